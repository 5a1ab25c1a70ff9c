// Host check of the tile element walk of the line kernels (the same source,
// compiled for the CPU): for every thread of a workgroup, across layouts,
// directions, workgroup sizes, line lengths and ragged tiles, the valid
// elements visited are exactly the tile's (pos, c) pairs, each once; their
// global offsets match the storage formula of the layout and stay inside the
// patch's storage; their LDS offsets are z[pos * ld + c]; the next-sample
// offset points at (pos + 1, c); every walk ends.  Prints the first failure
// and exits 1, else prints the number of cases and exits 0.
#include <cstdio>
#include <vector>

#include "../paper_2506_16076_amd/csrc/engine.h"

using namespace fcsd;

static long long layout_index(int i, int j, int n1, int nb1) {
  if (nb1) return 32LL * ((long long)(j >> 2) * nb1 + (i >> 3)) + 8 * (j & 3) + (i & 7);
  return (long long)j * n1 + i;
}

template <int DIR>
static bool check(int n1, int n2, int blocked, int line0, int nl, int ld, int bd) {
  const int nb1 = blocked ? (n1 + 7) / 8 : 0;
  const int N = DIR == 1 ? n1 : n2;
  const long long first = tile_first<DIR>(line0, nb1, n1);
  const long long storage = patch_storage(n1, n2, nb1);
  const unsigned gmax = 4u * (unsigned)(storage - 1 - first);
  std::vector<int> seen((size_t)N * nl, 0);
  for (int t = 0; t < bd; ++t) {
    Walk w = make_walk_t<DIR>(t, bd, N, nl, ld, nb1, n1);
    long long steps = 0;
    for (; w.more(); w.next()) {
      if (++steps > (long long)N * nl + 64) {
        printf("FAIL walk does not end: DIR %d n1 %d n2 %d blocked %d line0 %d nl %d ld %d bd %d t %d\n", DIR, n1,
               n2, blocked, line0, nl, ld, bd, t);
        return false;
      }
      if (!w.valid()) continue;
      const unsigned q = w.l / 8;
      const int pos = (int)(q / (unsigned)ld), c = (int)(q % (unsigned)ld);
      const int i = DIR == 1 ? pos : line0 + c, j = DIR == 1 ? line0 + c : pos;
      bool ok = w.l % 8 == 0 && w.g % 4 == 0 && pos < N && c < nl && w.g <= gmax;
      ok = ok && first + w.g / 4 == layout_index(i, j, n1, nb1) && w.g == tile_goff<DIR>(pos, c, nb1, n1);
      if (ok && pos + 1 < N) ok = w.g + w.gnext == tile_goff<DIR>(pos + 1, c, nb1, n1);
      if (ok) ok = ++seen[(size_t)pos * nl + c] == 1;
      if (!ok) {
        printf("FAIL element: DIR %d n1 %d n2 %d blocked %d line0 %d nl %d ld %d bd %d t %d pos %d c %d g %u l %u\n",
               DIR, n1, n2, blocked, line0, nl, ld, bd, t, pos, c, w.g, w.l);
        return false;
      }
    }
  }
  for (int pos = 0; pos < N; ++pos)
    for (int c = 0; c < nl; ++c)
      if (seen[(size_t)pos * nl + c] != 1) {
        printf("FAIL missed: DIR %d n1 %d n2 %d blocked %d line0 %d nl %d ld %d bd %d pos %d c %d\n", DIR, n1, n2,
               blocked, line0, nl, ld, bd, pos, c);
        return false;
      }
  // the end samples read for the side buffer stay inside the storage
  for (int c = 0; c < nl; ++c)
    for (int pos : {0, N - 1})
      if (tile_goff<DIR>(pos, c, nb1, n1) > gmax) {
        printf("FAIL end sample outside storage: DIR %d pos %d c %d\n", DIR, pos, c);
        return false;
      }
  return true;
}

int main() {
  const int sides[] = {11, 12, 13, 16, 31, 48, 57, 100, 129, 300, 512};
  const int bds[] = {64, 256, 512, 1024};
  long long cases = 0;
  for (int blocked = 0; blocked < 2; ++blocked)
    for (int n1 : sides)
      for (int n2 : {11, 20, 48, 97}) {
        for (int dir = 1; dir <= 2; ++dir) {
          const int nlines = dir == 1 ? n2 : n1;
          const int align = blocked ? (dir == 1 ? 4 : 8) : 1;
          for (int tile : {1, 3, 4, 8, 13, 24, 32, 64}) {
            int nlt = blocked ? (tile + align - 1) / align * align : tile;
            if (nlt > 64) nlt = 64;
            // tiles of nlt lines (the last one ragged) covering every line
            for (int line0 = 0; line0 < nlines; line0 += nlt) {
              const int nl = nlines - line0 < nlt ? nlines - line0 : nlt;
              for (int ld : {nl | 1, (2 * nl) | 1})
                for (int bd : bds) {
                  const bool ok = dir == 1 ? check<1>(n1, n2, blocked, line0, nl, ld, bd)
                                           : check<2>(n1, n2, blocked, line0, nl, ld, bd);
                  if (!ok) return 1;
                  ++cases;
                }
            }
          }
        }
      }
  printf("walk_check: %lld cases ok\n", cases);
  return 0;
}
