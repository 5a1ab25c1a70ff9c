// Host-side precomputation for the FC line engine (compiled with g++).
//
//  * FC-Gram continuation matrix A_r Q^T (paper Sec. 2.2, eq. "continuation").
//    The right blend of the d end samples is the least-squares
//    trigonometric polynomial (period P = 2(d + C) grid intervals, modes
//    0..K, K = 18) that matches the degree-(d-1) interpolant of the samples
//    on the matching interval [0, d-1] and vanishes on [d+C, 2d+C-1], both
//    sampled 20 times per interval; its values at d..d+C-1 form the tail.
//    The operator is linear in the samples, so column j of A_r Q^T is the
//    blend of the j-th Lagrange basis polynomial of the matching points.  (In
//    the Gram basis the same matrix factors as A_r Q^T; the Lagrange form
//    needs no orthogonalisation.)  The fit is solved by Householder QR in
//    IEEE binary128 (__float128), then rounded to double.
//  * The same rows differenced along the extension (the device derivative
//    transforms the first differences of the extension, see engine.h).
//  * Mixed-radix factorisation of the extension length L = N + C, the FP32
//    twiddle table exp(-2 pi i n / L) and the derivative multipliers,
//    computed in binary128.
#include <quadmath.h>

#include <cstdint>
#include <cstring>
#include <algorithm>
#include <array>
#include <vector>

namespace {

typedef __float128 qf;

const int kModes = 18;
const int kOversample = 20;

// cos and sin of 2 pi num / den with exact integer range reduction
void cis2pi(int64_t num, int64_t den, qf* c, qf* s) {
  num %= den;
  if (num < 0) num += den;
  qf a = 2 * M_PIq * (qf)num / (qf)den;
  *c = cosq(a);
  *s = sinq(a);
}

// A_r Q^T in binary128, C rows of d entries.
int fc_matrix_q(int d, int C, std::vector<qf>& out) {
  if (d < 1 || d > 8 || C < 1 || C > 256) return 1;
  const int P = 2 * (d + C);           // period in grid intervals
  const int ncol = 2 * kModes + 1;
  const int per = (d - 1) * kOversample + 1;
  const int nrow = (d == 1) ? 2 : 2 * per;
  // sample points in units of 1/kOversample grid intervals
  std::vector<int64_t> pts;
  for (int i = 0; i < per; ++i) pts.push_back(i);
  for (int i = 0; i < per; ++i) pts.push_back((int64_t)(d + C) * kOversample + i);
  const int m = (int)pts.size();
  (void)nrow;
  const int64_t den = (int64_t)P * kOversample;  // angle = 2 pi n s / (P * os)
  std::vector<qf> A((size_t)m * ncol);
  for (int r = 0; r < m; ++r) {
    A[(size_t)r * ncol] = 1;
    for (int n = 1; n <= kModes; ++n) {
      qf c, s;
      cis2pi((int64_t)n * pts[r], den, &c, &s);
      A[(size_t)r * ncol + 2 * n - 1] = c;
      A[(size_t)r * ncol + 2 * n] = s;
    }
  }
  // right-hand sides: Lagrange basis polynomial j on the matching interval, 0 on the zero interval
  std::vector<qf> B((size_t)m * d, 0);
  for (int r = 0; r < per; ++r) {
    qf t = (qf)pts[r] / kOversample;
    for (int j = 0; j < d; ++j) {
      qf v = 1;
      for (int k = 0; k < d; ++k)
        if (k != j) v *= (t - k) / (qf)(j - k);
      B[(size_t)r * d + j] = v;
    }
  }
  // Householder QR of A applied to B
  for (int k = 0; k < ncol; ++k) {
    qf nrm = 0;
    for (int r = k; r < m; ++r) nrm += A[(size_t)r * ncol + k] * A[(size_t)r * ncol + k];
    nrm = sqrtq(nrm);
    if (nrm == 0) return 2;
    qf akk = A[(size_t)k * ncol + k];
    qf alpha = akk > 0 ? -nrm : nrm;
    std::vector<qf> v(m - k);
    v[0] = akk - alpha;
    for (int r = k + 1; r < m; ++r) v[r - k] = A[(size_t)r * ncol + k];
    qf vv = 0;
    for (qf x : v) vv += x * x;
    if (vv == 0) continue;
    for (int c = k; c < ncol; ++c) {
      qf dot = 0;
      for (int r = k; r < m; ++r) dot += v[r - k] * A[(size_t)r * ncol + c];
      qf f = 2 * dot / vv;
      for (int r = k; r < m; ++r) A[(size_t)r * ncol + c] -= f * v[r - k];
    }
    for (int c = 0; c < d; ++c) {
      qf dot = 0;
      for (int r = k; r < m; ++r) dot += v[r - k] * B[(size_t)r * d + c];
      qf f = 2 * dot / vv;
      for (int r = k; r < m; ++r) B[(size_t)r * d + c] -= f * v[r - k];
    }
  }
  // back substitution R x = (Q^T B)[:ncol]
  std::vector<qf> X((size_t)ncol * d);
  for (int c = 0; c < d; ++c) {
    for (int i = ncol - 1; i >= 0; --i) {
      qf acc = B[(size_t)i * d + c];
      for (int j = i + 1; j < ncol; ++j) acc -= A[(size_t)i * ncol + j] * X[(size_t)j * d + c];
      X[(size_t)i * d + c] = acc / A[(size_t)i * ncol + i];
    }
  }
  // evaluate at the continuation points t = d .. d+C-1
  for (int mm = 0; mm < C; ++mm) {
    int64_t t = (int64_t)(d + mm) * kOversample;
    for (int c = 0; c < d; ++c) {
      qf acc = X[c];
      for (int n = 1; n <= kModes; ++n) {
        qf cs, sn;
        cis2pi((int64_t)n * t, den, &cs, &sn);
        acc += X[(size_t)(2 * n - 1) * d + c] * cs + X[(size_t)(2 * n) * d + c] * sn;
      }
      out[(size_t)mm * d + c] = acc;
    }
  }
  return 0;
}

}  // namespace

extern "C" int fcsd_host_fc_matrix(int d, int C, double* out) {
  if (!out) return 1;
  std::vector<qf> q((size_t)C * d > 0 ? (size_t)C * d : 1);
  const int r = fc_matrix_q(d, C, q);
  if (r) return r;
  for (size_t i = 0; i < (size_t)C * d; ++i) out[i] = (double)q[i];
  return 0;
}

// Differenced continuation rows.  With e_0 = f[N-1], e_{1+m} = tail[m]
// (m < C) and e_{C+1} = f[0] (the periodic wrap), row r = 0..C holds the
// coefficients of e_{r+1} - e_r on the 2d end samples: entries 0..d-1 act
// on f[N-d+j], entries d..2d-1 on f[j].  Differences are taken in binary128
// before rounding to double.
extern "C" int fcsd_host_fc_dmatrix(int d, int C, double* out) {
  if (!out) return 1;
  std::vector<qf> q((size_t)C * d > 0 ? (size_t)C * d : 1);
  const int rc = fc_matrix_q(d, C, q);
  if (rc) return rc;
  std::vector<qf> a(2 * d), b(2 * d);
  auto row = [&](int rr, std::vector<qf>& v) {
    for (auto& x : v) x = 0;
    if (rr == 0) {
      v[d - 1] = 1;
    } else if (rr == C + 1) {
      v[d] = 1;
    } else {
      const int m = rr - 1;
      for (int j = 0; j < d; ++j) {
        v[j] = q[(size_t)m * d + j];
        v[d + j] = q[(size_t)(C - 1 - m) * d + (d - 1 - j)];
      }
    }
  };
  for (int r = 0; r <= C; ++r) {
    row(r + 1, a);
    row(r, b);
    for (int k = 0; k < 2 * d; ++k) out[(size_t)r * 2 * d + k] = (double)(a[k] - b[k]);
  }
  return 0;
}

// Twiddle table w[n] = exp(-2 pi i n / L), n < L, interleaved (re, im) FP32.
extern "C" void fcsd_host_twiddles(int L, float* out) {
  for (int n = 0; n < L; ++n) {
    qf c, s;
    cis2pi(n, L, &c, &s);
    out[2 * n] = (float)c;
    out[2 * n + 1] = (float)(-s);
  }
}

// Radix plan of a transform of length L: the radices r_0 .. r_{s-1} (product
// L, at most 8) of the in-place stages.  The engine runs stages 0 .. s-2
// forward and again inverse, each with twiddles, and the last one fused with
// the multiplier and the first inverse butterfly, so a plan costs
// 2 sum_{i < s-1} c(r_i) + c_f(r_{s-1}).  c and c_f are the vector
// instructions per point of one stage of the generated code for gfx950 plus a
// fixed charge for the LDS round trip and the barrier of a stage; the search
// is exhaustive over the divisors of L.  Returns the number of stages, or 0 if
// L has a prime factor above 13 or needs more than 8 stages.
namespace {
struct RadixCost {
  int r;
  double stage, fused;
};
constexpr double kStageCharge = 4.0;
constexpr RadixCost kRadixCost[] = {
    {2, 13.0, 15.0},  {3, 13.3, 17.0},  {4, 12.75, 16.0}, {5, 15.4, 21.8},  {6, 13.7, 19.0},
    {7, 16.9, 25.6},  {8, 13.75, 19.5}, {9, 16.9, 25.9},  {10, 16.2, 24.6}, {11, 20.5, 33.4},
    {12, 14.8, 22.0}, {13, 22.5, 37.3}, {14, 18.1, 28.7}, {15, 17.9, 28.2}, {16, 16.4, 25.3},
};
}  // namespace

extern "C" int fcsd_host_factor(int L, int* rad) {
  if (L < 2) return 0;
  const double inf = 1e300;
  // best[n][k]: cheapest k twiddle stages with product n (forward + inverse)
  std::vector<std::array<double, 8>> best(L + 1);
  std::vector<std::array<int, 8>> pick(L + 1);
  for (int n = 0; n <= L; ++n) {
    best[n].fill(inf);
    pick[n].fill(0);
  }
  best[1][0] = 0.0;
  for (int n = 2; n <= L; ++n) {
    if (L % n) continue;
    for (int k = 1; k < 8; ++k)
      for (const RadixCost& c : kRadixCost) {
        if (n % c.r || best[n / c.r][k - 1] >= inf) continue;
        const double v = best[n / c.r][k - 1] + 2.0 * (c.stage + kStageCharge);
        if (v < best[n][k]) {
          best[n][k] = v;
          pick[n][k] = c.r;
        }
      }
  }
  double top = inf;
  int last = 0, kk = -1;
  for (const RadixCost& c : kRadixCost) {
    if (L % c.r) continue;
    for (int k = 0; k < 8; ++k) {
      const double v = best[L / c.r][k] + c.fused + kStageCharge;
      if (v < top) {
        top = v;
        last = c.r;
        kk = k;
      }
    }
  }
  if (kk < 0) return 0;
  int n = L / last, s = 0;
  for (int k = kk; k > 0; --k) {
    rad[s++] = pick[n][k];
    n /= pick[n][k];
  }
  std::sort(rad, rad + s, [](int a, int b) { return a > b; });
  rad[s++] = last;
  return s;
}

// Position -> signed wavenumber map of the in-place decimation-in-frequency
// output: position p = sum_s q_s m_s (m_s = L / (r_0 ... r_s)) holds the
// coefficient of frequency k = sum_s q_s (r_0 ... r_{s-1}).  Fills, as
// interleaved (re, im) pairs, the multiplier that turns the DFT of the
// differenced extension into that of the derivative: i w_k / (exp(2 pi i k
// / L) - 1) with w_k = 2 pi k (N-1) / L^2 (the FFT normalisation 1/L and
// the period beta = L/(N-1) folded in); k = 0 and the Nyquist of even L are
// zero.
namespace {
int64_t position_wavenumber(int p, int L, int nst, const int* rad) {
  int rem = p, M = L;
  int64_t k = 0, place = 1;
  for (int s = 0; s < nst; ++s) {
    int m = M / rad[s];
    int q = rem / m;
    rem -= q * m;
    k += (int64_t)q * place;
    place *= rad[s];
    M = m;
  }
  return k;
}
}  // namespace

extern "C" void fcsd_host_kmul(int N, int L, int nst, const int* rad, float* out, int periodic) {
  for (int p = 0; p < L; ++p) {
    const int64_t k = position_wavenumber(p, L, nst, rad);
    int64_t ks = (k <= L / 2) ? k : k - L;
    if (L % 2 == 0 && k == L / 2) ks = 0;
    // derivative w.r.t. q in [0, 1]: beta = L h, h = 1/(N-1); periodic mode h = 1/N, beta = 1
    const qf scale = periodic ? 2 * M_PIq / L : 2 * M_PIq * (N - 1) / ((qf)L * L);
    const qf w = scale * (qf)ks;
    // the engine transforms the differenced extension, whose DFT is
    // (exp(2 pi i k / L) - 1) times that of the extension:
    //   i w / (exp(i theta) - 1) = w exp(-i theta / 2) / (2 sin(theta / 2)),  theta = 2 pi k / L
    qf re = 0, im = 0;
    if (ks != 0) {
      qf c, sn;
      cis2pi(k, 2 * (int64_t)L, &c, &sn);
      const qf a = w / (2 * sn);
      re = a * c;
      im = -a * sn;
    }
    out[2 * p] = (float)re;
    out[2 * p + 1] = (float)im;
  }
}

// Filter factors by position of the same digit-reversed order (paper Sec.
// 4.3.1, eq. filtering): sigma(2k/L) / L = exp(-alpha (2k/L)^p) / L for the
// signed wavenumber k of the position (the FFT normalisation 1/L folded in),
// as (re, 0) pairs.  p is even, so the sign of k (and the side the Nyquist of
// an even L is counted on) does not matter.
extern "C" void fcsd_host_fmul(int L, int nst, const int* rad, double alpha, int p, float* out) {
  for (int pos = 0; pos < L; ++pos) {
    const int64_t k = position_wavenumber(pos, L, nst, rad);
    const int64_t ks = (k <= L / 2) ? k : k - L;
    const qf x = 2 * (qf)ks / L;
    const qf v = expq(-(qf)alpha * powq(x, p)) / L;
    out[2 * pos] = (float)v;
    out[2 * pos + 1] = 0.0f;
  }
}

// ------------------------------------------------------------------ embedded circulants
// A line operator of the engine is a circulant of the extension length
// L = N + C (the FC derivative, eq. fc_der, on the differenced extension;
// the spectral filter, eq. filtering).  When L has a prime factor above 13
// there is no mixed-radix plan of length L; the circulant is then applied as
// a cyclic convolution of a 13-smooth length M >= N + L: the line is padded
// with zeros to M and the kernel's first column h (period L) is wrapped as
// k[t mod M] = h[t mod L] for t in [-(L-1), N], zero elsewhere.  For the
// outputs n < N of inputs m < L (the forward operators) n - m lies in
// [-(L-1), N-1], for the transposes (inputs m <= N, outputs n < N) m - n in
// [-(N-1), N]; on both ranges k equals h's periodic continuation and the
// ranges do not wrap onto each other in M >= N + L, so the cyclic convolution
// of length M returns the circulant of length L exactly (in exact
// arithmetic) on the positions used.

// Smallest length M >= n whose prime factors are at most 13 and that has a
// radix plan of at most 8 stages; 0 if none up to 65536.
extern "C" int fcsd_host_embed_length(int n) {
  int rad[8];
  for (int M = std::max(n, 2); M <= 65536; ++M) {
    int m = M;
    for (int q : {2, 3, 5, 7, 11, 13})
      while (m % q == 0) m /= q;
    if (m == 1 && fcsd_host_factor(M, rad) > 0) return M;
  }
  return 0;
}

namespace {
typedef long double ldt;

// First column h[0..L-1] of a line circulant of length L.
// kind 0: derivative of the differenced extension, the multipliers
//   i w_k / (exp(2 pi i k / L) - 1), w_k = 2 pi k / beta (beta = L / (N-1),
//   or 1 for a periodic line), k = 0 and the Nyquist of an even L zero:
//   h[r] = (1/L) sum_{k=1}^{(L-1)/2} w_k cos(2 pi k (2r - 1) / (2L)) / sin(pi k / L);
// kind 1: spectral filter, sigma(2k/L) = exp(-alpha (2k/L)^p) on every k:
//   h[r] = (1/L) (sigma_0 + 2 sum_k sigma_k cos(2 pi k r / L) + [L even] sigma_{L/2} (-1)^r).
std::vector<ldt> circulant_column(int kind, int N, int L, int periodic, double alpha, int p) {
  std::vector<ldt> h(L, 0.0L);
  const int K = (L - 1) / 2;
  if (kind == 0) {
    const qf wscale = periodic ? 2 * M_PIq : 2 * M_PIq * (N - 1) / (qf)L;
    const int64_t L2 = 2 * (int64_t)L;
    std::vector<ldt> cs2(L2);  // cos(2 pi j / (2L))
    std::vector<ldt> inv_s(K + 1);
    for (int j = 0; j < L2; ++j) {
      qf c, sn;
      cis2pi(j, L2, &c, &sn);
      cs2[j] = (ldt)c;
      if (j >= 1 && j <= K) inv_s[j] = (ldt)(wscale * (qf)j / sn);  // w_j / sin(pi j / L)
    }
    for (int r = 0; r < L; ++r) {
      ldt acc = 0.0L;
      for (int k = 1; k <= K; ++k) {
        int64_t num = ((int64_t)k * (2 * (int64_t)r - 1)) % L2;
        if (num < 0) num += L2;
        acc += inv_s[k] * cs2[num];
      }
      h[r] = acc / (ldt)L;
    }
  } else {
    std::vector<ldt> sig(L / 2 + 1), cs(L);
    for (int k = 0; k <= L / 2; ++k) sig[k] = (ldt)expq(-(qf)alpha * powq(2 * (qf)k / L, p));
    for (int j = 0; j < L; ++j) {
      qf c, sn;
      cis2pi(j, L, &c, &sn);
      cs[j] = (ldt)c;
    }
    for (int r = 0; r < L; ++r) {
      ldt acc = sig[0];
      for (int k = 1; k <= K; ++k) acc += 2.0L * sig[k] * cs[(int)(((int64_t)k * r) % L)];
      if (L % 2 == 0) acc += sig[L / 2] * ((r & 1) ? -1.0L : 1.0L);
      h[r] = acc / (ldt)L;
    }
  }
  return h;
}

// Multiplier table of the wrapped kernel for the engine's transform of
// length M (plan rad): position pos holds DFT_M(k)[kappa] / M for the
// wavenumber kappa of the position (the inverse transform's 1/M folded in),
// as interleaved (re, im) FP32 pairs.
void embedded_table(const std::vector<ldt>& h, int N, int L, int M, int nst, const int* rad, float* out) {
  std::vector<ldt> k(M, 0.0L);
  for (int t = -(L - 1); t <= N; ++t) {
    int tm = t % M, tl = t % L;
    if (tm < 0) tm += M;
    if (tl < 0) tl += L;
    k[tm] = h[tl];
  }
  std::vector<ldt> cs(M), sn(M);
  for (int j = 0; j < M; ++j) {
    qf c, s;
    cis2pi(j, M, &c, &s);
    cs[j] = (ldt)c;
    sn[j] = (ldt)s;
  }
  for (int pos = 0; pos < M; ++pos) {
    const int64_t kap = position_wavenumber(pos, M, nst, rad);
    ldt re = 0.0L, im = 0.0L;
    for (int t = 0; t < M; ++t) {
      if (k[t] == 0.0L) continue;
      const int j = (int)((kap * t) % M);
      re += k[t] * cs[j];
      im -= k[t] * sn[j];
    }
    out[2 * pos] = (float)(re / (ldt)M);
    out[2 * pos + 1] = (float)(im / (ldt)M);
  }
}
}  // namespace

// Derivative multipliers of a line of N points with extension length L
// embedded in a transform of length M (see above).
extern "C" void fcsd_host_kmul_embedded(int N, int L, int M, int nst, const int* rad, float* out, int periodic) {
  embedded_table(circulant_column(0, N, L, periodic, 0.0, 0), N, L, M, nst, rad, out);
}

// Spectral filter factors (alpha, p) of an extension of length L embedded
// in a transform of length M.
extern "C" void fcsd_host_fmul_embedded(int N, int L, int M, int nst, const int* rad, double alpha, int p,
                                        float* out) {
  embedded_table(circulant_column(1, N, L, 0, alpha, p), N, L, M, nst, rad, out);
}

// Fold matrix of a transposed FC line operator (paper Sec. 2.2, eqs.
// continuation and fc_der, transposed).  A line operator of the engine is
// R K E: E extends the N samples by the continuation tail (T, C x 2d on the
// end samples), K is a circulant of length L = N + C with first column k,
// R keeps positions 0..N-1.  Its transpose is E^T K^T R^T: on positions
// < N the circulant's own transpose, plus the fold T^T (K^T)[N.., 0..N-1] of
// the tail onto the 2d end samples.  The fold's matrix entries reach ~1e4
// (T) times the circulant's, so the device applies it in FP64 straight to
// the cotangent instead of folding a tail rounded by an FP32 transform.
//   out[n * 2d + e] = sum_{m < C} T[m][e] k[(n - N - m) mod L],  n < N,
// e < d: right end sample N-d+e (T[m][e] = (A_r Q^T)[m][e]); e >= d: left end
// sample e-d (T[m][e] = (A_r Q^T)[C-1-m][2d-1-e]).
// kind 0: derivative, k[r] = (1/L) sum_kappa (2 pi i kappa / beta)
//   exp(2 pi i kappa r / L), beta = L/(N-1), |kappa| < L/2 (the Nyquist mode
//   of an even L is zero);
// kind 1: spectral filter (Sec. 4.3.1, eq. filtering), k[r] = (1/L) sum_kappa
//   sigma(2 kappa / L) exp(2 pi i kappa r / L), sigma(x) = exp(-alpha x^p),
//   Nyquist included.
// The circulant's column is summed in long double over binary128 sine and
// cosine tables.  arq: A_r Q^T in double, C rows of d.
extern "C" int fcsd_host_fold_matrix(int N, int C, int d, const double* arq, int kind, double alpha, int p,
                                     double* out) {
  if (!arq || !out || N < 2 * d || C < 1 || d < 1 || d > 8 || (kind != 0 && kind != 1)) return 1;
  const int L = N + C;
  typedef long double ld;
  std::vector<ld> sn(L), cs(L), k(L, 0.0L);
  for (int j = 0; j < L; ++j) {
    qf c, s;
    cis2pi(j, L, &c, &s);
    cs[j] = (ld)c;
    sn[j] = (ld)s;
  }
  const int M = (L - 1) / 2;  // kappa = 1..M pairs with -kappa; an even L's Nyquist L/2 is apart
  if (kind == 0) {
    // (1/L) (2 pi i kappa / beta) (e^{i phi} - e^{-i phi}) = -(2/L) (2 pi kappa / beta) sin(phi)
    const ld w = 2.0L * (ld)M_PIq * (ld)(N - 1) / ((ld)L * (ld)L);
    for (int r = 0; r < L; ++r) {
      ld acc = 0.0L;
      for (int kap = 1; kap <= M; ++kap) acc += (ld)kap * sn[(int)(((int64_t)kap * r) % L)];
      k[r] = -2.0L * w * acc;
    }
  } else {
    std::vector<ld> sig(L / 2 + 1);
    for (int kap = 0; kap <= L / 2; ++kap) sig[kap] = (ld)expq(-(qf)alpha * powq(2 * (qf)kap / L, p));
    for (int r = 0; r < L; ++r) {
      ld acc = sig[0];
      for (int kap = 1; kap <= M; ++kap) acc += 2.0L * sig[kap] * cs[(int)(((int64_t)kap * r) % L)];
      if (L % 2 == 0) acc += sig[L / 2] * ((r & 1) ? -1.0L : 1.0L);
      k[r] = acc / (ld)L;
    }
  }
  for (int n = 0; n < N; ++n)
    for (int e = 0; e < 2 * d; ++e) {
      ld acc = 0.0L;
      for (int m = 0; m < C; ++m) {
        const double t = e < d ? arq[(size_t)m * d + e] : arq[(size_t)(C - 1 - m) * d + (2 * d - 1 - e)];
        int r = (n - N - m) % L;
        if (r < 0) r += L;
        acc += (ld)t * k[r];
      }
      out[(size_t)n * 2 * d + e] = (double)acc;
    }
  return 0;
}
