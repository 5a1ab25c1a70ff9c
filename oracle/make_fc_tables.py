"""Writes tests/golden/fc_tables.npz: the oracle's FC-Gram continuation
matrices A_r Q^T (FP64) for d = 5 and d = 2 over a range of C.  Calls only
oracle.fcgram.build_continuation (40-digit least-squares fit).

Usage: python -m oracle.make_fc_tables
"""
import numpy as np

from oracle.fcgram import build_continuation, _TABLE


def main():
    out = {}
    for d in (5, 2):
        for C in range(27, 46):
            out[f"d{d}_C{C}"] = build_continuation(d, C)
            print(d, C, np.abs(out[f"d{d}_C{C}"]).max(), flush=True)
    np.savez(_TABLE, **out)


if __name__ == "__main__":
    main()
