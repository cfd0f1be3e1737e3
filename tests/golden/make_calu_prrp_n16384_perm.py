"""Writes the oracle's CALU_PRRP permutation for the full-size tournament
workload: n = 16384 N(0,1) matrix (seed 16384, PCG64, so every machine draws
the same bits), b = 128, tau = 2, 512-row tiles, binary tree (Section 3.1).
Calls only oracle/ and the seeded input generator; takes a few minutes.

    python tests/golden/make_calu_prrp_n16384_perm.py
"""
import gzip
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import lu as olu  # noqa: E402
from paper_1208_2451_amd import inputs  # noqa: E402

N, B, TAU, TILE, SEED = 16384, 128, 2.0, 512, 16384
OUT = os.path.join(HERE, "calu_prrp_n16384_b128_t512_binary_perm.txt.gz")


def main():
    A, _ = inputs.randn_system(N, SEED)
    f = olu.calu_prrp(A, B, TAU, tile_rows=TILE, tree="binary")
    with gzip.open(OUT, "wt") as fh:
        fh.write("# oracle CALU_PRRP permutation: n=%d b=%d tau=%g tile_rows=%d binary, "
                 "randn seed %d; g_W=%.6g tree_height=%d\n" % (N, B, TAU, TILE, SEED, f.g_W,
                                                               getattr(f, "tree_height", -1)))
        fh.write("\n".join(str(int(p)) for p in f.perm))
        fh.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
