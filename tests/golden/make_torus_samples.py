"""Writes torus_oracle_samples.txt: sampled cells of the FP64 oracle's multi-resolution solve
(Algorithm 2, Sec. 3) of the torus layout (8^3 base blocks of 16^3, two refinement levels,
interpolation order 6), for the full-size GPU parity test.  Calls only the oracle and the
seeded input generator; the oracle's solve takes one to two minutes on one core.

    python3 tests/golden/make_torus_samples.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import multires                      # noqa: E402
from paper_1911_10228_amd import workloads       # noqa: E402

PER_LEVEL = 170                                  # sampled cells per refinement level
SEED = 20


def input_digest(L) -> str:
    """SHA-256 of the layout and the source (detects a change of the input generator)."""
    h = hashlib.sha256()
    for a in (np.ascontiguousarray(L.blocks, dtype=np.int64), np.ascontiguousarray(L.levels, dtype=np.int64),
              np.ascontiguousarray(L.f, dtype=np.float64)):
        h.update(a.tobytes())
    h.update(f"{L.n_b} {L.interp_order}".encode())
    return h.hexdigest()


def main():
    L = workloads.torus()
    u = multires.solve(L.blocks, L.levels, L.f, L.n_b, L.interp_order)
    rng = np.random.default_rng(SEED)
    n3 = L.n_b ** 3
    lines = [
        "# Sampled cells of the FP64 oracle's multi-resolution solve (Algorithm 2, Sec. 3) of the",
        "# torus layout: workloads.torus() (8^3 base blocks of 16^3, two refinement levels,",
        "# interpolation order 6).  Written by make_torus_samples.py (oracle only).",
        f"input_sha256 {input_digest(L)}",
        f"max_abs_u {np.abs(u).max():.17g}",
        "# block cell value   (cell = (z n_b + y) n_b + x within the block)",
    ]
    levels = np.asarray(L.levels)
    for lv in range(int(levels.max()) + 1):
        ids = np.nonzero(levels == lv)[0]
        bs = rng.choice(ids, size=PER_LEVEL)
        cs = rng.integers(0, n3, size=PER_LEVEL)
        for b, c in zip(bs, cs):
            lines.append(f"{int(b)} {int(c)} {u.reshape(len(L.blocks), n3)[b, c]:.17g}")
    with open(os.path.join(HERE, "torus_oracle_samples.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
