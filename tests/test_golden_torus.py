"""The stored oracle samples of the full torus solve (tests/golden/torus_oracle_samples.txt,
written by tests/golden/make_torus_samples.py from the oracle alone) belong to the layout and
source the generator produces now, and cover every refinement level; the GPU test compares
the full-size solves with them."""
import importlib.util
import os

import numpy as np

from paper_1911_10228_amd import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_torus_samples_match_the_generator():
    spec = importlib.util.spec_from_file_location("make_torus_samples", os.path.join(GOLDEN, "make_torus_samples.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    digest, umax, rows = None, None, []
    for line in open(os.path.join(GOLDEN, "torus_oracle_samples.txt")):
        p = line.split()
        if not p or p[0].startswith("#"):
            continue
        if p[0] == "input_sha256":
            digest = p[1]
        elif p[0] == "max_abs_u":
            umax = float(p[1])
        else:
            rows.append((int(p[0]), int(p[1]), float(p[2])))
    L = workloads.torus()
    assert digest == mk.input_digest(L), "torus input changed: rerun tests/golden/make_torus_samples.py"
    levels = np.asarray(L.levels)
    b = np.array([r[0] for r in rows])
    c = np.array([r[1] for r in rows])
    v = np.array([r[2] for r in rows])
    assert len(rows) == 3 * mk.PER_LEVEL and (c >= 0).all() and (c < L.n_b ** 3).all()
    assert np.bincount(levels[b], minlength=3).tolist() == [mk.PER_LEVEL] * 3
    # a negative kernel convolved with a non-negative source: u <= 0, bounded by its maximum
    assert (v <= 0).all() and np.abs(v).max() <= umax
