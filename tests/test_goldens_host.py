"""The stored oracle results under tests/golden/ (written by
tests/golden/make_goldens.py from the oracle alone): the expected cases are
present and each file is consistent with the workload it names."""

import glob
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from make_goldens import load, cpqr_flops  # noqa: E402


def _cases():
    out = []
    for p in sorted(glob.glob(os.path.join(HERE, "golden", "c*_s*_eps*.json"))):
        parts = os.path.basename(p)[:-5].split("_")
        w, s, e = parts[:3]
        out.append((w, int(s[1:]), float(e[3:]), len(parts) == 3))
    return out


def test_expected_cases_present():
    have = set(_cases())
    for s in (0, 1, 2):
        for e in (1e-2, 1e-4, 1e-6):
            assert ("c2", s, e, True) in have
    assert ("c4", 0, 1e-2, True) in have and ("c3", 0, 1e-2, True) in have
    assert ("c2", 0, 1e-2, False) in have


def test_records_are_consistent():
    from problems import config_problem
    from oracle.ordering import order_grid
    orderings = {}
    for w, s, e, scale in _cases():
        g = load(w, s, e, scale)
        assert g.get("scale", True) == scale
        assert g["gmres_relres"] <= 1e-10 and g["gmres_iterations"] >= 1
        assert abs(cpqr_flops(g["cpqr_shapes"]) - g["cpqr_flops"]) <= 1e-9 * g["cpqr_flops"]
        # ranks never exceed the interface size or the number of columns
        P, m, r = g["cpqr_shapes"].T
        assert np.all(r <= np.minimum(P, m)) and np.all(r >= 0)
        if w not in orderings:
            prob = config_problem(w, seed=0)
            orderings[w] = order_grid(prob["dims"], prob["levels"])
        o = orderings[w]
        assert g["n"] == o.perm.size and g["levels"] == o.L
        for k, sizes in g["stage_sizes"].items():
            st, en, _, _ = o.stage_clusters(k)
            assert sizes.shape == st.shape
            # a cluster never holds more unknowns than its points
            assert np.all(sizes <= en - st) and np.all(sizes >= 0)
        # without sparsification below the first sparsified stage, sizes are whole
        top = max(g["sparsified_stages"])
        for k in range(g["levels"], top, -1):
            st, en, _, _ = o.stage_clusters(k)
            assert np.array_equal(g["stage_sizes"][k], en - st)
        assert g["sample_idx"].size == min(512, g["n"]) and np.all(np.diff(g["sample_idx"]) > 0)
