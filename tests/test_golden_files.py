"""The stored oracle outputs under tests/golden/ still match their recipe:
the inputs they were computed from are what the seeded input generators
produce now, and the files carry what the GPU tests read."""
import hashlib
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def test_tgv64_golden_matches_the_input_recipe():
    import sys
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_tgv64_golden as mk

    g = np.load(mk.OUT, allow_pickle=False)
    assert tuple(g["shape"]) == mk.SHAPE
    assert float(g["ma"]) == mk.MA and float(g["tau"]) == mk.TAU
    assert tuple(g["checkpoints"]) == mk.CHECKPOINTS
    fl = mk.input_fields()
    assert str(g["input_sha256"]) == mk.input_digest(fl)
    assert float(g["v0"]) == fl.meta["v0"]
    for n in mk.CHECKPOINTS:
        idx = g[f"sites_{n}"]
        assert np.array_equal(idx, mk.sample_sites(n))
        assert g[f"rho_{n}"].shape == idx.shape
        assert g[f"u_{n}"].shape == (3,) + idx.shape
        assert g[f"totals_{n}"].shape == (5,)
        # the stored samples lie within the stored full-grid maxima
        rmax, umax, tmax = g[f"max_{n}"]
        assert np.abs(g[f"rho_{n}"]).max() <= rmax
        assert np.sqrt((g[f"u_{n}"] ** 2).sum(0)).max() <= umax
        # mass is conserved by the stored run (Eq. conslaws)
        assert abs(g[f"totals_{n}"][0] - fl.rho.sum()) <= 1e-13 * fl.rho.sum()


def test_riemann_sensitivity_file_matches_its_recipe():
    import json
    import sys
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_riemann_sensitivity as mk

    with open(mk.OUT) as fh:
        rec = json.load(fh)
    assert tuple(rec["shape"]) == mk.SHAPE and rec["steps"] == mk.STEPS
    assert rec["tau"] == mk.TAU and rec["perturbation"] == mk.REL
    assert tuple(rec["seeds"]) == mk.SEEDS == tuple(range(len(rec["per_seed"])))
    for k, med in rec["median"].items():
        vals = sorted(e[k] for e in rec["per_seed"])
        assert vals[0] <= med <= vals[-1]
        # a rounding-level perturbation moves the result by far more than
        # rounding, but far less than the solution itself
        assert 1e-14 < med < 1e-10
