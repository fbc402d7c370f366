"""The oracle reproduces its stored results (tests/golden/oracle_small.json,
written by tests/golden/make_golden.py from the oracle alone) bit for bit."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden  # noqa: E402


def test_oracle_matches_golden(orc):
    with open(os.path.join(HERE, "golden", "oracle_small.json")) as f:
        gold = json.load(f)
    for name, kind, size, seed in make_golden.CASES:
        A, y = make_golden.system(kind, size, seed)
        for method in ("bicgstab", "cgnr"):
            g = gold[name][method]
            r = getattr(orc, method)(A, y, tol=1e-10, maxit=200)
            assert (r.info, r.iters, r.matvecs) == (g["info"], g["iters"],
                                                    g["matvecs"])
            x = np.array([complex(a, b) for a, b in g["x"]])
            assert np.array_equal(r.x, x), (name, method)
