"""Write the oracle's results on a few small seeded systems to
``oracle_small.json``.  Calls only the oracle and the input generators.

The paper prints no worked example (it has no tables or figures), so these
fixtures are regression values of the pinned oracle: test_golden checks that
the oracle still reproduces them bit for bit, so any later change to its
arithmetic shows up and has to be justified."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1208_4869_amd import inputs  # noqa: E402

CASES = [
    ("dense_n8_seed1", "dense", 8, 1),
    ("dense_n33_seed2", "dense", 33, 2),
    ("lattice_m3_seed3", "lattice", 3, 3),
]


def system(kind, size, seed):
    if kind == "dense":
        A, _, y = inputs.dense_system(size, seed)
    else:
        A = inputs.lattice_matrix(size)
        y = inputs.cn01(np.random.default_rng(seed), A.shape[0])
    return A, y


def cplx(v):
    return [[float(z.real), float(z.imag)] for z in np.asarray(v).ravel()]


def main():
    orc = oracle.get()
    out = {}
    for name, kind, size, seed in CASES:
        A, y = system(kind, size, seed)
        entry = {"kind": kind, "size": size, "seed": seed}
        for method in ("bicgstab", "cgnr"):
            r = getattr(orc, method)(A, y, tol=1e-10, maxit=200)
            entry[method] = {"info": r.info, "iters": r.iters,
                             "matvecs": r.matvecs, "x": cplx(r.x)}
        out[name] = entry
    with open(os.path.join(HERE, "oracle_small.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
