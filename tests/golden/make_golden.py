"""Writes the stored oracle values for the full-size (r = 50, N = 30) workload.

Calls only ``oracle/`` and ``synth/``.  One FP64 oracle step (eps = 1e-3, no
mask) from the seed-0 synthetic inputs; stores the scalars, block norms and a
fixed sample of residual / update / new 2-RDM elements, so the GPU test at the
full size does not have to rerun the ~40 s oracle.

    python tests/golden/make_golden.py        # -> tests/golden/r50_step.json
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import step as ost  # noqa: E402
from synth import generators as gen  # noqa: E402

EPS = 1e-3
NSAMPLE = 96


def sample_indices(r, n, seed):
    rng = np.random.default_rng(seed)
    return [tuple(int(x) for x in rng.integers(0, r, 4)) for _ in range(n)]


def main(name="r50", out="r50_step.json"):
    p = gen.named(name)
    r = p["r"]
    o = ost.step(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], EPS)
    idx = sample_indices(r, NSAMPLE, 1234)
    rec = dict(
        workload=name, r=r, N=p["N"], eps=EPS, seed=0,
        norm2=o["norm2"], energy0=o["energy0"], energy1=o["energy"],
        trace_scale=list(o["trace_scale"]),
        norms={k: float(np.linalg.norm(o[k])) for k in ("R_aa", "R_ab", "U_aa", "U_ab", "d2aa", "d2ab")},
        index=idx,
        samples={k: [float(o[k][t]) for t in idx] for k in ("R_aa", "R_ab", "U_aa", "U_ab", "d2aa", "d2ab")},
        gamma1=o["gamma"].tolist(),
    )
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", out, "norm2", o["norm2"], "E1", o["energy"])


if __name__ == "__main__":
    main()
