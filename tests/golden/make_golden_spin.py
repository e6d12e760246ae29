"""Writes the stored oracle values for the full-size open-shell workload
(r = 50, N_alpha = 16, N_beta = 14).

Calls only ``oracle/`` and ``synth/``.  One FP64 oracle step of the spin-block
form (eps = 1e-3, no mask) from the seed-0 synthetic inputs; stores the
scalars, block norms and a fixed sample of residual / update / new 2-RDM
elements of the three spin blocks, so the GPU test and the bench at the full
size do not rerun the oracle (about a minute).

    python tests/golden/make_golden_spin.py   # -> tests/golden/r50_spin_step.json
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
KEYS = ("R_aa", "R_bb", "R_ab", "U_aa", "U_bb", "U_ab", "d2aa", "d2bb", "d2ab")


def sample_indices(r, n, seed):
    rng = np.random.default_rng(seed)
    return [tuple(int(x) for x in rng.integers(0, r, 4)) for _ in range(n)]


def main(name="r50s", out="r50_spin_step.json"):
    p = gen.named_spin(name)
    r = p["r"]
    o = ost.step_spin(p["h"], p["V"], p["Na"], p["Nb"], p["gamma_a"], p["gamma_b"], p["d2aa"], p["d2bb"],
                      p["d2ab"], EPS)
    idx = sample_indices(r, NSAMPLE, 4321)
    rec = dict(
        workload=name, r=r, Na=p["Na"], Nb=p["Nb"], eps=EPS, seed=0,
        norm2=o["norm2"], energy0=o["energy0"], energy1=o["energy"],
        trace_scale=list(o["trace_scale"]),
        norms={k: float(np.linalg.norm(o[k])) for k in KEYS},
        index=idx,
        samples={k: [float(o[k][t]) for t in idx] for k in KEYS},
        gamma_a=o["gamma_a"].tolist(), gamma_b=o["gamma_b"].tolist(),
    )
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", out, "norm2", o["norm2"], "E1", o["energy"])


if __name__ == "__main__":
    main()
