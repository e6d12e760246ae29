"""Writes the stored oracle values of the full-size open-shell residual with
the NY 3-RDM (r = 50, N_alpha = 16, N_beta = 14, default open-shell
occupations).

Calls only ``oracle/`` and ``synth/``.  One FP64 oracle residual of the
spin-block form (Eq. (4) with the 3-RDM of Eq. (8)) from the seed-0 synthetic
inputs of the open-shell workload; stores ||R||^2, the block norms and a fixed
sample of elements of the three residual blocks, so the GPU test at the full
size does not rerun the oracle (a few minutes, about 10 GB of host memory).

    python tests/golden/make_golden_spin_ny.py   # -> tests/golden/r50_spin_ny_residual.json
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import step as ost  # noqa: E402
from synth import generators as gen  # noqa: E402

NSAMPLE = 96
KEYS = ("R_aa", "R_bb", "R_ab")


def sample_indices(r, n, seed):
    rng = np.random.default_rng(seed)
    return [tuple(int(x) for x in rng.integers(0, r, 4)) for _ in range(n)]


def main(name="r50s", out="r50_spin_ny_residual.json"):
    p = gen.named_spin(name)
    r = p["r"]
    sig = ost.sigma_open_shell(r, p["Na"], p["Nb"])
    raa, rbb, rab, n2 = ost.residual_spin(p["h"], p["V"], p["Na"], p["Nb"], p["gamma_a"], p["gamma_b"], p["d2aa"],
                                          p["d2bb"], p["d2ab"], sigma_so=sig)
    o = dict(R_aa=raa, R_bb=rbb, R_ab=rab)
    idx = sample_indices(r, NSAMPLE, 8642)
    rec = dict(
        workload=name, r=r, Na=p["Na"], Nb=p["Nb"], seed=0, sigma="open-shell default",
        norm2=n2,
        norms={k: float(np.linalg.norm(o[k])) for k in KEYS},
        index=idx,
        samples={k: [float(o[k][t]) for t in idx] for k in KEYS},
    )
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", out, "norm2", n2)


if __name__ == "__main__":
    main()
