"""Writes the stored oracle values of the Nakatsuji-Yasuda residual for the
full-size (r = 50, N = 30) workload.

Calls only ``oracle/`` and ``synth/``.  One FP64 oracle residual with the NY
3-RDM of Eq. (8) (sigma: orbitals 0 .. N/2 - 1 occupied) from the seed-0
synthetic inputs, in the factorised form whose agreement with the
materialised definition ``tests/test_oracle_ny.py`` pins; stores ||R||^2, the
block norms and the elements at the sample indices of ``r50_step.json``, so
the GPU test at the full size does not rerun the oracle (several minutes).

    python tests/golden/make_golden_ny.py     # -> tests/golden/r50_ny_residual.json
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import step as ost  # noqa: E402
from synth import generators as gen  # noqa: E402


def main(name="r50", out="r50_ny_residual.json"):
    p = gen.named(name)
    r, N = p["r"], p["N"]
    base = json.load(open(os.path.join(HERE, "r50_step.json")))
    idx = [tuple(t) for t in base["index"]]
    sigma = np.where(np.arange(r) < N // 2, 1.0, -1.0)
    t0 = time.time()
    raa, rab, n2 = ost.residual(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"], sigma=sigma)
    rec = dict(
        workload=name, r=r, N=N, seed=0, sigma="orbitals below N/2 occupied",
        norm2=n2,
        norms={"R_aa": float(np.linalg.norm(raa)), "R_ab": float(np.linalg.norm(rab))},
        index=[list(t) for t in idx],
        samples={"R_aa": [float(raa[t]) for t in idx], "R_ab": [float(rab[t]) for t in idx]},
    )
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", out, "norm2", n2, "in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
