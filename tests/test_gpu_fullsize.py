"""GPU parity at the full workload size and at the largest supported r.

* r = 50, N = 30 (the headline workload, in the launch configuration bench.py
  times: autotuned tile, one acse_step at eps = 1e-3): sampled elements of R,
  U and the new 2-RDM, the block norms, ||R||^2, E before and after the step
  and the new 1-RDM against the stored oracle values of
  tests/golden/r50_step.json (written by tests/golden/make_golden.py, which
  calls only the oracle).  FP64 at 1e-10 and |dE| < 1e-7 Eh; FP32 and split
  BF16 at the per-result tolerances stated below.
* r = 96 (the largest r the library accepts): a closed-shell determinant in a
  random orbital basis, for which the Valdemoro reconstruction is exact and the
  residual has a closed form (tests/determinant_forms.py, pinned against Fock
  space brute force and the oracle on the CPU): every element of R_aa and R_ab,
  ||R||^2 and the energy; then one step, checked through the identity
  E1 - E0 = -eps ||R||^2 (Tr(K U) = -<R, R>) and Tr U = 0 per block.
"""
import json
import os

import numpy as np
import pytest

import determinant_forms as dform
from synth import generators as gen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "r50_step.json")

# per-result bars: (R samples, U samples, |dE| / |E1 - E0|, ||R||^2 relative), all
# relative to the largest stored sample of the array
TOL = {"fp64": (1e-10, 1e-10, 1e-14, 1e-10),
       "fp32": (1e-5, 5e-6, 1e-6, 1e-7),
       "bf16x3": (5e-5, 2e-5, 2e-6, 1e-6),
       "int8crt": (1e-10, 1e-10, 1e-13, 1e-10)}


@pytest.fixture(scope="module")
def acse():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2604_02550_amd as acse
    return acse


@pytest.fixture(scope="module")
def r50(acse):
    g = json.load(open(GOLDEN))
    p = gen.named(g["workload"])
    assert p["r"] == g["r"] == 50 and p["N"] == g["N"]
    ctx = acse.Context(r_max=p["r"])
    yield acse, ctx, g, p
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "int8crt"])
def test_r50_step_vs_stored_oracle(r50, precision):
    acse, ctx, g, p = r50
    print(f"[fullsize] r50 step precision={precision}", flush=True)
    prob, _ = ctx.problem(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2)
    ctx.autotune_raw(prob, ctx.options(precision))
    out = ctx.step(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2, eps=g["eps"],
                   precision=precision, return_ru=True)
    tR, tU, tE, tN = TOL[precision]
    idx = tuple(np.array(g["index"]).T)
    for key, tol in (("R_aa", tR), ("R_ab", tR), ("U_aa", tU), ("U_ab", tU)):
        ref = np.array(g["samples"][key])
        got = out[key].cpu().numpy()
        assert np.abs(got[idx] - ref).max() <= tol * np.abs(ref).max(), key
        nrm = float(np.linalg.norm(got))
        assert abs(nrm - g["norms"][key]) <= tol * g["norms"][key], key
    # the new 2-RDM moves by eps U: its error is eps times U's
    umax = max(np.abs(np.array(g["samples"][k])).max() for k in ("U_aa", "U_ab"))
    for key in ("d2aa", "d2ab"):
        ref = np.array(g["samples"][key])
        got = out[key].cpu().numpy()
        assert np.abs(got[idx] - ref).max() <= max(tU * g["eps"] * umax, 1e-12 * np.abs(ref).max()), key
    dE = abs(out["energy"] - g["energy1"])
    assert dE <= tE * abs(g["energy1"] - g["energy0"])
    print(f"[fullsize] r50 {precision}: |dE| = {dE:.3e} Eh", flush=True)
    if precision in ("fp64", "int8crt"):
        assert dE < 1e-7
    assert abs(out["norm2"] - g["norm2"]) <= tN * g["norm2"]
    # the 1-RDM sums r elements of the new 2-RDM per entry, times 2 / (N - 1)
    g1 = np.array(g["gamma1"])
    fac = 2.0 * g["r"] / (g["N"] - 1)
    assert np.abs(out["d1"].cpu().numpy() - g1).max() <= max(fac * tU * g["eps"] * umax, 1e-12 * np.abs(g1).max())


@pytest.mark.parametrize("precision", ["fp64", "int8crt"])
def test_r96_determinant_closed_form(acse, precision):
    r, na = 96, 29
    eps = 1e-6  # eps ||R||^2 is a few percent of |E|: the energy identity is well conditioned
    print(f"[fullsize] r={r} closed-shell determinant, n_alpha={na}, {precision}", flush=True)
    rng = np.random.default_rng(96)
    h, V = gen.hamiltonian(rng, r, 96)
    g, d2aa, d2ab = dform.rdms(r, na)
    caa, cab = dform.residual_blocks(h, V, na)
    n2 = 2.0 * np.sum(caa ** 2) + 4.0 * np.sum(cab ** 2)
    e0 = dform.energy(h, V, na)
    U = gen.haar_orthogonal(rng, r)
    rot = dform.rot4
    inputs = (dform.rot2(h, U), rot(V, U), dform.rot2(g, U), rot(d2aa, U), rot(d2ab, U))
    del V, d2aa, d2ab
    exp_aa, exp_ab = rot(caa, U), rot(cab, U)
    del caa, cab
    ctx = acse.Context(r_max=r)
    try:
        Raa, Rab, gn2 = ctx.residual(*inputs, na, precision=precision)
        scale = max(np.abs(exp_aa).max(), np.abs(exp_ab).max())
        assert np.abs(Raa.cpu().numpy() - exp_aa).max() <= 1e-10 * scale
        assert np.abs(Rab.cpu().numpy() - exp_ab).max() <= 1e-10 * scale
        del Raa, Rab
        assert abs(gn2 - n2) <= 1e-10 * n2
        ge = ctx.energy(inputs[0], inputs[1], inputs[3], inputs[4], na)
        assert abs(ge - e0) <= 1e-10 * abs(e0)
        out = ctx.step(*inputs, na, eps=eps, return_ru=True, precision=precision)
        assert abs(out["norm2"] - n2) <= 1e-10 * n2
        assert abs((out["energy"] - ge) + eps * n2) <= 1e-9 * eps * n2
        Uaa, Uab = out["U_aa"], out["U_ab"]
        umax = max(float(Uaa.abs().max()), float(Uab.abs().max()))
        for Ub in (Uaa, Uab):
            tr = float(Ub.reshape(r * r, r * r).diagonal().sum())
            assert abs(tr) <= 1e-12 * umax * r * r
    finally:
        ctx.close()
