"""GPU parity of the Nakatsuji-Yasuda reconstruction (Eq. (8); App. D, NY
part) against the oracle (tier B with the NY share, pinned in
test_oracle_ny.py).

* Residual at r = 4, 9, 16, 24 (r^2 = 16 .. 576: one to five GEMM tiles with
  ragged edges) with the default reference occupations and with sigma patterns that
  are not a prefix; FP64 bar 1e-10 of the largest element, on the residual
  and, separately, on the NY share alone (NY residual minus Valdemoro
  residual, both from the same side), so a wrong share cannot hide below the
  Valdemoro part.
* One Euler step (both maps with the NY 3-RDM) and the Euler driver with the
  fixed control, against the oracle's step and iteration.
* r = 50 (the headline size): the residual in the launch configuration the
  bench times (autotuned tile), every precision, against the stored oracle
  values of tests/golden/r50_ny_residual.json (sampled elements, block norms,
  ||R||^2; written by tests/golden/make_golden_ny.py, which calls only the
  oracle); and the identities that hold at any size, E1 - E0 = -eps ||R||^2
  and Tr U = 0 per block.
* r = 96 (the largest r): a closed-shell determinant has 2Delta = 0, so the
  NY residual equals the closed form of the Valdemoro one.
* FP32 and split-BF16 block products (the combination FP64) at the bars of
  the Valdemoro mixed modes, 1e-5 and 5e-5 of the largest element, on the
  residual and on the step's update; the int8 exact-accumulation products at
  the FP64 bar (residual, share, step; r = 50 stored values).
* The batched residual with the NY 3-RDM (instances of r = 6, 9, 13 in one
  call) against the oracle per instance.
* Rejected combinations: an explicit sigma array in a batch, sigma entries
  other than +1 / -1; above r = 64 the adjoint, the quadratic control and the
  spin-block path (their spin-orbital tensors).
* Edges: r = 2 and 3; the step with the active-active mask on the
  general-size kernels; the update map on an anti-Hermitian direction that is
  not a residual; the backtracking control (rejected trials) with the input
  symmetry check on.
"""
import json
import os

import numpy as np
import pytest

import determinant_forms as dform
from oracle import rdm
from oracle import solve as sv
from oracle import step as ost
from synth import generators as gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def acse():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2604_02550_amd as acse
    return acse


def correlated(r, N, seed, scale=0.05):
    """A generated problem with a larger 2-cumulant (the NY share is quadratic in it)."""
    p = gen.problem(r, N, 8, seed=seed)
    extra = gen.symmetric_direction(np.random.default_rng(seed + 100), r, scale=scale)
    p["d2aa"] = p["d2aa"] + extra["d2aa"]
    p["d2ab"] = p["d2ab"] + extra["d2ab"]
    return p


def sigma_of(p, pattern):
    if pattern == "prefix":
        return np.where(np.arange(p["r"]) < p["N"] // 2, 1.0, -1.0)
    return np.array(pattern, dtype=float)


CASES = [(4, 4, 0, "prefix"), (4, 4, 1, (-1, 1, -1, 1)), (9, 8, 2, "prefix"),
         (9, 8, 3, (1, -1, 1, 1, -1, 1, -1, -1, 1)), (16, 10, 4, "prefix"), (24, 14, 6, "prefix")]


@pytest.mark.parametrize("r,N,seed,pattern", CASES)
def test_ny_residual_matches_oracle(acse, r, N, seed, pattern):
    p = correlated(r, N, seed)
    sig = sigma_of(p, pattern)
    print(f"[ny] residual r={r} N={N} seed={seed} sigma={pattern}", flush=True)
    oaa, oab, on2 = ost.residual(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"], sigma=sig)
    vaa, vab, _ = ost.residual(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"])
    ctx = acse.Context(r_max=r)
    try:
        arg = True if pattern == "prefix" else [int(x) for x in sig]
        Raa, Rab, n2 = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2, sigma=arg)
        Vaa, Vab, _ = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2)
        Raa, Rab, Vaa, Vab = (x.cpu().numpy() for x in (Raa, Rab, Vaa, Vab))
    finally:
        ctx.close()
    scale = max(np.abs(oaa).max(), np.abs(oab).max())
    assert np.abs(Raa - oaa).max() <= 1e-10 * scale
    assert np.abs(Rab - oab).max() <= 1e-10 * scale
    assert abs(n2 - on2) <= 1e-10 * on2
    share = max(np.abs(oaa - vaa).max(), np.abs(oab - vab).max())
    assert share > 1e-4 * scale
    assert np.abs((Raa - Vaa) - (oaa - vaa)).max() <= 1e-9 * share
    assert np.abs((Rab - Vab) - (oab - vab)).max() <= 1e-9 * share


def test_ny_step_matches_oracle(acse):
    r, N = 9, 8
    p = correlated(r, N, 5)
    sig = sigma_of(p, "prefix")
    print(f"[ny] step r={r}", flush=True)
    o = ost.step(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"], 1e-3, sigma=sig)
    ctx = acse.Context(r_max=r)
    try:
        g = ctx.step(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2, eps=1e-3, return_ru=True,
                     sigma=True)
        for key in ("R_aa", "R_ab", "U_aa", "U_ab", "d2aa", "d2ab"):
            x = g[key].cpu().numpy()
            assert np.abs(x - o[key]).max() <= 1e-10 * np.abs(o[key]).max(), key
        assert np.abs(g["d1"].cpu().numpy() - o["gamma"]).max() <= 1e-10 * np.abs(o["gamma"]).max()
        assert abs(g["energy"] - o["energy"]) <= 1e-12 * abs(o["energy"])
        assert abs(g["norm2"] - o["norm2"]) <= 1e-10 * o["norm2"]
    finally:
        ctx.close()


def test_ny_solve_matches_oracle(acse):
    r, N = 6, 4
    p = gen.problem(r, N, 12, seed=1)
    _, d2 = rdm.blocks_to_spin_orbital(np.eye(r), p["d2aa"], p["d2ab"])
    p["gamma"] = rdm.contract_to_1rdm(d2, N)[:r, :r]
    sig = sigma_of(p, "prefix")
    print(f"[ny] solve r={r}", flush=True)
    o = sv.euler(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"], eps=1e-3, de_tol=1e-9, max_iter=3,
                 control=sv.FIXED, sigma=sig)
    ctx = acse.Context(r_max=r)
    try:
        g = ctx.solve(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2, eps=1e-3, de_tol=1e-9,
                      max_iter=3, control="fixed", sigma=True)
    finally:
        ctx.close()
    assert g["iterations"] == o["iterations"] and len(g["trials"]) == len(o["trials"])
    for (ge, gE, gf, gn, ga), (oe, oE, of, on, oa) in zip(g["trials"], o["trials"]):
        assert gn == on and ga == oa and ge == oe
        assert abs(gE - oE) <= 1e-10 * max(1.0, abs(oE))
        assert abs(gf - of) <= 1e-10 * of
    for key in ("d2aa", "d2ab"):
        assert np.abs(g[key].cpu().numpy() - o[key]).max() <= 1e-10 * np.abs(o[key]).max(), key


def test_ny_r50_identities(acse):
    p = gen.named("r50")
    r, N = p["r"], p["N"]
    eps = 1e-3
    print(f"[ny] r={r} identities", flush=True)
    ctx = acse.Context(r_max=r)
    try:
        E0 = ctx.energy(p["h"], p["V"], p["d2aa"], p["d2ab"], N // 2)
        Vaa, Vab, _ = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2)
        out = ctx.step(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2, eps=eps, return_ru=True,
                       sigma=True)
        n2 = out["norm2"]
        assert abs((out["energy"] - E0) + eps * n2) <= 1e-9 * eps * n2
        for Ub in (out["U_aa"], out["U_ab"]):
            umax = float(Ub.abs().max())
            tr = float(Ub.reshape(r * r, r * r).diagonal().sum())
            assert abs(tr) <= 1e-12 * umax * r * r
        share = max(float((out["R_aa"] - Vaa).abs().max()), float((out["R_ab"] - Vab).abs().max()))
        assert share > 1e-8 * float(out["R_ab"].abs().max())
    finally:
        ctx.close()


def test_ny_r96_determinant(acse):
    r, na = 96, 29
    print(f"[ny] r={r} closed-shell determinant", flush=True)
    rng = np.random.default_rng(7)
    h, V = gen.hamiltonian(rng, r, 96)
    g, d2aa, d2ab = dform.rdms(r, na)
    caa, cab = dform.residual_blocks(h, V, na)
    U = gen.haar_orthogonal(rng, r)
    rot = dform.rot4
    inputs = (dform.rot2(h, U), rot(V, U), dform.rot2(g, U), rot(d2aa, U), rot(d2ab, U))
    del V, d2aa, d2ab
    exp_aa, exp_ab = rot(caa, U), rot(cab, U)
    del caa, cab
    ctx = acse.Context(r_max=r)
    try:
        Raa, Rab, _ = ctx.residual(*inputs, na, sigma=True)
        scale = max(np.abs(exp_aa).max(), np.abs(exp_ab).max())
        assert np.abs(Raa.cpu().numpy() - exp_aa).max() <= 1e-10 * scale
        assert np.abs(Rab.cpu().numpy() - exp_ab).max() <= 1e-10 * scale
        # the NY adjoint, the quadratic control with NY and the spin-block NY
        # share run their spin-orbital tensors up to r = 64
        with pytest.raises(acse.AcseError, match="UNSUPPORTED"):
            ctx.residual_vjp(*inputs, na, Raa, Rab, sigma=True)
        with pytest.raises(acse.AcseError, match="UNSUPPORTED"):
            ctx.solve(*inputs, na, control="quadratic", sigma=True, max_iter=1)
        with pytest.raises(acse.AcseError, match="UNSUPPORTED"):
            ctx.residual_spin(inputs[0], inputs[1], inputs[2], inputs[2], inputs[3], inputs[3], inputs[4], na,
                              na, sigma=True)
    finally:
        ctx.close()


def test_ny_rejected_combinations(acse):
    import torch
    p = correlated(4, 4, 0)
    ctx = acse.Context(r_max=4)
    z = [torch.zeros((4, 4, 4, 4), dtype=torch.float64, device="cuda") for _ in range(5)]
    try:
        with pytest.raises(acse.AcseError, match="ny_sigma"):
            ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], 2, sigma=[1, 0, -1, -1])
        bp, bkeep = ctx.problem(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], 2)
        with pytest.raises(acse.AcseError, match="ny_sigma must be NULL"):
            ctx.residual_batched_raw([bp], ctx.options("fp64", sigma=[1, 1, -1, -1]), [z[0]], [z[1]])
        # the Valdemoro path is unaffected afterwards
        Raa, Rab, n2 = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], 2)
        o = ost.residual(p["h"], p["V"], 4, p["gamma"], p["d2aa"], p["d2ab"])
        assert abs(n2 - o[2]) <= 1e-10 * o[2]
    finally:
        ctx.close()


@pytest.mark.parametrize("r,N", [(2, 2), (3, 4)])
def test_ny_smallest_sizes(acse, r, N):
    p = correlated(r, N, 20 + r)
    sig = sigma_of(p, "prefix")
    print(f"[ny] residual r={r} N={N}", flush=True)
    oaa, oab, on2 = ost.residual(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"], sigma=sig)
    ctx = acse.Context(r_max=r)
    try:
        Raa, Rab, n2 = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2, sigma=True)
    finally:
        ctx.close()
    scale = max(np.abs(oaa).max(), np.abs(oab).max())
    assert np.abs(Raa.cpu().numpy() - oaa).max() <= 1e-10 * scale
    assert np.abs(Rab.cpu().numpy() - oab).max() <= 1e-10 * scale
    assert abs(n2 - on2) <= 1e-10 * on2


def test_ny_step_active_mask_and_general_kernels(acse):
    """The NY step with the active-active mask, on the general-size kernels
    (the one-index transforms, stored G2, row-chunked assembly), against the
    oracle step with the same mask."""
    r, N = 10, 8
    p = correlated(r, N, 31)
    sig = np.array([1, -1, 1, 1, -1, 1, -1, 1, -1, -1], dtype=float)
    act = np.zeros(r, bool)
    act[2:7] = True
    print(f"[ny] step r={r} active={act.astype(int).tolist()} general kernels", flush=True)
    o = ost.step(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"], 1e-3, active=act, sigma=sig)
    ctx = acse.Context(r_max=r)
    try:
        g = ctx.step(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2, eps=1e-3, return_ru=True,
                     active=act, flags=acse.FLAG_GENERAL_KERNELS, sigma=[int(x) for x in sig])
        for key in ("R_aa", "R_ab", "U_aa", "U_ab", "d2aa", "d2ab"):
            x = g[key].cpu().numpy()
            assert np.abs(x - o[key]).max() <= 1e-10 * np.abs(o[key]).max(), key
        assert abs(g["energy"] - o["energy"]) <= 1e-12 * abs(o["energy"])
    finally:
        ctx.close()


def test_ny_update_map_random_x(acse):
    """acse_update_map with the NY 3-RDM on an anti-Hermitian direction that is
    not a residual (X_aa antisymmetric in each pair, both blocks pair-exchange
    symmetric and anti-Hermitian), against the oracle's anti-Hermitian branch."""
    import torch
    from oracle import residual as rs
    r, N = 7, 6
    p = correlated(r, N, 41)
    sig = sigma_of(p, "prefix")
    rng = np.random.default_rng(42)
    x = rng.normal(size=(r, r, r, r))
    xaa = x - x.transpose(1, 0, 2, 3) - x.transpose(0, 1, 3, 2) + x.transpose(1, 0, 3, 2)
    xaa = xaa - xaa.transpose(2, 3, 0, 1)
    x = rng.normal(size=(r, r, r, r))
    xab = x + x.transpose(1, 0, 3, 2)
    xab = xab - xab.transpose(2, 3, 0, 1)
    print(f"[ny] update map r={r}", flush=True)
    d1, d2 = rdm.blocks_to_spin_orbital(p["gamma"], p["d2aa"], p["d2ab"])
    _, Xso = rdm.blocks_to_spin_orbital(np.eye(r), xaa, xab)
    U = rs.residual_map(Xso, d1, d2, hermitian=False, sigma_so=rdm.sigma_spin_orbital(sig)).numpy()
    uaa, uab = rdm.spin_orbital_to_blocks(U)
    ctx = acse.Context(r_max=r)
    try:
        gaa, gab = ctx.update_map(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2,
                                  torch.from_numpy(xaa), torch.from_numpy(xab), sigma=True)
    finally:
        ctx.close()
    scale = max(np.abs(uaa).max(), np.abs(uab).max())
    assert np.abs(gaa.cpu().numpy() - uaa).max() <= 1e-10 * scale
    assert np.abs(gab.cpu().numpy() - uab).max() <= 1e-10 * scale


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16x3", 5e-5)])
def test_ny_mixed_precision(acse, precision, tol):
    r, N = 16, 10
    p = correlated(r, N, 51)
    sig = sigma_of(p, "prefix")
    print(f"[ny] step r={r} precision={precision}", flush=True)
    o = ost.step(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"], 1e-3, sigma=sig)
    ctx = acse.Context(r_max=r)
    try:
        g = ctx.step(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2, eps=1e-3, return_ru=True,
                     precision=precision, sigma=True)
        for key in ("R_aa", "R_ab", "U_aa", "U_ab"):
            x = g[key].cpu().numpy()
            assert np.abs(x - o[key]).max() <= tol * np.abs(o[key]).max(), key
        assert abs(g["norm2"] - o["norm2"]) <= tol * o["norm2"]
        # the share itself at the same relative bar
        vaa, vab, _ = ost.residual(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"])
        share = max(np.abs(o["R_aa"] - vaa).max(), np.abs(o["R_ab"] - vab).max())
        Vaa, Vab, _ = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2, precision=precision)
        got = max(np.abs((g["R_aa"] - Vaa).cpu().numpy() - (o["R_aa"] - vaa)).max(),
                  np.abs((g["R_ab"] - Vab).cpu().numpy() - (o["R_ab"] - vab)).max())
        assert got <= 10 * tol * share
    finally:
        ctx.close()


@pytest.mark.parametrize("r,N,seed,pattern", [CASES[1], CASES[3], CASES[5]])
def test_ny_int8crt_residual_and_step(acse, r, N, seed, pattern):
    """The int8 exact-accumulation products in the NY share (and the
    Valdemoro part) at the FP64 bar: residual and share against the oracle,
    one step's R, U, new 2-RDM and energy."""
    p = correlated(r, N, seed)
    sig = sigma_of(p, pattern)
    print(f"[ny int8crt] r={r} N={N} sigma={pattern}", flush=True)
    oaa, oab, on2 = ost.residual(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"], sigma=sig)
    vaa, vab, _ = ost.residual(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"])
    o = ost.step(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"], 1e-3, sigma=sig)
    ctx = acse.Context(r_max=r)
    try:
        arg = True if pattern == "prefix" else [int(x) for x in sig]
        args = (p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2)
        Raa, Rab, n2 = ctx.residual(*args, precision="int8crt", sigma=arg)
        Vaa, Vab, _ = ctx.residual(*args, precision="int8crt")
        Raa, Rab, Vaa, Vab = (x.cpu().numpy() for x in (Raa, Rab, Vaa, Vab))
        g = ctx.step(*args, eps=1e-3, return_ru=True, precision="int8crt", sigma=arg)
        for key in ("R_aa", "R_ab", "U_aa", "U_ab", "d2aa", "d2ab"):
            x = g[key].cpu().numpy()
            assert np.abs(x - o[key]).max() <= 1e-10 * np.abs(o[key]).max(), key
        assert abs(g["energy"] - o["energy"]) <= 1e-12 * abs(o["energy"])
    finally:
        ctx.close()
    scale = max(np.abs(oaa).max(), np.abs(oab).max())
    assert np.abs(Raa - oaa).max() <= 1e-10 * scale and np.abs(Rab - oab).max() <= 1e-10 * scale
    assert abs(n2 - on2) <= 1e-10 * on2
    share = max(np.abs(oaa - vaa).max(), np.abs(oab - vab).max())
    assert np.abs((Raa - Vaa) - (oaa - vaa)).max() <= 1e-9 * share
    assert np.abs((Rab - Vab) - (oab - vab)).max() <= 1e-9 * share


GOLDEN_NY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "r50_ny_residual.json")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5), ("bf16x3", 5e-5), ("int8crt", 1e-10)])
def test_ny_r50_residual_vs_stored_oracle(acse, precision, tol):
    g = json.load(open(GOLDEN_NY))
    p = gen.named(g["workload"])
    r, N = p["r"], p["N"]
    assert r == g["r"] == 50 and N == g["N"]
    print(f"[ny] r=50 residual vs stored oracle, precision={precision}", flush=True)
    ctx = acse.Context(r_max=r)
    try:
        prob, _ = ctx.problem(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2)
        ctx.autotune_raw(prob, ctx.options(precision))
        Raa, Rab, n2 = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2,
                                    precision=precision, sigma=True)
        idx = tuple(np.array(g["index"]).T)
        for key, got in (("R_aa", Raa), ("R_ab", Rab)):
            ref = np.array(g["samples"][key])
            x = got.cpu().numpy()
            assert np.abs(x[idx] - ref).max() <= tol * np.abs(ref).max(), key
            assert abs(float(np.linalg.norm(x)) - g["norms"][key]) <= tol * g["norms"][key], key
        assert abs(n2 - g["norm2"]) <= tol * g["norm2"]
    finally:
        ctx.close()


def test_ny_backtracking_solve_and_input_check(acse):
    """The backtracking control with the NY 3-RDM (a step size that overshoots
    first) against the oracle's iteration, with the input-symmetry check on."""
    r, N = 6, 4
    p = gen.problem(r, N, 12, seed=1)
    _, d2 = rdm.blocks_to_spin_orbital(np.eye(r), p["d2aa"], p["d2ab"])
    p["gamma"] = rdm.contract_to_1rdm(d2, N)[:r, :r]
    sig = np.array([1, -1, 1, -1, -1, 1], dtype=float)
    print(f"[ny] backtracking solve r={r}", flush=True)
    o = sv.euler(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"], eps=0.1, de_tol=0.0, max_iter=3,
                 control=sv.BACKTRACK, max_halvings=12, sigma=sig)
    assert any(not t[4] for t in o["trials"])  # at least one rejected trial
    ctx = acse.Context(r_max=r)
    try:
        g = ctx.solve(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2, eps=0.1, de_tol=0.0, max_iter=3,
                      control="backtrack", max_halvings=12, flags=acse.FLAG_CHECK_INPUTS,
                      sigma=[int(x) for x in sig])
    finally:
        ctx.close()
    assert g["stop"] == ("max_iter", "converged", "energy_rose", "norm_rose")[o["stop"]]
    assert len(g["trials"]) == len(o["trials"])
    for (ge, gE, gf, gn, ga), (oe, oE, of, on, oa) in zip(g["trials"], o["trials"]):
        assert gn == on and ga == oa and ge == oe
        assert abs(gE - oE) <= 1e-10 * max(1.0, abs(oE))
        assert abs(gf - of) <= 1e-10 * of
    for key in ("d2aa", "d2ab"):
        assert np.abs(g[key].cpu().numpy() - o[key]).max() <= 1e-10 * np.abs(o[key]).max(), key


def test_ny_batched_residual(acse):
    insts = [correlated(6, 4, 61), correlated(9, 8, 62), correlated(13, 8, 63)]
    print("[ny] batched residual r=6,9,13", flush=True)
    ctx = acse.Context(r_max=13)
    try:
        got = ctx.residual_batched(insts, ny=True)
        plain = ctx.residual_batched(insts)
    finally:
        ctx.close()
    for q, (Raa, Rab, n2), (Vaa, Vab, _) in zip(insts, got, plain):
        sig = sigma_of(q, "prefix")
        oaa, oab, on2 = ost.residual(q["h"], q["V"], q["N"], q["gamma"], q["d2aa"], q["d2ab"], sigma=sig)
        scale = max(np.abs(oaa).max(), np.abs(oab).max())
        assert np.abs(Raa.cpu().numpy() - oaa).max() <= 1e-10 * scale
        assert np.abs(Rab.cpu().numpy() - oab).max() <= 1e-10 * scale
        assert abs(n2 - on2) <= 1e-10 * on2
        assert np.abs((Raa - Vaa).cpu().numpy()).max() > 1e-6 * scale  # the NY share is there


@pytest.mark.parametrize("tile", [0, 1, 2])
def test_ny_every_tile_config(acse, tile):
    """acse_options.tile selects the tile configuration of the NY block
    products as of the Valdemoro ones."""
    r, N = 13, 8
    p = correlated(r, N, 71)
    sig = sigma_of(p, "prefix")
    print(f"[ny] residual r={r} tile={tile}", flush=True)
    oaa, oab, on2 = ost.residual(p["h"], p["V"], N, p["gamma"], p["d2aa"], p["d2ab"], sigma=sig)
    ctx = acse.Context(r_max=r)
    try:
        Raa, Rab, n2 = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2, tile=tile, sigma=True)
    finally:
        ctx.close()
    scale = max(np.abs(oaa).max(), np.abs(oab).max())
    assert np.abs(Raa.cpu().numpy() - oaa).max() <= 1e-10 * scale
    assert np.abs(Rab.cpu().numpy() - oab).max() <= 1e-10 * scale
    assert abs(n2 - on2) <= 1e-10 * on2
