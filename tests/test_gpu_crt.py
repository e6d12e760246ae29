"""The int8 exact-accumulation products (precision "int8crt") against the FP64
oracle through the C ABI.

The products are exact up to the rounding of each operand to k-bit integers
relative to its row's largest magnitude (k = 44 at K = 2500 with the default 13
moduli, more at smaller K), so the FP64 bar of the other parity tests applies:
normwise and max-elementwise relative error <= 1e-10 for every array.  The
modulus count is checked to matter: with fewer moduli (fewer bits per operand)
the error grows as 2^-k.
"""
import numpy as np
import pytest

from oracle import fermion as fm
from oracle import step as ost
from synth import generators as gen

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def acse():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2604_02550_amd as acse
    return acse


@pytest.fixture(scope="module")
def ctx(acse):
    return acse.Context(r_max=32)


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - b).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))


def maxrel(a, b):
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


def cpu(t):
    return t.detach().cpu().numpy()


def tiny():
    rng = np.random.default_rng(0)
    h, V = gen.hamiltonian(rng, 4, 6)
    p = fm.fci_singlet_problem(h, V, 4)
    return dict(r=4, N=4, h=h, V=V, gamma=p["gamma"], d2aa=p["d2aa"], d2ab=p["d2ab"])


PROBLEMS = {
    "tiny_fci": tiny,
    "r6": lambda: gen.problem(6, 4, 12, seed=1),
    "r13": lambda: gen.problem(13, 8, 26, seed=3),
    "r23": lambda: gen.problem(23, 14, 46, seed=4),
}


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_crt_residual_and_step(ctx, name):
    p = PROBLEMS[name]()
    na = p["N"] // 2
    print(f"[crt] {name} r={p['r']}", flush=True)
    raa, rab, n2 = ost.residual(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"])
    Raa, Rab, gn2 = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], na, precision="int8crt")
    for got, ref in ((Raa, raa), (Rab, rab)):
        assert rel(cpu(got), ref) < TOL and maxrel(cpu(got), ref) < TOL
    assert abs(gn2 - n2) <= TOL * n2
    o = ost.step(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], 1e-3)
    g = ctx.step(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], na, eps=1e-3, precision="int8crt",
                 return_ru=True)
    for key in ("R_aa", "R_ab", "U_aa", "U_ab", "d2aa", "d2ab"):
        assert rel(cpu(g[key]), o[key]) < TOL, key
        assert maxrel(cpu(g[key]), o[key]) < TOL, key
    assert maxrel(cpu(g["d1"]), o["gamma"]) < TOL
    assert abs(g["energy"] - o["energy"]) <= TOL * max(1.0, abs(o["energy"]))


@pytest.fixture(scope="module")
def r30():
    p = gen.named("r30")
    return p, ost.step(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], 1e-3)


def test_crt_r30_step(ctx, r30):
    """The r = 30, N = 20 workload: every array at the FP64 bar, and the energy
    after the step within 1e-9 Eh (the step moves it by ~1e3 Eh)."""
    p, o = r30
    print("[crt] r30 step", flush=True)
    g = ctx.step(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2, eps=1e-3,
                 precision="int8crt", return_ru=True)
    for key in ("R_aa", "R_ab", "U_aa", "U_ab", "d2aa", "d2ab"):
        assert rel(cpu(g[key]), o[key]) < TOL, key
        assert maxrel(cpu(g[key]), o[key]) < TOL, key
    dE = abs(g["energy"] - o["energy"])
    print(f"[crt] r30 |dE| = {dE:.3e} Eh (step {abs(o['energy'] - o['energy0']):.3e} Eh)", flush=True)
    assert dE < 1e-9
    assert abs(g["norm2"] - o["norm2"]) <= TOL * o["norm2"]


def test_crt_moduli_count_sets_the_accuracy(ctx):
    """Error against the oracle as the modulus count grows (8 .. 15 moduli:
    about 25 .. 51 bits per operand at this K): it falls, roughly by 2^-4 per
    extra modulus until the FP64 floor, and the default count meets the FP64 bar."""
    p = PROBLEMS["r13"]()
    raa, rab, _ = ost.residual(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"])
    errs = {}
    for nm in (8, 9, 10, 11, 12, 13, 15):
        Raa, Rab, _ = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2,
                                   precision="int8crt", moduli=nm)
        errs[nm] = max(rel(cpu(Raa), raa), rel(cpu(Rab), rab))
    print(f"[crt] r13 normwise error by modulus count: {errs}", flush=True)
    assert errs[8] > 1e-9             # few bits: the operand rounding shows
    for a, b in ((8, 10), (10, 12)):
        assert errs[b] < errs[a] / 20
    assert errs[13] < 1e-12 and errs[15] < 1e-12
    # the default (0) is 13 moduli
    Raa, Rab, _ = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2,
                               precision="int8crt")
    R13, _, _ = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2,
                             precision="int8crt", moduli=13)
    import torch
    assert torch.equal(Raa, R13)


@pytest.mark.parametrize("r,N", [(2, 2), (3, 6), (5, 10)])
def test_crt_edge_sizes(ctx, r, N):
    """Smallest sizes (one pair at r = 2, whose alpha-alpha residual is zero),
    every orbital doubly occupied."""
    p = gen.problem(r, N, 2 * r, seed=40 + r + N)
    print(f"[crt] edge r={r} N={N}", flush=True)
    o = ost.step(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], 1e-3)
    g = ctx.step(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2, eps=1e-3,
                 precision="int8crt", return_ru=True)
    for pair in (("R_aa", "R_ab"), ("U_aa", "U_ab"), ("d2aa", "d2ab")):
        scale = max(np.abs(o[k]).max() for k in pair)
        for key in pair:
            assert np.abs(cpu(g[key]) - o[key]).max() <= TOL * scale, key
    assert abs(g["energy"] - o["energy"]) <= TOL * max(1.0, abs(o["energy"]))


def test_crt_general_kernels_and_mask(acse, ctx):
    """With the general-size kernels (their FP64 operand writers feed the
    conversion) and a scattered active mask."""
    p = PROBLEMS["r13"]()
    act = np.zeros(13, bool)
    act[[0, 3, 4, 9]] = True
    o = ost.step(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], 1e-3, active=act)
    g = ctx.step(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2, eps=1e-3, active=act,
                 precision="int8crt", return_ru=True, flags=acse.FLAG_GENERAL_KERNELS)
    for key in ("R_aa", "R_ab", "U_aa", "U_ab", "d2aa", "d2ab"):
        assert rel(cpu(g[key]), o[key]) < TOL and maxrel(cpu(g[key]), o[key]) < TOL, key


def test_crt_deterministic_and_solve(acse, ctx):
    import torch
    p = PROBLEMS["r13"]()
    args = (p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2)
    a = ctx.residual(*args, precision="int8crt")
    b = ctx.residual(*args, precision="int8crt")
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2] == b[2]
    # the Euler iteration with the backtracking control takes the FP64 path's decisions
    r64 = ctx.solve(*args, eps=0.05, de_tol=0.0, max_iter=3, control="backtrack")
    rc = ctx.solve(*args, eps=0.05, de_tol=0.0, max_iter=3, control="backtrack", precision="int8crt")
    assert [t[4] for t in rc["trials"]] == [t[4] for t in r64["trials"]]
    for t1, t2 in zip(rc["trials"], r64["trials"]):
        assert abs(t1[1] - t2[1]) <= 1e-10 * abs(t2[1]) and abs(t1[2] - t2[2]) <= 1e-9 * t2[2]


def test_crt_quadratic_solve_takes_the_fp64_decisions(ctx):
    """The quadratic control in the int8 mode (its slope from the int8
    adjoint): the FP64 path's trials, decisions and second step sizes."""
    p = gen.problem(10, 6, 20, seed=2)
    # start from the 1-RDM contracted from the 2-RDM (an eps = 0 step)
    s0 = ctx.step(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], 3, eps=0.0)
    args = (p["h"], p["V"], cpu(s0["d1"]), cpu(s0["d2aa"]), cpu(s0["d2ab"]), 3)
    print("[crt] r10 quadratic solve", flush=True)
    r64 = ctx.solve(*args, eps=1e-3, de_tol=0.0, max_iter=5, control="quadratic")
    rc = ctx.solve(*args, eps=1e-3, de_tol=0.0, max_iter=5, control="quadratic", precision="int8crt")
    assert r64["iterations"] >= 3
    assert rc["stop"] == r64["stop"] and rc["iterations"] == r64["iterations"] and rc["maps"] == r64["maps"]
    assert [t[3:] for t in rc["trials"]] == [t[3:] for t in r64["trials"]]
    for t1, t2 in zip(rc["trials"], r64["trials"]):
        assert abs(t1[0] - t2[0]) <= 1e-8 * abs(t2[0])
        assert abs(t1[1] - t2[1]) <= 1e-9 * abs(t2[1]) and abs(t1[2] - t2[2]) <= 1e-8 * t2[2]


def test_crt_unsupported_combinations(acse, ctx):
    import torch
    p = PROBLEMS["r6"]()
    args = (p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2)
    inst = [dict(h=p["h"], V=p["V"], N=p["N"], gamma=p["gamma"], d2aa=p["d2aa"], d2ab=p["d2ab"])]
    with pytest.raises(acse.AcseError, match="UNSUPPORTED"):
        ctx.residual_batched(inst, precision="int8crt", flags=acse.FLAG_BATCH_PERSISTENT)
    with pytest.raises(acse.AcseError, match="UNSUPPORTED"):
        acse.residual_noalloc(*args, precision="int8crt")
    for bad in (7, 16, -1):
        with pytest.raises(acse.AcseError, match="moduli"):
            ctx.residual(*args, precision="int8crt", moduli=bad)
