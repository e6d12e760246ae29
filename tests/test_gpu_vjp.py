"""GPU parity of the hand-written adjoints (acse_residual_vjp, acse_energy_vjp).

* FP64 against the oracle adjoint (autograd of the oracle forward, projected)
  at r = 4 (FCI RDMs), 6, 10 and 13: relative 1e-10 per gradient.
* r = 30, N = 20 (the differentiation workload): central finite differences
  (step 1e-5) of the oracle's FP64 forward along one structured direction per
  input, against <gradient, direction>, FP64 and FP32.
* FP32 / split-BF16 contractions against the FP64 oracle adjoint, stated
  per-gradient tolerances; int8 exact-accumulation products at the FP64 bar
  (1e-10 against the oracle adjoint, the r = 30 finite differences at 1e-7).
* The torch.autograd.Function wrappers give the same gradients, and two calls
  are bitwise identical.
* With the NY 3-RDM (default and non-prefix occupations): FP64 and the int8
  products against the oracle's NY adjoint at 1e-10, and the autograd
  wrapper with sigma.
"""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import fermion as fm
from oracle import step as ost
from synth import generators as gen

pytestmark = pytest.mark.gpu

KEYS = ("h", "V", "gamma", "d2aa", "d2ab")
TOL64 = 1e-10
# normwise relative error of each gradient against the FP64 oracle adjoint
MIXED_TOL = {"fp32": 1e-5, "bf16x3": 5e-5}


@pytest.fixture(scope="module")
def acse():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2604_02550_amd as acse
    return acse


@pytest.fixture(scope="module")
def ctx(acse):
    return acse.Context(r_max=30)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def maxrel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def cpu(t):
    return t.detach().cpu().numpy()


def tiny_fci(seed=0):
    rng = np.random.default_rng(seed)
    h, V = gen.hamiltonian(rng, 4, 6)
    p = fm.fci_singlet_problem(h, V, 4)
    return dict(r=4, N=4, h=h, V=V, gamma=p["gamma"], d2aa=p["d2aa"], d2ab=p["d2ab"])


PROBLEMS = {
    "tiny_fci": lambda: tiny_fci(0),
    "r6": lambda: gen.problem(6, 4, 12, seed=1),
    "r10": lambda: gen.problem(10, 6, 20, seed=2),
    "r13": lambda: gen.problem(13, 8, 26, seed=3),
}


def gpu_vjp(ctx, p, Rb, precision="fp64", sigma=None):
    out = ctx.residual_vjp(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2,
                           Rb[0], Rb[1], precision=precision, sigma=sigma)
    return dict(zip(KEYS, [cpu(x) for x in out]))


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_residual_vjp_fp64_vs_oracle(ctx, name):
    p = PROBLEMS[name]()
    print(f"[residual_vjp_fp64] {name} r={p['r']}", flush=True)
    Rb = gen.cotangent(np.random.default_rng(21), p["r"])
    ref = adj.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], *Rb)
    got = gpu_vjp(ctx, p, Rb)
    for k in KEYS:
        assert rel(got[k], ref[k]) < TOL64, (k, rel(got[k], ref[k]))
        assert maxrel(got[k], ref[k]) < TOL64, (k, maxrel(got[k], ref[k]))


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_residual_vjp_int8crt_vs_oracle(ctx, name):
    """The adjoint with int8 exact-accumulation products: the FP64 bar
    against the oracle adjoint (operands rounded to k = 44+ bits, products
    exact)."""
    p = PROBLEMS[name]()
    print(f"[residual_vjp_int8crt] {name} r={p['r']}", flush=True)
    Rb = gen.cotangent(np.random.default_rng(22), p["r"])
    ref = adj.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], *Rb)
    got = gpu_vjp(ctx, p, Rb, "int8crt")
    for k in KEYS:
        assert rel(got[k], ref[k]) < TOL64, (k, rel(got[k], ref[k]))
        assert maxrel(got[k], ref[k]) < TOL64, (k, maxrel(got[k], ref[k]))


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32", 1e-5), ("bf16x3", 5e-5), ("int8crt", TOL64)])
def test_residual_vjp_general_kernels(acse, ctx, precision, tol):
    """The adjoint with the general-size kernels (ACSE_FLAG_GENERAL_KERNELS): the
    G2 kernel that stores G2, and the alpha-beta pp adjoint products packed
    over the pair-exchange symmetry (the form used from r = 40 on), in every
    precision of the contractions."""
    p = PROBLEMS["r13"]()
    print(f"[vjp_general] r13 {precision}", flush=True)
    Rb = gen.cotangent(np.random.default_rng(25), p["r"])
    ref = adj.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], *Rb)
    out = ctx.residual_vjp(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2, Rb[0], Rb[1],
                           precision=precision, flags=acse.FLAG_GENERAL_KERNELS)
    for k, x in zip(KEYS, out):
        assert rel(cpu(x), ref[k]) < tol, k


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_energy_vjp_fp64_vs_oracle(ctx, name):
    p = PROBLEMS[name]()
    ref = adj.energy_vjp(p["h"], p["V"], p["N"], p["d2aa"], p["d2ab"], Ebar=-1.3)
    got = ctx.energy_vjp(p["h"], p["V"], p["d2aa"], p["d2ab"], p["N"] // 2, Ebar=-1.3)
    for k, x in zip(("h", "V", "d2aa", "d2ab"), got):
        assert rel(cpu(x), ref[k]) < TOL64 and maxrel(cpu(x), ref[k]) < TOL64, k


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_residual_vjp_mixed_vs_oracle(ctx, precision):
    p = PROBLEMS["r13"]()
    Rb = gen.cotangent(np.random.default_rng(22), p["r"])
    ref = adj.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], *Rb)
    got = gpu_vjp(ctx, p, Rb, precision)
    for k in KEYS:
        e = rel(got[k], ref[k])
        print(f"[vjp {precision}] {k} rel {e:.2e}", flush=True)
        assert e < MIXED_TOL[precision], (k, e)


def oracle_loss(p, Rb, **over):
    q = {k: over.get(k, p[k]) for k in KEYS}
    raa, rab, _ = ost.residual(q["h"], q["V"], p["N"], q["gamma"], q["d2aa"], q["d2ab"])
    return float(np.sum(Rb[0] * raa) + np.sum(Rb[1] * rab))


@pytest.fixture(scope="module")
def vjp30():
    p = gen.named("vjp30")
    rng = np.random.default_rng(23)
    Rb = gen.cotangent(rng, p["r"])
    dirs = gen.symmetric_direction(rng, p["r"])
    t = 1e-5
    fd = {}
    for k in KEYS:
        print(f"[vjp30 fd] {k}", flush=True)
        fd[k] = (oracle_loss(p, Rb, **{k: p[k] + t * dirs[k]})
                 - oracle_loss(p, Rb, **{k: p[k] - t * dirs[k]})) / (2 * t)
    return p, Rb, dirs, fd


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-7), ("fp32", 1e-4), ("int8crt", 1e-7)])
def test_residual_vjp_r30_finite_difference(ctx, vjp30, precision, tol):
    p, Rb, dirs, fd = vjp30
    got = gpu_vjp(ctx, p, Rb, precision)
    for k in KEYS:
        an = float(np.sum(got[k] * dirs[k]))
        scale = max(abs(fd[k]), np.linalg.norm(got[k]))
        print(f"[vjp30 {precision}] {k} fd {fd[k]:.10e} an {an:.10e}", flush=True)
        assert abs(an - fd[k]) <= tol * scale, (k, an, fd[k])


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-7), ("fp32", 1e-4)])
def test_residual_vjp_r44_finite_difference(acse, precision, tol):
    """At r = 44 the alpha-beta pp adjoint products run packed (as from r = 40
    on): <gradient, direction> against central finite differences of
    <Rbar, R> along one structured direction per input, with R from the FP64
    residual on the GPU (itself checked against the oracle elsewhere)."""
    import torch
    p = gen.problem(44, 26, 88, seed=44)
    rng = np.random.default_rng(44)
    Rb = gen.cotangent(rng, p["r"])
    dirs = gen.symmetric_direction(rng, p["r"])
    ctx = acse.Context(r_max=p["r"])
    try:
        dev = ctx.device
        Rbt = [torch.as_tensor(a, device=dev) for a in Rb]

        def loss(**over):
            q = {k: over.get(k, p[k]) for k in KEYS}
            Raa, Rab, _ = ctx.residual(q["h"], q["V"], q["gamma"], q["d2aa"], q["d2ab"], p["N"] // 2)
            return float((Rbt[0] * Raa).sum() + (Rbt[1] * Rab).sum())

        got = gpu_vjp(ctx, p, Rb, precision)
        t = 1e-5
        for k in KEYS:
            fd = (loss(**{k: p[k] + t * dirs[k]}) - loss(**{k: p[k] - t * dirs[k]})) / (2 * t)
            an = float(np.sum(got[k] * dirs[k]))
            scale = max(abs(fd), np.linalg.norm(got[k]))
            print(f"[vjp44 {precision}] {k} fd {fd:.10e} an {an:.10e}", flush=True)
            assert abs(an - fd) <= tol * scale, (k, an, fd)
    finally:
        ctx.close()


def test_autograd_function_and_determinism(acse, ctx):
    import torch
    p = PROBLEMS["r10"]()
    dev = ctx.device
    x = [torch.tensor(p[k], device=dev, requires_grad=True) for k in KEYS]
    Rb = [torch.tensor(a, device=dev) for a in gen.cotangent(np.random.default_rng(24), p["r"])]
    Raa, Rab = acse.ACSEResidual.apply(ctx, *x, p["N"] // 2, "fp64")
    L = (Rb[0] * Raa).sum() + (Rb[1] * Rab).sum()
    L.backward()
    direct = ctx.residual_vjp(*[t.detach() for t in x], p["N"] // 2, Rb[0], Rb[1])
    again = ctx.residual_vjp(*[t.detach() for t in x], p["N"] // 2, Rb[0], Rb[1])
    for t, a, b in zip(x, direct, again):
        assert torch.equal(t.grad, a)
        assert torch.equal(a, b)
    # energy through its Function
    y = [torch.tensor(p[k], device=dev, requires_grad=True) for k in ("h", "V", "d2aa", "d2ab")]
    E = acse.ACSEEnergy.apply(ctx, *y, p["N"] // 2)
    assert abs(E.item() - ost.energy(p["h"], p["V"], p["N"], p["d2aa"], p["d2ab"])) < 1e-10 * abs(E.item())
    (2.0 * E).backward()
    ref = adj.energy_vjp(p["h"], p["V"], p["N"], p["d2aa"], p["d2ab"], Ebar=2.0)
    for t, k in zip(y, ("h", "V", "d2aa", "d2ab")):
        assert rel(cpu(t.grad), ref[k]) < TOL64, k


def test_vjp_argument_errors(acse, ctx):
    import torch
    p = PROBLEMS["r6"]()
    prob, keep = ctx.problem(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2)
    opts = ctx.options("fp64")
    out = [torch.empty_like(t) for t in keep]
    # the binding refuses a missing cotangent before the library sees it ...
    with pytest.raises(ValueError, match="Rbar_aa"):
        ctx.residual_vjp_raw(prob, opts, None, keep[3], *out)
    # ... and the library itself reports a NULL one
    import ctypes
    st = acse._lib.acse_residual_vjp(ctx._h, ctypes.byref(prob), ctypes.byref(opts), None,
                                     acse._ptr(keep[3]), *[acse._ptr(t) for t in out])
    assert st == 1   # ACSE_ERR_ARG
    with pytest.raises(acse.AcseError):
        ctx.energy_vjp_raw(prob, float("nan"), out[0], out[1], out[3], out[4])


def ny_sigma(p, kind):
    """Default occupations (orbitals below N/2) or a non-prefix pattern."""
    r, na = p["r"], p["N"] // 2
    if kind == "default":
        return [1 if q < na else -1 for q in range(r)]
    return [1 if (q * 7 + 3) % r < na else -1 for q in range(r)]


@pytest.mark.parametrize("kind", ["default", "scattered"])
@pytest.mark.parametrize("name", list(PROBLEMS))
def test_residual_vjp_ny_fp64_vs_oracle(ctx, name, kind):
    """The NY adjoint (the Valdemoro adjoint plus the NY share's, FP64 over
    spin-orbital tensors) against autograd of the oracle's NY residual."""
    p = PROBLEMS[name]()
    sig = ny_sigma(p, kind)
    print(f"[residual_vjp_ny] {name} r={p['r']} sigma={sig}", flush=True)
    Rb = gen.cotangent(np.random.default_rng(31), p["r"])
    ref = adj.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], *Rb, sigma=sig)
    got = gpu_vjp(ctx, p, Rb, sigma=sig if kind != "default" else True)
    for k in KEYS:
        assert rel(got[k], ref[k]) < TOL64, (k, rel(got[k], ref[k]))
        assert maxrel(got[k], ref[k]) < TOL64, (k, maxrel(got[k], ref[k]))
    # the NY share's adjoint is not zero here
    val = adj.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], *Rb)
    assert max(rel(val[k], ref[k]) for k in KEYS) > 1e-6


@pytest.mark.parametrize("r,N", [(2, 2), (3, 2), (3, 4)])
def test_residual_vjp_ny_smallest_sizes(ctx, r, N):
    """The NY adjoint at the smallest sizes (2r = 4 and 6 spin orbitals: one
    ragged tile in every spin-block product)."""
    p = gen.problem(r, N, 2 * r, seed=9)
    sig = [1 if q < N // 2 else -1 for q in range(r)]
    print(f"[residual_vjp_ny] r={r} N={N}", flush=True)
    Rb = gen.cotangent(np.random.default_rng(3), r)
    ref = adj.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], *Rb, sigma=sig)
    got = gpu_vjp(ctx, p, Rb, sigma=True)
    for k in KEYS:
        assert rel(got[k], ref[k]) < TOL64, (k, rel(got[k], ref[k]))
        assert maxrel(got[k], ref[k]) < TOL64, (k, maxrel(got[k], ref[k]))


@pytest.mark.parametrize("name", ["r6", "r10", "r13"])
def test_residual_vjp_ny_int8crt_vs_oracle(ctx, name):
    """The NY adjoint with int8 exact-accumulation products in both the
    Valdemoro part and the NY share's spin-orbital contractions, at the FP64 bar."""
    p = PROBLEMS[name]()
    sig = ny_sigma(p, "scattered")
    print(f"[residual_vjp_ny] {name} int8crt", flush=True)
    Rb = gen.cotangent(np.random.default_rng(32), p["r"])
    ref = adj.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], *Rb, sigma=sig)
    got = gpu_vjp(ctx, p, Rb, "int8crt", sigma=sig)
    for k in KEYS:
        assert rel(got[k], ref[k]) < TOL64, (k, rel(got[k], ref[k]))
        assert maxrel(got[k], ref[k]) < TOL64, (k, maxrel(got[k], ref[k]))


def test_autograd_function_ny(acse, ctx):
    import torch
    p = PROBLEMS["r6"]()
    sig = ny_sigma(p, "scattered")
    dev = ctx.device
    x = [torch.tensor(p[k], device=dev, requires_grad=True) for k in KEYS]
    Rb = [torch.tensor(a, device=dev) for a in gen.cotangent(np.random.default_rng(33), p["r"])]
    Raa, Rab = acse.ACSEResidual.apply(ctx, *x, p["N"] // 2, "fp64", sig)
    o = ost.residual(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], sigma=sig)
    assert np.abs(cpu(Raa) - o[0]).max() <= TOL64 * np.abs(o[0]).max()
    ((Rb[0] * Raa).sum() + (Rb[1] * Rab).sum()).backward()
    ref = adj.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], *[cpu(t) for t in Rb],
                           sigma=sig)
    for t, k in zip(x, KEYS):
        assert rel(cpu(t.grad), ref[k]) < TOL64, k


def test_residual_vjp_ny_r50_finite_difference(acse):
    """The NY adjoint at the size the bench times (r = 50, N = 30, default
    occupations): <gradient, direction> against central finite differences
    of <Rbar, R> along one structured direction per input, R from the NY
    residual on the GPU (itself checked against stored oracle values at this
    size in test_gpu_ny.py)."""
    import torch
    p = gen.named("r50")
    rng = np.random.default_rng(50)
    Rb = gen.cotangent(rng, p["r"])
    dirs = gen.symmetric_direction(rng, p["r"])
    ctx = acse.Context(r_max=p["r"])
    try:
        dev = ctx.device
        Rbt = [torch.as_tensor(a, device=dev) for a in Rb]

        def loss(**over):
            q = {k: over.get(k, p[k]) for k in KEYS}
            Raa, Rab, _ = ctx.residual(q["h"], q["V"], q["gamma"], q["d2aa"], q["d2ab"], p["N"] // 2, sigma=True)
            return float((Rbt[0] * Raa).sum() + (Rbt[1] * Rab).sum())

        print("[vjp50 ny] adjoint", flush=True)
        got = gpu_vjp(ctx, p, Rb, sigma=True)
        t = 1e-5
        for k in KEYS:
            fd = (loss(**{k: p[k] + t * dirs[k]}) - loss(**{k: p[k] - t * dirs[k]})) / (2 * t)
            an = float(np.sum(got[k] * dirs[k]))
            scale = max(abs(fd), np.linalg.norm(got[k]))
            print(f"[vjp50 ny] {k} fd {fd:.10e} an {an:.10e}", flush=True)
            assert abs(an - fd) <= 1e-7 * scale, (k, an, fd)
    finally:
        ctx.close()
