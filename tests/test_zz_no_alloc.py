"""acse_residual_noalloc: the residual with no context and no allocation (its
workspace is a fixed device array of the library, r <= 16), through the C ABI,
against acse_residual on the same inputs and against the FP64 oracle; calls in
a row on the shared array with the problem shrinking; errors beyond the
maximum size."""
import numpy as np
import pytest

from oracle import step as ost
from synth import generators as gen

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def maxrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def acse():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2604_02550_amd as acse
    return acse


def test_noalloc_equals_residual_with_shrinking_problems(acse):
    import torch
    ctx = acse.Context(r_max=16)
    stream = torch.cuda.Stream()   # a stream of the caller's, not the context's
    # the largest size first, then smaller ones: every later call finds the
    # previous call's contents in the shared array
    for r, N, seed in ((16, 10, 5), (13, 8, 3), (6, 4, 1)):
        p = gen.problem(r, N, 2 * r, seed=seed)
        args = (p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2)
        print(f"[noalloc] r={r} N={N}", flush=True)
        Raa, Rab, n2 = ctx.residual(*args)
        Gaa, Gab, g2 = acse.residual_noalloc(*args, stream=stream)
        torch.cuda.synchronize()
        # the same kernels and tile on the same inputs: bitwise equal
        assert torch.equal(Gaa, Raa) and torch.equal(Gab, Rab) and g2 == n2
        raa, rab, on2 = ost.residual(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"])
        for got, ref in ((Gaa, raa), (Gab, rab)):
            got = got.cpu().numpy()
            assert rel(got, ref) < TOL64 and maxrel(got, ref) < TOL64
        assert abs(g2 - on2) <= TOL64 * on2


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_noalloc_mixed_precision(acse, precision):
    import torch
    ctx = acse.Context(r_max=16)
    for r, N, seed in ((14, 8, 7), (9, 6, 2)):
        p = gen.problem(r, N, 2 * r, seed=seed)
        args = (p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], N // 2)
        print(f"[noalloc] {precision} r={r}", flush=True)
        Raa, Rab, n2 = ctx.residual(*args, precision=precision)
        Gaa, Gab, g2 = acse.residual_noalloc(*args, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(Gaa, Raa) and torch.equal(Gab, Rab) and g2 == n2


def test_noalloc_errors(acse):
    import torch
    p = gen.problem(17, 10, 34, seed=1)
    args = (p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], 5)
    with pytest.raises(acse.AcseError, match=r"outside \[2, 16\]"):
        acse.residual_noalloc(*args)
    q = gen.problem(6, 4, 12, seed=1)
    dev = torch.device("cuda", 0)
    t = [torch.as_tensor(q[k], device=dev).contiguous() for k in ("h", "V", "gamma", "d2aa", "d2ab")]
    prob = acse.Problem(6, 2, 2, *[x.data_ptr() for x in t])
    R = [torch.empty((6,) * 4, dtype=torch.float64, device=dev) for _ in range(2)]
    with pytest.raises(acse.AcseError, match="Valdemoro"):
        acse.residual_noalloc_raw(prob, acse.Context.options(sigma=True), R[0], R[1])
    bad = acse.Problem(6, 3, 2, *[x.data_ptr() for x in t])
    with pytest.raises(acse.AcseError, match="UNSUPPORTED"):
        acse.residual_noalloc_raw(bad, acse.Context.options(), R[0], R[1])
