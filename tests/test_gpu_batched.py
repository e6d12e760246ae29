"""GPU tests of the batched residual (acse_residual_batched): instances of
uneven r, each on its own side-stream lane (default) or with all products in
one persistent launch (ACSE_FLAG_BATCH_PERSISTENT).  Both strategies:

* A small mixed batch (r = 5, 6, 9, 13; ground and pinned excited states)
  against the FP64 oracle, 1e-10.
* The 12-instance workload (r in {20, 28, 36, 44}, 3 states each): every
  instance bitwise equal to its own single acse_residual call with the same
  tile configuration, and the r = 20 and r = 28 instances against the oracle.
* FP32 contractions against the FP64 oracle (stated tolerance).
* The batch autotuner, workspace reuse with a smaller second batch, and
  argument errors that name the failing instance.
"""
import numpy as np
import pytest

from oracle import step as ost
from synth import generators as gen

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-5


@pytest.fixture(scope="module")
def acse():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2604_02550_amd as acse
    return acse


@pytest.fixture(scope="module")
def ctx(acse):
    return acse.Context(r_max=44)


@pytest.fixture(scope="module")
def big_batch():
    return gen.batched_problems(seed=0)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def cpu(t):
    return t.detach().cpu().numpy()


def small_batch():
    out = []
    for r, N, seed in ((5, 4, 1), (6, 4, 2), (9, 6, 3), (13, 8, 4)):
        out.append(gen.problem(r, N, 2 * r, seed=seed))
        out.append(gen.problem(r, N, 2 * r, seed=seed + 100, pinned=(N // 2 - 1, N // 2)))
    return out


def check_oracle(p, Raa, Rab, n2, tol):
    raa, rab, rn2 = ost.residual(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"])
    assert rel(cpu(Raa), raa) < tol and rel(cpu(Rab), rab) < tol
    assert abs(n2 - rn2) <= tol * rn2


STRATEGIES = {"lanes": 0, "persistent": 4}


@pytest.mark.parametrize("strategy", list(STRATEGIES))
@pytest.mark.parametrize("tile", [-1, 0, 1, 2])
def test_small_batch_vs_oracle(ctx, tile, strategy):
    batch = small_batch()
    print(f"[batched small] {strategy} tile={tile} r={[p['r'] for p in batch]}", flush=True)
    res = ctx.residual_batched(batch, "fp64", tile, flags=STRATEGIES[strategy])
    for p, (Raa, Rab, n2) in zip(batch, res):
        check_oracle(p, Raa, Rab, n2, TOL64)


def test_small_batch_general_kernels(acse, ctx):
    batch = small_batch()
    res = ctx.residual_batched(batch, "fp64", -1, flags=acse.FLAG_GENERAL_KERNELS)
    for p, (Raa, Rab, n2) in zip(batch, res):
        check_oracle(p, Raa, Rab, n2, TOL64)


@pytest.mark.parametrize("strategy", list(STRATEGIES))
def test_big_batch_equals_single_launches(ctx, big_batch, strategy):
    import torch
    res = ctx.residual_batched(big_batch, "fp64", 1, flags=STRATEGIES[strategy])
    for i, (p, (Raa, Rab, n2)) in enumerate(zip(big_batch, res)):
        print(f"[batched big] {strategy} instance {i} r={p['r']}", flush=True)
        Saa, Sab, s2 = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2,
                                    "fp64", 1)
        assert torch.equal(Raa, Saa) and torch.equal(Rab, Sab), i
        assert n2 == s2
        if p["r"] <= 28:
            check_oracle(p, Raa, Rab, n2, TOL64)


@pytest.mark.parametrize("strategy", list(STRATEGIES))
def test_big_batch_fp32(ctx, big_batch, strategy):
    sub = [p for p in big_batch if p["r"] == 20]
    res = ctx.residual_batched(big_batch, "fp32", flags=STRATEGIES[strategy])
    k = 0
    for p, (Raa, Rab, n2) in zip(big_batch, res):
        if p["r"] != 20:
            continue
        check_oracle(p, Raa, Rab, n2, TOL32)
        k += 1
    assert k == len(sub) == 3


def test_autotune_batched_and_reuse(acse, ctx, big_batch):
    import torch
    probs, keep = [], []
    for p in big_batch:
        prob, t = ctx.problem(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2)
        probs.append(prob)
        keep.append(t)
    pers = acse.FLAG_BATCH_PERSISTENT
    best, times = ctx.autotune_batched_raw(probs, ctx.options("fp64", flags=pers))
    print(f"[batched autotune] persistent: best {best} times {times}", flush=True)
    assert 0 <= best < acse.NUM_TILE_CONFIGS and all(t > 0 for t in times)
    # the persistent launch takes the tuned configuration with tile = -1
    tuned = ctx.residual_batched(big_batch, "fp64", -1, flags=pers)
    fixed = ctx.residual_batched(big_batch, "fp64", best, flags=pers)
    for a, b in zip(tuned, fixed):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    # lanes: every r tuned as a single call; tile = -1 then gives each
    # instance's single-call result bitwise
    best, times = ctx.autotune_batched_raw(probs, ctx.options("fp64"))
    print(f"[batched autotune] lanes: best (r = 44) {best} times {times}", flush=True)
    assert 0 <= best < acse.NUM_TILE_CONFIGS and all(t > 0 for t in times)
    tuned = ctx.residual_batched(big_batch, "fp64", -1)
    for p, (Raa, Rab, n2) in zip(big_batch, tuned):
        Saa, Sab, s2 = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2, "fp64")
        assert torch.equal(Raa, Saa) and torch.equal(Rab, Sab) and n2 == s2
    # a smaller batch afterwards reuses the workspace
    small = small_batch()[:3]
    for p, (Raa, Rab, n2) in zip(small, ctx.residual_batched(small, "fp64")):
        check_oracle(p, Raa, Rab, n2, TOL64)


def test_batched_errors(acse, ctx):
    import torch
    good = gen.problem(6, 4, 12, seed=1)
    prob, keep = ctx.problem(good["h"], good["V"], good["gamma"], good["d2aa"], good["d2ab"], 2)
    out = [torch.empty((6,) * 4, dtype=torch.float64, device=ctx.device) for _ in range(2)]
    with pytest.raises(acse.AcseError):
        ctx.residual_batched_raw([], ctx.options("fp64"), [], [])
    bad_prob = acse.Problem(prob.r, 1, 2, prob.h, prob.V, prob.d1, prob.d2aa, prob.d2ab)
    with pytest.raises(acse.AcseError, match="instance 1"):
        ctx.residual_batched_raw([prob, bad_prob], ctx.options("fp64"), [out[0]] * 2, [out[1]] * 2)


def test_int8crt_batch_on_lanes(ctx, big_batch):
    """The int8 exact-accumulation products in a batch (lanes, one residue
    workspace per lane): the small mixed batch against the oracle at the FP64
    bar, and every instance of the 12-instance workload bitwise equal to its
    own single int8crt call."""
    import torch
    small = small_batch()
    print("[batched int8crt] small batch", flush=True)
    for p, (Raa, Rab, n2) in zip(small, ctx.residual_batched(small, "int8crt")):
        check_oracle(p, Raa, Rab, n2, TOL64)
    res = ctx.residual_batched(big_batch, "int8crt")
    for i, (p, (Raa, Rab, n2)) in enumerate(zip(big_batch, res)):
        Saa, Sab, s2 = ctx.residual(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2, "int8crt")
        assert torch.equal(Raa, Saa) and torch.equal(Rab, Sab) and n2 == s2, i
