"""Benchmark of the ACSE residual hot path on one MI355X.

A step is one pass of the whole hot path on the r = 50, N = 30 synthetic
workload (seed 0): the residual R of Eq. (4) with the Valdemoro 3-RDM, its
norm, the update map U = F(R), the Euler update of the 2-RDM blocks, trace
restoration, the 1-RDM contraction and the energy (one ``acse_step`` call).
Each step starts from the same input state: the 1-/2-RDM blocks are restored
on the device from a pristine copy inside the timed region (one r^4 device copy
per block, negligible next to the contractions).

Prints one JSON line.  ``value`` = steps per second of the first mode in
``--modes`` (one step = one ``acse_step``: the residual, the update map, the
Euler step and the energy); by default that is "int8crt", the exact-accumulation
int8 products, the fastest mode whose one-step energy meets |dE| < 1e-7 Eh.  ``residual_evals_per_s`` is the residual-only
rate (``acse_residual`` alone) of the same kernels.  Every mode is timed and
its one-step energy checked against the stored FP64 oracle values;
``accuracy_gate`` says per mode whether |dE| < 1e-7 Eh holds.

    python bench.py [--steps K] [--warmup W] [--modes int8crt,fp64,fp32,bf16x3] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2516.6, "int8crt": 5000.0}  # int8: dense TOP/s
CRT_MODULI = 13  # modulus count of the int8crt mode (the library default)
GOLDEN = os.path.join(ROOT, "tests", "golden", "r50_step.json")
TRAFFIC = os.path.join(ROOT, "profiles", "gemm_traffic_r50.json")
# the GEMM kernels and the descriptor they take (the traffic figures are those of these kernels)
TRAFFIC_SRCS = [os.path.join(ROOT, "paper_2604_02550_amd", "csrc", f)
                for f in ("gemm.hip", "gemm_crt.hip", "gemm_crt.h", "acse_internal.h")]


def gemm_flops(r):
    """Algorithmic flops of one grouped GEMM launch (one residual map): three
    particle-hole products r^2 x r^2 x r^2 and three packed particle-particle
    products (rows x r^2 x K with rows = K = r(r-1)/2, r(r+1)/2, r(r-1)/2)."""
    lt, le = r * (r - 1) // 2, r * (r + 1) // 2
    return 3 * 2 * r ** 6 + 2 * r * r * (lt * lt + le * le + lt * lt)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="r50")
    ap.add_argument("--modes", default="int8crt,fp64,fp32,bf16x3")
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--vjp-modes", default="int8crt,fp64,fp32",
                    help="precisions of the adjoint (VJP) measurement ('' to skip)")
    ap.add_argument("--batched-modes", default="int8crt,fp64,fp32",
                    help="precisions of the batched-instances measurement ('' to skip)")
    ap.add_argument("--solve-controls", default="fixed,backtrack,quadratic",
                    help="step controls of acse_solve timed on the workload (FP64); empty to skip")
    ap.add_argument("--solve-iters", type=int, default=5)
    ap.add_argument("--ny-steps", type=int, default=5,
                    help="steps of the Nakatsuji-Yasuda leg (FP64); 0 skips it")
    ap.add_argument("--spin-steps", type=int, default=5,
                    help="steps of the open-shell (N_alpha != N_beta) leg at r = 50 (FP64); 0 skips it")
    ap.add_argument("--spin-ny-steps", type=int, default=2,
                    help="steps of the open-shell leg with the NY 3-RDM at r = 50 (FP64); 0 skips it")
    ap.add_argument("--solve-eps", type=float, default=1e-5,
                    help="first step size of the acse_solve leg (the synthetic r = 50 integrals are "
                         "large: eps = 1e-3 raises ||R|| at the first trial)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


# GEMM tile shapes (BM, BN, BK, LDS stages) per configuration index, as instantiated in gemm.hip
TILE_SHAPES = {"fp64": [(128, 128, 16, 2), (64, 64, 16, 2), (128, 64, 16, 2)],
               "fp32": [(128, 128, 32, 2), (64, 64, 32, 2), (128, 128, 64, 1)],
               "bf16x3": [(128, 128, 32, 2), (64, 64, 32, 2), (128, 128, 64, 1)]}
TRAITS = {"fp64": "TrF64", "fp32": "TrF32", "bf16x3": "TrBF16x3"}


def gemm_kernel_name(prec, cfg):
    if prec == "int8crt":
        return "acse::(anonymous namespace)::gemm_mod_kernel"
    bm, bn, bk, ns = TILE_SHAPES[prec][cfg]
    wpe = 2 if prec == "fp64" and bm * bn >= 128 * 128 else 1   # register cap of the instantiation
    return f"acse::gemm_nt_kernel<acse::{TRAITS[prec]}, {bm}, {bn}, {bk}, {ns}, {wpe}>"


def bench_batched(acse, ctx, gen, torch, modes, steps, warmup):
    """Twelve instances (r in {20, 28, 36, 44}, ground + 2 excited states each):
    one acse_residual_batched call per step (default: each instance on its own
    side-stream lane; and with ACSE_FLAG_BATCH_PERSISTENT: all products in one
    persistent launch) against twelve acse_residual calls in order on one
    stream (each with its own autotuned tile configuration)."""
    dev = torch.device("cuda", 0)
    batch = gen.batched_problems(seed=0)
    probs, keep, outs = [], [], []
    for p in batch:
        prob, t = ctx.problem(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2)
        probs.append(prob)
        keep.append(t)
        r = p["r"]
        outs.append([torch.empty((r, r, r, r), dtype=torch.float64, device=dev) for _ in range(2)])
    Ra, Rb = [o[0] for o in outs], [o[1] for o in outs]
    flops = sum(gemm_flops(p["r"]) for p in batch)
    res = {}
    for mode in modes:
        opts = acse.Context.options(mode)
        popts = acse.Context.options(mode, flags=acse.FLAG_BATCH_PERSISTENT)
        ctx.autotune_batched_raw(probs, opts)          # every r, as single calls take them
        if mode != "int8crt":
            best, tile_ms = ctx.autotune_batched_raw(probs, popts)

        def timed(fn):
            for _ in range(warmup):
                fn()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(ctx.stream)
            for _ in range(steps):
                fn()
            b.record(ctx.stream)
            torch.cuda.synchronize()
            return a.elapsed_time(b) / steps

        def batched():
            ctx.residual_batched_raw(probs, opts, Ra, Rb, want_norm=False)

        def persistent():
            ctx.residual_batched_raw(probs, popts, Ra, Rb, want_norm=False)

        def sequential():
            for prob, o in zip(probs, outs):
                ctx.residual_raw(prob, opts, o[0], o[1], want_norm=False)

        ms_b = timed(batched)
        ms_s = timed(sequential)
        if mode == "int8crt":   # the persistent strategy runs the floating-point products only
            res[mode] = dict(instances=len(batch), sizes=sorted({p["r"] for p in batch}),
                             batched_ms=ms_b, sequential_ms=ms_s,
                             batched_evals_per_s=len(batch) * 1e3 / ms_b,
                             sequential_evals_per_s=len(batch) * 1e3 / ms_s,
                             speedup=ms_s / ms_b, useful_tflops=flops / (ms_b * 1e-3) / 1e12)
            continue
        ms_p = timed(persistent)
        ctx.profile(True)
        persistent()
        prof = ctx.profile_read()
        ctx.profile(False)
        gemm_ms = prof["gemm"][0]
        res[mode] = dict(instances=len(batch), sizes=sorted({p["r"] for p in batch}),
                         batched_ms=ms_b, persistent_ms=ms_p, sequential_ms=ms_s,
                         batched_evals_per_s=len(batch) * 1e3 / ms_b,
                         sequential_evals_per_s=len(batch) * 1e3 / ms_s,
                         speedup=ms_s / ms_b, persistent_speedup=ms_s / ms_p,
                         persistent_tile_config=best, persistent_tile_gemm_ms=tile_ms,
                         persistent_gemm_ms=gemm_ms,
                         persistent_gemm_tflops=flops / (gemm_ms * 1e-3) / 1e12,
                         useful_tflops=flops / (ms_b * 1e-3) / 1e12)
    return res


def bench_vjp(acse, gen, torch, modes, steps, warmup, ny_steps=2):
    """acse_residual_vjp with a seeded cotangent: on the differentiation workload
    (r = 30, N = 20) and on r = 50, N = 30, against the forward residual of the
    same problem (one context per size).  With ny_steps > 0 also the NY
    residual's adjoint ("ny_fp64": the FP64 Valdemoro adjoint plus the NY
    share's, FP64 over spin-orbital tensors), ny_steps timed calls after one
    warm-up, against the NY forward residual; "ny_int8crt" the same with the
    int8 exact-accumulation products in both adjoints."""
    dev = torch.device("cuda", 0)
    res = {}
    for wl in ("vjp30", "r50"):
        p = gen.named(wl)
        r = p["r"]
        ctx = acse.Context(r_max=r, device=0)
        prob, keep = ctx.problem(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2)
        Rb = [torch.as_tensor(a, device=dev).contiguous() for a in gen.cotangent(np.random.default_rng(5), r)]
        outs = [torch.empty_like(t) for t in keep]
        R = [torch.empty((r, r, r, r), dtype=torch.float64, device=dev) for _ in range(2)]
        for mode in list(modes) + (["ny_fp64", "ny_int8crt"] if ny_steps > 0 else []):
            ny = mode.startswith("ny_")
            opts = acse.Context.options(mode[3:] if ny else mode, sigma=True if ny else None)
            if not ny:
                ctx.autotune_raw(prob, opts)
            n_warm, n_steps = (1, ny_steps) if ny else (warmup, steps)

            def timed(fn):
                for _ in range(n_warm):
                    fn()
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(ctx.stream)
                for _ in range(n_steps):
                    fn()
                b.record(ctx.stream)
                torch.cuda.synchronize()
                return a.elapsed_time(b) / n_steps

            ms_vjp = timed(lambda: ctx.residual_vjp_raw(prob, opts, Rb[0], Rb[1], *outs))
            ms_fwd = timed(lambda: ctx.residual_raw(prob, opts, R[0], R[1], want_norm=False))
            res[f"{wl}_{mode}"] = dict(r=r, vjp_ms=ms_vjp, residual_ms=ms_fwd, vjp_over_residual=ms_vjp / ms_fwd,
                                       vjp_per_s=1e3 / ms_vjp)
        ctx.close()
        del keep, outs, R, Rb
        torch.cuda.empty_cache()
    return res


def bench_solve(acse, ctx, prob, work, pristine, torch, controls, iters, eps, step_ms):
    """acse_solve (the Euler iteration with the method section's stopping rules)
    on the headline workload, FP64, from the state whose 1-RDM is the
    contraction of its 2-RDM (one acse_step with eps = 0 makes it so).  Wall
    time per accepted step against the plain acse_step time: the driver's host
    decisions, copies and per-trial synchronisations are the difference."""
    opts = acse.Context.options("fp64")
    res = {}
    for control in controls:
        for w, q in zip(work, pristine):
            w.copy_(q)
        ctx.step_raw(prob, 0.0, opts, want=False)
        so = acse.SolveOptions(eps, 0.0, 0.0, iters, acse.CONTROLS[control], 8, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, trials = ctx.solve_raw(prob, opts, so)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[control] = dict(iterations=out.iterations, trials=out.trials, maps=out.maps,
                            stop=acse.STOP_REASONS[out.stop], wall_ms=wall * 1e3,
                            ms_per_accepted_step=wall * 1e3 / max(1, out.iterations),
                            ms_per_map=wall * 1e3 / max(1, out.maps),
                            energy0=out.energy0, energy=out.energy,
                            norm2_ratio=out.norm2 / out.norm2_0, eps_last=out.eps,
                            eps0=eps, acse_step_ms=step_ms)
    for w, q in zip(work, pristine):
        w.copy_(q)
    return res


def bench_solve_spin(acse, ctx, gen, torch, controls, iters, eps, step_ms, name="r50s"):
    """acse_solve_spin (the Euler iteration for a state of any S_z, FP64) with
    the fixed, backtracking and quadratic controls (the last with its slope
    from four more residual maps per step) on the open-shell workload, each from
    the state whose 1-RDMs are contracted from its 2-RDM (one acse_step_spin
    with eps = 0): wall time per accepted step and per map against the plain
    acse_step_spin time."""
    dev = torch.device("cuda", 0)
    p = gen.named_spin(name)
    r = p["r"]
    h = torch.as_tensor(p["h"], device=dev).contiguous()
    V = torch.as_tensor(p["V"], device=dev).contiguous()
    work = [torch.as_tensor(p[k], device=dev).contiguous() for k in ("gamma_a", "gamma_b", "d2aa", "d2bb", "d2ab")]
    pristine = [t.clone() for t in work]
    prob = acse.ProblemSpin(r, p["Na"], p["Nb"], h.data_ptr(), V.data_ptr(), *[t.data_ptr() for t in work])
    opts = acse.Context.options("fp64")
    res = {}
    for control in controls:
        for w, q in zip(work, pristine):
            w.copy_(q)
        ctx.step_spin_raw(prob, 0.0, opts, want=False)
        so = acse.SolveOptions(eps, 0.0, 0.0, iters, acse.CONTROLS[control], 8, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, trials = ctx.solve_spin_raw(prob, opts, so)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[control] = dict(iterations=out.iterations, trials=out.trials, maps=out.maps,
                            stop=acse.STOP_REASONS[out.stop], wall_ms=wall * 1e3,
                            ms_per_accepted_step=wall * 1e3 / max(1, out.iterations),
                            ms_per_map=wall * 1e3 / max(1, out.maps), energy0=out.energy0, energy=out.energy,
                            norm2_ratio=out.norm2 / out.norm2_0, eps_last=out.eps, eps0=eps,
                            acse_step_spin_ms=step_ms)
    return res


def ny_map_flops(r):
    """Flops the NY share's block products execute per map (the plan of
    ny_plan.h): 17 products of r^2 x r^2 x r^2 and one whose summed pair is
    packed to r(r-1)/2 columns."""
    return 2.0 * r ** 6 * (17 + (r * (r - 1) / 2) / r ** 2)


def bench_ny(acse, ctx, prob, work, pristine, torch, stream, steps, warmup, eps, v_step_ms, mode="fp64"):
    """One acse_step with the Nakatsuji-Yasuda 3-RDM (Eq. (8)) on the same
    workload, block products in `mode`: ms per step, the residual-only time,
    the stage split with the NY share's own stages, the share's rate in
    executed block-GEMM flops (ny_map_flops per map) per second of its whole
    stage, and the roofline of the block GEMM launches alone.  The check is
    E1 - E0 = -eps ||R||^2."""
    r = prob.r
    opts = acse.Context.options(mode, sigma=True)

    def restore():
        for w, q in zip(work, pristine):
            w.copy_(q)

    for _ in range(warmup):
        restore()
        ctx.step_raw(prob, eps, opts, want=False)
    torch.cuda.synchronize()
    ctx.profile(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        restore()
        ctx.step_raw(prob, eps, opts, want=False)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    prof = ctx.profile_read()
    ctx.profile(False)
    restore()
    E0 = ctx.energy_raw(prob)
    E1, n2 = ctx.step_raw(prob, eps, opts)
    restore()
    # residual-only rate with the NY 3-RDM (the oracle is timed on the same call)
    R = [torch.empty((r, r, r, r), dtype=torch.float64, device="cuda") for _ in range(2)]
    ctx.residual_raw(prob, opts, R[0], R[1], want_norm=False)
    torch.cuda.synchronize()
    s2 = torch.cuda.Event(enable_timing=True)
    e2 = torch.cuda.Event(enable_timing=True)
    s2.record(stream)
    for _ in range(steps):
        ctx.residual_raw(prob, opts, R[0], R[1], want_norm=False)
    e2.record(stream)
    torch.cuda.synchronize()
    res_ms = s2.elapsed_time(e2) / steps
    del R
    ny_ms = prof["ny_share"][0] / steps
    gemm_ms = prof["ny_gemm"][0] / steps
    flops = 2 * ny_map_flops(r)
    work = flops * (CRT_MODULI if mode == "int8crt" else 1)   # int8 ops: one product per modulus
    achieved = work / (gemm_ms * 1e-3) / 1e12
    return dict(ms_per_step=ms, steps_per_s=1e3 / ms, over_valdemoro_step=ms / v_step_ms,
                residual_ms=res_ms, residual_evals_per_s=1e3 / res_ms,
                stage_ms_per_step={k: v[0] / steps for k, v in prof.items()},
                ny_share_ms_per_step=ny_ms, ny_block_gemm_flops_per_step=flops,
                ny_share_tflops=flops / (ny_ms * 1e-3) / 1e12,
                roofline={"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[mode],
                          "unit": "TOP/s" if mode == "int8crt" else "TFLOP/s",
                          "frac": achieved / PEAK_TFLOPS[mode],
                          "kernel": "gemm_nt_kernel on the NY block products (18 per map, one with its summed pair packed; "
                                    "HIP-event time of their launches)"},
                energy_identity_rel=abs((E1 - E0) + eps * n2) / (eps * n2))


SPIN_GOLDEN = os.path.join(ROOT, "tests", "golden", "r50_spin_step.json")


def spin_map_flops(r):
    """Algorithmic flops of the block products of one spin-block map: 13
    products of r^2 x r^2 x r^2 (the mixed-spin Y and W H terms and the ten E
    terms) and the four same-spin Y and W H products with rows and summed pair
    packed to the pairs i < j, r < s (r(r-1)/2 x r^2 x r(r-1)/2)."""
    lt = r * (r - 1) // 2
    return 13 * 2.0 * r ** 6 + 4 * 2.0 * lt * r * r * lt


def bench_spin(acse, ctx, gen, torch, steps, warmup, eps, mode="fp64", name="r50s", ny=False):
    """One acse_step_spin per step on the open-shell workload (r = 50,
    N_alpha = 16, N_beta = 14): the residual, the update map, the per-block
    Euler step with trace restoration, the 1-RDMs per spin and the energy,
    with the block products in FP64 or as int8 exact-accumulation products
    ("int8crt").  Inputs restored from a pristine device copy inside the timed
    region.  Checked against the stored FP64 oracle values of the same step
    (Valdemoro).  With ``ny`` both maps add the NY share (default open-shell
    occupations) over spin-orbital tensors (2r = 100), its block products in
    the mode's precision."""
    dev = torch.device("cuda", 0)
    p = gen.named_spin(name)
    r = p["r"]
    h = torch.as_tensor(p["h"], device=dev).contiguous()
    V = torch.as_tensor(p["V"], device=dev).contiguous()
    keys = ("gamma_a", "gamma_b", "d2aa", "d2bb", "d2ab")
    pristine = [torch.as_tensor(p[k], device=dev).contiguous() for k in keys]
    work = [t.clone() for t in pristine]
    prob = acse.ProblemSpin(r, p["Na"], p["Nb"], h.data_ptr(), V.data_ptr(), *[t.data_ptr() for t in work])
    outs = [torch.empty((r, r, r, r), dtype=torch.float64, device=dev) for _ in range(6)]
    opts = acse.Context.options(mode, sigma=True if ny else None)
    stream = ctx.stream

    def restore():
        for w, q in zip(work, pristine):
            w.copy_(q)

    for _ in range(warmup):
        restore()
        ctx.step_spin_raw(prob, eps, opts, outs, want=False)
    torch.cuda.synchronize()
    ctx.profile(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        restore()
        ctx.step_spin_raw(prob, eps, opts, outs, want=False)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    prof = ctx.profile_read()
    ctx.profile(False)
    # residual-only rate
    R = outs[:3]
    ctx.residual_spin_raw(prob, opts, *R, want_norm=False)
    torch.cuda.synchronize()
    s2 = torch.cuda.Event(enable_timing=True)
    e2 = torch.cuda.Event(enable_timing=True)
    s2.record(stream)
    for _ in range(steps):
        ctx.residual_spin_raw(prob, opts, *R, want_norm=False)
    e2.record(stream)
    torch.cuda.synchronize()
    res_ms = s2.elapsed_time(e2) / steps
    restore()
    E1, n2 = ctx.step_spin_raw(prob, eps, opts, outs)
    err = None
    if os.path.exists(SPIN_GOLDEN) and not ny:
        g = json.load(open(SPIN_GOLDEN))
        idx = [tuple(t) for t in g["index"]]
        got = dict(zip(("R_aa", "R_bb", "R_ab", "U_aa", "U_bb", "U_ab"), [o.cpu().numpy() for o in outs]))
        got.update(zip(("d2aa", "d2bb", "d2ab"), [w.cpu().numpy() for w in work[2:]]))
        err = dict(dE=abs(E1 - g["energy1"]), meets_dE_1em7=bool(abs(E1 - g["energy1"]) < 1e-7),
                   norm2_rel=abs(n2 - g["norm2"]) / g["norm2"])
        for k, v in got.items():
            ref = np.array(g["samples"][k])
            val = np.array([v[t] for t in idx])
            err[f"{k}_sample_rel"] = float(np.abs(val - ref).max() / max(np.abs(ref).max(), 1e-300))
            err[f"{k}_norm_rel"] = abs(float(np.linalg.norm(v)) - g["norms"][k]) / max(g["norms"][k], 1e-300)
    restore()
    gemm_ms, gemm_n = prof["gemm"]
    flops = 2 * spin_map_flops(r)          # two maps per step
    work = flops * (CRT_MODULI if mode == "int8crt" else 1)   # int8 ops: one product per modulus
    achieved = work / (gemm_ms / steps * 1e-3) / 1e12
    kernel = ("gemm_mod_kernel on the 17 spin-block products per map (13 moduli; HIP-event time of its "
              "launches)" if mode == "int8crt" else
              "gemm_nt_kernel<TrF64> on the 17 spin-block products per map (HIP-event time of their launches)")
    extra = {}
    if ny:
        # two maps; six spin-orbital contractions each, of which ten r^2 x r^2 x r^2
        # spin-block products per contraction conserve spin and run
        ny_flops = 2 * 6 * 10 * 2 * r ** 6
        ny_ms, _ = prof["ny_share"]
        nyg_ms, _ = prof["ny_gemm"]
        rate = ny_flops / (nyg_ms / steps * 1e-3) / 1e12  # FP64-equivalent rate of the block products
        extra = dict(ny_share_ms_per_step=ny_ms / steps, ny_gemm_ms_per_step=nyg_ms / steps,
                     ny_gemm_flops_per_step=ny_flops, ny_gemm_tflops=rate)
        if mode == "int8crt":   # int8 ops: one product per modulus, against the int8 peak
            extra["ny_gemm_frac_int8"] = rate * CRT_MODULI / PEAK_TFLOPS["int8crt"]
        else:
            extra["ny_gemm_frac_fp64"] = rate / PEAK_TFLOPS["fp64"]
    return dict(
        workload=f"{name}: r={r}, N_alpha={p['Na']}, N_beta={p['Nb']}, three 2-RDM spin blocks, one "
                 f"acse_step_spin (eps={eps}) per step, products {mode}"
                 + (", NY 3-RDM (open-shell occupations)" if ny else ""),
        **extra,
        ms_per_step=ms, steps_per_s=1e3 / ms, residual_ms=res_ms, residual_evals_per_s=1e3 / res_ms,
        stage_ms_per_step={k: v[0] / steps for k, v in prof.items()},
        block_gemm_flops_per_step=flops, useful_tflops_step=flops / (ms * 1e-3) / 1e12,
        roofline={"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[mode],
                  "unit": "TOP/s" if mode == "int8crt" else "TFLOP/s",
                  "frac": achieved / PEAK_TFLOPS[mode], "kernel": kernel},
        error_vs_oracle=err, energy1=E1, norm2=n2)


def cpu_model():
    """CPU model string of the host (the 'model name' line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def time_oracle(fn, reps=3, warmup=1):
    """Median wall time of `reps` calls after `warmup` untimed ones."""
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), ts


def cpu_baseline(p, gen):
    """The FP64 oracle's residual (tier B, dense spin-orbital products of about
    384 r^6 flops; a correctness oracle, not a tuned CPU code) on this host:
    every usable core, 1 warm-up and the median of 3 at the bench workload, plus
    one 1-thread call on the r = 30, N = 20 workload for scale."""
    import torch
    from oracle import step as ost

    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    before = torch.get_num_threads()
    torch.set_num_threads(usable)
    args = (p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"])
    med, ts = time_oracle(lambda: ost.residual(*args))
    torch.set_num_threads(1)
    q = gen.named("r30")
    t1, _ = time_oracle(lambda: ost.residual(q["h"], q["V"], q["N"], q["gamma"], q["d2aa"], q["d2ab"]),
                        reps=1, warmup=0)
    torch.set_num_threads(before)
    r = p["r"]
    return {"value": 1.0 / med, "unit": "residual evals/s", "cores": usable, "kind": "oracle",
            "sample": f"FP64 oracle residual at r={r}, N={p['N']} (spin-orbital factorised form, about "
                      f"384 r^6 = {384 * r ** 6:.2e} flop): median of 3 after 1 warm-up on {usable} threads "
                      f"({', '.join(f'{t:.2f}' for t in ts)} s)",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "oracle_gflops": 384 * r ** 6 / med / 1e9,
            "one_thread_r30": {"seconds": t1, "evals_per_s": 1.0 / t1,
                               "sample": "one FP64 oracle residual at r=30, N=20 on 1 thread"}}


def src_hash():
    h = hashlib.sha256()
    for path in TRAFFIC_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU path is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_02550_amd as acse
    from synth import generators as gen

    dev = torch.device("cuda", 0)
    p = gen.named(args.workload)
    r, N = p["r"], p["N"]
    na = N // 2
    ctx = acse.Context(r_max=r, device=0)
    stream = ctx.stream
    h = torch.as_tensor(p["h"], device=dev).contiguous()
    V = torch.as_tensor(p["V"], device=dev).contiguous()
    pristine = [torch.as_tensor(p[k], device=dev).contiguous() for k in ("gamma", "d2aa", "d2ab")]
    work = [t.clone() for t in pristine]
    prob = acse.Problem(r, na, na, h.data_ptr(), V.data_ptr(), *[t.data_ptr() for t in work])
    R = [torch.empty((r, r, r, r), dtype=torch.float64, device=dev) for _ in range(2)]
    U = [torch.empty((r, r, r, r), dtype=torch.float64, device=dev) for _ in range(2)]

    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * 2 ** 20 // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    golden = json.load(open(GOLDEN)) if os.path.exists(GOLDEN) and args.workload == "r50" else None

    def restore():
        for w, q in zip(work, pristine):
            w.copy_(q)

    results = {}
    for mode in args.modes.split(","):
        opts = acse.Context.options(mode)
        best_tile, tile_ms = ctx.autotune_raw(prob, opts)
        # warmup
        for _ in range(args.warmup):
            restore()
            ctx.step_raw(prob, args.eps, opts, want=False)
        torch.cuda.synchronize()
        ctx.profile(True)
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start.record(stream)
        for _ in range(args.steps):
            restore()
            ctx.step_raw(prob, args.eps, opts, R[0], R[1], U[0], U[1], want=False)
        stop.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = start.elapsed_time(stop) / args.steps
        prof = ctx.profile_read()
        ctx.profile(False)
        gemm_ms, gemm_n = prof["gemm"]
        # residual-only rate of the same kernels
        res_steps = max(args.steps, 5)
        for _ in range(2):
            ctx.residual_raw(prob, opts, R[0], R[1], want_norm=False)
        torch.cuda.synchronize()
        s2 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        restore()
        s2.record(stream)
        for _ in range(res_steps):
            ctx.residual_raw(prob, opts, R[0], R[1], want_norm=False)
        e2.record(stream)
        torch.cuda.synchronize()
        res_ms = s2.elapsed_time(e2) / res_steps
        # one checked step against the stored oracle values
        restore()
        E1, n2 = ctx.step_raw(prob, args.eps, opts, R[0], R[1], U[0], U[1])
        err = None
        if golden is not None:
            idx = [tuple(t) for t in golden["index"]]
            got = {k: v.cpu().numpy() for k, v in
                   (("R_aa", R[0]), ("R_ab", R[1]), ("U_aa", U[0]), ("U_ab", U[1]))}
            err = dict(
                dE=abs(E1 - golden["energy1"]),
                meets_dE_1em7=bool(abs(E1 - golden["energy1"]) < 1e-7),
                dE_rel_to_step=abs(E1 - golden["energy1"]) / abs(golden["energy1"] - golden["energy0"]),
                norm2_rel=abs(n2 - golden["norm2"]) / golden["norm2"],
            )
            for k in got:
                ref = np.array(golden["samples"][k])
                val = np.array([got[k][t] for t in idx])
                err[f"{k}_sample_rel"] = float(np.abs(val - ref).max() / np.abs(ref).max())
                err[f"{k}_norm_rel"] = abs(float(np.linalg.norm(got[k])) - golden["norms"][k]) / golden["norms"][k]
        gemm_avg = gemm_ms / max(gemm_n, 1)
        # executed work of the dominant launch: int8 ops (one product per modulus) for
        # int8crt, floating-point operations otherwise
        gemm_work = gemm_flops(r) * (CRT_MODULI if mode == "int8crt" else 1)
        achieved = gemm_work / (gemm_avg * 1e-3) / 1e12
        results[mode] = dict(
            ms_per_step=ms, steps_per_s=1e3 / ms, wall_s=wall, residual_ms=res_ms,
            residual_evals_per_s=1e3 / res_ms,
            gemm_avg_ms=gemm_avg, gemm_launches=gemm_n, gemm_tflops=achieved,
            gemm_fp64_equivalent_tflops=gemm_flops(r) / (gemm_avg * 1e-3) / 1e12,
            stage_ms_per_step={k: v[0] / args.steps for k, v in prof.items()},
            useful_tflops_step=2 * gemm_flops(r) / (ms * 1e-3) / 1e12,
            error_vs_oracle=err, energy1=E1, norm2=n2,
            tile_config=best_tile, tile_gemm_ms=tile_ms,
        )

    head = args.modes.split(",")[0]
    hr = results[head]
    traffic = None
    if os.path.exists(TRAFFIC):
        t = json.load(open(TRAFFIC))
        k = t.get("kernels", {}).get(gemm_kernel_name(head, hr["tile_config"]))
        if t.get("src_sha256_16") == src_hash() and k is not None:
            traffic = k.get("bytes_per_launch")
    line = {
        "metric": "ACSE residual evals/s + TFLOP/s at r=50: FP64 vs mixed at |dE|<1e-7 Eh",
        "value": hr["steps_per_s"],
        "unit": "steps/s (one acse_step: residual, update map, Euler step, energy)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hr["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "int8crt": "i8 (CRT, FP64 result)"}[head],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: r={r} spatial orbitals, N={N}, singlet "
                               "alpha-alpha/alpha-beta blocks, one acse_step (eps=1e-3) per step",
                   "r": r, "N": N, "precision": head},
        "tflops": hr["useful_tflops_step"],
        "roofline": {"bound": "mfma", "achieved": hr["gemm_tflops"], "peak": PEAK_TFLOPS[head],
                     "unit": "TFLOP/s", "frac": hr["gemm_tflops"] / PEAK_TFLOPS[head],
                     "traffic": traffic,
                     "kernel": gemm_kernel_name(head, hr["tile_config"]) +
                               (" (13 moduli x (3 ph + 3 packed pp products) per launch; achieved and peak in "
                                "int8 TOP/s)" if head == "int8crt" else
                                " (grouped: 3 ph + 3 packed pp products per launch)")},
        "residual_evals_per_s": hr["residual_evals_per_s"],
        "accuracy_gate": {m: {"dE_Eh": (v["error_vs_oracle"] or {}).get("dE"),
                              "meets_dE_1e-7": (v["error_vs_oracle"] or {}).get("meets_dE_1em7"),
                              "steps_per_s": v["steps_per_s"], "residual_evals_per_s": v["residual_evals_per_s"]}
                          for m, v in results.items()},
        "modes": results,
    }
    if args.solve_controls:
        line["solve"] = bench_solve(acse, ctx, prob, work, pristine, torch, args.solve_controls.split(","),
                                    args.solve_iters, args.solve_eps, results.get("fp64", hr)["ms_per_step"])
    if args.ny_steps > 0:
        line["nakatsuji_yasuda"] = {
            mode: bench_ny(acse, ctx, prob, work, pristine, torch, stream, args.ny_steps, min(args.warmup, 2),
                           args.eps, results[mode]["ms_per_step"], mode)
            for mode in args.modes.split(",")}
    if args.spin_steps > 0:
        line["non_singlet"] = {m: bench_spin(acse, ctx, gen, torch, args.spin_steps, min(args.warmup, 2), args.eps, m)
                               for m in ("int8crt", "fp64")}
        if args.spin_ny_steps > 0:
            for m in ("int8crt", "fp64"):
                line["non_singlet"]["ny_" + m] = bench_spin(acse, ctx, gen, torch, args.spin_ny_steps, 1,
                                                            args.eps, m, ny=True)
        if args.solve_controls:
            line["non_singlet"]["solve_fp64"] = bench_solve_spin(
                acse, ctx, gen, torch, args.solve_controls.split(","), args.solve_iters, args.solve_eps,
                line["non_singlet"]["fp64"]["ms_per_step"])
    if args.vjp_modes:
        line["vjp"] = bench_vjp(acse, gen, torch, args.vjp_modes.split(","), max(3, args.steps // 2),
                                args.warmup)
    if args.batched_modes:
        line["batched_instances"] = bench_batched(acse, ctx, gen, torch, args.batched_modes.split(","),
                                                  args.steps, args.warmup)
    if not args.no_cpu_baseline:
        import torch as _t
        from oracle import step as ost
        line["cpu_baseline"] = cpu_baseline(p, gen)
        threads = line["cpu_baseline"]["cores"]
        _t.set_num_threads(threads)
        if args.ny_steps > 0 and "fp64" in line.get("nakatsuji_yasuda", {}):
            sigma = np.where(np.arange(r) < N // 2, 1.0, -1.0)
            t0 = time.perf_counter()
            ost.residual(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], sigma=sigma)
            dt = time.perf_counter() - t0
            line["nakatsuji_yasuda"]["fp64"]["cpu_baseline"] = {
                "value": 1.0 / dt, "unit": "residual evals/s", "cores": threads, "kind": "oracle",
                "sample": f"one FP64 oracle residual with the NY 3-RDM at r={r}, N={N} (spin-orbital "
                          f"factorised form, {dt:.1f} s)"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
