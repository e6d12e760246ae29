"""The Nakatsuji-Yasuda spin-block plan of the library (host logic,
paper_2604_02550_amd/csrc/ny_plan.h), checked on the CPU.

The plan is compiled with g++ (tests/ny_plan_dump.cpp prints it as JSON) and
executed here with numpy, operation by operation as the library's executor
does: operand builds (source blocks permuted or pair-packed into operand
layout, intermediates from their staging, sums and differences), the block
products with their output layouts and weights, the unscrambling passes, the
partial trace Y and the final combination

    B = 4 [sw(T_il) + T_pl - 2 sw(T_ir) - 2 T_pr],  C = B - B(k <-> l).

The alpha-alpha and alpha-beta blocks of C must equal the oracle's factorised
NY share (oracle/residual.py, contraction_b_ny, pinned against the
materialised definition in test_oracle_ny.py) for random singlet-structured
inputs and sigma patterns.  A wrong spin block, layout, weight or pairing in
the plan fails here without a GPU.
"""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import rdm
from oracle import residual as rs
from synth import generators as gen

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2604_02550_amd", "csrc")


@pytest.fixture(scope="module")
def plan(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("nyplan") / "ny_plan_dump")
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", CSRC, "-o", exe, os.path.join(HERE, "ny_plan_dump.cpp")],
                   check=True)
    return json.loads(subprocess.run([exe], check=True, capture_output=True, text=True).stdout)


def test_plan_counts(plan):
    # 18 block products per map (one packed), 5 crosswise pairs
    assert len(plan["products"]) == 18
    assert sum(1 for g in plan["products"] if g[9]) == 1
    assert len(plan["unscrambles"]) == 5
    assert all(g[8] in (1.0, 2.0) for g in plan["products"])


def execute(P, r, Xaa, Xab, gamma, d2aa, d2ab, sig):
    Daa = d2aa - 0.5 * (np.einsum('pr,qs->pqrs', gamma, gamma) - np.einsum('ps,qr->pqrs', gamma, gamma))
    Dab = d2ab - 0.5 * np.einsum('pr,qs->pqrs', gamma, gamma)

    def blocks(aa, ab):
        return {0: aa, 5: ab, 6: -ab.transpose(0, 1, 3, 2)}
    src = {0: blocks(Xaa, Xab), 1: blocks(Daa, Dab)}
    src[2] = {b: v * sig[None, None, :, None] for b, v in src[1].items()}
    staging = {(t, b): i for t, b, i in P["staging"]}
    st_arr, prod, bufs = {}, {}, {}
    stages = P["stages"]
    iu = np.triu_indices(r, 1)
    for phase in (0, 1):
        for t1, b1, t2, b2, c2, lay, ph, buf, packed in P["operands"]:
            if ph != phase:
                continue
            if lay >= 0:
                o = P["layouts"][lay]
                M = src[t1][b1].transpose(o)
                if t2 >= 0:
                    M = M + c2 * src[t2][b2].transpose(o)
            else:
                M = st_arr[staging[(t1, b1)]]
                if t2 >= 0:
                    M = M + c2 * st_arr[staging[(t2, b2)]]
            bufs[buf] = M.reshape(r * r, r, r)[:, iu[0], iu[1]] if packed else M.reshape(r * r, r * r)
        for a, bb, out, blk, stg, ph, acc, term, alpha, packed in P["products"]:
            if ph != phase:
                continue
            la, ra, lb, rb, lo = stages[stg]
            C = alpha * (bufs[a] @ bufs[bb].T).reshape(r, r, r, r)
            C = np.einsum(ra + rb + '->' + lo, C)
            if out >= 6:
                prod[(out, blk)] = C if not acc else prod[(out, blk)] + C
            else:
                i = staging[(out, blk)]
                st_arr[i] = C if not acc else st_arr[i] + C
        for out, bx, by, ph in P["unscrambles"]:
            if ph != phase:
                continue
            if out >= 6:
                x, y = prod[(out, bx)], prod[(out, by)]
                prod[(out, bx)], prod[(out, by)] = 0.5 * (x + y), 0.5 * (x - y)
            else:
                ix, iy = staging[(out, bx)], staging[(out, by)]
                x, y = st_arr[ix], st_arr[iy]
                st_arr[ix], st_arr[iy] = 0.5 * (x + y), 0.5 * (x - y)
    Y = np.einsum('pkpa->ka', st_arr[staging[(3, 0)]]) + np.einsum('pkpa->ka', st_arr[staging[(3, 5)]])

    def T(t, b):
        return prod[(t, b ^ 15 if b & 8 else b)]

    def Bv(b):
        bs = ((b >> 2) & 1) << 3 | ((b >> 3) & 1) << 2 | (b & 3)  # spins of i and j exchanged
        tpl = np.einsum('ka,ijal->ijkl', Y, src[2][b])
        return 4 * (T(6, b) - T(6, bs).transpose(1, 0, 2, 3) + tpl - 2 * T(7, b)
                    + 2 * T(7, bs).transpose(1, 0, 2, 3) - 2 * T(8, b))
    return Bv(0) - Bv(0).transpose(0, 1, 3, 2), Bv(5) - Bv(6).transpose(0, 1, 3, 2)


@pytest.mark.parametrize("r,seed,sig", [(3, 0, (1, -1, 1)), (4, 1, (1, -1, 1, -1)), (5, 2, (-1, 1, 1, -1, 1))])
def test_plan_matches_oracle_share(plan, r, seed, sig):
    p = gen.problem(r, 4, 8, seed=seed)
    rng = np.random.default_rng(seed + 50)
    ex = gen.symmetric_direction(rng, r, scale=0.05)
    d2aa, d2ab, g = p["d2aa"] + ex["d2aa"], p["d2ab"] + ex["d2ab"], p["gamma"]
    xd = gen.symmetric_direction(rng, r, scale=1.0)  # X_aa antisymmetric, X_ab pair-exchange symmetric
    sig = np.array(sig, dtype=float)
    caa_plan, cab_plan = execute(plan, r, xd["d2aa"], xd["d2ab"], g, d2aa, d2ab, sig)
    _, Xso = rdm.blocks_to_spin_orbital(np.eye(r), xd["d2aa"], xd["d2ab"])
    d1, d2 = rdm.blocks_to_spin_orbital(g, d2aa, d2ab)
    B = rs.contraction_b_ny(Xso, d1, d2, rdm.sigma_spin_orbital(sig)).numpy()
    caa, cab = rdm.spin_orbital_to_blocks(B - B.transpose(0, 1, 3, 2))
    scale = max(np.abs(caa).max(), np.abs(cab).max())
    assert scale > 1e-6
    assert np.abs(caa_plan - caa).max() <= 1e-12 * scale
    assert np.abs(cab_plan - cab).max() <= 1e-12 * scale
