"""GPU parity of the spin-block path (states of any S_z) with the FP64 oracle.

FP64 bar: normwise and max-elementwise relative error <= 1e-10 per block
(relative to the largest block of R, U or the 2-RDM respectively), scalars
relative 1e-10.  Sizes span several GEMM tiles with ragged tails (r^2 = 16 ...
576 against 64/128 tiles); electron counts cover doublets, triplets,
S_z = 3/2 and an empty beta shell.
"""
import json
import os

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
    return acse.Context(r_max=24)


def cpu(t):
    return t.detach().cpu().numpy()


def _args(p):
    return (p["h"], p["V"], p["gamma_a"], p["gamma_b"], p["d2aa"], p["d2bb"], p["d2ab"], p["Na"], p["Nb"])


def _oracle_args(p):
    return (p["h"], p["V"], p["Na"], p["Nb"], p["gamma_a"], p["gamma_b"], p["d2aa"], p["d2bb"], p["d2ab"])


def _check_blocks(g, o, keys):
    scale = max(np.abs(o[k]).max() for k in keys)
    for k in keys:
        got = cpu(g[k])
        assert np.abs(got - o[k]).max() <= TOL * scale, k
        assert np.linalg.norm(got - o[k]) <= TOL * max(np.linalg.norm(o[k]), 1e-300) + TOL * scale, k


def fock_problem(r, Na, Nb, seed, determinant=False):
    """Exact blocks of a Fock-space state (random or an open-shell determinant)."""
    rng = np.random.default_rng(seed)
    fock = fm.Fock(2 * r)
    if determinant:
        Ua, Ub = gen.haar_orthogonal(rng, r), gen.haar_orthogonal(rng, r)
        C = np.zeros((2 * r, Na + Nb))
        C[:r, :Na] = Ua[:, :Na]
        C[r:, Na:] = Ub[:, :Nb]
        psi = fm.rotated_determinant(fock, C)
    else:
        sec = fock.sector(Na + Nb, Na)
        psi = np.zeros(fock.dim)
        psi[sec] = rng.normal(size=sec.size)
        psi /= np.linalg.norm(psi)
    h, V = gen.hamiltonian(rng, r, 6)
    ga, gb, aa, bb, ab = fm.spin_blocks_from_state(fock, psi)
    return dict(r=r, Na=Na, Nb=Nb, N=Na + Nb, h=h, V=V, gamma_a=ga, gamma_b=gb, d2aa=aa, d2bb=bb, d2ab=ab)


PROBLEMS = {
    "fock_doublet_r3": lambda: fock_problem(3, 2, 1, 1),
    "fock_triplet_r4": lambda: fock_problem(4, 3, 1, 2),
    "det_sz1_r4": lambda: fock_problem(4, 1, 3, 3, determinant=True),
    "r6_4_2": lambda: gen.spin_problem(6, 4, 2, 12, seed=1),
    "r9_5_4": lambda: gen.spin_problem(9, 5, 4, 18, seed=2),
    "r13_8_5": lambda: gen.spin_problem(13, 8, 5, 26, seed=3),
    "r16_9_6": lambda: gen.spin_problem(16, 9, 6, 32, seed=4),
    "r24_14_10": lambda: gen.spin_problem(24, 14, 10, 48, seed=5),
}


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_spin_residual_and_step(ctx, name):
    p = PROBLEMS[name]()
    print(f"[spin] {name} r={p['r']} Na={p['Na']} Nb={p['Nb']}", flush=True)
    raa, rbb, rab, n2 = ost.residual_spin(*_oracle_args(p))
    Raa, Rbb, Rab, gn2 = ctx.residual_spin(*_args(p))
    _check_blocks(dict(R_aa=Raa, R_bb=Rbb, R_ab=Rab), dict(R_aa=raa, R_bb=rbb, R_ab=rab), ("R_aa", "R_bb", "R_ab"))
    assert abs(gn2 - n2) <= TOL * n2
    o = ost.step_spin(*_oracle_args(p), 1e-3)
    g = ctx.step_spin(*_args(p), eps=1e-3, return_ru=True)
    _check_blocks(g, o, ("R_aa", "R_bb", "R_ab"))
    _check_blocks(g, o, ("U_aa", "U_bb", "U_ab"))
    _check_blocks(g, o, ("d2aa", "d2bb", "d2ab"))
    for k, ok in (("d1a", "gamma_a"), ("d1b", "gamma_b")):
        assert np.abs(cpu(g[k]) - o[ok]).max() <= TOL * max(np.abs(o[ok]).max(), 1.0), k
    assert abs(g["energy"] - o["energy"]) <= TOL * max(1.0, abs(o["energy"]))
    assert abs(g["norm2"] - o["norm2"]) <= TOL * o["norm2"]
    e0 = ctx.energy_spin(p["h"], p["V"], p["d2aa"], p["d2bb"], p["d2ab"], p["Na"], p["Nb"])
    assert abs(e0 - o["energy0"]) <= TOL * max(1.0, abs(o["energy0"]))


@pytest.mark.parametrize("r,Na,Nb", [(4, 3, 0), (5, 2, 0), (5, 4, 1), (3, 1, 1)])
def test_spin_edge_counts(ctx, r, Na, Nb):
    """An empty beta shell (beta blocks zero), a single beta electron (beta-beta
    block zero) and the smallest open- and closed-shell counts."""
    p = gen.spin_problem(r, Na, Nb, 2 * r, seed=50 + r + Na)
    print(f"[spin edge] r={r} Na={Na} Nb={Nb}", flush=True)
    o = ost.step_spin(*_oracle_args(p), 1e-3)
    g = ctx.step_spin(*_args(p), eps=1e-3, return_ru=True)
    for keys in (("R_aa", "R_bb", "R_ab"), ("U_aa", "U_bb", "U_ab"), ("d2aa", "d2bb", "d2ab")):
        scale = max(np.abs(o[k]).max() for k in keys)
        for k in keys:
            assert np.abs(cpu(g[k]) - o[k]).max() <= TOL * max(scale, 1e-300), k
    assert abs(g["energy"] - o["energy"]) <= TOL * max(1.0, abs(o["energy"]))


def test_spin_masked_step_and_general_kernels(acse, ctx):
    p = PROBLEMS["r13_8_5"]()
    act = np.zeros(13, bool)
    act[[1, 2, 5, 8, 11]] = True
    print("[spin] masked step r13, general kernels", flush=True)
    o = ost.step_spin(*_oracle_args(p), 1e-3, active=act)
    for flags in (0, acse.FLAG_GENERAL_KERNELS):
        g = ctx.step_spin(*_args(p), eps=1e-3, active=act, return_ru=True, flags=flags)
        _check_blocks(g, o, ("R_aa", "R_bb", "R_ab"))
        _check_blocks(g, o, ("U_aa", "U_bb", "U_ab"))
        _check_blocks(g, o, ("d2aa", "d2bb", "d2ab"))
        assert abs(g["energy"] - o["energy"]) <= TOL * abs(o["energy"])


def test_spin_path_on_singlet_inputs_matches_singlet_path(ctx):
    """A singlet given as three spin blocks: the spin-block path equals the
    singlet path (different kernels, same map) and R_bb = R_aa."""
    p = gen.problem(10, 6, 20, seed=2)
    g = ctx.step_spin(p["h"], p["V"], p["gamma"], p["gamma"], p["d2aa"], p["d2aa"], p["d2ab"], 3, 3, eps=1e-3,
                      return_ru=True)
    s = ctx.step(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], 3, eps=1e-3, return_ru=True)
    for k in ("R_aa", "R_ab", "U_aa", "U_ab", "d2aa", "d2ab"):
        a, b = cpu(g[k]), cpu(s[k])
        assert np.abs(a - b).max() <= TOL * np.abs(b).max(), k
    assert np.abs(cpu(g["R_bb"]) - cpu(s["R_aa"])).max() <= TOL * np.abs(cpu(s["R_aa"])).max()
    assert abs(g["energy"] - s["energy"]) <= TOL * abs(s["energy"])
    assert abs(g["norm2"] - s["norm2"]) <= TOL * s["norm2"]


def test_spin_step_identities_and_errors(acse, ctx):
    """E1 - E0 = -eps ||R||^2 + O(eps^2) and the per-block traces; unsupported
    options are refused; the singlet calls refuse n_alpha != n_beta."""
    p = PROBLEMS["r16_9_6"]()
    eps = 1e-7
    e0 = ctx.energy_spin(p["h"], p["V"], p["d2aa"], p["d2bb"], p["d2ab"], p["Na"], p["Nb"])
    g = ctx.step_spin(*_args(p), eps=eps)
    assert abs((g["energy"] - e0) + eps * g["norm2"]) <= 1e-5 * eps * g["norm2"]
    tr = lambda x: float(np.einsum("pqpq->", cpu(x) if not isinstance(x, np.ndarray) else x))
    for k in ("d2aa", "d2bb", "d2ab"):
        assert abs(tr(g[k]) - tr(p[k])) <= 1e-13 * max(1.0, abs(tr(p[k])))
    prob, keep = ctx.problem_spin(*_args(p))
    import torch
    R = [torch.empty((16,) * 4, dtype=torch.float64, device=ctx.device) for _ in range(3)]
    with pytest.raises(acse.AcseError, match="UNSUPPORTED"):
        ctx.residual_spin_raw(prob, ctx.options("fp32"), *R)
    with pytest.raises(acse.AcseError, match="UNSUPPORTED"):
        ctx.residual_spin_raw(prob, ctx.options("bf16x3"), *R)
    # NY occupations: one per spin orbital, each +1 or -1
    with pytest.raises(acse.AcseError, match="ARG"):
        ctx.residual_spin_raw(prob, ctx.options(sigma=[1, 0] + [-1] * 30), *R)
    with pytest.raises(ValueError, match="2r = 32 spin orbitals"):
        ctx.residual_spin_raw(prob, ctx.options(sigma=[1] * 16), *R)
    singlet, _ = ctx.problem(p["h"], p["V"], p["gamma_a"], p["d2aa"], p["d2ab"], p["Na"], n_beta=p["Nb"])
    with pytest.raises(acse.AcseError, match="_spin calls"):
        ctx.residual_raw(singlet, ctx.options(), R[0], R[1])


SPIN_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "r50_spin_step.json")


def test_r50_spin_step_vs_stored_oracle(acse):
    """Full size (r = 50, N_alpha = 16, N_beta = 14), the configuration the
    bench times: sampled elements of the R, U and new 2-RDM blocks, the block
    norms, ||R||^2, E before and after the step and both new 1-RDMs against the
    stored oracle values (tests/golden/make_golden_spin.py), FP64 at 1e-10."""
    g = json.load(open(SPIN_GOLDEN))
    p = gen.named_spin(g["workload"])
    assert (p["r"], p["Na"], p["Nb"]) == (g["r"], g["Na"], g["Nb"]) == (50, 16, 14)
    print("[spin fullsize] r50s step", flush=True)
    ctx = acse.Context(r_max=50)
    try:
        e0 = ctx.energy_spin(p["h"], p["V"], p["d2aa"], p["d2bb"], p["d2ab"], p["Na"], p["Nb"])
        out = ctx.step_spin(*_args(p), eps=g["eps"], return_ru=True)
        idx = tuple(np.array(g["index"]).T)
        for k in g["samples"]:
            got = cpu(out[k])
            ref = np.array(g["samples"][k])
            assert np.abs(got[idx] - ref).max() <= TOL * np.abs(ref).max(), k
            assert abs(np.linalg.norm(got) - g["norms"][k]) <= TOL * g["norms"][k], k
        assert abs(out["norm2"] - g["norm2"]) <= TOL * g["norm2"]
        assert abs(e0 - g["energy0"]) <= TOL * abs(g["energy0"])
        assert abs(out["energy"] - g["energy1"]) <= 1e-13 * abs(g["energy1"])
        assert abs(out["energy"] - g["energy1"]) < 1e-7
        for k, ok in (("d1a", "gamma_a"), ("d1b", "gamma_b")):
            assert np.abs(cpu(out[k]) - np.array(g[ok])).max() <= TOL, k
    finally:
        ctx.close()


@pytest.mark.parametrize("name", ["fock_triplet_r4", "det_sz1_r4", "r9_5_4", "r16_9_6", "r24_14_10"])
def test_spin_int8crt_residual_and_step(ctx, name):
    """The int8 exact-accumulation products on the spin-block path: the same
    FP64 bar against the oracle (the products are exact for operands rounded
    to k = 44+ bits)."""
    p = PROBLEMS[name]()
    print(f"[spin int8crt] {name}", flush=True)
    raa, rbb, rab, n2 = ost.residual_spin(*_oracle_args(p))
    Raa, Rbb, Rab, gn2 = ctx.residual_spin(*_args(p), precision="int8crt")
    _check_blocks(dict(R_aa=Raa, R_bb=Rbb, R_ab=Rab), dict(R_aa=raa, R_bb=rbb, R_ab=rab), ("R_aa", "R_bb", "R_ab"))
    assert abs(gn2 - n2) <= TOL * n2
    o = ost.step_spin(*_oracle_args(p), 1e-3)
    g = ctx.step_spin(*_args(p), eps=1e-3, return_ru=True, precision="int8crt")
    for keys in (("R_aa", "R_bb", "R_ab"), ("U_aa", "U_bb", "U_ab"), ("d2aa", "d2bb", "d2ab")):
        _check_blocks(g, o, keys)
    assert abs(g["energy"] - o["energy"]) <= TOL * max(1.0, abs(o["energy"]))


def test_spin_int8crt_moduli_and_masked_step(acse, ctx):
    """Fewer moduli (fewer operand bits) raise the error as 2^-k; a masked
    int8 step matches the oracle."""
    p = PROBLEMS["r13_8_5"]()
    raa, rbb, rab, n2 = ost.residual_spin(*_oracle_args(p))
    errs = []
    for m in (8, 10, 13):
        Raa, Rbb, Rab, gn2 = ctx.residual_spin(*_args(p), precision="int8crt", moduli=m)
        errs.append(max(np.abs(cpu(x) - y).max() for x, y in ((Raa, raa), (Rbb, rbb), (Rab, rab))))
    print(f"[spin int8crt] max errors for 8, 10, 13 moduli: {errs}", flush=True)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] <= TOL * max(np.abs(raa).max(), np.abs(rab).max())
    act = np.zeros(13, bool)
    act[[0, 3, 4, 9]] = True
    o = ost.step_spin(*_oracle_args(p), 1e-3, active=act)
    g = ctx.step_spin(*_args(p), eps=1e-3, active=act, return_ru=True, precision="int8crt")
    for keys in (("R_aa", "R_bb", "R_ab"), ("U_aa", "U_bb", "U_ab"), ("d2aa", "d2bb", "d2ab")):
        _check_blocks(g, o, keys)


def test_r50_spin_int8crt_step_vs_stored_oracle(acse):
    """Full size in the int8 mode: the stored oracle step at 1e-10 and
    |dE| < 1e-7 Eh."""
    g = json.load(open(SPIN_GOLDEN))
    p = gen.named_spin(g["workload"])
    print("[spin fullsize] r50s int8crt step", flush=True)
    ctx = acse.Context(r_max=50)
    try:
        out = ctx.step_spin(*_args(p), eps=g["eps"], return_ru=True, precision="int8crt")
        idx = tuple(np.array(g["index"]).T)
        for k in g["samples"]:
            got = cpu(out[k])
            ref = np.array(g["samples"][k])
            assert np.abs(got[idx] - ref).max() <= TOL * np.abs(ref).max(), k
            assert abs(np.linalg.norm(got) - g["norms"][k]) <= TOL * g["norms"][k], k
        assert abs(out["norm2"] - g["norm2"]) <= TOL * g["norm2"]
        assert abs(out["energy"] - g["energy1"]) < 1e-7
    finally:
        ctx.close()
