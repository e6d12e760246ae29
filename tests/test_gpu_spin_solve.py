"""GPU parity of the open-shell Euler iteration (acse_solve_spin) with the
oracle's spin-block iteration.

Both sides take every accept/reject decision from their own E and ||R||^2;
the cases are chosen so that each decision clears its threshold by a relative
3e-3 or more in the oracle (far above the 1e-10 parity bar), so the two
trajectories must agree trial by trial: step sizes exactly, E and ||R||^2 of
every trial and the returned blocks and 1-RDMs to 1e-10 relative.  The cases
cover all four stop reasons, fixed and backtracking control, the active mask
and the int8 exact-accumulation products.
"""
import numpy as np
import pytest

from oracle import fermion as fm
from oracle import rdm
from oracle import solve as osv
from oracle import step as ost
from synth import generators as gen

pytestmark = pytest.mark.gpu

TOL = 1e-10
STOPS = {osv.STOP_MAX_ITER: "max_iter", osv.STOP_CONVERGED: "converged", osv.STOP_ENERGY_ROSE: "energy_rose",
         osv.STOP_NORM_ROSE: "norm_rose"}


@pytest.fixture(scope="module")
def acse():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2604_02550_amd as acse
    return acse


@pytest.fixture(scope="module")
def ctx(acse):
    return acse.Context(r_max=16)


def cpu(t):
    return t.detach().cpu().numpy()


def consistent(p):
    """The problem with both 1-RDMs replaced by the contraction of its 2-RDM."""
    r = p["h"].shape[0]
    z = np.zeros((r, r))
    _, d2 = rdm.spin_blocks_to_spin_orbital(z, z, p["d2aa"], p["d2bb"], p["d2ab"])
    g = rdm.contract_to_1rdm(d2, p["Na"] + p["Nb"])
    return dict(p, gamma_a=g[:r, :r].copy(), gamma_b=g[r:, r:].copy())


def fock_problem(r, Na, Nb, seed):
    """Exact blocks of a random state of the (Na, Nb) sector."""
    rng = np.random.default_rng(seed)
    fock = fm.Fock(2 * r)
    sec = fock.sector(Na + Nb, Na)
    psi = np.zeros(fock.dim)
    psi[sec] = rng.normal(size=sec.size)
    psi /= np.linalg.norm(psi)
    h, V = gen.hamiltonian(rng, r, 6)
    ga, gb, aa, bb, ab = fm.spin_blocks_from_state(fock, psi)
    return dict(r=r, Na=Na, Nb=Nb, h=h, V=V, gamma_a=ga, gamma_b=gb, d2aa=aa, d2bb=bb, d2ab=ab)


def compare(ctx, p, eps, de_tol, max_iter, control, max_halvings=8, active=None, precision="fp64"):
    o = osv.euler_spin(p["h"], p["V"], p["Na"], p["Nb"], p["gamma_a"], p["gamma_b"], p["d2aa"], p["d2bb"],
                       p["d2ab"], eps=eps, de_tol=de_tol, max_iter=max_iter,
                       control=osv.BACKTRACK if control == "backtrack" else osv.FIXED, max_halvings=max_halvings,
                       active=active)
    g = ctx.solve_spin(p["h"], p["V"], p["gamma_a"], p["gamma_b"], p["d2aa"], p["d2bb"], p["d2ab"], p["Na"],
                       p["Nb"], eps=eps, de_tol=de_tol, max_iter=max_iter, control=control,
                       max_halvings=max_halvings, active=active, precision=precision)
    assert g["stop"] == STOPS[o["stop"]]
    assert g["iterations"] == o["iterations"]
    assert g["trial_count"] == len(o["trials"])
    # one residual per state evaluated, one update direction per step taken
    assert g["maps"] == 1 + len(o["trials"]) + len({t[3] for t in o["trials"]})
    for a, b in zip(g["trials"], o["trials"]):
        assert a[0] == b[0] and a[3] == b[3] and a[4] == b[4]
        assert abs(a[1] - b[1]) <= TOL * max(1.0, abs(b[1]))
        assert abs(a[2] - b[2]) <= TOL * b[2]
    for k in ("energy0", "energy"):
        assert abs(g[k] - o[k]) <= TOL * max(1.0, abs(o[k])), k
    for k in ("norm2_0", "norm2"):
        assert abs(g[k] - o[k]) <= TOL * o[k], k
    assert g["eps"] == o["eps_last"]
    scale = max(np.abs(o[k]).max() for k in ("d2aa", "d2bb", "d2ab"))
    for k in ("d2aa", "d2bb", "d2ab"):
        assert np.abs(cpu(g[k]) - o[k]).max() <= TOL * scale, k
    for k, ok in (("d1a", "ga"), ("d1b", "gb")):
        assert np.abs(cpu(g[k]) - o[ok]).max() <= TOL * max(1.0, np.abs(o[ok]).max()), k
    return g, o


CASES = {
    # six accepted fixed steps
    "r6_fixed": (lambda: consistent(gen.spin_problem(6, 4, 2, 12, seed=1)), dict(eps=1e-2, de_tol=0.0, max_iter=6,
                                                                                control="fixed")),
    # the second trial raises ||R||: the state after one step comes back
    "r6_norm_rose": (lambda: consistent(gen.spin_problem(6, 4, 2, 12, seed=2)),
                     dict(eps=1e-2, de_tol=0.0, max_iter=6, control="fixed")),
    # |dE| of the fourth step (1.015) is the first below de_tol = 1.1
    "r6_converged": (lambda: consistent(gen.spin_problem(6, 4, 2, 12, seed=1)),
                     dict(eps=1e-2, de_tol=1.1, max_iter=10, control="fixed")),
    # a negative step size climbs: the first trial raises E
    "fock_energy_rose": (lambda: fock_problem(4, 3, 1, 2), dict(eps=-0.05, de_tol=0.0, max_iter=3, control="fixed")),
    # two halvings before each of two acceptances; the step size carries over
    "fock_backtrack": (lambda: fock_problem(4, 3, 1, 2),
                       dict(eps=0.1, de_tol=0.0, max_iter=4, control="backtrack", max_halvings=4)),
    # six halvings before the first acceptance; tiles with ragged tails (r^2 = 169)
    "r13_backtrack": (lambda: consistent(gen.spin_problem(13, 8, 5, 26, seed=3)),
                      dict(eps=0.05, de_tol=0.0, max_iter=3, control="backtrack", max_halvings=6)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_solve_spin_matches_oracle_iteration(ctx, name):
    make, kw = CASES[name]
    p = make()
    print(f"[solve_spin] {name} r={p['h'].shape[0]} Na={p['Na']} Nb={p['Nb']} {kw}", flush=True)
    compare(ctx, p, **kw)


@pytest.mark.parametrize("precision", ["fp64", "int8crt"])
def test_solve_spin_masked(ctx, precision):
    """The active mask (all-active elements of R dropped before the update
    direction) in both product modes."""
    p = consistent(gen.spin_problem(9, 5, 4, 18, seed=2))
    act = np.zeros(9, bool)
    act[[1, 2, 5, 7]] = True
    print(f"[solve_spin] r9 masked {precision}", flush=True)
    compare(ctx, p, eps=1e-3, de_tol=0.0, max_iter=3, control="fixed", active=act, precision=precision)


def test_solve_spin_int8crt_backtrack(ctx):
    p = fock_problem(4, 3, 1, 2)
    print("[solve_spin] fock backtrack int8crt", flush=True)
    compare(ctx, p, eps=0.1, de_tol=0.0, max_iter=4, control="backtrack", max_halvings=4, precision="int8crt")


def test_solve_spin_on_singlet_inputs_matches_singlet_solve(ctx):
    """A singlet given as three spin blocks: the spin-block iteration takes the
    singlet iteration's trials (different kernels, same method)."""
    p = gen.problem(8, 6, 16, seed=4)
    # the 1-RDM contracted from the 2-RDM: two halvings, then accepted steps
    g1 = consistent(dict(p, Na=3, Nb=3, d2bb=p["d2aa"]))["gamma_a"]
    print("[solve_spin] singlet inputs r8", flush=True)
    kw = dict(eps=1e-2, de_tol=0.0, max_iter=3, control="backtrack", max_halvings=3)
    g = ctx.solve_spin(p["h"], p["V"], g1, g1, p["d2aa"], p["d2aa"], p["d2ab"], 3, 3, **kw)
    s = ctx.solve(p["h"], p["V"], g1, p["d2aa"], p["d2ab"], 3, **kw)
    assert [t[4] for t in s["trials"]] == [False, False, True, True, True]
    assert g["stop"] == s["stop"] and g["iterations"] == s["iterations"]
    assert len(g["trials"]) == len(s["trials"])
    for a, b in zip(g["trials"], s["trials"]):
        assert a[0] == b[0] and a[3:] == b[3:]
        assert abs(a[1] - b[1]) <= TOL * abs(b[1]) and abs(a[2] - b[2]) <= TOL * b[2]
    for k, ref in (("d2aa", "d2aa"), ("d2bb", "d2aa"), ("d2ab", "d2ab"), ("d1a", "d1"), ("d1b", "d1")):
        a, b = cpu(g[k]), cpu(s[ref])
        assert np.abs(a - b).max() <= TOL * np.abs(b).max(), k


def test_solve_spin_zero_steps_and_refusals(acse, ctx):
    """max_iter = 0 evaluates the input state only and leaves it unchanged;
    unsupported precisions and bad options (an uphill step size for the
    quadratic control) are refused."""
    p = consistent(gen.spin_problem(6, 4, 2, 12, seed=1))
    args = (p["h"], p["V"], p["gamma_a"], p["gamma_b"], p["d2aa"], p["d2bb"], p["d2ab"], 4, 2)
    g = ctx.solve_spin(*args, eps=1e-2, max_iter=0)
    assert g["stop"] == "max_iter" and g["iterations"] == 0 and g["trial_count"] == 0 and g["maps"] == 1
    assert g["energy"] == g["energy0"] and g["norm2"] == g["norm2_0"]
    for k in ("d2aa", "d2bb", "d2ab"):
        assert np.array_equal(cpu(g[k]), p[k]), k
    e0 = ctx.energy_spin(p["h"], p["V"], p["d2aa"], p["d2bb"], p["d2ab"], 4, 2)
    assert abs(g["energy0"] - e0) <= TOL * max(1.0, abs(e0))
    with pytest.raises(acse.AcseError, match="ARG"):
        ctx.solve_spin(*args, control="quadratic", eps=-1e-2)
    with pytest.raises(acse.AcseError, match="UNSUPPORTED"):
        ctx.solve_spin(*args, precision="fp32")
    with pytest.raises(acse.AcseError, match="ARG"):
        ctx.solve_spin(*args, eps=0.0)
    with pytest.raises(acse.AcseError, match="ARG"):
        ctx.solve_spin(*args, max_halvings=61, control="backtrack")


# (problem, first step size, NY, precision): interpolated second trials that
# are taken, first trials kept after a second one (evaluated again), rejected
# first trials; every decision clears its threshold by 2.9e-4 relative or more
QUAD_CASES = {
    "r6": (lambda: consistent(gen.spin_problem(6, 4, 2, 12, seed=1)), 1e-2, False, "fp64"),
    "fock": (lambda: fock_problem(4, 3, 1, 2), 0.05, False, "fp64"),
    "fock_ny": (lambda: fock_problem(4, 3, 1, 2), 0.05, True, "fp64"),
    "r9_int8crt": (lambda: consistent(gen.spin_problem(9, 5, 4, 18, seed=2)), 1e-3, False, "int8crt"),
    "r6_ny": (lambda: consistent(gen.spin_problem(6, 4, 2, 12, seed=1)), 1e-2, True, "fp64"),
}


@pytest.mark.parametrize("name", list(QUAD_CASES))
def test_solve_spin_quadratic_matches_oracle_iteration(ctx, name):
    """The quadratic control for states of any S_z: the GPU takes f'(0) from the
    five-point central difference of R along the step (exact for the residual's
    polynomial dependence on the step), the oracle by autograd.  The second
    step size is a ratio of differences (two digits lost to cancellation), so
    the step sizes are compared at 1e-7 and the scalars and arrays at 1e-8, as
    for the singlet quadratic control."""
    make, eps, ny, precision = QUAD_CASES[name]
    p = make()
    r = p["h"].shape[0]
    sig = ost.sigma_open_shell(r, p["Na"], p["Nb"]) if ny else None
    print(f"[solve_spin quadratic] {name}", flush=True)
    o = osv.euler_spin(p["h"], p["V"], p["Na"], p["Nb"], p["gamma_a"], p["gamma_b"], p["d2aa"], p["d2bb"],
                       p["d2ab"], eps=eps, de_tol=0.0, max_iter=4, control=osv.QUADRATIC, max_halvings=6,
                       sigma_so=sig)
    g = ctx.solve_spin(p["h"], p["V"], p["gamma_a"], p["gamma_b"], p["d2aa"], p["d2bb"], p["d2ab"], p["Na"],
                       p["Nb"], eps=eps, de_tol=0.0, max_iter=4, control="quadratic", max_halvings=6,
                       precision=precision, sigma=True if ny else None)
    assert g["stop"] == STOPS[o["stop"]]
    assert g["iterations"] == o["iterations"]
    assert g["trial_count"] == len(o["trials"])
    # per step: U, four residuals along the line, one per trial (and one more
    # when a first trial is kept after a second)
    steps = len({t[3] for t in o["trials"]})
    assert g["maps"] >= 1 + 5 * steps + len(o["trials"])
    for a, b in zip(g["trials"], o["trials"]):
        assert a[3] == b[3] and a[4] == b[4]
        assert abs(a[0] - b[0]) <= 1e-7 * abs(b[0])
        assert abs(a[1] - b[1]) <= 1e-8 * max(1.0, abs(b[1]))
        assert abs(a[2] - b[2]) <= 1e-8 * b[2]
    scale = max(np.abs(o[k]).max() for k in ("d2aa", "d2bb", "d2ab"))
    for k in ("d2aa", "d2bb", "d2ab"):
        assert np.abs(cpu(g[k]) - o[k]).max() <= 1e-8 * scale, k


def test_solve_spin_quadratic_on_singlet_inputs_matches_singlet_solve(ctx):
    """On a singlet given as three blocks, the spin-block quadratic control
    (slope from the five-point difference along the line) takes the trials of
    the singlet quadratic control (slope from the hand-written adjoint)."""
    p = gen.problem(5, 4, 10, seed=3)
    g1 = consistent(dict(p, Na=2, Nb=2, d2bb=p["d2aa"]))["gamma_a"]
    print("[solve_spin quadratic] singlet inputs r5", flush=True)
    kw = dict(eps=1e-2, de_tol=0.0, max_iter=3, control="quadratic", max_halvings=4)
    g = ctx.solve_spin(p["h"], p["V"], g1, g1, p["d2aa"], p["d2aa"], p["d2ab"], 2, 2, **kw)
    s = ctx.solve(p["h"], p["V"], g1, p["d2aa"], p["d2ab"], 2, **kw)
    assert len(s["trials"]) > s["iterations"]  # second (interpolated) trials were taken
    assert g["stop"] == s["stop"] and g["iterations"] == s["iterations"]
    assert len(g["trials"]) == len(s["trials"])
    for a, b in zip(g["trials"], s["trials"]):
        assert a[3:] == b[3:]
        assert abs(a[0] - b[0]) <= 1e-7 * abs(b[0])
        assert abs(a[1] - b[1]) <= 1e-8 * abs(b[1]) and abs(a[2] - b[2]) <= 1e-8 * b[2]
