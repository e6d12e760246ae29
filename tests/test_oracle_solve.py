"""Pins of the oracle's Euler iteration (oracle/solve.py), CPU only.

* The slope f'(0) of f(eps) = ||R(2D + eps U)||^2 that the quadratic control
  takes from the adjoint equals central finite differences of the numpy
  forward along the step (trace restoration and the 1-RDM contraction
  included); without the 1-RDM term it does not (the pin sees that term).
* The quadratic model's step on parabolas with known minimisers, and its
  clamps.
* The fixed-step loop of the method section is repeated single Euler steps
  (oracle.step) while no rise occurs; it stops at the first rise of E or of
  ||R|| and returns the state before it; |dE| < de_tol stops it after the step.
* Backtracking halves the step size until a trial is acceptable; every
  rejected trial raises E or ||R||; the accepted one raises neither.
* Energies of accepted states decrease (E is linear along the step and its
  slope is -<R_m, R> up to a positive factor).
"""
import numpy as np
import pytest

from oracle import rdm
from oracle import solve as sv
from oracle import step as ost
from synth import generators as gen


def consistent(p):
    """The problem with gamma replaced by the contraction of its 2-RDM."""
    r = p["r"]
    _, d2 = rdm.blocks_to_spin_orbital(np.eye(r), p["d2aa"], p["d2ab"])
    q = dict(p)
    q["gamma"] = rdm.contract_to_1rdm(d2, p["N"])[:r, :r]
    return q


@pytest.fixture(scope="module")
def r6():
    return consistent(gen.problem(6, 4, 12, seed=1))


def run(p, **kw):
    return sv.euler(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], **kw)


@pytest.mark.parametrize("name", ["r4", "r6"])
def test_norm_slope_matches_finite_differences(name):
    p = consistent(gen.problem(4, 4, 6, seed=7) if name == "r4" else gen.problem(6, 4, 12, seed=1))
    o = ost.step(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], 0.0)
    g0 = sv.norm_slope(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], o["R_aa"], o["R_ab"],
                       o["U_aa"], o["U_ab"])
    K = rdm.reduced_hamiltonian(p["h"], p["V"], p["N"])

    def f(x):
        a, b, g1, _ = sv._trial(K, p["N"], p["d2aa"], p["d2ab"], o["U_aa"], o["U_ab"], x)
        return sv._residual(K, g1, a, b)[1]

    h = 1e-6
    fd = (f(h) - f(-h)) / (2 * h)
    assert abs(g0 - fd) <= 1e-6 * abs(fd)
    # the 1-RDM's dependence on 2D is part of the slope
    from oracle import adjoint
    g = adjoint.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"],
                             4.0 * o["R_aa"], 8.0 * o["R_ab"])
    g_no_gamma = float(np.sum(g["d2aa"] * o["U_aa"]) + np.sum(g["d2ab"] * o["U_ab"]))
    assert abs(g_no_gamma - fd) > 1e-3 * abs(fd)


@pytest.mark.parametrize("name", ["r4", "r6"])
def test_norm_slope_ny_matches_finite_differences(name):
    """The slope with the NY 3-RDM (its adjoint) against central differences
    of the NY norm along the NY update direction."""
    p = consistent(gen.problem(4, 4, 6, seed=7) if name == "r4" else gen.problem(6, 4, 12, seed=1))
    r = p["r"]
    sig = [1 if q % 3 != 2 else -1 for q in range(r)]
    sso = rdm.sigma_spin_orbital(sig)
    o = ost.step(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], 0.0, sigma=sig)
    g0 = sv.norm_slope(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], o["R_aa"], o["R_ab"],
                       o["U_aa"], o["U_ab"], sigma=sig)
    K = rdm.reduced_hamiltonian(p["h"], p["V"], p["N"])

    def f(x):
        a, b, g1, _ = sv._trial(K, p["N"], p["d2aa"], p["d2ab"], o["U_aa"], o["U_ab"], x)
        return sv._residual(K, g1, a, b, sso)[1]

    h = 1e-6
    fd = (f(h) - f(-h)) / (2 * h)
    assert abs(g0 - fd) <= 1e-6 * abs(fd)
    # the Valdemoro slope along the same direction is another number
    gv = sv.norm_slope(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], o["R_aa"], o["R_ab"],
                       o["U_aa"], o["U_ab"])
    assert abs(gv - fd) > 1e-3 * abs(fd)


def test_quadratic_trial_step():
    # f = 3 - 2x + 5x^2: minimiser 0.2
    f = lambda x: 3.0 - 2.0 * x + 5.0 * x * x
    assert sv.quadratic_trial_step(3.0, -2.0, 0.1, f(0.1), 1.0) == pytest.approx(0.2, rel=1e-14)
    # minimiser 1.0 clamped to 4 eps
    f = lambda x: 1.0 - 2.0 * x + x * x
    assert sv.quadratic_trial_step(1.0, -2.0, 0.1, f(0.1), 1.0) == pytest.approx(0.4, rel=1e-14)
    # ... and to eps_max
    assert sv.quadratic_trial_step(1.0, -2.0, 0.1, f(0.1), 0.3) == pytest.approx(0.3, rel=1e-14)
    # minimiser 0.001 clamped to eps/4
    f = lambda x: 1.0 - 2.0 * x + 1000.0 * x * x
    assert sv.quadratic_trial_step(1.0, -2.0, 0.1, f(0.1), 1.0) == pytest.approx(0.025, rel=1e-14)
    # non-positive curvature: 4 eps
    assert sv.quadratic_trial_step(1.0, -2.0, 0.1, 1.0 - 0.2 - 0.01, 1.0) == pytest.approx(0.4)
    # ascending start, and a minimiser within 5% of eps: no second trial
    assert sv.quadratic_trial_step(1.0, 2.0, 0.1, 1.3, 1.0) is None
    f = lambda x: 1.0 - 2.0 * x + 10.2 * x * x  # minimiser 0.098
    assert sv.quadratic_trial_step(1.0, -2.0, 0.1, f(0.1), 1.0) is None


def test_fixed_loop_is_repeated_euler_steps(r6):
    p = r6
    o = run(p, eps=1e-3, de_tol=0.0, max_iter=3)
    assert o["iterations"] == 3 and o["stop"] == sv.STOP_MAX_ITER
    g, a, b = p["gamma"], p["d2aa"], p["d2ab"]
    energies = []
    for _ in range(3):
        s = ost.step(p["h"], p["V"], p["N"], g, a, b, 1e-3)
        g, a, b = s["gamma"], s["d2aa"], s["d2ab"]
        energies.append(s["energy"])
    for x, y in ((o["d2aa"], a), (o["d2ab"], b), (o["gamma"], g)):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(y).max()
    assert [t[1] for t in o["trials"]] == pytest.approx(energies, rel=1e-13)
    assert all(t[4] for t in o["trials"])
    assert np.all(np.diff([o["energy0"]] + energies) < 0)


def test_stop_on_energy_rise_returns_input(r6):
    p = r6
    o = run(p, eps=-1e-3, de_tol=0.0, max_iter=5)
    assert o["stop"] == sv.STOP_ENERGY_ROSE and o["iterations"] == 0
    assert len(o["trials"]) == 1 and o["trials"][0][1] > o["energy0"]
    assert np.array_equal(o["d2aa"], p["d2aa"]) and np.array_equal(o["d2ab"], p["d2ab"])
    assert np.array_equal(o["gamma"], p["gamma"])
    assert o["energy"] == o["energy0"] and o["norm2"] == o["norm2_0"]


def test_stop_on_norm_rise_returns_input():
    # a 1-RDM that is not the contraction of the 2-RDM: the first step moves it
    # onto the contraction and the residual norm jumps up
    p = gen.problem(6, 4, 12, seed=1)
    o = run(p, eps=1e-3, de_tol=0.0, max_iter=5)
    assert o["stop"] == sv.STOP_NORM_ROSE and o["iterations"] == 0
    t = o["trials"][0]
    assert t[1] <= o["energy0"] and t[2] > o["norm2_0"]
    assert np.array_equal(o["d2aa"], p["d2aa"]) and np.array_equal(o["gamma"], p["gamma"])


def test_energy_change_threshold_stops_after_the_step(r6):
    o = run(r6, eps=1e-3, de_tol=1.0, max_iter=5)
    assert o["stop"] == sv.STOP_CONVERGED and o["iterations"] == 1
    s = ost.step(r6["h"], r6["V"], r6["N"], r6["gamma"], r6["d2aa"], r6["d2ab"], 1e-3)
    assert o["energy"] == pytest.approx(s["energy"], rel=1e-13)
    assert run(r6, max_iter=0)["trials"] == []


def test_backtracking_rule(r6):
    o = run(r6, eps=0.1, de_tol=0.0, max_iter=5, control=sv.BACKTRACK, max_halvings=20)
    E, f = o["energy0"], o["norm2_0"]
    steps = {}
    for t in o["trials"]:
        steps.setdefault(t[3], []).append(t)
    assert len(steps) >= 3
    eps = 0.1
    for n in sorted(steps):
        ts = steps[n]
        assert ts[0][0] == eps
        for a, b in zip(ts, ts[1:]):
            assert b[0] == 0.5 * a[0]
        for t in ts[:-1]:
            assert not t[4] and (t[1] > E or t[2] > f)
        last = ts[-1]
        if last[4]:
            assert last[1] <= E and last[2] <= f
            E, f, eps = last[1], last[2], last[0]
    assert steps[0][0][4] is False  # the first step at 0.1 overshoots
    assert o["energy"] == E and o["norm2"] == f


def test_quadratic_control_lowers_the_norm_faster(r6):
    fixed = run(r6, eps=1e-3, de_tol=0.0, max_iter=6)
    quad = run(r6, eps=1e-3, de_tol=0.0, max_iter=6, control=sv.QUADRATIC)
    assert fixed["iterations"] == quad["iterations"] == 6
    assert quad["norm2"] < 0.5 * fixed["norm2"]
    assert quad["energy"] < fixed["energy"]
    accepted = [t for t in quad["trials"] if t[4]]
    assert np.all(np.diff([quad["norm2_0"]] + [t[2] for t in accepted]) <= 0)


def test_euler_spin_on_singlet_inputs_is_the_singlet_iteration():
    """The spin-block iteration on a singlet given as three blocks (beta =
    alpha, pair-exchange symmetric alpha-beta) takes the singlet iteration's
    trials, decisions and final state; with backtracking from a step size that
    raises ||R|| the halvings agree too."""
    from oracle import solve as sv
    p = gen.problem(5, 4, 10, seed=3)
    args = (p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"])
    for eps, ctrl in ((1e-3, sv.FIXED), (0.2, sv.BACKTRACK)):
        s = sv.euler(*args, eps=eps, de_tol=0.0, max_iter=3, control=ctrl, max_halvings=4)
        g = sv.euler_spin(p["h"], p["V"], 2, 2, p["gamma"], p["gamma"], p["d2aa"], p["d2aa"], p["d2ab"],
                          eps=eps, de_tol=0.0, max_iter=3, control=ctrl, max_halvings=4)
        assert g["stop"] == s["stop"] and g["iterations"] == s["iterations"]
        assert len(g["trials"]) == len(s["trials"])
        for a, b in zip(g["trials"], s["trials"]):
            assert a[0] == b[0] and a[3:] == b[3:]
            assert abs(a[1] - b[1]) < 1e-11 * abs(b[1]) and abs(a[2] - b[2]) < 1e-11 * b[2]
        for k, ref in (("d2aa", s["d2aa"]), ("d2bb", s["d2aa"]), ("d2ab", s["d2ab"]), ("ga", s["gamma"])):
            assert np.abs(g[k] - ref).max() < 1e-12 * max(1.0, np.abs(ref).max()), k


def _spin_line(ny):
    """An open-shell state with its 1-RDMs contracted from its 2-RDM, the
    update direction U of its step and f(s) = ||R(2D + s U, 1D + s dD)||^2."""
    p = gen.spin_problem(5, 3, 1, 10, seed=2)
    z = np.zeros((5, 5))
    _, d2 = rdm.spin_blocks_to_spin_orbital(z, z, p["d2aa"], p["d2bb"], p["d2ab"])
    g = rdm.contract_to_1rdm(d2, 4)
    ga, gb = g[:5, :5].copy(), g[5:, 5:].copy()
    sig = ost.sigma_open_shell(5, 3, 1) if ny else None
    blocks = (p["d2aa"], p["d2bb"], p["d2ab"])
    o = ost.step_spin(p["h"], p["V"], 3, 1, ga, gb, *blocks, 0.0, sigma_so=sig)
    U = (o["U_aa"], o["U_bb"], o["U_ab"])
    _, u2 = rdm.spin_blocks_to_spin_orbital(z, z, *U)
    u1 = rdm.contract_to_1rdm(u2, 4)

    def R(s):
        bl = [b + s * u for b, u in zip(blocks, U)]
        return ost.residual_spin(p["h"], p["V"], 3, 1, ga + s * u1[:5, :5], gb + s * u1[5:, 5:], *bl, sigma_so=sig)

    return p, ga, gb, blocks, U, sig, R


@pytest.mark.parametrize("ny", [False, True])
def test_norm_slope_spin_matches_finite_differences(ny):
    """The open-shell slope (autograd along the line) against central
    differences of the numpy forward's ||R||^2."""
    from oracle import solve as sv
    p, ga, gb, blocks, U, sig, R = _spin_line(ny)
    g0 = sv.norm_slope_spin(p["h"], p["V"], 3, 1, ga, gb, *blocks, *U, sigma_so=sig)
    h = 1e-6
    fd = (R(h)[3] - R(-h)[3]) / (2 * h)
    assert abs(g0 - fd) <= 1e-8 * abs(fd)


@pytest.mark.parametrize("ny", [False, True])
def test_residual_is_quartic_along_a_line(ny):
    """Along a straight line in (2D, 1D) the residual is a polynomial of degree
    at most 4 in the line parameter (the Valdemoro 3-RDM cubic, the NY one
    quartic in the RDMs): the five-point central difference of R at a large
    step equals the exact directional derivative (the autograd slope), while
    the three-point one (exact to degree 2) does not."""
    from oracle import solve as sv
    p, ga, gb, blocks, U, sig, R = _spin_line(ny)
    g0 = sv.norm_slope_spin(p["h"], p["V"], 3, 1, ga, gb, *blocks, *U, sigma_so=sig)
    H = 0.3
    R0 = R(0.0)[:3]
    Rh, Rm, R2h, R2m = (R(x)[:3] for x in (H, -H, 2 * H, -2 * H))
    w = (1.0, 1.0, 4.0)  # spin-orbital norm weights of the aa, bb, ab blocks

    def slope(d):
        return 2.0 * sum(c * float(np.sum(a * b)) for c, a, b in zip(w, R0, d))
    five = slope([(8.0 * (a - b) - (c - e)) / (12.0 * H) for a, b, c, e in zip(Rh, Rm, R2h, R2m)])
    three = slope([(a - b) / (2.0 * H) for a, b in zip(Rh, Rm)])
    assert abs(five - g0) <= 1e-12 * abs(g0)
    assert abs(three - g0) > 1e-6 * abs(g0)


def test_euler_spin_quadratic_on_singlet_inputs_is_the_singlet_iteration():
    """The quadratic control of the spin-block iteration (its slope by
    autograd along the line) on a singlet given as three blocks takes the
    singlet iteration's trials (slope from the singlet adjoint)."""
    from oracle import solve as sv
    p = gen.problem(5, 4, 10, seed=3)
    _, d2 = rdm.blocks_to_spin_orbital(np.eye(5), p["d2aa"], p["d2ab"])
    g1 = rdm.contract_to_1rdm(d2, 4)[:5, :5]
    s = sv.euler(p["h"], p["V"], 4, g1, p["d2aa"], p["d2ab"], eps=1e-2, de_tol=0.0, max_iter=3,
                 control=sv.QUADRATIC, max_halvings=4)
    g = sv.euler_spin(p["h"], p["V"], 2, 2, g1, g1, p["d2aa"], p["d2aa"], p["d2ab"], eps=1e-2, de_tol=0.0,
                      max_iter=3, control=sv.QUADRATIC, max_halvings=4)
    assert len(s["trials"]) > s["iterations"]  # a second (interpolated) trial was taken
    assert g["stop"] == s["stop"] and g["iterations"] == s["iterations"]
    assert len(g["trials"]) == len(s["trials"])
    for a, b in zip(g["trials"], s["trials"]):
        assert abs(a[0] - b[0]) <= 1e-9 * abs(b[0]) and a[3:] == b[3:]
        assert abs(a[1] - b[1]) < 1e-10 * abs(b[1]) and abs(a[2] - b[2]) < 1e-10 * b[2]


@pytest.mark.parametrize("ny", [False, True])
def test_euler_spin_steps_are_step_spin_steps(ny):
    """Every accepted fixed-eps step of the spin-block iteration is one
    step_spin of the state before it (energy and blocks), with either 3-RDM
    reconstruction."""
    from oracle import rdm
    from oracle import solve as sv
    from oracle import step as st
    p = gen.spin_problem(5, 3, 1, 10, seed=2)
    z = np.zeros((5, 5))
    _, d2 = rdm.spin_blocks_to_spin_orbital(z, z, p["d2aa"], p["d2bb"], p["d2ab"])
    g = rdm.contract_to_1rdm(d2, 4)
    ga, gb = g[:5, :5].copy(), g[5:, 5:].copy()
    sig = st.sigma_open_shell(5, 3, 1) if ny else None
    o = sv.euler_spin(p["h"], p["V"], 3, 1, ga, gb, p["d2aa"], p["d2bb"], p["d2ab"], eps=1e-2, de_tol=0.0,
                      max_iter=2, sigma_so=sig)
    s1 = st.step_spin(p["h"], p["V"], 3, 1, ga, gb, p["d2aa"], p["d2bb"], p["d2ab"], 1e-2, sigma_so=sig)
    s2 = st.step_spin(p["h"], p["V"], 3, 1, s1["gamma_a"], s1["gamma_b"], s1["d2aa"], s1["d2bb"], s1["d2ab"], 1e-2,
                      sigma_so=sig)
    assert o["iterations"] == 2 and [t[4] for t in o["trials"]] == [True, True]
    assert abs(o["trials"][0][1] - s1["energy"]) < 1e-12 * abs(s1["energy"])
    assert abs(o["energy"] - s2["energy"]) < 1e-12 * abs(s2["energy"])
    for k in ("d2aa", "d2bb", "d2ab"):
        assert np.abs(o[k] - s2[k]).max() <= 1e-13 * np.abs(s2[k]).max(), k
