"""Pins of the oracle for states of any S_z (N_alpha != N_beta), against
Fock-space brute force (CPU).

The three unique spin blocks named in the Theory section (alpha-alpha,
beta-beta, alpha-beta) are lifted to spin orbitals by the fermionic
antisymmetry alone; every pin below would fail for a wrong sign or index order
of a mixed block, for beta blocks taken from the alpha ones, or for a norm or
energy that counted the mixed blocks twice.
"""
import numpy as np
import pytest

from oracle import fermion as fm
from oracle import rdm
from oracle import residual as rs
from oracle import step as st
from synth import generators as gen


def _state(r, Na, Nb, seed):
    rng = np.random.default_rng(seed)
    fock = fm.Fock(2 * r)
    sec = fock.sector(Na + Nb, Na)
    psi = np.zeros(fock.dim)
    psi[sec] = rng.normal(size=sec.size)
    return rng, fock, psi / np.linalg.norm(psi)


def _open_shell_determinant(fock, rng, r, Na, Nb):
    """A determinant with N_a alpha and N_b beta orbitals, each spin rotated by
    its own random orthogonal matrix (exact for the Valdemoro 3-RDM)."""
    Ua, Ub = gen.haar_orthogonal(rng, r), gen.haar_orthogonal(rng, r)
    C = np.zeros((2 * r, Na + Nb))
    C[:r, :Na] = Ua[:, :Na]
    C[r:, Na:] = Ub[:, :Nb]
    return fm.rotated_determinant(fock, C)


SECTORS = [(3, 2, 1), (4, 3, 1), (4, 1, 3), (4, 3, 0)]   # doublet, triplet, S_z = -1, S_z = 3/2


@pytest.mark.parametrize("r,Na,Nb", SECTORS)
def test_spin_block_lift_round_trip(r, Na, Nb):
    """The blocks of an exact Fock-space state lift back to its full spin-orbital
    1- and 2-RDM, zero blocks included."""
    rng, fock, psi = _state(r, Na, Nb, 11 + r + Na)
    d1 = fock.rdm1(psi)
    d2 = fock.rdm2(psi) / 2.0
    ga, gb, aa, bb, ab = fm.spin_blocks_from_state(fock, psi)
    l1, l2 = rdm.spin_blocks_to_spin_orbital(ga, gb, aa, bb, ab)
    assert np.abs(l1 - d1).max() < 1e-14
    assert np.abs(l2 - d2).max() < 1e-14
    # App. A traces of the three blocks and the 1-RDM contraction per spin
    tr = lambda b: np.einsum('pqpq->', b)
    assert abs(tr(aa) - Na * (Na - 1) / 2) < 1e-12 and abs(tr(bb) - Nb * (Nb - 1) / 2) < 1e-12
    assert abs(tr(ab) - Na * Nb / 2) < 1e-12
    g = rdm.contract_to_1rdm(l2, Na + Nb)
    assert np.abs(g[:r, :r] - ga).max() < 1e-12 and np.abs(g[r:, r:] - gb).max() < 1e-12


@pytest.mark.parametrize("r,Na,Nb", SECTORS)
def test_energy_spin_equals_expectation(r, Na, Nb):
    rng, fock, psi = _state(r, Na, Nb, 21 + r)
    h, V = gen.hamiltonian(rng, r, 6)
    hso, gso = fm.spin_orbital_integrals(h, V)
    H = fock.hamiltonian(hso, gso)
    _, _, aa, bb, ab = fm.spin_blocks_from_state(fock, psi)
    assert abs(st.energy_spin(h, V, Na, Nb, aa, bb, ab) - psi @ (H @ psi)) < 1e-12


@pytest.mark.parametrize("r,Na,Nb", SECTORS)
def test_residual_spin_for_open_shell_determinants(r, Na, Nb):
    """For a determinant the Valdemoro 3-RDM is exact, so the residual blocks
    equal those of the brute-force <[O, H]>, and so does the norm."""
    rng = np.random.default_rng(31 + r + Na)
    fock = fm.Fock(2 * r)
    psi = _open_shell_determinant(fock, rng, r, Na, Nb)
    g3 = fock.rdm3(psi)
    assert np.abs(rdm.gamma3_valdemoro_wform(fock.rdm1(psi), fock.rdm2(psi)) - g3).max() < 1e-12
    h, V = gen.hamiltonian(rng, r, 6)
    hso, gso = fm.spin_orbital_integrals(h, V)
    H = fock.hamiltonian(hso, gso)
    hpsi = H @ psi
    brute = fock.commutator_expectation(psi, hpsi, hpsi)
    ga, gb, aa, bb, ab = fm.spin_blocks_from_state(fock, psi)
    raa, rbb, rab, n2 = st.residual_spin(h, V, Na, Nb, ga, gb, aa, bb, ab)
    a, b = slice(0, r), slice(r, 2 * r)
    scale = np.abs(brute).max()
    assert scale > 1e-3
    for got, ref in ((raa, brute[a, a, a, a]), (rbb, brute[b, b, b, b]), (rab, brute[a, b, a, b])):
        assert np.abs(got - ref).max() < 1e-12 * scale
    assert abs(n2 - np.sum(brute ** 2)) < 1e-12 * np.sum(brute ** 2)


@pytest.mark.parametrize("r,Na,Nb", [(3, 2, 1), (4, 3, 1), (4, 3, 0)])
def test_update_spin_for_open_shell_determinants(r, Na, Nb):
    """The update blocks of one step equal 1/2 <[O, A]> with A = sum R a+a+aa in
    Fock space (exact 3-RDM of a determinant), and E1 - E0 = -eps ||R||^2 to
    first order."""
    rng = np.random.default_rng(41 + r + Na)
    fock = fm.Fock(2 * r)
    psi = _open_shell_determinant(fock, rng, r, Na, Nb)
    h, V = gen.hamiltonian(rng, r, 6)
    hso, gso = fm.spin_orbital_integrals(h, V)
    H = fock.hamiltonian(hso, gso)
    hpsi = H @ psi
    R = fock.commutator_expectation(psi, hpsi, hpsi)
    apsi = fock.apply_two_body(R, psi)
    brute = 0.5 * fock.commutator_expectation(psi, apsi, -apsi)
    ga, gb, aa, bb, ab = fm.spin_blocks_from_state(fock, psi)
    eps = 1e-7
    o = st.step_spin(h, V, Na, Nb, ga, gb, aa, bb, ab, eps)
    a, b = slice(0, r), slice(r, 2 * r)
    scale = np.abs(brute).max()
    for got, ref in ((o["U_aa"], brute[a, a, a, a]), (o["U_bb"], brute[b, b, b, b]), (o["U_ab"], brute[a, b, a, b])):
        assert np.abs(got - ref).max() < 1e-11 * scale
    de = o["energy"] - o["energy0"]
    assert abs(de + eps * o["norm2"]) < 1e-6 * eps * o["norm2"]


def test_step_spin_invariants_on_synthetic_input():
    """A synthetic open-shell state at r = 5: Tr U = 0 per block, every block
    keeps its input trace, Tr(K U) = -<R_m, R>, and the beta blocks differ from
    the alpha ones (the state is not a singlet)."""
    p = gen.spin_problem(5, 3, 1, 10, seed=2)
    args = (p["h"], p["V"], p["Na"], p["Nb"], p["gamma_a"], p["gamma_b"], p["d2aa"], p["d2bb"], p["d2ab"])
    act = np.array([0, 1, 1, 0, 1], dtype=bool)
    o = st.step_spin(*args, 1e-3, active=act, keep_spin_orbital=True)
    tr = lambda x: np.einsum('pqpq->', x)
    umax = max(np.abs(o[k]).max() for k in ("U_aa", "U_bb", "U_ab"))
    for k in ("U_aa", "U_bb", "U_ab"):
        assert abs(tr(o[k])) < 1e-12 * umax * 25
    for k in ("d2aa", "d2bb", "d2ab"):
        assert abs(tr(o[k]) - tr(p[k])) < 1e-13 * max(1.0, abs(tr(p[k])))
    assert abs(np.sum(o["K"] * o["U"]) + np.sum(o["Rm"] * o["R"])) < 1e-10 * o["norm2"]
    assert np.abs(o["R_aa"] - o["R_bb"]).max() > 1e-3 * np.abs(o["R_aa"]).max()


def test_spin_path_reduces_to_the_singlet_path():
    """Singlet inputs (beta blocks equal to alpha, pair-exchange symmetric
    alpha-beta block) give the singlet path's residual, update and energy, and
    R_bb = R_aa."""
    p = gen.problem(5, 4, 10, seed=3)
    s = st.step(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], 1e-3)
    g = st.step_spin(p["h"], p["V"], 2, 2, p["gamma"], p["gamma"], p["d2aa"], p["d2aa"], p["d2ab"], 1e-3)
    for k in ("R_aa", "R_ab", "U_aa", "U_ab", "d2aa", "d2ab"):
        assert np.abs(g[k] - s[k]).max() < 1e-12 * max(1.0, np.abs(s[k]).max()), k
    assert np.abs(g["R_bb"] - s["R_aa"]).max() < 1e-12 * np.abs(s["R_aa"]).max()
    assert abs(g["energy"] - s["energy"]) < 1e-12 * abs(s["energy"]) and abs(g["norm2"] - s["norm2"]) < 1e-12 * s["norm2"]
    assert np.abs(g["gamma_a"] - s["gamma"]).max() < 1e-12


def test_spin_lift_planted_mistakes_fail():
    """The round-trip pin catches a flipped sign of a mixed block and beta blocks
    taken from alpha ones."""
    r, Na, Nb = 4, 3, 1
    rng, fock, psi = _state(r, Na, Nb, 5)
    d2 = fock.rdm2(psi) / 2.0
    ga, gb, aa, bb, ab = fm.spin_blocks_from_state(fock, psi)

    def wrong_sign(ga, gb, aa, bb, ab):
        d1, t = rdm.spin_blocks_to_spin_orbital(ga, gb, aa, bb, ab)
        a, b = slice(0, r), slice(r, 2 * r)
        t[a, b, b, a] *= -1.0
        return d1, t

    def beta_from_alpha(ga, gb, aa, bb, ab):
        return rdm.spin_blocks_to_spin_orbital(ga, ga, aa, aa, ab)

    for wrong in (wrong_sign, beta_from_alpha):
        _, l2 = wrong(ga, gb, aa, bb, ab)
        assert np.abs(l2 - d2).max() > 1e-3, wrong.__name__


@pytest.mark.parametrize("Na,Nb", [(3, 0), (4, 1)])
def test_step_spin_blocks_of_fewer_than_two_electrons_stay_zero(Na, Nb):
    """A pair kind with fewer than two electrons has a zero block in every
    N-representable 2-RDM (its App. A trace is zero): the step keeps it zero,
    and the other blocks keep their traces."""
    p = gen.spin_problem(5, Na, Nb, 10, seed=7)
    args = (p["h"], p["V"], p["Na"], p["Nb"], p["gamma_a"], p["gamma_b"], p["d2aa"], p["d2bb"], p["d2ab"])
    assert not np.any(p["d2bb"]) and (Nb > 0) == bool(np.any(p["d2ab"]))
    o = st.step_spin(*args, 1e-3)
    assert not np.any(o["d2bb"])
    if Nb == 0:
        assert not np.any(o["d2ab"]) and not np.any(o["gamma_b"])
    tr = lambda x: np.einsum('pqpq->', x)
    for k in ("d2aa", "d2ab"):
        assert abs(tr(o[k]) - tr(p[k])) < 1e-13 * max(1.0, abs(tr(p[k])))
    assert np.all(np.isfinite(o["d2aa"])) and np.isfinite(o["energy"])


def test_spin_blocks_ny_on_singlet_inputs_is_the_singlet_ny_map():
    """The spin-block NY residual and step, given a singlet as three blocks and
    both spins' weights from the spatial ones, are the singlet NY ones (whose
    cumulant formula is pinned to the exact second-order 3-cumulant)."""
    p = gen.problem(6, 4, 12, seed=5)
    sig = np.array([1.0, 1.0, -1.0, 1.0, -1.0, -1.0])  # not a prefix
    sso = np.concatenate([sig, sig])
    args = (p["h"], p["V"], 2, 2, p["gamma"], p["gamma"], p["d2aa"], p["d2aa"], p["d2ab"])
    raa, rbb, rab, n2 = st.residual_spin(*args, sigma_so=sso)
    Raa, Rab = st.residual(p["h"], p["V"], 4, p["gamma"], p["d2aa"], p["d2ab"], sigma=sig)[:2]
    assert np.abs(raa - Raa).max() < 1e-12 * np.abs(Raa).max()
    assert np.abs(rbb - Raa).max() < 1e-12 * np.abs(Raa).max()
    assert np.abs(rab - Rab).max() < 1e-12 * np.abs(Rab).max()
    v = st.residual_spin(*args)
    assert np.abs(v[0] - raa).max() > 1e-6 * np.abs(raa).max()  # NY differs from V here
    o = st.step_spin(*args, 1e-3, sigma_so=sso)
    s1 = st.step(p["h"], p["V"], 4, p["gamma"], p["d2aa"], p["d2ab"], 1e-3, sigma=sig)
    assert abs(o["energy"] - s1["energy"]) < 1e-12 * abs(s1["energy"])
    assert np.abs(o["d2aa"] - s1["d2aa"]).max() < 1e-12 * np.abs(s1["d2aa"]).max()


@pytest.mark.parametrize("r,Na,Nb", [(4, 3, 1), (4, 1, 3), (5, 3, 2)])
def test_spin_blocks_ny_equals_v_for_a_determinant(r, Na, Nb):
    """For an open-shell determinant the 2-cumulant vanishes, so the NY
    3-cumulant does too and the NY residual is the (exact) Valdemoro one,
    whatever the weights."""
    rng = np.random.default_rng(r + 10 * Na)
    fock = fm.Fock(2 * r)
    Ua, Ub = gen.haar_orthogonal(rng, r), gen.haar_orthogonal(rng, r)
    C = np.zeros((2 * r, Na + Nb))
    C[:r, :Na] = Ua[:, :Na]
    C[r:, Na:] = Ub[:, :Nb]
    psi = fm.rotated_determinant(fock, C)
    h, V = gen.hamiltonian(rng, r, 6)
    ga, gb, aa, bb, ab = fm.spin_blocks_from_state(fock, psi)
    args = (h, V, Na, Nb, ga, gb, aa, bb, ab)
    v = st.residual_spin(*args)
    for sso in (st.sigma_open_shell(r, Na, Nb), -st.sigma_open_shell(r, Na, Nb)):
        n = st.residual_spin(*args, sigma_so=sso)
        for a, b in zip(n[:3], v[:3]):
            assert np.abs(a - b).max() <= 1e-11 * max(np.abs(v[0]).max(), np.abs(v[2]).max(), 1e-300)
