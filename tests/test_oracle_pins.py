"""Pins of the CPU oracle against brute force and closed forms (no GPU).

Every formula in ``oracle.rdm`` / ``oracle.residual`` / ``oracle.step`` is
checked here against something other than itself: Fock-space commutators
(Eqs. (4), (9)), exact eigenstates (the CSE/ACSE vanish there), single
determinants (Valdemoro is exact there; Slater-Condon closed forms), the
independent nine-term form of App. C, Eq. (C5), and exact identities.
"""
import numpy as np
import pytest

from oracle import fermion as fm
from oracle import rdm
from oracle import residual as rs
from oracle import step as st
from synth import generators as gen


def _random_state(fock, N, rng, n_alpha=None):
    sec = fock.sector(N, n_alpha)
    psi = np.zeros(fock.dim)
    psi[sec] = rng.normal(size=sec.size)
    return psi / np.linalg.norm(psi)


def _system(r, N, seed, n_chol=6):
    rng = np.random.default_rng(seed)
    h, V = gen.hamiltonian(rng, r, n_chol)
    fock = fm.Fock(2 * r)
    hso, gso = fm.spin_orbital_integrals(h, V)
    H = fock.hamiltonian(hso, gso)
    return rng, h, V, fock, hso, gso, H


# --------------------------------------------------------------------------
# T1: sign/scale of F and the fold of Eq. (2) against <[O, H]> in Fock space
# --------------------------------------------------------------------------

@pytest.mark.parametrize("r,N,seed,na", [(3, 4, 0, None), (3, 3, 1, None), (4, 4, 2, 2)])
def test_residual_equals_commutator_exact_rdms(r, N, seed, na):
    rng, h, V, fock, hso, gso, H = _system(r, N, seed)
    psi = _random_state(fock, N, rng, na)
    hpsi = H @ psi
    brute = fock.commutator_expectation(psi, hpsi, hpsi)
    K = rdm.reduced_hamiltonian(h, V, N)
    d2 = fock.rdm2(psi) / 2.0
    d3 = fock.rdm3(psi) / 6.0
    F = rs.residual_map_dense(K, d2, d3)
    assert np.abs(F - brute).max() < 1e-12 * max(1.0, np.abs(brute).max())
    # energy convention E = Tr(K 2D) = <H>
    assert abs(np.sum(K * d2) - psi @ hpsi) < 1e-12


def test_generic_map_for_non_hermitian_x():
    """F(X) = 1/2 <[O, sum X a+a+aa]> for an arbitrary pair-exchange-symmetric X."""
    r, N = 3, 3
    rng, h, V, fock, *_ = _system(r, N, 5)
    psi = _random_state(fock, N, rng)
    n = 2 * r
    X = rng.normal(size=(n, n, n, n))
    X = 0.5 * (X + X.transpose(1, 0, 3, 2))
    bpsi = fock.apply_two_body(X, psi)
    bdpsi = fock.apply_two_body(X.transpose(2, 3, 0, 1), psi)
    brute = 0.5 * fock.commutator_expectation(psi, bpsi, bdpsi)
    F = rs.residual_map_dense(X, fock.rdm2(psi) / 2.0, fock.rdm3(psi) / 6.0)
    assert np.abs(F - brute).max() < 1e-12 * np.abs(brute).max()


def test_eq5_as_printed_is_minus_commutator():
    """Reading of the sign: Eq. (5) with K of Eq. (2) equals -<[O,H]>."""
    r, N = 3, 4
    rng, h, V, fock, hso, gso, H = _system(r, N, 3)
    psi = _random_state(fock, N, rng)
    hpsi = H @ psi
    brute = fock.commutator_expectation(psi, hpsi, hpsi)
    K = rdm.reduced_hamiltonian(h, V, N)
    R5 = rs.eq5_as_printed(K, fock.rdm2(psi) / 2.0, fock.rdm3(psi) / 6.0)
    assert np.abs(R5 + brute).max() < 1e-12
    assert np.abs(brute).max() > 1e-2


# --------------------------------------------------------------------------
# T2: eigenstates.  The ACSE (and CSE) residual vanishes at any eigenstate.
# --------------------------------------------------------------------------

def test_residual_vanishes_at_eigenstates():
    r, N = 4, 4
    rng, h, V, fock, hso, gso, H = _system(r, N, 7)
    w, vecs = fm.fci(fock, H, N, nroots=3)
    K = rdm.reduced_hamiltonian(h, V, N)
    for k in range(3):
        psi = vecs[:, k]
        hpsi = H @ psi
        brute = fock.commutator_expectation(psi, hpsi, hpsi)
        assert np.abs(brute).max() < 1e-12
        F = rs.residual_map_dense(K, fock.rdm2(psi) / 2.0, fock.rdm3(psi) / 6.0)
        assert np.abs(F).max() < 1e-11
        assert abs(np.sum(K * fock.rdm2(psi) / 2.0) - w[k]) < 1e-11


def test_fci_singlet_blocks_reproduce_spin_orbital_rdms():
    """Block layout of the stored alpha-alpha / alpha-beta 2-RDM (spatial working
    equations with singlet beta-beta = alpha-alpha) against the full spin-orbital 2-RDM."""
    rng = np.random.default_rng(11)
    h, V = gen.hamiltonian(rng, 4, 6)
    p = fm.fci_singlet_problem(h, V, 4)
    d1, d2 = rdm.blocks_to_spin_orbital(p["gamma"], p["d2aa"], p["d2ab"])
    assert np.abs(d1 - p["fock"].rdm1(p["psi"])).max() < 1e-12
    assert np.abs(d2 - p["fock"].rdm2(p["psi"]) / 2.0).max() < 1e-12
    # App. A traces
    taa, tab = rdm.block_traces(p["d2aa"], p["d2ab"])
    assert abs(taa - 2 * 1 / 2) < 1e-12 and abs(tab - 2 * 2 / 2) < 1e-12
    assert abs(np.einsum('pqpq->', d2) - 4 * 3 / 2) < 1e-12
    # Eq. (6) 3-RDM traces of App. A (alpha-alpha-alpha, alpha-alpha-beta)
    d3 = p["fock"].rdm3(p["psi"]) / 6.0
    a, b = slice(0, 4), slice(4, 8)
    assert abs(np.einsum('pqtpqt->', d3[a, a, a, a, a, a]) - 0.0) < 1e-12
    assert abs(np.einsum('pqtpqt->', d3[a, a, b, a, a, b]) - 2 * 1 * 2 / 6) < 1e-12
    # 1-RDM from the 2-RDM contraction
    assert np.abs(rdm.contract_to_1rdm(d2, 4) - d1).max() < 1e-12


# --------------------------------------------------------------------------
# T3/T4: the Valdemoro reconstruction and the factorisation
# --------------------------------------------------------------------------

def test_valdemoro_exact_for_rotated_determinants():
    r, N = 4, 4
    rng = np.random.default_rng(4)
    fock = fm.Fock(2 * r)
    U = gen.haar_orthogonal(rng, r)
    C = np.zeros((2 * r, N))
    C[:r, 0:2] = U[:, :2]
    C[r:, 2:4] = U[:, :2]
    psi = fm.rotated_determinant(fock, C)
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-12
    g1, g2, g3 = fock.rdm1(psi), fock.rdm2(psi), fock.rdm3(psi)
    assert np.abs(6.0 * rdm.d3_valdemoro(g1, g2 / 2.0) - g3).max() < 1e-12
    assert np.abs(rdm.gamma3_valdemoro_wform(g1, g2) - g3).max() < 1e-12
    # and therefore the reconstructed residual equals the brute-force one
    h, V = gen.hamiltonian(rng, r, 6)
    hso, gso = fm.spin_orbital_integrals(h, V)
    H = fock.hamiltonian(hso, gso)
    hpsi = H @ psi
    brute = fock.commutator_expectation(psi, hpsi, hpsi)
    K = rdm.reduced_hamiltonian(h, V, N)
    RB = rs.residual_map(K, g1, g2 / 2.0, hermitian=True).numpy()
    assert np.abs(RB - brute).max() < 1e-12 * np.abs(brute).max()


def test_valdemoro_not_exact_for_correlated_state():
    """Guard: the pins above would be vacuous if Valdemoro were exact in general."""
    rng = np.random.default_rng(12)
    h, V = gen.hamiltonian(rng, 4, 6)
    p = fm.fci_singlet_problem(h, V, 4)
    g1, g2, g3 = (p["fock"].rdm1(p["psi"]), p["fock"].rdm2(p["psi"]), p["fock"].rdm3(p["psi"]))
    assert np.abs(rdm.gamma3_valdemoro_wform(g1, g2) - g3).max() > 1e-4


@pytest.mark.parametrize("r,seed", [(3, 0), (5, 1)])
def test_c5_form_equals_w_form_and_tiers_agree(r, seed):
    p = gen.problem(r, 4, 8, seed=seed)
    d1, d2 = rdm.blocks_to_spin_orbital(p["gamma"], p["d2aa"], p["d2ab"])
    d3 = rdm.d3_valdemoro(d1, d2)
    assert np.abs(6.0 * d3 - rdm.gamma3_valdemoro_wform(d1, 2.0 * d2)).max() < 1e-13
    # antisymmetry of M (App. C, Eq. (C4)) and of the reconstructed 3D
    M = rdm.m_intermediate(d1, d2)
    assert np.abs(M + M.transpose(1, 0, 2, 3)).max() < 1e-14
    assert np.abs(M + M.transpose(0, 1, 3, 2)).max() < 1e-14
    assert np.abs(d3 + d3.transpose(1, 0, 2, 3, 4, 5)).max() < 1e-14
    assert np.abs(d3 + d3.transpose(0, 2, 1, 3, 4, 5)).max() < 1e-14
    assert np.abs(d3 + d3.transpose(0, 1, 2, 3, 5, 4)).max() < 1e-14
    K = rdm.reduced_hamiltonian(p["h"], p["V"], p["N"])
    RA = rs.residual_map_dense(K, d2, d3)
    RB = rs.residual_map(K, d1, d2, hermitian=True).numpy()
    assert np.abs(RA - RB).max() < 1e-12 * np.abs(RA).max()
    # single-element evaluator
    n = 2 * r
    idx = [tuple(int(x) for x in np.random.default_rng(seed).integers(0, n, 4)) for _ in range(6)]
    el = rs.residual_elements(K, d1, d2, idx)
    assert np.abs(el - np.array([RA[t] for t in idx])).max() < 1e-12 * np.abs(RA).max()
    # update map, anti-Hermitian branch
    UA = rs.residual_map_dense(RA, d2, d3)
    UB = rs.residual_map(RA, d1, d2, hermitian=False).numpy()
    assert np.abs(UA - UB).max() < 1e-12 * np.abs(UA).max()


# --------------------------------------------------------------------------
# T5: the update of Eq. (9) against 1/2 <[O, A]> in Fock space
# --------------------------------------------------------------------------

def test_update_equals_commutator_with_residual_operator():
    r, N = 3, 4
    rng, h, V, fock, hso, gso, H = _system(r, N, 9)
    psi = _random_state(fock, N, rng)
    hpsi = H @ psi
    R = fock.commutator_expectation(psi, hpsi, hpsi)
    apsi = fock.apply_two_body(R, psi)
    brute = 0.5 * fock.commutator_expectation(psi, apsi, -apsi)
    U = rs.residual_map_dense(R, fock.rdm2(psi) / 2.0, fock.rdm3(psi) / 6.0)
    assert np.abs(U - brute).max() < 1e-11 * np.abs(brute).max()
    # U is d 2D / d eps along exp(eps A) psi: finite difference in Fock space
    from scipy.sparse.linalg import expm_multiply
    A = fock.two_body(R)
    eps = 1e-5
    dp = expm_multiply(eps * A, psi)
    dm = expm_multiply(-eps * A, psi)
    fd = (fock.rdm2(dp) - fock.rdm2(dm)) / (4.0 * eps)
    assert np.abs(fd - U).max() < 1e-6 * np.abs(U).max()


# --------------------------------------------------------------------------
# T6/T7: exact identities and symmetries at any size (tier B)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def step8():
    p = gen.problem(8, 6, 16, seed=3)
    return p, st.step(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], 1e-3,
                      keep_spin_orbital=True)


def test_update_identities(step8):
    p, o = step8
    # dE/deps = Tr(K U) = -<R_m, R>;  Tr U per block = 0
    assert abs(np.sum(o["K"] * o["U"]) + np.sum(o["Rm"] * o["R"])) < 1e-10 * np.sum(o["R"] ** 2)
    taa, tab = rdm.block_traces(o["U_aa"], o["U_ab"])
    assert abs(taa) < 1e-11 and abs(tab) < 1e-11
    # the step is first order: E1 = E0 + eps Tr(K U) up to the (tiny) trace rescale
    assert abs(o["energy"] - (o["energy0"] + 1e-3 * np.sum(o["K"] * o["U"]))) < 1e-9


def test_symmetries(step8):
    p, o = step8
    R, U = o["R"], o["U"]
    for T, herm in ((R, -1.0), (U, 1.0)):
        assert np.abs(T + T.transpose(1, 0, 2, 3)).max() < 1e-12
        assert np.abs(T + T.transpose(0, 1, 3, 2)).max() < 1e-12
        assert np.abs(T - herm * T.transpose(2, 3, 0, 1)).max() < 1e-11
    raa, rab = o["R_aa"], o["R_ab"]
    assert np.abs(rab - rab.transpose(1, 0, 3, 2)).max() < 1e-12
    # singlet-consistent inputs give a singlet-consistent residual and update
    assert np.abs(raa - (rab - rab.transpose(0, 1, 3, 2))).max() < 1e-12
    assert np.abs(o["U_aa"] - (o["U_ab"] - o["U_ab"].transpose(0, 1, 3, 2))).max() < 1e-11
    # beta-beta equals alpha-alpha
    r = p["r"]
    assert np.abs(R[r:, r:, r:, r:] - raa).max() < 1e-12
    # norm in blocks
    assert abs(o["norm2"] - (2 * np.sum(raa ** 2) + 4 * np.sum(rab ** 2))) < 1e-10 * o["norm2"]


def test_orbital_rotation_covariance():
    p = gen.problem(6, 4, 10, seed=8)
    U = gen.haar_orthogonal(np.random.default_rng(99), 6)
    raa, rab, n2 = st.residual(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"])
    e = np.einsum
    rot4 = lambda t: e('pqrs,pa,qb,rc,sd->abcd', t, U, U, U, U)
    raa2, rab2, n22 = st.residual(U.T @ p["h"] @ U, rot4(p["V"]), p["N"], U.T @ p["gamma"] @ U,
                                  rot4(p["d2aa"]), rot4(p["d2ab"]))
    assert np.abs(rot4(raa) - raa2).max() < 1e-12
    assert np.abs(rot4(rab) - rab2).max() < 1e-12
    assert abs(n2 - n22) < 1e-10 * n2


def _mask_pin_holds(mask_fn):
    """The active-mask rule (all four spatial indices active -> zeroed, in every
    spin block) on r = 5 with orbitals 1, 2, 3 active, checked against hand-picked
    spin-orbital elements and against a keep/zero table built with explicit index
    loops.  Returns True iff ``mask_fn(active, r)`` (True = kept) satisfies both."""
    r = 5
    active = [False, True, True, True, False]
    m = np.asarray(mask_fn(np.array(active), r), dtype=bool)
    if m.shape != (2 * r,) * 4:
        return False
    a, b = 0, r   # offsets of the alpha and beta spin orbitals
    zeroed = [(1 + a, 2 + a, 3 + a, 1 + a),          # alpha-alpha block
              (1 + b, 2 + b, 3 + b, 1 + b),          # beta-beta block
              (1 + a, 2 + b, 3 + a, 1 + b),          # (alpha beta | alpha beta)
              (1 + a, 2 + b, 3 + b, 1 + a),          # (alpha beta | beta alpha)
              (3 + b, 3 + a, 2 + b, 2 + a)]
    kept = [(0 + a, 2 + a, 3 + a, 1 + a), (1 + a, 2 + a, 3 + a, 4 + a),
            (0 + a, 2 + b, 3 + a, 1 + b), (1 + b, 2 + b, 3 + b, 4 + b),
            (1 + a, 4 + b, 3 + b, 1 + a), (0 + a, 0 + b, 0 + a, 0 + b)]
    if any(m[t] for t in zeroed) or not all(m[t] for t in kept):
        return False
    n = 2 * r
    for p in range(n):
        for q in range(n):
            for u in range(n):
                for v in range(n):
                    all_active = (active[p % r] and active[q % r] and active[u % r]
                                  and active[v % r])
                    if m[p, q, u, v] != (not all_active):
                        return False
    return True


def test_active_mask_pin():
    """C-9 (the method section's all-active option): the oracle's mask passes
    the pin; a rule that zeroes an element when ANY index is active, an
    inverted rule, and one that ignores the beta spin orbitals each fail it."""
    assert _mask_pin_holds(st.active_mask)

    def any_rule(active, r):
        so = np.concatenate([active, active])
        return ~(so[:, None, None, None] | so[None, :, None, None] | so[None, None, :, None]
                 | so[None, None, None, :])

    def inverted(active, r):
        return ~st.active_mask(active, r)

    def alpha_only(active, r):
        so = np.concatenate([active, np.zeros_like(active)])
        return ~(so[:, None, None, None] & so[None, :, None, None] & so[None, None, :, None]
                 & so[None, None, None, :])

    for wrong in (any_rule, inverted, alpha_only):
        assert not _mask_pin_holds(wrong), wrong.__name__


def test_active_mask_in_the_step():
    """The step zeroes exactly the all-active elements of R before the update
    map, keeps the rest unchanged, and takes the norm before masking."""
    p = gen.problem(5, 4, 8, seed=2)
    active = np.array([0, 1, 1, 1, 0], dtype=bool)
    o = st.step(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], 1e-3, active=active,
                keep_spin_orbital=True)
    n = 10
    for idx in np.ndindex(n, n, n, n):
        if all(active[x % 5] for x in idx):
            assert o["Rm"][idx] == 0.0
        else:
            assert o["Rm"][idx] == o["R"][idx]
    assert np.abs(o["R"][1, 2, 3, 1]) > 0.0    # the zeroed element was not zero already
    assert abs(o["norm2"] - np.sum(o["R"] ** 2)) < 1e-12 * o["norm2"]   # norm before masking
    assert abs(np.sum(o["K"] * o["U"]) + np.sum(o["Rm"] * o["R"])) < 1e-10 * o["norm2"]


def _explicit_traces(d2aa, d2ab):
    r = d2aa.shape[0]
    taa = tab = 0.0
    for p in range(r):
        for q in range(r):
            taa += d2aa[p, q, p, q]
            tab += d2ab[p, q, p, q]
    return taa, tab


def _restoration_pin_holds(fn):
    """Trace restoration (C-10, App. A traces) on blocks carrying a planted
    drift, different in the two blocks: the output traces must equal the input
    ones (hand-summed), and each output block must be its drifted input times
    one positive number (the restoration changes nothing but the scale)."""
    p = gen.problem(5, 4, 10, seed=3)
    t0 = _explicit_traces(p["d2aa"], p["d2ab"])
    rng = np.random.default_rng(7)
    drift_aa = 1.07 * p["d2aa"] + 1e-3 * rng.standard_normal(p["d2aa"].shape)
    drift_ab = 0.93 * p["d2ab"] + 1e-3 * rng.standard_normal(p["d2ab"].shape)
    out_aa, out_ab, _ = fn(drift_aa, drift_ab, t0)
    t1 = _explicit_traces(out_aa, out_ab)
    if abs(t1[0] - t0[0]) > 1e-13 * abs(t0[0]) or abs(t1[1] - t0[1]) > 1e-13 * abs(t0[1]):
        return False
    for out, drift in ((out_aa, drift_aa), (out_ab, drift_ab)):
        c = float(np.sum(out * drift) / np.sum(drift * drift))
        if not c > 0 or np.abs(out - c * drift).max() > 1e-14 * np.abs(out).max():
            return False
    return True


def test_trace_restoration_pin():
    """The oracle's restoration passes; an inverted ratio, one factor for the
    whole 2-RDM, and no restoration at all each fail."""
    assert _restoration_pin_holds(st.restore_traces)

    def inverted(aa, ab, t0):
        t1 = _explicit_traces(aa, ab)
        return aa * (t1[0] / t0[0]), ab * (t1[1] / t0[1]), None

    def whole(aa, ab, t0):
        t1 = _explicit_traces(aa, ab)
        s = (t0[0] + t0[1]) / (t1[0] + t1[1])
        return aa * s, ab * s, None

    def none(aa, ab, t0):
        return aa, ab, None

    for wrong in (inverted, whole, none):
        assert not _restoration_pin_holds(wrong), wrong.__name__


def test_step_keeps_app_a_traces():
    """After a step the blocks keep the App. A traces of the input state
    (N_a(N_a-1)/2 and N_a N_b/2 for the FCI singlet's 2-RDM)."""
    rng = np.random.default_rng(0)
    h, V = gen.hamiltonian(rng, 4, 6)
    p = fm.fci_singlet_problem(h, V, 4)
    o = st.step(h, V, 4, p["gamma"], p["d2aa"], p["d2ab"], 1e-2)
    taa, tab = _explicit_traces(o["d2aa"], o["d2ab"])
    assert abs(taa - 1.0) < 1e-13 and abs(tab - 2.0) < 1e-13


# --------------------------------------------------------------------------
# T8: determinants in their own basis: Slater-Condon closed forms at larger r
# --------------------------------------------------------------------------

def _closed_form_residual(hso, gso, occ):
    """R for a single determinant: R^{ij}_{ab} = <ij||ab> (i,j occupied, a,b virtual),
    R^{ij}_{aj} = f_ai (i != j occupied, a virtual), the rest by antisymmetry and
    anti-Hermiticity, all other elements zero."""
    n = hso.shape[0]
    o = np.zeros(n, bool)
    o[list(occ)] = True
    v = ~o
    anti = gso - gso.transpose(0, 1, 3, 2)
    f = hso + np.einsum('pmqm->pq', anti[:, o][:, :, :, o])
    D1 = anti * (o[:, None, None, None] & o[None, :, None, None] & v[None, None, :, None] & v[None, None, None, :])
    S1 = np.zeros((n, n, n, n))
    for i in np.flatnonzero(o):
        for j in np.flatnonzero(o):
            if i != j:
                for a in np.flatnonzero(v):
                    S1[i, j, a, j] = f[a, i]
    S2 = S1 - S1.transpose(1, 0, 2, 3) - S1.transpose(0, 1, 3, 2) + S1.transpose(1, 0, 3, 2)
    R = D1 + S2
    return R - R.transpose(2, 3, 0, 1), f


def test_closed_form_matches_brute_force():
    r, N = 3, 4
    rng, h, V, fock, hso, gso, H = _system(r, N, 13)
    occ = [0, 1, 3, 4]
    psi = fm.determinant(fock, occ)
    hpsi = H @ psi
    brute = fock.commutator_expectation(psi, hpsi, hpsi)
    Rc, _ = _closed_form_residual(hso, gso, occ)
    assert np.abs(Rc - brute).max() < 1e-12


@pytest.mark.parametrize("r,N", [(8, 6), (12, 8)])
def test_tier_b_matches_closed_form_for_determinants(r, N):
    rng = np.random.default_rng(r)
    h, V = gen.hamiltonian(rng, r, 2 * r)
    hso, gso = fm.spin_orbital_integrals(h, V)
    na = N // 2
    gamma = np.diag([1.0] * na + [0.0] * (r - na))
    d2aa = 0.5 * (np.einsum('pr,qs->pqrs', gamma, gamma) - np.einsum('ps,qr->pqrs', gamma, gamma))
    d2ab = 0.5 * np.einsum('pr,qs->pqrs', gamma, gamma)
    raa, rab, n2 = st.residual(h, V, N, gamma, d2aa, d2ab)
    occ = list(range(na)) + list(range(r, r + na))
    Rc, f = _closed_form_residual(hso, gso, occ)
    caa, cab = rdm.spin_orbital_to_blocks(Rc)
    scale = np.abs(Rc).max()
    assert np.abs(raa - caa).max() < 1e-12 * scale
    assert np.abs(rab - cab).max() < 1e-12 * scale
    assert abs(n2 - np.sum(Rc ** 2)) < 1e-10 * n2
    # HF energy expression
    o = np.zeros(2 * r, bool)
    o[occ] = True
    anti = gso - gso.transpose(0, 1, 3, 2)
    e_hf = np.trace(hso[o][:, o]) + 0.5 * np.einsum('ijij->', anti[o][:, o][:, :, o][:, :, :, o])
    assert abs(st.energy(h, V, N, d2aa, d2ab) - e_hf) < 1e-10
    # rotate to a random basis: covariance at larger r
    U = gen.haar_orthogonal(rng, r)
    e = np.einsum
    rot4 = lambda t: e('pqrs,pa,qb,rc,sd->abcd', t, U, U, U, U)
    raa2, rab2, _ = st.residual(U.T @ h @ U, rot4(V), N, U.T @ gamma @ U, rot4(d2aa), rot4(d2ab))
    assert np.abs(raa2 - rot4(caa)).max() < 1e-11 * scale
    assert np.abs(rab2 - rot4(cab)).max() < 1e-11 * scale


def test_planted_mistakes_are_caught():
    """A dropped term, a wrong sign and a transposed operand in F each break the
    brute-force pin (guards the strength of test_residual_equals_commutator_exact_rdms)."""
    r, N = 3, 4
    rng, h, V, fock, hso, gso, H = _system(r, N, 21)
    psi = _random_state(fock, N, rng)
    hpsi = H @ psi
    brute = fock.commutator_expectation(psi, hpsi, hpsi)
    K = rdm.reduced_hamiltonian(h, V, N)
    d2, d3 = fock.rdm2(psi) / 2.0, fock.rdm3(psi) / 6.0
    e = np.einsum
    good = rs.residual_map_dense(K, d2, d3)
    dropped = good - (6.0 * e('pqri,jpqrlk->ijkl', K, d3))
    flipped = good - 2.0 * (2.0 * e('klrs,ijrs->ijkl', K, d2))
    transposed = good + 6.0 * e('kprs,ijprsl->ijkl', K, d3) - 6.0 * e('pkrs,ijprsl->ijkl', K, d3)
    for bad in (dropped, flipped, transposed):
        assert np.abs(bad - brute).max() > 1e-3
