"""Pins of the oracle's Nakatsuji-Yasuda reconstruction (Eq. (8); App. D, NY
part), CPU only.

* Second order: for a determinant with a doubles admixture of amplitude t, the
  exact 3-cumulant (Fock-space 3-RDM minus the Valdemoro terms) is O(t^2) and
  the NY formula, evaluated on the exact 2-cumulant with sigma from the
  determinant's occupations, matches it up to O(t^3); for a prefix of
  occupied orbitals and for a scattered set (sigma follows the orbital, not
  its position).  This fixes the 1/6, the
  36-term antisymmetriser and the normalisation of 2Delta; a factor 2 or a
  sign flip leaves an O(t^2) error and fails.
* Invariants of the NY 3-cumulant: antisymmetric within the upper and within
  the lower triple, symmetric under upper <-> lower (so the transposition
  forms of App. B, Eqs. (B8)-(B9) hold for the NY 3-RDM as for the Valdemoro
  one); zero for a determinant (2Delta = 0).
* The factorised NY share of B (tier B, 9 products, 3-RDM never formed) equals
  the six-term map with the materialised NY 3-RDM (tier A) for both the
  Hermitian and the anti-Hermitian branch, with a sigma pattern that is not a
  prefix (a misplaced orbital index a would show).
"""
import itertools

import numpy as np
import pytest

from oracle import fermion as fm
from oracle import rdm
from oracle import residual as rs
from oracle import step as st
from synth import generators as gen


def _doubles_state(fock, occ, amp, t):
    n = fock.n
    virt = [p for p in range(n) if p not in occ]
    psi0 = fm.determinant(fock, occ)
    psi = psi0.copy()
    for i, j in itertools.combinations(occ, 2):
        for a, b in itertools.combinations(virt, 2):
            psi = psi + t * amp[i, j, a, b] * (fock.cre[a] @ (fock.cre[b] @ (fock.ann[j] @ (fock.ann[i] @ psi0))))
    return psi / np.linalg.norm(psi)


@pytest.fixture(scope="module", params=[(0, 1), (1, 3)], ids=["occ01", "occ13"])
def second_order(request):
    n = 8
    fock = fm.Fock(n)
    occ = [q for o in request.param for q in (o, o + 4)]  # both spins of the occupied spatial orbitals
    amp = np.random.default_rng(3).standard_normal((n, n, n, n))
    sigma = np.array([1.0 if p in occ else -1.0 for p in range(n)])
    out = []
    for t in (0.025, 0.0125, 0.00625):
        psi = _doubles_state(fock, occ, amp, t)
        d1 = fock.rdm1(psi)
        d2 = 0.5 * fock.rdm2(psi)
        c3 = fock.rdm3(psi) / 6.0 - rdm.d3_valdemoro(d1, d2)
        out.append((t, c3, rdm.d3_ny_cumulant(d1, d2, sigma)))
    return out


def test_ny_matches_exact_cumulant_through_second_order(second_order):
    errs, sizes = [], []
    for t, c3, ny in second_order:
        errs.append(np.abs(c3 - ny).max())
        sizes.append(np.abs(c3).max())
    # the cumulant itself falls by 4 per halving of t, the NY error by 8
    for a, b in zip(sizes, sizes[1:]):
        assert 3.0 < a / b < 5.0
    for a, b in zip(errs, errs[1:]):
        assert a / b > 6.5
    assert errs[-1] < 0.03 * sizes[-1]


@pytest.mark.parametrize("factor", [2.0, 0.5, -1.0])
def test_second_order_pin_rejects_wrong_scale(second_order, factor):
    t, c3, ny = second_order[-1]
    assert np.abs(c3 - factor * ny).max() > 0.3 * np.abs(c3).max()


def test_ny_cumulant_invariants():
    p = gen.problem(3, 4, 6, seed=5)
    d1, d2 = rdm.blocks_to_spin_orbital(p["gamma"], p["d2aa"], p["d2ab"])
    sigma = rdm.sigma_spin_orbital([1.0, -1.0, 1.0])
    c = rdm.d3_ny_cumulant(d1, d2, sigma)
    scale = np.abs(c).max()
    assert scale > 1e-6
    for perm in [(1, 0, 2), (0, 2, 1), (2, 1, 0)]:
        up = list(perm) + [3, 4, 5]
        lo = [0, 1, 2] + [3 + x for x in perm]
        assert np.abs(c + c.transpose(up)).max() < 1e-14 * scale
        assert np.abs(c + c.transpose(lo)).max() < 1e-14 * scale
    assert np.abs(c - c.transpose(3, 4, 5, 0, 1, 2)).max() < 1e-14 * scale


def test_ny_cumulant_vanishes_for_a_determinant():
    r, na = 4, 2
    g = np.diag([1.0, 1.0, 0.0, 0.0])
    d2aa = 0.5 * (np.einsum('pr,qs->pqrs', g, g) - np.einsum('ps,qr->pqrs', g, g))
    d2ab = 0.5 * np.einsum('pr,qs->pqrs', g, g)
    d1, d2 = rdm.blocks_to_spin_orbital(g, d2aa, d2ab)
    sigma = rdm.sigma_spin_orbital([1.0, 1.0, -1.0, -1.0])
    assert np.abs(rdm.d3_ny_cumulant(d1, d2, sigma)).max() == 0.0
    assert np.abs(rdm.d3_ny(d1, d2, sigma) - rdm.d3_valdemoro(d1, d2)).max() == 0.0


@pytest.mark.parametrize("r,seed,sig", [(3, 0, (1, -1, 1)), (4, 1, (-1, 1, 1, -1))])
def test_factorised_ny_map_equals_materialised(r, seed, sig):
    p = gen.problem(r, 4, 8, seed=seed)
    # a larger cumulant than the generator's default, so the NY share is not small
    rng = np.random.default_rng(seed + 10)
    extra = gen.symmetric_direction(rng, r, scale=0.05)
    d2aa, d2ab = p["d2aa"] + extra["d2aa"], p["d2ab"] + extra["d2ab"]
    d1, d2 = rdm.blocks_to_spin_orbital(p["gamma"], d2aa, d2ab)
    sso = rdm.sigma_spin_orbital(np.array(sig, dtype=float))
    d3 = rdm.d3_ny(d1, d2, sso)
    K = rdm.reduced_hamiltonian(p["h"], p["V"], p["N"])
    RA = rs.residual_map_dense(K, d2, d3)
    RB = rs.residual_map(K, d1, d2, hermitian=True, sigma_so=sso).numpy()
    assert np.abs(RA - RB).max() < 1e-12 * np.abs(RA).max()
    # the NY share is a visible part of the residual
    RV = rs.residual_map(K, d1, d2, hermitian=True).numpy()
    assert np.abs(RB - RV).max() > 1e-3 * np.abs(RB).max()
    UA = rs.residual_map_dense(RA, d2, d3)
    UB = rs.residual_map(RA, d1, d2, hermitian=False, sigma_so=sso).numpy()
    assert np.abs(UA - UB).max() < 1e-12 * np.abs(UA).max()


def test_ny_step_blocks_and_energy_identity():
    """The NY step on the stored blocks: E1 - E0 = -eps <R, R_m> holds as for V
    (E is linear along the step), and sigma = None is the V step."""
    p = gen.problem(4, 4, 8, seed=2)
    sig = np.array([1.0, 1.0, -1.0, -1.0])
    s = st.step(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], 1e-4, sigma=sig,
                keep_spin_orbital=True)
    v = st.step(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], 1e-4)
    assert np.abs(s["R_aa"] - v["R_aa"]).max() > 0.0
    K = s["K"]
    dE = float(np.sum(K * (s["U"]))) * 1e-4
    # trace restoration changes E only at O(eps * rounding)
    assert abs((s["energy"] - s["energy0"]) - dE) <= 1e-9 * abs(dE)
    assert abs(float(np.sum(K * s["U"])) + float(np.sum(s["R"] * s["Rm"]))) <= 1e-10 * s["norm2"]
