"""Pins of the closed-shell determinant closed forms (tests/determinant_forms.py),
CPU only: against Fock-space brute force of <[O, H]> for a determinant, and
against the oracle (tier B residual, energy) at larger r, in the orbital basis
and after a random rotation (covariance)."""
import numpy as np
import pytest

import determinant_forms as dform
from oracle import fermion as fm
from oracle import rdm
from oracle import step as ost
from synth import generators as gen


@pytest.mark.parametrize("r,na,seed", [(3, 1, 0), (4, 2, 1)])
def test_blocks_match_brute_force(r, na, seed):
    rng = np.random.default_rng(seed)
    h, V = gen.hamiltonian(rng, r, 6)
    fock = fm.Fock(2 * r)
    hso, gso = fm.spin_orbital_integrals(h, V)
    H = fock.hamiltonian(hso, gso)
    psi = fm.determinant(fock, list(range(na)) + list(range(r, r + na)))
    hpsi = H @ psi
    R = fock.commutator_expectation(psi, hpsi, hpsi)
    baa, bab = rdm.spin_orbital_to_blocks(R)
    caa, cab = dform.residual_blocks(h, V, na)
    scale = np.abs(R).max()
    assert np.abs(caa - baa).max() <= 1e-12 * scale
    assert np.abs(cab - bab).max() <= 1e-12 * scale
    assert abs(dform.energy(h, V, na) - float(psi @ hpsi)) <= 1e-12 * max(1.0, abs(float(psi @ hpsi)))


@pytest.mark.parametrize("r,na", [(8, 3), (11, 5)])
def test_blocks_match_oracle_and_rotate(r, na):
    rng = np.random.default_rng(r)
    h, V = gen.hamiltonian(rng, r, 2 * r)
    g, d2aa, d2ab = dform.rdms(r, na)
    raa, rab, n2 = ost.residual(h, V, 2 * na, g, d2aa, d2ab)
    caa, cab = dform.residual_blocks(h, V, na)
    scale = max(np.abs(caa).max(), np.abs(cab).max())
    assert np.abs(raa - caa).max() <= 1e-12 * scale
    assert np.abs(rab - cab).max() <= 1e-12 * scale
    assert abs(n2 - (2 * np.sum(caa ** 2) + 4 * np.sum(cab ** 2))) <= 1e-12 * n2
    assert abs(ost.energy(h, V, 2 * na, d2aa, d2ab) - dform.energy(h, V, na)) <= 1e-12 * abs(dform.energy(h, V, na))
    U = gen.haar_orthogonal(rng, r)
    R = dform.rot4
    raa2, rab2, _ = ost.residual(dform.rot2(h, U), R(V, U), 2 * na, dform.rot2(g, U), R(d2aa, U), R(d2ab, U))
    assert np.abs(raa2 - R(caa, U)).max() <= 1e-11 * scale
    assert np.abs(rab2 - R(cab, U)).max() <= 1e-11 * scale
