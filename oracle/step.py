"""One ACSE propagation step and the energy, on the stored singlet blocks (oracle).

Inputs are the spatial quantities the GPU library takes: h [r,r], chemists'
V [r,r,r,r], N, the alpha 1-RDM gamma [r,r] and the 2-RDM blocks d2aa, d2ab
[r,r,r,r] (Eq. (6) normalisation).  Everything is lifted to spin orbitals
(``rdm.blocks_to_spin_orbital``) and computed there; the returned blocks are
the alpha-alpha and (p_a q_b | r_a s_b) parts.

Readings:
* Active mask (the "all active" option of the method section): ``active`` is
  a per-spatial-orbital flag; a residual element is zeroed iff all four of its
  spatial indices are active, in every spin block.  The residual norm is
  taken before masking.
* Update scale: U = F(R_m) = 1/2 <[O, A]> = d 2D / d eps along exp(eps A) psi,
  with A = sum R_m a+a+aa;  2D_{n+1} = 2D_n + eps U  (Eq. (9)).
* Trace restoration: the paper describes none; Tr U = 0 per block in exact
  arithmetic, so each block is rescaled to its input trace (removes rounding
  drift only).
* 1-RDM after the step: the contraction 1D = 2/(N-1) sum_q 2D[p,q,r,q].
* Reconstruction: ``sigma`` None is the Valdemoro 3-RDM; a per-spatial-orbital
  array of +1 (occupied in the Hartree-Fock reference) / -1 selects the NY one
  (Eq. (8)) for both maps of the step.
"""
import numpy as np
import torch

from . import rdm
from .residual import residual_map


def active_mask(active, r):
    """Spin-orbital mask, True where the element is kept."""
    if active is None:
        return None
    act = np.asarray(active, dtype=bool)
    so = np.concatenate([act, act])
    all4 = so[:, None, None, None] & so[None, :, None, None] & so[None, None, :, None] & so[None, None, None, :]
    return ~all4


def _trace(d2):
    r = d2.shape[0]
    return float(sum(d2[p, q, p, q] for p in range(r) for q in range(r)))


def restore_block_traces(blocks, traces):
    """Trace restoration after the update: each 2-RDM spin block is multiplied
    by the ratio of the trace it must keep (its input trace, App. A) to the
    trace it has now, so every block trace returns to its input value and
    nothing else changes shape.  A block whose input trace is zero (fewer than
    two electrons of that pair kind: the block of the exact state vanishes) is
    set to zero.  Returns the rescaled blocks and the factors."""
    scales = tuple((t0 / _trace(b)) if t0 != 0.0 else 0.0 for b, t0 in zip(blocks, traces))
    return tuple(b * c for b, c in zip(blocks, scales)), scales


def restore_traces(d2aa, d2ab, traces):
    """restore_block_traces for the two stored singlet blocks (aa, ab)."""
    (aa, ab), scales = restore_block_traces((d2aa, d2ab), traces)
    return aa, ab, scales


def norm2_spin_orbital(t4):
    return float(np.sum(np.asarray(t4) ** 2))


def energy(h, V, N, d2aa, d2ab):
    """E = Tr(K 2D) over spin orbitals (Eq. (2) with Eq. (6))."""
    r = h.shape[0]
    K = rdm.reduced_hamiltonian(h, V, N)
    _, d2 = rdm.blocks_to_spin_orbital(np.eye(r), d2aa, d2ab)
    return float(np.sum(K * d2))


def _sigma_so(sigma):
    return None if sigma is None else rdm.sigma_spin_orbital(sigma)


def residual(h, V, N, gamma, d2aa, d2ab, sigma=None):
    """R = F(K) (Eq. (4)); returns (R_aa, R_ab, ||R||^2 over spin orbitals)."""
    K = rdm.reduced_hamiltonian(h, V, N)
    d1, d2 = rdm.blocks_to_spin_orbital(gamma, d2aa, d2ab)
    R = residual_map(K, d1, d2, hermitian=True, sigma_so=_sigma_so(sigma)).numpy()
    raa, rab = rdm.spin_orbital_to_blocks(R)
    return raa, rab, norm2_spin_orbital(R)


def step(h, V, N, gamma, d2aa, d2ab, eps, active=None, keep_spin_orbital=False, sigma=None):
    """One Euler step (Eq. (9)).  Returns a dict of blocks and scalars."""
    r = h.shape[0]
    K = rdm.reduced_hamiltonian(h, V, N)
    d1, d2 = rdm.blocks_to_spin_orbital(gamma, d2aa, d2ab)
    sso = _sigma_so(sigma)
    R = residual_map(K, d1, d2, hermitian=True, sigma_so=sso).numpy()
    n2 = norm2_spin_orbital(R)
    mask = active_mask(active, r)
    Rm = R if mask is None else R * mask
    U = residual_map(Rm, d1, d2, hermitian=False, sigma_so=sso).numpy()
    raa, rab = rdm.spin_orbital_to_blocks(R)
    uaa, uab = rdm.spin_orbital_to_blocks(U)
    d2aa_1, d2ab_1, scale = restore_traces(d2aa + eps * uaa, d2ab + eps * uab,
                                           rdm.block_traces(d2aa, d2ab))
    _, d2_1 = rdm.blocks_to_spin_orbital(gamma, d2aa_1, d2ab_1)
    gamma_1 = rdm.contract_to_1rdm(d2_1, N)[:r, :r]
    e1 = float(np.sum(K * d2_1))
    out = dict(R_aa=raa, R_ab=rab, norm2=n2, U_aa=uaa, U_ab=uab,
               d2aa=d2aa_1, d2ab=d2ab_1, gamma=gamma_1, energy=e1,
               energy0=float(np.sum(K * d2)),
               trace_scale=scale)
    if keep_spin_orbital:
        out.update(R=R, U=U, Rm=Rm, K=K, d1=d1, d2=d2)
    return out


# ---------------------------------------------------------------------------
# States of any S_z (N_alpha != N_beta): the three unique spin blocks
# ---------------------------------------------------------------------------

def energy_spin(h, V, Na, Nb, d2aa, d2bb, d2ab):
    """E = Tr(K 2D) over spin orbitals (Eq. (2) with Eq. (6))."""
    r = h.shape[0]
    K = rdm.reduced_hamiltonian(h, V, Na + Nb)
    _, d2 = rdm.spin_blocks_to_spin_orbital(np.eye(r), np.eye(r), d2aa, d2bb, d2ab)
    return float(np.sum(K * d2))


def sigma_open_shell(r, Na, Nb):
    """Spin-orbital NY weights of the open-shell Hartree-Fock reference: alpha
    orbitals below Na and beta orbitals below Nb occupied (+1), the rest -1;
    alpha orbitals first."""
    p = np.arange(r)
    return np.concatenate([np.where(p < Na, 1.0, -1.0), np.where(p < Nb, 1.0, -1.0)])


def residual_spin(h, V, Na, Nb, ga, gb, d2aa, d2bb, d2ab, sigma_so=None):
    """R = F(K) (Eq. (4)) of a state of any S_z; returns (R_aa, R_bb, R_ab,
    ||R||^2 over spin orbitals).  ``sigma_so`` (2r weights, alpha orbitals
    first, +1 occupied / -1 unoccupied in the reference) selects the NY 3-RDM
    (Eq. (8)); None is Valdemoro."""
    K = rdm.reduced_hamiltonian(h, V, Na + Nb)
    d1, d2 = rdm.spin_blocks_to_spin_orbital(ga, gb, d2aa, d2bb, d2ab)
    R = residual_map(K, d1, d2, hermitian=True, sigma_so=sigma_so).numpy()
    raa, rbb, rab = rdm.spin_orbital_to_spin_blocks(R)
    return raa, rbb, rab, norm2_spin_orbital(R)


def step_spin(h, V, Na, Nb, ga, gb, d2aa, d2bb, d2ab, eps, active=None, keep_spin_orbital=False, sigma_so=None):
    """One Euler step (Eq. (9)) of a state of any S_z, with the readings of
    ``step`` (mask, trace restoration per spin block, 1-RDM contraction); the
    1-RDM blocks after the step are those of the contraction of the new 2-RDM.
    ``sigma_so`` as for ``residual_spin`` (both maps of the step)."""
    r = h.shape[0]
    N = Na + Nb
    K = rdm.reduced_hamiltonian(h, V, N)
    d1, d2 = rdm.spin_blocks_to_spin_orbital(ga, gb, d2aa, d2bb, d2ab)
    R = residual_map(K, d1, d2, hermitian=True, sigma_so=sigma_so).numpy()
    n2 = norm2_spin_orbital(R)
    mask = active_mask(active, r)
    Rm = R if mask is None else R * mask
    U = residual_map(Rm, d1, d2, hermitian=False, sigma_so=sigma_so).numpy()
    raa, rbb, rab = rdm.spin_orbital_to_spin_blocks(R)
    uaa, ubb, uab = rdm.spin_orbital_to_spin_blocks(U)
    traces = tuple(_trace(b) for b in (d2aa, d2bb, d2ab))
    (aa1, bb1, ab1), scale = restore_block_traces((d2aa + eps * uaa, d2bb + eps * ubb, d2ab + eps * uab), traces)
    _, d2_1 = rdm.spin_blocks_to_spin_orbital(ga, gb, aa1, bb1, ab1)
    g1 = rdm.contract_to_1rdm(d2_1, N)
    a, b = rdm.spin_blocks(r)
    out = dict(R_aa=raa, R_bb=rbb, R_ab=rab, norm2=n2, U_aa=uaa, U_bb=ubb, U_ab=uab,
               d2aa=aa1, d2bb=bb1, d2ab=ab1, gamma_a=g1[a, a].copy(), gamma_b=g1[b, b].copy(),
               energy=float(np.sum(K * d2_1)), energy0=float(np.sum(K * d2)), trace_scale=scale)
    if keep_spin_orbital:
        out.update(R=R, U=U, Rm=Rm, K=K, d1=d1, d2=d2)
    return out
