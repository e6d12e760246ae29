"""Adjoints of the residual and the energy (oracle; test infrastructure only).

For a cotangent (Rbar_aa, Rbar_ab) on the residual blocks of Eq. (4) (with
the Valdemoro 3-RDM, or the NY one of Eq. (8) when occupations are given), the
vector-Jacobian product is the gradient of

    L = <Rbar_aa, R_aa> + <Rbar_ab, R_ab>

with respect to the spatial inputs (h, V, gamma, d2aa, d2ab).  For the energy
E = Tr(K 2D) (Eq. (2), Eq. (6)) it is the gradient of Ebar * E.

How it is computed: reverse-mode automatic differentiation (torch.autograd,
a library primitive) through the oracle's own torch forward.  That forward is
the spin-orbital reduced Hamiltonian of Eq. (2), the singlet embedding of the
blocks, and the factorised residual map of App. D.1 with Eqs. (B8)-(B9).
No hand-derived step is involved.

The inputs are structured: h and gamma are symmetric; V has the 8-fold
symmetry of (pq|rs); d2aa is antisymmetric within each pair and Hermitian;
d2ab is Hermitian and symmetric under (pq)(rs) -> (qp)(sr).  The gradient of
a function restricted to such a subspace is the orthogonal projection of the
unrestricted gradient onto it.  Each result here is projected that way
(reading: the adjoint is defined on the symmetric input space, which is what
finite differences along symmetry-respecting directions measure).

Pins (tests/test_oracle_adjoint.py):

* central finite differences of the numpy forward (oracle.step);
* exact linearity of R in (h, V), and bilinearity of E;
* idempotence of the projections.
"""
import numpy as np
import torch

from . import residual as rs

__all__ = ["proj_sym2", "proj_V", "proj_aa", "proj_ab", "reduced_hamiltonian_t",
           "blocks_to_spin_orbital_t", "residual_blocks_t", "energy_t", "residual_vjp",
           "energy_vjp"]

e = torch.einsum


def _t(x):
    if isinstance(x, torch.Tensor):
        return x.to(torch.float64)
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))


# --- projections onto the symmetry subspaces of the inputs ------------------

def proj_sym2(x):
    """Symmetric part of a matrix (h, gamma)."""
    return 0.5 * (x + x.transpose(0, 1))


def proj_V(x):
    """Average over the 8 index permutations that leave (pq|rs) invariant."""
    perms = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
             (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]
    return sum(x.permute(*p) for p in perms) / 8.0


def proj_aa(x):
    """Antisymmetric in (p,q) and in (r,s), then Hermitian under (pq) <-> (rs)."""
    y = 0.25 * (x - x.permute(1, 0, 2, 3) - x.permute(0, 1, 3, 2) + x.permute(1, 0, 3, 2))
    return 0.5 * (y + y.permute(2, 3, 0, 1))


def proj_ab(x):
    """Hermitian under (pq) <-> (rs), then symmetric under (pq)(rs) -> (qp)(sr)."""
    y = 0.5 * (x + x.permute(2, 3, 0, 1))
    return 0.5 * (y + y.permute(1, 0, 3, 2))


# --- differentiable forward ----------------------------------------------------

def reduced_hamiltonian_t(h, V, N):
    """Spin-orbital K of Eq. (2) in torch (same reading as oracle.rdm):
    K[p,q,r,s] = <pq|rs> + (h_pr d_qs + h_qs d_pr)/(N-1), <pq|rs> = (pr|qs)."""
    r = h.shape[0]
    n = 2 * r
    hso = torch.zeros((n, n), dtype=torch.float64)
    hso[:r, :r] = h
    hso[r:, r:] = h
    phys = V.permute(0, 2, 1, 3)
    eri = torch.zeros((n, n, n, n), dtype=torch.float64)
    for s1 in (slice(0, r), slice(r, n)):
        for s2 in (slice(0, r), slice(r, n)):
            eri[s1, s2, s1, s2] = phys
    eye = torch.eye(n, dtype=torch.float64)
    return eri + (e('pr,qs->pqrs', hso, eye) + e('qs,pr->pqrs', hso, eye)) / (N - 1)


def blocks_to_spin_orbital_t(gamma, d2aa, d2ab):
    """Spin-orbital (1D, 2D) from the singlet blocks, in torch (same embedding as
    oracle.rdm.blocks_to_spin_orbital)."""
    r = gamma.shape[0]
    n = 2 * r
    a, b = slice(0, r), slice(r, n)
    d1 = torch.zeros((n, n), dtype=torch.float64)
    d1[a, a] = gamma
    d1[b, b] = gamma
    d2 = torch.zeros((n, n, n, n), dtype=torch.float64)
    d2[a, a, a, a] = d2aa
    d2[b, b, b, b] = d2aa
    d2[a, b, a, b] = d2ab
    d2[b, a, b, a] = d2ab.permute(1, 0, 3, 2)
    d2[a, b, b, a] = -d2ab.permute(0, 1, 3, 2)
    d2[b, a, a, b] = -d2ab.permute(1, 0, 2, 3)
    return d1, d2


def residual_blocks_t(h, V, N, gamma, d2aa, d2ab, sigma_so=None):
    """(R_aa, R_ab) of Eq. (4) as a differentiable torch function; ``sigma_so``
    (2r spin-orbital occupations) selects the NY 3-RDM."""
    r = h.shape[0]
    K = reduced_hamiltonian_t(h, V, N)
    d1, d2 = blocks_to_spin_orbital_t(gamma, d2aa, d2ab)
    R = rs.residual_map(K, d1, d2, hermitian=True, sigma_so=sigma_so)
    return R[:r, :r, :r, :r], R[:r, r:, :r, r:]


def energy_t(h, V, N, d2aa, d2ab):
    """E = Tr(K 2D) over spin orbitals, differentiable."""
    K = reduced_hamiltonian_t(h, V, N)
    r = h.shape[0]
    _, d2 = blocks_to_spin_orbital_t(torch.zeros((r, r), dtype=torch.float64), d2aa, d2ab)
    return (K * d2).sum()


# --- vector-Jacobian products --------------------------------------------------

def residual_vjp(h, V, N, gamma, d2aa, d2ab, Rbar_aa, Rbar_ab, sigma=None):
    """Projected gradients of <Rbar, R> as numpy arrays:
    dict(h, V, gamma, d2aa, d2ab).  ``sigma`` (per spatial orbital, +1 / -1,
    the same for both spins) selects the NY 3-RDM; None is Valdemoro."""
    x = [_t(a).clone().requires_grad_(True) for a in (h, V, gamma, d2aa, d2ab)]
    sso = None if sigma is None else np.concatenate([np.asarray(sigma, float)] * 2)
    Raa, Rab = residual_blocks_t(x[0], x[1], N, x[2], x[3], x[4], sigma_so=sso)
    L = (_t(Rbar_aa) * Raa).sum() + (_t(Rbar_ab) * Rab).sum()
    g = torch.autograd.grad(L, x)
    proj = (proj_sym2, proj_V, proj_sym2, proj_aa, proj_ab)
    return {k: p(gi).detach().numpy() for k, p, gi in
            zip(("h", "V", "gamma", "d2aa", "d2ab"), proj, g)}


def energy_vjp(h, V, N, d2aa, d2ab, Ebar=1.0):
    """Projected gradients of Ebar * E as numpy arrays: dict(h, V, d2aa, d2ab)."""
    x = [_t(a).clone().requires_grad_(True) for a in (h, V, d2aa, d2ab)]
    E = energy_t(x[0], x[1], N, x[2], x[3])
    g = torch.autograd.grad(Ebar * E, x)
    proj = (proj_sym2, proj_V, proj_aa, proj_ab)
    return {k: p(gi).detach().numpy() for k, p, gi in zip(("h", "V", "d2aa", "d2ab"), proj, g)}
