"""Closed forms for a closed-shell Slater determinant in spatial spin blocks
(test helper, not a test module).

For a single determinant the Valdemoro reconstruction of Eq. (7) is exact, so
the residual of Eq. (4) is the exact commutator expectation, which the
Slater-Condon rules give in closed form.  In spin orbitals (o = occupied,
v = virtual, <pq||rs> = <pq|rs> - <pq|sr>, f the Fock matrix):

    X^{pq}_{rs} = <pq||rs> o_p o_q v_r v_s + S2^{pq}_{rs},
    S1^{pq}_{rs} = f_rp delta_qs o_p o_q v_r [p != q],
    S2 = S1 - S1(p<->q) - S1(r<->s) + S1(p<->q, r<->s),
    R = X - X^T   (T: (pq) <-> (rs)).

``tests/test_oracle_pins.py`` pins this spin-orbital form to Fock-space brute
force.  Written out on the spin blocks of a closed shell (orbitals 0..na-1
doubly occupied; <pq|rs> = (pr|qs) = V[p,r,q,s], zero unless the spins of p, r
and of q, s agree):

    alpha-alpha: <pq||rs> = Vt - Vt(r<->s) with Vt[p,q,r,s] = V[p,r,q,s]; the
                 S1 terms all stay in the block.
    alpha-beta:  <pq||rs> = Vt; of the S1 terms only S1 itself
                 (f_rp delta_qs o_p o_q v_r) and the doubly swapped one
                 (f_sq delta_pr o_p o_q v_s) survive the spin deltas.

with the closed-shell Fock matrix f = h + sum_{m occ} (2 (..|mm) - (.m|m.)) and
the energy E = 2 sum_i h_ii + sum_ij (2 (ii|jj) - (ij|ji)).
"""
import numpy as np


def occupation(r, na):
    o = np.zeros(r, bool)
    o[:na] = True
    return o


def rdms(r, na):
    """gamma, d2aa, d2ab of the determinant (Eq. (6) normalisation)."""
    g = np.diag(occupation(r, na).astype(np.float64))
    d2aa = 0.5 * (np.einsum('pr,qs->pqrs', g, g) - np.einsum('ps,qr->pqrs', g, g))
    d2ab = 0.5 * np.einsum('pr,qs->pqrs', g, g)
    return g, d2aa, d2ab


def fock(h, V, na):
    m = np.arange(na)
    return h + 2.0 * V[:, :, m, m].sum(axis=2) - V[:, m, m, :].sum(axis=1)


def energy(h, V, na):
    i = np.arange(na)
    J = V[i][:, i][:, :, i][:, :, :, i]
    return 2.0 * np.trace(h[:na, :na]) + 2.0 * np.einsum('iijj->', J) - np.einsum('ijji->', J)


def residual_blocks(h, V, na):
    """(R_aa, R_ab) of the determinant in its own orbital basis."""
    r = h.shape[0]
    o = occupation(r, na).astype(np.float64)
    v = 1.0 - o
    f = fock(h, V, na)
    Vt = np.ascontiguousarray(V.transpose(0, 2, 1, 3))
    mask = o[:, None, None, None] * o[None, :, None, None] * v[None, None, :, None] * v[None, None, None, :]
    eye = np.eye(r)
    # S1[p,q,r,s] = f[r,p] delta_qs o_p o_q v_r (p != q inside the block)
    fo = (f.T * o[:, None] * v[None, :])          # [p, r]: f[r,p] o_p v_r
    S1 = np.einsum('pr,qs->pqrs', fo, eye * o[:, None])
    S1aa = S1 * (1.0 - eye)[:, :, None, None]
    S2aa = S1aa - S1aa.transpose(1, 0, 2, 3) - S1aa.transpose(0, 1, 3, 2) + S1aa.transpose(1, 0, 3, 2)
    del S1aa
    Xaa = (Vt - Vt.transpose(0, 1, 3, 2)) * mask + S2aa
    del S2aa
    Raa = Xaa - Xaa.transpose(2, 3, 0, 1)
    del Xaa
    # alpha-beta: S1 + its doubly swapped partner f[s,q] delta_pr o_p o_q v_s
    Xab = Vt * mask + S1 + S1.transpose(1, 0, 3, 2)
    del S1, Vt, mask
    Rab = Xab - Xab.transpose(2, 3, 0, 1)
    return np.ascontiguousarray(Raa), np.ascontiguousarray(Rab)


def rot2(t, U):
    return U.T @ t @ U


def rot4(t, U):
    """t'[a,b,c,d] = sum t[p,q,r,s] U[p,a] U[q,b] U[r,c] U[s,d]."""
    x = t
    for _ in range(4):
        x = np.tensordot(x, U, axes=([0], [0]))
    return np.ascontiguousarray(x)
