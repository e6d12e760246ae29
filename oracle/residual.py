"""The ACSE residual map (oracle, test only).

For any two-body coefficient tensor X with the pair exchange symmetry
X^{pq}_{rs} = X^{qp}_{sr}, define

    F(X)^{ij}_{kl} = 1/2 sum_{pqrs} X^{pq}_{rs} <psi| [a+_i a+_j a_l a_k, a+_p a+_q a_s a_r] |psi>.

The residual of Eq. (4) is R = F(K) with the reduced Hamiltonian K of Eq. (2)
(H = 1/2 sum K a+a+aa on N electrons), and the update of Eq. (9) is
U = F(R_m) = 1/2 <[a+a+aa, A]> with A = sum R_m a+a+aa, i.e. the derivative of
2D along psi(eps) = exp(eps A) psi.

Normal ordering the commutator (the derivation of App. B, Eqs. (B1)-(B6),
using only the antisymmetry of the RDMs and the pair exchange of X) gives

    F(X)^{ij}_{kl} =  2 sum_rs  X^{kl}_{rs} 2D^{ij}_{rs}  - 2 sum_pq  X^{pq}_{ij} 2D^{pq}_{kl}
                    - 6 sum_prs X^{kp}_{rs} 3D^{ijp}_{rsl} + 6 sum_prs X^{lp}_{rs} 3D^{ijp}_{rsk}
                    - 6 sum_pqr X^{pq}_{rj} 3D^{ipq}_{rlk} + 6 sum_pqr X^{pq}_{ri} 3D^{jpq}_{rlk}.

Readings (each pinned by brute force in the tests):

* Sign.  Eq. (5) / (B6), read with K as above, equals -<[O,H]> term by term;
  Eq. (4) defines R = +<[O,H]>.  We follow Eq. (4).  The update U = F(F(K))
  is even in this sign, so the 2-RDM trajectory is the same either way.
* Transposition forms.  With A = 2 sum K^{kl}_{qp} 2D^{ij}_{qp} and
  B^{ij}_{kl} = 6 sum K^{kp}_{rq} 3D^{ijp}_{rql}, C = B - B(k<->l) of
  Eqs. (B8)-(B9), and T' denoting the exchange (ij) <-> (kl):
      Hermitian X (the residual):        F = A - A' - C + C'
      anti-Hermitian X (the update):     F = A + A' - C - C'
  i.e. for the update BOTH transposed terms change sign (App. B states only
  the C term).
* E intermediate of App. D.1, Eq. (D4) lies inside the 1/9.
"""
import numpy as np
import torch

from . import rdm


# ---------------------------------------------------------------------------
# Tier A: materialised 3-RDM (small n)
# ---------------------------------------------------------------------------

def residual_map_dense(X, d2, d3):
    """F(X) with a materialised 3D (axes [i,j,p,r,s,l]); any 3D (exact or reconstructed)."""
    e = np.einsum
    return (2.0 * e('klrs,ijrs->ijkl', X, d2) - 2.0 * e('pqij,pqkl->ijkl', X, d2)
            - 6.0 * e('kprs,ijprsl->ijkl', X, d3) + 6.0 * e('lprs,ijprsk->ijkl', X, d3)
            - 6.0 * e('pqrj,ipqrlk->ijkl', X, d3) + 6.0 * e('pqri,jpqrlk->ijkl', X, d3))


def eq5_as_printed(K, d2, d3):
    """Eq. (5) exactly as printed (documents reading C-1: it equals -F(K))."""
    e = np.einsum
    return (2.0 * e('ijqp,klqp->ijkl', K, d2) + 6.0 * e('kprq,ijprql->ijkl', K, d3)
            - 6.0 * e('lprq,ijprqk->ijkl', K, d3) - 2.0 * e('klqp,ijqp->ijkl', K, d2)
            - 6.0 * e('pqri,jpqrlk->ijkl', K, d3) + 6.0 * e('pqrj,ipqrlk->ijkl', K, d3))


# ---------------------------------------------------------------------------
# Tier B: factorised, the 3-RDM is never formed (App. D.1 and App. B)
# ---------------------------------------------------------------------------

def _t(x):
    if isinstance(x, torch.Tensor):
        return x.to(torch.float64)
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))


def _mm4(a, b, a_rows, a_cols, b_cols):
    """out[a_rows..., b_cols...] = sum over a_cols of a * b (b indexed [a_cols, b_cols]),
    as one matrix product of the flattened operands."""
    return a.reshape(a_rows, a_cols) @ b.reshape(a_cols, b_cols)


def contraction_b(X, d1, d2):
    """B^{ij}_{kl} = 6 sum_pqr X^{kp}_{rq} 3D_V^{ijp}_{rql} through the M intermediate of
    App. C, Eq. (C3) and the factorisation of App. D.1, Eqs. (D2)-(D4):

      sum_pqr X^{kp}_{rq} 3D^{ijp}_{rql} = 1/9 [ sum X^{kp}_{rq} M^{ij}_{rq} D^p_l
            - sum (X^{kp}_{rq} - X^{kp}_{qr}) M^{ij}_{lq} D^p_r + E^{ij}_{kl} - E^{ji}_{kl} ],
      E^{ij}_{kl} = sum (X^{kp}_{rq} - X^{kp}_{qr}) M^{ip}_{lq} D^j_r - X^{kp}_{rq} M^{ip}_{rq} D^j_l.

    Torch float64 so that the oracle is differentiable.  Axes [i,j,k,l].
    """
    X, d1, d2 = _t(X), _t(d1), _t(d2)
    n = d1.shape[0]
    wedge = 0.5 * (torch.einsum('ir,jq->ijrq', d1, d1) - torch.einsum('jr,iq->ijrq', d1, d1))
    M = 3.0 * (d2 - wedge) + wedge                                   # (C3)
    n2 = n * n
    # first term: sum_rq M^{ij}_{rq} (sum_p X^{kp}_{rq} D^p_l)
    xd = torch.einsum('kprq,pl->klrq', X, d1)
    term_a = (M.reshape(n2, n2) @ xd.reshape(n2, n2).T).reshape(n, n, n, n)
    del xd
    # second term: - sum_q (sum_pr (X^{kp}_{rq} - X^{kp}_{qr}) D^p_r) M^{ij}_{lq}
    xa = X - X.permute(0, 1, 3, 2)
    fq = torch.einsum('kprq,pr->kq', xa, d1)
    term_b = -torch.einsum('kq,ijlq->ijkl', fq, M)
    # E intermediate (D3)
    xaj = torch.einsum('kprq,jr->kjpq', xa, d1)                      # [k,j,(p,q)]
    mil = M.permute(0, 2, 1, 3)                                       # [i,l,p,q]
    e1 = (xaj.reshape(n2, n2) @ mil.reshape(n2, n2).T).reshape(n, n, n, n)  # [k,j,i,l]
    e1 = e1.permute(2, 1, 0, 3)                                       # [i,j,k,l]
    del xaj, xa
    tt = torch.einsum('iprq,kprq->ik', M, X)
    E = e1 - torch.einsum('ik,jl->ijkl', tt, d1)
    del e1
    bt = (term_a + term_b + E - E.permute(1, 0, 2, 3)) / 9.0
    return 6.0 * bt


def contraction_b_ny(X, d1, d2, sigma_so):
    """The NY cumulant's share of B: 6 sum_pqr X^{kp}_{rq} 3Delta^{ijp}_{rql}
    with the 3Delta of Eq. (8), never formed.

    Collapsing the 36 signed permutations with the pair antisymmetry of
    2Delta leaves 9 distinct products, each with weight 4: the upper index x
    of the first cumulant is i (+), j (-) or p (+, the second then carrying
    (i, j)); the lower index y of the second cumulant is l (+), r (-) or q (-),
    the first carrying the other two in their order.  Each product is two
    pairwise contractions with n^4 intermediates (n^6 work), summed over the
    orbital a with weight sigma_a.  The x = j products are the x = i ones with
    i and j exchanged.  Axes [i,j,k,l].  Torch float64 (differentiable).
    """
    X, d1, d2 = _t(X), _t(d1), _t(d2)
    s = _t(sigma_so)
    c2 = d2 - 0.5 * (torch.einsum('ir,jq->ijrq', d1, d1) - torch.einsum('jr,iq->ijrq', d1, d1))
    cs = c2 * s[None, None, :, None]          # sigma_a on the first lower index: 2Delta^{..}_{a.}
    e = torch.einsum
    # y = l: first cumulant lower (r, q), second (a, l)
    t_il = e('kpia,jpal->ijkl', e('kprq,iarq->kpia', X, c2), cs)
    t_pl = e('ka,ijal->ijkl', e('kprq,parq->ka', X, c2), cs)
    # y = r: first cumulant lower (l, q), second (a, r)
    t_ir = e('kqja,ialq->ijkl', e('kprq,jpar->kqja', X, cs), c2)
    t_pr = e('kral,ijar->ijkl', e('kprq,palq->kral', X, c2), cs)
    # y = q: first cumulant lower (r, l), second (a, q)
    t_iq = e('krja,iarl->ijkl', e('kprq,jpaq->krja', X, cs), c2)
    t_pq = e('kqal,ijaq->ijkl', e('kprq,parl->kqal', X, c2), cs)

    def sw(t):
        return t - t.permute(1, 0, 2, 3)
    return 4.0 * (sw(t_il) + t_pl - sw(t_ir) - t_pr - sw(t_iq) - t_pq)


def residual_map(X, d1, d2, hermitian, sigma_so=None):
    """F(X) via Eqs. (B8)-(B9) with the factorised B (tier B).

    A^{ij}_{kl} = 2 sum_qp X^{kl}_{qp} 2D^{ij}_{qp};  C = B - B(k<->l);
    Hermitian X:       F = A - A' - C + C'
    anti-Hermitian X:  F = A + A' - C - C'      (' : exchange (ij)<->(kl)).
    With sigma_so (spin-orbital HF occupations, +1 / -1) the 3-RDM is the NY
    one, 3D_V + 3Delta_NY (Eq. (8)); F is linear in 3D, so B gains the
    cumulant's share.
    """
    X, d1, d2 = _t(X), _t(d1), _t(d2)
    n = d1.shape[0]
    n2 = n * n
    A = 2.0 * (d2.reshape(n2, n2) @ X.reshape(n2, n2).T).reshape(n, n, n, n)
    B = contraction_b(X, d1, d2)
    if sigma_so is not None:
        B = B + contraction_b_ny(X, d1, d2, sigma_so)
    C = B - B.permute(0, 1, 3, 2)
    del B
    At = A.permute(2, 3, 0, 1)
    Ct = C.permute(2, 3, 0, 1)
    if hermitian:
        return A - At - C + Ct
    return A + At - C - Ct


# ---------------------------------------------------------------------------
# Single elements at any size (plain definition with 3D_V formed slice by slice)
# ---------------------------------------------------------------------------

_LET = 'abcdef'


def d3v_slice(M, D, upper, lower):
    """Slice of 3D_V^{abc}_{def} = 1/9 sum_{x,y} (-1)^{pos x + pos y} D_{xy} M^{abc minus x}_{def minus y}
    (the compact statement of App. C, Eq. (C5)).  Entries of ``upper``/``lower`` are
    ints (fixed) or None (free); the result has the free axes in order."""
    spec = list(upper) + list(lower)
    free = [_LET[t] for t, v in enumerate(spec) if v is None]
    out = 0.0
    for xi in range(3):
        for yi in range(3):
            sign = -1.0 if (xi + yi) % 2 else 1.0
            ux = [u for u in range(3) if u != xi]
            ly = [3 + w for w in range(3) if w != yi]
            m_pos = ux + ly
            d_pos = [xi, 3 + yi]
            m_idx = tuple(slice(None) if spec[t] is None else spec[t] for t in m_pos)
            d_idx = tuple(slice(None) if spec[t] is None else spec[t] for t in d_pos)
            m_let = ''.join(_LET[t] for t in m_pos if spec[t] is None)
            d_let = ''.join(_LET[t] for t in d_pos if spec[t] is None)
            term = np.einsum(f'{m_let},{d_let}->{"".join(free)}', M[m_idx], D[d_idx])
            out = out + sign * term
    return out / 9.0


def residual_elements(X, d1, d2, index_list):
    """F(X)^{ij}_{kl} for each (i,j,k,l) in index_list, from the six-term form in
    the module docstring with the Valdemoro 3D evaluated on the slices it needs."""
    M = rdm.m_intermediate(d1, d2)
    out = []
    for (i, j, k, l) in index_list:
        s_ijl = d3v_slice(M, d1, (i, j, None), (None, None, l))   # [p,r,s]
        s_ijk = d3v_slice(M, d1, (i, j, None), (None, None, k))
        s_ilk = d3v_slice(M, d1, (i, None, None), (None, l, k))   # [p,q,r]
        s_jlk = d3v_slice(M, d1, (j, None, None), (None, l, k))
        v = (2.0 * np.sum(X[k, l] * d2[i, j]) - 2.0 * np.sum(X[:, :, i, j] * d2[:, :, k, l])
             - 6.0 * np.sum(X[k] * s_ijl) + 6.0 * np.sum(X[l] * s_ijk)
             - 6.0 * np.sum(X[:, :, :, j] * s_ilk) + 6.0 * np.sum(X[:, :, :, i] * s_jlk))
        out.append(v)
    return np.array(out)
