"""Spin-orbital tensors of the ACSE from spatial inputs (oracle, test only).

Conventions (spin orbitals n = 2r, alpha first):

* 1D[p,r]          = <a+_p a_r>                          (Eq. (6) trace N)
* 2D[p,q,r,s]      = 1/2 <a+_p a+_q a_s a_r>             (Eq. (6))
* 3D[p,q,t,r,s,u]  = 1/6 <a+_p a+_q a+_t a_u a_s a_r>    (Eq. (6))
* K[p,q,r,s]       = coefficient of the reduced Hamiltonian of Eq. (2) such
                     that H = 1/2 sum K a+_p a+_q a_s a_r on N electrons and
                     E = Tr(K 2D).

Reading of Eq. (2): the printed prefactors mix a two-electron operator
without 1/2 (Eq. (1)) with an unhalved 1/(N-1) one-electron term; we take the
scale fixed by the operator identity  sum_pr h a+_p a_r =
1/(N-1) sum_pqr h a+_p a+_q a_q a_r  on the N-electron space, i.e.
K^{pq}_{rs} = <pq|rs> + (h_pr d_qs + h_qs d_pr)/(N-1), with the chemists'
integral V[p,q,r,s] = (pq|rs) and <pq|rs> = (pr|qs).
"""
import numpy as np


def spin_blocks(r):
    """Slices of the alpha and beta spin orbitals."""
    return slice(0, r), slice(r, 2 * r)


def reduced_hamiltonian(h, V, N):
    """Spin-orbital K of Eq. (2) (reading above)."""
    r = h.shape[0]
    n = 2 * r
    a, b = spin_blocks(r)
    hso = np.zeros((n, n))
    hso[a, a] = h
    hso[b, b] = h
    eri = np.zeros((n, n, n, n))
    phys = V.transpose(0, 2, 1, 3)
    for s1 in (a, b):
        for s2 in (a, b):
            eri[s1, s2, s1, s2] = phys
    eye = np.eye(n)
    one = (np.einsum('pr,qs->pqrs', hso, eye) + np.einsum('qs,pr->pqrs', hso, eye)) / (N - 1)
    return eri + one


def spatial_reduced_hamiltonian(h, V, N):
    """Spatial G_s[p,q,r,s] = V[p,r,q,s] + (h_pr d_qs + h_qs d_pr)/(N-1); the
    spin-orbital K is G_s on every block with d(s_p,s_r) d(s_q,s_s)."""
    r = h.shape[0]
    eye = np.eye(r)
    return (V.transpose(0, 2, 1, 3) + (np.einsum('pr,qs->pqrs', h, eye)
                                       + np.einsum('qs,pr->pqrs', h, eye)) / (N - 1))


def blocks_to_spin_orbital(gamma, d2aa, d2ab):
    """Spin-orbital (1D, 2D) from the stored singlet blocks (the alpha-alpha and
    alpha-beta 2-RDM blocks of the spatial-orbital working equations, with the
    beta-beta block equal to alpha-alpha for singlets).

    2D(pa qb | ra sb) = d2ab[p,q,r,s]; the other three mixed blocks follow from
    fermionic antisymmetry and the pair exchange (pq)(rs) -> (qp)(sr).
    """
    r = gamma.shape[0]
    n = 2 * r
    a, b = spin_blocks(r)
    d1 = np.zeros((n, n))
    d1[a, a] = gamma
    d1[b, b] = gamma
    d2 = np.zeros((n, n, n, n))
    d2[a, a, a, a] = d2aa
    d2[b, b, b, b] = d2aa
    d2[a, b, a, b] = d2ab
    d2[b, a, b, a] = d2ab.transpose(1, 0, 3, 2)
    d2[a, b, b, a] = -d2ab.transpose(0, 1, 3, 2)
    d2[b, a, a, b] = -d2ab.transpose(1, 0, 2, 3)
    return d1, d2


def spin_orbital_to_blocks(t4):
    """(alpha-alpha, alpha-beta) spatial blocks of a spin-orbital 4-index tensor."""
    r = t4.shape[0] // 2
    a, b = spin_blocks(r)
    return t4[a, a, a, a].copy(), t4[a, b, a, b].copy()


def spin_blocks_to_spin_orbital(ga, gb, d2aa, d2bb, d2ab):
    """Spin-orbital (1D, 2D) of a state of any S_z from its unique spin blocks
    (the fixed-spin blocks named in the Theory section: alpha-alpha,
    beta-beta and alpha-beta):
      1D(pa|ra) = ga, 1D(pb|rb) = gb;
      2D(pa qa|ra sa) = d2aa, 2D(pb qb|rb sb) = d2bb, 2D(pa qb|ra sb) = d2ab;
    the three other mixed blocks follow from the fermionic antisymmetry of
    each index pair alone: 2D(pb qa|rb sa) = d2ab[q,p,s,r],
    2D(pa qb|rb sa) = -d2ab[p,q,s,r], 2D(pb qa|ra sb) = -d2ab[q,p,r,s].
    With gb = ga and d2bb = d2aa (and d2ab invariant under (pq)(rs) ->
    (qp)(sr)) this is the singlet lift above."""
    r = ga.shape[0]
    n = 2 * r
    a, b = spin_blocks(r)
    d1 = np.zeros((n, n))
    d1[a, a] = ga
    d1[b, b] = gb
    d2 = np.zeros((n, n, n, n))
    d2[a, a, a, a] = d2aa
    d2[b, b, b, b] = d2bb
    d2[a, b, a, b] = d2ab
    d2[b, a, b, a] = d2ab.transpose(1, 0, 3, 2)
    d2[a, b, b, a] = -d2ab.transpose(0, 1, 3, 2)
    d2[b, a, a, b] = -d2ab.transpose(1, 0, 2, 3)
    return d1, d2


def spin_orbital_to_spin_blocks(t4):
    """(alpha-alpha, beta-beta, alpha-beta) spatial blocks of a spin-orbital 4-index tensor."""
    r = t4.shape[0] // 2
    a, b = spin_blocks(r)
    return t4[a, a, a, a].copy(), t4[b, b, b, b].copy(), t4[a, b, a, b].copy()


def block_traces(d2aa, d2ab):
    """Tr 2D_aa and Tr 2D_ab (App. A: N_a(N_a-1)/2 and N_a N_b/2)."""
    r = d2aa.shape[0]
    pq = np.arange(r)
    taa = sum(d2aa[p, q, p, q] for p in pq for q in pq)
    tab = sum(d2ab[p, q, p, q] for p in pq for q in pq)
    return float(taa), float(tab)


def contract_to_1rdm(d2, N):
    """1D[p,r] = 2/(N-1) sum_q 2D[p,q,r,q]  (Eq. (6) normalisations)."""
    return 2.0 * np.einsum('pqrq->pr', d2) / (N - 1)


# ---------------------------------------------------------------------------
# Cumulant expansion and the Valdemoro 3-RDM (Eq. (7), App. C)
# ---------------------------------------------------------------------------

def wedge11(d1):
    """(1D ^ 1D)^{ij}_{rq} = 1/2 (1D^i_r 1D^j_q - 1D^j_r 1D^i_q)  (App. C, Eq. (C2))."""
    return 0.5 * (np.einsum('ir,jq->ijrq', d1, d1) - np.einsum('jr,iq->ijrq', d1, d1))


def cumulant2(d1, d2):
    """2-body cumulant: 2D = 2Delta + 1D ^ 1D  (Eq. (7))."""
    return d2 - wedge11(d1)


def m_intermediate(d1, d2):
    """M^{ij}_{rq} = 3 2Delta^{ij}_{rq} + 1/2(1D^i_r 1D^j_q - 1D^j_r 1D^i_q)  (App. C, Eq. (C3))."""
    return 3.0 * cumulant2(d1, d2) + wedge11(d1)


def d3_valdemoro(d1, d2):
    """Valdemoro 3-RDM, 3Delta = 0, in the nine-term form of App. C, Eq. (C5):

    3D^{ijp}_{rql} = 1/9 ( M^{ij}_{rq} D^p_l - M^{ij}_{lq} D^p_r - M^{ij}_{rl} D^p_q
                         - M^{ip}_{rq} D^j_l + M^{ip}_{lq} D^j_r + M^{ip}_{rl} D^j_q
                         + M^{jp}_{rq} D^i_l - M^{jp}_{lq} D^i_r - M^{jp}_{rl} D^i_q ).

    Returned with axes [i, j, p, r, q, l].  Materialised: n^6 memory, small n only.
    """
    M = m_intermediate(d1, d2)
    D = d1
    e = np.einsum
    t = (e('ijrq,pl->ijprql', M, D) - e('ijlq,pr->ijprql', M, D) - e('ijrl,pq->ijprql', M, D)
         - e('iprq,jl->ijprql', M, D) + e('iplq,jr->ijprql', M, D) + e('iprl,jq->ijprql', M, D)
         + e('jprq,il->ijprql', M, D) - e('jplq,ir->ijprql', M, D) - e('jprl,iq->ijprql', M, D))
    return t / 9.0


def gamma3_valdemoro_wform(g1, g2):
    """Independent form of the same functional in unnormalised RDMs
    (Gamma1 = 1D, Gamma2 = 2 2D, Gamma3 = 6 3D):

    Gamma3^{abc}_{def} = sum_{x in (a,b,c), y in (d,e,f)} (-1)^{pos x + pos y}
                         Gamma1_{xy} W^{abc minus x}_{def minus y},
    W = Gamma2 - 2/3 (Gamma1 ^ Gamma1)_unnormalised.

    (1/3 of the antisymmetrised Gamma1 product inside W summed over the nine
    Laplace cofactors gives the full 3x3 determinant of Gamma1, and the
    cumulant part gives the nine 2Delta ^ 1D terms of Eq. (7) with 3Delta = 0.)
    Axes [a, b, c, d, e, f].
    """
    w = g2 - (2.0 / 3.0) * (np.einsum('ad,be->abde', g1, g1) - np.einsum('ae,bd->abde', g1, g1))
    e = np.einsum
    return (e('ad,bcef->abcdef', g1, w) - e('ae,bcdf->abcdef', g1, w) + e('af,bcde->abcdef', g1, w)
            - e('bd,acef->abcdef', g1, w) + e('be,acdf->abcdef', g1, w) - e('bf,acde->abcdef', g1, w)
            + e('cd,abef->abcdef', g1, w) - e('ce,abdf->abcdef', g1, w) + e('cf,abde->abcdef', g1, w))


# ---------------------------------------------------------------------------
# Nakatsuji-Yasuda approximation to the 3-cumulant (Eq. (8); App. D, NY part)
# ---------------------------------------------------------------------------

def sigma_spin_orbital(sigma):
    """Spin-orbital weights from the spatial ones (both spins of an orbital
    share its Hartree-Fock occupation): +1 occupied, -1 unoccupied."""
    s = np.asarray(sigma, dtype=np.float64)
    return np.concatenate([s, s])


def _perm_sign(p):
    p = list(p)
    sign = 1.0
    for i in range(len(p)):
        while p[i] != i:
            j = p[i]
            p[i], p[j] = p[j], p[i]
            sign = -sign
    return sign


def d3_ny_cumulant(d1, d2, sigma_so):
    """3Delta^{ijp}_{rql} = 1/6 sum_a sigma_a A[ 2Delta^{ia}_{rq} 2Delta^{jp}_{al} ]
    (Eq. (8)), A the sum over all signed permutations of the upper indices
    (i, j, p) and, independently, of the lower ones (r, q, l) -- 36 terms, a
    unit weight each, as the explicit expansion of the NY appendix lists them;
    a stays fixed.  2Delta is the cumulant of Eq. (7) in the normalisation of
    Eq. (6), so that 3D = 3D_V + 3Delta.

    The plain definition, materialised with axes [i, j, p, r, q, l]: n^6
    memory, small n only.  Pinned against the exact 3-cumulant of a
    determinant with a small doubles admixture, which it matches through
    second order.
    """
    c2 = cumulant2(d1, d2)
    prod = np.einsum('a,iarq,jpal->ijprql', np.asarray(sigma_so, dtype=np.float64), c2, c2)
    out = np.zeros_like(prod)
    import itertools
    for up in itertools.permutations(range(3)):
        for lo in itertools.permutations(range(3)):
            out += _perm_sign(up) * _perm_sign(lo) * prod.transpose(list(up) + [3 + x for x in lo])
    return out / 6.0


def d3_ny(d1, d2, sigma_so):
    """NY 3-RDM: the Valdemoro terms of Eq. (7) plus the NY 3-cumulant."""
    return d3_valdemoro(d1, d2) + d3_ny_cumulant(d1, d2, sigma_so)
