"""Brute-force second quantisation in the full Fock space (oracle, test only).

Spin-orbital convention used throughout the oracle: ``n = 2 r`` spin orbitals,
alpha first (P < r is alpha orbital P, P >= r is beta orbital P - r).  A Fock
basis state is the integer whose bit P is the occupation of spin orbital P.
Creation/annihilation operators are Jordan-Wigner matrices:
``a_P |..> = (-1)^(number of occupied Q < P) |.. without P>``.

Everything here is the plain definition: operators are sparse matrices and
expectation values are inner products of state vectors.  It is used only on
tiny systems (n <= 12) to pin the tensor formulas of the other modules.
"""
import numpy as np
import scipy.sparse as sp


def _popcount(x):
    x = np.asarray(x, dtype=np.int64)
    c = np.zeros_like(x)
    while np.any(x):
        c += x & 1
        x = x >> 1
    return c


class Fock:
    """Annihilation operators a_P (P = 0..n-1) on the 2^n Fock space."""

    def __init__(self, n):
        self.n = n
        self.dim = 1 << n
        idx = np.arange(self.dim, dtype=np.int64)
        self.ann = []
        for P in range(n):
            src = idx[((idx >> P) & 1) == 1]
            dst = src ^ (1 << P)
            sign = np.where(_popcount(src & ((1 << P) - 1)) % 2 == 0, 1.0, -1.0)
            self.ann.append(sp.csr_matrix((sign, (dst, src)), shape=(self.dim, self.dim)))
        self.cre = [a.T.tocsr() for a in self.ann]
        self.nel = _popcount(idx)

    def sector(self, N, n_alpha=None):
        """Basis indices with N electrons (and n_alpha alpha electrons if given)."""
        idx = np.arange(self.dim, dtype=np.int64)
        keep = self.nel == N
        if n_alpha is not None:
            r = self.n // 2
            keep &= _popcount(idx & ((1 << r) - 1)) == n_alpha
        return idx[keep]

    # ---- operators -------------------------------------------------------
    def one_body(self, h):
        """sum_PR h[P,R] a+_P a_R."""
        out = sp.csr_matrix((self.dim, self.dim))
        for P in range(self.n):
            for R in range(self.n):
                if h[P, R] != 0.0:
                    out = out + h[P, R] * (self.cre[P] @ self.ann[R])
        return out

    def two_body(self, X):
        """sum_PQRS X[P,Q,R,S] a+_P a+_Q a_S a_R  (no prefactor)."""
        n = self.n
        pair = {}
        for R in range(n):
            for S in range(n):
                if R != S:
                    pair[(R, S)] = self.ann[S] @ self.ann[R]  # a_S a_R
        out = sp.csr_matrix((self.dim, self.dim))
        for (P, Q), bpq in pair.items():
            acc = sp.csr_matrix((self.dim, self.dim))
            for (R, S), brs in pair.items():
                c = X[P, Q, R, S]
                if c != 0.0:
                    acc = acc + c * brs
            if acc.nnz:
                out = out + bpq.T @ acc  # (a_Q a_P)^+ = a+_P a+_Q
        return out.tocsr()

    def hamiltonian(self, h_so, g_so):
        """Eq. (1) with antisymmetry-free physicists' integrals:
        H = sum h a+a + 1/2 sum <PQ|RS> a+_P a+_Q a_S a_R."""
        return (self.one_body(h_so) + 0.5 * self.two_body(g_so)).tocsr()

    # ---- state-derived quantities ----------------------------------------
    def pair_vectors(self, psi):
        """Phi[P,Q] = a_Q a_P psi, shape (n, n, dim)."""
        n = self.n
        a1 = np.stack([self.ann[P] @ psi for P in range(n)])  # a_P psi
        return np.stack([np.stack([self.ann[Q] @ a1[P] for Q in range(n)]) for P in range(n)])

    def triple_vectors(self, psi):
        """Phi[P,Q,T] = a_T a_Q a_P psi, shape (n, n, n, dim)."""
        n = self.n
        a2 = self.pair_vectors(psi)
        return np.stack([np.stack([np.stack([self.ann[T] @ a2[P, Q] for T in range(n)])
                                   for Q in range(n)]) for P in range(n)])

    def rdm1(self, psi):
        """Gamma1[P,R] = <a+_P a_R>  (Eq. (6) normalisation of 1D, trace N)."""
        a1 = np.stack([self.ann[P] @ psi for P in range(self.n)])
        return a1 @ a1.T

    def rdm2(self, psi):
        """Gamma2[P,Q,R,S] = <a+_P a+_Q a_S a_R> = 2 * 2D of Eq. (6)."""
        n = self.n
        ph = self.pair_vectors(psi).reshape(n * n, -1)
        return (ph @ ph.T).reshape(n, n, n, n)

    def rdm3(self, psi):
        """Gamma3[P,Q,T,R,S,U] = <a+_P a+_Q a+_T a_U a_S a_R> = 6 * 3D of Eq. (6)."""
        n = self.n
        ph = self.triple_vectors(psi).reshape(n ** 3, -1)
        return (ph @ ph.T).reshape(n, n, n, n, n, n)

    def commutator_expectation(self, psi, b_psi, bdag_psi):
        """C[i,j,k,l] = <psi| [a+_i a+_j a_l a_k, B] |psi> for real states.

        <O B> = <a_j a_i psi | a_l a_k B psi> and
        <B O> = <a_j a_i B^+ psi | a_l a_k psi>.
        """
        n = self.n
        p0 = self.pair_vectors(psi).reshape(n * n, -1)
        pb = self.pair_vectors(b_psi).reshape(n * n, -1)
        pd = self.pair_vectors(bdag_psi).reshape(n * n, -1)
        return (p0 @ pb.T - pd @ p0.T).reshape(n, n, n, n)

    def apply_two_body(self, X, psi):
        """(sum_PQRS X[P,Q,R,S] a+_P a+_Q a_S a_R) psi without forming the operator."""
        n = self.n
        ph = self.pair_vectors(psi).reshape(n * n, -1)  # a_S a_R psi at [R,S]
        xi = (X.reshape(n * n, n * n) @ ph).reshape(n, n, -1)
        out = np.zeros(self.dim)
        for P in range(n):
            for Q in range(n):
                if np.any(xi[P, Q]):
                    out += self.cre[P] @ (self.cre[Q] @ xi[P, Q])
        return out


def spin_orbital_integrals(h, V):
    """Spin-orbital h_so[P,R] and physicists' <PQ|RS> from spatial h and
    chemists' V[p,q,r,s] = (pq|rs):  <PQ|RS> = (pr|qs) d(sP,sR) d(sQ,sS)."""
    r = h.shape[0]
    n = 2 * r
    h_so = np.zeros((n, n))
    h_so[:r, :r] = h
    h_so[r:, r:] = h
    g = np.zeros((n, n, n, n))
    phys = V.transpose(0, 2, 1, 3)  # <pq|rs> = (pr|qs)
    for sP in (0, 1):
        for sQ in (0, 1):
            g[sP * r:(sP + 1) * r, sQ * r:(sQ + 1) * r, sP * r:(sP + 1) * r, sQ * r:(sQ + 1) * r] = phys
    return h_so, g


def fci(fock, H, N, n_alpha=None, nroots=None):
    """Exact diagonalisation of H in the N-electron (optionally fixed-S_z) sector.
    Returns (energies, full-space eigenvectors as columns)."""
    sec = fock.sector(N, n_alpha)
    Hs = H[sec][:, sec].toarray()
    w, v = np.linalg.eigh(Hs)
    if nroots is not None:
        w, v = w[:nroots], v[:, :nroots]
    full = np.zeros((fock.dim, v.shape[1]))
    full[sec] = v
    return w, full


def s_squared(fock, psi):
    """<S^2> of a real state (alpha orbitals 0..r-1, beta r..2r-1)."""
    r = fock.n // 2
    sp_ = sum(fock.cre[p] @ fock.ann[p + r] for p in range(r))  # S+ = sum a+_pa a_pb
    na = sum(fock.cre[p] @ fock.ann[p] for p in range(r))
    nb = sum(fock.cre[p + r] @ fock.ann[p + r] for p in range(r))
    sz = 0.5 * (na - nb)
    s2 = sp_.T @ sp_ + sz @ sz + sz
    return float(psi @ (s2 @ psi))


def lowest_singlet(fock, H, N, tol=1e-8):
    """Lowest eigenstate with <S^2> < tol in the N_alpha = N_beta sector; ties by lowest index."""
    w, v = fci(fock, H, N, n_alpha=N // 2)
    for k in range(len(w)):
        if s_squared(fock, v[:, k]) < tol:
            return w[k], v[:, k]
    raise RuntimeError("no singlet found")


def determinant(fock, occ):
    """Basis vector of the determinant with the given occupied spin orbitals."""
    psi = np.zeros(fock.dim)
    psi[sum(1 << P for P in occ)] = 1.0
    return psi


def rotated_determinant(fock, C):
    """prod_k (sum_P C[P,k] a+_P) |vac>, k = 0..N-1 applied left to right, so the
    result is b+_{N-1} ... b+_0 |vac>.  C has orthonormal columns."""
    psi = np.zeros(fock.dim)
    psi[0] = 1.0
    for k in range(C.shape[1]):
        op = sum(C[P, k] * fock.cre[P] for P in range(fock.n) if C[P, k] != 0.0)
        psi = op @ psi
    return psi


def singlet_blocks_from_state(fock, psi):
    """(gamma, 2D_aa, 2D_ab) of a state (Eq. (6) normalisations; alpha orbitals first)."""
    r = fock.n // 2
    g1 = fock.rdm1(psi)
    g2 = fock.rdm2(psi)
    a, b = slice(0, r), slice(r, 2 * r)
    return g1[a, a].copy(), 0.5 * g2[a, a, a, a], 0.5 * g2[a, b, a, b]


def spin_blocks_from_state(fock, psi):
    """(gamma_a, gamma_b, 2D_aa, 2D_bb, 2D_ab) of a state of any S_z."""
    r = fock.n // 2
    g1 = fock.rdm1(psi)
    g2 = fock.rdm2(psi)
    a, b = slice(0, r), slice(r, 2 * r)
    return (g1[a, a].copy(), g1[b, b].copy(), 0.5 * g2[a, a, a, a], 0.5 * g2[b, b, b, b],
            0.5 * g2[a, b, a, b])


def fci_singlet_problem(h, V, N):
    """Lowest singlet of the Hamiltonian of Eq. (1) built from spatial (h, V):
    returns dict(energy, psi, fock, gamma, d2aa, d2ab)."""
    r = h.shape[0]
    fock = Fock(2 * r)
    hso, gso = spin_orbital_integrals(h, V)
    H = fock.hamiltonian(hso, gso)
    e0, psi = lowest_singlet(fock, H, N)
    g, d2aa, d2ab = singlet_blocks_from_state(fock, psi)
    return dict(energy=e0, psi=psi, fock=fock, H=H, gamma=g, d2aa=d2aa, d2ab=d2ab)
