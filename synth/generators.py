"""Seeded synthetic workloads (no method arithmetic here).

Recipe (one ``numpy.random.default_rng(seed)`` per problem, fixed draw order:
h diagonal, h upper triangle, Cholesky vectors, orbital rotation, cumulant):

* h: diagonal U[-2, 2]; off-diagonal N(0, 0.1^2), mirrored.
* V[p,q,r,s] = sum_k L^k_pq L^k_rs with L^k symmetric, upper triangle
  (with diagonal) N(0, 0.3^2): 8-fold symmetric and positive semidefinite.
* Spin-summed natural occupations n_i = 0.02 + 1.96 / (1 + exp((i - mu)/0.5)),
  mu bisected so that sum n = N; excited-state variants pin one pair of
  frontier orbitals at occupation 1.0 and re-bisect the rest.
* gamma = U diag(n/2) U^T, U Haar-random orthogonal (QR of a Gaussian).
* 2D_aa = 1/2 (g_pr g_qs - g_ps g_qr) + c Delta_aa,  2D_ab = 1/2 g_pr g_qs + c Delta_ab,
  c = 1e-2, Delta_ab a Gaussian tensor projected onto Hermitian + pair-exchange
  symmetry, Delta_aa = Delta_ab - Delta_ab(r<->s) (singlet-consistent), then one
  global scale so the spin-orbital trace 2 Tr 2D_aa + 2 Tr 2D_ab = N(N-1)/2.

States of any S_z (``spin_problem``, N_alpha != N_beta): per spin sigma the
occupations n_i = 0.01 + 0.98 / (1 + exp((i - mu)/0.5)) bisected to sum N_sigma
(all zero for N_sigma = 0, all one for N_sigma = r); gamma_sigma = U_sigma
diag(n_sigma) U_sigma^T with its own Haar rotation (drawn alpha then beta);
2D_ss = 1/2 (g_pr g_qs - g_ps g_qr) + c Delta_ss (Delta antisymmetric in each
pair and Hermitian, drawn aa then bb), 2D_ab = 1/2 ga_pr gb_qs + c Delta_ab
(Delta Hermitian only, drawn last); each block then scaled to its App. A trace
N_a(N_a-1)/2, N_b(N_b-1)/2, N_a N_b / 2.

These stand in for the molecular 1-/2-RDMs and integrals of the paper's
CASSCF-referenced runs (sizes r = 12 ... 116 spatial orbitals), which are not
available here.
"""
import numpy as np

# Named workloads: (r, N, n_chol).  "tiny" takes its RDMs from exact FCI.
CONFIGS = {
    "tiny": dict(r=4, N=4, n_chol=6),
    "r30": dict(r=30, N=20, n_chol=60),
    "r50": dict(r=50, N=30, n_chol=60),
    "vjp30": dict(r=30, N=20, n_chol=60),
}
# Named workloads of states of any S_z: (r, N_alpha, N_beta, n_chol).
SPIN_CONFIGS = {
    "r50s": dict(r=50, Na=16, Nb=14, n_chol=60),
}
BATCH_SIZES = (20, 28, 36, 44)


def hamiltonian(rng, r, n_chol):
    h = np.zeros((r, r))
    h[np.diag_indices(r)] = rng.uniform(-2.0, 2.0, size=r)
    iu = np.triu_indices(r, 1)
    off = rng.normal(0.0, 0.1, size=iu[0].size)
    h[iu] = off
    h[(iu[1], iu[0])] = off
    iu0 = np.triu_indices(r)
    L = np.zeros((n_chol, r, r))
    for k in range(n_chol):
        v = rng.normal(0.0, 0.3, size=iu0[0].size)
        L[k][iu0] = v
        L[k][(iu0[1], iu0[0])] = v
    Lm = L.reshape(n_chol, r * r)
    V = (Lm.T @ Lm).reshape(r, r, r, r)
    return h, V


def _occ(x, mu):
    return 0.02 + 1.96 / (1.0 + np.exp((x - mu) / 0.5))


def fermi_occupations(r, N, pinned=()):
    """Spin-summed occupations summing to N; indices in ``pinned`` are fixed at 1.0."""
    idx = np.arange(r, dtype=np.float64)
    free = np.ones(r, dtype=bool)
    free[list(pinned)] = False
    target = N - 1.0 * len(pinned)
    lo, hi = -50.0, r + 50.0
    for _ in range(200):
        mu = 0.5 * (lo + hi)
        s = _occ(idx[free], mu).sum()
        if s < target:
            lo = mu
        else:
            hi = mu
    n = np.ones(r)
    n[free] = _occ(idx[free], 0.5 * (lo + hi))
    return n


def haar_orthogonal(rng, r):
    z = rng.normal(size=(r, r))
    q, rr = np.linalg.qr(z)
    return q * np.sign(np.diag(rr))


def rdm_blocks(rng, r, N, occ, cumulant_scale=1e-2):
    U = haar_orthogonal(rng, r)
    g = (U * (occ / 2.0)) @ U.T
    g = 0.5 * (g + g.T)
    d2aa = 0.5 * (np.einsum('pr,qs->pqrs', g, g) - np.einsum('ps,qr->pqrs', g, g))
    d2ab = 0.5 * np.einsum('pr,qs->pqrs', g, g)
    x = rng.normal(size=(r, r, r, r))
    dab = 0.25 * (x + x.transpose(2, 3, 0, 1) + x.transpose(1, 0, 3, 2) + x.transpose(3, 2, 1, 0))
    daa = dab - dab.transpose(0, 1, 3, 2)
    d2aa = d2aa + cumulant_scale * daa
    d2ab = d2ab + cumulant_scale * dab
    tr = 2.0 * np.einsum('pqpq->', d2aa) + 2.0 * np.einsum('pqpq->', d2ab)
    c = (N * (N - 1) / 2.0) / tr
    return g, d2aa * c, d2ab * c


def problem(r, N, n_chol, seed=0, pinned=()):
    """(h, V, gamma, d2aa, d2ab) of one synthetic singlet instance."""
    rng = np.random.default_rng(seed)
    h, V = hamiltonian(rng, r, n_chol)
    occ = fermi_occupations(r, N, pinned)
    g, d2aa, d2ab = rdm_blocks(rng, r, N, occ)
    return dict(r=r, N=N, h=h, V=V, gamma=g, d2aa=d2aa, d2ab=d2ab)


def named(name, seed=0):
    c = CONFIGS[name]
    return problem(c["r"], c["N"], c["n_chol"], seed)


def named_spin(name, seed=0):
    c = SPIN_CONFIGS[name]
    return spin_problem(c["r"], c["Na"], c["Nb"], c["n_chol"], seed)


def batched_problems(seed=0, sizes=BATCH_SIZES):
    """Ground + two excited-state-like instances per size, one (h, V) per size.
    N = 2 round(0.3 r); the excited variants pin HONO/LUNO (then HONO-1/LUNO+1)
    at occupation 1.0."""
    rng = np.random.default_rng(seed)
    out = []
    for r in sizes:
        N = 2 * int(round(0.3 * r))
        h, V = hamiltonian(rng, r, 2 * r)
        homo, lumo = N // 2 - 1, N // 2
        for pinned in ((), (homo, lumo), (homo - 1, lumo + 1)):
            occ = fermi_occupations(r, N, pinned)
            g, d2aa, d2ab = rdm_blocks(rng, r, N, occ)
            out.append(dict(r=r, N=N, h=h, V=V, gamma=g, d2aa=d2aa, d2ab=d2ab))
    return out


def symmetric_direction(rng, r, scale=1.0):
    """A random direction in the structured input space: h and gamma symmetric,
    V with the 8-fold symmetry of (pq|rs), d2aa antisymmetric in each pair and
    Hermitian, d2ab Hermitian and pair-exchange symmetric (each unit Frobenius
    norm times ``scale``).  Used for finite-difference checks of adjoints."""
    def sym2():
        x = rng.normal(size=(r, r))
        return 0.5 * (x + x.T)

    x = rng.normal(size=(r, r, r, r))
    perms = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
             (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]
    V = sum(x.transpose(p) for p in perms) / 8.0
    x = rng.normal(size=(r, r, r, r))
    y = x - x.transpose(1, 0, 2, 3) - x.transpose(0, 1, 3, 2) + x.transpose(1, 0, 3, 2)
    daa = y + y.transpose(2, 3, 0, 1)
    x = rng.normal(size=(r, r, r, r))
    dab = x + x.transpose(2, 3, 0, 1) + x.transpose(1, 0, 3, 2) + x.transpose(3, 2, 1, 0)
    out = dict(h=sym2(), V=V, gamma=sym2(), d2aa=daa, d2ab=dab)
    return {k: scale * v / np.linalg.norm(v) for k, v in out.items()}


def cotangent(rng, r):
    """A seeded Gaussian cotangent (Rbar_aa, Rbar_ab) on the residual blocks."""
    return rng.normal(size=(r, r, r, r)), rng.normal(size=(r, r, r, r))


def _spin_occupations(r, Ns):
    if Ns == 0:
        return np.zeros(r)
    if Ns >= r:
        return np.ones(r)
    idx = np.arange(r, dtype=np.float64)
    occ = lambda mu: 0.01 + 0.98 / (1.0 + np.exp((idx - mu) / 0.5))
    lo, hi = -50.0, r + 50.0
    for _ in range(200):
        mu = 0.5 * (lo + hi)
        if occ(mu).sum() < Ns:
            lo = mu
        else:
            hi = mu
    return occ(0.5 * (lo + hi))


def _scaled(block, target):
    tr = np.einsum('pqpq->', block)
    return block * (target / tr) if target != 0.0 else np.zeros_like(block)


def spin_problem(r, Na, Nb, n_chol, seed=0, cumulant_scale=1e-2):
    """(h, V, gamma_a, gamma_b, d2aa, d2bb, d2ab) of one synthetic state with
    N_a alpha and N_b beta electrons (any S_z)."""
    rng = np.random.default_rng(seed)
    h, V = hamiltonian(rng, r, n_chol)
    g = []
    for Ns in (Na, Nb):
        U = haar_orthogonal(rng, r)
        gs = (U * _spin_occupations(r, Ns)) @ U.T
        g.append(0.5 * (gs + gs.T))
    ga, gb = g
    blocks = []
    for gs in (ga, gb):
        x = rng.normal(size=(r, r, r, r))
        x = x - x.transpose(1, 0, 2, 3)
        x = x - x.transpose(0, 1, 3, 2)
        x = 0.125 * (x + x.transpose(2, 3, 0, 1))
        mf = 0.5 * (np.einsum('pr,qs->pqrs', gs, gs) - np.einsum('ps,qr->pqrs', gs, gs))
        blocks.append(mf + cumulant_scale * x)
    x = rng.normal(size=(r, r, r, r))
    dab = 0.5 * np.einsum('pr,qs->pqrs', ga, gb) + cumulant_scale * 0.5 * (x + x.transpose(2, 3, 0, 1))
    d2aa = _scaled(blocks[0], Na * (Na - 1) / 2.0)
    d2bb = _scaled(blocks[1], Nb * (Nb - 1) / 2.0)
    d2ab = _scaled(dab, Na * Nb / 2.0)
    return dict(r=r, Na=Na, Nb=Nb, N=Na + Nb, h=h, V=V, gamma_a=ga, gamma_b=gb, d2aa=d2aa, d2bb=d2bb,
                d2ab=d2ab)
