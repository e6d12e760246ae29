"""The Euler iteration of Eq. (9) with the method section's stopping rules,
and two step-size controls (oracle; test infrastructure only).

The method section propagates 2D_{n+1} = 2D_n + eps U_n with a fixed eps
(1e-3 by default) and ends the iteration when the energy or the residual norm
increases, or when the energy changes by less than 1e-6 Eh.

Readings (the paper is silent on these points):

* "Increase" compares the trial state with the current one: a trial 2D' is
  acceptable iff E(2D') <= E_n and ||R(2D')||^2 <= ||R_n||^2 (the residual
  norm over spin orbitals, before the active mask).  On an increase the
  iteration ends and the state before the step is returned: the rise is not
  kept.
* The energy test is made after an accepted step: |E_{n+1} - E_n| < de_tol
  ends the iteration with the new state.
* BACKTRACK: instead of ending at a rise, eps is halved (the same U_n, a new
  trial from 2D_n) at most ``max_halvings`` times; the step size of an
  accepted step carries over to the next step.
* QUADRATIC (Newton-like control from the adjoint): along the step,
  f(eps) = ||R(2D_n + eps U_n)||^2 has the slope
      f'(0) = <dbar_aa, U_aa> + <dbar_ab, U_ab> + <gbar, d gamma/d eps>,
  where (gbar, dbar_aa, dbar_ab) is the vector-Jacobian product of the
  residual map for the cotangent (4 R_aa, 8 R_ab) (the gradient of
  2||R_aa||^2 + 4||R_ab||^2) and d gamma/d eps = 2/(N-1) Tr_2 U (the 1-RDM is
  contracted from the 2-RDM after each step).  After the first trial at eps,
  f is modelled as f(0) + f'(0) x + c x^2 through f(eps); when f'(0) < 0 the
  model's minimiser (or 4 eps when c <= 0), clamped to [eps/4, min(4 eps,
  eps_max)], is tried as well unless it lies within 5% of eps.  Of the
  acceptable trials the one with the smaller f is kept (the first on a tie);
  if neither is acceptable, plain halving continues from the smaller of the
  two step sizes.
* Trace restoration and the 1-RDM follow ``step.step``: each block is
  rescaled to its trace before the step; gamma' = 2/(N-1) Tr_2 2D'.

Every quantity is evaluated with the oracle's own residual, energy and
adjoint; the GPU driver shares none of this code.
"""
import numpy as np

from . import adjoint, rdm
from .residual import residual_map
from .step import active_mask, restore_block_traces, restore_traces

FIXED, BACKTRACK, QUADRATIC = 0, 1, 2
STOP_MAX_ITER, STOP_CONVERGED, STOP_ENERGY_ROSE, STOP_NORM_ROSE = 0, 1, 2, 3


def _residual(K, gamma, d2aa, d2ab, sigma_so=None):
    d1, d2 = rdm.blocks_to_spin_orbital(gamma, d2aa, d2ab)
    R = residual_map(K, d1, d2, hermitian=True, sigma_so=sigma_so).numpy()
    return R, float(np.sum(R ** 2)), d1, d2


def _trial(K, N, d2aa, d2ab, uaa, uab, eps):
    """2D' = (2D + eps U) rescaled per block to the trace of 2D; gamma'; E'."""
    r = d2aa.shape[0]
    a, b, _ = restore_traces(d2aa + eps * uaa, d2ab + eps * uab, rdm.block_traces(d2aa, d2ab))
    _, d2 = rdm.blocks_to_spin_orbital(np.eye(r), a, b)
    gamma = rdm.contract_to_1rdm(d2, N)[:r, :r]
    return a, b, gamma, float(np.sum(K * d2))


def norm_slope(h, V, N, gamma, d2aa, d2ab, Raa, Rab, uaa, uab, sigma=None):
    """f'(0) for f(eps) = ||R(2D + eps U)||^2 over spin orbitals, from the
    residual's vector-Jacobian product (cotangent 4 R_aa, 8 R_ab), with the
    3-RDM ``sigma`` selects (None: Valdemoro, else NY)."""
    r = h.shape[0]
    g = adjoint.residual_vjp(h, V, N, gamma, d2aa, d2ab, 4.0 * Raa, 8.0 * Rab, sigma=sigma)
    _, u = rdm.blocks_to_spin_orbital(np.zeros((r, r)), uaa, uab)
    dgamma = rdm.contract_to_1rdm(u, N)[:r, :r]
    return float(np.sum(g["d2aa"] * uaa) + np.sum(g["d2ab"] * uab) + np.sum(g["gamma"] * dgamma))


def norm_slope_spin(h, V, Na, Nb, ga, gb, d2aa, d2bb, d2ab, uaa, ubb, uab, sigma_so=None):
    """f'(0) for f(s) = ||R(2D + s U, 1D + s dD)||^2 over spin orbitals of a
    state of any S_z, dD the 1-RDMs contracted from U (the contraction is
    linear): reverse-mode differentiation (torch.autograd) of the torch
    residual map with respect to s, along the straight line in the RDMs."""
    import torch
    r = h.shape[0]
    N = Na + Nb
    K = torch.from_numpy(rdm.reduced_hamiltonian(np.asarray(h, float), np.asarray(V, float), N))
    d1, d2 = rdm.spin_blocks_to_spin_orbital(ga, gb, d2aa, d2bb, d2ab)
    z = np.zeros((r, r))
    _, u2 = rdm.spin_blocks_to_spin_orbital(z, z, uaa, ubb, uab)
    u1 = rdm.contract_to_1rdm(u2, N)
    a, b = rdm.spin_blocks(r)
    u1[a, b] = 0.0   # the 1-RDM blocks are spin-diagonal
    u1[b, a] = 0.0
    sv = torch.zeros((), dtype=torch.float64, requires_grad=True)
    D1 = torch.from_numpy(d1) + sv * torch.from_numpy(u1)
    D2 = torch.from_numpy(d2) + sv * torch.from_numpy(u2)
    R = residual_map(K, D1, D2, hermitian=True, sigma_so=sigma_so)
    (g,) = torch.autograd.grad((R * R).sum(), sv)
    return float(g)


def quadratic_trial_step(f0, g0, eps, f_eps, eps_max):
    """Second step size of QUADRATIC, or None: the minimiser of the parabola
    through f(0) = f0 with slope g0 and f(eps) = f_eps, clamped to
    [eps/4, min(4 eps, eps_max)]; 4 eps (clamped) when the curvature is not
    positive.  None when g0 >= 0 or the result is within 5% of eps."""
    if not g0 < 0.0:
        return None
    c = (f_eps - f0 - g0 * eps) / (eps * eps)
    hi = min(4.0 * eps, eps_max)
    x = -g0 / (2.0 * c) if c > 0.0 else hi
    x = min(max(x, 0.25 * eps), hi)
    if abs(x - eps) <= 0.05 * abs(eps):
        return None
    return x


def euler(h, V, N, gamma, d2aa, d2ab, eps=1e-3, de_tol=1e-6, max_iter=100, control=FIXED,
          max_halvings=8, eps_max=0.0, active=None, sigma=None):
    """Run the iteration; returns a dict with the final gamma, d2aa, d2ab, the
    energies and norms of the input and returned states, the stop reason, the
    accepted-step count and the list of trials (eps, E, ||R||^2, step index,
    accepted).  ``sigma`` (per spatial orbital, +1 / -1) selects the NY
    3-RDM of Eq. (8) for every map and for the quadratic control's slope."""
    sso = None if sigma is None else rdm.sigma_spin_orbital(sigma)
    h = np.asarray(h, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    r = h.shape[0]
    K = rdm.reduced_hamiltonian(h, V, N)
    mask = active_mask(active, r)
    eps_max = eps_max if eps_max > 0.0 else 16.0 * abs(eps)
    gamma = np.array(gamma, dtype=np.float64)
    d2aa = np.array(d2aa, dtype=np.float64)
    d2ab = np.array(d2ab, dtype=np.float64)
    _, d2 = rdm.blocks_to_spin_orbital(gamma, d2aa, d2ab)
    E = float(np.sum(K * d2))
    R, f, d1, d2 = _residual(K, gamma, d2aa, d2ab, sso)
    out = dict(energy0=E, norm2_0=f, trials=[], iterations=0, stop=STOP_MAX_ITER, eps_last=0.0)
    e = eps

    def ok(Et, ft):
        return Et <= E and ft <= f

    def why(Et):
        return STOP_ENERGY_ROSE if Et > E else STOP_NORM_ROSE

    for n in range(max_iter):
        Rm = R if mask is None else R * mask
        U = residual_map(Rm, d1, d2, hermitian=False, sigma_so=sso).numpy()
        uaa, uab = rdm.spin_orbital_to_blocks(U)
        raa, rab = rdm.spin_orbital_to_blocks(R)

        def run(x):
            a, b, g1, Et = _trial(K, N, d2aa, d2ab, uaa, uab, x)
            Rt, ft, _, _ = _residual(K, g1, a, b, sso)
            return dict(eps=x, d2aa=a, d2ab=b, gamma=g1, E=Et, f=ft, R=Rt)

        trials = []

        def attempt(x):
            q = run(x)
            trials.append(q)
            return q

        t = attempt(e)
        chosen = t if ok(t["E"], t["f"]) else None
        cand = e
        if control == QUADRATIC:
            g0 = norm_slope(h, V, N, gamma, d2aa, d2ab, raa, rab, uaa, uab, sigma=sigma)
            x = quadratic_trial_step(f, g0, e, t["f"], eps_max)
            if x is not None:
                t2 = attempt(x)
                good = [q for q in (t, t2) if ok(q["E"], q["f"])]
                chosen = min(good, key=lambda q: q["f"]) if good else None  # first on a tie
                cand = min(e, x)
        halvings = 0
        while chosen is None and control != FIXED and halvings < max_halvings:
            cand = 0.5 * cand
            halvings += 1
            t = attempt(cand)
            if ok(t["E"], t["f"]):
                chosen = t
        stop = None if chosen is not None else why(trials[-1]["E"])
        for q in trials:
            out["trials"].append((q["eps"], q["E"], q["f"], n, q is chosen))
        if chosen is None:
            out["stop"] = stop
            break
        dE = chosen["E"] - E
        d2aa, d2ab, gamma = chosen["d2aa"], chosen["d2ab"], chosen["gamma"]
        E, f, R = chosen["E"], chosen["f"], chosen["R"]
        d1, d2 = rdm.blocks_to_spin_orbital(gamma, d2aa, d2ab)
        e = chosen["eps"]
        out["iterations"] = n + 1
        out["eps_last"] = e
        if abs(dE) < de_tol:
            out["stop"] = STOP_CONVERGED
            break
    out.update(gamma=gamma, d2aa=d2aa, d2ab=d2ab, energy=E, norm2=f)
    return out


def euler_spin(h, V, Na, Nb, ga, gb, d2aa, d2bb, d2ab, eps=1e-3, de_tol=1e-6, max_iter=100, control=FIXED,
               max_halvings=8, active=None, sigma_so=None, eps_max=0.0):
    """The iteration of ``euler`` for a state of any S_z, on its three 2-RDM
    spin blocks (alpha-alpha, beta-beta, alpha-beta) and one 1-RDM per spin:
    the same stopping rules and the three step controls (QUADRATIC with its
    slope from ``norm_slope_spin``); each block is rescaled to its own trace
    before the step (a block of trace zero is set to zero) and both 1-RDMs are
    contracted from the new 2-RDM.  ``sigma_so``
    (2r reference occupations, alpha orbitals first) selects the NY 3-RDM of
    Eq. (8) in both maps; None is Valdemoro.  Returns a dict with ga, gb,
    d2aa, d2bb, d2ab of the returned state and the fields of ``euler``."""
    if control not in (FIXED, BACKTRACK, QUADRATIC):
        raise ValueError("unknown step control")
    eps_max = eps_max if eps_max > 0.0 else 16.0 * abs(eps)
    h = np.asarray(h, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    r = h.shape[0]
    N = Na + Nb
    K = rdm.reduced_hamiltonian(h, V, N)
    mask = active_mask(active, r)
    blocks = tuple(np.array(x, dtype=np.float64) for x in (d2aa, d2bb, d2ab))
    ga = np.array(ga, dtype=np.float64)
    gb = np.array(gb, dtype=np.float64)
    z = np.zeros((r, r))

    def residual(ga, gb, blocks):
        d1, d2 = rdm.spin_blocks_to_spin_orbital(ga, gb, *blocks)
        R = residual_map(K, d1, d2, hermitian=True, sigma_so=sigma_so).numpy()
        return R, float(np.sum(R ** 2)), d1, d2, float(np.sum(K * d2))

    R, f, d1, d2, E = residual(ga, gb, blocks)
    out = dict(energy0=E, norm2_0=f, trials=[], iterations=0, stop=STOP_MAX_ITER, eps_last=0.0)
    e = eps
    for n in range(max_iter):
        Rm = R if mask is None else R * mask
        U = residual_map(Rm, d1, d2, hermitian=False, sigma_so=sigma_so).numpy()
        ublocks = rdm.spin_orbital_to_spin_blocks(U)
        traces = tuple(float(np.einsum('pqpq->', b)) for b in blocks)

        def run(x):
            new, _ = restore_block_traces(tuple(b + x * u for b, u in zip(blocks, ublocks)), traces)
            _, d2n = rdm.spin_blocks_to_spin_orbital(z, z, *new)
            g1 = rdm.contract_to_1rdm(d2n, N)
            g1a, g1b = g1[:r, :r].copy(), g1[r:, r:].copy()
            Rt, ft, d1t, d2t, Et = residual(g1a, g1b, new)
            return dict(eps=x, blocks=new, ga=g1a, gb=g1b, E=Et, f=ft, R=Rt, d1=d1t, d2=d2t)

        trials = [run(e)]
        chosen = trials[0] if (trials[0]["E"] <= E and trials[0]["f"] <= f) else None
        cand = e
        if control == QUADRATIC:
            g0 = norm_slope_spin(h, V, Na, Nb, ga, gb, *blocks, *ublocks, sigma_so=sigma_so)
            x = quadratic_trial_step(f, g0, e, trials[0]["f"], eps_max)
            if x is not None:
                trials.append(run(x))
                good = [q for q in trials if q["E"] <= E and q["f"] <= f]
                chosen = min(good, key=lambda q: q["f"]) if good else None  # first on a tie
                cand = min(e, x)
        halvings = 0
        while chosen is None and control != FIXED and halvings < max_halvings:
            cand = 0.5 * cand
            halvings += 1
            t = run(cand)
            trials.append(t)
            if t["E"] <= E and t["f"] <= f:
                chosen = t
        for q in trials:
            out["trials"].append((q["eps"], q["E"], q["f"], n, q is chosen))
        if chosen is None:
            out["stop"] = STOP_ENERGY_ROSE if trials[-1]["E"] > E else STOP_NORM_ROSE
            break
        dE = chosen["E"] - E
        blocks, ga, gb = chosen["blocks"], chosen["ga"], chosen["gb"]
        E, f, R, d1, d2 = chosen["E"], chosen["f"], chosen["R"], chosen["d1"], chosen["d2"]
        e = chosen["eps"]
        out["iterations"] = n + 1
        out["eps_last"] = e
        if abs(dE) < de_tol:
            out["stop"] = STOP_CONVERGED
            break
    out.update(ga=ga, gb=gb, d2aa=blocks[0], d2bb=blocks[1], d2ab=blocks[2], energy=E, norm2=f)
    return out
