"""Pins of the oracle adjoints (oracle/adjoint.py), CPU only.

The adjoint is reverse-mode differentiation of the oracle's torch forward,
projected onto the symmetric input space.  It is checked here against things
that do not share its derivation:

* central finite differences (step 1e-5) of the numpy forward (oracle.step);
* R is linear in K, so <grad_(h,V), (dh, dV)> = L evaluated at (dh, dV);
* E is bilinear in K and 2D, which gives two exact identities;
* the projections are idempotent and self-adjoint, and they fix the
  generator's structured directions.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint as adj
from oracle import fermion as fm
from oracle import rdm
from oracle import step as ost
from synth import generators as gen

KEYS = ("h", "V", "gamma", "d2aa", "d2ab")


def tiny_fci(seed=0):
    rng = np.random.default_rng(seed)
    h, V = gen.hamiltonian(rng, 4, 6)
    p = fm.fci_singlet_problem(h, V, 4)
    return dict(r=4, N=4, h=h, V=V, gamma=p["gamma"], d2aa=p["d2aa"], d2ab=p["d2ab"])


PROBLEMS = {
    "tiny_fci": lambda: tiny_fci(0),
    "r5": lambda: gen.problem(5, 6, 10, seed=4),
}


def loss(p, Rb, sigma=None, **over):
    q = {k: over.get(k, p[k]) for k in KEYS}
    raa, rab, _ = ost.residual(q["h"], q["V"], p["N"], q["gamma"], q["d2aa"], q["d2ab"], sigma=sigma)
    return float(np.sum(Rb[0] * raa) + np.sum(Rb[1] * rab))


def test_torch_forward_matches_numpy():
    p = PROBLEMS["r5"]()
    K = adj.reduced_hamiltonian_t(torch.tensor(p["h"]), torch.tensor(p["V"]), p["N"]).numpy()
    assert np.array_equal(K, rdm.reduced_hamiltonian(p["h"], p["V"], p["N"]))
    d1, d2 = adj.blocks_to_spin_orbital_t(*[torch.tensor(p[k]) for k in ("gamma", "d2aa", "d2ab")])
    n1, n2 = rdm.blocks_to_spin_orbital(p["gamma"], p["d2aa"], p["d2ab"])
    assert np.array_equal(d1.numpy(), n1) and np.array_equal(d2.numpy(), n2)
    Raa, Rab = adj.residual_blocks_t(*[torch.tensor(p[k]) for k in ("h", "V")], p["N"],
                                     *[torch.tensor(p[k]) for k in ("gamma", "d2aa", "d2ab")])
    raa, rab, _ = ost.residual(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"])
    assert np.abs(Raa.numpy() - raa).max() <= 1e-13 * np.abs(raa).max()
    assert np.abs(Rab.numpy() - rab).max() <= 1e-13 * np.abs(rab).max()
    E = adj.energy_t(torch.tensor(p["h"]), torch.tensor(p["V"]), p["N"], torch.tensor(p["d2aa"]),
                     torch.tensor(p["d2ab"])).item()
    assert abs(E - ost.energy(p["h"], p["V"], p["N"], p["d2aa"], p["d2ab"])) <= 1e-13 * abs(E)


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("key", KEYS)
def test_residual_vjp_finite_difference(name, key):
    p = PROBLEMS[name]()
    r = p["r"]
    rng = np.random.default_rng(11)
    Rb = gen.cotangent(rng, r)
    d = gen.symmetric_direction(rng, r)[key]
    g = adj.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], *Rb)
    t = 1e-5
    fd = (loss(p, Rb, **{key: p[key] + t * d}) - loss(p, Rb, **{key: p[key] - t * d})) / (2 * t)
    an = float(np.sum(g[key] * d))
    scale = max(abs(an), np.linalg.norm(g[key]))
    assert abs(fd - an) <= 1e-7 * scale, (fd, an)


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_residual_vjp_exact_linearity_in_hamiltonian(name):
    p = PROBLEMS[name]()
    r = p["r"]
    rng = np.random.default_rng(12)
    Rb = gen.cotangent(rng, r)
    d = gen.symmetric_direction(rng, r)
    g = adj.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], *Rb)
    lin = loss(p, Rb, h=d["h"], V=d["V"])
    an = float(np.sum(g["h"] * d["h"]) + np.sum(g["V"] * d["V"]))
    assert abs(lin - an) <= 1e-12 * max(1.0, abs(lin))


def test_energy_vjp_bilinear():
    p = PROBLEMS["r5"]()
    r, N = p["r"], p["N"]
    rng = np.random.default_rng(13)
    d = gen.symmetric_direction(rng, r)
    g = adj.energy_vjp(p["h"], p["V"], N, p["d2aa"], p["d2ab"], Ebar=0.7)
    e_rdm = ost.energy(p["h"], p["V"], N, d["d2aa"], d["d2ab"])
    an = float(np.sum(g["d2aa"] * d["d2aa"]) + np.sum(g["d2ab"] * d["d2ab"]))
    assert abs(0.7 * e_rdm - an) <= 1e-12 * max(1.0, abs(an))
    e_ham = ost.energy(d["h"], d["V"], N, p["d2aa"], p["d2ab"])
    an = float(np.sum(g["h"] * d["h"]) + np.sum(g["V"] * d["V"]))
    assert abs(0.7 * e_ham - an) <= 1e-12 * max(1.0, abs(an))


def test_projections():
    rng = np.random.default_rng(14)
    r = 4
    d = gen.symmetric_direction(rng, r)
    pairs = (("h", adj.proj_sym2), ("V", adj.proj_V), ("gamma", adj.proj_sym2),
             ("d2aa", adj.proj_aa), ("d2ab", adj.proj_ab))
    for k, P in pairs:
        shape = d[k].shape
        x = torch.tensor(rng.normal(size=shape))
        y = torch.tensor(rng.normal(size=shape))
        px = P(x)
        assert torch.allclose(P(px), px, rtol=0, atol=1e-14)                        # idempotent
        assert abs(float((px * y).sum() - (x * P(y)).sum())) < 1e-12                # self-adjoint
        dd = torch.tensor(d[k])
        assert torch.allclose(P(dd), dd, rtol=0, atol=1e-14)                        # fixes the subspace
        assert float(torch.linalg.norm(px)) < float(torch.linalg.norm(x))          # a proper projection


def test_planted_unprojected_gradient_breaks_symmetry():
    """Without the projection the raw autograd gradient of d2ab is not in the
    symmetric subspace (so a GPU result that is symmetric could not match it)."""
    p = PROBLEMS["r5"]()
    rng = np.random.default_rng(15)
    Rb = gen.cotangent(rng, p["r"])
    x = [torch.tensor(p[k], requires_grad=True) for k in KEYS]
    Raa, Rab = adj.residual_blocks_t(x[0], x[1], p["N"], x[2], x[3], x[4])
    L = (torch.tensor(Rb[0]) * Raa).sum() + (torch.tensor(Rb[1]) * Rab).sum()
    raw = torch.autograd.grad(L, x)[4]
    assert float(torch.linalg.norm(raw - adj.proj_ab(raw))) > 1e-3 * float(torch.linalg.norm(raw))


# occupations of the NY pins: not a prefix, so that the sigma weights matter
NY_SIGMA = {"tiny_fci": [1, -1, 1, -1], "r5": [1, 1, -1, 1, -1]}


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("key", KEYS)
def test_residual_vjp_ny_finite_difference(name, key):
    """The NY adjoint (autograd through the factorised NY share) against
    central finite differences of the numpy NY forward."""
    p = PROBLEMS[name]()
    r = p["r"]
    sig = NY_SIGMA[name]
    rng = np.random.default_rng(13)
    Rb = gen.cotangent(rng, r)
    d = gen.symmetric_direction(rng, r)[key]
    g = adj.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], *Rb, sigma=sig)
    t = 1e-5
    fd = (loss(p, Rb, sig, **{key: p[key] + t * d}) - loss(p, Rb, sig, **{key: p[key] - t * d})) / (2 * t)
    an = float(np.sum(g[key] * d))
    scale = max(abs(an), np.linalg.norm(g[key]))
    assert abs(fd - an) <= 1e-7 * scale, (fd, an)
    # the NY share moves this gradient: the Valdemoro one differs
    gv = adj.residual_vjp(p["h"], p["V"], p["N"], p["gamma"], p["d2aa"], p["d2ab"], *Rb)
    assert np.linalg.norm(gv[key] - g[key]) > 1e-6 * np.linalg.norm(g[key])
