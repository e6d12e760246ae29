"""Host-side checks of the Python binding (CPU): shapes and option arrays are
validated before any pointer reaches the library, and the checkpoint tag
covers every option that changes the Euler iteration."""
import numpy as np
import pytest
import torch

import paper_2604_02550_amd as acse


class _NoLibrary:
    """Stands in for the loaded library: any call is a test failure."""

    def __getattr__(self, name):
        raise AssertionError(f"the library was called ({name}) although the arguments are invalid")


@pytest.fixture
def no_lib(monkeypatch):
    monkeypatch.setattr(acse, "_lib", _NoLibrary())


@pytest.fixture
def ctx(no_lib):
    # a context object that never reached acse_create: only its device is set
    c = object.__new__(acse.Context)
    c.device = torch.device("cuda", 0)
    c._h = None
    c.r_max = 8
    return c


def _arrays(r):
    rng = np.random.default_rng(0)
    return dict(h=rng.standard_normal((r, r)), V=rng.standard_normal((r,) * 4),
                d1=rng.standard_normal((r, r)), d2aa=rng.standard_normal((r,) * 4),
                d2ab=rng.standard_normal((r,) * 4))


@pytest.mark.parametrize("key,bad", [("h", (4, 5)), ("d1", (5, 5)), ("V", (4, 4, 4, 5)),
                                     ("d2aa", (5, 5, 5, 5)), ("d2ab", (4, 4, 4))])
def test_problem_shapes_rejected_before_the_library(ctx, key, bad):
    a = _arrays(4)
    a[key] = np.zeros(bad)
    with pytest.raises(ValueError, match=key if key != "h" else "h must"):
        ctx.problem(a["h"], a["V"], a["d1"], a["d2aa"], a["d2ab"], 2)
    with pytest.raises(ValueError):
        ctx.residual(a["h"], a["V"], a["d1"], a["d2aa"], a["d2ab"], 2)
    with pytest.raises(ValueError):
        ctx.step(a["h"], a["V"], a["d1"], a["d2aa"], a["d2ab"], 2)


def test_valid_shapes_accepted():
    a = _arrays(5)
    assert acse.check_problem_shapes(a["h"], a["V"], a["d1"], a["d2aa"], a["d2ab"]) == 5
    # flat 4-index arrays of the right size are accepted too
    assert acse.check_problem_shapes(a["h"], a["V"].ravel(), a["d1"], a["d2aa"], a["d2ab"].ravel()) == 5


def test_option_arrays_must_cover_r(ctx):
    prob = acse.Problem(5, 2, 2, 0, 0, 0, 0, 0)
    for opts in (acse.Context.options(active=[1, 0, 1]), acse.Context.options(sigma=[1, 1, -1, -1])):
        with pytest.raises(ValueError, match="entries"):
            ctx.step_raw(prob, 1e-3, opts)
        with pytest.raises(ValueError, match="entries"):
            ctx.solve_raw(prob, opts, acse.SolveOptions())
    acse._check_opts(acse.Context.options(active=[1, 0, 1, 0, 0], sigma=[1, 1, -1, -1, -1]), 5)


def test_spin_calls_take_occupations_per_spin_orbital(ctx):
    """The _spin calls take 2r NY occupations (alpha orbitals first), the
    singlet calls r; the binding refuses the other length before the library."""
    prob = acse.ProblemSpin(4, 3, 1, 0, 0, 0, 0, 0, 0, 0)
    with pytest.raises(ValueError, match="2r = 8 spin orbitals"):
        ctx.step_spin_raw(prob, 1e-3, acse.Context.options(sigma=[1, 1, -1, -1]))
    with pytest.raises(ValueError, match="2r = 8 spin orbitals"):
        ctx.solve_spin_raw(prob, acse.Context.options(sigma=[1] * 4), acse.SolveOptions())
    acse._check_opts(acse.Context.options(sigma=[1, 1, 1, -1, 1, -1, -1, -1]), 4, spin=True)
    with pytest.raises(ValueError, match="r = 4 orbitals"):
        acse._check_opts(acse.Context.options(sigma=[1, 1, 1, -1, 1, -1, -1, -1]), 4)


def test_outputs_checked_before_the_library(ctx):
    prob = acse.Problem(4, 2, 2, 0, 0, 0, 0, 0)
    opts = acse.Context.options()
    host = torch.zeros((4, 4, 4, 4), dtype=torch.float64)
    with pytest.raises(ValueError, match="R_aa"):
        ctx.residual_raw(prob, opts, host, host)        # not on the device
    with pytest.raises(ValueError, match="U_aa"):
        ctx.step_raw(prob, 1e-3, opts, U_aa=host)
    with pytest.raises(ValueError, match="Rbar_aa"):
        ctx.residual_vjp_raw(prob, opts, host, host, None, None, None, None, None)
    with pytest.raises(ValueError, match="one R_aa"):
        ctx.residual_batched_raw([prob, prob], opts, [host], [host])


def test_update_map_and_vjp_check_their_tensors(ctx):
    a = _arrays(4)
    # the problem would be moved to the device first; X of the wrong size must be caught
    # without a device, so check the helper that guards it
    with pytest.raises(ValueError):
        acse._check_dev4(torch.zeros(3, 3, 3, 3, dtype=torch.float64), 4, "X_aa", torch.device("cpu"))
    with pytest.raises(ValueError):
        acse._check_dev4(torch.zeros(4, 4, 4, 4, dtype=torch.float32), 4, "X_aa", torch.device("cpu"))
    with pytest.raises(ValueError):
        acse._check_dev2(torch.zeros(4, 5, dtype=torch.float64), 4, "h_bar", torch.device("cpu"))
    acse._check_dev4(torch.zeros(4, 4, 4, 4, dtype=torch.float64), 4, "X_aa", torch.device("cpu"))
    assert a["h"].shape == (4, 4)


def test_checkpoint_tag_covers_the_iteration_options():
    a = _arrays(4)
    base = acse.checkpoint_tag(a["h"], a["V"], 2)
    assert base == acse.checkpoint_tag(a["h"], a["V"], 2, de_tol=1e-6, control="fixed", precision="fp64")
    assert base == acse.checkpoint_tag(a["h"], a["V"], 2, eps=0.5)   # the step size is not part of it
    changed = [dict(precision="fp32"), dict(active=[1, 1, 0, 0]), dict(control="backtrack"),
               dict(max_halvings=3), dict(eps_max=1.0), dict(de_tol=1e-8), dict(sigma=True),
               dict(sigma=[1, -1, 1, -1])]
    tags = {acse.checkpoint_tag(a["h"], a["V"], 2, **kw) for kw in changed}
    assert base not in tags and len(tags) == len(changed)
    assert acse.checkpoint_tag(a["h"], a["V"], 1) != base
    h2 = a["h"].copy()
    h2[0, 0] += 1e-12
    assert acse.checkpoint_tag(h2, a["V"], 2) != base
