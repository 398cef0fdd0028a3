"""Breakdown restarts and staged halo values, through the C-ABI.

Restarts (reading R8 of the breakdown rule): a breakdown forced from the host
at full iteration n (WFA_OPT_FORCE_BREAKDOWN) restarts from b - A x_{n-1}.
The iterates that follow are compared with the oracle's solve forced the same
way, at the trajectory bar of tests/parity_bars.py, for the textbook form,
the two-reduction form and its hashed shadow residual.

Staging: the passes that apply an operator to a vector they form on the fly
(p' in both BiCGStab organisations, r' in CG with one reduction) compute each
cell's value twice, once where it is stored and once on every neighbouring
tile's halo.  Both copies must round the same way: the stored v' must be the
operator applied to the stored p', bit for bit, on grids whose tiles are
ragged in x, y and z.
"""
import numpy as np
import pytest

from paper_2209_13768_amd import inputs
from tests.oracle_helpers import rel_l2
from tests.parity_bars import check, sensitivity, trajectory_bound
from tests.test_gpu_parity import to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wfa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_13768_amd import wfa as w
    w.lib()
    return w


FORMS = {
    "textbook": dict(method="bicgstab", shadow=0),
    "two_reduction": dict(method="bicgstab2", shadow=0),
    "two_reduction_hashed": dict(method="bicgstab2", shadow=1),
}


def _oracle_forced(o, form, b, x0, k, n):
    if form == "textbook":
        return o.bicgstab(b, x0, 1e-300, k, force_breakdown=n)
    return o.bicgstab2(b, x0, 1e-300, k, force_breakdown=n,
                       hashed_shadow=FORMS[form]["shadow"] == 1)


@pytest.mark.parametrize("form", sorted(FORMS))
def test_forced_restart_trajectory(wfa, oracle_mod, form):
    prob = inputs.random_problem(108, 37, 21, 18, cell=True, u=(1.0, 0.5, 0.25),
                                 bc_kind=inputs.MIXED_BC_KIND)
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    n = 4
    for k in (3, 4, 5, 8, 12):
        xo, io = _oracle_forced(o, form, b, prob.T0, k, n)
        assert io.iterations == k and io.restarts == (1 if k >= n else 0)
        g = wfa.Grid.from_problem(prob, precision=wfa.F64)
        g.set_option(wfa.OPT_SHADOW, FORMS[form]["shadow"])
        g.set_option(wfa.OPT_FORCE_BREAKDOWN, n)
        x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e-300, maxit=k,
                          method=FORMS[form]["method"], check=False)
        assert info.status == wfa.ERR_NOCONV, (k, info)
        assert info.iterations == k and info.restarts == io.restarts, (k, info, io)
        sx = sensitivity(lambda bb, xx: _oracle_forced(o, form, bb, xx, k, n)[0], b, prob.T0,
                         seeds=(0,))
        # 2k products of the iterations and one for the restart's residual
        check(f"forced restart {form} n={n} k={k} x", rel_l2(to_np(x), xo),
              trajectory_bound(sx, 2 * k + 1), sx)


@pytest.mark.parametrize("form", sorted(FORMS))
def test_forced_restart_converges_like_oracle(wfa, oracle_mod, form):
    """A solve that restarts still reaches the oracle's converged solution
    (well-conditioned case, both to 1e-13)."""
    prob = inputs.random_problem(110, 22, 16, 10, cell=True, u=(2.0, 1.0, 0.0))
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    xo, io = _oracle_forced(o, form, b, prob.T0, 3000, 5)
    assert io.status == oracle_mod.OK and io.restarts == 1
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    g.set_option(wfa.OPT_SHADOW, FORMS[form]["shadow"])
    g.set_option(wfa.OPT_FORCE_BREAKDOWN, 5)
    x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e-13, maxit=3000,
                      method=FORMS[form]["method"])
    assert info.status == wfa.OK and info.restarts == 1
    check(f"forced restart {form} converged x", rel_l2(to_np(x), xo), 1e-11)
    assert o.true_relres(b, to_np(x)) <= 1e-13


STAGED = {
    "textbook": dict(method="bicgstab", shadow=0, pairs=((3, 5), (4, 6))),
    "two_reduction_hashed": dict(method="bicgstab2", shadow=1, pairs=((3, 5), (4, 6))),
    "two_reduction": dict(method="bicgstab2", shadow=0, pairs=((3, 5), (4, 6))),
    "cg1": dict(method="cg1", shadow=0, pairs=((0, 5), (8, 6))),
}
# (rows per wave, z planes per workgroup): 70 x 45 x 38 leaves ragged tiles in
# x (64 + 6), y (4 ry rows per tile) and z for each of these
TILINGS = [(0, 0), (1, 4), (2, 16), (4, 32)]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name", sorted(STAGED))
def test_staged_vector_is_what_the_operator_saw(wfa, name, precision):
    spec = STAGED[name]
    u = (0.0, 0.0, 0.0) if name == "cg1" else (1.0, -0.5, 2.0)
    prob = inputs.random_problem(120, 70, 45, 38, cell=True, u=u, bc_kind=inputs.MIXED_BC_KIND)
    for ry, zc in TILINGS:
        g = wfa.Grid.from_problem(prob, precision=wfa.PRECISIONS[precision])
        g.set_option(wfa.OPT_SHADOW, spec["shadow"])
        if ry:
            g.set_option(wfa.OPT_RY, ry)
            g.set_option(wfa.OPT_ZCHUNK, zc)
        b = g.rhs(g.field(prob.T0))
        x, info = g.solve(b, g.field(prob.T0), tol=1e-300, maxit=3, method=spec["method"],
                          check=False)
        assert info.status == wfa.ERR_NOCONV and info.iterations == 3, (ry, zc, info)
        for src, dst in spec["pairs"]:
            staged = g.vector(src).clone()
            stored = g.vector(dst).clone()
            assert staged.abs().max().item() > 0.0
            again = g.apply(staged)
            same = bool((again == stored).all().item())
            diff = (again - stored).abs().max().item()
            assert same, (name, precision, ry, zc, src, dst, diff)
