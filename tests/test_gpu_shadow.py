"""Two-reduction BiCGStab with the index-hashed shadow residual
(WFA_OPT_SHADOW = 1) against the oracle's same variant: trajectories,
converged solves, a time step, and FP32."""
import numpy as np
import pytest

from paper_2209_13768_amd import inputs
from tests.oracle_helpers import rel_l2
from tests.parity_bars import FP32_TOL, FP64_TOL, check, sensitivity, trajectory_bound
from tests.test_gpu_parity import VARIANTS, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wfa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_13768_amd import wfa as w
    w.lib()
    return w


def _grid(wfa, prob, precision):
    g = wfa.Grid.from_problem(prob, precision=precision)
    g.set_option(wfa.OPT_SHADOW, 1)
    return g


def _sensitivity(o, b, x0, k):
    """How far the oracle's own k-th iterate moves under a one-ulp
    perturbation of b (and x0): BiCGStab amplifies rounding."""
    return sensitivity(lambda bb, xx: o.bicgstab2(bb, xx, 1e-300, k, hashed_shadow=True)[0],
                       b, x0)


@pytest.mark.parametrize("k", [1, 2, 5, 10, 20])
@pytest.mark.parametrize("name", ["cell_upwind_mixed", "const_dirichlet"])
def test_hashed_shadow_trajectory_fp64(wfa, oracle_mod, name, k):
    prob = inputs.random_problem(141, 37, 21, 18, **VARIANTS[name])
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    x0 = np.zeros(prob.shape)
    xo, io = o.bicgstab2(b, x0, 1e-300, k, hashed_shadow=True)
    g = _grid(wfa, prob, wfa.F64)
    x, info = g.solve(g.field(b), g.field(), tol=1e-300, maxit=k, method="bicgstab2")
    assert info.status == wfa.ERR_NOCONV and info.iterations == k == io.iterations
    sx = _sensitivity(o, b, x0, k)
    check(f"hashed bicgstab2 f64 {name} k={k} x", rel_l2(to_np(x), xo), trajectory_bound(sx, 2 * k),
          sx)
    # a different shadow vector gives different iterates: the option took effect
    xr, _ = o.bicgstab2(b, x0, 1e-300, k)
    if k >= 2:
        assert rel_l2(to_np(x), xr) > 1e-9


@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_hashed_shadow_converged_matches_oracle(wfa, oracle_mod, name):
    prob = inputs.random_problem(142, 24, 18, 14, **VARIANTS[name])
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    xo, _ = o.bicgstab2(b, prob.T0, 1e-14, 2000, hashed_shadow=True)
    g = _grid(wfa, prob, wfa.F64)
    x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e-14, maxit=2000, method="bicgstab2")
    assert info.status == wfa.OK
    assert rel_l2(to_np(x), xo) <= FP64_TOL
    assert o.true_relres(b, to_np(x)) <= 1e-13


def test_hashed_shadow_timestep_restart_and_fp32(wfa, oracle_mod):
    prob = inputs.convdiff(n=40, seed=9)
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    g = _grid(wfa, prob, wfa.F64)
    g.set_option(wfa.OPT_METHOD, wfa.METHOD_BICGSTAB2)
    T = g.field(prob.T0)
    info = g.timestep(T, 1, tol=1e-10, maxit=5000)[0]
    assert info.status == wfa.OK
    assert o.true_relres(b, to_np(T)) <= 1e-10
    g.set_option(wfa.OPT_FORCE_BREAKDOWN, 5)
    x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e-10, maxit=5000, method="bicgstab2")
    assert info.status == wfa.OK and info.restarts == 1
    assert o.true_relres(b, to_np(x)) <= 1e-10
    g32 = _grid(wfa, prob, wfa.F32)
    b32 = g32.rhs(g32.field(prob.T0))
    x, info = g32.solve(b32, g32.field(prob.T0), tol=1e-5, maxit=5000, method="bicgstab2")
    assert info.status == wfa.OK and info.rel_res_true <= 2e-5
    # FP32 first iterates against the FP64 oracle
    p2 = inputs.heat_32(n=24)
    o2 = oracle_mod.Oracle(p2)
    b2 = o2.rhs(p2.T0)
    xo, _ = o2.bicgstab2(b2, p2.T0, 1e-300, 5, hashed_shadow=True)
    g2 = _grid(wfa, p2, wfa.F32)
    x2, _ = g2.solve(g2.field(b2), g2.field(p2.T0), tol=1e-300, maxit=5, method="bicgstab2",
                     check=False)
    assert rel_l2(to_np(x2), xo) <= FP32_TOL


def test_hashed_shadow_inside_refinement(wfa, oracle_mod):
    """FP32-in-FP64 refinement whose inner two-reduction solves use the
    hashed shadow: same FP64 accuracy as with r^ = r0."""
    prob = inputs.convdiff(n=40, seed=4, u=(4.0, 2.0, 1.0))
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    xs = []
    for shadow in (0, 1):
        g = wfa.Grid.from_problem(prob, precision=wfa.F32_IR64)
        g.set_option(wfa.OPT_SHADOW, shadow)
        x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e-12, maxit=5000)
        assert info.status == wfa.OK, info
        assert o.true_relres(b, to_np(x)) <= 1e-12
        xs.append(to_np(x))
    assert rel_l2(xs[1], xs[0]) <= 1e-9
    assert not np.array_equal(xs[0], xs[1])          # the option took effect
