"""Pass 1 of the two-reduction BiCGStab forming t = A s again
(WFA_OPT_RECOMPUTE_T) against the passes that store t and read it back.

The fused pass stages s with pass 2's operations and applies the same
operator, so t, every store and every partial sum are bitwise those of the
stored-t passes: x, the iteration count and the residuals must be identical
bit for bit, on grids whose tiles are ragged in x, y and z, for every tiling
the autotuner may pick (one plane per workgroup included), both shadow
residuals, Jacobi scaling, refinement's FP32 inner solve, restarts and
graph replay.  The oracle check of the same path is in the trajectory and
converged-solve tests, which these runs match bit for bit.
"""
import pytest

from paper_2209_13768_amd import inputs
from tests.oracle_helpers import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wfa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_13768_amd import wfa as w
    w.lib()
    w.tune_clear()
    return w


PROBLEMS = {
    "cell_upwind_mixed_70x45x38": (dict(cell=True, u=(1.0, -0.5, 2.0), bc_kind=inputs.MIXED_BC_KIND),
                                   (70, 45, 38)),
    "const_33x17x5": (dict(cell=False), (33, 17, 5)),
    "cell_7x1x40": (dict(cell=True, u=(0.5, 0.0, -1.0)), (7, 1, 40)),
    "cell_1x1x1": (dict(cell=True), (1, 1, 1)),
    "cell_130x9x3": (dict(cell=True, bc_kind=(inputs.ZEROFLUX,) * 6), (130, 9, 3)),
}
TILINGS = [(0, 0), (1, 1), (1, 4), (2, 1), (2, 2), (2, 16), (4, 1), (4, 3), (4, 32)]


def _pair(wfa, prob, precision, ry, zc):
    """Two grids of the problem on the same tiling: t stored, t formed again."""
    out = []
    for rec in (0, 1):
        g = wfa.Grid.from_problem(prob, precision=wfa.PRECISIONS[precision])
        if ry:
            g.set_option(wfa.OPT_RY, ry)
            g.set_option(wfa.OPT_ZCHUNK, min(zc, prob.nz))
        g.set_option(wfa.OPT_RECOMPUTE_T, rec)
        out.append(g)
    return out


def _same(a, b):
    import torch
    return bool(torch.equal(a, b))


def _info_same(i0, i1):
    return (i0.status, i0.iterations, i0.restarts, i0.refinements, i0.rel_res_recursive,
            i0.rel_res_true) == (i1.status, i1.iterations, i1.restarts, i1.refinements,
                                 i1.rel_res_recursive, i1.rel_res_true)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_recompute_t_bitwise_over_tilings(wfa, name, precision):
    kw, shape = PROBLEMS[name]
    prob = inputs.random_problem(501, *shape, **kw)
    for ry, zc in TILINGS:
        for shadow in (0, 1):
            g0, g1 = _pair(wfa, prob, precision, ry, zc)
            for g in (g0, g1):
                g.set_option(wfa.OPT_SHADOW, shadow)
            b = g0.rhs(g0.field(prob.T0))
            for maxit in (1, 2, 7):
                x0, i0 = g0.solve(b, g0.field(prob.T0), tol=1e-300, maxit=maxit,
                                  method="bicgstab2", check=False)
                x1, i1 = g1.solve(b, g1.field(prob.T0), tol=1e-300, maxit=maxit,
                                  method="bicgstab2", check=False)
                assert _same(x0, x1), (name, precision, ry, zc, shadow, maxit)
                assert _info_same(i0, i1), (name, precision, ry, zc, shadow, maxit, i0, i1)
        del g0, g1


@pytest.mark.parametrize("precision", ["f64", "f32", "f32_ir64"])
def test_recompute_t_bitwise_converged_and_timesteps(wfa, oracle_mod, precision):
    prob = inputs.random_problem(502, 70, 45, 38, cell=True, u=(1.0, 0.5, 0.25),
                                 bc_kind=inputs.MIXED_BC_KIND)
    tol = 1e-5 if precision == "f32" else 1e-10
    for shadow in (0, 1):
        g0, g1 = _pair(wfa, prob, precision, 0, 0)
        for g in (g0, g1):
            g.set_option(wfa.OPT_SHADOW, shadow)
            g.set_option(wfa.OPT_METHOD, wfa.METHOD_BICGSTAB2)
        T0, T1 = g0.field(prob.T0), g1.field(prob.T0)
        i0 = g0.timestep(T0, 3, tol=tol, maxit=5000)
        i1 = g1.timestep(T1, 3, tol=tol, maxit=5000)
        assert _same(T0, T1), (precision, shadow)
        assert all(_info_same(a, b) for a, b in zip(i0, i1)), (precision, shadow, i0, i1)
        if precision != "f32":
            o = oracle_mod.Oracle(prob)
            To, _ = o.timestep(prob.T0, 3, tol, 5000)
            assert rel_l2(T1.cpu().double().numpy(), To) <= 1e-6


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_recompute_t_bitwise_jacobi_restart_graph(wfa, precision):
    prob = inputs.random_problem(503, 66, 40, 21, cell=True, u=(2.0, -1.0, 0.5),
                                 bc_kind=inputs.MIXED_BC_KIND, sigma=2.0)
    # Jacobi scaling
    g0, g1 = _pair(wfa, prob, precision, 0, 0)
    for g in (g0, g1):
        g.set_option(wfa.OPT_JACOBI, 1)
    b = g0.rhs(g0.field(prob.T0))
    x0, i0 = g0.solve(b, g0.field(prob.T0), tol=1e-300, maxit=9, method="bicgstab2", check=False)
    x1, i1 = g1.solve(b, g1.field(prob.T0), tol=1e-300, maxit=9, method="bicgstab2", check=False)
    assert _same(x0, x1) and _info_same(i0, i1)
    # a forced breakdown and restart
    g0, g1 = _pair(wfa, prob, precision, 0, 0)
    for g in (g0, g1):
        g.set_option(wfa.OPT_FORCE_BREAKDOWN, 4)
    x0, i0 = g0.solve(b, g0.field(prob.T0), tol=1e-300, maxit=9, method="bicgstab2", check=False)
    x1, i1 = g1.solve(b, g1.field(prob.T0), tol=1e-300, maxit=9, method="bicgstab2", check=False)
    assert i0.restarts == 1 and _same(x0, x1) and _info_same(i0, i1)
    # graph replay of the fused passes against plain launches
    g0, g1 = _pair(wfa, prob, precision, 0, 0)
    g0.set_option(wfa.OPT_RECOMPUTE_T, 1)
    g1.set_option(wfa.OPT_GRAPH, 1)
    g1.set_option(wfa.OPT_CHECK_EVERY, 16)
    for _ in range(2):   # replays after the first capture too
        x0, i0 = g0.solve(b, g0.field(prob.T0), tol=1e-300, maxit=33, method="bicgstab2",
                          check=False)
        x1, i1 = g1.solve(b, g1.field(prob.T0), tol=1e-300, maxit=33, method="bicgstab2",
                          check=False)
        assert _same(x0, x1) and _info_same(i0, i1)


def test_recompute_t_option_validated(wfa):
    prob = inputs.random_problem(504, 8, 8, 8)
    g = wfa.Grid.from_problem(prob)
    with pytest.raises(wfa.WfaError) as e:
        g.set_option(wfa.OPT_RECOMPUTE_T, 2)
    assert e.value.code == wfa.ERR_INVALID
