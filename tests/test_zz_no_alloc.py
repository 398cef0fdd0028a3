"""wfa_bicgstab_solve_static, the solve that allocates nothing, against
wfa_bicgstab_solve on a grid over a caller workspace.

The two must give bitwise the same x and info: the same kernels run with the
same tiling over a workspace that differs only in where it lives.  Two calls
in a row per precision, the second on a smaller grid over what the first
left in the static workspace, and the oracle's operator on the results.
"""
import numpy as np
import pytest

from paper_2209_13768_amd import inputs
from tests.parity_bars import check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wfa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_13768_amd import wfa as w
    w.lib()
    w.tune_clear()          # default tiling for both paths
    return w


def _grid_args(prob, precision):
    import torch
    kappa = torch.from_numpy(prob.kappa).cuda() if prob.kappa is not None else None
    return dict(nx=prob.nx, ny=prob.ny, nz=prob.nz, h=prob.h, dt=prob.dt, alpha=prob.alpha,
                kappa=kappa, u=prob.u, bc=prob.bc_kind, bc_value=prob.bc_value,
                precision=precision)


CALLS = [(70, 45, 38), (33, 17, 5)]        # the second call is smaller


@pytest.mark.parametrize("precision", ["f64", "f32", "f32_ir64"])
def test_static_solve_equals_workspace_solve(wfa, oracle_mod, precision):
    import torch
    prec = wfa.PRECISIONS[precision]
    tol = 1e-5 if precision == "f32" else 1e-10
    for shape in CALLS:
        prob = inputs.random_problem(401, *shape, cell=True, u=(1.0, -0.5, 0.25),
                                     bc_kind=inputs.MIXED_BC_KIND)
        g = wfa.Grid.from_problem(prob, precision=prec)
        b = g.rhs(g.field(prob.T0))
        x_ref, i_ref = g.solve(b, g.field(prob.T0), tol=tol, maxit=3000, method="bicgstab")
        x_st, i_st = wfa.solve_static(_grid_args(prob, prec), b.clone(), g.field(prob.T0),
                                      tol=tol, maxit=3000)
        torch.cuda.synchronize()
        assert i_ref.status == wfa.OK, (shape, i_ref)
        assert bool(torch.equal(x_st, x_ref)), (precision, shape)
        for f in ("status", "iterations", "restarts", "refinements", "rel_res_recursive",
                  "rel_res_true"):
            assert getattr(i_st, f) == getattr(i_ref, f), (precision, shape, f)
        o = oracle_mod.Oracle(prob)
        xo = x_st.cpu().double().numpy()
        bo = b.cpu().double().numpy()
        check(f"static solve {precision} {'x'.join(map(str, shape))} true residual",
              o.true_relres(bo, xo), 2e-5 if precision == "f32" else tol)


def test_static_solve_limits(wfa):
    """A grid whose workspace exceeds the static array is refused before
    any launch (WFA_ERR_NOMEM); bad arguments give WFA_ERR_INVALID."""
    import torch
    n = 256
    prob = inputs.Problem(n, n, n, h=inputs.grid_spacing(n, n, n), dt=1e-3, alpha=1.0)
    assert wfa.workspace_bytes(n, n, n, wfa.F64) > wfa.STATIC_WORKSPACE_BYTES
    f = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(wfa.WfaError) as e:
        wfa.solve_static(_grid_args(prob, wfa.F64), f, f.clone(), tol=1e-8, maxit=10)
    assert e.value.code == wfa.ERR_NOMEM
    small = inputs.Problem(8, 8, 8, h=inputs.grid_spacing(8, 8, 8), dt=1e-3, alpha=1.0)
    g = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(wfa.WfaError) as e:
        wfa.solve_static(_grid_args(small, wfa.F64), g, g.clone(), tol=-1.0, maxit=10)
    assert e.value.code == wfa.ERR_INVALID
    # b = 0 gives x = 0
    x, info = wfa.solve_static(_grid_args(small, wfa.F64), g, g.clone() + 1.0, tol=1e-10,
                               maxit=10)
    assert info.status == wfa.OK and info.iterations == 0 and not bool(x.any())
