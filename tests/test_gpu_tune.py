"""Tile-shape autotuner on the GPU: it picks one of its candidates, the grid
and every later grid of the same key use it, the solver options survive,
solves on the tuned tiling still match the oracle, and the serving path
takes the tuned plane depth (bitwise the single-grid result on it)."""
import numpy as np
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
    yield w
    w.tune_clear()


def test_autotune_applies_and_records(wfa, oracle_mod, tmp_path):
    prob = inputs.random_problem(131, 70, 45, 38, cell=True, u=(1.0, -0.5, 2.0),
                                 bc_kind=inputs.MIXED_BC_KIND)
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    g.set_option(wfa.OPT_METHOD, wfa.METHOD_BICGSTAB2)
    res = g.autotune("bicgstab2", iters=6)
    assert res["ry"] in (1, 2, 4) and 1 <= res["zc"] <= 38
    assert res["candidates"] >= 10
    assert res["us_per_iter"] <= res["us_per_iter_default"]
    tx, ty, zc, blocks = g.tiling()
    assert (ty, zc) == (4 * res["ry"], res["zc"])
    g2 = wfa.Grid.from_problem(prob, precision=wfa.F64)
    assert g2.tiling() == g.tiling()
    # options survive: timestep uses the method set before tuning, on the tuned tiling
    o = oracle_mod.Oracle(prob)
    To, _ = o.timestep(prob.T0, 1, 1e-13, 5000)
    T = g.field(prob.T0)
    info = g.timestep(T, 1, tol=1e-13, maxit=5000)[0]
    assert info.status == wfa.OK
    assert rel_l2(T.cpu().numpy(), To) <= 1e-10
    T2 = g2.field(prob.T0)
    g2.set_option(wfa.OPT_METHOD, wfa.METHOD_BICGSTAB2)
    g2.timestep(T2, 1, tol=1e-13, maxit=5000)
    assert np.array_equal(T.cpu().numpy(), T2.cpu().numpy())
    path = tmp_path / "table.txt"
    wfa.tune_save(str(path))
    line = [ln for ln in path.read_text().splitlines() if ln.startswith("70 45 38 0 1 ")]
    assert len(line) == 1 and line[0].split()[5:7] == [str(res["ry"]), str(res["zc"])]


def test_server_uses_tuned_plane_depth(wfa, tmp_path):
    """FP64 requests: the reduction order (hence the tiling) reaches the
    iterates' last bits, so bitwise equality with the single-grid solve on
    the tuned tiling, and inequality with the default tiling, show which
    tiling the server ran.  (With FP32 inner vectors the FP64-accumulated
    scalars almost never round differently, so the result does not depend
    on the tiling at all.)"""
    import torch
    rq = inputs.Request(0, 0.0, 64, 40, 36)
    prob = rq.problem()
    g0 = wfa.Grid.from_problem(prob, precision=wfa.F64)
    g0.set_option(wfa.OPT_METHOD, wfa.METHOD_BICGSTAB2)   # the server's method
    g0.set_option(wfa.OPT_SHADOW, 1)                      # and shadow residual
    ry = g0.tiling()[1] // 4
    path = tmp_path / "t.txt"
    path.write_text(f"64 40 36 {wfa.F64} 0 {ry} 3 1.0\n")
    wfa.tune_load(str(path))
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    g.set_option(wfa.OPT_METHOD, wfa.METHOD_BICGSTAB2)
    g.set_option(wfa.OPT_SHADOW, 1)
    assert g.tiling()[2] == 3 and g0.tiling()[2] != 3
    T = g.field(prob.T0)
    gi = g.timestep(T, 1, tol=1e-10, maxit=20000)[0]
    sv = wfa.Server(1 << 30, max_slots=2)
    Ts = torch.from_numpy(prob.T0).to("cuda", torch.float64)
    t = sv.submit_problem(prob, Ts, precision=wfa.F64, tol=1e-10, maxit=20000)
    sv.drain()
    code, info = sv.poll(t)
    sv.close()
    assert code == wfa.OK
    assert np.array_equal(Ts.cpu().numpy(), T.cpu().numpy())
    assert info.iterations == gi.iterations
    T0 = g0.field(prob.T0)
    g0.timestep(T0, 1, tol=1e-10, maxit=20000)
    assert not np.array_equal(T0.cpu().numpy(), T.cpu().numpy())
    wfa.tune_clear()


@pytest.mark.parametrize("iters", [20, 150])
def test_autotune_fp32_convection_diffusion_256(wfa, iters):
    """The 256^3 convection-diffusion grid in FP32: the timed solves may stop
    early on their own numbers (a diverging FP32 BiCGStab), which must not
    end the tuning; every candidate is timed and one is chosen."""
    prob = inputs.convdiff(n=256)
    g = wfa.Grid.from_problem(prob, precision=wfa.F32)
    g.set_option(wfa.OPT_METHOD, wfa.METHOD_BICGSTAB2)
    g.set_option(wfa.OPT_SHADOW, 1)
    res = g.autotune("bicgstab2", iters=iters)
    assert res["ry"] in (1, 2, 4) and 1 <= res["zc"] <= 64
    assert res["candidates"] >= 20
    assert 0.0 < res["us_per_iter"] <= res["us_per_iter_default"]
    # a sane cost: 56 bytes per cell and iteration at no more than 8 TB/s
    assert res["us_per_iter"] >= 56 * prob.cells / 8e12 * 1e6
    wfa.tune_clear()
