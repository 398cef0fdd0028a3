"""CG with one reduction per iteration (Chronopoulos-Gear) on the GPU against
the oracle's same method and its textbook CG.

Bars (relative L2):
  trajectories (same x0, k <= 20 iterations): 1e-12 FP64, or 100x the
    oracle's own change under a one-ulp perturbation of b or of x0 where
    rounding is amplified beyond that; 1e-5 FP32;
  converged solves (both sides to 1e-14): 1e-11, against the one-reduction
    oracle and against classic CG (the same iterates in exact arithmetic);
  the 32^3 heat workload's 10 steps: as the classic solver's heat test.
The fused pass applies each iteration's update while it forms the next
operator product, so the halo cells recompute the neighbours' new residual:
the trajectory tests run on tilings with many tiles and ragged tails.
As the inner FP32 solve of refinement it must reach FP64 accuracy (1e-12
under the oracle's operator), including after a forced inner divergence.
"""
import numpy as np
import pytest

from paper_2209_13768_amd import inputs
from paper_2209_13768_amd.inputs import DIRICHLET, ZEROFLUX
from tests.oracle_helpers import rel_l2
from tests.parity_bars import FP32_TOL, FP64_TOL, check, sensitivity, trajectory_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wfa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_13768_amd import wfa as w
    w.lib()
    return w


def to_np(t):
    return t.detach().cpu().double().numpy()


SYMMETRIC = {
    "const_dirichlet": dict(shape=(64, 16, 16), cell=False),
    "cell_mixed": dict(shape=(130, 37, 19), cell=True, bc_kind=inputs.MIXED_BC_KIND),
    "cell_zeroflux_mostly": dict(shape=(33, 17, 5), cell=True,
                                 bc_kind=(ZEROFLUX, ZEROFLUX, DIRICHLET, ZEROFLUX, ZEROFLUX,
                                          ZEROFLUX)),
}


def _problem(name, seed=301):
    v = dict(SYMMETRIC[name])
    nx, ny, nz = v.pop("shape")
    return inputs.random_problem(seed, nx, ny, nz, **v)


def _sensitivity(o, b, x0, k):
    """How far the oracle's own k-th iterate moves when b, or x0, is perturbed
    by one ulp in a random direction.  On the nearly all-zero-flux grid the
    recurrences amplify rounding of x0 far more than rounding of b (by 1e3 at
    k = 20), so both are taken."""
    return sensitivity(lambda bb, xx: o.cg1(bb, xx, 1e-300, k)[0], b, x0, seeds=(0,))


@pytest.mark.parametrize("k", [1, 2, 5, 10, 20])
@pytest.mark.parametrize("name", sorted(SYMMETRIC))
def test_cg1_trajectory_fp64(wfa, oracle_mod, name, k):
    prob = _problem(name)
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    xo, io = o.cg1(b, prob.T0, 1e-300, k)
    assert io.iterations == k
    sx = _sensitivity(o, b, prob.T0, k)
    bound = trajectory_bound(sx, k + 1)     # k iterations after w0 = A r0
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e-300, maxit=k, method="cg1",
                      check=False)
    assert info.status == wfa.ERR_NOCONV and info.iterations == k
    check(f"cg1 f64 {name} k={k} x", rel_l2(to_np(x), xo), bound, sx)
    # the recursive residual norm the library reports (relative to ||b||) is
    # the oracle's; a wrong reduction would move it at O(1)
    assert abs(info.rel_res_recursive - io.rel_res_recursive) <= 1e-8


@pytest.mark.parametrize("k", [1, 5])
def test_cg1_trajectory_fp32(wfa, oracle_mod, k):
    prob = _problem("cell_mixed")
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    xo, _ = o.cg1(b, prob.T0, 1e-300, k)
    g = wfa.Grid.from_problem(prob, precision=wfa.F32)
    x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e-300, maxit=k, method="cg1",
                      check=False)
    assert info.iterations == k
    assert rel_l2(to_np(x), xo) <= FP32_TOL


@pytest.mark.parametrize("name", sorted(SYMMETRIC))
def test_cg1_converged_matches_oracle_and_classic_cg(wfa, oracle_mod, name):
    prob = _problem(name, seed=302)
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    x1, i1 = o.cg1(b, prob.T0, 1e-14, 5000)
    xc, ic = o.cg(b, prob.T0, 1e-14, 5000)
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e-14, maxit=5000, method="cg1")
    assert info.status == wfa.OK and i1.status == ic.status == 0
    # ~1000 iterations on the mixed grid: rounding shifts the stopping
    # iteration by a few
    assert abs(info.iterations - i1.iterations) <= max(2, i1.iterations // 50)
    assert info.rel_res_true <= max(1e-13, 4 * i1.rel_res_true)
    assert rel_l2(to_np(x), x1) <= 1e-11
    assert rel_l2(to_np(x), xc) <= 1e-11


def test_cg1_heat_32_ten_steps(wfa, oracle_mod):
    """The 32^3 heat workload, 10 backward-Euler steps to 1e-10 with the
    one-reduction CG; cond(A) ~ 13.6, so the steps agree with the oracle's
    (BiCGStab) steps to ~cond * tol each, and to 1e-12 when both solve to
    1e-14.  The first step's solve takes the oracle's one-reduction CG's
    iteration count."""
    prob = inputs.heat_32()
    o = oracle_mod.Oracle(prob)
    To, _ = o.timestep(prob.T0, 10, 1e-10, 1000)
    _, i1 = o.cg1(o.rhs(prob.T0), prob.T0, 1e-10, 1000)
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    g.set_option(wfa.OPT_METHOD, wfa.METHOD_CG1)
    T = g.field(prob.T0)
    infos = g.timestep(T, 10, tol=1e-10, maxit=1000)
    assert all(i.status == wfa.OK for i in infos)
    assert abs(infos[0].iterations - i1.iterations) <= 1
    assert rel_l2(to_np(T), To) <= 10 * 14 * 2e-10
    To2, _ = o.timestep(prob.T0, 2, 1e-14, 1000)
    T2 = g.field(prob.T0)
    g.timestep(T2, 2, tol=1e-14, maxit=1000)
    assert rel_l2(to_np(T2), To2) <= FP64_TOL


def test_cg1_status_paths(wfa, oracle_mod):
    prob = _problem("cell_mixed", seed=303)
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    # b == 0 -> x = 0, zero iterations
    x, info = g.solve(g.field(), g.field(prob.T0), tol=1e-10, maxit=50, method="cg1")
    assert info.status == wfa.OK and info.iterations == 0 and not to_np(x).any()
    # converged at the initial guess: zero iterations, x untouched
    x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e3, maxit=50, method="cg1")
    assert info.status == wfa.OK and info.iterations == 0
    assert np.array_equal(to_np(x), prob.T0)
    # maxit -> NOCONV with the last iterate
    xo, _ = o.cg1(b, prob.T0, 1e-300, 1)
    x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e-14, maxit=1, method="cg1",
                      check=False)
    assert info.status == wfa.ERR_NOCONV and info.iterations == 1
    assert rel_l2(to_np(x), xo) <= FP64_TOL
    # NaN -> NONFINITE
    bad = b.copy()
    bad[3, 4, 5] = np.nan
    x, info = g.solve(g.field(bad), g.field(prob.T0), tol=1e-10, maxit=50, method="cg1",
                      check=False)
    assert info.status == wfa.ERR_NONFINITE
    # what the method does not cover is rejected before any launch
    nonsym = inputs.random_problem(304, 12, 10, 8, cell=True, u=(1.0, 0.0, 0.0))
    gn = wfa.Grid.from_problem(nonsym, precision=wfa.F64)
    with pytest.raises(wfa.WfaError) as e:
        gn.solve(gn.field(), gn.field(), tol=1e-10, maxit=10, method="cg1")
    assert e.value.code == wfa.ERR_INVALID
    gi = wfa.Grid.from_problem(prob, precision=wfa.F32_IR64)
    with pytest.raises(wfa.WfaError) as e:
        gi.solve(gi.field(b), gi.field(), tol=1e-10, maxit=10, method="cg")
    assert e.value.code == wfa.ERR_INVALID
    gj = wfa.Grid.from_problem(prob, precision=wfa.F64)
    gj.set_option(wfa.OPT_JACOBI, 1)
    with pytest.raises(wfa.WfaError) as e:
        gj.solve(gj.field(b), gj.field(), tol=1e-10, maxit=10, method="cg1")
    assert e.value.code == wfa.ERR_INVALID


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_cg1_chunking_graphs_and_profiling_are_bitwise_identical(wfa, precision):
    """Chunk sizes (host checks every 1, 7 or 64 iterations, or adaptive),
    graph replay and the profiled path change when the host looks, never what
    the kernels compute; two runs are identical bit for bit."""
    prob = _problem("cell_mixed", seed=305)
    prec = wfa.PRECISIONS[precision]
    tol = 1e-5 if precision == "f32" else 1e-10
    ref = None
    for check_every, graph, profile in ((0, 0, 0), (0, 0, 0), (1, 0, 0), (7, 0, 0), (64, 0, 0),
                                        (0, 1, 0), (13, 1, 0), (5, 0, 1)):
        g = wfa.Grid.from_problem(prob, precision=prec)
        g.set_option(wfa.OPT_CHECK_EVERY, check_every)
        g.set_option(wfa.OPT_GRAPH, graph)
        g.set_option(wfa.OPT_PROFILE, profile)
        b = g.rhs(g.field(prob.T0))
        x, info = g.solve(b, g.field(prob.T0), tol=tol, maxit=3000, method="cg1")
        assert info.status == wfa.OK
        out = (to_np(x), info.iterations, info.rel_res_recursive, info.rel_res_true)
        if ref is None:
            ref = out
            continue
        assert np.array_equal(out[0], ref[0]), (check_every, graph, profile)
        assert out[1:] == ref[1:], (check_every, graph, profile)
        if profile:
            # one pass per iteration plus the pass that forms w0 = A r0, and
            # the rest of the chunk that ended the solve (those exit at once)
            n, ms, by = g.kernel_stats(wfa.K_CG1)
            assert info.iterations + 1 <= n < info.iterations + 1 + check_every and ms > 0
            w = 4 if precision == "f32" else 8
            assert by == (10 * w + 4) * prob.cells


def test_cg1_needs_half_the_passes_of_classic_cg(wfa):
    """Iteration counts of the two CG forms agree; the one-reduction form
    launches one operator pass per iteration (and one for w0 = A r0), classic
    CG two.  An iteration limit makes the launch counts exact."""
    prob = _problem("const_dirichlet", seed=306)
    out = {}
    for method, kernels in (("cg", (wfa.K_CG_A, wfa.K_CG_B)), ("cg1", (wfa.K_CG1,))):
        g = wfa.Grid.from_problem(prob, precision=wfa.F64)
        b = g.rhs(g.field(prob.T0))
        _, info = g.solve(b, g.field(), tol=1e-10, maxit=3000, method=method)
        assert info.status == wfa.OK
        g.set_option(wfa.OPT_PROFILE, 1)
        _, cap = g.solve(b, g.field(), tol=1e-300, maxit=40, method=method, check=False)
        assert cap.status == wfa.ERR_NOCONV and cap.iterations == 40
        out[method] = (info.iterations, sum(g.kernel_stats(k)[0] for k in kernels))
    assert abs(out["cg"][0] - out["cg1"][0]) <= 1
    assert out["cg"][1] == 2 * 40
    assert out["cg1"][1] == 40 + 1


def test_cg1_refinement_reaches_fp64_accuracy(wfa, oracle_mod):
    """FP32 one-reduction CG (on A itself) inside FP64 refinement, on the
    log-normal-diffusivity grid without velocity: the result meets 1e-12
    under the oracle's operator, and the host's chunking leaves it unchanged
    bit for bit."""
    prob = inputs.convdiff(n=40, seed=4, u=(0.0, 0.0, 0.0))
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    xo, _ = o.cg1(b, prob.T0, 1e-13, 5000)
    outs = []
    for check_every in (0, 5):
        g = wfa.Grid.from_problem(prob, precision=wfa.F32_IR64)
        g.set_option(wfa.OPT_CHECK_EVERY, check_every)
        x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e-12, maxit=5000, method="cg1")
        assert info.status == wfa.OK, info
        assert info.refinements >= 2
        assert o.true_relres(b, to_np(x)) <= 1e-12
        assert info.rel_res_true <= 1e-12
        assert rel_l2(to_np(x), xo) <= 1e-7
        outs.append((to_np(x), info.iterations, info.refinements))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1:] == outs[1][1:]


def test_cg1_refinement_recovers_from_a_diverged_inner_solve(wfa, oracle_mod):
    """An inner CG solve declared diverged from the host at inner iteration 7
    is repeated once, stopped at its smallest residual, and its correction
    applied: the solve still reaches 1e-12, with one more residual pass."""
    prob = inputs.convdiff(n=40, seed=4, u=(0.0, 0.0, 0.0))
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    runs = []
    for force in (0, 7):
        g = wfa.Grid.from_problem(prob, precision=wfa.F32_IR64)
        g.set_option(wfa.OPT_PROFILE, 1)
        g.set_option(wfa.OPT_FORCE_DIVERGE, force)
        x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e-12, maxit=5000, method="cg1")
        assert info.status == wfa.OK, (force, info)
        assert o.true_relres(b, to_np(x)) <= 1e-12
        runs.append((to_np(x), info, g.kernel_stats(wfa.K_RESIDUAL)[0]))
    (x0, i0, n0), (x1, i1, n1) = runs
    assert n0 == i0.refinements + 1
    assert n1 == i1.refinements + 2
    assert rel_l2(x1, x0) <= 1e-9


def test_cg1_heat_refinement_matches_oracle(wfa, oracle_mod):
    prob = inputs.heat_32()
    o = oracle_mod.Oracle(prob)
    To, _ = o.timestep(prob.T0, 3, 1e-12, 1000)
    g = wfa.Grid.from_problem(prob, precision=wfa.F32_IR64)
    g.set_option(wfa.OPT_METHOD, wfa.METHOD_CG1)
    T = g.field(prob.T0)
    infos = g.timestep(T, 3, tol=1e-12, maxit=1000)
    assert all(i.status == wfa.OK and i.refinements >= 2 for i in infos)
    assert rel_l2(to_np(T), To) <= 3 * 14 * 2e-12


EDGE_SHAPES = [(1, 1, 1), (1, 7, 3), (65, 3, 2), (7, 1, 40), (33, 17, 5), (200, 9, 33)]
EDGE_VARIANTS = {
    "cell_mixed": dict(cell=True, bc_kind=inputs.MIXED_BC_KIND),
    "const_zeroflux": dict(cell=False, bc_kind=(ZEROFLUX,) * 6),
}


@pytest.mark.parametrize("shape", EDGE_SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("name", sorted(EDGE_VARIANTS))
def test_cg1_degenerate_and_ragged_grids(wfa, oracle_mod, shape, name):
    """Single cells, single rows and columns, ragged tiles, all faces
    zero-flux: converged solves agree with the oracle's, and on grids with
    more than a few cells the first two iterates do too."""
    prob = inputs.random_problem(330, *shape, **EDGE_VARIANTS[name])
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    xo, io = o.cg1(b, prob.T0, 1e-13, 5000)
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e-13, maxit=5000, method="cg1")
    assert info.status == wfa.OK and io.status == 0
    assert rel_l2(to_np(x), xo) <= 1e-11
    if prob.cells >= 8:
        xk, _ = o.cg1(b, prob.T0, 1e-300, 2)
        sx = _sensitivity(o, b, prob.T0, 2)
        x2, i2 = g.solve(g.field(b), g.field(prob.T0), tol=1e-300, maxit=2, method="cg1",
                         check=False)
        assert i2.iterations == 2
        check(f"cg1 f64 edge {name} {'x'.join(map(str, shape))} k=2 x", rel_l2(to_np(x2), xk),
              trajectory_bound(sx, 3), sx)
