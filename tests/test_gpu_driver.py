"""Host driver of the Krylov solves on the GPU.

The true residual of a plain solve comes back with the chunk of iterations
that ends it: a residual pass is queued behind every chunk and runs only once
the solve has converged or used its iterations.  Here that figure must equal a
separate true-residual computation bit for bit (same pass, same inputs), for
a converged solve, one stopped by its iteration limit and one that converges
at its initial residual.  A profiled grid takes the separate path; its
iterates and reports must be identical.  Torch work after a solve must see
no stale HIP error from the driver's polling.
"""
import numpy as np
import pytest

from paper_2209_13768_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wfa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_13768_amd import wfa as w
    w.lib()
    return w


CASES = [(m, p) for m in ("bicgstab", "bicgstab2", "cg", "cg1") for p in ("f64", "f32")]


def _solve(wfa, prob, prec, method, tol, maxit, profile):
    g = wfa.Grid.from_problem(prob, precision=prec)
    if profile:
        g.set_option(wfa.OPT_PROFILE, 1)
    b = g.rhs(g.field(prob.T0))
    x, info = g.solve(b, g.field(prob.T0), tol=tol, maxit=maxit, method=method, check=False)
    return g, b, x, info


@pytest.mark.parametrize("method,precision", CASES, ids=[f"{m}-{p}" for m, p in CASES])
def test_residual_with_last_chunk_equals_separate_pass(wfa, method, precision):
    import torch
    u = (0.0, 0.0, 0.0) if method.startswith("cg") else (1.0, -0.5, 0.25)
    prob = inputs.random_problem(151, 40, 33, 21, cell=True, u=u, bc_kind=inputs.MIXED_BC_KIND)
    prec = wfa.PRECISIONS[precision]
    tol = 1e-5 if precision == "f32" else 1e-10
    for tol, maxit, status, iters in ((tol, 5000, wfa.OK, None), (1e-300, 7, wfa.ERR_NOCONV, 7),
                                      (10.0, 100, wfa.OK, 0)):
        g, b, x, info = _solve(wfa, prob, prec, method, tol, maxit, False)
        assert info.status == status, (tol, info)
        if iters is not None:
            assert info.iterations == iters
        assert info.rel_res_true == g.true_residual(b, x)
        y = (x * 2).sum()               # torch work right after the solve
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        _, _, xp, ip = _solve(wfa, prob, prec, method, tol, maxit, True)
        assert np.array_equal(xp.cpu().numpy(), x.cpu().numpy())
        assert (ip.status, ip.iterations, ip.restarts) == (info.status, info.iterations, info.restarts)
        assert ip.rel_res_true == info.rel_res_true
        assert ip.rel_res_recursive == info.rel_res_recursive


def test_restarts_and_refinement_unchanged_by_profiling(wfa):
    """A forced breakdown (restart queued without a readback) and FP32-in-FP64
    refinement (outer scalars read back with the inner chunks): identical
    with and without the profiled path."""
    prob = inputs.convdiff(n=36, seed=12)
    out = []
    for profile in (0, 1):
        g = wfa.Grid.from_problem(prob, precision=wfa.F64)
        g.set_option(wfa.OPT_PROFILE, profile)
        g.set_option(wfa.OPT_FORCE_BREAKDOWN, 4)
        b = g.rhs(g.field(prob.T0))
        x, info = g.solve(b, g.field(prob.T0), tol=1e-10, maxit=5000, method="bicgstab2")
        assert info.status == wfa.OK and info.restarts == 1
        gi = wfa.Grid.from_problem(prob, precision=wfa.F32_IR64)
        gi.set_option(wfa.OPT_PROFILE, profile)
        bi = gi.rhs(gi.field(prob.T0))
        xi, ii = gi.solve(bi, gi.field(prob.T0), tol=1e-12, maxit=5000)
        assert ii.status == wfa.OK and ii.refinements >= 2
        assert gi.true_residual(bi, xi) <= 1e-12
        out.append((x.cpu().numpy(), info.iterations, info.rel_res_true, xi.cpu().numpy(),
                    ii.iterations, ii.refinements, ii.rel_res_true))
    for a, c in zip(out[0], out[1]):
        if isinstance(a, np.ndarray):
            assert np.array_equal(a, c)
        else:
            assert a == c


@pytest.mark.parametrize("precision", ["f64", "f32_ir64"])
def test_first_chunk_hint_leaves_results_unchanged(wfa, precision):
    """The first chunk of a solve is sized from the grid's previous solve:
    results on a grid that has solved before (the hint set) must equal, bit
    for bit, those of fresh grids (no hint), for repeated solves and for
    time steps; and a hint far too large or too small changes nothing."""
    prob = inputs.convdiff(n=30, seed=21)
    prec = wfa.PRECISIONS[precision]
    tol = 1e-10

    def fresh_step(T):
        g = wfa.Grid.from_problem(prob, precision=prec)
        g.set_option(wfa.OPT_METHOD, wfa.METHOD_BICGSTAB2)
        return g.timestep(T, 1, tol=tol, maxit=5000)[0]

    warm = wfa.Grid.from_problem(prob, precision=prec)
    warm.set_option(wfa.OPT_METHOD, wfa.METHOD_BICGSTAB2)
    Tw = warm.field(prob.T0)
    Tf = warm.field(prob.T0)
    for step in range(4):
        iw = warm.timestep(Tw, 1, tol=tol, maxit=5000)[0]
        i_f = fresh_step(Tf)
        assert iw.status == wfa.OK and i_f.status == wfa.OK
        assert (iw.iterations, iw.refinements) == (i_f.iterations, i_f.refinements), step
        assert iw.rel_res_true == i_f.rel_res_true
        assert np.array_equal(Tw.cpu().numpy(), Tf.cpu().numpy()), step
    # a solve of a much easier system right after (hint far too large), then
    # the original again (hint far too small)
    b = warm.rhs(warm.field(prob.T0))
    _, ie = warm.solve(b, warm.field(prob.T0), tol=1e-2, maxit=5000, method="bicgstab2")
    x1, i1 = warm.solve(b, warm.field(prob.T0), tol=tol, maxit=5000, method="bicgstab2")
    g2 = wfa.Grid.from_problem(prob, precision=prec)
    x2, i2 = g2.solve(b, g2.field(prob.T0), tol=tol, maxit=5000, method="bicgstab2")
    assert ie.status == wfa.OK and ie.iterations < i1.iterations
    assert (i1.iterations, i1.rel_res_true) == (i2.iterations, i2.rel_res_true)
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())


def test_sampled_launch_timing(wfa):
    """WFA_OPT_PROFILE = n times the first and then every n-th launch of each
    kernel: a fixed-length solve times ceil(launches / n) of each kernel's
    launches, and the iterates do not depend on the timing."""
    prob = inputs.random_problem(152, 70, 20, 33, cell=True, u=(0.5, 0.0, -1.0))
    counts, xs = {}, {}
    for n in (1, 3, 8):
        g = wfa.Grid.from_problem(prob, precision=wfa.F64)
        g.set_option(wfa.OPT_PROFILE, n)
        b = g.rhs(g.field(prob.T0))
        x, info = g.solve(b, g.field(prob.T0), tol=1e-300, maxit=25, method="bicgstab2",
                          check=False)
        assert info.iterations == 25
        counts[n] = [g.kernel_stats(k)[0] for k in range(wfa.K_COUNT)]
        xs[n] = x.cpu().numpy()
        ms = [g.kernel_stats(k)[1] for k in range(wfa.K_COUNT)]
        assert all(m > 0 for c, m in zip(counts[n], ms) if c > 0)
    assert counts[1][wfa.K_PHASE_AC] >= 25 and counts[1][wfa.K_PHASE_B2] >= 25
    for n in (3, 8):
        assert counts[n] == [-(-c // n) for c in counts[1]], (n, counts[n], counts[1])
        assert np.array_equal(xs[n], xs[1])
