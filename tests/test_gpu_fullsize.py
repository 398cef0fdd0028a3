"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (default tiling, two-reduction BiCGStab with the hashed
shadow residual where the benchmark uses it).

* 256^3 convection-diffusion (log-normal diffusivity, upwind, mixed faces):
  the whole operator and right-hand side in FP64 and FP32, the first
  iterates against the oracle's same variant, and one backward-Euler step
  whose result the oracle's operator must see at the benchmark's tolerance.
* 512x512x1024 smooth-diffusivity diffusion in FP32: the whole operator, the
  first iterate, two iterations of the one-reduction CG, and the sixth
  iterate of the benchmarked solve against the FP64 oracle.
* 384^3 convection-diffusion (velocity x4): FP32 inside FP64 refinement to
  1e-12, judged by the oracle's FP64 operator.
* The serving stream's first requests (their real grid sizes), batched
  together: each result meets 1e-10 under the oracle's operator, and equals
  the same request served alone, bit for bit.

Where BiCGStab amplifies rounding, an iterate is held to the trajectory bar
of tests/parity_bars.py: 15 sqrt(m) times the oracle's own change under a
one-ulp perturbation of b (m operator applications), floored at the FP64
bar (the FP32 bar and a one-FP32-ulp perturbation for FP32 iterates).
"""
import numpy as np
import pytest

from paper_2209_13768_amd import inputs
from tests.oracle_helpers import rel_l2
from tests.parity_bars import check, sensitivity, trajectory_bound

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def wfa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_13768_amd import wfa as w
    w.lib()
    return w


def _np(t):
    return t.detach().cpu().double().numpy()


@pytest.fixture(scope="module")
def convdiff256():
    return inputs.convdiff(n=256)


def _sensitivity(o, b, x0, k):
    """How far the oracle's own k-th iterate moves when b (and x0) is
    perturbed by one ulp in a random direction."""
    return sensitivity(lambda bb, xx: o.bicgstab2(bb, xx, 1e-300, k, hashed_shadow=True)[0],
                       b, x0, seeds=(0,))


def test_convdiff256_operator(wfa, oracle_mod, convdiff256):
    prob = convdiff256
    o = oracle_mod.Oracle(prob)
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    x = g.field(prob.T0)
    assert rel_l2(_np(g.apply(x)), o.apply(prob.T0)) <= FP64_TOL
    assert rel_l2(_np(g.rhs(x)), o.rhs(prob.T0)) <= FP64_TOL
    g32 = wfa.Grid.from_problem(prob, precision=wfa.F32)
    x32 = g32.field(prob.T0)
    x32n = _np(x32)
    assert rel_l2(_np(g32.apply(x32)), o.apply(x32n)) <= FP32_TOL
    assert rel_l2(_np(g32.rhs(x32)), o.rhs(x32n)) <= FP32_TOL


@pytest.mark.parametrize("k", [1, 2])
def test_convdiff256_first_iterates(wfa, oracle_mod, convdiff256, k):
    prob = convdiff256
    o = oracle_mod.Oracle(prob)
    b = o.rhs(prob.T0)
    xo, io = o.bicgstab2(b, prob.T0, 1e-300, k, hashed_shadow=True)
    sx = _sensitivity(o, b, prob.T0, k)
    bound = trajectory_bound(sx, 2 * k)
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    g.set_option(wfa.OPT_SHADOW, 1)
    x, info = g.solve(g.field(b), g.field(prob.T0), tol=1e-300, maxit=k, method="bicgstab2",
                      check=False)
    assert info.status == wfa.ERR_NOCONV and info.iterations == k == io.iterations
    check(f"convdiff256 hashed bicgstab2 f64 k={k} x", rel_l2(_np(x), xo), bound, sx)
    g32 = wfa.Grid.from_problem(prob, precision=wfa.F32)
    g32.set_option(wfa.OPT_SHADOW, 1)
    x32, _ = g32.solve(g32.field(b), g32.field(prob.T0), tol=1e-300, maxit=k,
                       method="bicgstab2", check=False)
    assert rel_l2(_np(x32), xo) <= FP32_TOL


def test_convdiff256_timestep_as_benchmarked(wfa, oracle_mod, convdiff256):
    """The benchmark's first step: tolerance 1e-8, two-reduction BiCGStab,
    hashed shadow residual, default tiling.  The condition number is ~1e5,
    so the iterate is judged by the oracle's own FP64 residual."""
    prob = convdiff256
    o = oracle_mod.Oracle(prob)
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    g.set_option(wfa.OPT_METHOD, wfa.METHOD_BICGSTAB2)
    g.set_option(wfa.OPT_SHADOW, 1)
    T = g.field(prob.T0)
    info = g.timestep(T, 1, tol=1e-8, maxit=5000)[0]
    assert info.status == wfa.OK and info.iterations > 100
    rel = o.true_relres(o.rhs(prob.T0), _np(T))
    assert rel <= 1e-8
    # the library's own FP64 true residual agrees with the oracle's
    assert abs(info.rel_res_true - rel) <= 1e-3 * rel


def test_poisson_512x512x1024_operator_and_first_iterate(wfa, oracle_mod):
    prob = inputs.poisson_large()
    o = oracle_mod.Oracle(prob)
    g = wfa.Grid.from_problem(prob, precision=wfa.F32)
    x = g.field(prob.T0)
    xn = _np(x)
    assert rel_l2(_np(g.apply(x)), o.apply(xn)) <= FP32_TOL
    b = o.rhs(xn)
    xo, _ = o.bicgstab2(b, np.zeros_like(b), 1e-300, 1, hashed_shadow=True)
    g.set_option(wfa.OPT_SHADOW, 1)
    x1, info = g.solve(g.field(b), g.field(), tol=1e-300, maxit=1, method="bicgstab2",
                       check=False)
    assert info.iterations == 1
    assert rel_l2(_np(x1), xo) <= FP32_TOL
    # the symmetric workload's one-reduction CG: two iterations (the second
    # pass is the first with the fused update)
    xc, _ = o.cg1(b, np.zeros_like(b), 1e-300, 2)
    x2, info = g.solve(g.field(b), g.field(), tol=1e-300, maxit=2, method="cg1", check=False)
    assert info.iterations == 2
    assert rel_l2(_np(x2), xc) <= FP32_TOL


def test_poisson_512x512x1024_fp32_trajectory(wfa, oracle_mod):
    """The headline solve's first iterates beyond the first: FP32 on the GPU
    against the FP64 oracle's same method (two-reduction, hashed shadow),
    from the benchmark's x0 = T0.  FP32 arithmetic rounds every operator
    application and every stored vector at 2^-24, and the iteration
    amplifies it; the bar is the FP64 one's derivation (tests/parity_bars.py)
    with a one-FP32-ulp perturbation of b and x0 in place of a one-FP64-ulp
    one: 15 sqrt(m + 1) times the oracle's own change under it (m operator
    applications, one more for the rounding of b and x0 to FP32), floored
    at the FP32 bar."""
    k = 6
    prob = inputs.poisson_large()
    o = oracle_mod.Oracle(prob)
    x0 = prob.T0.astype(np.float32).astype(np.float64)
    b = o.rhs(prob.T0)
    run = lambda bb, xx: o.bicgstab2(bb, xx, 1e-300, k, hashed_shadow=True)[0]
    xo = run(b, x0)
    s32 = sensitivity(run, b, x0, eps=2.0 ** -23, seeds=(0,))
    g = wfa.Grid.from_problem(prob, precision=wfa.F32)
    g.set_option(wfa.OPT_SHADOW, 1)
    xk, info = g.solve(g.field(b), g.field(x0), tol=1e-300, maxit=k, method="bicgstab2",
                       check=False)
    assert info.iterations == k
    bound = trajectory_bound(s32, 2 * k + 1, floor=FP32_TOL)
    check(f"poisson512x512x1024 fp32 k={k}", rel_l2(_np(xk), xo), bound, s32)


def test_mixed_precision_384_reaches_1e12(wfa, oracle_mod):
    prob = inputs.convdiff_384()
    o = oracle_mod.Oracle(prob)
    g = wfa.Grid.from_problem(prob, precision=wfa.F32_IR64)
    g.set_option(wfa.OPT_METHOD, wfa.METHOD_BICGSTAB2)
    T = g.field(prob.T0)
    info = g.timestep(T, 1, tol=1e-12, maxit=100000)[0]
    assert info.status == wfa.OK and info.refinements >= 2
    assert o.true_relres(o.rhs(prob.T0), _np(T)) <= 1e-12


def test_serving_stream_head(wfa, oracle_mod):
    """The benchmark's request stream, its first 24 requests at their real
    sizes, submitted together into a server with the benchmark's budget and
    slot count."""
    import torch
    reqs = inputs.request_stream()[:24]

    def serve(batch):
        sv = wfa.Server(64 << 30, max_slots=64)
        outs, tickets = [], []
        for rq in batch:
            prob = rq.problem()
            T = torch.from_numpy(prob.T0).to("cuda", torch.float64)
            tickets.append(sv.submit_problem(prob, T, precision=wfa.F32_IR64, tol=1e-10,
                                             maxit=20000))
            outs.append(T)
        sv.drain()
        infos = [sv.poll(t) for t in tickets]
        sv.close()
        return [_np(t) for t in outs], infos

    mix, infos = serve(reqs)
    for rq, T, (code, info) in zip(reqs, mix, infos):
        assert code == wfa.OK, (rq, code)
        prob = rq.problem()
        o = oracle_mod.Oracle(prob)
        assert o.true_relres(o.rhs(prob.T0), T) <= 1e-10, rq
    for q in (0, 7, 23):
        alone, _ = serve([reqs[q]])
        assert np.array_equal(alone[0], mix[q]), reqs[q]
