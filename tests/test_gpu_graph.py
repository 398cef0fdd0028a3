"""Graph replay of iteration chunks against plain launches.

A chunk of iterations between host checks can be replayed from a captured
HIP graph; the kernels and their arguments are those of the plain launches,
so every result must be bitwise identical.  Each graph is replayed many
times, with other device work and synchronisations in between, and every
replay's result is checked against plain launches.
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


def _solve(wfa, prob, precision, graph, method, check_every=0, tol=1e-10, maxit=2000, ry=0):
    g = wfa.Grid.from_problem(prob, precision=precision)
    g.set_option(wfa.OPT_GRAPH, graph)
    if method == "bicgstab2_hashed":
        method = "bicgstab2"
        g.set_option(wfa.OPT_SHADOW, 1)
    g.set_option(wfa.OPT_CHECK_EVERY, check_every)
    if ry:
        g.set_option(wfa.OPT_RY, ry)
    b = g.rhs(g.field(prob.T0))
    x, info = g.solve(b, g.field(prob.T0), tol=tol, maxit=maxit, method=method)
    return x.cpu().numpy(), info


CASES = [
    ("bicgstab", "f64"), ("bicgstab", "f32"), ("bicgstab", "f32_ir64"),
    ("bicgstab2", "f64"), ("bicgstab2", "f32"), ("bicgstab2_hashed", "f64"),
    ("bicgstab2_hashed", "f32_ir64"), ("cg", "f64"), ("cg", "f32"), ("cg1", "f64"), ("cg1", "f32"),
]


@pytest.mark.parametrize("check_every", [0, 13, 64])
@pytest.mark.parametrize("method,precision", CASES, ids=[f"{m}-{p}" for m, p in CASES])
def test_graph_replay_is_bitwise_identical(wfa, method, precision, check_every):
    u = (0.0, 0.0, 0.0) if method.startswith("cg") else (1.0, -0.5, 0.25)
    prob = inputs.random_problem(121, 45, 30, 21, cell=True, u=u, bc_kind=inputs.MIXED_BC_KIND)
    tol = 1e-5 if precision == "f32" else 1e-10
    prec = wfa.PRECISIONS[precision]
    xs, infos = [], []
    for graph in (0, 1):
        x, info = _solve(wfa, prob, prec, graph, method, check_every, tol=tol)
        assert info.status == wfa.OK, info
        xs.append(x)
        infos.append(info)
    assert infos[0].iterations == infos[1].iterations
    assert infos[0].refinements == infos[1].refinements
    assert np.array_equal(xs[0], xs[1])


def test_graph_replays_with_other_work_between(wfa):
    """One grid, graphs on: solves with fresh x tensors (new addresses), the
    same x tensor reused, other device work and synchronisations between,
    and an option change that re-tiles the grid; each result must equal the
    plain-launch result for the same inputs."""
    import torch
    prob = inputs.random_problem(122, 50, 24, 19, cell=True, u=(2.0, 1.0, -1.0),
                                 bc_kind=inputs.MIXED_BC_KIND)
    ref = {}
    for ry in (2, 1):
        ref[ry], _ = _solve(wfa, prob, wfa.F64, 0, "bicgstab2", 16, ry=ry)
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    g.set_option(wfa.OPT_GRAPH, 1)
    g.set_option(wfa.OPT_CHECK_EVERY, 16)
    b = g.rhs(g.field(prob.T0))
    keep = g.field(prob.T0)
    junk = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(6):
        ry = 1 if rep >= 4 else 2
        if rep == 4:
            g.set_option(wfa.OPT_RY, 1)
        if rep % 2:
            x = keep
            x.copy_(g.field(prob.T0))
        else:
            x = g.field(prob.T0)
        junk.add_(1.0)  # unrelated eager work on the same stream
        torch.cuda.synchronize()
        x, info = g.solve(b, x, tol=1e-10, maxit=2000, method="bicgstab2")
        assert info.status == wfa.OK
        assert np.array_equal(x.cpu().numpy(), ref[ry]), f"replay {rep} differs"
    assert float(junk[0]) == 6.0
