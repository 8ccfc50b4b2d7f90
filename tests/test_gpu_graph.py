"""GPU tests of the graph option of feast_solve: loop 1 runs eagerly, then
one loop (B*Y, the sweeps of all nodes, Q, the projection, the reduced
problem, X = Q Phi, the residuals, Y <- X) is captured as a HIP graph and
launched for every later loop, with the host reading the convergence data
between launches.  The graph runs the same kernels on the same data in the
same order as the eager loop, so every output must be bitwise equal to the
eager solve, which the oracle pins (here and in the parity tests)."""
import numpy as np
import pytest

from oracle import feast_oracle as O
from paper_0901_2665_amd import workloads as W
from test_gpu_parity import check_against_oracle, dev, gpencil, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a HIP device"
    return _t


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_0901_2665_amd import feast as F
    c = F.Context(0)
    yield c
    c.close()


def same(a, b):
    assert (a.status, a.M, a.loops, a.rr_sweeps, a.fallback) == \
        (b.status, b.M, b.loops, b.rr_sweeps, b.fallback)
    assert a.traces == b.traces and a.counts == b.counts
    for x, y in ((a.lam, b.lam), (a.X, b.X), (a.res, b.res)):
        assert np.array_equal(host(x), host(y), equal_nan=True)  # NaN: dropped slots


def test_graph_equals_eager(ctx, torch):
    p, emin, emax, m0, ne, Y0 = W.make_workload("chain800")
    gp, y = gpencil(p), dev(torch, Y0)
    eager = ctx.solve(gp, emin, emax, m0, ne, y)
    g = ctx.solve(gp, emin, emax, m0, ne, y, graph=1)
    assert eager.status == 0 and eager.loops >= 3  # the graph launched twice at least
    same(g, eager)
    check_against_oracle(g, O.feast(p, emin, emax, m0, ne, Y0), p, emin, emax)


def test_graph_replays(ctx, torch):
    # tol = 1e-20: the residual gate (sqrt(tol) = 1e-10) still counts the
    # converged pairs, but the trace test passes only on equal traces, so
    # the loop goes on and the graph is launched for loops 2, 3, ..., each
    # launch checked through the final outputs and the per-loop trace
    # history; then a second graph solve in the same context and an eager
    # one again
    p = W.dense_random_pencil(7, 16, 6)
    lam = O.bruteforce(p)[0]
    emin, emax = 0.5 * (lam[29] + lam[30]), 0.5 * (lam[39] + lam[40])
    Y0 = dev(torch, W.random_subspace(p.n, 18, 106))
    gp = gpencil(p)
    kw = dict(tol=1e-20, max_loops=7)
    eager = ctx.solve(gp, emin, emax, 18, 8, Y0, **kw)
    assert eager.loops >= 3 and eager.M == 10
    for graph in (1, 1, 0):
        same(ctx.solve(gp, emin, emax, 18, 8, Y0, graph=graph, **kw), eager)


def test_graph_batched(ctx, torch):
    # the batched call passes the option to every problem (each worker
    # captures on its own stream)
    probs = []
    for seed, (nc, b, k0, m) in enumerate([(6, 8, 10, 12), (11, 20, 60, 15), (4, 5, 5, 6)]):
        p = W.dense_random_pencil(nc, b, seed + 1)
        lam = O.bruteforce(p)[0]
        emin, emax = 0.5 * (lam[k0 - 1] + lam[k0]), 0.5 * (lam[k0 + m - 1] + lam[k0 + m])
        m0 = min(m + 6, p.n)
        probs.append((gpencil(p), emin, emax, m0, 8,
                      dev(torch, W.random_subspace(p.n, m0, seed + 50))))
    st, rs = ctx.solve_batched(probs, tol=1e-13, max_loops=40, workers=3, graph=1)
    assert st in (0, 2)
    for pr, r in zip(probs, rs):
        same(r, ctx.solve(*pr, tol=1e-13, max_loops=40, partitions=1))  # batched: 0 reads as 1


def test_graph_bad_option(ctx, torch):
    from paper_0901_2665_amd import feast as F
    p = W.dense_random_pencil(3, 8, 9)
    Y0 = dev(torch, W.random_subspace(p.n, 4, 3))
    with pytest.raises(F.FeastError) as e:
        ctx.solve(gpencil(p), 0.0, 1.0, 4, 8, Y0, graph=3)
    assert e.value.status == -7
    with pytest.raises(F.FeastError) as e:   # graph 2 keeps a history of 64 loops
        ctx.solve(gpencil(p), 0.0, 1.0, 4, 8, Y0, graph=2, max_loops=65)
    assert e.value.status == -7


# graph = 2: the convergence decision on the device, the loops captured four
# at a time with kernels that return at once after convergence; same
# kernels, same data, same order and the same decisions as the eager loop,
# so every output must be bitwise equal to it
def test_device_graph_equals_eager(ctx, torch):
    p, emin, emax, m0, ne, Y0 = W.make_workload("chain800")
    gp, y = gpencil(p), dev(torch, Y0)
    eager = ctx.solve(gp, emin, emax, m0, ne, y)
    g = ctx.solve(gp, emin, emax, m0, ne, y, graph=2)
    same(g, eager)
    assert g.trace_rel == eager.trace_rel
    check_against_oracle(g, O.feast(p, emin, emax, m0, ne, Y0), p, emin, emax)


@pytest.mark.parametrize("max_loops", [3, 4, 5, 9])
def test_device_graph_chunks(ctx, torch, max_loops):
    # tol = 1e-20: the trace test passes only on equal traces, here in loop 5;
    # below that the solve stops at max_loops (status 1) inside or at the end
    # of the first graph launch, else it converges in the second launch; the
    # final Ritz vectors come from y or x by the parity of the loop count
    p = W.dense_random_pencil(7, 16, 6)
    lam = O.bruteforce(p)[0]
    emin, emax = 0.5 * (lam[29] + lam[30]), 0.5 * (lam[39] + lam[40])
    Y0 = dev(torch, W.random_subspace(p.n, 18, 106))
    gp = gpencil(p)
    kw = dict(tol=1e-20, max_loops=max_loops)
    eager = ctx.solve(gp, emin, emax, 18, 8, Y0, **kw)
    assert eager.loops == min(max_loops, 5)
    assert eager.status == (1 if max_loops < 5 else 0)
    same(ctx.solve(gp, emin, emax, 18, 8, Y0, graph=2, **kw), eager)


def test_device_graph_batched_and_tb6400(ctx, torch):
    probs = []
    for seed, (nc, b, k0, m) in enumerate([(6, 8, 10, 12), (11, 20, 60, 15), (4, 5, 5, 6)]):
        p = W.dense_random_pencil(nc, b, seed + 1)
        lam = O.bruteforce(p)[0]
        emin, emax = 0.5 * (lam[k0 - 1] + lam[k0]), 0.5 * (lam[k0 + m - 1] + lam[k0 + m])
        m0 = min(m + 6, p.n)
        probs.append((gpencil(p), emin, emax, m0, 8,
                      dev(torch, W.random_subspace(p.n, m0, seed + 50))))
    st, rs = ctx.solve_batched(probs, tol=1e-13, max_loops=40, workers=3, graph=2)
    assert st in (0, 2)
    for pr, r in zip(probs, rs):
        same(r, ctx.solve(*pr, tol=1e-13, max_loops=40, partitions=1))
    p, emin, emax, m0, ne, Y0 = W.make_workload("tb6400")
    gp, y = gpencil(p), dev(torch, Y0)
    same(ctx.solve(gp, emin, emax, m0, ne, y, graph=2), ctx.solve(gp, emin, emax, m0, ne, y))


def test_device_graph_wide_blocks(ctx, torch):
    # 64 < b <= 96: the wide kernels take the same flag
    p = W.dense_random_pencil(6, 96, 81)
    lam = O.bruteforce(p)[0]
    emin, emax = 0.5 * (lam[149] + lam[150]), 0.5 * (lam[169] + lam[170])
    Y0 = dev(torch, W.random_subspace(p.n, 40, 181))
    gp = gpencil(p)
    eager = ctx.solve(gp, emin, emax, 40, 8, Y0, tol=1e-13, max_loops=40)
    assert eager.M == 20
    for graph in (1, 2):
        same(ctx.solve(gp, emin, emax, 40, 8, Y0, tol=1e-13, max_loops=40, graph=graph), eager)
