"""GPU parity: every step of the HIP path against the CPU oracle.

All calls go through the C ABI (paper_0901_2665_amd.feast -> libfeast.so).
Tolerances: float64 throughout; a step that is a plain product or sum is
held to a few units of rounding times the problem scale; the shifted solves
to their conditioning; FEAST outputs to the contract (same M, eigenvalues
within 1e-10 relative, residuals <= 1e-9).
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import feast_oracle as O
from paper_0901_2665_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


def dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def gpencil(p):
    from paper_0901_2665_amd import feast as F
    return F.Pencil(p.Ad, p.Au, p.Bd, p.Bu)


U64 = np.finfo(np.float64).eps / 2   # unit roundoff of float64


def assert_columnwise(out, ref, rel):
    """Element by element: every entry within rel times the largest entry of
    its own reference column (so a few wrong rows of a tall result fail)."""
    out = np.asarray(out)
    ref = np.asarray(ref)
    assert out.shape == ref.shape
    scale = np.max(np.abs(ref), axis=0, keepdims=True)
    err = np.abs(out - ref)
    bad = err > rel * scale
    assert not np.any(bad), (f"{int(bad.sum())} entries off; worst "
                             f"{float(np.max(err / np.maximum(scale, 1e-300))):.3e} of the column max")


def chain_small(nc, b, seed):
    if b == 64:
        return W.chain_pencil(nc, b, seed)
    return W.dense_random_pencil(nc, b, seed)


SHAPES = [(1, 5, 3), (2, 16, 16), (3, 17, 30), (20, 40, 30), (7, 64, 128), (5, 33, 100),
          (9, 48, 8), (4, 64, 1), (40, 16, 8), (67, 32, 20)]


@pytest.mark.parametrize("nc,b,m", SHAPES)
def test_bt_multiply(ctx, torch, nc, b, m):
    p = chain_small(nc, b, 100 + nc)
    V = np.random.default_rng(nc * b).standard_normal((p.n, m))
    gp = gpencil(p)
    for which, (d, u) in enumerate([(p.Ad, p.Au), (p.Bd, p.Bu)]):
        out = host(ctx.bt_multiply(gp, which, dev(torch, V)))
        ref = O.bt_multiply(d, u, V)
        # componentwise bound of a sum of 3b products, every entry
        bound = 2 * (3 * b) * U64 * O.bt_multiply(np.abs(d), np.abs(u), np.abs(V))
        assert np.all(np.abs(out - ref) <= bound + 1e-300)


@pytest.mark.parametrize("nc,b,m", SHAPES)
def test_shifted_solve(ctx, torch, nc, b, m):
    p = chain_small(nc, b, 200 + nc)
    R = np.random.default_rng(7 * nc + b).standard_normal((p.n, m))
    z = 0.37 + 0.05j
    xr, xi = ctx.shifted_solve(gpencil(p), z, dev(torch, R))
    X = host(xr) + 1j * host(xi)
    ref = O.shifted_solve(p, z, R)
    M = O.shifted_matrix(p, z)
    berr = np.linalg.norm(R - M @ X, axis=0) / (spla.norm(M) * np.linalg.norm(X, axis=0))
    assert np.max(berr) <= 1e-14
    assert_columnwise(X, ref, 1e-10)


# 64 < b <= 96: the wide kernels (one top-down chain per shift, blocks padded
# to 96), single and padded blocks, up to 128 right-hand sides
WIDE_SHAPES = [(1, 96, 8), (2, 65, 3), (5, 80, 24), (12, 96, 40), (3, 96, 128), (40, 70, 16)]


@pytest.mark.parametrize("nc,b,m", WIDE_SHAPES)
def test_shifted_solve_wide_blocks(ctx, torch, nc, b, m):
    p = W.dense_random_pencil(nc, b, 300 + nc + b)
    R = np.random.default_rng(11 * nc + b).standard_normal((p.n, m))
    z = 0.37 + 0.05j
    xr, xi = ctx.shifted_solve(gpencil(p), z, dev(torch, R))
    X = host(xr) + 1j * host(xi)
    ref = O.shifted_solve(p, z, R)
    M = O.shifted_matrix(p, z)
    berr = np.linalg.norm(R - M @ X, axis=0) / (spla.norm(M) * np.linalg.norm(X, axis=0))
    assert np.max(berr) <= 1e-14
    assert_columnwise(X, ref, 1e-10)


@pytest.mark.parametrize("eta", [5e-2, 1e-3, 1e-4])
def test_shifted_solve_wide_near_axis(ctx, torch, eta):
    # the benchmark chain recipe at b = 96, shifts inside the spectrum
    p = W.chain_pencil(60, 96, 4243)
    B = O.assemble(p.Bd, p.Bu)
    bmin = spla.eigsh(B, k=1, which="SA", return_eigenvectors=False)[0]
    z = 0.1234 + 1j * eta
    R = np.random.default_rng(19).standard_normal((p.n, 24))
    xr, xi = ctx.shifted_solve(gpencil(p), z, dev(torch, R))
    X = host(xr) + 1j * host(xi)
    M = O.shifted_matrix(p, z)
    berr = np.linalg.norm(R - M @ X, axis=0) / (spla.norm(M) * np.linalg.norm(X, axis=0))
    print(f"wide near axis: Im z {eta:g}  backward error {np.max(berr):.2e}")
    bar = WIDE_NEAR_AXIS_BAR[eta]
    assert np.max(berr) <= bar
    ref = O.shifted_solve(p, z, R)
    cond = spla.norm(M) / (eta * bmin)
    assert_columnwise(X, ref, max(1e-12, 10 * bar * cond))


# measured: 6.1e-17, 3.4e-15, 5.7e-14 (one chain, no partitions)
WIDE_NEAR_AXIS_BAR = {5e-2: 1e-15, 1e-3: 2e-14, 1e-4: 3e-13}


def near_axis_chain():
    """A chain of the benchmark recipe long enough for several partitions
    of the factorisation (nc = 160, b = 32: 10 per half chain)."""
    return W.chain_pencil(160, 32, 4242)


# Backward-error bars of one shifted solve near the real axis, from the
# measured values (one partition / automatic, here 10 per half chain):
#   Im z = 5e-2: 1.5e-16 / 1.2e-16;  1e-3: 2.7e-14 / 1.1e-12;  1e-4: 8.1e-14 / 4.6e-12.
# The unpivoted inversion of blocks whose smallest singular value is of the
# order of Im z costs up to three digits against LAPACK's pivoted banded LU
# (about 1e-16 here), and the interface step of the partitioned factorisation
# up to two more.
NEAR_AXIS_BAR = {(5e-2, 1): 1e-15, (5e-2, 0): 1e-15, (1e-3, 1): 2e-13, (1e-3, 0): 1e-11,
                 (1e-4, 1): 5e-13, (1e-4, 0): 3e-11}


@pytest.mark.parametrize("parts", [1, 0])
@pytest.mark.parametrize("eta", [5e-2, 1e-3, 1e-4])
def test_shifted_solve_near_axis(ctx, torch, eta, parts):
    # contour points next to the real axis (Ne = 16 puts its outermost pair at
    # Im Z = 0.017 r, with r down to a few 1e-3 on the batch problems): the
    # shift's real part sits inside the dense part of the spectrum
    p = near_axis_chain()
    B = O.assemble(p.Bd, p.Bu)
    bmin = spla.eigsh(B, k=1, which="SA", return_eigenvectors=False)[0]
    z = 0.1234 + 1j * eta   # inside the spectrum (about [-7, 7] for this recipe)
    R = np.random.default_rng(17).standard_normal((p.n, 24))
    xr, xi = ctx.shifted_solve(gpencil(p), z, dev(torch, R), partitions=parts)
    X = host(xr) + 1j * host(xi)
    M = O.shifted_matrix(p, z)
    berr = np.linalg.norm(R - M @ X, axis=0) / (spla.norm(M) * np.linalg.norm(X, axis=0))
    bar = NEAR_AXIS_BAR[(eta, parts)]
    assert np.max(berr) <= bar
    ref = O.shifted_solve(p, z, R)
    # forward error: at most the backward error times the condition number
    # (||M^-1|| <= 1 / (Im z lambda_min(B)))
    cond = spla.norm(M) / (eta * bmin)
    assert_columnwise(X, ref, max(1e-12, 10 * bar * cond))


@pytest.mark.parametrize("name_or_shape", ["chain800", (9, 16, 24, 4), (3, 3, 5, 16),
                                           (13, 64, 40, 8)])
def test_filter(ctx, torch, name_or_shape):
    if isinstance(name_or_shape, str):
        p, emin, emax, m0, ne, Y = W.make_workload(name_or_shape)
    else:
        nc, b, m0, ne = name_or_shape
        p = chain_small(nc, b, 300 + nc)
        lam = O.bruteforce(p)[0]
        k0 = p.n // 3
        emin, emax = 0.5 * (lam[k0 - 1] + lam[k0]), 0.5 * (lam[k0 + 3] + lam[k0 + 4])
        Y = W.random_subspace(p.n, m0, nc)
    Q = host(ctx.filter(gpencil(p), emin, emax, ne, dev(torch, Y)))
    ref = O.filter_apply(p, emin, emax, ne, Y)
    assert_columnwise(Q, ref, 1e-11)


@pytest.mark.parametrize("nc,b,m0", [(20, 40, 30), (6, 64, 128), (3, 7, 5)])
def test_project(ctx, torch, nc, b, m0):
    p = chain_small(nc, b, 400 + nc)
    Q = np.random.default_rng(nc).standard_normal((p.n, m0))
    AQ, BQ = ctx.project(gpencil(p), dev(torch, Q))
    ra, rb = O.project(p, Q)
    # componentwise bound of Q^T (T Q): sums of N (3b)-term products
    aQ = np.abs(Q)
    for out, ref, (d, u) in [(AQ, ra, (p.Ad, p.Au)), (BQ, rb, (p.Bd, p.Bu))]:
        bound = 2 * (3 * b + p.n) * U64 * (aQ.T @ O.bt_multiply(np.abs(d), np.abs(u), aQ))
        assert np.all(np.abs(host(out) - ref) <= bound)
    assert np.array_equal(host(AQ), host(AQ).T)


def spd_pair(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    mu = np.geomspace(1.0, 1.0 / cond, n)
    BQ = (Qm * mu) @ Qm.T
    AQ = rng.standard_normal((n, n))
    return 0.5 * (AQ + AQ.T), 0.5 * (BQ + BQ.T)


def feast_like_pair(n, seed, smallest=1e-6):
    """Reduced matrices as FEAST produces them near convergence: Q ~ X D with
    a filter-like scaling D, so B_Q ~ D^2 is ill conditioned while the pencil
    keeps well separated, well conditioned eigenvalues."""
    rng = np.random.default_rng(seed)
    lam = np.sort(rng.uniform(-3, 3, n))
    d = np.geomspace(1.0, smallest, n)
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    G = Qm * d                       # columns scaled
    E = 1e-3 * rng.standard_normal((n, n))
    G = (np.eye(n) + E) @ G
    AQ = G.T @ np.diag(lam) @ G
    BQ = G.T @ G
    return 0.5 * (AQ + AQ.T), 0.5 * (BQ + BQ.T), lam


def rr_backward_error(AQ, BQ, eps, Phi):
    r = AQ @ Phi - (BQ @ Phi) * eps
    den = (np.linalg.norm(AQ, 2) + np.abs(eps) * np.linalg.norm(BQ, 2)) * \
        np.linalg.norm(Phi, axis=0)
    return np.max(np.linalg.norm(r, axis=0) / den)


@pytest.mark.parametrize("n,cond", [(1, 1.0), (7, 10.0), (17, 10.0), (30, 1e2), (33, 1e2), (64, 1e3),
                                    (100, 1e3), (128, 1e3)])
def test_reduced_eig_well_conditioned(ctx, torch, n, cond):
    AQ, BQ = spd_pair(n, n, cond)
    eps, Phi, fb = ctx.reduced_eig(dev(torch, AQ), dev(torch, BQ))
    eps, Phi = host(eps), host(Phi)
    ref, _, rfb = O.reduced_eig(AQ, BQ)
    assert not fb and not rfb
    assert np.max(np.abs(eps - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(Phi.T @ BQ @ Phi - np.eye(n))) <= 1e-12
    assert rr_backward_error(AQ, BQ, eps, Phi) <= 1e-14
    assert np.all(np.diff(eps) >= 0)


@pytest.mark.parametrize("n,smallest", [(30, 1e-5), (80, 1e-6), (128, 1e-7)])
def test_reduced_eig_feast_like(ctx, torch, n, smallest):
    AQ, BQ, lam = feast_like_pair(n, n + 1, smallest)
    eps, Phi, fb = ctx.reduced_eig(dev(torch, AQ), dev(torch, BQ))
    eps, Phi = host(eps), host(Phi)
    ref, _, rfb = O.reduced_eig(AQ, BQ)
    assert not fb and not rfb
    assert np.max(np.abs(eps - ref)) <= 1e-11 * np.max(np.abs(ref))
    assert np.max(np.abs(Phi.T @ BQ @ Phi - np.eye(n))) <= 1e-9


@pytest.mark.parametrize("n,cond", [(30, 1e6), (127, 1e8), (128, 1e10)])
def test_reduced_eig_ill_conditioned_backward_stable(ctx, torch, n, cond):
    # with cond(B_Q) large, a Cholesky-based reduction has a backward error
    # growing with cond(B_Q) (so does LAPACK's): hold the GPU to the oracle's
    # own backward error, and the eigenvalues to eps * cond(B_Q).
    AQ, BQ = spd_pair(n, n, cond)
    eps, Phi, fb = ctx.reduced_eig(dev(torch, AQ), dev(torch, BQ))
    eps, Phi = host(eps), host(Phi)
    ref, rPhi, _ = O.reduced_eig(AQ, BQ)
    assert not fb
    assert rr_backward_error(AQ, BQ, eps, Phi) <= 10 * rr_backward_error(AQ, BQ, ref, rPhi) + 1e-15
    assert np.max(np.abs(eps - ref)) <= 1e-15 * cond * np.max(np.abs(ref))


def test_reduced_eig_scaled_columns_keep_cholesky(ctx, torch):
    # a diagonal B_Q down to 1e-14: the pivot test is scale-invariant, so
    # no fallback, as in the oracle
    mu = np.geomspace(1.0, 1e-14, 9)
    BQ = np.diag(mu)
    AQ = np.diag(np.arange(1.0, 10.0)) * mu
    eps, Phi, fb = ctx.reduced_eig(dev(torch, AQ), dev(torch, BQ))
    ref, _, rfb = O.reduced_eig(AQ, BQ)
    assert not fb and not rfb
    assert np.allclose(host(eps), np.arange(1.0, 10.0), rtol=1e-12)


@pytest.mark.parametrize("d2,fallback", [(1e-14, True), (1e-13, True), (1e-11, False)])
def test_reduced_eig_pivot_cut(ctx, torch, d2, fallback):
    # B_Q = Q^T Q with Q = [e1, e1 + d e2, e3]: relative pivot d^2 / (1 + d^2)
    BQ = np.array([[1.0, 1.0, 0.0], [1.0, 1.0 + d2, 0.0], [0.0, 0.0, 1.0]])
    Q = np.array([[1.0, 1.0, 0.0], [0.0, np.sqrt(d2), 0.0], [0.0, 0.0, 1.0]])
    AQ = Q.T @ np.diag([1.0, 2.0, 3.0]) @ Q
    eps, Phi, fb = ctx.reduced_eig(dev(torch, AQ), dev(torch, BQ))
    ref, _, rfb = O.reduced_eig(AQ, BQ)
    assert fb == rfb == fallback
    eps = host(eps)
    if fallback:
        assert np.sum(np.isfinite(eps)) == 2 and np.isnan(eps[2])
        assert np.allclose(eps[:2], ref[:2], rtol=1e-8)
    else:
        assert np.allclose(eps, [1.0, 2.0, 3.0], rtol=1e-4)


def test_reduced_eig_fallback(ctx, torch):
    rng = np.random.default_rng(8)
    G = rng.standard_normal((10, 6))
    BQ = G @ G.T
    AQ = G @ np.diag(np.arange(1.0, 7.0)) @ G.T
    eps, Phi, fb = ctx.reduced_eig(dev(torch, AQ), dev(torch, BQ))
    eps, Phi = host(eps), host(Phi)
    ref, _, rfb = O.reduced_eig(AQ, BQ)
    assert fb and rfb
    assert np.sum(np.isfinite(eps)) == np.sum(np.isfinite(ref)) == 6
    assert np.allclose(eps[:6], ref[:6], atol=1e-8)
    assert np.all(np.isnan(eps[6:])) and np.all(Phi[:, 6:] == 0)


def check_against_oracle(r, ref, p, emin, emax):
    assert r.M == ref.M
    M = r.M
    lam = host(r.lam)
    scale = np.maximum(np.abs(ref.lam[:M]), (emax - emin) / 2)
    assert np.max(np.abs(lam[:M] - ref.lam[:M]) / scale, initial=0) <= 1e-10
    res = host(r.res)
    assert np.max(res[:M], initial=0) <= 1e-9
    assert abs(r.loops - ref.loops) <= 1
    X = host(r.X)[:, :M]
    B = O.assemble(p.Bd, p.Bu)
    assert np.max(np.abs(X.T @ (B @ X) - np.eye(M)), initial=0) <= 1e-9
    # the in-interval subspaces agree (principal angles)
    if M:
        Xo = ref.X[:, :M]
        G = Xo.T @ (B @ X)
        s = np.linalg.svd(G, compute_uv=False)
        assert np.min(s) >= 1 - 1e-9


def test_solve_chain800(ctx, torch):
    p, emin, emax, m0, ne, Y0 = W.make_workload("chain800")
    r = ctx.solve(gpencil(p), emin, emax, m0, ne, dev(torch, Y0))
    ref = O.feast(p, emin, emax, m0, ne, Y0)
    assert r.status == 0
    assert r.m0_small == 0  # M0 = 30 = 1.5 M
    check_against_oracle(r, ref, p, emin, emax)
    lam_b = O.bruteforce(p)[0]
    assert np.max(np.abs(host(r.lam)[:20] - lam_b[200:220]) / np.abs(lam_b[200:220])) <= 1e-12


@pytest.mark.parametrize("nc,b,seed,k0,m,extra", [
    (2, 3, 1, 1, 2, 2), (3, 4, 2, 3, 4, 3), (4, 5, 3, 5, 6, 4), (6, 8, 4, 10, 12, 6),
    (1, 9, 5, 2, 3, 2), (7, 16, 6, 30, 10, 8), (11, 20, 7, 60, 15, 9),
    (10, 20, 8, 50, 40, 40), (12, 16, 9, 40, 50, 50)])  # M0 = 80, 100: 5 and 7 column tiles
def test_solve_small(ctx, torch, nc, b, seed, k0, m, extra):
    p = W.dense_random_pencil(nc, b, seed)
    lam = O.bruteforce(p)[0]
    emin, emax = 0.5 * (lam[k0 - 1] + lam[k0]), 0.5 * (lam[k0 + m - 1] + lam[k0 + m])
    m0 = min(m + extra, p.n)
    Y0 = W.random_subspace(p.n, m0, seed + 100)
    r = ctx.solve(gpencil(p), emin, emax, m0, 8, dev(torch, Y0), tol=1e-13, max_loops=40)
    ref = O.feast(p, emin, emax, m0, 8, Y0, tol=1e-13, max_loops=40)
    assert r.status == ref.status
    check_against_oracle(r, ref, p, emin, emax)


@pytest.mark.parametrize("parts", [1, 2, 3, 5])
def test_solve_partitioned_factor(ctx, torch, parts):
    # the partitioned factorisation is exact: results agree with the oracle
    # for any number of partitions per half chain
    p, emin, emax, m0, ne, Y0 = W.make_workload("chain800")
    r = ctx.solve(gpencil(p), emin, emax, m0, ne, dev(torch, Y0), partitions=parts)
    ref = O.feast(p, emin, emax, m0, ne, Y0)
    assert r.status == 0
    check_against_oracle(r, ref, p, emin, emax)


def test_solve_tb6400_golden(ctx, torch):
    g = json.load(open(os.path.join(GOLDEN, "feast_tb6400.json")))
    p, emin, emax, m0, ne, Y0 = W.make_workload("tb6400")
    r = ctx.solve(gpencil(p), emin, emax, m0, ne, dev(torch, Y0))
    assert r.status == 0 and r.M == g["M"] == 80
    lam = host(r.lam)[:80]
    ref = np.array(g["lam"])
    assert np.max(np.abs(lam - ref) / np.abs(ref)) <= 1e-10
    assert np.max(host(r.res)[:80]) <= 1e-9
    assert abs(r.loops - g["loops"]) <= 1


def test_solve_tb128k_full_size(ctx, torch):
    """The full-size workload (nc=2000, b=64, n=128000, M0=128, Ne=8) in the
    launch configuration the benchmark times: eigenvalues against the stored
    oracle result, residuals recomputed on the host for a sample of pairs,
    and B-orthonormality of that sample."""
    g = json.load(open(os.path.join(GOLDEN, "feast_tb128k.json")))
    p, emin, emax, m0, ne, Y0 = W.make_workload("tb128k")
    r = ctx.solve(gpencil(p), emin, emax, m0, ne, dev(torch, Y0))
    assert r.status == 0 and r.M == g["M"] == 80
    lam = host(r.lam)[:80]
    ref = np.array(g["lam"])
    assert np.max(np.abs(lam - ref) / np.abs(ref)) <= 1e-10
    res = host(r.res)
    assert np.max(res[:80]) <= 1e-9
    assert abs(r.loops - g["loops"]) <= 1
    cols = [0, 13, 27, 40, 53, 66, 79]
    X = host(r.X)[:, cols]
    AX = O.bt_multiply(p.Ad, p.Au, X)
    BX = O.bt_multiply(p.Bd, p.Bu, X)
    res_host = O.residuals(p, lam[cols], X, emin, emax)
    assert np.max(res_host) <= 1e-9
    assert np.allclose(res_host, res[cols], rtol=1e-3, atol=1e-14)
    assert np.max(np.abs(X.T @ BX - np.eye(len(cols)))) <= 1e-9
    assert np.max(np.abs(AX - BX * lam[cols]), initial=0) <= 1e-9 * np.max(np.abs(AX))


def test_solve_multiplicity_k_copies(ctx, torch):
    # k copies of a chain joined by zero coupling blocks (the replicated
    # systems of Sec. IV.B, Table IV): every eigenvalue is k-fold; the zero
    # junctions fall inside partitions of the factorisation
    k = 4
    p1 = W.dense_random_pencil(6, 16, 61)
    lam1 = O.bruteforce(p1)[0]
    emin, emax = 0.5 * (lam1[29] + lam1[30]), 0.5 * (lam1[34] + lam1[35])
    z = np.zeros((1, 16, 16))
    Ad = np.concatenate([p1.Ad] * k)
    Bd = np.concatenate([p1.Bd] * k)
    Au = np.concatenate(sum([[p1.Au, z] for _ in range(k)], [])[:-1])
    Bu = np.concatenate(sum([[p1.Bu, z] for _ in range(k)], [])[:-1])
    p = W.Pencil(Ad, Au, Bd, Bu)
    Y0 = W.random_subspace(p.n, 32, 62)
    r = ctx.solve(gpencil(p), emin, emax, 32, 8, dev(torch, Y0), max_loops=40)
    ref = O.feast(p, emin, emax, 32, 8, Y0, max_loops=40)
    assert r.status == ref.status == 0 and r.M == 5 * k
    check_against_oracle(r, ref, p, emin, emax)
    got = np.sort(host(r.lam)[:r.M]).reshape(5, k)
    assert np.max(np.abs(got - lam1[30:35, None])) <= 1e-10 * np.max(np.abs(lam1))


def test_solve_warm_start_one_loop(ctx, torch):
    # Y0 = exact B-orthonormal eigenvectors (Sec. III.B (i)): the first
    # contour integration already returns the exact eigenvalues
    p = W.dense_random_pencil(8, 16, 71)
    lam, Xe = O.bruteforce(p)
    k0, m = 40, 6
    emin, emax = 0.5 * (lam[k0 - 1] + lam[k0]), 0.5 * (lam[k0 + m - 1] + lam[k0 + m])
    cols = np.argsort(np.abs(lam - 0.5 * (emin + emax)))[:10]
    Y0 = np.ascontiguousarray(Xe[:, cols])
    r = ctx.solve(gpencil(p), emin, emax, 10, 8, dev(torch, Y0), max_loops=1)
    assert r.status == 1 and r.loops == 1 and r.M == m
    got = host(r.lam)[:m]
    assert np.max(np.abs(got - lam[k0:k0 + m])) <= 1e-12 * np.max(np.abs(lam))
    assert np.max(host(r.res)[:m]) <= 1e-12


@pytest.mark.parametrize("seed,n,m0", [(0, 800, 30), (987654321, 1000, 7), (2 ** 64 - 1, 3, 1)])
def test_random_start_block(ctx, torch, seed, n, m0):
    # the start block of Y0 = NULL (Fig. 2 step 1) against the oracle's own
    # implementation of the same generator, element by element (the two sides
    # differ only in the last bits of log, cos and sin)
    Y = host(ctx.random_start(seed, n, m0))
    ref = O.random_start(seed, n, m0)
    assert np.all(np.abs(Y - ref) <= 1e-14 * np.maximum(np.abs(ref), 1.0))


@pytest.mark.parametrize("seed", [0, 987654321])
def test_solve_random_start(ctx, torch, seed):
    # a solve with Y0 = NULL agrees with the oracle started from the same block
    p, emin, emax, m0, ne, _ = W.make_workload("chain800")
    Y0 = O.random_start(seed, p.n, m0)
    r = ctx.solve(gpencil(p), emin, emax, m0, ne, None, seed=seed)
    ref = O.feast(p, emin, emax, m0, ne, Y0)
    assert r.status == ref.status == 0
    check_against_oracle(r, ref, p, emin, emax)


def test_empty_interval(ctx, torch):
    p = W.dense_random_pencil(3, 8, 9)
    lam = O.bruteforce(p)[0]
    gap = np.argmax(np.diff(lam))
    emin = lam[gap] + 0.3 * (lam[gap + 1] - lam[gap])
    emax = lam[gap] + 0.7 * (lam[gap + 1] - lam[gap])
    Y0 = W.random_subspace(p.n, 4, 3)
    r = ctx.solve(gpencil(p), emin, emax, 4, 8, dev(torch, Y0))
    assert r.status == 3 and r.M == 0


@pytest.mark.parametrize("k0,m", [(5, 3), (10, 2)])
def test_subspace_just_large_enough(ctx, torch, k0, m):
    # M0 = M: status 4 (Fig. 2 asks for M0 > M), the pairs still found
    p = W.dense_random_pencil(3, 8, 9)
    lam = O.bruteforce(p)[0]
    emin, emax = 0.5 * (lam[k0 - 1] + lam[k0]), 0.5 * (lam[k0 + m - 1] + lam[k0 + m])
    Y0 = W.random_subspace(p.n, m, 3)
    r = ctx.solve(gpencil(p), emin, emax, m, 8, dev(torch, Y0), max_loops=40)
    ref = O.feast(p, emin, emax, m, 8, Y0, max_loops=40)
    assert r.status == ref.status == 4 and r.M == ref.M == m
    assert r.m0_small == 1  # M0 = M < 1.5 M
    check_against_oracle(r, ref, p, emin, emax)


def test_not_converged(ctx, torch):
    # one loop cannot converge (the trace test needs two): status 1, and the
    # outputs hold that loop, as the oracle's
    p = W.dense_random_pencil(3, 8, 9)
    lam = O.bruteforce(p)[0]
    emin, emax = 0.5 * (lam[4] + lam[5]), 0.5 * (lam[8] + lam[9])
    Y0 = W.random_subspace(p.n, 8, 3)
    r = ctx.solve(gpencil(p), emin, emax, 8, 8, dev(torch, Y0), max_loops=1)
    ref = O.feast(p, emin, emax, 8, 8, Y0, max_loops=1)
    assert r.status == ref.status == 1 and r.loops == 1 and r.M == ref.M
    lam_g = host(r.lam)[:r.M]
    assert np.max(np.abs(lam_g - ref.lam[:ref.M]) / np.abs(ref.lam[:ref.M])) <= 1e-10


def test_bad_arguments(ctx, torch):
    from paper_0901_2665_amd import feast as F
    p = W.dense_random_pencil(3, 8, 9)
    gp = gpencil(p)
    Y0 = dev(torch, W.random_subspace(p.n, 4, 3))
    with pytest.raises(F.FeastError) as e:
        ctx.solve(gp, 1.0, 0.0, 4, 8, Y0)
    assert e.value.status == -2
    with pytest.raises(F.FeastError) as e:
        ctx.solve(gp, 0.0, 1.0, 4, 0, Y0)
    assert e.value.status == -4
    with pytest.raises(F.FeastError) as e:
        ctx.solve(gp, 0.0, 1.0, 4, 8, Y0, tol=0.0)
    assert e.value.status == -7
    with pytest.raises(F.FeastError) as e:
        ctx.solve(gp, 0.0, 1.0, 4, 8, Y0, max_loops=0)
    assert e.value.status == -7
    with pytest.raises(F.FeastError) as e:  # M0 > N (checked before Y0 is read)
        ctx.solve(gp, 0.0, 1.0, p.n + 1, 8, Y0)
    assert e.value.status == -3
    bad = W.Pencil(p.Ad.copy(), p.Au, p.Bd, p.Bu)
    bad.Ad[1, 2, 3] = np.nan
    with pytest.raises(F.FeastError) as e:
        ctx.solve(gpencil(bad), 0.0, 1.0, 4, 8, Y0)
    assert e.value.status == -6


def test_deterministic(ctx, torch):
    p, emin, emax, m0, ne, Y0 = W.make_workload("chain800")
    gp, y = gpencil(p), dev(torch, Y0)
    a = ctx.solve(gp, emin, emax, m0, ne, y)
    b = ctx.solve(gp, emin, emax, m0, ne, y)
    assert torch.equal(a.lam, b.lam) and torch.equal(a.X, b.X) and torch.equal(a.res, b.res)


@pytest.mark.parametrize("nc,b,seed,k0,m,extra", [(6, 96, 81, 150, 20, 20), (4, 80, 82, 90, 12, 30),
                                                  (2, 65, 83, 40, 5, 3), (30, 96, 84, 700, 24, 16),
                                                  (8, 90, 86, 200, 60, 40)])
def test_solve_blocks_above_64(ctx, torch, nc, b, seed, k0, m, extra):
    # b > 64: the wide kernels (factorisation, sweeps, B Y, projection,
    # residuals), up to M0 = 100, against the oracle and brute force
    p = W.dense_random_pencil(nc, b, seed)
    lam = O.bruteforce(p)[0]
    emin, emax = 0.5 * (lam[k0 - 1] + lam[k0]), 0.5 * (lam[k0 + m - 1] + lam[k0 + m])
    m0 = m + extra
    Y0 = W.random_subspace(p.n, m0, seed + 100)
    r = ctx.solve(gpencil(p), emin, emax, m0, 8, dev(torch, Y0), tol=1e-13, max_loops=40)
    ref = O.feast(p, emin, emax, m0, 8, Y0, tol=1e-13, max_loops=40)
    # status 2 (B_Q fallback) where M0 is well above M, on both sides alike
    assert r.status == ref.status and r.status in (0, 2)
    check_against_oracle(r, ref, p, emin, emax)
    assert np.max(np.abs(host(r.lam)[:m] - lam[k0:k0 + m]) / np.abs(lam[k0:k0 + m])) <= 1e-10


def test_blocks_above_64_limits(ctx, torch):
    from paper_0901_2665_amd import feast as F
    p = W.dense_random_pencil(2, 96, 85)
    y = dev(torch, W.random_subspace(p.n, 129, 1))
    with pytest.raises(F.FeastError) as e:          # M0 above 128
        ctx.solve(gpencil(p), 0.0, 1.0, 129, 8, y)
    assert e.value.status == -3
    with pytest.raises(F.FeastError) as e:          # no mixed precision there
        ctx.solve(gpencil(p), 0.0, 1.0, 8, 8, dev(torch, W.random_subspace(p.n, 8, 1)),
                  precision=1)
    assert e.value.status == -7
    q = W.dense_random_pencil(2, 97, 86)
    with pytest.raises(F.FeastError) as e:          # above 96
        ctx.solve(gpencil(q), 0.0, 1.0, 8, 8, dev(torch, W.random_subspace(q.n, 8, 1)))
    assert e.value.status == -1
