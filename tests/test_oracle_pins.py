"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each pin is chosen so that a plausible slip in the oracle fails one of them:
the quadrature rule (printed table, polynomial exactness), the contour and
accumulation weights (closed-form filter values at the centre and the ends
of the interval), the solve + accumulation (spectral closed form of one
contour integration), the Rayleigh-Ritz output (dense brute force, Sylvester
inertia, B-orthonormality, multiplicity, warm start).  The last tests plant
mistakes in the oracle and check that the pins catch them.
"""
import os

import numpy as np
import pytest

from oracle import feast_oracle as O
from paper_0901_2665_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_pencil(nc, b, seed):
    return W.dense_random_pencil(nc, b, seed)


def diagonal_pencil(values, b=2):
    """Block-diagonal pencil (zero couplings) with A = diag(values), B = I."""
    v = np.asarray(values, dtype=np.float64)
    assert len(v) % b == 0
    nc = len(v) // b
    Ad = np.zeros((nc, b, b))
    for i in range(nc):
        Ad[i] = np.diag(v[i * b:(i + 1) * b])
    Bd = np.broadcast_to(np.eye(b), (nc, b, b)).copy()
    return W.Pencil(Ad, np.zeros((nc - 1, b, b)), Bd, np.zeros((nc - 1, b, b)))


def gap_interval(lam, k0, m):
    return 0.5 * (lam[k0 - 1] + lam[k0]), 0.5 * (lam[k0 + m - 1] + lam[k0 + m])


# ----------------------------------------------------------------- quadrature

def test_gauss_legendre_matches_printed_table():
    tab = np.loadtxt(os.path.join(GOLDEN, "gauss_legendre_ne8.txt"))
    order = np.argsort(tab[:, 1])
    xp, wp = tab[order, 1], tab[order, 2]
    x, w = O.gauss_legendre(8)
    assert np.max(np.abs(x - xp)) <= 1e-15
    assert np.max(np.abs(w - wp)) <= 1e-15


@pytest.mark.parametrize("ne", [1, 2, 3, 4, 5, 8, 12, 16, 24])
def test_gauss_legendre_polynomial_exactness(ne):
    x, w = O.gauss_legendre(ne)
    for j in range(2 * ne):
        exact = 2.0 / (j + 1) if j % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** j) - exact) <= 1e-14
    assert np.all(np.diff(x) > 0) and np.all(w > 0)


@pytest.mark.parametrize("ne", [4, 8, 16])
def test_gauss_legendre_vs_library(ne):
    x, w = O.gauss_legendre(ne)
    xl, wl = np.polynomial.legendre.leggauss(ne)
    assert np.max(np.abs(x - xl)) <= 1e-15
    assert np.max(np.abs(w - wl)) <= 2e-15


# ------------------------------------------------------------- random start

@pytest.mark.parametrize("seed", [0, 5, 2 ** 63 + 12345])
def test_philox_matches_numpy_bit_generator(seed):
    # numpy's Philox bit generator is Philox4x64-10; it increments its
    # counter before the first block, so its block q is our counter q + 1
    bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64),
                          counter=np.zeros(4, dtype=np.uint64))
    raw = bg.random_raw(4 * 64).reshape(64, 4)
    q = np.arange(1, 65, dtype=np.uint64)
    z = np.zeros_like(q)
    w = O.philox4x64_10([q, z, z, z], (seed, 0))
    assert np.array_equal(np.stack(w, axis=1), raw)


def test_random_start_is_standard_normal():
    import scipy.stats
    Y = O.random_start(11, 1000, 200)
    v = Y.ravel()
    assert abs(v.mean()) < 5e-3 and abs(v.std() - 1.0) < 5e-3
    assert scipy.stats.kstest(v, "norm").pvalue > 1e-3
    # the four normals of one counter are independent of each other
    C = np.corrcoef(v.reshape(-1, 4).T)
    assert np.max(np.abs(C - np.eye(4))) < 1e-2
    # deterministic, and a different seed gives a different block
    assert np.array_equal(Y, O.random_start(11, 1000, 200))
    assert not np.allclose(Y[:5], O.random_start(12, 1000, 200)[:5])


# ----------------------------------------------------------- contour filter

def filter_values(values, emin, emax, ne):
    """Diagonal of -Q for the pencil (diag(values), I) and Y = I.  For this
    pencil Q = -diag(f(values)) with f the rational filter of the contour."""
    p = diagonal_pencil(values)
    Y = np.eye(p.n)
    Q = O.filter_apply(p, emin, emax, ne, Y)
    off = Q - np.diag(np.diag(Q))
    assert np.max(np.abs(off)) <= 1e-14
    return -np.diag(Q)


@pytest.mark.parametrize("ne", [4, 8, 16])
def test_filter_closed_form_points(ne):
    # f(c) = 1 because the weights sum to 2; f(emin) = f(emax) = 1/2 because
    # Re{e^{i t} / (e^{i t} -/+ 1)} = 1/2 for every t.
    emin, emax = -1.3, 2.1
    c = 0.5 * (emin + emax)
    f = filter_values([c, emin, emax, c], emin, emax, ne)
    assert abs(f[0] - 1.0) <= 1e-14
    assert abs(f[1] - 0.5) <= 1e-14
    assert abs(f[2] - 0.5) <= 1e-14


def test_filter_shape():
    # inside the interval the filter is close to 1, far outside close to 0,
    # and it improves with Ne (Table III: more nodes, smaller residual)
    emin, emax = 0.0, 2.0
    f8 = filter_values([0.2, 1.8, 4.0, -3.0], emin, emax, 8)
    f16 = filter_values([0.2, 1.8, 4.0, -3.0], emin, emax, 16)
    assert np.all(np.abs(f8[:2] - 1) < 0.05) and np.all(np.abs(f8[2:]) < 1e-3)
    assert np.all(np.abs(f16[2:]) < np.abs(f8[2:]))


# ---------------------------------------------- solve + accumulation (eq. 15)

def test_shifted_solve_backward_error():
    p = tiny_pencil(5, 6, 11)
    R = np.random.default_rng(1).standard_normal((p.n, 7))
    z = 0.3 + 0.05j
    X = O.shifted_solve(p, z, R)
    M = O.shifted_matrix(p, z).toarray()
    be = np.linalg.norm(R - M @ X) / (np.linalg.norm(M) * np.linalg.norm(X))
    assert be <= 1e-15
    Xd = np.linalg.solve(M, R)
    assert np.linalg.norm(X - Xd) <= 1e-12 * np.linalg.norm(Xd)


@pytest.mark.parametrize("seed", [3, 4])
def test_one_contour_integration_spectral_form(seed):
    # With B-orthonormal eigenpairs, (zB - A)^{-1} = sum_j x_j x_j^T / (z - lam_j),
    # so one contour integration is Q = X diag(g) X^T B Y with g the filter of
    # the diagonal pencil holding the same eigenvalues.
    p = tiny_pencil(4, 5, seed)
    lam, X = O.bruteforce(p)
    emin, emax = gap_interval(lam, 6, 5)
    Y = np.random.default_rng(seed).standard_normal((p.n, 9))
    Q = O.filter_apply(p, emin, emax, 8, Y)
    g = -filter_values(lam, emin, emax, 8)
    B = O.assemble(p.Bd, p.Bu)
    ref = X @ (g[:, None] * (X.T @ (B @ Y)))
    assert np.linalg.norm(Q - ref) <= 1e-12 * np.linalg.norm(ref)


# ------------------------------------------------------- converged output

@pytest.mark.parametrize("nc,b,seed,k0,m,extra", [
    (2, 3, 1, 1, 2, 2), (3, 4, 2, 3, 4, 3), (4, 5, 3, 5, 6, 4), (6, 8, 4, 10, 12, 6),
    (5, 2, 5, 2, 3, 2), (3, 7, 6, 4, 1, 2)])
def test_feast_matches_bruteforce(nc, b, seed, k0, m, extra):
    p = tiny_pencil(nc, b, seed)
    lam, _ = O.bruteforce(p)
    emin, emax = gap_interval(lam, k0, m)
    m0 = min(m + extra, p.n)
    Y0 = W.random_subspace(p.n, m0, seed + 100)
    r = O.feast(p, emin, emax, m0, 8, Y0, tol=1e-13, max_loops=40)
    assert r.status in (0, 4)
    assert r.M == m
    ref = lam[k0:k0 + m]
    scale = np.maximum(np.abs(ref), (emax - emin) / 2)
    assert np.max(np.abs(r.lam[:m] - ref) / scale) <= 1e-12
    B = O.assemble(p.Bd, p.Bu)
    Xm = r.X[:, :m]
    assert np.max(np.abs(Xm.T @ (B @ Xm) - np.eye(m))) <= 1e-12
    assert r.max_res <= 1e-12


def test_feast_chain800_matches_bruteforce():
    p, emin, emax, m0, ne, Y0 = W.make_workload("chain800")
    lam, _ = O.bruteforce(p)
    r = O.feast(p, emin, emax, m0, ne, Y0)
    assert r.status == 0 and r.M == 20
    ref = lam[200:220]
    assert np.max(np.abs(r.lam[:20] - ref) / np.abs(ref)) <= 1e-12
    assert r.max_res <= 1e-12
    assert 2 <= r.loops <= 6


def test_inertia_count_vs_bruteforce():
    p = tiny_pencil(6, 5, 9)
    lam, _ = O.bruteforce(p)
    for s in np.linspace(lam[0] - 1, lam[-1] + 1, 23):
        assert O.inertia_count(p, s) == int(np.sum(lam < s))


def test_multiplicity_k_copies():
    # k copies on the diagonal (zero coupling at the junctions): every
    # eigenvalue is k-fold and k*M pairs are found with the same Ne solves.
    k = 3
    p1 = tiny_pencil(3, 4, 21)
    lam1, _ = O.bruteforce(p1)
    emin, emax = gap_interval(lam1, 3, 3)
    Ad = np.concatenate([p1.Ad] * k)
    Bd = np.concatenate([p1.Bd] * k)
    z = np.zeros((1, 4, 4))
    Au = np.concatenate(sum([[p1.Au, z] for _ in range(k)], [])[:-1])
    Bu = np.concatenate(sum([[p1.Bu, z] for _ in range(k)], [])[:-1])
    p = W.Pencil(Ad, Au, Bd, Bu)
    Y0 = W.random_subspace(p.n, 14, 5)
    r = O.feast(p, emin, emax, 14, 8, Y0, max_loops=40)
    assert r.M == 3 * k
    got = r.lam[:r.M].reshape(3, k)
    assert np.max(np.abs(got - lam1[3:6, None])) <= 1e-10


def test_warm_start_one_loop():
    # Y = exact B-orthonormal eigenvectors: rho B X = X, so the first loop
    # already returns the exact eigenvalues (Sec. III.B (i)).
    p = tiny_pencil(5, 6, 31)
    lam, X = O.bruteforce(p)
    emin, emax = gap_interval(lam, 10, 4)
    cols = np.argsort(np.abs(lam - 0.5 * (emin + emax)))[:8]
    Q = O.filter_apply(p, emin, emax, 8, X[:, cols])
    AQ, BQ = O.project(p, Q)
    eps, _, fb = O.reduced_eig(AQ, BQ)
    assert not fb
    assert np.max(np.abs(np.sort(eps) - np.sort(lam[cols]))) <= 1e-12


def test_reduced_eig_b_orthonormal():
    rng = np.random.default_rng(7)
    G = rng.standard_normal((12, 12))
    BQ = G @ G.T + 0.1 * np.eye(12)
    AQ = rng.standard_normal((12, 12))
    AQ = AQ + AQ.T
    eps, Phi, fb = O.reduced_eig(AQ, BQ)
    assert not fb and np.all(np.diff(eps) >= 0)
    assert np.max(np.abs(Phi.T @ BQ @ Phi - np.eye(12))) <= 1e-12
    assert np.max(np.abs(AQ @ Phi - BQ @ Phi * eps)) <= 1e-11


def test_reduced_eig_scaled_columns_keep_cholesky():
    # B_Q diagonal with entries down to 1e-14: every Cholesky pivot equals
    # its own diagonal entry, so the scale-invariant test keeps the Cholesky
    # path and the eigenvalues are exact
    mu = np.geomspace(1.0, 1e-14, 9)
    BQ = np.diag(mu)
    AQ = np.diag(np.arange(1.0, 10.0)) * mu
    eps, Phi, fb = O.reduced_eig(AQ, BQ)
    assert not fb
    assert np.allclose(eps, np.arange(1.0, 10.0), rtol=1e-12)


@pytest.mark.parametrize("d2,fallback", [(1e-14, True), (1e-13, True), (1e-11, False)])
def test_reduced_eig_pivot_cut(d2, fallback):
    # Q = [e1, e1 + d e2, e3]: B_Q = Q^T Q has the pivot d^2 / (1 + d^2)
    # relative to its diagonal in row 2; at or below 1e-12 it falls back
    BQ = np.array([[1.0, 1.0, 0.0], [1.0, 1.0 + d2, 0.0], [0.0, 0.0, 1.0]])
    Q = np.array([[1.0, 1.0, 0.0], [0.0, np.sqrt(d2), 0.0], [0.0, 0.0, 1.0]])
    AQ = Q.T @ np.diag([1.0, 2.0, 3.0]) @ Q
    eps, Phi, fb = O.reduced_eig(AQ, BQ)
    assert fb == fallback
    if fallback:  # B_Q's eigenvalue ~ d^2 / 2 <= 1e-10 max is dropped
        assert np.sum(np.isfinite(eps)) == 2 and np.isnan(eps[2])
    else:
        assert np.allclose(eps, [1.0, 2.0, 3.0], rtol=1e-4)


def test_reduced_eig_fallback_rank_deficient():
    rng = np.random.default_rng(8)
    G = rng.standard_normal((10, 6))
    BQ = G @ G.T  # rank 6
    AQ = G @ np.diag(np.arange(1.0, 7.0)) @ G.T
    eps, Phi, fb = O.reduced_eig(AQ, BQ)
    assert fb
    assert np.sum(np.isfinite(eps)) == 6
    assert np.allclose(np.sort(eps[np.isfinite(eps)]), np.arange(1.0, 7.0), atol=1e-8)


def test_residual_of_exact_pairs_is_tiny():
    p = tiny_pencil(4, 4, 41)
    lam, X = O.bruteforce(p)
    res = O.residuals(p, lam, X, lam[0], lam[-1])
    assert np.max(res) <= 1e-13
    # a perturbed vector has a residual of the size of the perturbation
    Xp = X + 1e-6 * np.random.default_rng(0).standard_normal(X.shape)
    assert np.min(O.residuals(p, lam, Xp, lam[0], lam[-1])) > 1e-9


def _hand_pencil():
    """Two cells of b = 2 with small integer entries:
    A = [[2 1 1 2], [1 3 0 1], [1 0 4 0], [2 1 0 -1]],
    B = [[2 0 0 1], [0 1 0 0], [0 0 1 0], [1 0 0 2]] (eigenvalues 1, 1, 1, 3)."""
    Ad = np.array([[[2, 1], [1, 3]], [[4, 0], [0, -1]]], dtype=np.float64)
    Au = np.array([[[1, 2], [0, 1]]], dtype=np.float64)
    Bd = np.array([[[2, 0], [0, 1]], [[1, 0], [0, 2]]], dtype=np.float64)
    Bu = np.array([[[0, 1], [0, 0]]], dtype=np.float64)
    return W.Pencil(Ad, Au, Bd, Bu)


# Worked by hand (Table I caption: ||A x - lam B x||_1 / ||A x||_1):
#   x1 = (1, -1, 2, 0), lam1 = 2:   A x1 = (3, -2, 9, 1), ||.||_1 = 15;
#       B x1 = (2, -1, 2, 1), ||.||_1 = 6;  A x1 - 2 B x1 = (-1, 0, 5, -1), ||.||_1 = 7.
#   x2 = (0, 1, 0, 1), lam2 = 1/2:  A x2 = (3, 4, 0, 0), ||.||_1 = 7;
#       B x2 = (1, 1, 0, 2), ||.||_1 = 4;  A x2 - B x2 / 2 = (5/2, 7/2, 0, -1), ||.||_1 = 7.
# On [1, 3] (r = 1) no guard applies: 7/15 and 7/7.  On [-10, 10] (r = 10)
# ||A x||_1 < r ||B x||_1 for both, so the denominators are ||B x||_1 * 10:
# 7/60 and 7/40.
HAND_X = np.array([[1.0, 0.0], [-1.0, 1.0], [2.0, 0.0], [0.0, 1.0]])
HAND_LAM = np.array([2.0, 0.5])


def test_residual_hand_worked_values():
    p = _hand_pencil()
    res = O.residuals(p, HAND_LAM, HAND_X, 1.0, 3.0)
    assert np.allclose(res, [7.0 / 15.0, 1.0], rtol=1e-15, atol=0)


def test_residual_small_ax_guard_hand_worked():
    p = _hand_pencil()
    res = O.residuals(p, HAND_LAM, HAND_X, -10.0, 10.0)
    assert np.allclose(res, [7.0 / 60.0, 7.0 / 40.0], rtol=1e-15, atol=0)


@pytest.mark.parametrize("variant", ["bx_denominator", "two_norm", "no_guard"])
def test_planted_residual_mistakes_are_caught(monkeypatch, variant):
    # each plausible misreading of the Table I caption changes a hand value
    def bad(p, lam, X, emin, emax):
        A = O.assemble(p.Ad, p.Au)
        B = O.assemble(p.Bd, p.Bu)
        AX, BX = A @ X, B @ X
        D = AX - BX * lam[None, :]
        r = (emax - emin) / 2.0
        if variant == "bx_denominator":
            return np.sum(np.abs(D), axis=0) / np.sum(np.abs(BX), axis=0)
        if variant == "two_norm":
            return np.linalg.norm(D, axis=0) / np.linalg.norm(AX, axis=0)
        return np.sum(np.abs(D), axis=0) / np.sum(np.abs(AX), axis=0)
    monkeypatch.setattr(O, "residuals", bad)
    p = _hand_pencil()
    r1 = O.residuals(p, HAND_LAM, HAND_X, 1.0, 3.0)
    r2 = O.residuals(p, HAND_LAM, HAND_X, -10.0, 10.0)
    ok = (np.allclose(r1, [7.0 / 15.0, 1.0], rtol=1e-12) and
          np.allclose(r2, [7.0 / 60.0, 7.0 / 40.0], rtol=1e-12))
    assert not ok


# ------------------------------------------- counting gate and convergence

def _slow_pair_case(seed, frac, extra, side="hi"):
    """Eigenvalues 10..17 of a dense-coupling chain inside the interval, one end
    placed at ``frac`` of the gap from the nearest inside eigenvalue, so that
    eigenvalue's filter value is close to 1/2 and its pair converges slowly."""
    p = tiny_pencil(6, 8, seed)
    lam, _ = O.bruteforce(p)
    k0, m = 10, 8
    if side == "hi":
        emin = 0.5 * (lam[k0 - 1] + lam[k0])
        emax = lam[k0 + m - 1] + frac * (lam[k0 + m] - lam[k0 + m - 1])
    else:
        emax = 0.5 * (lam[k0 + m - 1] + lam[k0 + m])
        emin = lam[k0] - frac * (lam[k0] - lam[k0 - 1])
    Y0 = W.random_subspace(p.n, m + extra, seed + 7)
    return p, lam, emin, emax, m + extra, Y0


@pytest.mark.parametrize("seed,frac,extra,side", [
    (3, 1e-3, 2, "hi"), (6, 1e-2, 2, "hi"), (23, 0.1, 2, "hi"),
    (29, 1e-2, 2, "hi"), (43, 1e-3, 1, "hi"), (16, 0.3, 4, "lo"), (5, 1e-3, 1, "lo")])
def test_slow_pairs_are_not_dropped(seed, frac, extra, side):
    # With M0 barely above M every true pair can still sit above the counting
    # gate (residual <= sqrt(tol)) after two loops; the counted set at
    # convergence must still be the brute-force set.
    p, lam, emin, emax, m0, Y0 = _slow_pair_case(seed, frac, extra, side)
    r = O.feast(p, emin, emax, m0, 8, Y0, tol=1e-12, max_loops=60)
    ref = lam[(lam >= emin) & (lam <= emax)]
    assert r.status == 0
    assert r.M == len(ref) == 8
    assert np.max(np.abs(r.lam[:r.M] - ref)) <= 1e-10 * np.max(np.abs(ref))
    # an in-interval Ritz value left uncounted at convergence is a mixture,
    # not one of the true eigenvalues
    rest = r.lam[r.M:]
    left = rest[(rest >= emin) & (rest <= emax)]
    for v in left:
        assert np.min(np.abs(ref - v)) > 1e-8


def test_planted_gate_without_convergence_wait_is_caught(monkeypatch):
    # without the wait for uncounted in-interval pairs that are still
    # converging, two loops with no pair below the gate end the iteration
    # with M = 0 (seed 3 above)
    monkeypatch.setattr(O, "UNCOUNTED_DROP", 0.0)
    p, lam, emin, emax, m0, Y0 = _slow_pair_case(3, 1e-3, 2)
    r = O.feast(p, emin, emax, m0, 8, Y0, tol=1e-12, max_loops=60)
    assert r.M != 8


# ------------------------------------------------------ planted mistakes

def _spectral_error(monkeypatch=None):
    p = tiny_pencil(4, 5, 3)
    lam, X = O.bruteforce(p)
    emin, emax = gap_interval(lam, 6, 5)
    Y = np.random.default_rng(3).standard_normal((p.n, 9))
    Q = O.filter_apply(p, emin, emax, 8, Y)
    dp = diagonal_pencil(lam)
    g = np.diag(O.filter_apply(dp, emin, emax, 8, np.eye(dp.n)))
    B = O.assemble(p.Bd, p.Bu)
    ref = X @ (g[:, None] * (X.T @ (B @ Y)))
    return np.linalg.norm(Q - ref) / np.linalg.norm(ref)


def test_planted_theta_sign_is_caught(monkeypatch):
    # accumulation phase e^{-i theta} instead of e^{+i theta}
    good = O.contour

    def bad(emin, emax, ne):
        ct = good(emin, emax, ne)
        ct.theta = -ct.theta
        return ct
    monkeypatch.setattr(O, "contour", bad)
    emin, emax = -1.3, 2.1
    c = 0.5 * (emin + emax)
    f = -np.diag(O.filter_apply(diagonal_pencil([c, emin, emax, c]), emin, emax, 8,
                                np.eye(4)))
    assert abs(f[0] - 1.0) > 1e-3 or abs(f[1] - 0.5) > 1e-3


def test_planted_rhs_without_b_is_caught(monkeypatch):
    assert _spectral_error() <= 1e-12

    def bad(p, emin, emax, ne, Y, factors=None):
        # right-hand side Y instead of B Y
        ct = O.contour(emin, emax, ne)
        Q = np.zeros(Y.shape)
        for e in range(ne):
            Qe = O.factor_shift(p, ct.Z[e]).solve(Y)
            Q -= (ct.w[e] / 2.0) * np.real(ct.r * np.exp(1j * ct.theta[e]) * Qe)
        return Q
    monkeypatch.setattr(O, "filter_apply", bad)
    assert _spectral_error() > 1e-6


def test_planted_untransposed_coupling_is_caught(monkeypatch):
    p = tiny_pencil(4, 4, 51)
    good = O.assemble

    def bad(diag, up):
        M = good(diag, up).tolil()
        b = diag.shape[1]
        for i in range(diag.shape[0] - 1):
            M[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = up[i]  # not transposed
        return M.tocsr()
    lam_ref, _ = O.bruteforce(p)
    emin, emax = gap_interval(lam_ref, 4, 3)
    monkeypatch.setattr(O, "assemble", bad)
    Y0 = W.random_subspace(p.n, 6, 1)
    r = O.feast(p, emin, emax, 6, 8, Y0, max_loops=10)
    ok = (r.M == 3 and np.max(np.abs(r.lam[:3] - lam_ref[4:7])) <= 1e-10)
    assert not ok


# ------------------------------------------------- Hermitian A (eq. 12)

def test_hermitian_pencil_is_hermitian_definite():
    p = W.hermitian_pencil(4, 6, 1)
    A = O.assemble_hermitian(p.Ad, p.Au).toarray()
    B = O.assemble(p.Bd, p.Bu).toarray()
    assert np.max(np.abs(A - A.conj().T)) == 0.0 and np.max(np.abs(A.imag)) > 0.1
    assert np.min(np.linalg.eigvalsh(B)) > 0.5


@pytest.mark.parametrize("maker", ["dense", "chain"])
def test_hermitian_inertia_count_vs_bruteforce(maker):
    p = W.hermitian_pencil(5, 6, 3) if maker == "dense" else W.hermitian_chain_pencil(6, 8, 5)
    lam, _ = O.bruteforce_hermitian(p)
    for s in np.linspace(lam[0] - 1, lam[-1] + 1, 29):
        assert O.inertia_count_hermitian(p, s) == int(np.sum(lam < s))


def test_hermitian_chain_pencil_is_hermitian_definite():
    # genuinely complex (phases on every hopping), the sparsity of the real
    # recipe, B that recipe's B
    p = W.hermitian_chain_pencil(5, 8, 11)
    q = W.chain_pencil(5, 8, 11)
    A = O.assemble_hermitian(p.Ad, p.Au).toarray()
    assert np.max(np.abs(A - A.conj().T)) == 0.0 and np.max(np.abs(A.imag)) > 0.1
    assert np.allclose(np.abs(p.Ad), np.abs(q.Ad), rtol=1e-15, atol=0)
    assert np.allclose(np.abs(p.Au), np.abs(q.Au), rtol=1e-15, atol=0)
    assert np.array_equal(p.Ad != 0, q.Ad != 0) and np.array_equal(p.Au != 0, q.Au != 0)
    assert np.array_equal(p.Bd, q.Bd) and np.array_equal(p.Bu, q.Bu)


def test_hermitian_adjoint_solve():
    # the adjoint solve of the factorised z B - A is a solve with z* B - A
    p = W.hermitian_pencil(4, 5, 2)
    z = 0.2 + 0.07j
    R = W.random_complex_subspace(p.n, 3, 3)
    lu = O.factor_shift_hermitian(p, z)
    M = O.shifted_matrix_hermitian(p, z).toarray()
    assert np.allclose(lu.solve(R), np.linalg.solve(M, R), rtol=1e-12, atol=1e-13)
    Mc = O.shifted_matrix_hermitian(p, np.conj(z)).toarray()
    assert np.allclose(M.conj().T, Mc, rtol=0, atol=1e-15)
    assert np.allclose(lu.solve(R, adjoint=True), np.linalg.solve(Mc, R), rtol=1e-12, atol=1e-13)


def _hermitian_spectral_error(p, emin, emax, Y, filt):
    lam, X = O.bruteforce_hermitian(p)
    Q = filt(p, emin, emax, 8, Y)
    f = filter_values(lam, emin, emax, 8)
    B = O.assemble(p.Bd, p.Bu)
    ref = -X @ (f[:, None] * (X.conj().T @ (B @ Y)))
    return np.linalg.norm(Q - ref) / np.linalg.norm(ref)


def test_hermitian_contour_integration_spectral_form():
    # with B-orthonormal eigenvectors G(Z) = X (Z - Lambda)^-1 X^H and
    # G(Z)^H = X (conj Z - Lambda)^-1 X^H, so eq. 12 is Q = -X diag(f) X^H B Y
    # with the same rational filter f as the real case
    p = W.hermitian_pencil(4, 5, 4)
    lam, _ = O.bruteforce_hermitian(p)
    emin, emax = gap_interval(lam, 6, 5)
    Y = W.random_complex_subspace(p.n, 7, 5)
    assert _hermitian_spectral_error(p, emin, emax, Y, O.filter_apply_hermitian) <= 1e-12


def test_planted_missing_adjoint_term_is_caught():
    # G(Z_e) in both terms of eq. 12 instead of G(Z_e) and G(Z_e)^H
    def bad(p, emin, emax, ne, Y):
        ct = O.contour(emin, emax, ne)
        R = O.assemble(p.Bd, p.Bu) @ Y
        Q = np.zeros(R.shape, dtype=np.complex128)
        for e in range(ne):
            x = O.factor_shift_hermitian(p, ct.Z[e]).solve(R)
            ph = np.exp(1j * ct.theta[e])
            Q -= (ct.w[e] / 4.0) * ct.r * (ph * x + np.conj(ph) * x)
        return Q
    p = W.hermitian_pencil(4, 5, 4)
    lam, _ = O.bruteforce_hermitian(p)
    emin, emax = gap_interval(lam, 6, 5)
    Y = W.random_complex_subspace(p.n, 7, 5)
    assert _hermitian_spectral_error(p, emin, emax, Y, bad) > 1e-3


@pytest.mark.parametrize("nc,b,seed,k0,m,extra", [
    (2, 3, 1, 1, 2, 2), (4, 5, 3, 5, 6, 4), (6, 8, 4, 10, 12, 6), (3, 7, 6, 4, 1, 2),
    (8, 16, 7, 40, 10, 8)])
def test_hermitian_feast_matches_bruteforce(nc, b, seed, k0, m, extra):
    p = W.hermitian_pencil(nc, b, seed)
    lam, Xb = O.bruteforce_hermitian(p)
    emin, emax = gap_interval(lam, k0, m)
    m0 = min(m + extra, p.n)
    Y0 = W.random_complex_subspace(p.n, m0, seed + 100)
    r = O.feast_hermitian(p, emin, emax, m0, 8, Y0, tol=1e-13, max_loops=40)
    assert r.status in (0, 4) and r.M == m
    ref = lam[k0:k0 + m]
    scale = np.maximum(np.abs(ref), (emax - emin) / 2)
    assert np.max(np.abs(r.lam[:m] - ref) / scale) <= 1e-12
    B = O.assemble(p.Bd, p.Bu)
    Xm = r.X[:, :m]
    assert np.max(np.abs(Xm.conj().T @ (B @ Xm) - np.eye(m))) <= 1e-12
    assert r.max_res <= 1e-11
    # the subspace is the brute-force one (principal angles)
    s = np.linalg.svd(Xb[:, k0:k0 + m].conj().T @ (B @ Xm), compute_uv=False)
    assert np.min(s) >= 1 - 1e-10


def test_hermitian_real_case_matches_real_path():
    # with a zero imaginary part, eq. 12 reduces to eq. 15 and the Hermitian
    # path returns the eigenvalues of the real symmetric one
    pr = tiny_pencil(5, 6, 8)
    ph = W.HermitianPencil(pr.Ad.astype(np.complex128), pr.Au.astype(np.complex128),
                           pr.Bd, pr.Bu)
    lam, _ = O.bruteforce(pr)
    emin, emax = gap_interval(lam, 8, 5)
    Y0 = W.random_subspace(pr.n, 9, 3)
    rr = O.feast(pr, emin, emax, 9, 8, Y0, tol=1e-13, max_loops=40)
    rh = O.feast_hermitian(ph, emin, emax, 9, 8, Y0.astype(np.complex128), tol=1e-13,
                           max_loops=40)
    assert rr.M == rh.M == 5
    assert np.max(np.abs(rr.lam[:5] - rh.lam[:5])) <= 1e-12 * np.max(np.abs(lam))
    Qr = O.filter_apply(pr, emin, emax, 8, Y0)
    Qh = O.filter_apply_hermitian(ph, emin, emax, 8, Y0.astype(np.complex128))
    assert np.max(np.abs(Qh.imag)) <= 1e-14 * np.max(np.abs(Qr))
    assert np.allclose(Qh.real, Qr, rtol=1e-12, atol=1e-14 * np.max(np.abs(Qr)))
