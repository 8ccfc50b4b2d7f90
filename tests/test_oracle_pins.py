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
