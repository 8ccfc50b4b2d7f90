"""CPU FP64 oracle for the FEAST hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module.  It shares no code with
the HIP library and must never be used as a fallback for it.

It follows E. Polizzi, "A Density Matrix-based Algorithm for Solving
Eigenvalue Problems", Sec. III, for a real symmetric A and s.p.d. B given in
block-tridiagonal storage (diag[nc][b][b], up[nc-1][b][b], lower block =
transpose of the upper one).  Everything is float64 / complex128.  Library
primitives serve as single steps: sparse matrix products, LAPACK's banded LU
(zgbtrf / zgbtrs) for the shifted solves, and LAPACK's symmetric-definite
eigensolver for the reduced problem.  There is no blocking, fusion or
reordering beyond what the paper's steps state.

Readings of points the paper leaves open (the same on the GPU path):
  * RHS of every refinement loop is B.Y with Y = Y0 first and Y = X after
    (Fig. 2 solves with Y at the first loop and with Y = BX later; one code
    path, equally random at the first loop).
  * An in-interval Ritz pair counts as an eigenvalue solution (Fig. 2 step
    5) once its relative residual is <= sqrt(tol): for a symmetric pencil the
    eigenvalue error is of the order of the squared residual, so such a pair
    is accurate to tol.  Pairs inside the interval with larger residuals are
    not counted (with M0 well above M, mixtures of eigenvectors from both
    sides of the interval that share a filter value give in-interval Ritz
    values with large residuals that persist over many loops).
  * Convergence: from the second loop on, stop when the number M of counted
    pairs is unchanged, the relative change of their trace
    |T_k - T_{k-1}| / max(|T_k|, M*r) is below tol (Sec. III.B (i) and Sec.
    IV.A give the trace test without fixing its denominator), and no
    uncounted in-interval pair is still converging: the smallest residual
    among them has not fallen below half its value of the previous loop.
    Without that last condition a slowly converging true pair that stays
    above the gate for two loops would be left out of M (with a small M0
    every pair can still be above it at loops 1 and 2, which ended the
    iteration with M = 0).  Fig. 2 step 5 counts every in-interval Ritz
    value, so loop counts differ from that literal rule (the nc=100 chain:
    3 loops here, 5 with the literal rule).
  * Residual of a pair: ||A x - lam B x||_1 / ||A x||_1 (Table I caption); if
    ||A x||_1 < r ||B x||_1 the denominator is ||B x||_1 max(|emin|,|emax|,r).
  * B_Q counts as numerically s.p.d. when its Cholesky factorisation exists
    with every pivot above 1e-12 times B_Q's diagonal entry in the same row
    (a scale-invariant test: scaling Q's columns leaves it unchanged).  If not
    (Sec. III.B (ii)), B_Q is diagonalised, directions with eigenvalue
    <= 1e-10 * max are dropped, and the dropped Ritz slots are returned last
    with lam = NaN, x = 0, status 2.
  * Output order: the M counted pairs first (ascending), then the other Ritz
    values (ascending), NaN slots last.  Membership is inclusive.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg
import scipy.sparse as sp
from scipy.linalg import lapack

# --------------------------------------------------------------------------
# Quadrature (Sec. III.B, eqs. 13-15 and the Gauss-Legendre rule of Fig. 2)
# --------------------------------------------------------------------------


def legendre_and_derivative(n: int, x: np.ndarray):
    """P_n(x) and P_n'(x) by the three-term recurrence
    (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}."""
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    # derivative: (1 - x^2) P_n' = n (P_{n-1} - x P_n)
    dp = n * (p0 - x * p1) / (1.0 - x * x)
    return p1, dp


def gauss_legendre(ne: int):
    """Nodes x_e (ascending) and weights w_e of the ne-point Gauss-Legendre rule
    on [-1, 1]: Newton's method on the roots of P_ne, w = 2 / ((1-x^2) P'(x)^2)."""
    if ne < 1:
        raise ValueError("ne must be >= 1")
    i = np.arange(1, ne + 1)
    x = np.cos(np.pi * (i - 0.25) / (ne + 0.5))
    for _ in range(100):
        p, dp = legendre_and_derivative(ne, x)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    p, dp = legendre_and_derivative(ne, x)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    order = np.argsort(x)
    return x[order], w[order]


@dataclasses.dataclass
class Contour:
    """Half-circle contour over [emin, emax] (eqs. 13-14) and the weights of
    the real-symmetric accumulation Q = -sum_e (w_e/2) Re{r e^{i theta_e} Q_e}
    (eq. 15 / Fig. 2 step 2), written as Q = sum_e Re(kappa_e Q_e)."""
    x: np.ndarray
    w: np.ndarray
    c: float
    r: float
    theta: np.ndarray
    Z: np.ndarray
    kappa: np.ndarray


def contour(emin: float, emax: float, ne: int) -> Contour:
    x, w = gauss_legendre(ne)
    r = (emax - emin) / 2.0
    c = (emax + emin) / 2.0
    theta = -(np.pi / 2.0) * (x - 1.0)
    Z = c + r * np.exp(1j * theta)
    kappa = -(w / 2.0) * r * np.exp(1j * theta)
    return Contour(x, w, c, r, theta, Z, kappa)


# --------------------------------------------------------------------------
# Random start (Fig. 2 step 1: M0 random vectors), seeded
# --------------------------------------------------------------------------
# Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
# as 1, 2, 3", SC'11): ten rounds of two 64x64 -> 128-bit products on a
# four-word counter, with a Weyl-sequence key schedule.

_PHILOX_MUL = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
_PHILOX_WEYL = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
_U32 = np.uint64(0xFFFFFFFF)


def _mulhilo64(a: np.ndarray, m: int):
    """High and low 64-bit words of a * m (a uint64 array, m a constant)."""
    m = np.uint64(m)
    a_lo, a_hi = a & _U32, a >> np.uint64(32)
    m_lo, m_hi = m & _U32, m >> np.uint64(32)
    ll, lh, hl, hh = a_lo * m_lo, a_lo * m_hi, a_hi * m_lo, a_hi * m_hi
    mid = (ll >> np.uint64(32)) + (lh & _U32) + (hl & _U32)
    hi = hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))
    return hi, a * m


def philox4x64_10(counter, key):
    """Philox4x64-10 of counters (4 uint64 arrays) under key (2 ints);
    returns the four output words."""
    c = [np.asarray(w, dtype=np.uint64).copy() for w in counter]
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = _mulhilo64(c[0], _PHILOX_MUL[0])
            hi1, lo1 = _mulhilo64(c[2], _PHILOX_MUL[1])
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
            k0 = k0 + np.uint64(_PHILOX_WEYL[0])
            k1 = k1 + np.uint64(_PHILOX_WEYL[1])
    return c


def random_start(seed: int, n: int, m0: int) -> np.ndarray:
    """Y0 [n][m0], standard normal: element t = i*m0 + j uses the Philox words
    of counter (t // 4, 0, 0, 0) under key (seed, 0); each word w gives the
    uniform u = (w >> 11) 2^-53 + 2^-54 in (0, 1), and Box-Muller on (u0, u1)
    and (u2, u3) gives sqrt(-2 ln u_a) cos(2 pi u_b) and ... sin(2 pi u_b);
    element t takes normal number t % 4."""
    t = np.arange(n * m0, dtype=np.uint64)
    zero = np.zeros_like(t)
    w = philox4x64_10([t >> np.uint64(2), zero, zero, zero], (seed, 0))
    u = [(wk >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 + 2.0 ** -54 for wk in w]
    lane = (t & np.uint64(3)).astype(np.int64)
    ua = np.where(lane < 2, u[0], u[2])
    ub = np.where(lane < 2, u[1], u[3])
    rho = np.sqrt(-2.0 * np.log(ua))
    ang = 2.0 * np.pi * ub
    z = np.where(lane % 2 == 0, rho * np.cos(ang), rho * np.sin(ang))
    return z.reshape(n, m0)


# --------------------------------------------------------------------------
# Block-tridiagonal matrices
# --------------------------------------------------------------------------


def assemble(diag: np.ndarray, up: np.ndarray) -> sp.csr_matrix:
    """Sparse matrix of a block-tridiagonal operator (lower block = up^T)."""
    nc = diag.shape[0]
    blocks = [[None] * nc for _ in range(nc)]
    for i in range(nc):
        blocks[i][i] = sp.csr_matrix(diag[i])
        if i + 1 < nc:
            blocks[i][i + 1] = sp.csr_matrix(up[i])
            blocks[i + 1][i] = sp.csr_matrix(up[i].T)
    if nc == 1:
        return sp.csr_matrix(diag[0])
    return sp.bmat(blocks, format="csr")


def bt_multiply(diag: np.ndarray, up: np.ndarray, V: np.ndarray) -> np.ndarray:
    """T @ V for a block-tridiagonal T given by (diag, up)."""
    return assemble(diag, up) @ V


# --------------------------------------------------------------------------
# Shifted solves (Fig. 2 step 2): (Z B - A) Q_e = R, LAPACK banded LU
# --------------------------------------------------------------------------


def shifted_matrix(p, z: complex) -> sp.csr_matrix:
    """z B - A as a complex sparse matrix."""
    A = assemble(p.Ad, p.Au).astype(np.complex128)
    B = assemble(p.Bd, p.Bu).astype(np.complex128)
    return (z * B - A).tocsr()


def band_storage(M: sp.spmatrix, kl: int, ku: int) -> np.ndarray:
    """LAPACK general band storage with kl extra rows for the LU fill:
    ab[kl + ku + i - j, j] = M[i, j]."""
    n = M.shape[0]
    ab = np.zeros((2 * kl + ku + 1, n), dtype=np.complex128)
    Mc = M.tocsr()
    for d in range(-kl, ku + 1):
        dg = Mc.diagonal(d)
        if d >= 0:
            ab[kl + ku - d, d:] = dg
        else:
            ab[kl + ku - d, :n + d] = dg
    return ab


class BandedLU:
    """Banded LU with partial pivoting of one shifted matrix (zgbtrf)."""

    def __init__(self, M: sp.spmatrix, half_band: int):
        self.n = M.shape[0]
        self.kl = self.ku = half_band
        ab = band_storage(M, self.kl, self.ku)
        self.lu, self.piv, info = lapack.zgbtrf(ab, self.kl, self.ku)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrf info={info}")

    def solve(self, R: np.ndarray, adjoint: bool = False) -> np.ndarray:
        """M^{-1} R, or M^{-H} R with ``adjoint`` (LAPACK trans = 'C')."""
        x, info = lapack.zgbtrs(self.lu, self.kl, self.ku,
                                np.asarray(R, dtype=np.complex128), self.piv,
                                trans=2 if adjoint else 0)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrs info={info}")
        return x


def factor_shift(p, z: complex) -> BandedLU:
    b = p.b
    half_band = 2 * b - 1 if p.nc > 1 else b - 1
    return BandedLU(shifted_matrix(p, z), max(half_band, 0))


def shifted_solve(p, z: complex, R: np.ndarray) -> np.ndarray:
    """Solve (z B - A) X = R (complex result)."""
    return factor_shift(p, z).solve(R)


# --------------------------------------------------------------------------
# One contour integration (Fig. 2 step 2) and the Rayleigh-Ritz steps
# --------------------------------------------------------------------------


def filter_apply(p, emin: float, emax: float, ne: int, Y: np.ndarray,
                 factors=None) -> np.ndarray:
    """Q = -sum_e (w_e/2) Re{ r e^{i theta_e} (Z_e B - A)^{-1} B Y }  (eq. 15)."""
    ct = contour(emin, emax, ne)
    B = assemble(p.Bd, p.Bu)
    R = B @ Y
    Q = np.zeros(R.shape, dtype=np.float64)
    for e in range(ne):
        lu = factors[e] if factors is not None else factor_shift(p, ct.Z[e])
        Qe = lu.solve(R)
        Q -= (ct.w[e] / 2.0) * np.real(ct.r * np.exp(1j * ct.theta[e]) * Qe)
    return Q


def project(p, Q: np.ndarray):
    """A_Q = Q^T A Q and B_Q = Q^T B Q (eq. 7), symmetrised."""
    A = assemble(p.Ad, p.Au)
    B = assemble(p.Bd, p.Bu)
    AQ = Q.T @ (A @ Q)
    BQ = Q.T @ (B @ Q)
    return 0.5 * (AQ + AQ.T), 0.5 * (BQ + BQ.T)


def reduced_eig(AQ: np.ndarray, BQ: np.ndarray):
    """Solve A_Q Phi = eps B_Q Phi with Phi^T B_Q Phi = I (eqs. 6-9).

    Returns (eps ascending, Phi, fallback_used).  B_Q is taken as s.p.d.
    when its Cholesky pivots L_kk^2 all exceed 1e-12 * B_Q(k, k): a pivot
    at rounding level relative to its own column means a numerically null
    direction (a column that depends on the ones before it), whose whitening
    would amplify rounding errors; the test does not depend on the scaling
    of Q's columns, which the filter spreads over many orders of magnitude.
    If it is not, the problem is solved in the span of B_Q's eigenvectors
    with eigenvalue > 1e-10 * max; dropped slots get eps = NaN and Phi
    column 0, last."""
    m0 = AQ.shape[0]
    spd = False
    try:
        L = np.linalg.cholesky(BQ)
        spd = bool(np.all(np.diag(L) ** 2 > 1e-12 * np.diag(BQ)))
    except np.linalg.LinAlgError:
        pass
    if spd:
        try:
            eps, Phi = scipy.linalg.eigh(AQ, BQ)
            return eps, Phi, False
        except np.linalg.LinAlgError:
            pass
    mu, V = np.linalg.eigh(BQ)
    keep = mu > 1e-10 * np.max(mu)
    T = V[:, keep] / np.sqrt(mu[keep])
    eps_k, W = np.linalg.eigh(T.T @ AQ @ T)
    eps = np.full(m0, np.nan)
    Phi = np.zeros((m0, m0))
    k = int(keep.sum())
    eps[:k] = eps_k
    Phi[:, :k] = T @ W
    return eps, Phi, True


def residuals(p, lam: np.ndarray, X: np.ndarray, emin: float, emax: float) -> np.ndarray:
    """Per column ||A x - lam B x||_1 / ||A x||_1 (Table I caption), with the
    small-||Ax|| guard described in the module docstring."""
    A = assemble(p.Ad, p.Au)
    B = assemble(p.Bd, p.Bu)
    AX = A @ X
    BX = B @ X
    r = (emax - emin) / 2.0
    num = np.sum(np.abs(AX - BX * lam[None, :]), axis=0)
    na = np.sum(np.abs(AX), axis=0)
    nb = np.sum(np.abs(BX), axis=0)
    den = np.where(na < r * nb, nb * max(abs(emin), abs(emax), r), na)
    with np.errstate(invalid="ignore", divide="ignore"):
        return num / den


def counted(eps: np.ndarray, res: np.ndarray, emin: float, emax: float,
            tol: float) -> np.ndarray:
    """Mask of the Ritz pairs that count as eigenvalue solutions: inside the
    interval (inclusive) with relative residual <= sqrt(tol)."""
    with np.errstate(invalid="ignore"):
        return (eps >= emin) & (eps <= emax) & (res <= np.sqrt(tol))


# An uncounted in-interval pair whose residual fell below this fraction of
# the previous loop's smallest uncounted residual is still converging.
UNCOUNTED_DROP = 0.5


def smallest_uncounted_residual(eps: np.ndarray, res: np.ndarray, mask: np.ndarray,
                                emin: float, emax: float) -> float:
    """Smallest residual among the in-interval Ritz pairs that are not counted
    (inf if there is none).  Convergence waits while it keeps falling: a true
    eigenpair that has not yet reached the counting gate shrinks its residual
    every loop, a mixture of eigenvectors from both sides of the interval
    does not."""
    with np.errstate(invalid="ignore"):
        left = (eps >= emin) & (eps <= emax) & ~mask
    return float(np.min(res[left])) if left.any() else np.inf


def order_ritz(eps: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Permutation: counted pairs first (ascending), then the other finite
    Ritz values (ascending), NaN slots last."""
    idx = np.arange(len(eps))
    finite = np.isfinite(eps)
    a = idx[mask]
    b_ = idx[~mask & finite]
    c = idx[~finite]
    return np.concatenate([a[np.argsort(eps[a], kind="stable")],
                           b_[np.argsort(eps[b_], kind="stable")], c])


@dataclasses.dataclass
class FeastResult:
    lam: np.ndarray
    X: np.ndarray
    res: np.ndarray
    M: int
    loops: int
    trace: float
    trace_rel: float
    max_res: float
    status: int
    traces: list
    counts: list


def feast(p, emin: float, emax: float, m0: int, ne: int, Y0: np.ndarray,
          tol: float = 1e-12, max_loops: int = 20, log=None) -> FeastResult:
    """Fig. 2: FEAST for A x = lam B x, A real symmetric, B s.p.d.
    ``log(k, M_k, T_k, trace_rel)`` is called after every loop if given."""
    ct = contour(emin, emax, ne)
    factors = [factor_shift(p, ct.Z[e]) for e in range(ne)]   # once (Sec. V (ii))
    Y = np.array(Y0, dtype=np.float64, copy=True)
    traces, counts = [], []
    converged = False
    fallback = False
    trace_rel = np.inf
    prev_left_min = np.inf
    for k in range(1, max_loops + 1):
        Q = filter_apply(p, emin, emax, ne, Y, factors)
        AQ, BQ = project(p, Q)
        eps, Phi, fallback = reduced_eig(AQ, BQ)
        X = Q @ Phi
        res = residuals(p, eps, X, emin, emax)
        inside = counted(eps, res, emin, emax, tol)
        left_min = smallest_uncounted_residual(eps, res, inside, emin, emax)
        still_converging = left_min < UNCOUNTED_DROP * prev_left_min
        prev_left_min = left_min
        Mk = int(inside.sum())
        Tk = float(np.sum(eps[inside]))
        if k >= 2:
            if Mk == 0 and counts[-1] == 0:
                trace_rel = 0.0
            else:
                trace_rel = abs(Tk - traces[-1]) / max(abs(Tk), Mk * ct.r)
        traces.append(Tk)
        counts.append(Mk)
        if log is not None:
            log(k, Mk, Tk, trace_rel)
        if k >= 2 and Mk == counts[-2] and trace_rel < tol and not still_converging:
            converged = True
            break
        Y = X
    perm = order_ritz(eps, inside)
    lam = eps[perm]
    X = X[:, perm]
    res = res[perm]
    M = counts[-1]
    max_res = float(np.max(res[:M])) if M > 0 else 0.0
    if not converged:
        status = 1
    elif fallback:
        status = 2
    elif M == m0:
        status = 4
    elif M == 0:
        status = 3
    else:
        status = 0
    return FeastResult(lam, X, res, M, len(traces), traces[-1], float(trace_rel),
                       max_res, status, traces, counts)


# --------------------------------------------------------------------------
# Hermitian A (Sec. III.B, eq. 12 and the changes listed after Fig. 2)
# --------------------------------------------------------------------------
# A complex Hermitian, B real s.p.d.; Y, Q, Phi and X complex.  Same readings
# as above (RHS B Y, counting gate, convergence, residual, B_Q test).


def assemble_hermitian(diag: np.ndarray, up: np.ndarray) -> sp.csr_matrix:
    """Sparse matrix of a block-tridiagonal Hermitian operator (lower block =
    conjugate transpose of the upper one)."""
    nc = diag.shape[0]
    if nc == 1:
        return sp.csr_matrix(diag[0])
    blocks = [[None] * nc for _ in range(nc)]
    for i in range(nc):
        blocks[i][i] = sp.csr_matrix(diag[i])
        if i + 1 < nc:
            blocks[i][i + 1] = sp.csr_matrix(up[i])
            blocks[i + 1][i] = sp.csr_matrix(up[i].conj().T)
    return sp.bmat(blocks, format="csr")


def shifted_matrix_hermitian(p, z: complex) -> sp.csr_matrix:
    """z B - A for a Hermitian pencil."""
    A = assemble_hermitian(p.Ad, p.Au)
    B = assemble(p.Bd, p.Bu).astype(np.complex128)
    return (z * B - A).tocsr()


def factor_shift_hermitian(p, z: complex) -> BandedLU:
    b = p.b
    half_band = 2 * b - 1 if p.nc > 1 else b - 1
    return BandedLU(shifted_matrix_hermitian(p, z), max(half_band, 0))


def filter_apply_hermitian(p, emin: float, emax: float, ne: int, Y: np.ndarray,
                           factors=None) -> np.ndarray:
    """Eq. 12 with RHS B Y: Q = -sum_e (w_e/4) r (e^{i theta_e} G(Z_e)
    + e^{-i theta_e} G(Z_e)^H) B Y, G(Z) = (Z B - A)^{-1}; the adjoint solve
    reuses the factorisation of Z_e B - A (G(conj Z) = G(Z)^H)."""
    ct = contour(emin, emax, ne)
    B = assemble(p.Bd, p.Bu)
    R = B @ np.asarray(Y, dtype=np.complex128)
    Q = np.zeros(R.shape, dtype=np.complex128)
    for e in range(ne):
        lu = factors[e] if factors is not None else factor_shift_hermitian(p, ct.Z[e])
        x = lu.solve(R)
        y = lu.solve(R, adjoint=True)
        ph = np.exp(1j * ct.theta[e])
        Q -= (ct.w[e] / 4.0) * ct.r * (ph * x + np.conj(ph) * y)
    return Q


def project_hermitian(p, Q: np.ndarray):
    """A_Q = Q^H A Q and B_Q = Q^H B Q, Hermitian parts."""
    A = assemble_hermitian(p.Ad, p.Au)
    B = assemble(p.Bd, p.Bu)
    AQ = Q.conj().T @ (A @ Q)
    BQ = Q.conj().T @ (B @ Q)
    return 0.5 * (AQ + AQ.conj().T), 0.5 * (BQ + BQ.conj().T)


def reduced_eig_hermitian(AQ: np.ndarray, BQ: np.ndarray):
    """Complex Hermitian version of reduced_eig (same B_Q test and fallback)."""
    m0 = AQ.shape[0]
    spd = False
    try:
        L = np.linalg.cholesky(BQ)
        spd = bool(np.all(np.abs(np.diag(L)) ** 2 > 1e-12 * np.real(np.diag(BQ))))
    except np.linalg.LinAlgError:
        pass
    if spd:
        try:
            eps, Phi = scipy.linalg.eigh(AQ, BQ)
            return eps, Phi, False
        except np.linalg.LinAlgError:
            pass
    mu, V = np.linalg.eigh(BQ)
    keep = mu > 1e-10 * np.max(mu)
    T = V[:, keep] / np.sqrt(mu[keep])
    eps_k, W = np.linalg.eigh(T.conj().T @ AQ @ T)
    eps = np.full(m0, np.nan)
    Phi = np.zeros((m0, m0), dtype=np.complex128)
    k = int(keep.sum())
    eps[:k] = eps_k
    Phi[:, :k] = T @ W
    return eps, Phi, True


def residuals_hermitian(p, lam: np.ndarray, X: np.ndarray, emin: float,
                        emax: float) -> np.ndarray:
    """Per column ||A x - lam B x||_1 / ||A x||_1 with complex moduli, and the
    small-||Ax|| guard of the real case."""
    A = assemble_hermitian(p.Ad, p.Au)
    B = assemble(p.Bd, p.Bu)
    AX = A @ X
    BX = B @ X
    r = (emax - emin) / 2.0
    num = np.sum(np.abs(AX - BX * lam[None, :]), axis=0)
    na = np.sum(np.abs(AX), axis=0)
    nb = np.sum(np.abs(BX), axis=0)
    den = np.where(na < r * nb, nb * max(abs(emin), abs(emax), r), na)
    with np.errstate(invalid="ignore", divide="ignore"):
        return num / den


def feast_hermitian(p, emin: float, emax: float, m0: int, ne: int, Y0: np.ndarray,
                    tol: float = 1e-12, max_loops: int = 20) -> FeastResult:
    """Fig. 2 with the Hermitian changes: complex Y, Q, Phi and X, eq. 12."""
    ct = contour(emin, emax, ne)
    factors = [factor_shift_hermitian(p, ct.Z[e]) for e in range(ne)]
    Y = np.array(Y0, dtype=np.complex128, copy=True)
    traces, counts = [], []
    converged = False
    fallback = False
    trace_rel = np.inf
    prev_left_min = np.inf
    for k in range(1, max_loops + 1):
        Q = filter_apply_hermitian(p, emin, emax, ne, Y, factors)
        AQ, BQ = project_hermitian(p, Q)
        eps, Phi, fallback = reduced_eig_hermitian(AQ, BQ)
        X = Q @ Phi
        res = residuals_hermitian(p, eps, X, emin, emax)
        inside = counted(eps, res, emin, emax, tol)
        left_min = smallest_uncounted_residual(eps, res, inside, emin, emax)
        still_converging = left_min < UNCOUNTED_DROP * prev_left_min
        prev_left_min = left_min
        Mk = int(inside.sum())
        Tk = float(np.sum(eps[inside]))
        if k >= 2:
            if Mk == 0 and counts[-1] == 0:
                trace_rel = 0.0
            else:
                trace_rel = abs(Tk - traces[-1]) / max(abs(Tk), Mk * ct.r)
        traces.append(Tk)
        counts.append(Mk)
        if k >= 2 and Mk == counts[-2] and trace_rel < tol and not still_converging:
            converged = True
            break
        Y = X
    perm = order_ritz(eps, inside)
    lam, X, res = eps[perm], X[:, perm], res[perm]
    M = counts[-1]
    max_res = float(np.max(res[:M])) if M > 0 else 0.0
    if not converged:
        status = 1
    elif fallback:
        status = 2
    elif M == m0:
        status = 4
    elif M == 0:
        status = 3
    else:
        status = 0
    return FeastResult(lam, X, res, M, len(traces), traces[-1], float(trace_rel),
                       max_res, status, traces, counts)


def bruteforce_hermitian(p):
    """All eigenpairs of the dense Hermitian pencil (LAPACK)."""
    A = assemble_hermitian(p.Ad, p.Au).toarray()
    B = assemble(p.Bd, p.Bu).toarray()
    return scipy.linalg.eigh(A, B)


# --------------------------------------------------------------------------
# Independent references used to pin the oracle
# --------------------------------------------------------------------------


def bruteforce(p):
    """All eigenpairs of the dense pencil (LAPACK symmetric-definite solver)."""
    A = assemble(p.Ad, p.Au).toarray()
    B = assemble(p.Bd, p.Bu).toarray()
    return scipy.linalg.eigh(A, B)


def inertia_count_hermitian(p, sigma: float) -> int:
    """Number of eigenvalues below sigma of a Hermitian pencil (A complex
    Hermitian, B real s.p.d.): negative eigenvalues of the block LDL^H Schur
    complements S_1 = K_11, S_{i+1} = K_{i+1,i+1} - C_i^H S_i^{-1} C_i of
    K = A - sigma B (Sylvester's law of inertia for Hermitian forms)."""
    K = p.Ad - sigma * p.Bd
    C = p.Au - sigma * p.Bu
    count = 0
    S = K[0].copy()
    for i in range(p.nc):
        ev = np.linalg.eigvalsh(0.5 * (S + S.conj().T))
        count += int(np.sum(ev < 0))
        if i + 1 < p.nc:
            S = K[i + 1] - C[i].conj().T @ np.linalg.solve(S, C[i])
    return count


def inertia_count(p, sigma: float) -> int:
    """Number of eigenvalues of (A, B) below sigma: negative eigenvalues of
    A - sigma B (Sylvester's law of inertia), summed over the block LDL^T
    Schur complements S_1 = K_11, S_{i+1} = K_{i+1,i+1} - C_i^T S_i^{-1} C_i
    (Haynsworth inertia additivity)."""
    K = p.Ad - sigma * p.Bd
    C = p.Au - sigma * p.Bu
    count = 0
    S = K[0].copy()
    for i in range(p.nc):
        ev = np.linalg.eigvalsh(0.5 * (S + S.T))
        count += int(np.sum(ev < 0))
        if i + 1 < p.nc:
            S = K[i + 1] - C[i].T @ np.linalg.solve(S, C[i])
    return count
