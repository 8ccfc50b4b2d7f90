// Reduced generalized eigenproblem of the Rayleigh-Ritz step (Sec. III.A,
// eqs. 6-9): A_Q Phi = eps B_Q Phi with Phi^T B_Q Phi = I, for M0 <= 128, in
// one workgroup, all in float64.
//
//  1. Whitening T with T^T B_Q T = I: T = L^{-T} from the Cholesky factor
//     B_Q = L L^T.  If a Cholesky pivot is not positive (B_Q not numerically
//     s.p.d., Sec. III.B (ii)), B_Q = V diag(mu) V^T is diagonalised instead,
//     T = V diag(mu^{-1/2}) on the directions with mu > 1e-14 max(mu), and
//     the other columns of T are zero.
//  2. C = T^T A_Q T, diagonalised by cyclic two-sided Jacobi rotations in a
//     round-robin order (all n/2 disjoint rotations of a round at once);
//     a rotation is skipped when |c_pq| <= 2^-53 sqrt(|c_pp c_qq|) or
//     |c_pq| <= 2^-56 ||C||_F, and the sweeps stop after a sweep without
//     rotations.
//  3. eps ascending (dropped directions: NaN, last), Phi = T V.
#include "common.h"
#include "kernels.h"

namespace feast {
namespace {

constexpr int kThreads = 1024;
constexpr int kMaxN = 128;

struct RRShared {
  int pp[kMaxN / 2], pq[kMaxN / 2];
  double cs[kMaxN / 2], sn[kMaxN / 2];
  int rot;
  int fail;
  double norm;
  double red[kThreads];
  int dropped[kMaxN];
  int rank[kMaxN];
  double diag[kMaxN];
};

__device__ __forceinline__ int rr_player(int s, int i, int nn) {
  // circle method: player 0 fixed, the others rotate by one place a round
  return i == 0 ? 0 : 1 + ((i - 1 + s) % (nn - 1));
}

// Cyclic Jacobi on the nn x nn symmetric matrix C (LDS, row stride ldc);
// V (global, nn x nn, row-major) accumulates the rotations.
__device__ int jacobi(double *C, int ldc, double *V, int nn, RRShared &sh) {
  const int tid = threadIdx.x;
  const int half = nn / 2;
  const double eps = 1.1102230246251565e-16;  // 2^-53
  // absolute floor: off-diagonal entries below eps * ||C||_F / 8 are rounding
  // noise of earlier rotations and are not rotated away
  {
    double part = 0.0;
    for (int idx = tid; idx < nn * nn; idx += kThreads) {
      const double v = C[(idx / nn) * ldc + idx % nn];
      part += v * v;
    }
    sh.red[tid] = part;
  }
  __syncthreads();
  if (tid == 0) {  // fixed summation order: bitwise reproducible
    double s = 0.0;
    for (int i = 0; i < kThreads; ++i) s += sh.red[i];
    sh.norm = s;
  }
  __syncthreads();
  const double floor_abs = 0.125 * eps * sqrt(sh.norm);
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    if (tid == 0) sh.rot = 0;
    __syncthreads();
    for (int s = 0; s < nn - 1; ++s) {
      if (tid < half) {
        int u = rr_player(s, tid, nn), v = rr_player(s, nn - 1 - tid, nn);
        int p = u < v ? u : v, q = u < v ? v : u;
        double app = C[p * ldc + p], aqq = C[q * ldc + q], apq = C[p * ldc + q];
        double c = 1.0, sgn = 0.0;
        if (fabs(apq) > floor_abs && fabs(apq) > eps * sqrt(fabs(app * aqq))) {
          double tau = (aqq - app) / (2.0 * apq);
          double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sgn = t * c;
          atomicAdd(&sh.rot, 1);
        }
        sh.pp[tid] = p;
        sh.pq[tid] = q;
        sh.cs[tid] = c;
        sh.sn[tid] = sgn;
      }
      __syncthreads();
      // C <- J^T C J on 2x2 blocks (a <= b), mirrored to keep C symmetric
      for (int idx = tid; idx < half * half; idx += kThreads) {
        const int a = idx / half, bq = idx % half;
        if (a > bq) continue;
        const int pa = sh.pp[a], qa = sh.pq[a], pb = sh.pp[bq], qb = sh.pq[bq];
        const double ca = sh.cs[a], sa = sh.sn[a], cb = sh.cs[bq], sb = sh.sn[bq];
        if (a == bq) {
          const double app = C[pa * ldc + pa], aqq = C[qa * ldc + qa], apq = C[pa * ldc + qa];
          if (sa != 0.0) {
            const double t = sa / ca;
            C[pa * ldc + pa] = app - t * apq;
            C[qa * ldc + qa] = aqq + t * apq;
            C[pa * ldc + qa] = 0.0;
            C[qa * ldc + pa] = 0.0;
          }
          continue;
        }
        const double x11 = C[pa * ldc + pb], x12 = C[pa * ldc + qb];
        const double x21 = C[qa * ldc + pb], x22 = C[qa * ldc + qb];
        const double y11 = cb * x11 - sb * x12, y12 = sb * x11 + cb * x12;
        const double y21 = cb * x21 - sb * x22, y22 = sb * x21 + cb * x22;
        const double z11 = ca * y11 - sa * y21, z21 = sa * y11 + ca * y21;
        const double z12 = ca * y12 - sa * y22, z22 = sa * y12 + ca * y22;
        C[pa * ldc + pb] = z11; C[pb * ldc + pa] = z11;
        C[pa * ldc + qb] = z12; C[qb * ldc + pa] = z12;
        C[qa * ldc + pb] = z21; C[pb * ldc + qa] = z21;
        C[qa * ldc + qb] = z22; C[qb * ldc + qa] = z22;
      }
      // V <- V J
      for (int idx = tid; idx < nn * half; idx += kThreads) {
        const int r = idx / half, a = idx % half;
        const double sa = sh.sn[a];
        if (sa == 0.0) continue;
        const double ca = sh.cs[a];
        const int pa = sh.pp[a], qa = sh.pq[a];
        const double vp = V[r * nn + pa], vq = V[r * nn + qa];
        V[r * nn + pa] = ca * vp - sa * vq;
        V[r * nn + qa] = sa * vp + ca * vq;
      }
      __syncthreads();
    }
    const int rot = sh.rot;
    __syncthreads();
    if (rot == 0) break;
  }
  return sweep;
}

__global__ __launch_bounds__(kThreads) void reduced_eig_kernel(const double *AQ, const double *BQ,
                                                               int n, double *eps, double *Phi,
                                                               double *scratch, int *flag) {
  extern __shared__ double C[];
  __shared__ RRShared sh;
  const int tid = threadIdx.x;
  const int nn = n + (n & 1);
  const int ldc = nn + 1;
  double *T = scratch;                 // nn x nn whitening
  double *T1 = scratch + nn * nn;      // nn x nn product
  double *V = scratch + 2 * nn * nn;   // nn x nn rotations
  double *Lg = scratch + 3 * nn * nn;  // nn x nn L^{-1}

  for (int idx = tid; idx < nn * nn; idx += kThreads) {
    const int i = idx / nn, j = idx % nn;
    C[i * ldc + j] = (i < n && j < n) ? BQ[i * n + j] : 0.0;
  }
  if (tid == 0) sh.fail = 0;
  if (tid < kMaxN) sh.dropped[tid] = (tid >= n);
  __syncthreads();

  // ---- Cholesky B_Q = L L^T (lower triangle of C) ----
  for (int k = 0; k < n; ++k) {
    const double d = C[k * ldc + k];
    if (!(d > 0.0) || !isfinite(d)) {  // uniform decision
      if (tid == 0) sh.fail = 1;
      break;
    }
    const double lkk = sqrt(d);
    __syncthreads();
    for (int i = k + tid; i < n; i += kThreads)
      C[i * ldc + k] = (i == k) ? lkk : C[i * ldc + k] / lkk;
    __syncthreads();
    const int m = n - k - 1;
    for (int idx = tid; idx < m * m; idx += kThreads) {
      const int i = k + 1 + idx / m, j = k + 1 + idx % m;
      if (j <= i) C[i * ldc + j] -= C[i * ldc + k] * C[j * ldc + k];
    }
    __syncthreads();
  }
  __syncthreads();
  const bool fallback = sh.fail != 0;

  if (!fallback) {
    // L^{-1} by columns (forward substitution), then T = L^{-T}
    if (tid < n) {
      const int j = tid;
      for (int i = 0; i < n; ++i) {
        double x;
        if (i < j) {
          x = 0.0;
        } else if (i == j) {
          x = 1.0 / C[i * ldc + i];
        } else {
          double s = 0.0;
          for (int k = j; k < i; ++k) s += C[i * ldc + k] * Lg[k * nn + j];
          x = -s / C[i * ldc + i];
        }
        Lg[i * nn + j] = x;
      }
    }
    __syncthreads();
    for (int idx = tid; idx < nn * nn; idx += kThreads) {
      const int i = idx / nn, j = idx % nn;
      T[idx] = (i < n && j < n) ? Lg[j * nn + i] : 0.0;
    }
  } else {
    // eigen-decomposition of B_Q, drop directions with mu <= 1e-14 max
    for (int idx = tid; idx < nn * nn; idx += kThreads) {
      const int i = idx / nn, j = idx % nn;
      C[i * ldc + j] = (i < n && j < n) ? BQ[i * n + j] : 0.0;
      V[idx] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int fsweeps = jacobi(C, ldc, V, nn, sh);
    if (tid == 0) flag[2] = fsweeps;
    if (tid < nn) sh.diag[tid] = C[tid * ldc + tid];
    __syncthreads();
    double mumax = 0.0;
    for (int i = 0; i < n; ++i) mumax = fmax(mumax, sh.diag[i]);
    if (tid < n) sh.dropped[tid] = !(sh.diag[tid] > 1e-14 * mumax);
    __syncthreads();
    for (int idx = tid; idx < nn * nn; idx += kThreads) {
      const int i = idx / nn, j = idx % nn;
      T[idx] = (i < n && j < n && !sh.dropped[j]) ? V[idx] / sqrt(sh.diag[j]) : 0.0;
    }
  }
  __syncthreads();

  // ---- C = T^T A_Q T ----
  for (int idx = tid; idx < nn * nn; idx += kThreads) {
    const int i = idx / nn, j = idx % nn;
    double s = 0.0;
    if (i < n)
      for (int k = 0; k < n; ++k) s += AQ[i * n + k] * T[k * nn + j];
    T1[idx] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < nn * nn; idx += kThreads) {
    const int i = idx / nn, j = idx % nn;
    if (j < i) continue;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += T[k * nn + i] * T1[k * nn + j];
    C[i * ldc + j] = s;
    C[j * ldc + i] = s;
  }
  for (int idx = tid; idx < nn * nn; idx += kThreads) V[idx] = (idx / nn == idx % nn) ? 1.0 : 0.0;
  __syncthreads();

  const int sweeps = jacobi(C, ldc, V, nn, sh);
  if (tid == 0) flag[1] = sweeps;

  // ---- sort ascending, dropped directions (NaN) last ----
  if (tid < nn) sh.diag[tid] = C[tid * ldc + tid];
  __syncthreads();
  if (tid < n) {
    const int i = tid;
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const bool dj = sh.dropped[j], di = sh.dropped[i];
      bool before;
      if (di != dj) before = !dj;            // kept ones come first
      else if (di) before = j < i;           // dropped: keep index order
      else before = (sh.diag[j] < sh.diag[i]) || (sh.diag[j] == sh.diag[i] && j < i);
      rk += before;
    }
    sh.rank[i] = rk;
    eps[rk] = sh.dropped[i] ? __longlong_as_double(0x7ff8000000000000LL) : sh.diag[i];
  }
  __syncthreads();
  // Phi[:, rank[i]] = T V[:, i]
  for (int idx = tid; idx < n * n; idx += kThreads) {
    const int r = idx / n, i = idx % n;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += T[r * nn + k] * V[k * nn + i];
    Phi[r * n + sh.rank[i]] = s;
  }
  if (tid == 0) flag[0] = fallback ? 1 : 0;
}

}  // namespace

hipError_t launch_reduced_eig(const double *AQ, const double *BQ, int n, double *eps, double *Phi,
                              double *scratch, int *flag, hipStream_t st) {
  if (n < 1 || n > kMaxN) return hipErrorInvalidValue;
  const int nn = n + (n & 1);
  const size_t shm = (size_t)nn * (nn + 1) * sizeof(double);
  hipError_t err = hipFuncSetAttribute((const void *)reduced_eig_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(reduced_eig_kernel, dim3(1), dim3(kThreads), shm, st, AQ, BQ, n, eps, Phi,
                     scratch, flag);
  return hipGetLastError();
}

}  // namespace feast
