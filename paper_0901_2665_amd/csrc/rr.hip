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
//     a rotation is skipped when |c_pq| <= u sqrt(|c_pp c_qq|) or
//     |c_pq| <= u ||C||_F / 8 (u = 2^-53), and the sweeps stop after a sweep
//     without rotations.
//  3. eps ascending (dropped directions: NaN, last), Phi = T V.
#include "common.h"
#include "kernels.h"

namespace feast {
namespace {

constexpr int kThreads = 1024;
constexpr int kMaxN = 128;

struct RRShared {
  double2 csn[kMaxN / 2];  // (cos, sin) of the rotation of each pair slot
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
  // (0 <= s < nn - 1, so one conditional subtraction is the modulo)
  if (i == 0) return 0;
  int x = i - 1 + s;
  if (x >= nn - 1) x -= nn - 1;
  return 1 + x;
}

constexpr int kMaxSweeps = 60;

// Cyclic Jacobi on the nn x nn symmetric matrix C (LDS, row stride ldc).
// The rotations of every round are appended to rlog (global, 2 * nn/2
// doubles a round: cosines then sines); the eigenvectors are rebuilt from
// the log afterwards (replay_rotations), so a round touches only C.
// Returns the number of sweeps that rotated (the final check sweep, which
// rotates nothing, is not counted).
__device__ int jacobi(double *C, int ldc, double *rlog, int nn, RRShared &sh) {
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
  // The sweeps keep only the upper triangle of C up to date (entry (i, j) is
  // read and written at (min, max)).  The 2x2 blocks (a, b), a <= b, of the
  // pair slots are dealt out to the threads once; a thread keeps its blocks
  // (at most 3 for nn <= 128) in registers.
  constexpr int kPer = (kMaxN / 2 * (kMaxN / 2 + 1) / 2 + kThreads - 1) / kThreads;
  const int nblk = half * (half + 1) / 2;
  int ba[kPer], bb[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    int idx = tid + t * kThreads;
    ba[t] = -1;
    bb[t] = -1;
    if (idx < nblk) {  // row a of the block triangle holds half - a blocks
      int a = 0;
      while (idx >= half - a) {
        idx -= half - a;
        ++a;
      }
      ba[t] = a;
      bb[t] = a + idx;
    }
  }
  auto at = [&](int i, int j) -> double & {
    return i < j ? C[i * ldc + j] : C[j * ldc + i];
  };
  int sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) sh.rot = 0;
    __syncthreads();
    for (int s = 0; s < nn - 1; ++s) {
      if (tid < half) {  // one wave: rotation of slot tid
        const int u = rr_player(s, tid, nn), v = rr_player(s, nn - 1 - tid, nn);
        const int p = u < v ? u : v, q = u < v ? v : u;
        const double app = C[p * ldc + p], aqq = C[q * ldc + q], apq = C[p * ldc + q];
        double c = 1.0, sgn = 0.0;
        const bool rotate =
            fabs(apq) > floor_abs && fabs(apq) > eps * sqrt(fabs(app * aqq));
        if (rotate) {
          // t = tan of the rotation angle: the smaller root of t^2 + 2 tau t - 1
          const double tau = (aqq - app) * rcp_newton(2.0 * apq);
          const double ata = fabs(tau);
          const double root = ata < 1e150 ? sqrt(1.0 + tau * tau) : ata;
          const double t = (tau >= 0.0 ? 1.0 : -1.0) * rcp_newton(ata + root);
          c = rcp_newton(sqrt(1.0 + t * t));
          sgn = t * c;
        }
        const unsigned long long m = __ballot(rotate);
        if (tid == 0) sh.rot += __popcll(m);
        sh.csn[tid] = double2{c, sgn};
        double *lg = rlog + (size_t)(sweep * (nn - 1) + s) * 2 * half;
        lg[tid] = c;
        lg[half + tid] = sgn;
      }
      __syncthreads();
      // C <- J^T C J on the thread's 2x2 blocks
#pragma unroll
      for (int t = 0; t < kPer; ++t) {
        const int a = ba[t], bq = bb[t];
        if (a < 0) continue;
        const double2 ra = sh.csn[a], rb = sh.csn[bq];
        const double ca = ra.x, sa = ra.y, cb = rb.x, sb = rb.y;
        int pa = rr_player(s, a, nn), qa = rr_player(s, nn - 1 - a, nn);
        if (pa > qa) { const int x = pa; pa = qa; qa = x; }
        if (a == bq) {
          if (sa != 0.0) {
            const double app = C[pa * ldc + pa], aqq = C[qa * ldc + qa], apq = C[pa * ldc + qa];
            const double tq = sa / ca;
            C[pa * ldc + pa] = app - tq * apq;
            C[qa * ldc + qa] = aqq + tq * apq;
            C[pa * ldc + qa] = 0.0;
          }
          continue;
        }
        if (sa == 0.0 && sb == 0.0) continue;
        int pb = rr_player(s, bq, nn), qb = rr_player(s, nn - 1 - bq, nn);
        if (pb > qb) { const int x = pb; pb = qb; qb = x; }
        double &e11 = at(pa, pb), &e12 = at(pa, qb), &e21 = at(qa, pb), &e22 = at(qa, qb);
        const double x11 = e11, x12 = e12, x21 = e21, x22 = e22;
        const double y11 = cb * x11 - sb * x12, y12 = sb * x11 + cb * x12;
        const double y21 = cb * x21 - sb * x22, y22 = sb * x21 + cb * x22;
        e11 = ca * y11 - sa * y21;
        e21 = sa * y11 + ca * y21;
        e12 = ca * y12 - sa * y22;
        e22 = sa * y12 + ca * y22;
      }
      __syncthreads();
    }
    const int rot = sh.rot;
    __syncthreads();
    if (rot == 0) break;
  }
  return sweep;  // sweeps with at least one rotation (all of them if not converged)
}

// V = J_1 J_2 ... J_R for the logged rounds, V (LDS, row stride ldv) starts
// as the identity.  A round rotates column pairs, so the rows of V evolve
// independently: each wave owns nn/16 rows (eight lanes a row, each lane a
// fixed set of pairs) and runs through all rounds without workgroup
// barriers; LDS accesses of one wave are ordered by a wave-level fence.
__device__ void replay_rotations(double *V, int ldv, const double *rlog, int rounds, int nn) {
  const int tid = threadIdx.x;
  const int half = nn / 2;
  for (int idx = tid; idx < nn * nn; idx += kThreads)
    V[(idx / nn) * ldv + idx % nn] = (idx / nn == idx % nn) ? 1.0 : 0.0;
  __syncthreads();
  const int w = tid >> 6, l = tid & 63;
  const int rows_per_wave = (nn + 15) / 16;   // <= 8
  const int row = w * rows_per_wave + (l >> 3);
  const int j = l & 7;
  const bool act = (l >> 3) < rows_per_wave && row < nn;
  constexpr int PA = kMaxN / 16;  // pairs a lane handles (a = j, j + 8, ...)
  double cn[PA], sn[PA];          // rotation of the next round, loaded ahead
#pragma unroll
  for (int t = 0; t < PA; ++t) {
    const int a = j + 8 * t;
    cn[t] = (rounds > 0 && a < half) ? rlog[a] : 1.0;
    sn[t] = (rounds > 0 && a < half) ? rlog[half + a] : 0.0;
  }
  int s = 0;
  for (int g = 0; g < rounds; ++g) {
    double cc[PA], ss[PA];
#pragma unroll
    for (int t = 0; t < PA; ++t) {
      cc[t] = cn[t];
      ss[t] = sn[t];
    }
    if (g + 1 < rounds) {
      const double *lg = rlog + (size_t)(g + 1) * 2 * half;
#pragma unroll
      for (int t = 0; t < PA; ++t) {
        const int a = j + 8 * t;
        cn[t] = a < half ? lg[a] : 1.0;
        sn[t] = a < half ? lg[half + a] : 0.0;
      }
    }
    if (act) {
#pragma unroll
      for (int t = 0; t < PA; ++t) {
        const int a = j + 8 * t;
        if (a < half && ss[t] != 0.0) {
          const int u = rr_player(s, a, nn), v = rr_player(s, nn - 1 - a, nn);
          const int p = u < v ? u : v, q = u < v ? v : u;
          const double vp = V[row * ldv + p], vq = V[row * ldv + q];
          V[row * ldv + p] = cc[t] * vp - ss[t] * vq;
          V[row * ldv + q] = ss[t] * vp + cc[t] * vq;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (++s == nn - 1) s = 0;
  }
  __syncthreads();
}

// Dense product of the workgroup on the matrix cores, n <= 128:
//   out(r, c) = sum_k a(r, k) b(k, c),   0 <= r, c < nt*16,
// with operand readers a, b (zero outside the matrices) and a writer.  The
// 16 waves share the (nt x nt) output tiles.
template <typename FA, typename FB, typename FO>
__device__ __forceinline__ void wg_gemm(int nt, FA a, FB b, FO out) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int kl = l >> 4;
  for (int t = w; t < nt * nt; t += kThreads / 64) {
    const int r0 = (t / nt) * 16, c0 = (t % nt) * 16;
    d4 acc0 = d4zero(), acc1 = d4zero();
    for (int k0 = 0; k0 < nt * 16; k0 += 8) {
      acc0 = mfma(a(r0 + (l & 15), k0 + kl), b(k0 + kl, c0 + (l & 15)), acc0);
      acc1 = mfma(a(r0 + (l & 15), k0 + 4 + kl), b(k0 + 4 + kl, c0 + (l & 15)), acc1);
    }
    const d4 acc = acc0 + acc1;
#pragma unroll
    for (int r = 0; r < 4; ++r) out(r0 + (l >> 4) + 4 * r, c0 + (l & 15), acc[r]);
  }
}

__global__ __launch_bounds__(kThreads) void reduced_eig_kernel(const double *AQ, const double *BQ,
                                                               int n, double *eps, double *Phi,
                                                               double *scratch, int *flag) {
  extern __shared__ double C[];
  __shared__ RRShared sh;
  const int tid = threadIdx.x;
  const int nn = n + (n & 1);
  const int ldc = nn + 1;
  const int nt = (nn + 15) / 16;
  double *T = scratch;                 // nn x nn whitening
  double *T1 = scratch + nn * nn;      // nn x nn product
  double *V = scratch + 2 * nn * nn;   // nn x nn eigenvectors of B_Q (fallback)
  double *rlog = scratch + 3 * nn * nn;  // rotation log

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
    // X = L^{-1}, row by row: X_ii = 1/L_ii, X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj;
    // X_ij (j < i) is kept in the free upper triangle of C at (j, i).
    // Eight threads share one dot product and combine it with shuffles.
    for (int i = 0; i < n; ++i) {
      const double dii = 1.0 / C[i * ldc + i];
      const int j = tid >> 3, part = tid & 7;
      double sum = 0.0;
      if (j < i) {
        for (int k = j + part; k < i; k += 8) {
          const double xkj = (k == j) ? sh.diag[k] : C[j * ldc + k];
          sum += C[i * ldc + k] * xkj;
        }
      }
      sum += __shfl_xor(sum, 1);
      sum += __shfl_xor(sum, 2);
      sum += __shfl_xor(sum, 4);
      if (j < i && part == 0) C[j * ldc + i] = -dii * sum;
      if (tid == 0) sh.diag[i] = dii;
      __syncthreads();
    }
    // T = L^{-T} = X^T (upper triangular)
    for (int idx = tid; idx < nn * nn; idx += kThreads) {
      const int i = idx / nn, j = idx % nn;
      double v = 0.0;
      if (i < n && j < n) v = (i < j) ? C[i * ldc + j] : (i == j ? sh.diag[i] : 0.0);
      T[idx] = v;
    }
  } else {
    // eigen-decomposition of B_Q, drop directions with mu <= 1e-14 max
    for (int idx = tid; idx < nn * nn; idx += kThreads) {
      const int i = idx / nn, j = idx % nn;
      C[i * ldc + j] = (i < n && j < n) ? BQ[i * n + j] : 0.0;
    }
    __syncthreads();
    const int fsweeps = jacobi(C, ldc, rlog, nn, sh);
    if (tid == 0) flag[2] = fsweeps;
    if (tid < nn) sh.diag[tid] = C[tid * ldc + tid];
    __syncthreads();
    replay_rotations(C, ldc, rlog, fsweeps * (nn - 1), nn);
    for (int idx = tid; idx < nn * nn; idx += kThreads) V[idx] = C[(idx / nn) * ldc + idx % nn];
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

  // ---- C = T^T A_Q T on the matrix cores ----
  const int nlim = nt * 16;
  wg_gemm(
      nt, [&](int r, int k) { return (r < n && k < n) ? AQ[k * n + r] : 0.0; },  // symmetric
      [&](int k, int c) { return (k < nn && c < nn) ? T[k * nn + c] : 0.0; },
      [&](int r, int c, double v) { if (r < nn && c < nn) T1[r * nn + c] = v; });
  __syncthreads();
  wg_gemm(
      nt, [&](int r, int k) { return (r < nn && k < nn) ? T[k * nn + r] : 0.0; },
      [&](int k, int c) { return (k < nn && c < nn) ? T1[k * nn + c] : 0.0; },
      [&](int r, int c, double v) { if (r < nn && c < nn) C[r * ldc + c] = v; });
  (void)nlim;
  __syncthreads();
  // symmetrise: C <- (C + C^T) / 2
  for (int idx = tid; idx < nn * nn; idx += kThreads) {
    const int i = idx / nn, j = idx % nn;
    if (j > i) {
      const double v = 0.5 * (C[i * ldc + j] + C[j * ldc + i]);
      C[i * ldc + j] = v;
      C[j * ldc + i] = v;
    }
  }
  __syncthreads();

  const int sweeps = jacobi(C, ldc, rlog, nn, sh);
  if (tid == 0) flag[1] = sweeps;

  // ---- sort ascending, dropped directions (NaN) last ----
  if (tid < nn) sh.diag[tid] = C[tid * ldc + tid];
  __syncthreads();
  double *VL = C;  // eigenvectors of C, rebuilt in LDS from the rotation log
  replay_rotations(VL, ldc, rlog, sweeps * (nn - 1), nn);
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
  wg_gemm(
      nt, [&](int r, int k) { return (r < nn && k < nn) ? T[r * nn + k] : 0.0; },
      [&](int k, int c) { return (k < nn && c < nn) ? VL[k * ldc + c] : 0.0; },
      [&](int r, int c, double v) { if (r < n && c < n) Phi[r * n + sh.rank[c]] = v; });
  if (tid == 0) flag[0] = fallback ? 1 : 0;
}

}  // namespace

size_t reduced_eig_scratch_doubles() {
  return 3 * (size_t)kMaxN * kMaxN + (size_t)kMaxSweeps * (kMaxN - 1) * kMaxN;
}

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
