// Reduced generalized eigenproblem of the Rayleigh-Ritz step (Sec. III.A,
// eqs. 6-9): A_Q Phi = eps B_Q Phi with Phi^T B_Q Phi = I, for M0 <= 128,
// all in float64.
//
//  1. Whitening T with T^T B_Q T = I: T = L^{-T} from the Cholesky factor
//     B_Q = L L^T.  If a Cholesky pivot is not above 1e-12 B_Q(k, k) (B_Q
//     not numerically s.p.d., Sec. III.B (ii): a pivot at rounding level
//     relative to its own column is a numerically null direction, whose
//     whitening would amplify rounding errors; the test does not depend on
//     the scaling of Q's columns), B_Q = V diag(mu) V^T is diagonalised instead,
//     T = V diag(mu^{-1/2}) on the directions with mu > 1e-10 max(mu), and
//     the other columns of T are zero.
//  2. C = T^T A_Q T, diagonalised by cyclic two-sided Jacobi rotations in a
//     round-robin order (all n/2 disjoint rotations of a round at once);
//     a rotation is skipped when |c_pq| <= u sqrt(|c_pp c_qq|) or
//     |c_pq| <= u ||C||_F / 8 (u = 2^-53), and the sweeps stop when no pair
//     would rotate.
//  3. eps ascending (dropped directions: NaN, last), Phi = T V.
//
// kSplit workgroups run steps 1-2 on identical data with identical
// arithmetic, so their rotations agree bit for bit; each keeps only its own
// rows of V (the rows of V evolve independently), which cuts the per-round
// eigenvector work of a workgroup by kSplit.  Workgroup 0 sorts; a second
// kernel forms Phi = T V.
#include "common.h"
#include "kernels.h"

namespace feast {
namespace {

constexpr int kThreads = 1024;
constexpr int kMaxN = 128;
constexpr int kSplit = 4;  // workgroups; each keeps kMaxN / kSplit rows of V

struct RRShared {
  double2 csn[2][kMaxN / 2];  // (cos, sin) of each pair slot, rounds of even / odd parity
  double4 dnew[kMaxN / 2];    // a round's new diagonal block of each slot
  int rot;
  int fail;
  double norm;
  double red[kThreads];
  int dropped[kMaxN];
  double diag[kMaxN];
};

constexpr int kMaxSweeps = 60;

// Eigenvector layout: VT (LDS, row stride kVTld, rows 16-byte aligned)
// holds VT[c][r] = V[r][c].
constexpr int kVTld = kMaxN + 2;

// v from lane l+1 (wave_rol:1, lane 63 from lane 0) and from lane l-1
// (wave_ror:1, lane 0 from lane 63), 64-bit
__device__ __forceinline__ double readlane_d(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_rol(double v) {
  const u32x2 x = __builtin_bit_cast(u32x2, v);
  return __builtin_bit_cast(double,
                            (u32x2){(unsigned)__builtin_amdgcn_mov_dpp((int)x[0], 0x134, 0xf, 0xf, false),
                                    (unsigned)__builtin_amdgcn_mov_dpp((int)x[1], 0x134, 0xf, 0xf, false)});
}
__device__ __forceinline__ double lane_ror(double v) {
  const u32x2 x = __builtin_bit_cast(u32x2, v);
  return __builtin_bit_cast(double,
                            (u32x2){(unsigned)__builtin_amdgcn_mov_dpp((int)x[0], 0x13c, 0xf, 0xf, false),
                                    (unsigned)__builtin_amdgcn_mov_dpp((int)x[1], 0x13c, 0xf, 0xf, false)});
}

// Cyclic Jacobi on the nn x nn symmetric matrix C (LDS, row stride ldc),
// round-robin by the circle method: circle position x holds a player (an
// index of C), pair slot a joins the positions a ("top") and nn-1-a
// ("bottom"), and after each round every player but the one at position 0
// moves one position down the circle (position 1 wraps to nn-1).
//
// During a sweep C is held in circle-position coordinates: entry (x, y) is
// C at the players standing at x and y, upper triangle only (kept at
// (min, max)).  A thread's 2x2 blocks (slots a < b) thus stay at fixed
// addresses, and each round writes its rotated entries to where their
// players stand in the next round, also fixed addresses: all index work is
// done once per call.  After nn-1 rounds every player is back at its start,
// so between sweeps C is in plain coordinates.  The rotation of slot a is
// taken in (top, bottom) order, x_top' = c x_top - s x_bot,
// x_bot' = s x_top + c x_bot; the lanes of wave 0 compute the rotations and
// also update the slots' diagonal 2x2 blocks.
//
// The eigenvectors V = J_1 J_2 ... accumulate in registers while C is
// rotated: every row of V evolves on its own, so wave w keeps the rows
// [8w, 8w+8) of V (16 waves cover 128) and lane a the two columns of slot a.
// After each round the columns move with their players: a lane takes its
// new top column from lane a+1 and its new bottom column from lane a-1
// (wavefront lane shifts), with the turning points at lanes 0 and half-1.
// A wave keeps R rows of V, the workgroup the rows [row0, row0 + 16 R).
// On return sh.diag holds the eigenvalues (diagonal of C), and the
// eigenvectors are in VT (which overlays C; R = 8, all rows) or, for R < 8,
// the workgroup's rows in Vout (Vout[c * nn + r] = V[r][c]).  Returns the
// number of sweeps that rotated.
template <int R>
__device__ __forceinline__ int jacobi(double *C, int ldc, int nn, RRShared &sh, int row0,
                                      double *Vout) {
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
  // where the player at position x stands in the next round, and the
  // offset of entry (x, y) in the upper triangle
  auto mv = [&](int x) { return x == 0 ? 0 : (x == 1 ? nn - 1 : x - 1); };
  auto sym = [&](int x, int y) { return x < y ? x * ldc + y : y * ldc + x; };
  // The off-diagonal 2x2 blocks (a, b), a < b, of the pair slots are dealt
  // out to the threads once (at most 2 each for nn <= 128); entry k of a
  // block is (top/bottom of a, top/bottom of b) = (k >> 1, k & 1).
  constexpr int kPer = (kMaxN / 2 * (kMaxN / 2 - 1) / 2 + kThreads - 1) / kThreads;
  const int nblk = half * (half - 1) / 2;
  int ba[kPer], bb[kPer], rd[kPer][4], wr[kPer][4];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    int idx = tid + t * kThreads;
    ba[t] = -1;
    bb[t] = 0;
    if (idx < nblk) {  // row a of the block triangle holds half - 1 - a blocks
      int a = 0;
      while (idx >= half - 1 - a) {
        idx -= half - 1 - a;
        ++a;
      }
      ba[t] = a;
      bb[t] = a + 1 + idx;
    }
    const int xa[2] = {ba[t] < 0 ? 0 : ba[t], nn - 1 - (ba[t] < 0 ? 0 : ba[t])};
    const int xb[2] = {bb[t], nn - 1 - bb[t]};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      rd[t][k] = sym(xa[k >> 1], xb[k & 1]);
      wr[t][k] = sym(mv(xa[k >> 1]), mv(xb[k & 1]));
    }
  }

  const int lw = tid >> 6, la = tid & 63;
  const int r0 = row0 + R * lw;
  // V[r0 + k][player at position la / nn-1-la].  Every round applies the
  // rotations of the round before and then moves the players, the first
  // round too, with identity rotations: V starts as the identity in the
  // positions of the round before, where position x holds player mv(x).
  double top[R], bot[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    top[k] = (la < half && mv(la) == r0 + k) ? 1.0 : 0.0;
    bot[k] = (la < half && mv(nn - 1 - la) == r0 + k) ? 1.0 : 0.0;
  }
  if (tid < half) sh.csn[1][tid] = double2{1.0, 0.0};
  // V <- V J with the rotations rv of a round, then the players move one
  // circle position (player 0 stays): a lane's new top column comes from
  // lane a+1 and its new bottom column from lane a-1, with the turning
  // points at lanes 0 and half-1.  Each round's update runs during the next
  // round's rotation phase (its rotations stay in the other half of the
  // double-buffered csn).  Lanes a >= half carry values that are never used.
  auto v_update = [&](const double2 *rv) {
    const double2 r = rv[la];
    const double c = r.x, sg = r.y;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const double t = top[k], b = bot[k];
      top[k] = c * t - sg * b;
      bot[k] = sg * t + c * b;
    }
    if (nn > 2) {
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const double rt = lane_rol(top[k]), rb = lane_ror(bot[k]);
        top[k] = la == 0 ? top[k] : (la == half - 1 ? bot[k] : rt);
        bot[k] = la == 0 ? rt : rb;
      }
    }
  };
  int g = 0;  // rounds done; csn[g & 1] holds the current round's rotations
  int sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) sh.rot = 0;
    __syncthreads();
    for (int s = 0; s < nn - 1; ++s) {
      double2 *csn = sh.csn[g & 1];
      if (tid < half) {  // one wave: rotation of slot tid and its diagonal block
        const int xt = tid, xbt = nn - 1 - tid;
        const double app = C[xt * ldc + xt], aqq = C[xbt * ldc + xbt], apq = C[xt * ldc + xbt];
        double c = 1.0, sgn = 0.0, t = 0.0;
        const bool rotate =
            fabs(apq) > floor_abs && fabs(apq) > eps * sqrt(fabs(app * aqq));
        if (rotate) {
          // t = tan of the rotation angle: the smaller root of t^2 + 2 tau t - 1
          const double tau = (aqq - app) * rcp_newton(2.0 * apq);
          const double ata = fabs(tau);
          const double root = ata < 1e150 ? sqrt(1.0 + tau * tau) : ata;
          t = (tau >= 0.0 ? 1.0 : -1.0) * rcp_newton(ata + root);
          c = rcp_newton(sqrt(1.0 + t * t));
          sgn = t * c;
        }
        // the new diagonal block, written to C after the barrier
        sh.dnew[tid] = double4{app - t * apq, aqq + t * apq, rotate ? 0.0 : apq, 0.0};
        const unsigned long long m = __ballot(rotate);
        if (tid == 0) sh.rot += __popcll(m);
        csn[tid] = double2{c, sgn};
      }
      v_update(sh.csn[(g & 1) ^ 1]);
      // the blocks' entries: every entry is read before the barrier, as the
      // writes after it go to other threads' entries
      double x[kPer][4];
#pragma unroll
      for (int t = 0; t < kPer; ++t) {
        if (ba[t] < 0) continue;
#pragma unroll
        for (int k = 0; k < 4; ++k) x[t][k] = C[rd[t][k]];
      }
      __syncthreads();
      // C <- J^T C J, written in the next round's positions
      if (tid < half) {
        const int xt = mv(tid), xbt = mv(nn - 1 - tid);
        const double4 d = sh.dnew[tid];
        C[xt * ldc + xt] = d.x;
        C[xbt * ldc + xbt] = d.y;
        C[sym(xt, xbt)] = d.z;
      }
#pragma unroll
      for (int t = 0; t < kPer; ++t) {
        if (ba[t] < 0) continue;
        const double2 ra = csn[ba[t]], rb = csn[bb[t]];
        const double ca = ra.x, sa = ra.y, cb = rb.x, sb = rb.y;
        const double x11 = x[t][0], x12 = x[t][1], x21 = x[t][2], x22 = x[t][3];
        const double y11 = cb * x11 - sb * x12, y12 = sb * x11 + cb * x12;
        const double y21 = cb * x21 - sb * x22, y22 = sb * x21 + cb * x22;
        C[wr[t][0]] = ca * y11 - sa * y21;
        C[wr[t][1]] = ca * y12 - sa * y22;
        C[wr[t][2]] = sa * y11 + ca * y21;
        C[wr[t][3]] = sa * y12 + ca * y22;
      }
      __syncthreads();
      ++g;
    }
    const int rot = sh.rot;
    __syncthreads();
    if (rot == 0) break;
    // Would a further sweep rotate anything?  C does not change during a
    // sweep without rotations, so testing every pair at once decides it as
    // that sweep would, without its nn - 1 rounds.
    bool need = false;
    for (int idx = tid; idx < nn * nn; idx += kThreads) {
      const int p = idx / nn, q = idx % nn;
      if (p < q) {
        const double apq = C[p * ldc + q];
        need |= fabs(apq) > floor_abs &&
                fabs(apq) > eps * sqrt(fabs(C[p * ldc + p] * C[q * ldc + q]));
      }
    }
    if (!__syncthreads_or(need)) {
      ++sweep;  // this sweep rotated; none is left to do
      break;
    }
  }
  v_update(sh.csn[(g & 1) ^ 1]);
  // every sweep ends with each player at its start: lane la holds the
  // columns la and nn-1-la
  if (tid < nn) sh.diag[tid] = C[tid * ldc + tid];
  __syncthreads();
  if constexpr (R == 8) {
    if (la < half && r0 < nn) {  // rows r0..r0+7 of every column: all of VT that is read
      double2 *xt2 = reinterpret_cast<double2 *>(C + la * kVTld + r0);
      double2 *xb2 = reinterpret_cast<double2 *>(C + (nn - 1 - la) * kVTld + r0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        xt2[k] = double2{top[2 * k], top[2 * k + 1]};
        xb2[k] = double2{bot[2 * k], bot[2 * k + 1]};
      }
    }
  } else if (la < half) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
      if (r0 + k < nn) {
        Vout[la * nn + r0 + k] = top[k];
        Vout[(nn - 1 - la) * nn + r0 + k] = bot[k];
      }
    }
  }
  __syncthreads();
  return sweep;  // sweeps with at least one rotation (all of them if not converged)
}

// Dense product of the workgroup on the matrix cores, n <= 128:
//   out(r, c) = sum_k a(r, k) b(k, c),   0 <= r, c < nl = nt*16,
// with operand readers a, b (global memory, zero outside the matrices) and
// a writer.  The operands pass through LDS (stage: kStageDoubles) in
// 32-deep slices loaded with consecutive threads on consecutive k-major
// elements; the 16 waves share the (nt x nt) output tiles and keep them in
// registers until the last slice, so the writer may overwrite stage.
constexpr int kSlice = 32;
constexpr int kSA = kSlice + 1;      // row stride of the a slice [nl][kSA]
constexpr int kSB = kMaxN + 1;       // row stride of the b slice [kSlice][kSB]
constexpr int kStageDoubles = kMaxN * kSA + kSlice * kSB;
template <typename FA, typename FB, typename FO>
__device__ __forceinline__ void wg_gemm(int nt, double *stage, FA a, FB b, FO out) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, kl = l >> 4;
  const int nl = nt * 16;
  double *sa = stage, *sb = stage + kMaxN * kSA;
  constexpr int kPerW = kMaxN / 16 * (kMaxN / 16) / (kThreads / 64);  // tiles per wave, nt = 8
  d4 acc[kPerW];
#pragma unroll
  for (int q = 0; q < kPerW; ++q) acc[q] = d4zero();
  for (int k0 = 0; k0 < nl; k0 += kSlice) {
    const int kw = nl - k0 < kSlice ? nl - k0 : kSlice;
    for (int idx = tid; idx < kw * nl; idx += kThreads) {
      const int kk = idx / nl, x = idx % nl;
      sa[x * kSA + kk] = a(x, k0 + kk);
      sb[kk * kSB + x] = b(k0 + kk, x);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPerW; ++q) {
      const int t = w + q * (kThreads / 64);
      if (t < nt * nt) {
        const int r0 = (t / nt) * 16, c0 = (t % nt) * 16;
        for (int kq = 0; kq < kw; kq += 4) {
          const double av = sa[(r0 + (l & 15)) * kSA + kq + kl];
          const double bv = sb[(kq + kl) * kSB + c0 + (l & 15)];
          acc[q] = mfma(av, bv, acc[q]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kPerW; ++q) {
    const int t = w + q * (kThreads / 64);
    if (t < nt * nt) {
      const int r0 = (t / nt) * 16, c0 = (t % nt) * 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) out(r0 + (l >> 4) + 4 * r, c0 + (l & 15), acc[q][r]);
    }
  }
}

__global__ __launch_bounds__(kThreads) void reduced_eig_kernel(const double *AQ, const double *BQ,
                                                               int n, double *eps, double *Phi,
                                                               double *scratch, int *flag,
                                                               const int *skip) {
  if (skip && *skip) return;  // a converged solve: later loops of a captured solve do nothing
  extern __shared__ __align__(16) double C[];  // nn x (nn + 1) matrix, or nn x kVTld VT
  __shared__ RRShared sh;
  const int tid = threadIdx.x;
  const int nn = n + (n & 1);
  const int ldc = nn + 1;
  const int nt = (nn + 15) / 16;
  // per workgroup: whitening T, product T1, eigenvectors V of B_Q (fallback),
  // each nn x nn; then the shared outputs VT (kMaxN^2) and rank (kMaxN ints)
  double *T = scratch + (size_t)blockIdx.x * 3 * kMaxN * kMaxN;
  double *T1 = T + nn * nn;
  double *V = T + 2 * nn * nn;
  double *VTg = scratch + (size_t)kSplit * 3 * kMaxN * kMaxN;
  int *rank_g = reinterpret_cast<int *>(VTg + kMaxN * kMaxN);

  for (int idx = tid; idx < nn * nn; idx += kThreads) {
    const int i = idx / nn, j = idx % nn;
    C[i * ldc + j] = (i < n && j < n) ? BQ[i * n + j] : 0.0;
  }
  if (tid == 0) sh.fail = 0;
  if (tid < kMaxN) sh.dropped[tid] = (tid >= n);
  __syncthreads();

  // ---- Cholesky B_Q = L L^T (lower triangle of C), by 16-column panels ----
  // Wave 0 factors the panel (its rows held in registers, two per lane,
  // pivot column values broadcast with readlane); then every wave applies
  // the panel to the trailing matrix on the matrix cores.  Entries above the
  // diagonal are not kept.
  // B_Q's own diagonal, for the pivot test (wave 0: lane l holds rows l, l + 64)
  double od[2] = {0.0, 0.0};
  if (tid < 64) {
    od[0] = tid < n ? C[tid * ldc + tid] : 0.0;
    od[1] = tid + 64 < n ? C[(tid + 64) * ldc + tid + 64] : 0.0;
  }
  for (int k0 = 0; k0 < n; k0 += 16) {
    const int kw = n - k0 < 16 ? n - k0 : 16;
    if (tid < 64) {
      const int i0 = k0 + tid, i1 = k0 + 64 + tid;  // this lane's rows
      double pr[2][16];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        pr[0][jj] = (i0 < n && jj < kw) ? C[i0 * ldc + k0 + jj] : 0.0;
        pr[1][jj] = (i1 < n && jj < kw) ? C[i1 * ldc + k0 + jj] : 0.0;
      }
      bool ok = true;  // uniform: every test below is on wave-uniform values
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const double d = readlane_d(pr[0][kk], kk);  // pivot (k0+kk, k0+kk)
        const double bkk = readlane_d(k0 < 64 ? od[0] : od[1], (k0 + kk) & 63);
        if (kk < kw && ok) {
          if (!(d > 1e-12 * bkk) || !isfinite(d)) {
            ok = false;
          } else {
            const double lkk = sqrt(d), rl = 1.0 / lkk;
            pr[0][kk] = tid > kk ? pr[0][kk] * rl : (tid == kk ? lkk : pr[0][kk]);
            pr[1][kk] *= rl;
#pragma unroll
            for (int jj = kk + 1; jj < 16; ++jj) {
              const double ljk = readlane_d(pr[0][kk], jj);  // L(k0+jj, k0+kk)
              pr[0][jj] -= pr[0][kk] * ljk;  // (columns jj >= kw are not stored)
              pr[1][jj] -= pr[1][kk] * ljk;
            }
          }
        }
      }
      if (!ok) {
        if (tid == 0) sh.fail = 1;
      } else {
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
          if (jj < kw && i0 < n) C[i0 * ldc + k0 + jj] = pr[0][jj];
          if (jj < kw && i1 < n) C[i1 * ldc + k0 + jj] = pr[1][jj];
        }
      }
    }
    __syncthreads();
    if (sh.fail) break;  // uniform
    // trailing update C(i, j) -= sum_k L(i, k) L(j, k), k in the panel,
    // j <= i, over the 16 x 16 tiles below the panel
    // (a panel narrower than 16 is the last one: nothing trails it, and
    // otherwise t0 is a multiple of 16)
    const int t0 = k0 + kw, tt0 = t0 / 16, ntr = nt - tt0;
    if (t0 < n) {
      const int l = tid & 63, kl = l >> 4;
      for (int t = tid >> 6; t < ntr * ntr; t += kThreads / 64) {
        const int ti = tt0 + t / ntr, tj = tt0 + t % ntr;
        if (tj > ti) continue;
        const int ra = ti * 16 + (l & 15), rb = tj * 16 + (l & 15);
        d4 acc = d4zero();
#pragma unroll
        for (int q = 0; q < 16; q += 4) {
          const int k = q + kl;
          const double a = (ra < n && k < kw) ? C[ra * ldc + k0 + k] : 0.0;
          const double bv = (rb < n && k < kw) ? C[rb * ldc + k0 + k] : 0.0;
          acc = mfma(a, bv, acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = ti * 16 + (l >> 4) + 4 * r, j = tj * 16 + (l & 15);
          if (i < n && j <= i && j >= t0) C[i * ldc + j] -= acc[r];
        }
      }
    }
    __syncthreads();
  }
  __syncthreads();
  const bool fallback = sh.fail != 0;

  if (!fallback) {
    // X = L^{-1} by 16 x 16 blocks; X_ij (j < i) is kept in the free upper
    // triangle of C at (j, i), X_ii = 1/L_ii in sh.diag.
    // (a) diagonal blocks, one wave each: lane c (< 16) forms column c of
    //     X_II by forward substitution, X_ic = (delta_ic - sum_k L_ik X_kc) / L_ii
    //     (the entries above the diagonal come out zero).
    const int nb = (n + 15) / 16;
    {
      const int w = tid >> 6, c = tid & 63, o = 16 * w;
      if (w < nb && c < 16) {
        double x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          x[i] = 0.0;
          if (o + i < n) {  // uniform in the wave
            const double dii = 1.0 / C[(o + i) * ldc + o + i];
            double sum = (i == c) ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < i; ++k) sum -= C[(o + i) * ldc + o + k] * x[k];
            x[i] = sum * dii;
            if (i == c) sh.diag[o + i] = dii;
          }
        }
        if (o + c < n) {
#pragma unroll
          for (int i = 0; i < 16; ++i)
            if (i > c && o + i < n) C[(o + c) * ldc + o + i] = x[i];
        }
      }
    }
    __syncthreads();
    // (b) X_IJ = -X_II sum_{K=J}^{I-1} L_IK X_KJ, one block diagonal I - J = d
    //     at a time (one wave per block, on the matrix cores).  The sum S is
    //     parked in X_IJ's place and read back by the same wave.
    auto xval = [&](int k, int c) {  // X(k, c), k >= c
      return k > c ? C[c * ldc + k] : (k == c ? sh.diag[k] : 0.0);
    };
    for (int d = 1; d < nb; ++d) {
      const int w = tid >> 6, l = tid & 63, kl = l >> 4;
      if (w < nb - d) {
        const int oj = 16 * w, oi = 16 * (w + d);
        const int rr = oi + (l & 15), cc = oj + (l & 15);
        d4 acc = d4zero();
        for (int ok = oj; ok < oi; ok += 16) {
#pragma unroll
          for (int q = 0; q < 16; q += 4) {
            const int k = ok + q + kl;
            const double a = (rr < n && k < n) ? C[rr * ldc + k] : 0.0;  // L(rr, k)
            const double bv = (k < n && cc < n && k >= cc) ? xval(k, cc) : 0.0;
            acc = mfma(a, bv, acc);
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = oi + (l >> 4) + 4 * q, c = oj + (l & 15);
          if (r < n && c < n) C[c * ldc + r] = acc[q];
        }
        d4 acc2 = d4zero();
#pragma unroll
        for (int q = 0; q < 16; q += 4) {
          const int k = oi + q + kl;
          const double a = (rr < n && k < n && rr >= k) ? xval(rr, k) : 0.0;  // X_II(rr, k)
          const double bv = (k < n && cc < n) ? C[cc * ldc + k] : 0.0;       // S(k, cc)
          acc2 = mfma(a, bv, acc2);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = oi + (l >> 4) + 4 * q, c = oj + (l & 15);
          if (r < n && c < n) C[c * ldc + r] = -acc2[q];
        }
      }
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
    // eigen-decomposition of B_Q, drop directions with mu <= 1e-10 max
    for (int idx = tid; idx < nn * nn; idx += kThreads) {
      const int i = idx / nn, j = idx % nn;
      C[i * ldc + j] = (i < n && j < n) ? BQ[i * n + j] : 0.0;
    }
    __syncthreads();
    const int fsweeps = jacobi<8>(C, ldc, nn, sh, 0, nullptr);
    if (tid == 0 && blockIdx.x == 0) flag[2] = fsweeps;
    for (int idx = tid; idx < nn * nn; idx += kThreads) V[idx] = C[(idx % nn) * kVTld + idx / nn];
    __syncthreads();
    double mumax = 0.0;
    for (int i = 0; i < n; ++i) mumax = fmax(mumax, sh.diag[i]);
    if (tid < n) sh.dropped[tid] = !(sh.diag[tid] > 1e-10 * mumax);
    __syncthreads();
    for (int idx = tid; idx < nn * nn; idx += kThreads) {
      const int i = idx / nn, j = idx % nn;
      T[idx] = (i < n && j < n && !sh.dropped[j]) ? V[idx] / sqrt(sh.diag[j]) : 0.0;
    }
  }
  __syncthreads();

  // ---- C = T^T A_Q T on the matrix cores ----
  const int nlim = nt * 16;
  // (C's storage is free here and serves as the staging area)
  wg_gemm(
      nt, C, [&](int r, int k) { return (r < n && k < n) ? AQ[k * n + r] : 0.0; },  // symmetric
      [&](int k, int c) { return (k < nn && c < nn) ? T[k * nn + c] : 0.0; },
      [&](int r, int c, double v) { if (r < nn && c < nn) T1[r * nn + c] = v; });
  __syncthreads();
  wg_gemm(
      nt, C, [&](int r, int k) { return (r < nn && k < nn) ? T[k * nn + r] : 0.0; },
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

  constexpr int kR = 8 / kSplit;
  const int sweeps = jacobi<kR>(C, ldc, nn, sh, blockIdx.x * 16 * kR, VTg);
  if (blockIdx.x != 0) return;
  if (tid == 0) flag[1] = sweeps;

  // ---- sort ascending, dropped directions (NaN) last ----
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
    rank_g[i] = rk;
    eps[rk] = sh.dropped[i] ? __longlong_as_double(0x7ff8000000000000LL) : sh.diag[i];
  }
  if (tid == 0) flag[0] = fallback ? 1 : 0;
}

// Phi[:, rank[c]] = T V[:, c] with T (nn x nn, row-major) of workgroup 0 and
// VT[c * nn + r] = V[r][c]: one wave per 16 x 16 output tile.
__global__ __launch_bounds__(64) void phi_kernel(const double *scratch, int n, double *Phi,
                                                 const int *skip) {
  if (skip && *skip) return;  // a converged solve: later loops of a captured solve do nothing
  const int nn = n + (n & 1);
  const int nt = (nn + 15) / 16;
  const double *T = scratch;
  const double *VT = scratch + (size_t)kSplit * 3 * kMaxN * kMaxN;
  const int *rank = reinterpret_cast<const int *>(VT + kMaxN * kMaxN);
  const int l = threadIdx.x, kl = l >> 4;
  const int r0 = blockIdx.y * 16, c0 = blockIdx.x * 16;
  const int r = r0 + (l & 15), c = c0 + (l & 15);
  d4 acc0 = d4zero(), acc1 = d4zero();
  for (int k0 = 0; k0 < nt * 16; k0 += 8) {
    const int ka = k0 + kl, kb = k0 + 4 + kl;
    const double a0 = (r < nn && ka < nn) ? T[r * nn + ka] : 0.0;
    const double a1 = (r < nn && kb < nn) ? T[r * nn + kb] : 0.0;
    const double b0 = (c < nn && ka < nn) ? VT[c * nn + ka] : 0.0;
    const double b1 = (c < nn && kb < nn) ? VT[c * nn + kb] : 0.0;
    acc0 = mfma(a0, b0, acc0);
    acc1 = mfma(a1, b1, acc1);
  }
  const d4 acc = acc0 + acc1;
  if (c < n) {
    const int rc = rank[c];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = r0 + (l >> 4) + 4 * i;
      if (rr < n) Phi[rr * n + rc] = acc[i];
    }
  }
}

}  // namespace

size_t reduced_eig_scratch_doubles() {
  return (3 * kSplit + 1) * (size_t)kMaxN * kMaxN + kMaxN / 2;
}

// Device-resident scratch of the allocation-free entry point: one reduced
// eigensolve at the largest size (kMaxN) followed by its flags (four ints in
// the last two doubles); 1.7 MB, held by every GPU the library runs on until
// the process ends.  Host code must use the address returned by
// reduced_eig_static_scratch, never this name.
namespace {
constexpr size_t kStaticScratchDoubles = (3 * kSplit + 1) * (size_t)kMaxN * kMaxN + kMaxN / 2 + 2;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];
}  // namespace

hipError_t reduced_eig_static_scratch(double **ptr, int **flag) {
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  *ptr = static_cast<double *>(p);
  *flag = reinterpret_cast<int *>(*ptr + reduced_eig_scratch_doubles());
  return hipSuccess;
}

// LDS of the reduced eigensolver for size m: the matrix or the eigenvector
// transpose, or the products' staging area
size_t reduced_eig_lds_bytes(int m) {
  const int mm = m + (m & 1);
  size_t d = (size_t)mm * (kVTld > mm + 1 ? kVTld : mm + 1);
  if (d < (size_t)kStageDoubles) d = kStageDoubles;
  return d * sizeof(double);
}

hipError_t reduced_eig_set_lds() {
  return hipFuncSetAttribute((const void *)reduced_eig_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)reduced_eig_lds_bytes(kMaxN));
}

hipError_t launch_reduced_eig(const double *AQ, const double *BQ, int n, double *eps, double *Phi,
                              double *scratch, int *flag, hipStream_t st, const int *skip) {
  if (n < 1 || n > kMaxN) return hipErrorInvalidValue;
  const int nn = n + (n & 1);
  const size_t shm = reduced_eig_lds_bytes(n);
  // the limit is set for the largest n (so calls of any size, from any
  // thread, agree on it), and not while the stream is being captured into a
  // graph: a captured loop always follows an eager call on the device
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t err = hipStreamIsCapturing(st, &cs);
  if (err != hipSuccess) return err;
  if (cs == hipStreamCaptureStatusNone) {
    err = reduced_eig_set_lds();
    if (err != hipSuccess) return err;
  }
  hipLaunchKernelGGL(reduced_eig_kernel, dim3(kSplit), dim3(kThreads), shm, st, AQ, BQ, n, eps, Phi,
                     scratch, flag, skip);
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int nt = (nn + 15) / 16;
  hipLaunchKernelGGL(phi_kernel, dim3(nt, nt), dim3(64), 0, st, scratch, n, Phi, skip);
  return hipGetLastError();
}

}  // namespace feast
