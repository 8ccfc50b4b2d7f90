// Dense kernels around the shifted solves: block-tridiagonal products
// (B Y, A Q, B Q, A X, B X), the quadrature sum over nodes (eq. 15), the
// projections A_Q = Q^T A Q and B_Q = Q^T B Q (eq. 7), the Ritz vectors
// X = Q Phi (eq. 9), the residuals of the Table I caption, and layout
// conversion between the caller's [N][M0] arrays and the padded internal
// layout [nc][BP][M0P].  Every reduction runs in a fixed order, so results do
// not depend on scheduling.
#include "common.h"
#include "kernels.h"

namespace feast {
namespace {

__global__ void pack_kernel(const double *src, int nc, int b, int bp, int m, int ldd,
                            double *dst) {
  const size_t total = (size_t)nc * bp * ldd;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(i % ldd);
    const size_t rr = i / ldd;
    const int r = (int)(rr % bp);
    const size_t c = rr / bp;
    dst[i] = (r < b && j < m) ? src[(c * b + r) * m + j] : 0.0;
  }
}

__global__ void unpack_kernel(const double *src, int nc, int b, int bp, int m, int lds,
                              const int *perm, double *dst) {
  const size_t total = (size_t)nc * b * m;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(i % m);
    const size_t rr = i / m;
    const int r = (int)(rr % b);
    const size_t c = rr / b;
    const int js = perm ? perm[j] : j;
    dst[i] = src[(c * bp + r) * lds + js];
  }
}

// ---------------------------------------------------------------------------
// Per-cell products.  One workgroup of kCellThreads threads walks the cells
// c = g, g + G, ... (G = gridDim.x) and forms (T V)_c = U_{c-1}^T V_{c-1} +
// D_c V_c + U_c V_{c+1} for all ld columns as a small GEMM: each of the (up
// to) three blocks is staged in LDS with the matching 64-row slab of V while
// the global loads of the next block are in flight, and the 16 waves share
// the 16x16 output tiles.  The consumers (plain product, projection, residual
// norms) use the cell's result right away and accumulate per workgroup in a
// fixed order.
// ---------------------------------------------------------------------------
constexpr int kCellThreads = 1024;
constexpr int kCellWaves = kCellThreads / 64;
constexpr int kCellGroups = 256;
constexpr int kVld = 128 + 16;  // LDS row stride of V slabs: rows 4 apart fall on other banks

// LDS of a cell workgroup: region r0 holds the A operands during the
// stages and (T V)_c (row stride kVld) in the epilogue; V holds the slab of
// the current stage, which is V_c in the last stage of every cell.
template <int BP, int NOP>
struct CellLds {
  static constexpr int ALD = BP + 1;
  static constexpr int R0 = NOP * BP * ALD > BP * kVld ? NOP * BP * ALD : BP * kVld;
  double r0[R0];
  double V[BP * kVld];
  __device__ double *A(int op) { return r0 + op * BP * ALD; }
  __device__ const double *A(int op) const { return r0 + op * BP * ALD; }
};

// The stages of cell c, in order: 0 = U_{c-1}^T with V_{c-1} (c > 0),
// 2 = U_c with V_{c+1} (c + 1 < nc), 1 = D_c with V_c (always, last).
__device__ __forceinline__ int stage_first(int c, int nc) {
  return c > 0 ? 0 : (c + 1 < nc ? 2 : 1);
}
__device__ __forceinline__ int stage_next(int c, int nc, int blk) {  // -1: cell done
  return blk == 0 ? (c + 1 < nc ? 2 : 1) : blk == 2 ? 1 : -1;
}

template <int BP, int NOP>
struct StageRegs {
  static constexpr int NA = (BP * BP + kCellThreads - 1) / kCellThreads;
  static constexpr int NV = (BP * 128 / 2 + kCellThreads - 1) / kCellThreads;  // pairs
  double a[NOP][NA];
  double2 v[NV];
};

template <int BP, int NOP>
__device__ __forceinline__ void stage_load(StageRegs<BP, NOP> &r, const double *const *D,
                                           const double *const *U, int nc, int b,
                                           const double *V, int ld, int c, int blk) {
  const int tid = threadIdx.x;
  const size_t bb = (size_t)b * b;
#pragma unroll
  for (int op = 0; op < NOP; ++op) {
    const double *M = blk == 0 ? U[op] + (size_t)(c - 1) * bb
                               : blk == 1 ? D[op] + (size_t)c * bb : U[op] + (size_t)c * bb;
#pragma unroll
    for (int i = 0; i < StageRegs<BP, NOP>::NA; ++i) {
      const int idx = tid + i * kCellThreads;
      const int x = idx / BP, y = idx % BP;  // memory order: row x, column y of M
      r.a[op][i] = (idx < BP * BP && x < b && y < b) ? M[x * b + y] : 0.0;
    }
  }
  const int cell = c - 1 + blk;
  const double2 *Vc = reinterpret_cast<const double2 *>(V + (size_t)cell * BP * ld);
  const int half = ld / 2;
#pragma unroll
  for (int i = 0; i < StageRegs<BP, NOP>::NV; ++i) {
    const int idx = tid + i * kCellThreads;
    r.v[i] = idx < BP * half ? Vc[idx] : double2{0.0, 0.0};
  }
}

// A operand in LDS as A[r][k]: U_{c-1}^T and D_c (symmetric) come from memory
// row k, column r; U_c from memory row r, column k.
template <int BP, int NOP>
__device__ __forceinline__ void stage_store(const StageRegs<BP, NOP> &r, CellLds<BP, NOP> &s,
                                            int ld, int blk) {
  constexpr int ALD = CellLds<BP, NOP>::ALD;
  const int tid = threadIdx.x;
#pragma unroll
  for (int op = 0; op < NOP; ++op)
#pragma unroll
    for (int i = 0; i < StageRegs<BP, NOP>::NA; ++i) {
      const int idx = tid + i * kCellThreads;
      const int x = idx / BP, y = idx % BP;
      if (idx < BP * BP) s.A(op)[blk == 2 ? x * ALD + y : y * ALD + x] = r.a[op][i];
    }
  const int half = ld / 2;
#pragma unroll
  for (int i = 0; i < StageRegs<BP, NOP>::NV; ++i) {
    const int idx = tid + i * kCellThreads;
    if (idx < BP * half) {
      const int k = idx / half, j = 2 * (idx % half);
      s.V[k * kVld + j] = r.v[i].x;
      s.V[k * kVld + j + 1] = r.v[i].y;
    }
  }
}

constexpr int kCellTiles = 2;  // output tiles a wave: (64 / 16) * (128 / 16) / 16

template <int BP, int NOP>
__device__ __forceinline__ void stage_mfma(const CellLds<BP, NOP> &s, int ld,
                                           d4 (&acc)[NOP][kCellTiles]) {
  constexpr int NR = BP / 16, ALD = CellLds<BP, NOP>::ALD;
  const int nct = ld / 16;
  const int l = lane_id(), w = wave_id(), kl = l >> 4;
#pragma unroll
  for (int i = 0; i < kCellTiles; ++i) {
    const int t = w + i * kCellWaves;
    if (t < NR * nct) {
      const int row = (t % NR) * 16 + (l & 15), col = (t / NR) * 16 + (l & 15);
#pragma unroll
      for (int ks = 0; ks < BP / 4; ++ks) {
        const int k = 4 * ks + kl;
        const double bv = s.V[k * kVld + col];
#pragma unroll
        for (int op = 0; op < NOP; ++op) acc[op][i] = mfma(s.A(op)[row * ALD + k], bv, acc[op][i]);
        if ((ks & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bounded register use
      }
    }
  }
}

// Runs the stages of every cell of this workgroup; epi(c, acc) is called
// with all threads after the last stage of cell c (LDS free to reuse until
// it returns, acc reset afterwards).
template <int BP, int NOP, typename EPI>
__device__ __forceinline__ void cell_loop(CellLds<BP, NOP> &s, const double *const *D,
                                          const double *const *U, int nc, int b,
                                          const double *V, int ld, EPI epi) {
  d4 acc[NOP][kCellTiles];
#pragma unroll
  for (int op = 0; op < NOP; ++op)
#pragma unroll
    for (int i = 0; i < kCellTiles; ++i) acc[op][i] = d4zero();
  int c = blockIdx.x;
  if (c >= nc) return;
  int blk = stage_first(c, nc);
  StageRegs<BP, NOP> r;
  stage_load<BP, NOP>(r, D, U, nc, b, V, ld, c, blk);
  while (true) {
    stage_store<BP, NOP>(r, s, ld, blk);
    __syncthreads();
    // next stage (possibly of the next cell) loads while this one computes
    int nc_ = c, nb = stage_next(c, nc, blk);
    if (nb < 0) {
      nc_ = c + gridDim.x;
      nb = nc_ < nc ? stage_first(nc_, nc) : 0;
    }
    if (nc_ < nc) stage_load<BP, NOP>(r, D, U, nc, b, V, ld, nc_, nb);
    stage_mfma<BP, NOP>(s, ld, acc);
    __syncthreads();
    if (nc_ != c) {
      epi(c, acc);
#pragma unroll
      for (int op = 0; op < NOP; ++op)
#pragma unroll
        for (int i = 0; i < kCellTiles; ++i) acc[op][i] = d4zero();
      if (nc_ >= nc) break;
    }
    c = nc_;
    blk = nb;
  }
}

// out = T V, all cells
template <int BP>
__global__ __launch_bounds__(kCellThreads) void cell_apply_kernel(const double *D, const double *U,
                                                                  int nc, int b, const double *V,
                                                                  int ld, double *out,
                                                                  const int *skip) {
  if (skip && *skip) return;  // a converged solve: later loops of a captured solve do nothing
  __shared__ CellLds<BP, 1> s;
  constexpr int NR = BP / 16;
  const int nct = ld / 16;
  const int l = lane_id(), w = wave_id();
  const double *Ds[1] = {D}, *Us[1] = {U};
  cell_loop<BP, 1>(s, Ds, Us, nc, b, V, ld, [&](int c, d4 (&acc)[1][kCellTiles]) {
#pragma unroll
    for (int i = 0; i < kCellTiles; ++i) {
      const int t = w + i * kCellWaves;
      if (t < NR * nct) {
        const int col = (t / NR) * 16 + acc_col(l);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          out[((size_t)c * BP + (t % NR) * 16 + acc_row(l, r)) * ld + col] = acc[0][i][r];
      }
    }
  });
}

// partial[g] = sum over the group's cells of Q_c^T (T Q)_c  (ld x ld)
constexpr int kProjTiles = 4;  // (128 / 16)^2 / 16

template <int BP>
__global__ __launch_bounds__(kCellThreads) void cell_project_kernel(const double *D,
                                                                    const double *U, int nc,
                                                                    int b, const double *Q,
                                                                    int ld, double *partial,
                                                                    const int *skip) {
  if (skip && *skip) return;  // a converged solve: later loops of a captured solve do nothing
  __shared__ CellLds<BP, 1> s;
  constexpr int NR = BP / 16;
  const int nct = ld / 16;
  const int l = lane_id(), w = wave_id(), kl = l >> 4;
  d4 pacc[kProjTiles];
#pragma unroll
  for (int i = 0; i < kProjTiles; ++i) pacc[i] = d4zero();
  // output tiles of this wave: ti = w % 8, tj = w / 8 + 2 i
  const int ti = w % 8;
  const double *Ds[1] = {D}, *Us[1] = {U};
  cell_loop<BP, 1>(s, Ds, Us, nc, b, Q, ld, [&](int c, d4 (&acc)[1][kCellTiles]) {
    // (T Q)_c into r0, then pacc += Q_c^T (T Q)_c with Q_c = the V slab
#pragma unroll
    for (int i = 0; i < kCellTiles; ++i) {
      const int t = w + i * kCellWaves;
      if (t < NR * nct) {
        const int col = (t / NR) * 16 + acc_col(l);
#pragma unroll
        for (int r = 0; r < 4; ++r) s.r0[((t % NR) * 16 + acc_row(l, r)) * kVld + col] = acc[0][i][r];
      }
    }
    __syncthreads();
    if (ti < nct) {
#pragma unroll
      for (int ks = 0; ks < BP / 4; ++ks) {
        const int k = 4 * ks + kl;
        const double a = s.V[k * kVld + ti * 16 + (l & 15)];
        // every tile, also those past nct (columns < 128 <= kVld stay inside
        // r0; their sums are never stored): no branch around the products
#pragma unroll
        for (int i = 0; i < kProjTiles; ++i) {
          const int tj = w / 8 + 2 * i;
          pacc[i] = mfma(a, s.r0[k * kVld + tj * 16 + (l & 15)], pacc[i]);
        }
        if ((ks & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bounded register use
      }
    }
    __syncthreads();
  });
  double *out = partial + (size_t)blockIdx.x * ld * ld;
  if (ti < nct)
#pragma unroll
    for (int i = 0; i < kProjTiles; ++i) {
      const int tj = w / 8 + 2 * i;
      if (tj < nct)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          out[(size_t)(ti * 16 + acc_row(l, r)) * ld + tj * 16 + acc_col(l)] = pacc[i][r];
    }
}

// M = 0.5 (S + S^T), S = sum over the groups' partials (group order), m0 x m0
// S = sum over the groups of their partial products, written to M: 64
// outputs per block, each summed by four threads over interleaved groups and
// combined in a fixed order (bitwise reproducible); symmetrize_kernel then
// forms (S + S^T) / 2.
__global__ __launch_bounds__(256) void cell_project_reduce_kernel(const double *partial, int groups,
                                                                  int ld, int m0, double *M,
                                                                  const int *skip) {
  if (skip && *skip) return;  // a converged solve: later loops of a captured solve do nothing
  __shared__ double red[4][64];
  const int e = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int idx = blockIdx.x * 64 + e;
  const bool in = idx < m0 * m0;
  const int i = in ? idx / m0 : 0, j = in ? idx % m0 : 0;
  double sum = 0.0;
  if (in) {
#pragma unroll 8
    for (int g = sl; g < groups; g += 4) sum += partial[((size_t)g * ld + i) * ld + j];
  }
  red[sl][e] = sum;
  __syncthreads();
  if (sl == 0 && in) M[idx] = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
}

// M <- (M + M^T) / 2 in place (m0 x m0), one thread per pair i < j.
__global__ void symmetrize_kernel(double *M, int m0, const int *skip) {
  if (skip && *skip) return;  // a converged solve: later loops of a captured solve do nothing
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m0 * m0) return;
  const int i = idx / m0, j = idx % m0;
  if (j <= i) return;
  const double v = 0.5 * (M[i * m0 + j] + M[j * m0 + i]);
  M[i * m0 + j] = v;
  M[j * m0 + i] = v;
}

// partial[g][3][ld] = per column: sum |A x - lam B x|, sum |A x|, sum |B x|
// over the group's cells (rows >= b of a cell are zero padding and add 0)
template <int BP>
__global__ __launch_bounds__(kCellThreads) void cell_residual_kernel(
    const double *Ad, const double *Au, const double *Bd, const double *Bu, int nc, int b,
    const double *X, int ld, const double *lam, int m0, double *partial, const int *skip) {
  if (skip && *skip) return;  // a converged solve: later loops of a captured solve do nothing
  __shared__ CellLds<BP, 2> s;
  constexpr int NR = BP / 16;
  const int nct = ld / 16;
  const int l = lane_id(), w = wave_id();
  double sums[kCellTiles][3];
  double lj[kCellTiles];
#pragma unroll
  for (int i = 0; i < kCellTiles; ++i) {
    const int t = w + i * kCellWaves;
    const int col = (t / NR) * 16 + acc_col(l);
    lj[i] = (t < NR * nct && col < m0) ? lam[col] : 0.0;
    sums[i][0] = sums[i][1] = sums[i][2] = 0.0;
  }
  const double *Ds[2] = {Ad, Bd}, *Us[2] = {Au, Bu};
  cell_loop<BP, 2>(s, Ds, Us, nc, b, X, ld, [&](int c, d4 (&acc)[2][kCellTiles]) {
#pragma unroll
    for (int i = 0; i < kCellTiles; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double a = acc[0][i][r], v = acc[1][i][r];
        sums[i][0] += fabs(a - lj[i] * v);
        sums[i][1] += fabs(a);
        sums[i][2] += fabs(v);
      }
  });
  // lanes l, l+16, l+32, l+48 hold the same column: fold them, then the waves
  // of equal column tile through LDS in wave order
#pragma unroll
  for (int i = 0; i < kCellTiles; ++i)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double v = sums[i][q];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      sums[i][q] = v;
    }
  double *red = s.r0;  // [3][kCellWaves * kCellTiles][16]
  __syncthreads();
  if (l < 16)
#pragma unroll
    for (int i = 0; i < kCellTiles; ++i)
#pragma unroll
      for (int q = 0; q < 3; ++q) red[(q * kCellWaves * kCellTiles + i * kCellWaves + w) * 16 + l] = sums[i][q];
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid < ld) {
    const int ct = tid / 16, lane = tid % 16;
    double tot[3] = {0.0, 0.0, 0.0};
    for (int t = ct * NR; t < (ct + 1) * NR; ++t) {  // tiles of this column tile
      const int i = t / kCellWaves, wv = t % kCellWaves;
#pragma unroll
      for (int q = 0; q < 3; ++q) tot[q] += red[(q * kCellWaves * kCellTiles + i * kCellWaves + wv) * 16 + lane];
    }
    double *out = partial + (size_t)blockIdx.x * 3 * ld;
#pragma unroll
    for (int q = 0; q < 3; ++q) out[q * ld + tid] = tot[q];
  }
}

// Float64 residuals of the shifted systems for the mixed-precision solves:
// r_e = R - (Z_e B - A) x_e with x_e = xr + i xi, in two passes over the
// planes of x_e so that each pass is one cell loop over A and B:
//   pass 0:  re = R + A xr - zr B xr,   im = -zi B xr
//   pass 1:  re += zi B xi,             im += A xi - zr B xi
// Node e = blockIdx.y.  Per column and group, pass P writes the sums
// partial[e][g][3 P + q][ld]: q = 0 |A x_P|^2, q = 1 |B x_P|^2 and q = 2
// R^2 (pass 0) or |r_e|^2 (pass 1), with x_0 = xr, x_1 = xi.
constexpr int kShiftSums = 6;

template <int BP, int PASS>
__global__ __launch_bounds__(kCellThreads) void cell_shift_residual_kernel(
    const double *Ad, const double *Au, const double *Bd, const double *Bu, int nc, int b,
    const double *X, const double *R, int ld, size_t plane, Shifts sh, double *Rout,
    double *partial) {
  __shared__ CellLds<BP, 2> s;
  constexpr int NR = BP / 16;
  const int nct = ld / 16;
  const int l = lane_id(), w = wave_id();
  const int e = blockIdx.y;
  const double zr = sh.zre[e], zi = sh.zim[e];
  const double *V = X + (2 * e + PASS) * plane;
  double *Ore = Rout + 2 * e * plane;
  double *Oim = Ore + plane;
  double sums[kCellTiles][3];
#pragma unroll
  for (int i = 0; i < kCellTiles; ++i) sums[i][0] = sums[i][1] = sums[i][2] = 0.0;
  const double *Ds[2] = {Ad, Bd}, *Us[2] = {Au, Bu};
  cell_loop<BP, 2>(s, Ds, Us, nc, b, V, ld, [&](int c, d4 (&acc)[2][kCellTiles]) {
#pragma unroll
    for (int i = 0; i < kCellTiles; ++i) {
      const int t = w + i * kCellWaves;
      if (t < NR * nct) {
        const int col = (t / NR) * 16 + acc_col(l);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const size_t idx = ((size_t)c * BP + (t % NR) * 16 + acc_row(l, r)) * ld + col;
          const double a = acc[0][i][r], bx = acc[1][i][r];
          double re, im;
          if (PASS == 0) {
            const double rv = R[idx];
            re = rv + a - zr * bx;
            im = -zi * bx;
            sums[i][2] += rv * rv;
          } else {
            re = Ore[idx] + zi * bx;
            im = Oim[idx] + a - zr * bx;
            sums[i][2] += re * re + im * im;
          }
          sums[i][0] += a * a;
          sums[i][1] += bx * bx;
          Ore[idx] = re;
          Oim[idx] = im;
        }
      }
    }
  });
  // lanes l, l+16, l+32, l+48 hold the same column: fold them, then the waves
  // of equal column tile through LDS in wave order
#pragma unroll
  for (int i = 0; i < kCellTiles; ++i)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double v = sums[i][q];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      sums[i][q] = v;
    }
  double *red = s.r0;  // [3][tile t = w + i kCellWaves][16]
  constexpr int NT = kCellWaves * kCellTiles;
  __syncthreads();
  if (l < 16)
#pragma unroll
    for (int i = 0; i < kCellTiles; ++i)
#pragma unroll
      for (int q = 0; q < 3; ++q) red[(q * NT + i * kCellWaves + w) * 16 + l] = sums[i][q];
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid < ld) {
    const int ct = tid / 16, lane = tid % 16;
    double tot[3] = {0.0, 0.0, 0.0};
    for (int t = ct * NR; t < (ct + 1) * NR; ++t)
#pragma unroll
      for (int q = 0; q < 3; ++q) tot[q] += red[(q * NT + t) * 16 + lane];
    double *out = partial + (((size_t)e * gridDim.x + blockIdx.x) * kShiftSums + 3 * PASS) * ld;
#pragma unroll
    for (int q = 0; q < 3; ++q) out[q * ld + tid] = tot[q];
  }
}

// ratio[e][j] = ||r_j|| / (||R_j|| + |Z_e| ||B x_j|| + ||A x_j||) (2-norms),
// the residual relative to the size of the terms it is computed from, for
// node e and column j < m0 (one thread each; group sums in group order).
__global__ __launch_bounds__(256) void shift_residual_ratio_kernel(const double *partial,
                                                                   int groups, int ld, int m0,
                                                                   int Ne, Shifts sh,
                                                                   double *ratio) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Ne * m0) return;
  const int e = idx / m0, j = idx % m0;
  double t[kShiftSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int g = 0; g < groups; ++g)
#pragma unroll
    for (int q = 0; q < kShiftSums; ++q)
      t[q] += partial[(((size_t)e * groups + g) * kShiftSums + q) * ld + j];
  const double za = sqrt(sh.zre[e] * sh.zre[e] + sh.zim[e] * sh.zim[e]);
  const double den = sqrt(t[2]) + za * sqrt(t[1] + t[4]) + sqrt(t[0] + t[3]);
  const double num = sqrt(t[5]);
  ratio[idx] = den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
}

// worst = max of the count ratios (one workgroup); a NaN (non-finite
// iterate) counts as infinity, so it never passes the refinement test
__global__ __launch_bounds__(256) void max_ratio_kernel(const double *ratio, int count,
                                                        double *worst) {
  __shared__ double red[256];
  double mx = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) {
    const double q = ratio[i];
    mx = (q == q) ? fmax(mx, q) : INFINITY;
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *worst = red[0];
}

// Q = sum_e (kr_e xr_e - ki_e xi_e), nodes in order.
__global__ void sum_nodes_complex_kernel(Shifts sh, int Ne, const double *X, size_t plane,
                                         double *Q) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < plane;
       i += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int e = 0; e < Ne; ++e)
      s += sh.kre[e] * X[2 * e * plane + i] - sh.kim[e] * X[(2 * e + 1) * plane + i];
    Q[i] = s;
  }
}

__global__ void sum_nodes_kernel(const double *P, int Ne, size_t count, double *Q,
                                 const int *skip) {
  if (skip && *skip) return;  // a converged solve: later loops of a captured solve do nothing
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int e = 0; e < Ne; ++e) s += P[(size_t)e * count + i];
    Q[i] = s;
  }
}

// X[row][j] = sum_{k<m0} Q[row][k] Phi[k][j]; columns m0..m0p-1 are zero
// (m0p = 16 NCT).  One wave per 16 rows and every column tile, so each row
// of Q is read once from memory; Phi (m0 x m0, finite) is read through the
// caches, its padding zeroed by a 0/1 factor on an unconditional in-bounds
// load (a select lets the compiler put the load behind a branch).
template <int NCT>
__global__ __launch_bounds__(256) void gemm_qphi_kernel(const double *Q, size_t rows, int m0,
                                                        const double *Phi, double *X,
                                                        const int *skip) {
  if (skip && *skip) return;  // a converged solve: later loops of a captured solve do nothing
  constexpr int M0P = 16 * NCT;
  const int l = lane_id(), w = wave_id();
  const size_t rbase = ((size_t)blockIdx.x * 4 + w) * 16;
  if (rbase >= rows) return;
  const int kl = l >> 4;
  const size_t row = rbase + (l & 15);
  d4 acc[NCT];
#pragma unroll
  for (int q = 0; q < NCT; ++q) acc[q] = d4zero();
#pragma unroll
  for (int k0 = 0; k0 < M0P; k0 += 4) {
    const int ka = k0 + kl;
    const double a = Q[row * M0P + ka];
    const int kc = ka < m0 ? ka : m0 - 1;
#pragma unroll
    for (int q = 0; q < NCT; ++q) {
      const int col = q * 16 + (l & 15);
      const double v = Phi[(size_t)kc * m0 + (col < m0 ? col : m0 - 1)];
      acc[q] = mfma(a, v * ((ka < m0 && col < m0) ? 1.0 : 0.0), acc[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < NCT; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      X[(rbase + acc_row(l, r)) * M0P + q * 16 + acc_col(l)] = acc[q][r];
}

// One block per column: 256 threads sum interleaved chunks, then a fixed
// tree in LDS (bitwise reproducible).
__global__ __launch_bounds__(256) void residual_reduce_kernel(const double *partial, int nchunks,
                                                              int m0p, int m0, double emin,
                                                              double emax, double *res,
                                                              const int *skip) {
  if (skip && *skip) return;  // a converged solve: later loops of a captured solve do nothing
  __shared__ double red[3][256];
  const int j = blockIdx.x, t = threadIdx.x;
  double num = 0.0, na = 0.0, nb = 0.0;
  for (int c = t; c < nchunks; c += 256) {
    const double *p = partial + (size_t)c * 3 * m0p;
    num += p[j];
    na += p[m0p + j];
    nb += p[2 * m0p + j];
  }
  red[0][t] = num;
  red[1][t] = na;
  red[2][t] = nb;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      red[0][t] += red[0][t + h];
      red[1][t] += red[1][t + h];
      red[2][t] += red[2][t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double r = 0.5 * (emax - emin);
    const double big = fmax(fmax(fabs(emin), fabs(emax)), r);
    const double den = (red[1][0] < r * red[2][0]) ? red[2][0] * big : red[1][0];
    res[j] = red[0][0] / den;
  }
}

// ---- blocks of 64 < b <= 96: products with the packed planes of the wide
// factorisation (layout fpos, see factor.hip) ----
//
// Tile (row block w, column tile tj) of (T V)_c for T = A (which = 0) or B (1):
//   D_c V_c + U_c V_{c+1} + U_{c-1}^T V_{c-1},
// the matrix operands as fragments of the packed planes (D_c symmetric: its
// own plane; U_c: the plane of U_c^T; U_{c-1}^T: the plane of U_{c-1}), the
// vector operand V[k][tj*16 + lane%16] from memory (V padded [nc][96][ld]).
constexpr int kWideB = 96;

__device__ __forceinline__ d4 wide_tile(const WidePack &pk, int which, int nc, int c, int w,
                                        int tj, const double *V, int ld) {
  constexpr int KS = kWideB / 4;
  const size_t per = (size_t)kWideB * kWideB;
  const int l = lane_id(), kl = l >> 4, n = l & 15;
  d4 a0 = d4zero(), a1 = d4zero(), a2 = d4zero();
  double f[KS];
  frag_plane_load<kWideB>(f, pk.dia + ((size_t)c * 2 + which) * per, w, true);
  const double *v0 = V + (size_t)c * kWideB * ld + tj * 16 + n;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) a0 = mfma(f[ks], v0[(size_t)(4 * ks + kl) * ld], a0);
  if (c + 1 < nc) {
    frag_plane_load<kWideB>(f, pk.cplt + ((size_t)c * 2 + which) * per, w, true);
    const double *v1 = v0 + (size_t)kWideB * ld;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a1 = mfma(f[ks], v1[(size_t)(4 * ks + kl) * ld], a1);
  }
  if (c > 0) {
    frag_plane_load<kWideB>(f, pk.cpl + ((size_t)(c - 1) * 2 + which) * per, w, true);
    const double *vm = v0 - (size_t)kWideB * ld;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a2 = mfma(f[ks], vm[(size_t)(4 * ks + kl) * ld], a2);
  }
  return (a0 + a1) + a2;
}

// out = T V; one workgroup of six waves per (cell, 16-column tile)
__global__ __launch_bounds__(384) void wide_apply_kernel(WidePack pk, int which, int nc,
                                                         const double *V, int ld, double *out,
                                                         const int *skip) {
  if (skip && *skip) return;
  const int c = blockIdx.x, tj = blockIdx.y, w = wave_id(), l = lane_id();
  const d4 acc = wide_tile(pk, which, nc, c, w, tj, V, ld);
#pragma unroll
  for (int r = 0; r < 4; ++r)
    out[((size_t)c * kWideB + w * 16 + acc_row(l, r)) * ld + tj * 16 + acc_col(l)] = acc[r];
}

// partial[c][3][ld]: per column j < m0 of cell c, the sums of |A x - lam_j B x|,
// |A x| and |B x| over the cell's rows (fixed order: rows within a lane,
// then the four lanes of a column, then the six row blocks)
__global__ __launch_bounds__(384) void wide_residual_kernel(WidePack pk, int nc, const double *X,
                                                            int ld, const double *lam, int m0,
                                                            double *partial, const int *skip) {
  if (skip && *skip) return;
  __shared__ double red[3][6][16];
  const int c = blockIdx.x, tj = blockIdx.y, w = wave_id(), l = lane_id();
  const d4 ax = wide_tile(pk, 0, nc, c, w, tj, X, ld);
  const d4 bx = wide_tile(pk, 1, nc, c, w, tj, X, ld);
  const int j = tj * 16 + acc_col(l);
  const double lj = j < m0 ? lam[j] : 0.0;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    s0 += fabs(ax[r] - lj * bx[r]);
    s1 += fabs(ax[r]);
    s2 += fabs(bx[r]);
  }
  // lanes n, n+16, n+32, n+48 hold the same column
  s0 += __shfl_xor(s0, 16);
  s1 += __shfl_xor(s1, 16);
  s2 += __shfl_xor(s2, 16);
  s0 += __shfl_xor(s0, 32);
  s1 += __shfl_xor(s1, 32);
  s2 += __shfl_xor(s2, 32);
  if (l < 16) {
    red[0][w][l] = s0;
    red[1][w][l] = s1;
    red[2][w][l] = s2;
  }
  __syncthreads();
  if (threadIdx.x < 48) {
    const int q = threadIdx.x / 16, n = threadIdx.x % 16;
    double s = 0.0;
    for (int ww = 0; ww < 6; ++ww) s += red[q][ww][n];
    partial[((size_t)c * 3 + q) * ld + tj * 16 + n] = s;
  }
}

__global__ void check_finite_kernel(const double *x, size_t count, int *flag) {
  int bad = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) bad = 1;
  if (bad) atomicOr(flag, 1);
}

__global__ void gather_kernel(const double *src, const int *perm, int m, double *dst) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) dst[j] = src[perm[j]];
}

int grid_for(size_t n, int threads) {
  size_t g = (n + threads - 1) / threads;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

// ---- random start (Fig. 2 step 1: M0 random vectors) ----
//
// Element t = i*m + j of the start block Y0[N][m] is standard normal, drawn
// from the counter-based generator Philox4x64-10 (Salmon, Moraes, Dror and
// Shaw, SC'11): counter (t/4, 0, 0, 0), key (seed, 0); its four 64-bit words
// give four uniforms u_k = (w_k >> 11) 2^-53 + 2^-54 in (0, 1), and the
// Box-Muller pairs (u0, u1), (u2, u3) give four normals
// sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b); element t takes normal t % 4.

__device__ inline void philox4x64_10(unsigned long long c[4], unsigned long long k0,
                                     unsigned long long k1) {
  const unsigned long long m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
  const unsigned long long w0 = 0x9E3779B97F4A7C15ull, w1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const unsigned long long hi0 = __umul64hi(m0, c[0]), lo0 = m0 * c[0];
    const unsigned long long hi1 = __umul64hi(m1, c[2]), lo1 = m1 * c[2];
    const unsigned long long n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += w0;
    k1 += w1;
  }
}

__global__ void random_start_kernel(unsigned long long seed, int nc, int b, int bp, int m,
                                    int ldd, double *dst) {
  const size_t total = (size_t)nc * bp * ldd;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(i % ldd);
    const size_t rr = i / ldd;
    const int r = (int)(rr % bp);
    const size_t c = rr / bp;
    double v = 0.0;
    if (r < b && j < m) {
      const unsigned long long t = (unsigned long long)((c * b + r) * m + j);
      unsigned long long w[4] = {t >> 2, 0ull, 0ull, 0ull};
      philox4x64_10(w, seed, 0ull);
      const int lane = (int)(t & 3);
      const int pa = lane & 2;  // the pair (u0, u1) or (u2, u3)
      const double ua = (double)(w[pa] >> 11) * 0x1p-53 + 0x1p-54;
      const double ub = (double)(w[pa + 1] >> 11) * 0x1p-53 + 0x1p-54;
      const double rho = sqrt(-2.0 * log(ua));
      const double ang = 2.0 * M_PI * ub;
      v = (lane & 1) ? rho * sin(ang) : rho * cos(ang);
    }
    dst[i] = v;
  }
}

hipError_t launch_random_start(unsigned long long seed, int nc, int b, int bp, int m, int ldd,
                               double *dst, hipStream_t st) {
  size_t n = (size_t)nc * bp * ldd;
  hipLaunchKernelGGL(random_start_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, seed, nc, b,
                     bp, m, ldd, dst);
  return hipGetLastError();
}

hipError_t launch_pack(const double *src, int nc, int b, int bp, int m, int ldd, double *dst,
                       hipStream_t st) {
  size_t n = (size_t)nc * bp * ldd;
  hipLaunchKernelGGL(pack_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, src, nc, b, bp, m,
                     ldd, dst);
  return hipGetLastError();
}

hipError_t launch_unpack(const double *src, int nc, int b, int bp, int m, int lds,
                         const int *perm, double *dst, hipStream_t st) {
  size_t n = (size_t)nc * b * m;
  hipLaunchKernelGGL(unpack_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, src, nc, b, bp, m,
                     lds, perm, dst);
  return hipGetLastError();
}

hipError_t launch_sum_nodes(const double *P, int Ne, size_t count, double *Q, hipStream_t st,
                            const int *skip) {
  hipLaunchKernelGGL(sum_nodes_kernel, dim3(grid_for(count, 256)), dim3(256), 0, st, P, Ne, count,
                     Q, skip);
  return hipGetLastError();
}

hipError_t launch_gemm_qphi(const double *Q, size_t rows, int m0p, int m0, const double *Phi,
                            double *X, hipStream_t st,
                            const int *skip) {
  if (m0 < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((rows + 63) / 64)), block(256);
  switch (m0p) {
    case 16: hipLaunchKernelGGL(gemm_qphi_kernel<1>, grid, block, 0, st, Q, rows, m0, Phi, X, skip); break;
    case 32: hipLaunchKernelGGL(gemm_qphi_kernel<2>, grid, block, 0, st, Q, rows, m0, Phi, X, skip); break;
    case 48: hipLaunchKernelGGL(gemm_qphi_kernel<3>, grid, block, 0, st, Q, rows, m0, Phi, X, skip); break;
    case 64: hipLaunchKernelGGL(gemm_qphi_kernel<4>, grid, block, 0, st, Q, rows, m0, Phi, X, skip); break;
    case 80: hipLaunchKernelGGL(gemm_qphi_kernel<5>, grid, block, 0, st, Q, rows, m0, Phi, X, skip); break;
    case 96: hipLaunchKernelGGL(gemm_qphi_kernel<6>, grid, block, 0, st, Q, rows, m0, Phi, X, skip); break;
    case 112: hipLaunchKernelGGL(gemm_qphi_kernel<7>, grid, block, 0, st, Q, rows, m0, Phi, X, skip); break;
    case 128: hipLaunchKernelGGL(gemm_qphi_kernel<8>, grid, block, 0, st, Q, rows, m0, Phi, X, skip); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

namespace {

// One loop's convergence decision on the device, in the host loop's order
// and arithmetic (see launch_converge in kernels.h).
__global__ void converge_kernel(const double *eps, const double *res, const int *flag, int m0,
                                double emin, double emax, double gate, double tol, double r,
                                double drop, int max_loops, DevConv *s) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (s->done) return;
  const int k = s->k + 1;
  const int fb = flag[0];
  s->fallback = fb;
  s->rr_sweeps += flag[1] + (fb ? flag[2] : 0);
  int mk = 0;
  double tk = 0.0, left_min = INFINITY;
  for (int j = 0; j < m0; ++j) {
    const double e = eps[j], rj = res[j];
    const bool in = e >= emin && e <= emax;
    if (in && rj <= gate) {
      ++mk;
      tk += e;
    } else if (in) {
      left_min = rj < left_min ? rj : left_min;
    }
  }
  const bool still = left_min < drop * s->prev_left_min;
  s->prev_left_min = left_min;
  double trace_rel = s->trace_rel;
  if (k >= 2) {
    if (mk == 0 && s->last_count == 0) {
      trace_rel = 0.0;
    } else {
      const double a = fabs(tk), c = mk * r;
      trace_rel = fabs(tk - s->last_trace) / (a < c ? c : a);
    }
  }
  const bool conv = k >= 2 && mk == s->last_count && trace_rel < tol && !still;
  if (k <= 64) {
    s->counts[k - 1] = mk;
    s->traces[k - 1] = tk;
  }
  s->last_trace = tk;
  s->last_count = mk;
  s->trace_rel = trace_rel;
  s->k = k;
  s->converged = conv ? 1 : 0;
  s->done = (conv || k >= max_loops) ? 1 : 0;
}

}  // namespace

hipError_t launch_converge(const double *eps, const double *res, const int *flag, int m0,
                           double emin, double emax, double gate, double tol, double r,
                           double drop, int max_loops, DevConv *st_dev, hipStream_t st) {
  hipLaunchKernelGGL(converge_kernel, dim3(1), dim3(64), 0, st, eps, res, flag, m0, emin, emax,
                     gate, tol, r, drop, max_loops, st_dev);
  return hipGetLastError();
}

hipError_t launch_wide_apply(const Pencil &p, const WidePack &pk, int which, const double *V,
                             int ld, double *out, hipStream_t st, const int *skip) {
  if (p.bp != kWideB || ld % 16 != 0 || ld > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL(wide_apply_kernel, dim3(p.nc, ld / 16), dim3(384), 0, st, pk, which, p.nc, V,
                     ld, out, skip);
  return hipGetLastError();
}

size_t wide_residual_partial_doubles(int nc, int ld) { return (size_t)nc * 3 * ld; }

hipError_t launch_wide_residuals(const Pencil &p, const WidePack &pk, const double *X, int ld,
                                 const double *lam, int m0, double emin, double emax,
                                 double *partial, double *res, hipStream_t st, const int *skip) {
  if (p.bp != kWideB || ld % 16 != 0 || ld > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL(wide_residual_kernel, dim3(p.nc, ld / 16), dim3(384), 0, st, pk, p.nc, X, ld,
                     lam, m0, partial, skip);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(residual_reduce_kernel, dim3(m0), dim3(256), 0, st, (const double *)partial,
                     p.nc, ld, m0, emin, emax, res, skip);
  return hipGetLastError();
}

// A_Q = Q^T (A Q), B_Q = Q^T (B Q), each symmetrised: the wide products into
// tmp, the cross Gram products (warm.hip) over all padded rows.
hipError_t launch_wide_project(const Pencil &p, const WidePack &pk, const double *Q, int ld,
                               int m0, double *tmp, double *partial, double *AQ, double *BQ,
                               hipStream_t st, const int *skip) {
  const long long rows = (long long)p.nc * kWideB;
  for (int z = 0; z < 2; ++z) {
    hipError_t err = launch_wide_apply(p, pk, z, Q, ld, tmp, st, skip);
    if (err != hipSuccess) return err;
    double *M = z ? BQ : AQ;
    if ((err = launch_cross_gram(Q, ld, tmp, ld, rows, m0, m0, partial, M, st)) != hipSuccess)
      return err;
    hipLaunchKernelGGL(symmetrize_kernel, dim3((m0 * m0 + 255) / 256), dim3(256), 0, st, M, m0,
                       skip);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t launch_check_finite(const double *x, size_t count, int *flag, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(check_finite_kernel, dim3(grid_for(count, 256)), dim3(256), 0, st, x, count,
                     flag);
  return hipGetLastError();
}

hipError_t launch_gather(const double *src, const int *perm, int m, double *dst, hipStream_t st) {
  hipLaunchKernelGGL(gather_kernel, dim3((m + 127) / 128), dim3(128), 0, st, src, perm, m, dst);
  return hipGetLastError();
}


int cell_groups(int nc) { return nc < kCellGroups ? nc : kCellGroups; }

size_t cell_partial_doubles(int nc, int ld) {
  return (size_t)cell_groups(nc) * ld * ld;
}

template <int BP>
hipError_t cell_apply_bp(const double *D, const double *U, int nc, int b, const double *V, int ld,
                         double *out, hipStream_t st, const int *skip) {
  hipLaunchKernelGGL(cell_apply_kernel<BP>, dim3(cell_groups(nc)), dim3(kCellThreads), 0, st, D,
                     U, nc, b, V, ld, out, skip);
  return hipGetLastError();
}

hipError_t launch_cell_apply(const Pencil &p, int which, const double *V, int ld, double *out,
                             hipStream_t st, const int *skip) {
  const double *D = which ? p.Bd : p.Ad;
  const double *U = which ? p.Bu : p.Au;
  if (ld % 16 != 0 || ld > 128) return hipErrorInvalidValue;
  switch (p.bp) {
    case 16: return cell_apply_bp<16>(D, U, p.nc, p.b, V, ld, out, st, skip);
    case 32: return cell_apply_bp<32>(D, U, p.nc, p.b, V, ld, out, st, skip);
    case 48: return cell_apply_bp<48>(D, U, p.nc, p.b, V, ld, out, st, skip);
    case 64: return cell_apply_bp<64>(D, U, p.nc, p.b, V, ld, out, st, skip);
    default: return hipErrorInvalidValue;
  }
}

template <int BP>
hipError_t cell_project_bp(const Pencil &p, const double *Q, int ld, int m0, double *partial,
                           double *AQ, double *BQ, hipStream_t st, const int *skip) {
  const int G = cell_groups(p.nc);
  for (int z = 0; z < 2; ++z) {
    const double *D = z ? p.Bd : p.Ad;
    const double *U = z ? p.Bu : p.Au;
    hipLaunchKernelGGL(cell_project_kernel<BP>, dim3(G), dim3(kCellThreads), 0, st, D, U, p.nc,
                       p.b, Q, ld, partial, skip);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(cell_project_reduce_kernel, dim3((m0 * m0 + 63) / 64), dim3(256), 0, st,
                       (const double *)partial, G, ld, m0, z ? BQ : AQ, skip);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(symmetrize_kernel, dim3((m0 * m0 + 255) / 256), dim3(256), 0, st,
                       z ? BQ : AQ, m0, skip);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t launch_cell_project(const Pencil &p, const double *Q, int ld, int m0, double *partial,
                               double *AQ, double *BQ, hipStream_t st, const int *skip) {
  if (ld % 16 != 0 || ld > 128) return hipErrorInvalidValue;
  switch (p.bp) {
    case 16: return cell_project_bp<16>(p, Q, ld, m0, partial, AQ, BQ, st, skip);
    case 32: return cell_project_bp<32>(p, Q, ld, m0, partial, AQ, BQ, st, skip);
    case 48: return cell_project_bp<48>(p, Q, ld, m0, partial, AQ, BQ, st, skip);
    case 64: return cell_project_bp<64>(p, Q, ld, m0, partial, AQ, BQ, st, skip);
    default: return hipErrorInvalidValue;
  }
}

template <int BP>
hipError_t cell_residual_bp(const Pencil &p, const double *X, int ld, const double *lam, int m0,
                            double emin, double emax, double *partial, double *res,
                            hipStream_t st, const int *skip) {
  const int G = cell_groups(p.nc);
  hipLaunchKernelGGL(cell_residual_kernel<BP>, dim3(G), dim3(kCellThreads), 0, st, p.Ad, p.Au,
                     p.Bd, p.Bu, p.nc, p.b, X, ld, lam, m0, partial, skip);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(residual_reduce_kernel, dim3(m0), dim3(256), 0, st,
                     (const double *)partial, G, ld, m0, emin, emax, res, skip);
  return hipGetLastError();
}

hipError_t launch_cell_residuals(const Pencil &p, const double *X, int ld, const double *lam,
                                 int m0, double emin, double emax, double *partial, double *res,
                                 hipStream_t st, const int *skip) {
  if (ld % 16 != 0 || ld > 128) return hipErrorInvalidValue;
  switch (p.bp) {
    case 16: return cell_residual_bp<16>(p, X, ld, lam, m0, emin, emax, partial, res, st, skip);
    case 32: return cell_residual_bp<32>(p, X, ld, lam, m0, emin, emax, partial, res, st, skip);
    case 48: return cell_residual_bp<48>(p, X, ld, lam, m0, emin, emax, partial, res, st, skip);
    case 64: return cell_residual_bp<64>(p, X, ld, lam, m0, emin, emax, partial, res, st, skip);
    default: return hipErrorInvalidValue;
  }
}

size_t shift_residual_partial_doubles(int nc, int ld, int Ne) {
  return (size_t)cell_groups(nc) * ld * Ne * kShiftSums + (size_t)Ne * ld;  // + ratios
}

template <int BP>
hipError_t shift_residual_bp(const Pencil &p, const Shifts &s, int Ne, const double *X,
                             const double *R, int ld, int m0, double *Rout, double *partial,
                             double *worst, hipStream_t st) {
  const int G = cell_groups(p.nc);
  const size_t plane = (size_t)p.nc * p.bp * ld;
  const dim3 grid(G, Ne);
  hipLaunchKernelGGL((cell_shift_residual_kernel<BP, 0>), grid, dim3(kCellThreads), 0, st, p.Ad,
                     p.Au, p.Bd, p.Bu, p.nc, p.b, X, R, ld, plane, s, Rout, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((cell_shift_residual_kernel<BP, 1>), grid, dim3(kCellThreads), 0, st, p.Ad,
                     p.Au, p.Bd, p.Bu, p.nc, p.b, X, R, ld, plane, s, Rout, partial);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  double *ratio = partial + (size_t)G * ld * Ne * kShiftSums;
  hipLaunchKernelGGL(shift_residual_ratio_kernel, dim3((Ne * m0 + 255) / 256), dim3(256), 0, st,
                     (const double *)partial, G, ld, m0, Ne, s, ratio);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(max_ratio_kernel, dim3(1), dim3(256), 0, st, (const double *)ratio, Ne * m0,
                     worst);
  return hipGetLastError();
}

hipError_t launch_shift_residuals(const Pencil &p, const Shifts &s, int Ne, const double *X,
                                  const double *R, int ld, int m0, double *Rout, double *partial,
                                  double *worst, hipStream_t st) {
  if (ld % 16 != 0 || ld > 128 || Ne < 1 || Ne > kMaxNe) return hipErrorInvalidValue;
  switch (p.bp) {
    case 16: return shift_residual_bp<16>(p, s, Ne, X, R, ld, m0, Rout, partial, worst, st);
    case 32: return shift_residual_bp<32>(p, s, Ne, X, R, ld, m0, Rout, partial, worst, st);
    case 48: return shift_residual_bp<48>(p, s, Ne, X, R, ld, m0, Rout, partial, worst, st);
    case 64: return shift_residual_bp<64>(p, s, Ne, X, R, ld, m0, Rout, partial, worst, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sum_nodes_complex(const Shifts &s, int Ne, const double *X, size_t plane,
                                    double *Q, hipStream_t st) {
  hipLaunchKernelGGL(sum_nodes_complex_kernel, dim3(grid_for(plane, 256)), dim3(256), 0, st, s,
                     Ne, X, plane, Q);
  return hipGetLastError();
}

}  // namespace feast
