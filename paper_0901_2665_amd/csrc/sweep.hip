// Forward and back sweeps of the twisted block factorisation: the shifted
// solves (Z_e B - A) Q_e = B Y of Fig. 2 step 2 for every node e and every
// right-hand side, fused with the quadrature weight of eq. 15.
//
// One workgroup runs one chain: (node e, tile of 8 complex right-hand sides,
// top or bottom half).  With complex symmetric factors (Sinv_j = Sinv_j^T,
// U_j^T Sinv_j = W_j^T) the forward sweep needs one product on its critical
// path:
//   h_0 = R_0,  h_{j+1} = R_{j+1} - W_j^T h_j,   g_j = Sinv_j h_j,
// the twist cell solves x_{m-1} = T (h_{m-1} - W~_m^T h~_m) and the back
// sweep is
//   x_j = g_j - W_j x_{j+1}   (top),   x_j = g~_j - W~_j x_{j-1}   (bottom).
// The back sweep writes P_e = Re(kappa_e x) so that Q = sum_e P_e.
//
// Products run on V_MFMA_F64_16X16X4_F64 with the complex product written as
// one real product over a doubled inner dimension:
//   [Mr | Mi] (16 x 2BP)  x  [[hr | hi]; [-hi | hr]] (2BP x 16)  =  [Re | Im].
// The matrix operand streams from global memory (L2); the vector operand
// comes from LDS, where each step leaves its result for the next one.
#include "common.h"
#include "kernels.h"

namespace feast {
namespace {

// LDS vector tile [plane][row][col] of BP x 8 complex values: the second
// plane starts 16 doubles after the packed position, so that the two planes
// of the rows one half-wave touches fall on different LDS banks.
template <int BP>
struct VecLds {
  static constexpr int PL = BP * kTile + 16;  // plane stride (doubles)
  double v[2][2 * PL];                        // [buffer][plane ...]
};

// Matrix-operand fragments of one stored block for this lane: the product
// uses the transpose of the stored block, A'[row][k] = M_plane[k][row].  In
// the factor layout (fpos) the k-steps 2p and 2p+1 of this lane are adjacent,
// so each 16-byte load fetches two of them and a wave reads 1 KB
// contiguously.  rb is the 16-row block of the output that the calling wave
// computes.  Fragments of the next cell are loaded one step ahead, so that
// the L2/HBM latency hides behind the current step's matrix-core work.
template <int BP>
struct Frag {
  double v[BP / 2];  // [plane][k-step]: BP/4 k-steps per plane
};

// The loads go through a buffer resource spanning exactly the one block (or
// nothing, valid = false), so that the per-pair displacement sits in a
// scalar offset and every load of the lane shares one address register.
template <int BP>
__device__ __forceinline__ void frag_load(Frag<BP> &f, const double *M, int rb, bool valid) {
  const int l = lane_id();
  const int row = rb * 16 + (l & 15), kl = l >> 4;
  const auto rs = buf_rsrc(M, valid ? 2 * BP * BP * 8 : 0);
  const int vo = fpos<BP>(kl, row) * 8;  // pair p = 0; fpos(8p + kl, row) adds 8 p BP
#pragma unroll
  for (int p = 0; p < BP / 8; ++p) {
    const auto v0 = __builtin_amdgcn_raw_buffer_load_b128(rs, vo, p * 8 * BP * 8, 0);
    const auto v1 =
        __builtin_amdgcn_raw_buffer_load_b128(rs, vo, (BP * BP + p * 8 * BP) * 8, 0);
    f.v[2 * p] = __builtin_bit_cast(double, (u32x2){v0[0], v0[1]});
    f.v[2 * p + 1] = __builtin_bit_cast(double, (u32x2){v0[2], v0[3]});
    f.v[BP / 4 + 2 * p] = __builtin_bit_cast(double, (u32x2){v1[0], v1[1]});
    f.v[BP / 4 + 2 * p + 1] = __builtin_bit_cast(double, (u32x2){v1[2], v1[3]});
  }
}

// Vector operand B' = [[hr | hi]; [-hi | hr]] of this lane, read from the LDS
// vector tile hv in one batch (b[ks] for k < BP, b[BP/4 + ks] for k >= BP).
// (Reading one plane and taking the other from lane n+8 by a row shift
// halves the LDS reads but makes the matrix cores wait for all of them:
// measured slower.)
template <int BP>
__device__ __forceinline__ void bvec_load(double (&b)[BP / 2], const double *hv) {
  constexpr int PL = VecLds<BP>::PL;
  const int l = lane_id();
  const int kl = l >> 4, n = l & 15, col = n & 7;
  const double *h0 = (n < 8) ? hv : hv + PL;  // k < BP
  const double *h1 = (n < 8) ? hv + PL : hv;  // k >= BP
  const double s1 = (n < 8) ? -1.0 : 1.0;
#pragma unroll
  for (int ks = 0; ks < BP / 4; ++ks) {
    b[ks] = h0[(4 * ks + kl) * kTile + col];
    b[BP / 4 + ks] = s1 * h1[(4 * ks + kl) * kTile + col];
  }
}

template <int BP>
__device__ __forceinline__ d4 frag_mfma(const d4 &acc0, const Frag<BP> &f,
                                        const double (&b)[BP / 2]) {
  d4 a0 = acc0, a1 = d4zero(), a2 = d4zero(), a3 = d4zero();
#pragma unroll
  for (int ks = 0; ks < BP / 2; ks += 4) {
    a0 = mfma(f.v[ks], b[ks], a0);
    a1 = mfma(f.v[ks + 1], b[ks + 1], a1);
    a2 = mfma(f.v[ks + 2], b[ks + 2], a2);
    a3 = mfma(f.v[ks + 3], b[ks + 3], a3);
  }
  return (a0 + a1) + (a2 + a3);
}

// Accumulator tile <-> vector tile [2][BP][8]: plain accesses (LDS or
// global) and buffer accesses that become no-ops when valid is false.
template <int BP>
__device__ __forceinline__ int vec_off(int rb, int r) {
  const int l = lane_id();
  const int n = l & 15, plane = n >> 3, col = n & 7;
  return (plane * BP + rb * 16 + acc_row(l, r)) * kTile + col;
}

template <int BP>
__device__ __forceinline__ void acc_store_vec(double *dst, const d4 &acc, int rb) {
#pragma unroll
  for (int r = 0; r < 4; ++r) dst[vec_off<BP>(rb, r)] = acc[r];
}

template <int BP>
__device__ __forceinline__ d4 acc_load_vec(const double *src, int rb) {
  d4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) a[r] = src[vec_off<BP>(rb, r)];
  return a;
}

// Accumulator tile <-> LDS vector tile (padded plane stride).
template <int BP>
__device__ __forceinline__ int lds_off(int rb, int r) {
  const int l = lane_id();
  const int n = l & 15;
  return (n >> 3) * VecLds<BP>::PL + (rb * 16 + acc_row(l, r)) * kTile + (n & 7);
}

template <int BP>
__device__ __forceinline__ void lds_store_vec(double *dst, const d4 &acc, int rb) {
#pragma unroll
  for (int r = 0; r < 4; ++r) dst[lds_off<BP>(rb, r)] = acc[r];
}

template <int BP>
__device__ __forceinline__ d4 lds_load_vec(const double *src, int rb) {
  d4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) a[r] = src[lds_off<BP>(rb, r)];
  return a;
}

template <int BP>
__device__ __forceinline__ void vec_store_buf(double *dst, const d4 &acc, int rb, bool valid) {
  const auto rs = buf_rsrc(dst, valid ? 2 * BP * kTile * 8 : 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) buf_store(acc[r], rs, vec_off<BP>(rb, r) * 8, 0);
}

template <int BP>
__device__ __forceinline__ d4 vec_load_buf(const double *src, int rb, bool valid) {
  const auto rs = buf_rsrc(src, valid ? 2 * BP * kTile * 8 : 0);
  d4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) a[r] = buf_load(rs, vec_off<BP>(rb, r) * 8, 0);
  return a;
}

// Accumulator <- real right-hand side tile of one cell (rows of length m0p,
// 8 columns from R; imaginary part 0).
template <int BP>
__device__ __forceinline__ d4 rhs_load(const double *R, int m0p, int rb, bool valid) {
  const int l = lane_id();
  const int n = l & 15;
  const auto rs = buf_rsrc(R, valid ? BP * m0p * 8 : 0);
  d4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = rb * 16 + acc_row(l, r);
    a[r] = buf_load(rs, n < 8 ? (row * m0p + n) * 8 : kBufferOff, 0);
  }
  return a;
}

struct SweepArgs {
  Pencil p;
  Factors f;
  SolveBufs sb;
  const double *R;   // padded [nc][bp][m0p]
  double *P;         // [Ne][nc][bp][m0p]  (or Xre for the complex variant)
  double *Xim;       // complex variant only
  int m0p, ntiles;
  double kre[kMaxNe], kim[kMaxNe];
  const int *skip;   // non-zero: a converged solve, the kernels do nothing
};

// Forward sweep.  The workgroup has two wave sets of BP/16 waves each: the
// first computes the critical-path product h_{j+1} = R_{j+1} - W_j^T h_j,
// the second g_j = Sinv_j h_j, so that every SIMD holds two waves and one
// hides the other's latencies.  LDS keeps u_j = -h_j (the sign then folds
// into the accumulator initialisation instead of every matrix operand).
// Every step issues the same memory operations on every wave (inactive ones
// through empty buffer resources), so the waits for the operands loaded a
// step ahead never cover the loads just issued.
template <int BP>
__global__ __launch_bounds__(BP * 8) void forward_kernel(SweepArgs a) {
  if (a.skip && *a.skip) return;
  __shared__ VecLds<BP> s;
  constexpr int NW = BP / 16;
  const int item = xcd_item(blockIdx.x, gridDim.x, a.ntiles);
  const int tau = item % a.ntiles;
  const int grp = item / a.ntiles;
  const int e = grp >> 1;
  const bool top = (grp & 1) == 0;
  const int nc = a.p.nc, m = a.f.m;
  const int len = top ? m : nc - m;
  if (len <= 0) return;
  const int dir = top ? 1 : -1;
  const int start = top ? 0 : nc - 1;
  const size_t blk = 2 * (size_t)BP * BP;
  const size_t vt = 2 * (size_t)BP * kTile;
  const int wv = wave_id();
  const bool wrole = wv < NW;  // wave-uniform
  const int rb = wrole ? wv : wv - NW;
  // the W role carries the recurrence from step to step: its instructions go
  // first when both roles of a SIMD are ready
  if (wrole) __builtin_amdgcn_s_setprio(2);
  const double *M = (wrole ? a.f.W : a.f.Sinv) + (size_t)e * nc * blk;
  double *G = a.sb.G + ((size_t)e * a.ntiles + tau) * nc * vt;
  double *TV = a.sb.TV + ((size_t)e * a.ntiles + tau) * 2 * vt;
  const double *R = a.R + tau * kTile;
  const size_t rstride = (size_t)BP * a.m0p;
  // the top chain's last cell is the twist cell: no product there
  const int nsteps = top ? len - 1 : len;

  if (wrole) {
    const d4 h = rhs_load<BP>(R + start * rstride, a.m0p, rb, true);
    lds_store_vec<BP>(s.v[0], -h, rb);
  }
  // matrix fragments and right-hand side tiles are loaded two steps ahead
  // (three buffers each)
  Frag<BP> f0, f1, f2;
  frag_load<BP>(f0, M + start * blk, rb, nsteps > 0);
  frag_load<BP>(f1, M + (start + dir) * blk, rb, nsteps > 1);
  d4 r0 = rhs_load<BP>(R + (start + dir) * rstride, a.m0p, rb, wrole && len > 1);
  d4 r1 = rhs_load<BP>(R + (start + 2 * dir) * rstride, a.m0p, rb, wrole && len > 2);
  d4 r2 = d4zero();
  __syncthreads();
  int cur = 0;
  // one step on cell c with operands (f, r = R_{c+dir}); loads the
  // fragments of cell c+2dir and R_{c+3dir} for step j+2
  auto step = [&](int j, const Frag<BP> &f, const d4 &r, Frag<BP> &nf2, d4 &nr2) {
    const int c = start + dir * j;
    frag_load<BP>(nf2, M + (c + 2 * dir) * blk, rb, j + 2 < nsteps);
    nr2 = rhs_load<BP>(R + (c + 3 * dir) * rstride, a.m0p, rb, wrole && j + 3 < len);
    double b[BP / 2];
    bvec_load<BP>(b, s.v[cur]);
    const bool more = j < len - 1;
    // W role: R_{j+1} + W_j^T u_j = h_{j+1};  Sinv role: Sinv_j u_j = -g_j
    const d4 acc = frag_mfma<BP>((wrole && more) ? r : d4zero(), f, b);
    vec_store_buf<BP>(G + c * vt, -acc, rb, !wrole);
    if (wrole) {
      if (more)
        lds_store_vec<BP>(s.v[cur ^ 1], -acc, rb);
      else
        acc_store_vec<BP>(TV + vt, acc, rb);  // c = -W~_m^T h~_m
    }
    __syncthreads();
    cur ^= 1;
  };
  // whole rounds of three steps without branches (exact waits), then the rest
  int j = 0;
  for (; j + 3 <= nsteps; j += 3) {
    step(j, f0, r0, f2, r2);
    step(j + 1, f1, r1, f0, r0);
    step(j + 2, f2, r2, f1, r1);
  }
  if (j < nsteps) step(j, f0, r0, f2, r2);
  if (j + 1 < nsteps) step(j + 1, f1, r1, f0, r0);
  if (top && wrole) {
    const d4 u = lds_load_vec<BP>(s.v[cur], rb);
    acc_store_vec<BP>(TV, -u, rb);  // h_{m-1}
  }
}

// Back sweep, one wave per 16-row block.  LDS keeps v = -x of the previous
// cell, so that x_c = g_c + W_c v accumulates onto g_c.
template <int BP, bool COMPLEX_OUT>
__global__ __launch_bounds__(BP * 4) void back_kernel(SweepArgs a) {
  if (a.skip && *a.skip) return;
  __shared__ VecLds<BP> s;
  const int item = xcd_item(blockIdx.x, gridDim.x, a.ntiles);
  const int tau = item % a.ntiles;
  const int grp = item / a.ntiles;
  const int e = grp >> 1;
  const bool top = (grp & 1) == 0;
  const int nc = a.p.nc, m = a.f.m;
  const int len = top ? m : nc - m;
  if (len <= 0) return;
  const size_t blk = 2 * (size_t)BP * BP;
  const size_t vt = 2 * (size_t)BP * kTile;
  const double *Sinv = a.f.Sinv + (size_t)e * nc * blk;
  const double *WT = a.f.WT + (size_t)e * nc * blk;
  const double *G = a.sb.G + ((size_t)e * a.ntiles + tau) * nc * vt;
  const double *TV = a.sb.TV + ((size_t)e * a.ntiles + tau) * 2 * vt;
  const size_t pstride = (size_t)BP * a.m0p;
  double *P = (COMPLEX_OUT ? a.P : a.P + (size_t)e * nc * pstride) + tau * kTile;
  double *Xim = COMPLEX_OUT ? a.Xim + tau * kTile : nullptr;
  const double kr = a.kre[e], ki = a.kim[e];
  const int l = lane_id();
  const int rb = wave_id();
  const int n = l & 15;
  const int pbytes = BP * a.m0p * 8;

  // P_c = Re(kappa_e x_c) (or x_c itself for the complex variant)
  auto emit = [&](int c, const d4 &x) {
    const auto rp = buf_rsrc(P + c * pstride, pbytes);
    const auto ri = buf_rsrc(COMPLEX_OUT ? Xim + c * pstride : nullptr,
                             COMPLEX_OUT ? pbytes : 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double other = __shfl_xor(x[r], 8);
      const int off = ((rb * 16 + acc_row(l, r)) * a.m0p + (n & 7)) * 8;
      if (COMPLEX_OUT) {
        buf_store(x[r], rp, n < 8 ? off : kBufferOff, 0);
        buf_store(x[r], ri, n < 8 ? kBufferOff : off, 0);
      } else {
        buf_store(kr * x[r] - ki * other, rp, n < 8 ? off : kBufferOff, 0);
      }
    }
  };
  const int count = top ? m - 1 : nc - m;
  auto cell = [&](int j) { return top ? (m - 2 - j) : (m + j); };

  // twist cell: x_{m-1} = T (h_{m-1} + c)
  Frag<BP> f0, f1;
  frag_load<BP>(f0, Sinv + (m - 1) * blk, rb, true);
  {
    d4 t = acc_load_vec<BP>(TV, rb);
    if (nc - m > 0) t += acc_load_vec<BP>(TV + vt, rb);
    lds_store_vec<BP>(s.v[1], t, rb);
  }
  frag_load<BP>(f1, WT + cell(0) * blk, rb, count > 0);
  d4 ga = vec_load_buf<BP>(G + cell(0) * vt, rb, count > 0), gb = d4zero();
  __syncthreads();
  {
    double b[BP / 2];
    bvec_load<BP>(b, s.v[1]);
    const d4 x = frag_mfma<BP>(d4zero(), f0, b);
    lds_store_vec<BP>(s.v[0], -x, rb);
    if (top) emit(m - 1, x);
  }
  __syncthreads();
  int cur = 0;
  // x_c = g_c + W_c v with operands (f, g); loads the next cell's W^T
  // fragments and g tile one step ahead
  auto step = [&](int j, const Frag<BP> &f, const d4 &g, Frag<BP> &nf, d4 &ng) {
    const int c = cell(j);
    const bool nx = j + 1 < count;
    frag_load<BP>(nf, WT + cell(j + 1) * blk, rb, nx);
    ng = vec_load_buf<BP>(G + cell(j + 1) * vt, rb, nx);
    double b[BP / 2];
    bvec_load<BP>(b, s.v[cur]);
    const d4 x = frag_mfma<BP>(g, f, b);
    lds_store_vec<BP>(s.v[cur ^ 1], -x, rb);
    emit(c, x);
    __syncthreads();
    cur ^= 1;
  };
  for (int j = 0; j < count; j += 2) {
    step(j, f1, ga, f0, gb);
    if (j + 1 < count) step(j + 1, f0, gb, f1, ga);
  }
}


// ---- blocks of 64 < b <= 96 (BP = 96): one chain per contour point ----
//
// The factorisation of these blocks runs top-down over all cells (no twist,
// see factor.hip), so the sweeps are the plain block forward and back
// substitutions:  h_0 = R_0,  g_c = Sinv_c h_c,  h_{c+1} = R_{c+1} - W_c^T h_c;
// x_last = g_last,  x_c = g_c - W_c x_{c+1}.  A fragment of a 96 x 96 complex
// block takes 96 registers, so one wave per 16-row block computes both
// products of a forward step from fragments of its own (the B operand is
// read from LDS inside the product, not staged in registers), and reloads
// each fragment array as soon as its product has consumed it: the load of
// W_{c+1} overlaps the Sinv_c product and that of Sinv_{c+1} the next W
// product.
constexpr int kWideBP = 96;
constexpr int kWideThreads = kWideBP / 16 * 64;

// acc0 + A' B' for fragments f and the vector tile hv in LDS (the operand
// bvec_load builds, read one k-step at a time).
template <int BP>
__device__ __forceinline__ d4 frag_mfma_lds(const d4 &acc0, const Frag<BP> &f, const double *hv) {
  constexpr int PL = VecLds<BP>::PL;
  const int l = lane_id();
  const int kl = l >> 4, n = l & 15, col = n & 7;
  const double *h0 = (n < 8) ? hv : hv + PL;
  const double *h1 = (n < 8) ? hv + PL : hv;
  const double s1 = (n < 8) ? -1.0 : 1.0;
  d4 a0 = acc0, a1 = d4zero(), a2 = d4zero(), a3 = d4zero();
#pragma unroll
  for (int ks = 0; ks < BP / 4; ks += 2) {
    a0 = mfma(f.v[ks], h0[(4 * ks + kl) * kTile + col], a0);
    a1 = mfma(f.v[ks + 1], h0[(4 * ks + 4 + kl) * kTile + col], a1);
    a2 = mfma(f.v[BP / 4 + ks], s1 * h1[(4 * ks + kl) * kTile + col], a2);
    a3 = mfma(f.v[BP / 4 + ks + 1], s1 * h1[(4 * ks + 4 + kl) * kTile + col], a3);
  }
  return (a0 + a1) + (a2 + a3);
}

__global__ __launch_bounds__(kWideThreads) void forward_wide_kernel(SweepArgs a) {
  if (a.skip && *a.skip) return;
  constexpr int BP = kWideBP;
  __shared__ VecLds<BP> s;
  const int item = xcd_item(blockIdx.x, gridDim.x, a.ntiles);
  const int tau = item % a.ntiles;
  const int e = item / a.ntiles;
  const int nc = a.p.nc;
  const size_t blk = 2 * (size_t)BP * BP;
  const size_t vt = 2 * (size_t)BP * kTile;
  const int rb = wave_id();
  const double *Wm = a.f.W + (size_t)e * nc * blk;
  const double *Sm = a.f.Sinv + (size_t)e * nc * blk;
  double *G = a.sb.G + ((size_t)e * a.ntiles + tau) * nc * vt;
  const double *R = a.R + tau * kTile;
  const size_t rstride = (size_t)BP * a.m0p;

  // LDS keeps u_c = -h_c
  lds_store_vec<BP>(s.v[0], -rhs_load<BP>(R, a.m0p, rb, true), rb);
  Frag<BP> fw, fs;
  frag_load<BP>(fw, Wm, rb, nc > 1);
  frag_load<BP>(fs, Sm, rb, true);
  d4 rn = rhs_load<BP>(R + rstride, a.m0p, rb, nc > 1);
  __syncthreads();
  int cur = 0;
  for (int c = 0; c < nc; ++c) {
    const bool more = c + 1 < nc;
    // h_{c+1} = R_{c+1} + W_c^T u_c (W_{c+1} exists while c + 2 < nc)
    const d4 h = frag_mfma_lds<BP>(more ? rn : d4zero(), fw, s.v[cur]);
    frag_load<BP>(fw, Wm + (c + 1) * blk, rb, c + 2 < nc);
    rn = rhs_load<BP>(R + (c + 2) * rstride, a.m0p, rb, c + 2 < nc);
    if (more) lds_store_vec<BP>(s.v[cur ^ 1], -h, rb);
    // Sinv_c u_c = -g_c
    const d4 g = frag_mfma_lds<BP>(d4zero(), fs, s.v[cur]);
    frag_load<BP>(fs, Sm + (c + 1) * blk, rb, more);
    vec_store_buf<BP>(G + c * vt, -g, rb, true);
    __syncthreads();
    cur ^= 1;
  }
}

// x_c = g_c + W_c v with v = -x_{c+1} in LDS; output as in back_kernel.
// Two fragment arrays: the W^T fragments of the next cell load during the
// current product.
template <bool COMPLEX_OUT>
__global__ __launch_bounds__(kWideThreads) void back_wide_kernel(SweepArgs a) {
  if (a.skip && *a.skip) return;
  constexpr int BP = kWideBP;
  __shared__ VecLds<BP> s;
  const int item = xcd_item(blockIdx.x, gridDim.x, a.ntiles);
  const int tau = item % a.ntiles;
  const int e = item / a.ntiles;
  const int nc = a.p.nc;
  const size_t blk = 2 * (size_t)BP * BP;
  const size_t vt = 2 * (size_t)BP * kTile;
  const double *WT = a.f.WT + (size_t)e * nc * blk;
  const double *G = a.sb.G + ((size_t)e * a.ntiles + tau) * nc * vt;
  const size_t pstride = (size_t)BP * a.m0p;
  double *P = (COMPLEX_OUT ? a.P : a.P + (size_t)e * nc * pstride) + tau * kTile;
  double *Xim = COMPLEX_OUT ? a.Xim + tau * kTile : nullptr;
  const double kr = a.kre[e], ki = a.kim[e];
  const int l = lane_id();
  const int rb = wave_id();
  const int n = l & 15;
  const int pbytes = BP * a.m0p * 8;
  auto emit = [&](int c, const d4 &x) {
    const auto rp = buf_rsrc(P + c * pstride, pbytes);
    const auto ri = buf_rsrc(COMPLEX_OUT ? Xim + c * pstride : nullptr, COMPLEX_OUT ? pbytes : 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double other = __shfl_xor(x[r], 8);
      const int off = ((rb * 16 + acc_row(l, r)) * a.m0p + (n & 7)) * 8;
      if (COMPLEX_OUT) {
        buf_store(x[r], rp, n < 8 ? off : kBufferOff, 0);
        buf_store(x[r], ri, n < 8 ? kBufferOff : off, 0);
      } else {
        buf_store(kr * x[r] - ki * other, rp, n < 8 ? off : kBufferOff, 0);
      }
    }
  };
  // x_last = g_last
  {
    const d4 x = vec_load_buf<BP>(G + (nc - 1) * vt, rb, true);
    lds_store_vec<BP>(s.v[0], -x, rb);
    emit(nc - 1, x);
  }
  Frag<BP> f0, f1;
  frag_load<BP>(f0, WT + (nc - 2) * blk, rb, nc > 1);
  d4 ga = vec_load_buf<BP>(G + (nc - 2) * vt, rb, nc > 1), gb = d4zero();
  __syncthreads();
  int cur = 0;
  auto step = [&](int c, const Frag<BP> &f, const d4 &g, Frag<BP> &nf, d4 &ng) {
    frag_load<BP>(nf, WT + (c - 1) * blk, rb, c >= 1);
    ng = vec_load_buf<BP>(G + (c - 1) * vt, rb, c >= 1);
    const d4 x = frag_mfma_lds<BP>(g, f, s.v[cur]);
    lds_store_vec<BP>(s.v[cur ^ 1], -x, rb);
    emit(c, x);
    __syncthreads();
    cur ^= 1;
  };
  for (int c = nc - 2; c >= 0; c -= 2) {
    step(c, f0, ga, f1, gb);
    if (c - 1 >= 0) step(c - 1, f1, gb, f0, ga);
  }
}

hipError_t launch_wide(SweepArgs &a, int Ne, bool complex_out, int part, hipStream_t st) {
  const int nblocks = Ne * a.ntiles;
  if (part & 1) {
    hipLaunchKernelGGL(forward_wide_kernel, dim3(nblocks), dim3(kWideThreads), 0, st, a);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  if (part & 2) {
    if (complex_out)
      hipLaunchKernelGGL(back_wide_kernel<true>, dim3(nblocks), dim3(kWideThreads), 0, st, a);
    else
      hipLaunchKernelGGL(back_wide_kernel<false>, dim3(nblocks), dim3(kWideThreads), 0, st, a);
  }
  return hipGetLastError();
}

// Spike solves of the partitioned factorisation.  For a chain with local
// matrix T (factored by its own top-down recurrence: Sinv_j, W_j) and
// E_1 = first block column of the identity, y = T^{-1} E_1 follows from
//   h_0 = I,  h_{j+1} = -W_j^T h_j,  g_j = Sinv_j h_j,
//   y_last = g_last,  y_j = g_j - W_j y_{j+1};
// the kernel keeps y_first = [T^-1]_{first,first} and
// y_last = [T^-1]_{last,first}.  One workgroup per chain computes all BP
// columns, so every factor block it streams feeds BP/8 column tiles.  In the
// forward part the first BP/16 waves form h_{j+1} (one 16-row block each) and
// the other BP/16 waves g_j; in the back part every wave owns one row block
// and half of the column tiles.
struct SpikeArgs {
  Pencil p;
  Factors f;
  const Chain *chains;
  int parts, gtiles;
  double *G, *G11, *GL1;
};

// A complex BP x BP block in LDS: row k holds, per 8-column tile, the 8 real
// parts then the 8 imaginary parts, and rows are 2 BP + 16 doubles apart, so
// that the 64 lanes reading one k-step of the MFMA vector operand (four rows,
// both planes, eight columns) fall on distinct banks.
template <int BP>
struct SpikeLds {
  static constexpr int RS = 2 * BP + 16;
  double h[2][BP * RS];  // [buffer]
  __device__ static int at(int k, int col, int plane) {
    return k * RS + (col >> 3) * 16 + plane * 8 + (col & 7);
  }
};

// B' operand of column tile tau of the LDS block hv at k-step ks for this lane.
template <int BP>
__device__ __forceinline__ double spike_b(const double *hv, int tau, int ks) {
  const int l = lane_id();
  const int kl = l >> 4, n = l & 15, col = tau * kTile + (n & 7);
  const int k = 4 * (ks % (BP / 4)) + kl;
  if (ks < BP / 4) return hv[SpikeLds<BP>::at(k, col, n >> 3)];
  const double v = hv[SpikeLds<BP>::at(k, col, 1 - (n >> 3))];
  return n < 8 ? -v : v;
}

// Accumulator of output row block rb, column tile tau <-> LDS block.
template <int BP>
__device__ __forceinline__ void spike_store_lds(double *hv, const d4 &acc, int rb, int tau) {
  const int l = lane_id();
  const int n = l & 15, plane = n >> 3, col = tau * kTile + (n & 7);
#pragma unroll
  for (int r = 0; r < 4; ++r) hv[SpikeLds<BP>::at(rb * 16 + acc_row(l, r), col, plane)] = acc[r];
}

template <int BP>
__device__ __forceinline__ void acc_store_block_cols(double *dst, const d4 &acc, int rb, int tau) {
  const int l = lane_id();
  const int n = l & 15, plane = n >> 3, col = n & 7;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = rb * 16 + acc_row(l, r);
    dst[(size_t)plane * BP * BP + row * BP + tau * kTile + col] = acc[r];
  }
}

template <int BP>
__global__ __launch_bounds__(BP * 8) void spike_kernel(SpikeArgs a) {
  extern __shared__ double spike_smem[];
  SpikeLds<BP> &s = *reinterpret_cast<SpikeLds<BP> *>(spike_smem);
  constexpr int NW = BP / 16, NT = BP / kTile;
  const Chain ch = a.chains[blockIdx.x];
  const int e = ch.e, start = ch.start, dir = ch.dir, len = ch.len;
  if (len <= 0) return;
  const int nc = a.p.nc;
  const size_t blk = 2 * (size_t)BP * BP;
  const size_t vt = 2 * (size_t)BP * kTile;
  const double *Sinv = a.f.Sinv + (size_t)e * nc * blk;
  const double *W = a.f.W + (size_t)e * nc * blk;
  const double *WT = a.f.WT + (size_t)e * nc * blk;
  // G tile tau of cell c: G + (tau * nc + c) * vt
  double *G = a.G + (size_t)e * a.gtiles * nc * vt;
  const size_t out = ((size_t)(e * 2 + ch.half) * a.parts + ch.part) * blk;
  const int tid = threadIdx.x, wv = wave_id();
  const bool wrole = wv < NW;  // wave-uniform
  const int rb = wrole ? wv : wv - NW;

  // h_0 = E_1: the identity block
  for (int idx = tid; idx < BP * BP; idx += BP * 8) {
    const int r = idx / BP, c = idx % BP;
    s.h[0][SpikeLds<BP>::at(r, c, 0)] = r == c ? 1.0 : 0.0;
    s.h[0][SpikeLds<BP>::at(r, c, 1)] = 0.0;
  }
  __syncthreads();
  // ---- forward: h_{j+1} = -W_j^T h_j (first wave set), g_j = Sinv_j h_j ----
  // The column tiles are done in two halves (fewer live accumulators); the
  // matrix fragments of the next cell are loaded a step ahead.
  constexpr int NH = NT / 2;  // tiles per half (NT is even)
  const double *M = wrole ? W : Sinv;
  Frag<BP> f0, f1;
  frag_load<BP>(f0, M + start * blk, rb, !(wrole && len == 1));
  int cur = 0;
  auto fstep = [&](int j, const Frag<BP> &f, Frag<BP> &nf) {
    const int c = start + dir * j;
    const bool last = j == len - 1;
    frag_load<BP>(nf, M + (c + dir) * blk, rb, j + 1 < len && !(wrole && j + 1 == len - 1));
    if (!(wrole && last)) {
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        d4 acc[NH];
#pragma unroll
        for (int q = 0; q < NH; ++q) acc[q] = d4zero();
#pragma unroll
        for (int ks = 0; ks < BP / 2; ++ks) {
#pragma unroll
          for (int q = 0; q < NH; ++q)
            acc[q] = mfma(f.v[ks], spike_b<BP>(s.h[cur], hf * NH + q, ks), acc[q]);
          // keep the vector-operand reads of later k-steps from being
          // hoisted all at once (register pressure)
          if ((ks & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int q = 0; q < NH; ++q) {
          const int t = hf * NH + q;
          if (wrole) {
            spike_store_lds<BP>(s.h[cur ^ 1], -acc[q], rb, t);
          } else {
            vec_store_buf<BP>(G + (t * nc + c) * vt, acc[q], rb, true);
            if (last) acc_store_block_cols<BP>(a.GL1 + out, acc[q], rb, t);
          }
        }
      }
    }
    __syncthreads();
    cur ^= 1;
  };
  for (int j = 0; j < len; j += 2) {
    fstep(j, f0, f1);
    if (j + 1 < len) fstep(j + 1, f1, f0);
  }
  // ---- back: LDS keeps v = -y of the previous cell, y_j = g_j + W_j v ----
  // Every wave owns one row block and NT/2 column tiles.  g_j is loaded at
  // the start of the step and added at its end; the W^T fragments of the
  // next cell are loaded a step ahead.
  const int rb2 = wv % NW, t0 = (wv / NW) * NH;
  {
    // -y_last = -g_last into the LDS buffer the loop reads first
    const int c = start + dir * (len - 1);
#pragma unroll
    for (int q = 0; q < NH; ++q) {
      const d4 g = vec_load_buf<BP>(G + ((t0 + q) * nc + c) * vt, rb2, true);
      spike_store_lds<BP>(s.h[0], -g, rb2, t0 + q);
    }
  }
  frag_load<BP>(f0, WT + (start + dir * (len - 2)) * blk, rb2, len >= 2);
  __syncthreads();
  cur = 0;
  auto bstep = [&](int j, const Frag<BP> &f, Frag<BP> &nf) {
    const int c = start + dir * j;
    frag_load<BP>(nf, WT + (c - dir) * blk, rb2, j >= 1);
    d4 g[NH], acc[NH];
#pragma unroll
    for (int q = 0; q < NH; ++q) {
      g[q] = vec_load_buf<BP>(G + ((t0 + q) * nc + c) * vt, rb2, true);
      acc[q] = d4zero();
    }
#pragma unroll
    for (int ks = 0; ks < BP / 2; ++ks) {
#pragma unroll
      for (int q = 0; q < NH; ++q) acc[q] = mfma(f.v[ks], spike_b<BP>(s.h[cur], t0 + q, ks), acc[q]);
      if ((ks & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int q = 0; q < NH; ++q) spike_store_lds<BP>(s.h[cur ^ 1], -(g[q] + acc[q]), rb2, t0 + q);
    __syncthreads();
    cur ^= 1;
  };
  for (int j = len - 2; j >= 0; j -= 2) {
    bstep(j, f0, f1);
    if (j - 1 >= 0) bstep(j - 1, f1, f0);
  }
  // y_first: -v in the current buffer
#pragma unroll
  for (int q = 0; q < NH; ++q) {
    const int t = t0 + q;
    const int l = lane_id();
    const int n = l & 15, plane = n >> 3, col = t * kTile + (n & 7);
    d4 y;
#pragma unroll
    for (int r = 0; r < 4; ++r) y[r] = -s.h[cur][SpikeLds<BP>::at(rb2 * 16 + acc_row(l, r), col, plane)];
    acc_store_block_cols<BP>(a.G11 + out, y, rb2, t);
  }
}

// part: 1 = forward sweep, 2 = back sweep, 3 = both
template <int BP>
hipError_t launch_sweeps_bp(SweepArgs &a, int Ne, bool complex_out, int part, hipStream_t st) {
  const int nblocks = Ne * 2 * a.ntiles;
  if (part & 1) {
    hipLaunchKernelGGL(forward_kernel<BP>, dim3(nblocks), dim3(BP * 8), 0, st, a);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  if (part & 2) {
    if (complex_out)
      hipLaunchKernelGGL((back_kernel<BP, true>), dim3(nblocks), dim3(BP * 4), 0, st, a);
    else
      hipLaunchKernelGGL((back_kernel<BP, false>), dim3(nblocks), dim3(BP * 4), 0, st, a);
  }
  return hipGetLastError();
}

template <int BP>
hipError_t launch_spike_bp(SpikeArgs &a, dim3 grid, hipStream_t st) {
  const int shm = (int)sizeof(SpikeLds<BP>);
  hipError_t err = hipFuncSetAttribute((const void *)spike_kernel<BP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, shm);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(spike_kernel<BP>, grid, dim3(BP * 8), shm, st, a);
  return hipGetLastError();
}

// ---- Hermitian A: both solves of eq. 12 on the matrix cores (b <= 64) ----
//
// The twisted factors of the non-symmetric M = Z B - A (hfactor_part_kernel)
// are complex blocks Sinv_c, W_c, V_c in the 4 x 4 tiled layout of
// kernels.h (the twist cell's T in Sinv_{m-1}).  Solve 0 is M x = R (forward h_next = R_next - V_c h_c,
// g_c = Sinv_c h_c; back x_c = g_c - W_c x_prev), solve 1 is M^H y = R with
// the same blocks conjugate-transposed (W_c^H, Sinv_c^H forward, V_c^H back):
// the top half runs from cell 0 and the bottom half from cell nc-1 towards
// the twist cell.
// The products are the real sweeps' single real product over a doubled inner
// dimension; the matrix operand op(M)[row][k] is M[row][k] or conj(M[k][row]),
// one complex element (sixteen bytes) a lane and k-step, zero outside b x b.
struct HSweepArgs {
  HPencil p;
  const double *Sinv, *W, *V;  // [Ne][nc] tiled blocks (kernels.h), complex
  const double *R;             // [N][m] complex
  double *G;                   // [Ne][2][N][m] complex: g, then the solutions;
                               // then the twist slots [Ne][2][ntiles][2][2][BP][8]
  int m, ntiles, Ne;
};

// Fragments of M[row][k] (adj: M[k][row]; the conjugate comes from the
// vector operand's sign2 = -1) from a block in the 4 x 4 tiled layout of the
// factors (tiled) or a plain [b][b] block of the pencil.  Rows at or beyond
// b load zeros; columns k >= b meet zero rows of the vector operand, so they
// may hold any finite value (padding, the next row's or block's entries, or
// zeros past the buffer).
template <int BP>
__device__ __forceinline__ void hfrag_load(Frag<BP> &f, const double *M, int b, int rb, bool adj,
                                           bool valid, bool tiled = true) {
  const int l = lane_id();
  const int row = rb * 16 + (l & 15), kl = l >> 4;
  const int bt = htile_dim(b) / 4;  // tiles a block row
  const int bytes = tiled ? (int)hfactor_block_elems(b) * 16 : 2 * b * b * 8;
  const auto rs = buf_rsrc(M, valid ? bytes : 0);
  // k-step ks: tiled, tile column ks (M) or tile row ks (M^H) of the row's
  // tiles; plain, four columns (M) or four rows (M^H) further
  int vo, kstride;
  if (tiled) {
    vo = adj ? (row >> 2) * 16 + kl * 4 + (row & 3) : (row >> 2) * bt * 16 + (row & 3) * 4 + kl;
    kstride = adj ? 256 * bt : 256;
  } else {
    vo = adj ? kl * b + row : row * b + kl;
    kstride = adj ? 64 * b : 64;
  }
  vo = row < b ? vo * 16 : kBufferOff;
#pragma unroll
  for (int ks = 0; ks < BP / 4; ++ks) {
    const auto x = __builtin_amdgcn_raw_buffer_load_b128(rs, vo, ks * kstride, 0);
    f.v[ks] = __builtin_bit_cast(double, (u32x2){x[0], x[1]});
    f.v[BP / 4 + ks] = __builtin_bit_cast(double, (u32x2){x[2], x[3]});
  }
}

// bvec_load with the second half (k >= BP) times sign2: sign2 = -1 makes
// the product use -Mi in place of Mi, the conjugate of the matrix operand.
template <int BP>
__device__ __forceinline__ void hbvec_load(double (&b)[BP / 2], const double *hv, double sign2) {
  constexpr int PL = VecLds<BP>::PL;
  const int l = lane_id();
  const int kl = l >> 4, n = l & 15, col = n & 7;
  const double *h0 = (n < 8) ? hv : hv + PL;  // k < BP
  const double *h1 = (n < 8) ? hv + PL : hv;  // k >= BP
  const double s1 = ((n < 8) ? -1.0 : 1.0) * sign2;
#pragma unroll
  for (int ks = 0; ks < BP / 4; ++ks) {
    b[ks] = h0[(4 * ks + kl) * kTile + col];
    b[BP / 4 + ks] = s1 * h1[(4 * ks + kl) * kTile + col];
  }
}

// Accumulator tile (rows of row block rb of cell c, the 8 columns of tile
// tau as [re | im]) <-> complex interleaved [N][m].
template <int BP>
__device__ __forceinline__ int hvec_off(int b, int m, int c, int rb, int r, int tau, bool &in) {
  const int l = lane_id();
  const int n = l & 15, row = rb * 16 + acc_row(l, r), col = tau * kTile + (n & 7);
  in = row < b && col < m;
  return (((c * b + row) * m + col) * 2 + (n >> 3)) * 8;
}

template <int BP>
__device__ __forceinline__ d4 hvec_load(const double *X, int nbytes, int b, int m, int c, int rb,
                                        int tau, bool valid) {
  const auto rs = buf_rsrc(X, valid ? nbytes : 0);
  d4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    bool in;
    const int off = hvec_off<BP>(b, m, c, rb, r, tau, in);
    a[r] = buf_load(rs, in ? off : kBufferOff, 0);
  }
  return a;
}

template <int BP>
__device__ __forceinline__ void hvec_store(double *X, int nbytes, int b, int m, int c, int rb,
                                           int tau, const d4 &a) {
  const auto rs = buf_rsrc(X, nbytes);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    bool in;
    const int off = hvec_off<BP>(b, m, c, rb, r, tau, in);
    buf_store(a[r], rs, in ? off : kBufferOff, 0);
  }
}

// Twisted sweeps of one (node, solve, half, tile) over the twisted factors
// of hfactor_part_kernel (top chain cells 0..m-1, bottom chain nc-1..m, the
// twist cell m-1 holding T).  Forward: the first wave set carries
// h_next = R_next - op(F_c) h_c (F = V, or W for the adjoint; the bottom
// chain's last cell leaves the twist term -op(F_m) h_m instead), the second
// computes g_c = op(Sinv_c) h_c into G; LDS keeps u_c = -h_c.  The top chain
// ends with h_{m-1}.  Both go to the tile's two slots TV[0], TV[1] at the end
// of G.
template <int BP>
__global__ __launch_bounds__(BP * 8) void hforward_kernel(HSweepArgs a) {
  __shared__ VecLds<BP> s;
  constexpr int NW = BP / 16;
  const int item = xcd_item(blockIdx.x, gridDim.x, a.ntiles);  // the tiles of a group on one XCD
  const int tau = item % a.ntiles;
  const int grp = item / a.ntiles;  // (node * 2 + solve) * 2 + half
  const int e = grp >> 2;
  const bool adj = (grp & 2) != 0, top = (grp & 1) == 0;
  const int nc = a.p.nc, b = a.p.b, m = a.m, mt = nc - nc / 2;
  const int len = top ? mt : nc - mt;
  if (len <= 0) return;
  const int start = top ? 0 : nc - 1, dir = top ? 1 : -1;
  const int nsteps = top ? len - 1 : len;  // no product at the twist cell
  const size_t bb = hfactor_block_elems(b);  // factor block (tiled)
  const size_t vt = 2 * (size_t)BP * kTile;
  const int wv = wave_id();
  const bool wrole = wv < NW;  // wave-uniform
  const int rb = wrole ? wv : wv - NW;
  if (wrole) __builtin_amdgcn_s_setprio(2);
  const double *Mat = (wrole ? (adj ? a.W : a.V) : a.Sinv) + 2 * (size_t)e * nc * bb;
  const int nbytes = nc * b * m * 16;
  const size_t slab = 2 * (size_t)nc * b * m;
  double *G = a.G + ((size_t)e * 2 + (adj ? 1 : 0)) * slab;
  double *TV = a.G + (size_t)a.Ne * 2 * slab +
               (((size_t)e * 2 + (adj ? 1 : 0)) * a.ntiles + tau) * 2 * vt;
  if (wrole) {
    const d4 h = hvec_load<BP>(a.R, nbytes, b, m, start, rb, tau, true);
    lds_store_vec<BP>(s.v[0], -h, rb);
  }
  // fragments and right-hand side tiles one step ahead (two buffers each)
  Frag<BP> f0, f1;
  hfrag_load<BP>(f0, Mat + 2 * (size_t)start * bb, b, rb, adj, nsteps > 0);
  d4 r0 = hvec_load<BP>(a.R, nbytes, b, m, start + dir, rb, tau, wrole && len > 1);
  d4 r1 = d4zero();
  __syncthreads();
  int cur = 0;
  // step j on cell c with operands (f = op(Mat_c), r = R_{c+dir}); loads the
  // fragments of cell c+dir and R_{c+2dir}
  auto step = [&](int j, const Frag<BP> &f, const d4 &r, Frag<BP> &nf, d4 &nr) {
    const int c = start + dir * j;
    hfrag_load<BP>(nf, Mat + 2 * (size_t)(c + dir) * bb, b, rb, adj, j + 1 < nsteps);
    nr = hvec_load<BP>(a.R, nbytes, b, m, c + 2 * dir, rb, tau, wrole && j + 2 < len);
    double bv[BP / 2];
    hbvec_load<BP>(bv, s.v[cur], adj ? -1.0 : 1.0);
    const bool more = j < len - 1;
    // coupling role: R_{c+dir} + op(F_c) u_c = h_{c+dir};  Sinv role: op(Sinv_c) u_c = -g_c
    const d4 acc = frag_mfma<BP>((wrole && more) ? r : d4zero(), f, bv);
    if (wrole) {
      if (more)
        lds_store_vec<BP>(s.v[cur ^ 1], -acc, rb);
      else
        acc_store_vec<BP>(TV + vt, acc, rb);  // -op(F_m) h_m (bottom chain)
    } else {
      hvec_store<BP>(G, nbytes, b, m, c, rb, tau, -acc);
    }
    __syncthreads();
    cur ^= 1;
  };
  for (int j = 0; j < nsteps; j += 2) {
    step(j, f0, r0, f1, r1);
    if (j + 1 < nsteps) step(j + 1, f1, r1, f0, r0);
  }
  if (top && wrole) {
    const d4 u = lds_load_vec<BP>(s.v[cur], rb);
    acc_store_vec<BP>(TV, -u, rb);  // h_{m-1}
  }
}

// Back sweep of one (node, solve, half, tile): the twist cell
// x_{m-1} = op(T) (h_{m-1} - op(F_m) h_m) (written by the top half), then
// x_c = g_c - op(B_c) x_prev outwards (B = W, or V for the adjoint),
// overwriting g in G; LDS keeps v = -x.
template <int BP>
__global__ __launch_bounds__(BP * 4) void hback_kernel(HSweepArgs a) {
  __shared__ VecLds<BP> s;
  const int item = xcd_item(blockIdx.x, gridDim.x, a.ntiles);
  const int tau = item % a.ntiles;
  const int grp = item / a.ntiles;
  const int e = grp >> 2;
  const bool adj = (grp & 2) != 0, top = (grp & 1) == 0;
  const int nc = a.p.nc, b = a.p.b, m = a.m, mt = nc - nc / 2;
  const size_t bb = hfactor_block_elems(b);  // factor block (tiled)
  const size_t vt = 2 * (size_t)BP * kTile;
  const int rb = wave_id();
  const double *Sm = a.Sinv + 2 * (size_t)e * nc * bb;
  const double *Mat = (adj ? a.V : a.W) + 2 * (size_t)e * nc * bb;
  const int nbytes = nc * b * m * 16;
  const size_t slab = 2 * (size_t)nc * b * m;
  double *G = a.G + ((size_t)e * 2 + (adj ? 1 : 0)) * slab;
  const double *TV = a.G + (size_t)a.Ne * 2 * slab +
                     (((size_t)e * 2 + (adj ? 1 : 0)) * a.ntiles + tau) * 2 * vt;
  const int count = top ? mt - 1 : nc - mt;
  if (!top && count <= 0) return;
  auto cell = [&](int j) { return top ? (mt - 2 - j) : (mt + j); };
  // twist cell
  Frag<BP> f0, f1;
  hfrag_load<BP>(f0, Sm + 2 * (size_t)(mt - 1) * bb, b, rb, adj, true);
  {
    d4 t = acc_load_vec<BP>(TV, rb);
    if (nc - mt > 0) t += acc_load_vec<BP>(TV + vt, rb);
    lds_store_vec<BP>(s.v[1], t, rb);
  }
  hfrag_load<BP>(f1, Mat + 2 * (size_t)cell(0) * bb, b, rb, adj, count > 0);
  d4 ga = hvec_load<BP>(G, nbytes, b, m, cell(0), rb, tau, count > 0), gb = d4zero();
  __syncthreads();
  {
    double bv[BP / 2];
    hbvec_load<BP>(bv, s.v[1], adj ? -1.0 : 1.0);
    const d4 x = frag_mfma<BP>(d4zero(), f0, bv);
    lds_store_vec<BP>(s.v[0], -x, rb);
    if (top) hvec_store<BP>(G, nbytes, b, m, mt - 1, rb, tau, x);
  }
  __syncthreads();
  int cur = 0;
  // x_c = g_c + op(B_c) v with operands (f, g); loads the next cell's
  auto step = [&](int j, const Frag<BP> &f, const d4 &g, Frag<BP> &nf, d4 &ng) {
    const int c = cell(j);
    const bool nx = j + 1 < count;
    hfrag_load<BP>(nf, Mat + 2 * (size_t)(nx ? cell(j + 1) : c) * bb, b, rb, adj, nx);
    ng = hvec_load<BP>(G, nbytes, b, m, nx ? cell(j + 1) : c, rb, tau, nx);
    double bv[BP / 2];
    hbvec_load<BP>(bv, s.v[cur], adj ? -1.0 : 1.0);
    const d4 x = frag_mfma<BP>(g, f, bv);
    lds_store_vec<BP>(s.v[cur ^ 1], -x, rb);
    hvec_store<BP>(G, nbytes, b, m, c, rb, tau, x);
    __syncthreads();
    cur ^= 1;
  };
  for (int j = 0; j < count; j += 2) {
    step(j, f1, ga, f0, gb);
    if (j + 1 < count) step(j + 1, f0, gb, f1, ga);
  }
}

// out = T V for a Hermitian pencil's block-tridiagonal operator T (which 0:
// A complex Hermitian, blocks (c, c+1) = Au[c], (c+1, c) = Au[c]^H; which 1:
// B real symmetric), V and out complex [N][m]; one workgroup per (cell,
// 8-column tile), one wave per row block: the three block products of the
// cell accumulate in one tile, the vector tiles of the cell and its two
// neighbours staged in LDS.
template <int BP>
struct HApplyLds {
  double t[3][2 * VecLds<BP>::PL];
};

// Fragments of a real block (row-wise, or column-wise for the transpose):
// imaginary parts zero.
template <int BP>
__device__ __forceinline__ void rfrag_load(Frag<BP> &f, const double *M, int b, int rb, bool tr) {
  const int l = lane_id();
  const int row = rb * 16 + (l & 15), kl = l >> 4;
  const auto rs = buf_rsrc(M, b * b * 8);
  const int vo = row < b ? (tr ? kl * b + row : row * b + kl) * 8 : kBufferOff;
  const int kstride = tr ? 32 * b : 32;
#pragma unroll
  for (int ks = 0; ks < BP / 4; ++ks) {
    f.v[ks] = buf_load(rs, vo, ks * kstride);
    f.v[BP / 4 + ks] = 0.0;
  }
}

template <int BP>
__global__ __launch_bounds__(BP * 4) void happly_mfma_kernel(HPencil p, int which, const double *V,
                                                             int m, int ntiles, double *out,
                                                             double *out2) {
  __shared__ HApplyLds<BP> s;
  const int c = blockIdx.x / ntiles, tau = blockIdx.x % ntiles;
  const int nc = p.nc, b = p.b, rb = wave_id();
  const size_t bb = (size_t)b * b;
  const int nbytes = nc * b * m * 16;
  // vector tiles of cells c-1, c, c+1 (zero outside the chain)
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int cq = c - 1 + q;
    const d4 v = hvec_load<BP>(V, nbytes, b, m, cq, rb, tau, cq >= 0 && cq < nc);
    lds_store_vec<BP>(s.t[q], v, rb);
  }
  __syncthreads();
  d4 acc = d4zero();
  Frag<BP> f;
  double bv[BP / 2];
  if (which != 1) {  // A V (which 0, or the first output of which 2)
    hfrag_load<BP>(f, p.Ad + 2 * (size_t)c * bb, b, rb, false, true, false);
    hbvec_load<BP>(bv, s.t[1], 1.0);
    acc = frag_mfma<BP>(acc, f, bv);
    if (c + 1 < nc) {
      hfrag_load<BP>(f, p.Au + 2 * (size_t)c * bb, b, rb, false, true, false);
      hbvec_load<BP>(bv, s.t[2], 1.0);
      acc = frag_mfma<BP>(acc, f, bv);
    }
    if (c > 0) {  // Au[c-1]^H: column-wise, conjugate through the vector operand
      hfrag_load<BP>(f, p.Au + 2 * (size_t)(c - 1) * bb, b, rb, true, true, false);
      hbvec_load<BP>(bv, s.t[0], -1.0);
      acc = frag_mfma<BP>(acc, f, bv);
    }
  }
  if (which == 2) {
    hvec_store<BP>(out, nbytes, b, m, c, rb, tau, acc);
    acc = d4zero();
  }
  if (which != 0) {  // B V
    rfrag_load<BP>(f, p.Bd + (size_t)c * bb, b, rb, false);
    hbvec_load<BP>(bv, s.t[1], 1.0);
    acc = frag_mfma<BP>(acc, f, bv);
    if (c + 1 < nc) {
      rfrag_load<BP>(f, p.Bu + (size_t)c * bb, b, rb, false);
      hbvec_load<BP>(bv, s.t[2], 1.0);
      acc = frag_mfma<BP>(acc, f, bv);
    }
    if (c > 0) {
      rfrag_load<BP>(f, p.Bu + (size_t)(c - 1) * bb, b, rb, true);
      hbvec_load<BP>(bv, s.t[0], 1.0);
      acc = frag_mfma<BP>(acc, f, bv);
    }
  }
  hvec_store<BP>(which == 2 ? out2 : out, nbytes, b, m, c, rb, tau, acc);
}

template <int BP>
hipError_t launch_happly_bp(const HPencil &p, int which, const double *V, int m, double *out,
                            double *out2, hipStream_t st) {
  const int ntiles = (m + kTile - 1) / kTile;
  hipLaunchKernelGGL(happly_mfma_kernel<BP>, dim3(p.nc * ntiles), dim3(BP * 4), 0, st, p, which,
                     V, m, ntiles, out, out2);
  return hipGetLastError();
}

template <int BP>
hipError_t launch_hsweeps_bp(HSweepArgs &a, int Ne, hipStream_t st) {
  const int nblocks = Ne * 2 * 2 * a.ntiles;
  hipLaunchKernelGGL(hforward_kernel<BP>, dim3(nblocks), dim3(BP * 8), 0, st, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(hback_kernel<BP>, dim3(nblocks), dim3(BP * 4), 0, st, a);
  return hipGetLastError();
}

hipError_t dispatch(SweepArgs &a, int Ne, bool complex_out, int part, hipStream_t st) {
  switch (a.p.bp) {
    case 16: return launch_sweeps_bp<16>(a, Ne, complex_out, part, st);
    case 32: return launch_sweeps_bp<32>(a, Ne, complex_out, part, st);
    case 48: return launch_sweeps_bp<48>(a, Ne, complex_out, part, st);
    case 64: return launch_sweeps_bp<64>(a, Ne, complex_out, part, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_sweeps(const Pencil &p, const Shifts &s, int Ne, const Factors &f,
                         const SolveBufs &sb, const double *R, int m0p, double *P, int part,
                         hipStream_t st, const int *skip) {
  SweepArgs a;
  a.p = p; a.f = f; a.sb = sb; a.R = R; a.P = P; a.Xim = nullptr; a.skip = skip;
  a.m0p = m0p; a.ntiles = m0p / kTile;
  for (int e = 0; e < kMaxNe; ++e) { a.kre[e] = s.kre[e]; a.kim[e] = s.kim[e]; }
  return dispatch(a, Ne, false, part, st);
}

hipError_t launch_spikes(const Pencil &p, const Factors &f, const Chain *chains, int nchains,
                         int parts, int gtiles, double *G, double *G11, double *GL1,
                         hipStream_t st) {
  if (nchains <= 0) return hipSuccess;
  SpikeArgs a;
  a.p = p; a.f = f; a.chains = chains; a.parts = parts; a.gtiles = gtiles;
  a.G = G; a.G11 = G11; a.GL1 = GL1;
  const dim3 grid(nchains);
  switch (p.bp) {
    case 16: return launch_spike_bp<16>(a, grid, st);
    case 32: return launch_spike_bp<32>(a, grid, st);
    case 48: return launch_spike_bp<48>(a, grid, st);
    case 64: return launch_spike_bp<64>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sweeps_wide(const Pencil &p, const Shifts &s, int Ne, const Factors &f,
                              const SolveBufs &sb, const double *R, int m0p, double *P,
                              double *Xim, int part, hipStream_t st, const int *skip) {
  if (p.bp != kWideBP) return hipErrorInvalidValue;
  SweepArgs a;
  a.p = p; a.f = f; a.sb = sb; a.R = R; a.P = P; a.Xim = Xim; a.skip = skip;
  a.m0p = m0p; a.ntiles = m0p / kTile;
  for (int e = 0; e < kMaxNe; ++e) { a.kre[e] = s.kre[e]; a.kim[e] = s.kim[e]; }
  return launch_wide(a, Ne, Xim != nullptr, part, st);
}

hipError_t launch_happly_mfma(const HPencil &p, int which, const double *V, int m, double *out,
                              hipStream_t st, double *out2) {
  if (p.b < 1 || p.b > 64 || m < 1 || which < 0 || which > 2 || (which == 2 && !out2) ||
      (size_t)p.nc * p.b * m * 16 > 0x7fffffffu)
    return hipErrorInvalidValue;
  switch ((p.b + 15) / 16 * 16) {
    case 16: return launch_happly_bp<16>(p, which, V, m, out, out2, st);
    case 32: return launch_happly_bp<32>(p, which, V, m, out, out2, st);
    case 48: return launch_happly_bp<48>(p, which, V, m, out, out2, st);
    default: return launch_happly_bp<64>(p, which, V, m, out, out2, st);
  }
}

size_t hsweep_work_doubles(const HPencil &p, int Ne, int m) {
  const size_t slabs = (size_t)Ne * 2 * 2 * p.nc * p.b * m;
  const size_t twist = (size_t)Ne * 2 * ((m + kTile - 1) / kTile) * 2 * (2 * 64 * kTile);
  return slabs + twist;
}

hipError_t launch_hsweeps_mfma(const HPencil &p, int Ne, const double *Sinv, const double *W,
                               const double *V, const double *R, int m, double *G,
                               hipStream_t st) {
  // byte offsets of one [N][m] complex slab stay within 32 bits
  if (p.b < 1 || p.b > 64 || m < 1 || Ne < 1 ||
      (size_t)p.nc * p.b * m * 16 > 0x7fffffffu)
    return hipErrorInvalidValue;
  HSweepArgs a;
  a.p = p; a.Sinv = Sinv; a.W = W; a.V = V; a.R = R; a.G = G; a.m = m; a.Ne = Ne;
  a.ntiles = (m + kTile - 1) / kTile;
  switch ((p.b + 15) / 16 * 16) {
    case 16: return launch_hsweeps_bp<16>(a, Ne, st);
    case 32: return launch_hsweeps_bp<32>(a, Ne, st);
    case 48: return launch_hsweeps_bp<48>(a, Ne, st);
    default: return launch_hsweeps_bp<64>(a, Ne, st);
  }
}

hipError_t launch_sweeps_complex(const Pencil &p, const Shifts &s, const Factors &f,
                                 const SolveBufs &sb, const double *R, int m0p,
                                 double *Xre, double *Xim, hipStream_t st) {
  SweepArgs a;
  a.p = p; a.f = f; a.sb = sb; a.R = R; a.P = Xre; a.Xim = Xim; a.skip = nullptr;
  a.m0p = m0p; a.ntiles = m0p / kTile;
  for (int e = 0; e < kMaxNe; ++e) { a.kre[e] = s.kre[e]; a.kim[e] = s.kim[e]; }
  return dispatch(a, 1, true, 3, st);
}

}  // namespace feast
