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

template <int BP>
struct VecLds {
  double v[2][2][BP][kTile];  // [buffer][plane][row][col]
};

// Matrix-operand fragments of one stored block for this lane: the product
// uses the transpose of the stored block, A'[row][k] = M_plane[k][row], so
// each load instruction reads 16 consecutive doubles of four rows.  Loading
// the next cell's fragments one step ahead hides the L2/HBM latency behind
// the current step's matrix-core work.
template <int BP>
struct Frag {
  double v[BP / 2];  // [plane][k-step]: BP/4 k-steps per plane
};

template <int BP>
__device__ __forceinline__ void frag_load(Frag<BP> &f, const double *__restrict__ M) {
  const int l = lane_id(), w = wave_id();
  const int row = w * 16 + (l & 15), kl = l >> 4;
#pragma unroll
  for (int ks = 0; ks < BP / 4; ++ks) {
    f.v[ks] = M[(4 * ks + kl) * BP + row];
    f.v[BP / 4 + ks] = M[BP * BP + (4 * ks + kl) * BP + row];
  }
}

// acc0/acc1 (+)= sign * A' * B', B' = stacked complex vector [[hr|hi];[-hi|hr]]
// from LDS buffer hv; even and odd k-steps go to separate accumulators.
template <int BP>
__device__ __forceinline__ void frag_mfma(d4 &acc0, d4 &acc1, const Frag<BP> &f,
                                          const double (*hv)[BP][kTile], double sign) {
  const int l = lane_id();
  const int kl = l >> 4;
  const int n = l & 15;
  const int col = n & 7;
  const double *h0 = (n < 8) ? &hv[0][0][0] : &hv[1][0][0];  // k < BP
  const double *h1 = (n < 8) ? &hv[1][0][0] : &hv[0][0][0];  // k >= BP
  const double s1 = (n < 8) ? -1.0 : 1.0;
#pragma unroll
  for (int ks = 0; ks < BP / 4; ks += 2) {
    const double b0 = h0[(4 * ks + kl) * kTile + col];
    const double b1 = h0[(4 * ks + 4 + kl) * kTile + col];
    acc0 = mfma(sign * f.v[ks], b0, acc0);
    acc1 = mfma(sign * f.v[ks + 1], b1, acc1);
  }
#pragma unroll
  for (int ks = 0; ks < BP / 4; ks += 2) {
    const double b0 = s1 * h1[(4 * ks + kl) * kTile + col];
    const double b1 = s1 * h1[(4 * ks + 4 + kl) * kTile + col];
    acc0 = mfma(sign * f.v[BP / 4 + ks], b0, acc0);
    acc1 = mfma(sign * f.v[BP / 4 + ks + 1], b1, acc1);
  }
}

// Accumulator tile <-> vector tile [2][BP][8] (global or LDS).
template <int BP>
__device__ __forceinline__ void acc_store_vec(double *dst, const d4 &acc) {
  const int l = lane_id(), w = wave_id();
  const int n = l & 15, plane = n >> 3, col = n & 7;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = w * 16 + acc_row(l, r);
    dst[(plane * BP + row) * kTile + col] = acc[r];
  }
}

template <int BP>
__device__ __forceinline__ d4 acc_load_vec(const double *src) {
  const int l = lane_id(), w = wave_id();
  const int n = l & 15, plane = n >> 3, col = n & 7;
  d4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = w * 16 + acc_row(l, r);
    a[r] = src[(plane * BP + row) * kTile + col];
  }
  return a;
}

// Accumulator <- real right-hand side tile (imaginary part 0).
template <int BP>
__device__ __forceinline__ d4 acc_load_rhs(const double *R, int m0p) {
  const int l = lane_id(), w = wave_id();
  const int n = l & 15;
  d4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = w * 16 + acc_row(l, r);
    a[r] = (n < 8) ? R[(size_t)row * m0p + n] : 0.0;
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
};

template <int BP>
__global__ __launch_bounds__(BP * 4) void forward_kernel(SweepArgs a) {
  __shared__ VecLds<BP> s;
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
  const double *Sinv = a.f.Sinv + (size_t)e * nc * blk;
  const double *W = a.f.W + (size_t)e * nc * blk;
  double *G = a.sb.G + ((size_t)e * a.ntiles + tau) * nc * vt;
  double *TV = a.sb.TV + ((size_t)e * a.ntiles + tau) * 2 * vt;
  const double *R = a.R + tau * kTile;
  const size_t rstride = (size_t)BP * a.m0p;
  // the top chain's last cell is the twist cell: no product there
  const int nsteps = top ? len - 1 : len;

  {
    d4 h = acc_load_rhs<BP>(R + start * rstride, a.m0p);
    acc_store_vec<BP>(&s.v[0][0][0][0], h);
  }
  Frag<BP> fs0, fw0, fs1, fw1;
  if (nsteps > 0) {
    frag_load<BP>(fs0, Sinv + start * blk);
    frag_load<BP>(fw0, W + start * blk);
  }
  __syncthreads();
  int cur = 0;
  // one chain step on cell c with fragments (fs, fw); prefetch cell c+dir
  auto step = [&](int j, const Frag<BP> &fs, const Frag<BP> &fw, Frag<BP> &ns, Frag<BP> &nw) {
    const int c = start + dir * j;
    if (j + 1 < nsteps) {
      frag_load<BP>(ns, Sinv + (c + dir) * blk);
      frag_load<BP>(nw, W + (c + dir) * blk);
    }
    const bool more = (j < len - 1);
    d4 h0 = more ? acc_load_rhs<BP>(R + (c + dir) * rstride, a.m0p) : d4zero();
    d4 h1 = d4zero(), g0 = d4zero(), g1 = d4zero();
    const auto hv = s.v[cur];
    frag_mfma<BP>(h0, h1, fw, hv, -1.0);  // h_{j+1} = R - W^T h_j (critical path)
    frag_mfma<BP>(g0, g1, fs, hv, 1.0);   // g_j = Sinv_j h_j
    if (more)
      acc_store_vec<BP>(&s.v[cur ^ 1][0][0][0], h0 + h1);
    else
      acc_store_vec<BP>(TV + vt, h0 + h1);  // c = -W~_m^T h~_m
    acc_store_vec<BP>(G + c * vt, g0 + g1);
    __syncthreads();
    cur ^= 1;
  };
  for (int j = 0; j < nsteps; j += 2) {
    step(j, fs0, fw0, fs1, fw1);
    if (j + 1 < nsteps) step(j + 1, fs1, fw1, fs0, fw0);
  }
  if (top) {
    d4 h = acc_load_vec<BP>(&s.v[cur][0][0][0]);
    acc_store_vec<BP>(TV, h);  // h_{m-1}
  }
}

template <int BP, bool COMPLEX_OUT>
__global__ __launch_bounds__(BP * 4) void back_kernel(SweepArgs a) {
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
  double *P = COMPLEX_OUT ? a.P : a.P + (size_t)e * nc * pstride;
  const double kr = a.kre[e], ki = a.kim[e];
  const int l = lane_id(), w = wave_id();
  const int n = l & 15;

  auto emit = [&](int c, const d4 &x) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double other = __shfl_xor(x[r], 8);
      const int row = w * 16 + acc_row(l, r);
      const size_t off = (size_t)c * pstride + (size_t)row * a.m0p + tau * kTile + (n & 7);
      if (COMPLEX_OUT) {
        if (n < 8) a.P[off] = x[r];
        else a.Xim[off] = x[r];
      } else if (n < 8) {
        P[off] = kr * x[r] - ki * other;
      }
    }
  };
  const int count = top ? m - 1 : nc - m;
  auto cell = [&](int j) { return top ? (m - 2 - j) : (m + j); };

  // twist cell: x_{m-1} = T (h_{m-1} + c)
  Frag<BP> f0, f1;
  frag_load<BP>(f0, Sinv + (m - 1) * blk);
  {
    d4 t = acc_load_vec<BP>(TV);
    if (nc - m > 0) t += acc_load_vec<BP>(TV + vt);
    acc_store_vec<BP>(&s.v[1][0][0][0], t);
  }
  __syncthreads();
  {
    d4 x0 = d4zero(), x1 = d4zero();
    frag_mfma<BP>(x0, x1, f0, s.v[1], 1.0);
    d4 x = x0 + x1;
    acc_store_vec<BP>(&s.v[0][0][0][0], x);
    if (top) emit(m - 1, x);
  }
  d4 gnext = d4zero();
  if (count > 0) {
    frag_load<BP>(f1, WT + cell(0) * blk);
    gnext = acc_load_vec<BP>(G + cell(0) * vt);
  }
  __syncthreads();
  int cur = 0;
  // x_c = g_c - W_c x_prev; prefetch the next cell's W^T fragments and g tile
  auto step = [&](int j, const Frag<BP> &fw, Frag<BP> &nw) {
    const int c = cell(j);
    d4 x0 = gnext, x1 = d4zero();
    if (j + 1 < count) {
      frag_load<BP>(nw, WT + cell(j + 1) * blk);
      gnext = acc_load_vec<BP>(G + cell(j + 1) * vt);
    }
    frag_mfma<BP>(x0, x1, fw, s.v[cur], -1.0);
    d4 x = x0 + x1;
    acc_store_vec<BP>(&s.v[cur ^ 1][0][0][0], x);
    emit(c, x);
    __syncthreads();
    cur ^= 1;
  };
  for (int j = 0; j < count; j += 2) {
    step(j, f1, f0);
    if (j + 1 < count) step(j + 1, f0, f1);
  }
}


// Spike solves of the partitioned factorisation.  For a chain with local
// matrix T (factored by its own top-down recurrence: Sinv_j, W_j) and
// E_1 = first block column of the identity, y = T^{-1} E_1 follows from
//   h_0 = I,  h_{j+1} = -W_j^T h_j,  g_j = Sinv_j h_j,
//   y_last = g_last,  y_j = g_j - W_j y_{j+1};
// the kernel keeps y_first = [T^-1]_{first,first} and
// y_last = [T^-1]_{last,first}.  One workgroup per (chain, tile of 8 columns).
struct SpikeArgs {
  Pencil p;
  Factors f;
  const Chain *chains;
  int parts, gtiles;
  double *G, *G11, *GL1;
};

template <int BP>
__device__ __forceinline__ void acc_store_block_cols(double *dst, const d4 &acc, int tau) {
  const int l = lane_id(), w = wave_id();
  const int n = l & 15, plane = n >> 3, col = n & 7;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = w * 16 + acc_row(l, r);
    dst[(size_t)plane * BP * BP + row * BP + tau * kTile + col] = acc[r];
  }
}

template <int BP>
__global__ __launch_bounds__(BP * 4) void spike_kernel(SpikeArgs a) {
  __shared__ VecLds<BP> s;
  constexpr int NTILE = BP / kTile;
  const int ci = blockIdx.x / NTILE, tau = blockIdx.x % NTILE;
  const Chain ch = a.chains[ci];
  const int e = ch.e, start = ch.start, dir = ch.dir, len = ch.len;
  if (len <= 0) return;
  const int nc = a.p.nc;
  const size_t blk = 2 * (size_t)BP * BP;
  const size_t vt = 2 * (size_t)BP * kTile;
  const double *Sinv = a.f.Sinv + (size_t)e * nc * blk;
  const double *W = a.f.W + (size_t)e * nc * blk;
  const double *WT = a.f.WT + (size_t)e * nc * blk;
  double *G = a.G + ((size_t)e * a.gtiles + tau) * nc * vt;
  const size_t out = ((size_t)(e * 2 + ch.half) * a.parts + ch.part) * blk;
  const int l = lane_id(), w = wave_id();
  {
    d4 h;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + acc_row(l, r), n = l & 15;
      h[r] = (n < 8 && row == tau * kTile + n) ? 1.0 : 0.0;
    }
    acc_store_vec<BP>(&s.v[0][0][0][0], h);
  }
  __syncthreads();
  int cur = 0;
  Frag<BP> fa, fb;
  d4 g = d4zero();
  for (int j = 0; j < len; ++j) {
    const int c = start + dir * j;
    frag_load<BP>(fa, Sinv + c * blk);
    d4 g0 = d4zero(), g1 = d4zero();
    frag_mfma<BP>(g0, g1, fa, s.v[cur], 1.0);
    g = g0 + g1;
    acc_store_vec<BP>(G + c * vt, g);
    if (j < len - 1) {
      frag_load<BP>(fb, W + c * blk);
      d4 h0 = d4zero(), h1 = d4zero();
      frag_mfma<BP>(h0, h1, fb, s.v[cur], -1.0);
      acc_store_vec<BP>(&s.v[cur ^ 1][0][0][0], h0 + h1);
    }
    __syncthreads();
    cur ^= 1;
  }
  acc_store_block_cols<BP>(a.GL1 + out, g, tau);
  acc_store_vec<BP>(&s.v[0][0][0][0], g);
  __syncthreads();
  cur = 0;
  for (int j = len - 2; j >= 0; --j) {
    const int c = start + dir * j;
    frag_load<BP>(fa, WT + c * blk);
    d4 x0 = acc_load_vec<BP>(G + c * vt), x1 = d4zero();
    frag_mfma<BP>(x0, x1, fa, s.v[cur], -1.0);
    g = x0 + x1;
    acc_store_vec<BP>(&s.v[cur ^ 1][0][0][0], g);
    __syncthreads();
    cur ^= 1;
  }
  acc_store_block_cols<BP>(a.G11 + out, g, tau);
}

// part: 1 = forward sweep, 2 = back sweep, 3 = both
template <int BP>
hipError_t launch_sweeps_bp(SweepArgs &a, int Ne, bool complex_out, int part, hipStream_t st) {
  const int nblocks = Ne * 2 * a.ntiles;
  if (part & 1) {
    hipLaunchKernelGGL(forward_kernel<BP>, dim3(nblocks), dim3(BP * 4), 0, st, a);
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
                         hipStream_t st) {
  SweepArgs a;
  a.p = p; a.f = f; a.sb = sb; a.R = R; a.P = P; a.Xim = nullptr;
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
  const dim3 grid(nchains * (p.bp / kTile));
  switch (p.bp) {
    case 16: hipLaunchKernelGGL(spike_kernel<16>, grid, dim3(64), 0, st, a); break;
    case 32: hipLaunchKernelGGL(spike_kernel<32>, grid, dim3(128), 0, st, a); break;
    case 48: hipLaunchKernelGGL(spike_kernel<48>, grid, dim3(192), 0, st, a); break;
    case 64: hipLaunchKernelGGL(spike_kernel<64>, grid, dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sweeps_complex(const Pencil &p, const Shifts &s, const Factors &f,
                                 const SolveBufs &sb, const double *R, int m0p,
                                 double *Xre, double *Xim, hipStream_t st) {
  SweepArgs a;
  a.p = p; a.f = f; a.sb = sb; a.R = R; a.P = Xre; a.Xim = Xim;
  a.m0p = m0p; a.ntiles = m0p / kTile;
  for (int e = 0; e < kMaxNe; ++e) { a.kre[e] = s.kre[e]; a.kim[e] = s.kim[e]; }
  return dispatch(a, 1, true, 3, st);
}

}  // namespace feast
