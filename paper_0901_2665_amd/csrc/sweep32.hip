// Mixed-precision shifted solves: the forward and back sweeps of the twisted
// block factorisation with the factor blocks rounded to float32 and the
// products on V_MFMA_F32_16X16X4F32, for a complex right-hand side per node.
//
// The caller refines in float64 around them (iterative refinement):
//   x_e = S(R),  then  x_e <- x_e + S(R - (Z_e B - A) x_e)  until the
// float64 residual of every column is small, where S is this float32 solve.
// Each step multiplies the error by about cond(Z_e B - A) u_32, so the
// refined x_e are float64 solutions of the systems of Fig. 2 step 2 as long
// as that product stays well below one.
//
// The sweep recurrences are those of the float64 kernels (see sweep.hip):
//   h_0 = r_0,  h_{j+1} = r_{j+1} - W_j^T h_j,   g_j = Sinv_j h_j,
//   twist x_{m-1} = T (h_{m-1} - W~_m^T h~_m),   x_j = g_j - W_j x_{j+1}.
// Right-hand sides are read in float64 and rounded on load; the back sweep
// writes (or adds to) the float64 iterate.
#include "common.h"
#include "kernels.h"

namespace feast {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f4 f4zero() { return f4{0.f, 0.f, 0.f, 0.f}; }

// V_MFMA_F32_16X16X4F32 takes its operands like the float64 instruction
// (lane l: A[l%16][l/16], B[l/16][l%16]) but keeps accumulator element r of
// lane l at row 4 (l/16) + r, column l%16 (checked on the device).
__device__ __forceinline__ int acc_row32(int l, int r) { return 4 * (l >> 4) + r; }

// Float32 factor layout: position of element (i, j) of one BP x BP plane.
// The product reads the stored block M as A'[r][k] = M[k][r] with
// k = 4 ks + kl; here the k-steps 4q .. 4q+3 of one (kl, r) are adjacent, so
// one 16-byte load per lane fetches four of them.
template <int BP>
__host__ __device__ constexpr int fpos32(int i, int j) {
  return ((((i >> 4) << 2) + (i & 3)) * BP + j) * 4 + ((i >> 2) & 3);
}

__device__ __forceinline__ void buf_store32(float v, __amdgpu_buffer_rsrc_t rs, int voff,
                                            int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, voff, soff, 0);
}

__device__ __forceinline__ float buf_load32(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
}

// Float64 factor plane (fpos order) -> float32 plane (fpos32 order), for
// nplanes consecutive planes.  Threads walk the destination in order.
template <int BP>
__global__ void round_factors_kernel(const double *src, float *dst, size_t nplanes) {
  const size_t total = nplanes * BP * BP;
  for (size_t d = blockIdx.x * (size_t)blockDim.x + threadIdx.x; d < total;
       d += (size_t)gridDim.x * blockDim.x) {
    const size_t pl = d / (BP * BP);
    const int w = (int)(d % (BP * BP));
    const int s = w & 3, t = (w >> 2) / BP, j = (w >> 2) % BP;
    const int i = ((t >> 2) << 4) + (s << 2) + (t & 3);  // inverse of fpos32
    dst[d] = (float)src[pl * BP * BP + fpos<BP>(i, j)];
  }
}

template <int BP>
struct VecLds32 {
  float v[2][2][BP][kTile];  // [buffer][plane][row][col]
};

// Matrix-operand fragments of one stored block for this lane (see Frag in
// sweep.hip): [plane][k-step], BP/4 k-steps a plane.
template <int BP>
struct Frag32 {
  float v[BP / 2];
};

template <int BP>
__device__ __forceinline__ void frag_load32(Frag32<BP> &f, const float *M, int rb, bool valid) {
  const int l = lane_id();
  const int row = rb * 16 + (l & 15), kl = l >> 4;
  const auto rs = buf_rsrc(M, valid ? 2 * BP * BP * 4 : 0);
  const int vo = fpos32<BP>(kl, row) * 4;  // quad q = 0; fpos32(16q + kl, row) adds 16 q BP
  // (the whole 128-bit result is reinterpreted at once: a bit cast of one
  // element of the loaded vector compiles to a reload of element 0)
#pragma unroll
  for (int q = 0; q < BP / 16; ++q) {
    const f4 v0 =
        __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, q * 16 * BP * 4, 0));
    const f4 v1 = __builtin_bit_cast(
        f4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, (BP * BP + q * 16 * BP) * 4, 0));
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      f.v[4 * q + s] = v0[s];
      f.v[BP / 4 + 4 * q + s] = v1[s];
    }
  }
}

// Vector operand B' = [[hr | hi]; [-hi | hr]] of this lane from the LDS tile.
template <int BP>
__device__ __forceinline__ void bvec_load32(float (&b)[BP / 2], const float (*hv)[BP][kTile]) {
  const int l = lane_id();
  const int kl = l >> 4, n = l & 15, col = n & 7;
  const float *h0 = (n < 8) ? &hv[0][0][0] : &hv[1][0][0];  // k < BP
  const float *h1 = (n < 8) ? &hv[1][0][0] : &hv[0][0][0];  // k >= BP
  const float s1 = (n < 8) ? -1.f : 1.f;
#pragma unroll
  for (int ks = 0; ks < BP / 4; ++ks) {
    b[ks] = h0[(4 * ks + kl) * kTile + col];
    b[BP / 4 + ks] = s1 * h1[(4 * ks + kl) * kTile + col];
  }
}

// acc0 + A' * B' over four independent accumulator chains
template <int BP>
__device__ __forceinline__ f4 frag_mfma32(const f4 &acc0, const Frag32<BP> &f,
                                          const float (&b)[BP / 2]) {
  f4 a0 = acc0, a1 = f4zero(), a2 = f4zero(), a3 = f4zero();
#pragma unroll
  for (int ks = 0; ks < BP / 2; ks += 4) {
    a0 = mfma32(f.v[ks], b[ks], a0);
    a1 = mfma32(f.v[ks + 1], b[ks + 1], a1);
    a2 = mfma32(f.v[ks + 2], b[ks + 2], a2);
    a3 = mfma32(f.v[ks + 3], b[ks + 3], a3);
  }
  return (a0 + a1) + (a2 + a3);
}

template <int BP>
__device__ __forceinline__ int vec_off32(int rb, int r) {
  const int l = lane_id();
  const int n = l & 15, plane = n >> 3, col = n & 7;
  return (plane * BP + rb * 16 + acc_row32(l, r)) * kTile + col;
}

template <int BP>
__device__ __forceinline__ void acc_store_vec32(float *dst, const f4 &acc, int rb) {
#pragma unroll
  for (int r = 0; r < 4; ++r) dst[vec_off32<BP>(rb, r)] = acc[r];
}

template <int BP>
__device__ __forceinline__ f4 acc_load_vec32(const float *src, int rb) {
  f4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) a[r] = src[vec_off32<BP>(rb, r)];
  return a;
}

template <int BP>
__device__ __forceinline__ void vec_store_buf32(float *dst, const f4 &acc, int rb, bool valid) {
  const auto rs = buf_rsrc(dst, valid ? 2 * BP * kTile * 4 : 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) buf_store32(acc[r], rs, vec_off32<BP>(rb, r) * 4, 0);
}

template <int BP>
__device__ __forceinline__ f4 vec_load_buf32(const float *src, int rb, bool valid) {
  const auto rs = buf_rsrc(src, valid ? 2 * BP * kTile * 4 : 0);
  f4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) a[r] = buf_load32(rs, vec_off32<BP>(rb, r) * 4, 0);
  return a;
}

struct Sweep32Args {
  int nc, m, m0p, ntiles;
  Factors32 f;
  SolveBufs32 sb;
  const double *R;  // node e: R + e * rnode (real plane), imaginary plane at + plane
  size_t rnode;
  int rcomplex;     // 0: no imaginary plane (real right-hand side)
  size_t plane;     // rows * m0p
  double *X;        // node e: X + 2 e plane (real plane), then the imaginary plane
};

// Float32 accumulator <- right-hand side tile of one cell (8 complex columns;
// lanes 0-7 of each row group read the real plane, lanes 8-15 the imaginary
// one).  Both loads are issued on every lane, one of them through an offset
// beyond its resource, so every path issues the same memory operations.
template <int BP>
__device__ __forceinline__ f4 rhs_load32(const double *Rre, const double *Rim, int m0p,
                                         bool cplx, int rb, bool valid) {
  const int l = lane_id();
  const int n = l & 15;
  const int bytes = BP * m0p * 8;
  const auto rr = buf_rsrc(Rre, valid ? bytes : 0);
  const auto ri = buf_rsrc(Rim, (valid && cplx) ? bytes : 0);
  f4 a;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int off = ((rb * 16 + acc_row32(l, r)) * m0p + (n & 7)) * 8;
    const double re = buf_load(rr, n < 8 ? off : kBufferOff, 0);
    const double im = buf_load(ri, n < 8 ? kBufferOff : off, 0);
    a[r] = (float)(re + im);
  }
  return a;
}

// Forward sweep (same wave roles and prefetch depth as the float64 kernel).
template <int BP>
__global__ __launch_bounds__(BP * 8) void forward32_kernel(Sweep32Args a) {
  __shared__ VecLds32<BP> s;
  constexpr int NW = BP / 16;
  const int item = xcd_item(blockIdx.x, gridDim.x, a.ntiles);
  const int tau = item % a.ntiles;
  const int grp = item / a.ntiles;
  const int e = grp >> 1;
  const bool top = (grp & 1) == 0;
  const int nc = a.nc, m = a.m;
  const int len = top ? m : nc - m;
  if (len <= 0) return;
  const int dir = top ? 1 : -1;
  const int start = top ? 0 : nc - 1;
  const size_t blk = 2 * (size_t)BP * BP;
  const size_t vt = 2 * (size_t)BP * kTile;
  const int wv = wave_id();
  const bool wrole = wv < NW;  // wave-uniform
  const int rb = wrole ? wv : wv - NW;
  if (wrole) __builtin_amdgcn_s_setprio(2);  // the recurrence's role goes first
  const float *M = (wrole ? a.f.W : a.f.Sinv) + (size_t)e * nc * blk;
  float *G = a.sb.G + ((size_t)e * a.ntiles + tau) * nc * vt;
  float *TV = a.sb.TV + ((size_t)e * a.ntiles + tau) * 2 * vt;
  const double *Rre = a.R + e * a.rnode + tau * kTile;
  const double *Rim = Rre + a.plane;
  const bool cplx = a.rcomplex != 0;
  const size_t rstride = (size_t)BP * a.m0p;
  const int nsteps = top ? len - 1 : len;
  auto rhs = [&](int c, bool valid) {
    return rhs_load32<BP>(Rre + c * rstride, Rim + c * rstride, a.m0p, cplx, rb, valid);
  };

  if (wrole) {
    const f4 h = rhs(start, true);
    acc_store_vec32<BP>(&s.v[0][0][0][0], -h, rb);
  }
  Frag32<BP> f0, f1, f2;
  frag_load32<BP>(f0, M + start * blk, rb, nsteps > 0);
  frag_load32<BP>(f1, M + (start + dir) * blk, rb, nsteps > 1);
  f4 r0 = rhs(start + dir, wrole && len > 1);
  f4 r1 = rhs(start + 2 * dir, wrole && len > 2);
  f4 r2 = f4zero();
  __syncthreads();
  int cur = 0;
  auto step = [&](int j, const Frag32<BP> &f, const f4 &r, Frag32<BP> &nf2, f4 &nr2) {
    const int c = start + dir * j;
    frag_load32<BP>(nf2, M + (c + 2 * dir) * blk, rb, j + 2 < nsteps);
    nr2 = rhs(c + 3 * dir, wrole && j + 3 < len);
    float b[BP / 2];
    bvec_load32<BP>(b, s.v[cur]);
    const bool more = j < len - 1;
    const f4 acc = frag_mfma32<BP>((wrole && more) ? r : f4zero(), f, b);
    vec_store_buf32<BP>(G + c * vt, -acc, rb, !wrole);
    if (wrole) {
      if (more)
        acc_store_vec32<BP>(&s.v[cur ^ 1][0][0][0], -acc, rb);
      else
        acc_store_vec32<BP>(TV + vt, acc, rb);  // c = -W~_m^T h~_m
    }
    __syncthreads();
    cur ^= 1;
  };
  int j = 0;
  for (; j + 3 <= nsteps; j += 3) {
    step(j, f0, r0, f2, r2);
    step(j + 1, f1, r1, f0, r0);
    step(j + 2, f2, r2, f1, r1);
  }
  if (j < nsteps) step(j, f0, r0, f2, r2);
  if (j + 1 < nsteps) step(j + 1, f1, r1, f0, r0);
  if (top && wrole) {
    const f4 u = acc_load_vec32<BP>(&s.v[cur][0][0][0], rb);
    acc_store_vec32<BP>(TV, -u, rb);  // h_{m-1}
  }
}

// Back sweep; ACCUM adds the solution to the float64 iterate X instead of
// writing it.  The iterate's tile of the next cell is loaded a step ahead.
template <int BP, bool ACCUM>
__global__ __launch_bounds__(BP * 4) void back32_kernel(Sweep32Args a) {
  __shared__ VecLds32<BP> s;
  const int item = xcd_item(blockIdx.x, gridDim.x, a.ntiles);
  const int tau = item % a.ntiles;
  const int grp = item / a.ntiles;
  const int e = grp >> 1;
  const bool top = (grp & 1) == 0;
  const int nc = a.nc, m = a.m;
  const int len = top ? m : nc - m;
  if (len <= 0) return;
  const size_t blk = 2 * (size_t)BP * BP;
  const size_t vt = 2 * (size_t)BP * kTile;
  const float *Sinv = a.f.Sinv + (size_t)e * nc * blk;
  const float *WT = a.f.WT + (size_t)e * nc * blk;
  const float *G = a.sb.G + ((size_t)e * a.ntiles + tau) * nc * vt;
  const float *TV = a.sb.TV + ((size_t)e * a.ntiles + tau) * 2 * vt;
  const size_t cs = (size_t)BP * a.m0p;
  double *Xre = a.X + 2 * e * a.plane + tau * kTile;
  double *Xim = Xre + a.plane;
  const int l = lane_id();
  const int rb = wave_id();
  const int n = l & 15;
  const int cbytes = BP * a.m0p * 8;
  auto xoff = [&](int r) { return ((rb * 16 + acc_row32(l, r)) * a.m0p + (n & 7)) * 8; };
  // this lane's four elements of the iterate at cell c (its own plane)
  auto xload = [&](int c, bool valid) {
    d4 v = d4zero();
    if (ACCUM) {
      const auto rr = buf_rsrc(Xre + c * cs, valid ? cbytes : 0);
      const auto ri = buf_rsrc(Xim + c * cs, valid ? cbytes : 0);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        v[r] = buf_load(rr, n < 8 ? xoff(r) : kBufferOff, 0) +
               buf_load(ri, n < 8 ? kBufferOff : xoff(r), 0);
    }
    return v;
  };
  auto emit = [&](int c, const f4 &x, const d4 &old) {
    const auto rr = buf_rsrc(Xre + c * cs, cbytes);
    const auto ri = buf_rsrc(Xim + c * cs, cbytes);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double v = old[r] + (double)x[r];
      buf_store(v, rr, n < 8 ? xoff(r) : kBufferOff, 0);
      buf_store(v, ri, n < 8 ? kBufferOff : xoff(r), 0);
    }
  };
  const int count = top ? m - 1 : nc - m;
  auto cell = [&](int j) { return top ? (m - 2 - j) : (m + j); };

  // twist cell: x_{m-1} = T (h_{m-1} + c)
  Frag32<BP> f0, f1;
  frag_load32<BP>(f0, Sinv + (m - 1) * blk, rb, true);
  const d4 xt = xload(m - 1, top);
  {
    f4 t = acc_load_vec32<BP>(TV, rb);
    if (nc - m > 0) t += acc_load_vec32<BP>(TV + vt, rb);
    acc_store_vec32<BP>(&s.v[1][0][0][0], t, rb);
  }
  frag_load32<BP>(f1, WT + cell(0) * blk, rb, count > 0);
  f4 ga = vec_load_buf32<BP>(G + cell(0) * vt, rb, count > 0), gb = f4zero();
  d4 xa = xload(cell(0), count > 0), xb = d4zero();
  __syncthreads();
  {
    float b[BP / 2];
    bvec_load32<BP>(b, s.v[1]);
    const f4 x = frag_mfma32<BP>(f4zero(), f0, b);
    acc_store_vec32<BP>(&s.v[0][0][0][0], -x, rb);
    if (top) emit(m - 1, x, xt);
  }
  __syncthreads();
  int cur = 0;
  auto step = [&](int j, const Frag32<BP> &f, const f4 &g, const d4 &xo, Frag32<BP> &nf, f4 &ng,
                  d4 &nxo) {
    const int c = cell(j);
    const bool nx = j + 1 < count;
    frag_load32<BP>(nf, WT + cell(j + 1) * blk, rb, nx);
    ng = vec_load_buf32<BP>(G + cell(j + 1) * vt, rb, nx);
    nxo = xload(cell(j + 1), nx);
    float b[BP / 2];
    bvec_load32<BP>(b, s.v[cur]);
    const f4 x = frag_mfma32<BP>(g, f, b);
    acc_store_vec32<BP>(&s.v[cur ^ 1][0][0][0], -x, rb);
    emit(c, x, xo);
    __syncthreads();
    cur ^= 1;
  };
  for (int j = 0; j < count; j += 2) {
    step(j, f1, ga, xa, f0, gb, xb);
    if (j + 1 < count) step(j + 1, f0, gb, xb, f1, ga, xa);
  }
}

template <int BP>
hipError_t sweeps32_bp(const Sweep32Args &a, int Ne, bool accumulate, int part,
                       hipStream_t st) {
  const int nblocks = Ne * 2 * a.ntiles;
  if (part & 1) {
    hipLaunchKernelGGL(forward32_kernel<BP>, dim3(nblocks), dim3(BP * 8), 0, st, a);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  if (part & 2) {
    if (accumulate)
      hipLaunchKernelGGL((back32_kernel<BP, true>), dim3(nblocks), dim3(BP * 4), 0, st, a);
    else
      hipLaunchKernelGGL((back32_kernel<BP, false>), dim3(nblocks), dim3(BP * 4), 0, st, a);
  }
  return hipGetLastError();
}

template <int BP>
hipError_t round_bp(const Factors &f, const Factors32 &g, size_t nplanes, hipStream_t st) {
  const double *src[3] = {f.Sinv, f.W, f.WT};
  float *dst[3] = {g.Sinv, g.W, g.WT};
  const size_t total = nplanes * BP * BP;
  size_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  for (int k = 0; k < 3; ++k) {
    hipLaunchKernelGGL(round_factors_kernel<BP>, dim3((unsigned)blocks), dim3(256), 0, st, src[k],
                       dst[k], nplanes);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_round_factors(const Pencil &p, int Ne, const Factors &f, const Factors32 &g,
                                hipStream_t st) {
  const size_t nplanes = (size_t)Ne * p.nc * 2;
  switch (p.bp) {
    case 16: return round_bp<16>(f, g, nplanes, st);
    case 32: return round_bp<32>(f, g, nplanes, st);
    case 48: return round_bp<48>(f, g, nplanes, st);
    case 64: return round_bp<64>(f, g, nplanes, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sweeps32(const Pencil &p, int Ne, const Factors32 &f, const SolveBufs32 &sb,
                           const double *R, size_t rnode, int rcomplex, int m0p, double *X,
                           int accumulate, int part, hipStream_t st) {
  Sweep32Args a;
  a.nc = p.nc; a.m = f.m; a.m0p = m0p; a.ntiles = m0p / kTile;
  a.f = f; a.sb = sb;
  a.R = R; a.rnode = rnode; a.rcomplex = rcomplex;
  a.plane = (size_t)p.nc * p.bp * m0p;
  a.X = X;
  switch (p.bp) {
    case 16: return sweeps32_bp<16>(a, Ne, accumulate != 0, part, st);
    case 32: return sweeps32_bp<32>(a, Ne, accumulate != 0, part, st);
    case 48: return sweeps32_bp<48>(a, Ne, accumulate != 0, part, st);
    case 64: return sweeps32_bp<64>(a, Ne, accumulate != 0, part, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace feast
