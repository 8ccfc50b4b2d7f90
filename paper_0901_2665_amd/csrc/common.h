// Shared device helpers for the FEAST kernels (gfx950 / CDNA4).
//
// Layout conventions used by every kernel of the library:
//  * A complex b x b block is stored as two real planes (re, im), each
//    BP x BP row-major, BP = b rounded up to a multiple of 16; padding rows
//    and columns hold the identity (diagonal blocks) or zero.
//  * Dense real N x M0 arrays are kept padded as [nc][BP][M0P], M0P = M0
//    rounded up to 16; padding is zero.
//  * Complex solve vectors are split in tiles of 8 complex columns:
//    [node][tile][cell][plane][BP][8].
//
// The matrix-core primitive is V_MFMA_F64_16X16X4_F64.  Lane l of a wave
// supplies A[l%16][l/16] and B[l/16][l%16] of a 16x4 by 4x16 product; the
// 16x16 accumulator is held as four doubles per lane, element r at row
// l/16 + 4r, column l%16 (checked on the device).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace feast {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ d4 d4zero() { return d4{0.0, 0.0, 0.0, 0.0}; }

// Raw buffer access.  Word 3 of an unformatted, unswizzled buffer resource
// on gfx9-class parts; an access whose offset lies at or beyond the
// resource's byte count touches no memory (loads return zero, stores are
// dropped).  A resource of 0 bytes therefore turns an access into a no-op
// without a branch, which keeps the number of memory operations in flight
// the same on every path (so waits on earlier loads stay exact).
constexpr int kBufferWord3 = 0x00020000;
constexpr int kBufferOff = 0x40000000;  // an offset beyond every resource here
typedef unsigned int u32x2 __attribute__((__vector_size__(8)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, bytes,
                                          kBufferWord3);
}

__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
}

__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t rs, int voff,
                                          int soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, voff, soff, 0);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
// Stored layout of the blocks of the shifted factorisation (Sinv, W, W^T):
// position of element (i, j) of one BP x BP plane.  The sweeps use a stored
// block M as the matrix operand A'[r][k] = M[k][r] with k = 4 ks + kl (ks the
// k-step of V_MFMA_F64_16X16X4_F64, kl = lane / 16); here the k-steps 2p and
// 2p+1 of one (kl, r) sit next to each other, so one 16-byte load per lane
// fetches both and the 64 lanes of a wave read 1 KB contiguously.
template <int BP>
__host__ __device__ constexpr int fpos(int i, int j) {
  return ((((i >> 3) << 2) + (i & 3)) * BP + j) * 2 + ((i >> 2) & 1);
}

// Matrix-operand fragments of one real BP x BP plane stored in the layout
// fpos (above) for this lane: v[ks] = M[4 ks + kl][rb * 16 + lane % 16],
// kl = lane / 16, i.e. the operand A'[r][k] = M[k][r] of row block rb (and,
// the lane mapping of A and B being the same, the operand B[k][n] = M[k][n]
// of column block rb).  Sixteen-byte loads through a buffer resource that
// covers the plane (or nothing: valid = false, the loads then return zero).
template <int BP>
__device__ __forceinline__ void frag_plane_load(double (&v)[BP / 4], const double *M, int rb,
                                                bool valid) {
  const int l = threadIdx.x & 63;
  const int row = rb * 16 + (l & 15), kl = l >> 4;
  const auto rs = buf_rsrc(M, valid ? BP * BP * 8 : 0);
  const int vo = fpos<BP>(kl, row) * 8;  // pair p adds 8 p BP elements
#pragma unroll
  for (int p = 0; p < BP / 8; ++p) {
    const auto x = __builtin_amdgcn_raw_buffer_load_b128(rs, vo, p * 8 * BP * 8, 0);
    v[2 * p] = __builtin_bit_cast(double, (u32x2){x[0], x[1]});
    v[2 * p + 1] = __builtin_bit_cast(double, (u32x2){x[2], x[3]});
  }
}

// wave index, known to the compiler as uniform across the wave
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Accumulator element r of lane l sits at (row, col) of its 16x16 tile.
__device__ __forceinline__ int acc_row(int l, int r) { return (l >> 4) + 4 * r; }
__device__ __forceinline__ int acc_col(int l) { return l & 15; }

// Complex helpers on (re, im) pairs.
struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx crecip(cplx a) {
  // Smith's scaling keeps the quotient finite for tiny or huge pivots.
  if (fabs(a.re) >= fabs(a.im)) {
    double t = a.im / a.re, d = a.re + a.im * t;
    return {1.0 / d, -t / d};
  } else {
    double t = a.re / a.im, d = a.re * t + a.im;
    return {t / d, -1.0 / d};
  }
}

// 1/a by Newton's iteration for the reciprocal, x <- x (2 - d x), started
// from the hardware estimate: two steps reach full double precision for the
// normal-range pivots met here (no denormal or overflow scaling).
__device__ __forceinline__ double rcp_newton(double d) {
  double x = __builtin_amdgcn_rcp(d);
  double e = fma(-d, x, 1.0);
  x = fma(x, e, x);
  e = fma(-d, x, 1.0);
  return fma(x, e, x);
}
// 1/(a + ib) = (a - ib) / (a^2 + b^2), with a and b first scaled by the
// power of two 2^-e of the larger component (exact), so that the squares
// neither overflow nor underflow: 1/(a + ib) = 2^-e / (a' + ib').
__device__ __forceinline__ cplx crecip_fast(cplx a) {
  const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(a.re), fabs(a.im)));
  const double ar = __builtin_amdgcn_ldexp(a.re, -e), ai = __builtin_amdgcn_ldexp(a.im, -e);
  const double inv = rcp_newton(fma(ar, ar, ai * ai));
  return {__builtin_amdgcn_ldexp(ar * inv, -e), __builtin_amdgcn_ldexp(-ai * inv, -e)};
}

// Grid position -> work item, placing consecutive groups of `per_group`
// items on one XCD (workgroups are dispatched to the 8 XCDs round-robin, so
// items that read the same factor stream share that XCD's L2).
__device__ __forceinline__ int xcd_item(int bid, int nblocks, int per_group) {
  const int nx = 8;
  if (nblocks % nx != 0 || (nblocks / nx) % per_group != 0) return bid;
  int xcd = bid % nx, slot = bid / nx;
  int per_xcd = nblocks / nx;
  return xcd * per_xcd + slot;
}

}  // namespace feast
