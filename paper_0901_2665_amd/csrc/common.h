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

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

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
// 1/(a + ib) = (a - ib) / (a^2 + b^2), with the common factor scaled by the
// larger component so that the squares neither overflow nor underflow.
__device__ __forceinline__ cplx crecip_fast(cplx a) {
  const double s = fmax(fabs(a.re), fabs(a.im));
  const double rs = rcp_newton(s);
  const double ar = a.re * rs, ai = a.im * rs;
  const double inv = rcp_newton(ar * ar + ai * ai) * rs;
  return {ar * inv, -ai * inv};
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
