// Twisted block factorisation of the shifted matrices M_e = Z_e B - A
// (the linear systems of Fig. 2 step 2), one chain of cells per workgroup.
//
// M_e is complex symmetric (A, B real symmetric) with Im M_e = Im(Z_e) B
// positive definite, so every Schur complement met below exists and stays
// complex symmetric; no pivoting between blocks is needed.
//
// Top chain (cells 0..m-1, top-down):    S_0 = D_0,
//   Sinv_j = S_j^{-1},  W_j = Sinv_j U_j,  S_{j+1} = D_{j+1} - U_j^T W_j.
// Bottom chain (cells nc-1..m, bottom-up) runs the same recurrence on the
// reversed chain (coupling of cell j towards j-1 is U_{j-1}^T).
// Twist cell m-1: T = (S_{m-1} - U_{m-1} W~_m)^{-1}.
// Here D_j = Z B_jj - A_jj and U_j = Z B_{j,j+1} - A_{j,j+1} are formed on the
// fly from the real blocks.  Every inverse is symmetrised, so Sinv may be read
// transposed.  The factors are computed once per solve and reused by every
// refinement loop (Sec. V, parallelism (ii)).
#include "common.h"
#include "kernels.h"

namespace feast {
namespace {

constexpr int kThreads = 256;

template <int BP>
struct Lds {
  static constexpr int LD = BP + 1;  // odd stride: conflict-free column reads
  static constexpr int PLANE = BP * LD;
  double A[2 * PLANE];                // slot A (re plane, im plane)
  double B[2 * PLANE];                // slot B
  double row[2][2][BP];               // Gauss-Jordan pivot row (double buffered)
  double col[2][2][BP];               // Gauss-Jordan pivot column
};

// slot <- z*Bblk - Ablk (or its transpose), identity padding on the diagonal.
template <int BP>
__device__ void form_block(double *slot, const double *Ablk, const double *Bblk, int b,
                           double zr, double zi, bool transpose, bool diag_pad) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  for (int idx = threadIdx.x; idx < BP * BP; idx += kThreads) {
    int r = idx / BP, c = idx % BP;
    double re, im;
    if (r < b && c < b) {
      int src = transpose ? c * b + r : r * b + c;
      double bv = Bblk[src], av = Ablk[src];
      re = zr * bv - av;
      im = zi * bv;
    } else {
      re = (diag_pad && r == c) ? 1.0 : 0.0;
      im = 0.0;
    }
    slot[r * LD + c] = re;
    slot[PLANE + r * LD + c] = im;
  }
}

// slot <- complex block from global planes [2][BP][BP].
template <int BP>
__device__ void load_block(double *slot, const double *g) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  for (int idx = threadIdx.x; idx < BP * BP; idx += kThreads) {
    int r = idx / BP, c = idx % BP;
    slot[r * LD + c] = g[idx];
    slot[PLANE + r * LD + c] = g[BP * BP + idx];
  }
}

template <int BP>
__device__ void store_block(double *g, const double *slot, bool transpose) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  for (int idx = threadIdx.x; idx < BP * BP; idx += kThreads) {
    int r = idx / BP, c = idx % BP;
    int s = transpose ? c * LD + r : r * LD + c;
    g[idx] = slot[s];
    g[BP * BP + idx] = slot[PLANE + s];
  }
}

// In-place Gauss-Jordan inversion of the complex block in slot A, without
// pivoting (every leading principal minor of a complex symmetric matrix with
// positive definite imaginary part is non-zero).  Each thread keeps a 4x4
// patch in registers; pivot row and column travel through LDS, one barrier
// per elimination step.  The result is symmetrised, written back to slot A
// and, if gout != nullptr, to global memory.
template <int BP>
__device__ void gj_invert(Lds<BP> &s, double *gout) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  const int t = threadIdx.x;
  const int ti = t >> 4, tj = t & 15;
  const bool act = (4 * ti < BP) && (4 * tj < BP);
  double ar[4][4], ai[4][4];
  if (act) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        ar[u][v] = s.A[(4 * ti + u) * LD + 4 * tj + v];
        ai[u][v] = s.A[PLANE + (4 * ti + u) * LD + 4 * tj + v];
      }
    if (ti == 0)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        s.row[0][0][4 * tj + v] = ar[0][v];
        s.row[0][1][4 * tj + v] = ai[0][v];
      }
    if (tj == 0)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        s.col[0][0][4 * ti + u] = ar[u][0];
        s.col[0][1][4 * ti + u] = ai[u][0];
      }
  }
  __syncthreads();
  for (int k = 0; k < BP; ++k) {
    const int q = k & 1;
    cplx piv = crecip(cplx{s.row[q][0][k], s.row[q][1][k]});
    if (act) {
      cplx rk[4], ck[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) rk[v] = cmul(cplx{s.row[q][0][4 * tj + v], s.row[q][1][4 * tj + v]}, piv);
#pragma unroll
      for (int u = 0; u < 4; ++u) ck[u] = cplx{s.col[q][0][4 * ti + u], s.col[q][1][4 * ti + u]};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool on_row = (4 * ti + u) == k;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool on_col = (4 * tj + v) == k;
          cplx a{ar[u][v], ai[u][v]};
          cplx upd;
          if (on_row && on_col) {
            upd = piv;
          } else if (on_row) {
            upd = rk[v];
          } else if (on_col) {
            cplx m = cmul(ck[u], piv);
            upd = cplx{-m.re, -m.im};
          } else {
            cplx m = cmul(ck[u], rk[v]);
            upd = cplx{a.re - m.re, a.im - m.im};
          }
          ar[u][v] = upd.re;
          ai[u][v] = upd.im;
        }
      }
      // publish row and column k+1 (register indices stay compile-time)
      const int k1 = k + 1;
      if (k1 < BP) {
        const int qn = k1 & 1;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (k1 == 4 * ti + u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              s.row[qn][0][4 * tj + v] = ar[u][v];
              s.row[qn][1][4 * tj + v] = ai[u][v];
            }
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (k1 == 4 * tj + v)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              s.col[qn][0][4 * ti + u] = ar[u][v];
              s.col[qn][1][4 * ti + u] = ai[u][v];
            }
      }
    }
    __syncthreads();
  }
  // symmetrise: S <- (S + S^T) / 2
  if (act) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        s.A[(4 * ti + u) * LD + 4 * tj + v] = ar[u][v];
        s.A[PLANE + (4 * ti + u) * LD + 4 * tj + v] = ai[u][v];
      }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        ar[u][v] = 0.5 * (ar[u][v] + s.A[(4 * tj + v) * LD + 4 * ti + u]);
        ai[u][v] = 0.5 * (ai[u][v] + s.A[PLANE + (4 * tj + v) * LD + 4 * ti + u]);
      }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * ti + u, c = 4 * tj + v;
        s.A[r * LD + c] = ar[u][v];
        s.A[PLANE + r * LD + c] = ai[u][v];
        if (gout) {
          gout[r * BP + c] = ar[u][v];
          gout[BP * BP + r * BP + c] = ai[u][v];
        }
      }
  }
  __syncthreads();
}

// Complex product on the matrix cores, operands in LDS slots:
//   acc (+)= sign * op(X) * Y,   op(X) = X or X^T.
// Wave w (< BP/16) owns row block w and all column blocks; acc[tj] holds
// the re / im 16x16 tiles.
template <int BP>
__device__ void cgemm_lds(d4 (&accr)[BP / 16], d4 (&acci)[BP / 16], const double *X,
                          bool transX, const double *Y, double sign) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE, NT = BP / 16;
  const int w = wave_id(), l = lane_id();
  if (w >= NT) return;
  const int row = w * 16 + (l & 15);
  const int kl = l >> 4;
  for (int k0 = 0; k0 < BP; k0 += 4) {
    const int k = k0 + kl;
    const int xa = transX ? k * LD + row : row * LD + k;
    const double xr = sign * X[xa], xi = sign * X[PLANE + xa];
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) {
      const int yb = k * LD + tj * 16 + (l & 15);
      const double yr = Y[yb], yi = Y[PLANE + yb];
      accr[tj] = mfma(xr, yr, accr[tj]);
      accr[tj] = mfma(-xi, yi, accr[tj]);
      acci[tj] = mfma(xr, yi, acci[tj]);
      acci[tj] = mfma(xi, yr, acci[tj]);
    }
  }
}

template <int BP>
__device__ void acc_to_lds(double *slot, const d4 (&accr)[BP / 16], const d4 (&acci)[BP / 16]) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE, NT = BP / 16;
  const int w = wave_id(), l = lane_id();
  if (w >= NT) return;
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + acc_row(l, r), col = tj * 16 + acc_col(l);
      slot[row * LD + col] = accr[tj][r];
      slot[PLANE + row * LD + col] = acci[tj][r];
    }
}

template <int BP>
__device__ void acc_to_global(double *g, const d4 (&accr)[BP / 16], const d4 (&acci)[BP / 16]) {
  constexpr int NT = BP / 16;
  const int w = wave_id(), l = lane_id();
  if (w >= NT) return;
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + acc_row(l, r), col = tj * 16 + acc_col(l);
      g[row * BP + col] = accr[tj][r];
      g[BP * BP + row * BP + col] = acci[tj][r];
    }
}

// acc <- z*Bblk - Ablk (diagonal block, identity padding).
template <int BP>
__device__ void acc_from_diag(d4 (&accr)[BP / 16], d4 (&acci)[BP / 16], const double *Ablk,
                              const double *Bblk, int b, double zr, double zi) {
  constexpr int NT = BP / 16;
  const int w = wave_id(), l = lane_id();
  if (w >= NT) return;
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + acc_row(l, r), col = tj * 16 + acc_col(l);
      double re, im;
      if (row < b && col < b) {
        double bv = Bblk[row * b + col], av = Ablk[row * b + col];
        re = zr * bv - av;
        im = zi * bv;
      } else {
        re = (row == col) ? 1.0 : 0.0;
        im = 0.0;
      }
      accr[tj][r] = re;
      acci[tj][r] = im;
    }
}

template <int BP>
__device__ void acc_from_global(d4 (&accr)[BP / 16], d4 (&acci)[BP / 16], const double *g) {
  constexpr int NT = BP / 16;
  const int w = wave_id(), l = lane_id();
  if (w >= NT) return;
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + acc_row(l, r), col = tj * 16 + acc_col(l);
      accr[tj][r] = g[row * BP + col];
      acci[tj][r] = g[BP * BP + row * BP + col];
    }
}

template <int BP>
__global__ __launch_bounds__(kThreads) void factor_chain_kernel(Pencil p, Shifts sh, Factors f) {
  extern __shared__ double smem_raw[];
  Lds<BP> &s = *reinterpret_cast<Lds<BP> *>(smem_raw);
  constexpr int NT = BP / 16;
  const int e = blockIdx.x >> 1;
  const bool top = (blockIdx.x & 1) == 0;
  const int nc = p.nc, b = p.b, m = f.m;
  const int start = top ? 0 : nc - 1;
  const int dir = top ? 1 : -1;
  const int len = top ? m : nc - m;
  if (len <= 0) return;
  const double zr = sh.zre[e], zi = sh.zim[e];
  const size_t blk = 2 * (size_t)BP * BP;
  const size_t bb = (size_t)b * b;
  double *Sinv = f.Sinv + (size_t)e * nc * blk;
  double *Wg = f.W + (size_t)e * nc * blk;
  double *WTg = f.WT + (size_t)e * nc * blk;

  form_block<BP>(s.A, p.Ad + start * bb, p.Bd + start * bb, b, zr, zi, false, true);
  __syncthreads();
  for (int j = 0; j < len; ++j) {
    const int c = start + dir * j;
    const bool last = (j == len - 1);
    if (top && last) {
      // raw Schur complement at the twist cell, finished by twist_kernel
      store_block<BP>(f.TW + (size_t)e * blk, s.A, false);
      break;
    }
    // coupling from c to the next cell in chain order
    if (top)
      form_block<BP>(s.B, p.Au + c * bb, p.Bu + c * bb, b, zr, zi, false, false);
    else
      form_block<BP>(s.B, p.Au + (c - 1) * bb, p.Bu + (c - 1) * bb, b, zr, zi, true, false);
    gj_invert<BP>(s, Sinv + c * blk);  // ends with a barrier
    d4 wr[NT], wi[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) { wr[q] = d4zero(); wi[q] = d4zero(); }
    cgemm_lds<BP>(wr, wi, s.A, true, s.B, 1.0);  // W = Sinv * Cpl
    __syncthreads();
    acc_to_lds<BP>(s.A, wr, wi);
    acc_to_global<BP>(Wg + c * blk, wr, wi);
    __syncthreads();
    store_block<BP>(WTg + c * blk, s.A, true);
    if (!last) {
      const int cn = c + dir;
      d4 sr[NT], si[NT];
      acc_from_diag<BP>(sr, si, p.Ad + cn * bb, p.Bd + cn * bb, b, zr, zi);
      cgemm_lds<BP>(sr, si, s.B, true, s.A, -1.0);  // S_next = D - Cpl^T W
      __syncthreads();
      acc_to_lds<BP>(s.A, sr, si);
      __syncthreads();
    }
  }
}

// Twist cell: Sinv[m-1] = (S_{m-1} - U_{m-1} W~_m)^{-1}  (no bottom chain:
// Sinv[m-1] = S_{m-1}^{-1}).
template <int BP>
__global__ __launch_bounds__(kThreads) void twist_kernel(Pencil p, Shifts sh, Factors f) {
  extern __shared__ double smem_raw[];
  Lds<BP> &s = *reinterpret_cast<Lds<BP> *>(smem_raw);
  constexpr int NT = BP / 16;
  const int e = blockIdx.x;
  const int nc = p.nc, b = p.b, m = f.m;
  const double zr = sh.zre[e], zi = sh.zim[e];
  const size_t blk = 2 * (size_t)BP * BP;
  const size_t bb = (size_t)b * b;
  const double *TW = f.TW + (size_t)e * blk;
  if (nc - m == 0) {
    load_block<BP>(s.A, TW);
    __syncthreads();
  } else {
    load_block<BP>(s.A, f.W + ((size_t)e * nc + m) * blk);
    form_block<BP>(s.B, p.Au + (m - 1) * bb, p.Bu + (m - 1) * bb, b, zr, zi, false, false);
    __syncthreads();
    d4 sr[NT], si[NT];
    acc_from_global<BP>(sr, si, TW);
    cgemm_lds<BP>(sr, si, s.B, false, s.A, -1.0);
    __syncthreads();
    acc_to_lds<BP>(s.A, sr, si);
    __syncthreads();
  }
  gj_invert<BP>(s, f.Sinv + ((size_t)e * nc + (m - 1)) * blk);
}

template <int BP>
hipError_t launch_factor_bp(const Pencil &p, const Shifts &s, int Ne, const Factors &f,
                            hipStream_t st) {
  const size_t shm = sizeof(Lds<BP>);
  hipError_t err = hipFuncSetAttribute((const void *)factor_chain_kernel<BP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (err != hipSuccess) return err;
  err = hipFuncSetAttribute((const void *)twist_kernel<BP>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(factor_chain_kernel<BP>, dim3(2 * Ne), dim3(kThreads), shm, st, p, s, f);
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(twist_kernel<BP>, dim3(Ne), dim3(kThreads), shm, st, p, s, f);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_factor(const Pencil &p, const Shifts &s, int Ne, const Factors &f,
                         hipStream_t st) {
  switch (p.bp) {
    case 16: return launch_factor_bp<16>(p, s, Ne, f, st);
    case 32: return launch_factor_bp<32>(p, s, Ne, f, st);
    case 48: return launch_factor_bp<48>(p, s, Ne, f, st);
    case 64: return launch_factor_bp<64>(p, s, Ne, f, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace feast
