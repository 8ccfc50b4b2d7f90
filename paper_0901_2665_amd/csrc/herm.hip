// Hermitian A (Sec. III.B, eq. 12 and the changes listed after Fig. 2):
// A complex Hermitian, B real s.p.d., the start block Y, the subspace Q, the
// reduced eigenvectors Phi and the Ritz vectors X complex.  Complex values are
// interleaved (re, im) double pairs; dense blocks are [N][m] row-major,
// matrix blocks [b][b] row-major.
//
// For each contour point the block LU of M = Z B - A (no longer complex
// symmetric) is computed once:
//   S_0 = D_0,  Sinv_i = S_i^{-1},  W_i = Sinv_i C_i,  V_i = L_i Sinv_i,
//   S_{i+1} = D_{i+1} - L_i W_i,
// with D_i = Z B_ii - A_ii, C_i = Z B_{i,i+1} - A_{i,i+1} (upper coupling)
// and L_i = Z B_{i,i+1}^T - A_{i,i+1}^H (lower coupling).  Every principal
// submatrix of M has a positive definite imaginary part Im(Z) B, so every
// S_i exists without pivoting.  The same factors give both solves of eq. 12:
//   M x = R:    h_0 = R_0, g_i = Sinv_i h_i, h_{i+1} = R_{i+1} - V_i h_i;
//               x_last = g_last, x_i = g_i - W_i x_{i+1};
//   M^H y = R:  k_0 = R_0, z_i = Sinv_i^H k_i, k_{i+1} = R_{i+1} - W_i^H k_i;
//               y_last = z_last, y_i = z_i - V_i^H y_{i+1}
// (M = L U with unit lower L of blocks V_i and upper U of blocks S_i, C_i;
// M^H = U^H L^H).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace feast {

namespace {

struct cd {
  double r, i;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cd cmulc(cd a, cd b) {  // conj(a) * b
  return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cd cinv(cd a) {
  // 1/a with the larger component scaled away (Smith's method)
  if (fabs(a.r) >= fabs(a.i)) {
    const double t = a.i / a.r, d = a.r + a.i * t;
    return {1.0 / d, -t / d};
  }
  const double t = a.r / a.i, d = a.i + a.r * t;
  return {t / d, -1.0 / d};
}
__device__ __forceinline__ cd ld(const double *p, size_t k) { return {p[2 * k], p[2 * k + 1]}; }
__device__ __forceinline__ void st(double *p, size_t k, cd v) {
  p[2 * k] = v.r;
  p[2 * k + 1] = v.i;
}

constexpr int kT = 256;

// Element (r, c) of the shifted blocks from the caller's blocks.
__device__ __forceinline__ cd shifted_diag(const HPencil &p, int cell, int r, int c, double zr,
                                           double zi) {
  const size_t o = ((size_t)cell * p.b + r) * p.b + c;
  const double bv = p.Bd[o];
  return {zr * bv - p.Ad[2 * o], zi * bv - p.Ad[2 * o + 1]};
}
__device__ __forceinline__ cd shifted_upper(const HPencil &p, int cell, int r, int c, double zr,
                                            double zi) {  // C_cell (r, c)
  const size_t o = ((size_t)cell * p.b + r) * p.b + c;
  const double bv = p.Bu[o];
  return {zr * bv - p.Au[2 * o], zi * bv - p.Au[2 * o + 1]};
}
__device__ __forceinline__ cd shifted_lower(const HPencil &p, int cell, int r, int c, double zr,
                                            double zi) {  // L_cell (r, c) = Z Bu(c, r) - conj(Au(c, r))
  const size_t o = ((size_t)cell * p.b + c) * p.b + r;
  const double bv = p.Bu[o];
  return {zr * bv - p.Au[2 * o], zi * bv + p.Au[2 * o + 1]};
}

constexpr int kMaxOut = 36;  // outputs per thread of a b x b block (b <= 96)

// One workgroup per contour point, sequential over the cells.  Dynamic LDS:
// the complex b x (b+1) block S (Sinv after the inversion); the products read
// the couplings from the caller's blocks and W back from global memory (its
// lines are written once per cell and not read before, so no stale copy can
// sit in the vector cache).
__global__ __launch_bounds__(kT) void hfactor_kernel(HPencil p, Shifts sh, double *Sinv,
                                                     double *W, double *V) {
  extern __shared__ double hsm[];
  const int b = p.b, nc = p.nc, ldb = b + 1, e = blockIdx.x, t = threadIdx.x;
  double *S = hsm;                     // [b][ldb] complex
  const double zr = sh.zre[e], zi = sh.zim[e];
  const size_t bb = (size_t)b * b;
  const int nout = b * b;
  double *Se = Sinv + 2 * (size_t)e * nc * bb;
  double *We = W + 2 * (size_t)e * (nc > 1 ? nc - 1 : 1) * bb;
  double *Ve = V + 2 * (size_t)e * (nc > 1 ? nc - 1 : 1) * bb;
  for (int o = t; o < nout; o += kT) st(S, (o / b) * ldb + o % b, shifted_diag(p, 0, o / b, o % b, zr, zi));
  __syncthreads();
  for (int cell = 0; cell < nc; ++cell) {
    // in-place Gauss-Jordan inverse without pivoting
    for (int k = 0; k < b; ++k) {
      const cd piv = cinv(ld(S, k * ldb + k));
      __syncthreads();
      for (int j = t; j < b; j += kT)
        if (j != k) st(S, k * ldb + j, cmul(ld(S, k * ldb + j), piv));
      __syncthreads();
      for (int o = t; o < nout; o += kT) {
        const int r = o / b, j = o % b;
        if (r != k && j != k) st(S, r * ldb + j, csub(ld(S, r * ldb + j), cmul(ld(S, r * ldb + k), ld(S, k * ldb + j))));
      }
      __syncthreads();
      for (int r = t; r < b; r += kT) {
        if (r != k) {
          const cd v = cmul(ld(S, r * ldb + k), piv);
          st(S, r * ldb + k, {-v.r, -v.i});
        } else {
          st(S, k * ldb + k, piv);
        }
      }
      __syncthreads();
    }
    for (int o = t; o < nout; o += kT) st(Se + 2 * (size_t)cell * bb, o, ld(S, (o / b) * ldb + o % b));
    if (cell == nc - 1) break;
    double *Wc = We + 2 * (size_t)cell * bb;
    // W = Sinv C, V = L Sinv (outputs o = t + kT q)
    for (int q = 0; q < kMaxOut; ++q) {
      const int o = t + kT * q;
      if (o >= nout) break;
      const int r = o / b, c = o % b;
      cd w = {0.0, 0.0}, v = {0.0, 0.0};
      for (int k = 0; k < b; ++k) {
        w = cadd(w, cmul(ld(S, r * ldb + k), shifted_upper(p, cell, k, c, zr, zi)));
        v = cadd(v, cmul(shifted_lower(p, cell, r, k, zr, zi), ld(S, k * ldb + c)));
      }
      st(Wc, o, w);
      st(Ve + 2 * (size_t)cell * bb, o, v);
    }
    __syncthreads();  // W complete (stores done) and Sinv no longer read
    // S_next = D_{cell+1} - L W straight over Sinv in LDS (this phase reads
    // only the caller's blocks and W)
    for (int q = 0; q < kMaxOut; ++q) {
      const int o = t + kT * q;
      if (o >= nout) break;
      const int r = o / b, c = o % b;
      cd s = shifted_diag(p, cell + 1, r, c, zr, zi);
      for (int k = 0; k < b; ++k) s = csub(s, cmul(shifted_lower(p, cell, r, k, zr, zi), ld(Wc, (size_t)k * b + c)));
      st(S, r * ldb + c, s);
    }
    __syncthreads();
  }
}

constexpr int kCols = 16;  // right-hand sides per sweep workgroup

constexpr int kTileOut = 6;  // outputs per thread of a b x kCols tile (b <= 96)

// y (b x kCols tile in LDS, complex, leading dim kCols) = op(Mat) * x, with
// op = identity or conjugate transpose; Mat [b][b] complex in global memory.
// Every thread keeps its outputs in out[] (o = t + kT q).
__device__ __forceinline__ void tile_apply(const double *Mat, bool adj, const double *x, int b,
                                           int ncol, cd (&out)[kTileOut]) {
  const int t = threadIdx.x;
  for (int q = 0; q < kTileOut; ++q) {
    const int o = t + kT * q;
    out[q] = {0.0, 0.0};
    if (o >= b * kCols) continue;
    const int r = o / kCols, c = o % kCols;
    if (c >= ncol) continue;
    cd s = {0.0, 0.0};
    if (!adj) {
      for (int k = 0; k < b; ++k) s = cadd(s, cmul(ld(Mat, (size_t)r * b + k), ld(x, k * kCols + c)));
    } else {
      for (int k = 0; k < b; ++k) s = cadd(s, cmulc(ld(Mat, (size_t)k * b + r), ld(x, k * kCols + c)));
    }
    out[q] = s;
  }
}

// Forward and back sweeps, one workgroup per (contour point, solve, column
// tile): solve 0 is M x = R, solve 1 is M^H y = R.  G [Ne][2][N][m] holds the
// forward results and is overwritten by the solutions.
__global__ __launch_bounds__(kT) void hsweep_kernel(HPencil p, const double *Sinv, const double *W,
                                                    const double *V, const double *R, int m,
                                                    double *G) {
  __shared__ double xs[2 * 96 * kCols];
  const int e = blockIdx.x, adj = blockIdx.y, c0 = blockIdx.z * kCols;
  const int b = p.b, nc = p.nc, t = threadIdx.x;
  const int ncol = m - c0 < kCols ? m - c0 : kCols;
  const size_t bb = (size_t)b * b, N = (size_t)nc * b;
  const double *Se = Sinv + 2 * (size_t)e * nc * bb;
  const size_t nf = nc > 1 ? nc - 1 : 1;
  const double *We = W + 2 * (size_t)e * nf * bb;
  const double *Ve = V + 2 * (size_t)e * nf * bb;
  double *Ge = G + 2 * ((size_t)e * 2 + adj) * N * m;
  const double *Fwd = adj ? We : Ve;   // coupling of the forward recursion
  const double *Bwd = adj ? Ve : We;   // coupling of the back recursion
  cd out[kTileOut];
  // h_0 = R_0
  for (int o = t; o < b * kCols; o += kT) {
    const int r = o / kCols, c = o % kCols;
    st(xs, o, c < ncol ? ld(R, (size_t)r * m + c0 + c) : cd{0.0, 0.0});
  }
  __syncthreads();
  for (int cell = 0; cell < nc; ++cell) {
    tile_apply(Se + 2 * (size_t)cell * bb, adj, xs, b, ncol, out);  // g = Sinv h (or Sinv^H k)
    for (int q = 0; q < kTileOut; ++q) {
      const int o = t + kT * q;
      if (o >= b * kCols) break;
      const int r = o / kCols, c = o % kCols;
      if (c < ncol) st(Ge, ((size_t)cell * b + r) * m + c0 + c, out[q]);
    }
    if (cell == nc - 1) break;
    tile_apply(Fwd + 2 * (size_t)cell * bb, adj, xs, b, ncol, out);  // V h (or W^H k)
    __syncthreads();
    for (int q = 0; q < kTileOut; ++q) {
      const int o = t + kT * q;
      if (o >= b * kCols) break;
      const int r = o / kCols, c = o % kCols;
      const cd rv = c < ncol ? ld(R, ((size_t)(cell + 1) * b + r) * m + c0 + c) : cd{0.0, 0.0};
      st(xs, o, csub(rv, out[q]));
    }
    __syncthreads();
  }
  // back sweep: x_last = g_last (in G and, as the running vector, in xs)
  __syncthreads();
  for (int o = t; o < b * kCols; o += kT) {
    const int r = o / kCols, c = o % kCols;
    st(xs, o, c < ncol ? ld(Ge, ((size_t)(nc - 1) * b + r) * m + c0 + c) : cd{0.0, 0.0});
  }
  __syncthreads();
  for (int cell = nc - 2; cell >= 0; --cell) {
    tile_apply(Bwd + 2 * (size_t)cell * bb, adj, xs, b, ncol, out);  // W x (or V^H y)
    __syncthreads();
    for (int q = 0; q < kTileOut; ++q) {
      const int o = t + kT * q;
      if (o >= b * kCols) break;
      const int r = o / kCols, c = o % kCols;
      if (c >= ncol) {
        st(xs, o, cd{0.0, 0.0});
        continue;
      }
      const size_t gi = ((size_t)cell * b + r) * m + c0 + c;
      const cd v = csub(ld(Ge, gi), out[q]);
      st(Ge, gi, v);
      st(xs, o, v);
    }
    __syncthreads();
  }
}

// Q = sum_e (c_e x_e + conj(c_e) y_e), c_e = -(w_e/4) r e^{i theta_e}
// (eq. 12), nodes in order.
__global__ void haccumulate_kernel(const double *G, int Ne, size_t Nm, const double *cre,
                                   const double *cim, double *Q) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < Nm;
       i += (size_t)gridDim.x * blockDim.x) {
    cd s = {0.0, 0.0};
    for (int e = 0; e < Ne; ++e) {
      const cd c = {cre[e], cim[e]};
      const cd x = ld(G + 2 * (size_t)(2 * e) * Nm, i);
      const cd y = ld(G + 2 * (size_t)(2 * e + 1) * Nm, i);
      s = cadd(s, cadd(cmul(c, x), cmulc(c, y)));
    }
    st(Q, i, s);
  }
}

// out = T V for T = A (complex Hermitian, which = 0) or B (real, which = 1);
// V, out complex [N][m].
__global__ void happly_kernel(HPencil p, int which, const double *Vin, int m, double *out) {
  const int b = p.b, nc = p.nc;
  const size_t total = (size_t)nc * b * m;
  const size_t bb = (size_t)b * b;
  for (size_t o = blockIdx.x * (size_t)blockDim.x + threadIdx.x; o < total;
       o += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(o % m);
    const size_t row = o / m;
    const int cell = (int)(row / b), r = (int)(row % b);
    cd s = {0.0, 0.0};
    for (int k = 0; k < b; ++k) {  // diagonal block
      const size_t ai = (size_t)cell * bb + (size_t)r * b + k;
      const cd a = which == 0 ? ld(p.Ad, ai) : cd{p.Bd[ai], 0.0};
      s = cadd(s, cmul(a, ld(Vin, ((size_t)cell * b + k) * m + j)));
    }
    if (cell + 1 < nc) {  // upper coupling (cell, cell+1)
      for (int k = 0; k < b; ++k) {
        const size_t ai = (size_t)cell * bb + (size_t)r * b + k;
        const cd a = which == 0 ? ld(p.Au, ai) : cd{p.Bu[ai], 0.0};
        s = cadd(s, cmul(a, ld(Vin, ((size_t)(cell + 1) * b + k) * m + j)));
      }
    }
    if (cell > 0) {  // lower coupling (cell, cell-1): conjugate transpose of the upper one
      for (int k = 0; k < b; ++k) {
        const size_t ai = (size_t)(cell - 1) * bb + (size_t)k * b + r;
        const cd a = which == 0 ? cd{p.Au[2 * ai], -p.Au[2 * ai + 1]} : cd{p.Bu[ai], 0.0};
        s = cadd(s, cmul(a, ld(Vin, ((size_t)(cell - 1) * b + k) * m + j)));
      }
    }
    st(out, o, s);
  }
}

constexpr int kHGramRows = 128;

// partial[blk][i][j] = sum over rows of X(row, i)^* V(row, j), m <= 64.
__global__ __launch_bounds__(kT) void hgram_kernel(const double *X, const double *Vin, long long N,
                                                   int m, double *partial) {
  __shared__ double xs[2 * 16 * 64];
  __shared__ double vs[2 * 16 * 64];
  const long long r0 = (long long)blockIdx.x * kHGramRows;
  const long long r1 = r0 + kHGramRows < N ? r0 + kHGramRows : N;
  const int nout = m * m;
  // a thread's outputs: i = ti + 16u, j = tj + 16v (u, v < 4)
  const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
  cd acc[4][4];
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) acc[u][v] = {0.0, 0.0};
  for (long long rb = r0; rb < r1; rb += 16) {
    const int nr = (int)((r1 - rb) < 16 ? (r1 - rb) : 16);
    __syncthreads();
    for (int idx = threadIdx.x; idx < 16 * 64; idx += kT) {
      const int rr = idx / 64, c = idx % 64;
      const bool in = rr < nr && c < m;
      st(xs, idx, in ? ld(X, (size_t)(rb + rr) * m + c) : cd{0.0, 0.0});
      st(vs, idx, in ? ld(Vin, (size_t)(rb + rr) * m + c) : cd{0.0, 0.0});
    }
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      cd xv[4], vv[4];
      for (int u = 0; u < 4; ++u) xv[u] = ld(xs, rr * 64 + ti + 16 * u);
      for (int v = 0; v < 4; ++v) vv[v] = ld(vs, rr * 64 + tj + 16 * v);
      for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) acc[u][v] = cadd(acc[u][v], cmulc(xv[u], vv[v]));
    }
  }
  double *out = partial + 2 * (size_t)blockIdx.x * nout;
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) {
      const int i = ti + 16 * u, j = tj + 16 * v;
      if (i < m && j < m) st(out, i * m + j, acc[u][v]);
    }
}

// S = sum of the blocks' partial products: 64 outputs a workgroup, four
// slices of the blocks a output (coalesced rows of the partials), the
// slices added in a fixed order.
__global__ __launch_bounds__(256) void hgram_sum_kernel(const double *partial, int nblk, int m,
                                                        double *S) {
  __shared__ cd red[4][64];
  const int ol = threadIdx.x & 63, slice = threadIdx.x >> 6;
  const int o = blockIdx.x * 64 + ol;
  const size_t mm = (size_t)m * m;
  cd s = {0.0, 0.0};
  if (o < (int)mm)
    for (int k = slice; k < nblk; k += 4) s = cadd(s, ld(partial + 2 * (size_t)k * mm, o));
  red[slice][ol] = s;
  __syncthreads();
  if (slice == 0 && o < (int)mm)
    st(S, o, cadd(cadd(red[0][ol], red[1][ol]), cadd(red[2][ol], red[3][ol])));
}

// G = Hermitian part of S (m x m).
__global__ void hermitian_part_kernel(const double *S, int m, double *G) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= m * m) return;
  const int i = o / m, j = o % m;
  const cd a = ld(S, o), b = ld(S, (size_t)j * m + i);
  st(G, o, {0.5 * (a.r + b.r), 0.5 * (a.i - b.i)});
}

// Real embedding of a Hermitian m x m matrix H = Hr + i Hi:
// E = [[Hr, -Hi], [Hi, Hr]] (2m x 2m, real symmetric); both A_Q and B_Q.
__global__ void hembed_kernel(const double *AQ, const double *BQ, int m, double *EA, double *EB) {
  const int n = 2 * m;
  for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < n * n; o += gridDim.x * blockDim.x) {
    const int r = o / n, c = o % n;
    const int i = r % m, j = c % m;
    const bool top = r < m, left = c < m;
    const size_t k = (size_t)i * m + j;
    const double ar = AQ[2 * k], ai = AQ[2 * k + 1], br = BQ[2 * k], bi = BQ[2 * k + 1];
    const double sa = top == left ? ar : (top ? -ai : ai);
    const double sb = top == left ? br : (top ? -bi : bi);
    EA[o] = sa;
    EB[o] = sb;
  }
}

// Eigenpairs of the embedded pencil come in pairs (lambda, [a; b]) and
// (lambda, [-b; a]); pair j gives eps[j] = eps2[2j] and Phi[:, j] = a + i b
// from the first vector of the pair (Phi2 [2m][2m] row-major).
__global__ void hextract_kernel(const double *eps2, const double *Phi2, int m, double *eps,
                                double *Phi) {
  const int n = 2 * m;
  for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < m * m; o += gridDim.x * blockDim.x) {
    const int r = o / m, j = o % m;
    st(Phi, o, cd{Phi2[(size_t)r * n + 2 * j], Phi2[(size_t)(r + m) * n + 2 * j]});
    if (r == 0) eps[j] = eps2[2 * j];
  }
}

// T[row][j] = sum_i X[row][i] G[i][j] (complex, X [N][m], G [m][m2], m, m2
// <= 64): 64 rows a workgroup, G and the rows staged in LDS (re and im
// planes), a thread computes rows t/16 + 16u and columns t%16 + 16v.
constexpr int kTallRows = 64, kTallLD = 65;
struct TallLds {
  double gr[64 * kTallLD], gi[64 * kTallLD];
  double xr[kTallRows * kTallLD], xi[kTallRows * kTallLD];
};

__global__ __launch_bounds__(256) void htall_gemm_kernel(const double *X, const double *G,
                                                         long long N, int m, int m2, double *T) {
  extern __shared__ double smem_raw[];
  TallLds &s = *reinterpret_cast<TallLds *>(smem_raw);
  const long long r0 = (long long)blockIdx.x * kTallRows;
  const int nr = (int)(N - r0 < kTallRows ? N - r0 : kTallRows);
  for (int o = threadIdx.x; o < m * m2; o += 256) {
    const int k = o / m2, j = o % m2;
    const cd g = ld(G, o);
    s.gr[k * kTallLD + j] = g.r;
    s.gi[k * kTallLD + j] = g.i;
  }
  for (int o = threadIdx.x; o < nr * m; o += 256) {
    const int r = o / m, k = o % m;
    const cd x = ld(X, (size_t)r0 * m + o);
    s.xr[r * kTallLD + k] = x.r;
    s.xi[r * kTallLD + k] = x.i;
  }
  __syncthreads();
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
  cd acc[4][4];
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) acc[u][v] = {0.0, 0.0};
  for (int k = 0; k < m; ++k) {
    cd xv[4], gv[4];
    for (int u = 0; u < 4; ++u) xv[u] = {s.xr[(tr + 16 * u) * kTallLD + k], s.xi[(tr + 16 * u) * kTallLD + k]};
    for (int v = 0; v < 4; ++v) gv[v] = {s.gr[k * kTallLD + tc + 16 * v], s.gi[k * kTallLD + tc + 16 * v]};
    for (int u = 0; u < 4; ++u)
      for (int v = 0; v < 4; ++v) acc[u][v] = cadd(acc[u][v], cmul(xv[u], gv[v]));
  }
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) {
      const int r = tr + 16 * u, j = tc + 16 * v;
      if (r < nr && j < m2) st(T, (size_t)(r0 + r) * m2 + j, acc[u][v]);
    }
}

// Per column j: the 1-norms ||AX_j - lam_j BX_j||, ||AX_j||, ||BX_j|| (complex
// moduli), one workgroup per column, fixed reduction order; then the
// residual of the Table I caption with the small-||Ax|| guard.
constexpr int kResRows = 128;  // rows of one partial sum

// Partial 1-norms over kResRows rows for every column: a thread takes column
// t % 64 of every fourth row (rows read whole), the four row sets added in a
// fixed order; partial[blk][3][m].
__global__ __launch_bounds__(kT) void hresidual_kernel(const double *AX, const double *BX,
                                                       const double *lam, long long N, int m,
                                                       double *partial) {
  __shared__ double red[3][kT];
  const int t = threadIdx.x, j = t & 63, rs = t >> 6;
  const long long r0 = (long long)blockIdx.x * kResRows;
  const long long r1 = r0 + kResRows < N ? r0 + kResRows : N;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (j < m) {
    const double l = lam[j];
    for (long long r = r0 + rs; r < r1; r += kT / 64) {
      const cd a = ld(AX, (size_t)r * m + j), bx = ld(BX, (size_t)r * m + j);
      s0 += hypot(a.r - l * bx.r, a.i - l * bx.i);
      s1 += hypot(a.r, a.i);
      s2 += hypot(bx.r, bx.i);
    }
  }
  red[0][t] = s0;
  red[1][t] = s1;
  red[2][t] = s2;
  __syncthreads();
  if (t < 64 && j < m) {
    double *out = partial + (size_t)blockIdx.x * 3 * m;
    for (int q = 0; q < 3; ++q)
      out[q * m + j] = (red[q][j] + red[q][64 + j]) + (red[q][128 + j] + red[q][192 + j]);
  }
}

// The partials (16 slices of the blocks, added in a fixed order), then the
// residual of the Table I caption with the small-||Ax|| guard.
__global__ __launch_bounds__(1024) void hresidual_sum_kernel(const double *partial, int nblk,
                                                             int m, double emin, double emax,
                                                             double *res) {
  __shared__ double red[3][16][64];
  const int t = threadIdx.x, j = t & 63, sl = t >> 6;
  double s[3] = {0.0, 0.0, 0.0};
  if (j < m)
    for (int k = sl; k < nblk; k += 16)
      for (int q = 0; q < 3; ++q) s[q] += partial[((size_t)k * 3 + q) * m + j];
  for (int q = 0; q < 3; ++q) red[q][sl][j] = s[q];
  __syncthreads();
  if (t >= m) return;
  for (int q = 0; q < 3; ++q) {
    s[q] = 0.0;
    for (int w = 0; w < 16; ++w) s[q] += red[q][w][t];
  }
  const double r = 0.5 * (emax - emin);
  const double scale = fmax(fmax(fabs(emin), fabs(emax)), r);
  const double den = s[1] < r * s[2] ? s[2] * scale : s[1];
  res[t] = s[0] / den;
}

// out[r][j] = in[r][perm[j]] (complex [N][m]).
__global__ void hgather_kernel(const double *in, const int *perm, long long N, int m, double *out) {
  const long long total = N * m;
  for (long long o = blockIdx.x * (long long)blockDim.x + threadIdx.x; o < total;
       o += (long long)gridDim.x * blockDim.x) {
    const long long r = o / m;
    const int j = (int)(o % m);
    st(out, o, ld(in, (size_t)r * m + perm[j]));
  }
}

int grid_of(size_t n) {
  size_t g = (n + 255) / 256;
  return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

// ---- reduced problem A_Q Phi = eps B_Q Phi, complex Hermitian (eqs. 6-9) ----
//
// htridiag_kernel (one workgroup of 1024 threads, m <= 64) brings the
// complex problem to a real symmetric tridiagonal one of size m for the
// real eigensolver (reduced_eig_kernel with B = I):
//  1. B_Q = L L^H (Hermitian part, right-looking Cholesky); a pivot L_kk^2
//     not above 1e-12 B_Q(k, k) stops the kernel with flag[3] = 1 and
//     nothing else written (the caller then takes the real embedding, whose
//     fallback handles a singular B_Q);
//  2. C = L^-1 A_Q L^-H;
//  3. Householder reduction C = Q C3 Q^H, C3 Hermitian tridiagonal:
//     x = C[k+1:, k], alpha = -(x_0 / |x_0|) ||x||, v = x - alpha e_1,
//     H = I - tau v v^H with tau = 2 / ||v||^2, C <- H C H through
//     p = tau C v, w = p - (tau / 2)(v^H p) v, C <- C - v w^H - w v^H;
//  4. D = diag(d), d_0 = 1, d_k+1 = d_k beta_k / |beta_k| (beta_k =
//     C3[k+1][k]) makes T = D^H C3 D real: diagonal Re C3[k][k], off
//     diagonal |beta_k|.
// Outputs: T and I (real [m][m]), Z = L^-H Q D (complex [m][m]); the
// eigenvectors are Phi = Z V_T for T = V_T diag(eps) V_T^T.  Linv:
// 2 (m+1)^2 doubles of scratch.  flag[3] = 0 on success.
constexpr int kRN = 64, kRLD = kRN + 1, kRThreads = 1024;

typedef unsigned int hu32x2 __attribute__((__vector_size__(8)));

// Sums across lanes by DPP row shifts (the whole wave active): after
// row_scan16 lane 16r + 15 holds the sum of row r's sixteen lanes;
// wave_sum adds the four row sums (every lane gets the same value).
template <int CTRL>
__device__ __forceinline__ double dpp_shifted(double v) {
  const auto u = __builtin_bit_cast(hu32x2, v);
  hu32x2 w;
  w[0] = (unsigned)__builtin_amdgcn_update_dpp(0, (int)u[0], CTRL, 0xf, 0xf, true);
  w[1] = (unsigned)__builtin_amdgcn_update_dpp(0, (int)u[1], CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, w);
}

__device__ __forceinline__ double row_scan16(double v) {
  v += dpp_shifted<0x111>(v);  // row_shr:1
  v += dpp_shifted<0x112>(v);  // row_shr:2
  v += dpp_shifted<0x114>(v);  // row_shr:4
  v += dpp_shifted<0x118>(v);  // row_shr:8
  return v;
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  const auto u = __builtin_bit_cast(hu32x2, v);
  hu32x2 w;
  w[0] = (unsigned)__builtin_amdgcn_readlane((int)u[0], lane);
  w[1] = (unsigned)__builtin_amdgcn_readlane((int)u[1], lane);
  return __builtin_bit_cast(double, w);
}

__device__ __forceinline__ double wave_sum(double v) {
  v = row_scan16(v);
  return (lane_value(v, 15) + lane_value(v, 31)) + (lane_value(v, 47) + lane_value(v, 63));
}

struct HTriLds {
  double Cr[kRN * kRLD], Ci[kRN * kRLD];  // C; first L^-1
  double Vr[kRN * kRLD], Vi[kRN * kRLD];  // Q; first B_Q -> L, then A_Q -> A_Q L^-H
  double vr[kRN], vi[kRN];                 // Householder vector
  double pr[kRN], pi[kRN];                 // p
  double qr[kRN], qi[kRN];                 // Q v
  double dr[kRN], di[kRN];                 // D
  double bdiag[kRN];
  double tau, alpha_r, alpha_i, kr, ki;
  int skip;
};

__global__ __launch_bounds__(kRThreads) void htridiag_kernel(const double *AQ, const double *BQ,
                                                             int m, double *T, double *I,
                                                             double *Z, double *Linv, int *flag) {
  extern __shared__ double smem_raw[];
  HTriLds &s = *reinterpret_cast<HTriLds *>(smem_raw);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n2 = m + (m & 1), np = n2 / 2;
  double *Cr = s.Cr, *Ci = s.Ci, *Vr = s.Vr, *Vi = s.Vi;
  auto at = [](int i, int j) { return i * kRLD + j; };
  // Hermitian part of B_Q, identity padding
  for (int o = tid; o < n2 * n2; o += kRThreads) {
    const int i = o / n2, j = o % n2;
    double re = i == j ? 1.0 : 0.0, im = 0.0;
    if (i < m && j < m) {
      const cd a = ld(BQ, (size_t)i * m + j), b = ld(BQ, (size_t)j * m + i);
      re = 0.5 * (a.r + b.r);
      im = 0.5 * (a.i - b.i);
    }
    Vr[at(i, j)] = re;
    Vi[at(i, j)] = im;
    if (i == j) s.bdiag[i] = re;
  }
  __syncthreads();
  // 1. Cholesky (lower triangle of V)
  bool fail = false;
  for (int k = 0; k < n2; ++k) {
    const double d = Vr[at(k, k)];
    if (!(d > 1e-12 * s.bdiag[k]) || !isfinite(d)) {  // same values in every thread
      fail = true;
      break;
    }
    const double lkk = sqrt(d), inv = 1.0 / lkk;
    __syncthreads();
    if (tid == 0) {
      Vr[at(k, k)] = lkk;
      Vi[at(k, k)] = 0.0;
    }
    for (int i = k + 1 + tid; i < n2; i += kRThreads) {
      Vr[at(i, k)] *= inv;
      Vi[at(i, k)] *= inv;
    }
    __syncthreads();
    {  // 16 threads a row of the trailing lower triangle
      const int i = k + 1 + (tid >> 4);
      if (i < n2) {
        const double lr = Vr[at(i, k)], li = Vi[at(i, k)];
        for (int j = k + 1 + (tid & 15); j <= i; j += 16) {
          const double jr = Vr[at(j, k)], ji = Vi[at(j, k)];
          Vr[at(i, j)] -= lr * jr + li * ji;  // L_ik conj(L_jk)
          Vi[at(i, j)] -= li * jr - lr * ji;
        }
      }
    }
    __syncthreads();
  }
  if (fail) {
    if (tid == 0) flag[3] = 1;
    return;
  }
  // 2. L^-1 (lower) into C row by row (16 threads a column); a copy to global
  for (int i = 0; i < n2; ++i) {
    const int j = tid >> 4, part = tid & 15;
    double sr = 0.0, si = 0.0;
    if (j < i)
      for (int k = j + part; k < i; k += 16) {
        const double lr = Vr[at(i, k)], li = Vi[at(i, k)], xr = Cr[at(k, j)], xi = Ci[at(k, j)];
        sr += lr * xr - li * xi;
        si += lr * xi + li * xr;
      }
    sr = row_scan16(sr);  // the column's sum in its last lane
    si = row_scan16(si);
    if (part == 15 && j < n2) {
      const double inv = 1.0 / Vr[at(i, i)];
      Cr[at(i, j)] = j < i ? -sr * inv : (j == i ? inv : 0.0);
      Ci[at(i, j)] = j < i ? -si * inv : 0.0;
    }
    __syncthreads();
  }
  for (int o = tid; o < n2 * n2; o += kRThreads) {
    const int i = o / n2, j = o % n2;
    Linv[2 * o] = Cr[at(i, j)];
    Linv[2 * o + 1] = Ci[at(i, j)];
    double re = 0.0, im = 0.0;  // Hermitian part of A_Q into V (zero padding)
    if (i < m && j < m) {
      const cd a = ld(AQ, (size_t)i * m + j), b = ld(AQ, (size_t)j * m + i);
      re = 0.5 * (a.r + b.r);
      im = 0.5 * (a.i - b.i);
    }
    Vr[at(i, j)] = re;
    Vi[at(i, j)] = im;
  }
  __syncthreads();
  // A_Q L^-H, then C = L^-1 (A_Q L^-H): 2 x 2 output blocks a thread
  const bool blk = (tid >> 5) < np && (tid & 31) < np;
  const int r0 = 2 * (tid >> 5), c0 = 2 * (tid & 31);
  cd acc[2][2];
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) acc[u][v] = {0.0, 0.0};
  if (blk)
    for (int k = 0; k < n2; ++k)
      for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
          const cd a = {Vr[at(r0 + u, k)], Vi[at(r0 + u, k)]};
          const cd l = {Cr[at(c0 + v, k)], Ci[at(c0 + v, k)]};  // conj(L^-1[c][k]) below
          acc[u][v] = cadd(acc[u][v], {a.r * l.r + a.i * l.i, a.i * l.r - a.r * l.i});
        }
  __syncthreads();
  if (blk)
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) {
        Vr[at(r0 + u, c0 + v)] = acc[u][v].r;
        Vi[at(r0 + u, c0 + v)] = acc[u][v].i;
        acc[u][v] = {0.0, 0.0};
      }
  __syncthreads();
  if (blk)
    for (int k = 0; k < n2; ++k)
      for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
          const cd l = {Cr[at(r0 + u, k)], Ci[at(r0 + u, k)]};
          const cd t = {Vr[at(k, c0 + v)], Vi[at(k, c0 + v)]};
          acc[u][v] = cadd(acc[u][v], cmul(l, t));
        }
  __syncthreads();
  if (blk)
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) {
        Cr[at(r0 + u, c0 + v)] = acc[u][v].r;
        Ci[at(r0 + u, c0 + v)] = acc[u][v].i;
      }
  __syncthreads();
  // Hermitian part of C; Q = I
  if (blk)
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) {
        const int i = r0 + u, j = c0 + v;
        acc[u][v] = {0.5 * (Cr[at(i, j)] + Cr[at(j, i)]), 0.5 * (Ci[at(i, j)] - Ci[at(j, i)])};
      }
  __syncthreads();
  if (blk)
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) {
        const int i = r0 + u, j = c0 + v;
        Cr[at(i, j)] = acc[u][v].r;
        Ci[at(i, j)] = acc[u][v].i;
        Vr[at(i, j)] = i == j ? 1.0 : 0.0;
        Vi[at(i, j)] = 0.0;
      }
  __syncthreads();
  // 3. Householder reduction of the leading m x m block
  for (int k = 0; k + 2 < m; ++k) {
    const int n1 = m - k - 1;  // length of x
    if (wv == 0) {
      double xr = 0.0, xi = 0.0;
      if (lane < n1) {
        xr = Cr[at(k + 1 + lane, k)];
        xi = Ci[at(k + 1 + lane, k)];
      }
      const double nx2 = wave_sum(xr * xr + xi * xi);
      const double x0r = Cr[at(k + 1, k)], x0i = Ci[at(k + 1, k)];
      const double nx = sqrt(nx2), a0 = sqrt(x0r * x0r + x0i * x0i);
      const double phr = a0 > 0.0 ? x0r / a0 : 1.0, phi = a0 > 0.0 ? x0i / a0 : 0.0;
      const double alr = -phr * nx, ali = -phi * nx;
      // ||v||^2 = ||x||^2 - |x_0|^2 + (|x_0| + ||x||)^2
      const double vn2 = 2.0 * nx * (nx + a0);
      s.vr[lane] = lane == 0 ? xr - alr : xr;
      s.vi[lane] = lane == 0 ? xi - ali : xi;
      if (lane == 0) {
        s.skip = !(vn2 > 0.0);
        s.tau = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
        s.alpha_r = alr;
        s.alpha_i = ali;
      }
    }
    __syncthreads();
    if (s.skip) {  // uniform: x = 0, nothing to reduce
      __syncthreads();
      continue;
    }
    const double tau = s.tau;
    // p = tau C_sub v (rows < n1) and q = Q_sub v (rows < m): 16 threads a row
    {
      const int row = tid >> 4, part = tid & 15;
      for (int pass = 0; pass < 2; ++pass) {
        const int rr = row + 64 * pass;  // 0..n1-1: p, n1..n1+m-1: q
        const bool isp = rr < n1, isq = !isp && rr - n1 < m;
        double sr = 0.0, si = 0.0;
        if (isp || isq) {
          const int i = isp ? k + 1 + rr : rr - n1;
          const double *Mr = isp ? Cr : Vr, *Mi = isp ? Ci : Vi;
          for (int j = part; j < n1; j += 16) {
            const double mr = Mr[at(i, k + 1 + j)], mi = Mi[at(i, k + 1 + j)];
            sr += mr * s.vr[j] - mi * s.vi[j];
            si += mr * s.vi[j] + mi * s.vr[j];
          }
        }
        sr = row_scan16(sr);  // the row's sum in its last lane
        si = row_scan16(si);
        if (part == 15) {
          if (isp) {
            s.pr[rr] = tau * sr;
            s.pi[rr] = tau * si;
          } else if (isq) {
            s.qr[rr - n1] = sr;
            s.qi[rr - n1] = si;
          }
        }
      }
    }
    __syncthreads();
    if (wv == 0) {  // K = (tau / 2) v^H p
      double kr = 0.0, ki = 0.0;
      if (lane < n1) {
        kr = s.vr[lane] * s.pr[lane] + s.vi[lane] * s.pi[lane];
        ki = s.vr[lane] * s.pi[lane] - s.vi[lane] * s.pr[lane];
      }
      kr = wave_sum(kr);
      ki = wave_sum(ki);
      if (lane == 0) {
        s.kr = 0.5 * tau * kr;
        s.ki = 0.5 * tau * ki;
      }
    }
    __syncthreads();
    // C_sub -= v w^H + w v^H with w = p - K v; column and row k; Q_sub -= tau q v^H
    {
      const double kr = s.kr, ki = s.ki;
      const int i = tid >> 4;
      if (i < n1) {
        const double vir = s.vr[i], vii = s.vi[i];
        const double wir = s.pr[i] - (kr * vir - ki * vii), wii = s.pi[i] - (kr * vii + ki * vir);
        for (int j = tid & 15; j < n1; j += 16) {
          const double vjr = s.vr[j], vji = s.vi[j];
          const double wjr = s.pr[j] - (kr * vjr - ki * vji), wji = s.pi[j] - (kr * vji + ki * vjr);
          // v_i conj(w_j) + w_i conj(v_j)
          const double ur = vir * wjr + vii * wji + wir * vjr + wii * vji;
          const double ui = vii * wjr - vir * wji + wii * vjr - wir * vji;
          Cr[at(k + 1 + i, k + 1 + j)] -= ur;
          Ci[at(k + 1 + i, k + 1 + j)] -= ui;
        }
      }
      if (i < m) {
        const double qr = tau * s.qr[i], qi = tau * s.qi[i];
        for (int j = tid & 15; j < n1; j += 16) {
          const double vjr = s.vr[j], vji = s.vi[j];
          Vr[at(i, k + 1 + j)] -= qr * vjr + qi * vji;  // tau q_i conj(v_j)
          Vi[at(i, k + 1 + j)] -= qi * vjr - qr * vji;
        }
      }
    }
    if (tid < n1) {
      const double ar = tid == 0 ? s.alpha_r : 0.0, ai = tid == 0 ? s.alpha_i : 0.0;
      Cr[at(k + 1 + tid, k)] = ar;
      Ci[at(k + 1 + tid, k)] = ai;
      Cr[at(k, k + 1 + tid)] = ar;
      Ci[at(k, k + 1 + tid)] = -ai;
    }
    __syncthreads();
  }
  // 4. D, T, I, Z = L^-H Q D
  if (tid == 0) {
    double dr = 1.0, di = 0.0;
    s.dr[0] = 1.0;
    s.di[0] = 0.0;
    for (int k = 0; k + 1 < m; ++k) {
      const double br = Cr[at(k + 1, k)], bi = Ci[at(k + 1, k)];
      const double ab = sqrt(br * br + bi * bi);
      if (ab > 0.0) {
        const double er = br / ab, ei = bi / ab;
        const double nr = dr * er - di * ei, ni = dr * ei + di * er;
        dr = nr;
        di = ni;
      }
      s.dr[k + 1] = dr;
      s.di[k + 1] = di;
    }
  }
  for (int o = tid; o < m * m; o += kRThreads) {
    const int i = o / m, j = o % m;
    double t = 0.0;
    if (i == j) t = Cr[at(i, i)];
    else if (i == j + 1 || j == i + 1) {
      const int hi = i > j ? i : j, lo = i > j ? j : i;
      const double br = Cr[at(hi, lo)], bi = Ci[at(hi, lo)];
      t = sqrt(br * br + bi * bi);
    }
    T[o] = t;
    I[o] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int o = tid; o < n2 * n2; o += kRThreads) {  // L^-1 back into C
    const int i = o / n2, j = o % n2;
    Cr[at(i, j)] = Linv[2 * o];
    Ci[at(i, j)] = Linv[2 * o + 1];
  }
  __syncthreads();
  if (blk) {
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) acc[u][v] = {0.0, 0.0};
    for (int k = 0; k < n2; ++k)
      for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
          const cd l = {Cr[at(k, r0 + u)], Ci[at(k, r0 + u)]};  // conj(L^-1[k][r]) below
          const cd x = {Vr[at(k, c0 + v)], Vi[at(k, c0 + v)]};
          acc[u][v] = cadd(acc[u][v], cmulc(l, x));
        }
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) {
        const int i = r0 + u, j = c0 + v;
        if (i < m && j < m) st(Z, (size_t)i * m + j, cmul(acc[u][v], {s.dr[j], s.di[j]}));
      }
  }
  if (tid == 0) flag[3] = 0;
}

// Phi[r][j] = sum_k Z[r][k] VT[k][j] (Z complex, VT real, [m][m]).
__global__ void hcombine_kernel(const double *Z, const double *VT, int m, double *Phi) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= m * m) return;
  const int r = o / m, j = o % m;
  cd acc = {0.0, 0.0};
  for (int k = 0; k < m; ++k) {
    const cd z = ld(Z, (size_t)r * m + k);
    const double v = VT[(size_t)k * m + j];
    acc = {acc.r + z.r * v, acc.i + z.i * v};
  }
  st(Phi, o, acc);
}

}  // namespace

size_t hfactor_lds_bytes(int b) { return 2 * (size_t)b * (b + 1) * sizeof(double); }

hipError_t launch_hfactor(const HPencil &p, const Shifts &s, int Ne, double *Sinv, double *W,
                          double *V, int parts, double *work, hipStream_t st) {
  if (p.b < 1 || p.b > kMaxHBlock) return hipErrorInvalidValue;
  if (p.b <= 64) return launch_hfactor_mfma(p, s, Ne, Sinv, W, V, parts, work, st);
  const size_t lds = hfactor_lds_bytes(p.b);
  hipError_t e = hipFuncSetAttribute((const void *)hfactor_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)hfactor_lds_bytes(kMaxHBlock));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hfactor_kernel, dim3(Ne), dim3(kT), lds, st, p, s, Sinv, W, V);
  return hipGetLastError();
}

hipError_t launch_hsweeps(const HPencil &p, int Ne, const double *Sinv, const double *W,
                          const double *V, const double *R, int m, double *G, hipStream_t st) {
  if (p.b > kMaxHBlock || m < 1) return hipErrorInvalidValue;
  if (p.b <= 64) return launch_hsweeps_mfma(p, Ne, Sinv, W, V, R, m, G, st);
  dim3 grid(Ne, 2, (m + kCols - 1) / kCols);
  hipLaunchKernelGGL(hsweep_kernel, grid, dim3(kT), 0, st, p, Sinv, W, V, R, m, G);
  return hipGetLastError();
}

hipError_t launch_haccumulate(const double *G, int Ne, size_t Nm, const double *cre,
                              const double *cim, double *Q, hipStream_t st) {
  hipLaunchKernelGGL(haccumulate_kernel, dim3(grid_of(Nm)), dim3(256), 0, st, G, Ne, Nm, cre, cim, Q);
  return hipGetLastError();
}

hipError_t launch_happly_pair(const HPencil &p, const double *Vin, int m, double *outA,
                              double *outB, hipStream_t st) {
  if (p.b <= 64) return launch_happly_mfma(p, 2, Vin, m, outA, st, outB);
  hipError_t e = launch_happly(p, 0, Vin, m, outA, st);
  return e == hipSuccess ? launch_happly(p, 1, Vin, m, outB, st) : e;
}

hipError_t launch_happly(const HPencil &p, int which, const double *Vin, int m, double *out,
                         hipStream_t st) {
  if (p.b <= 64) return launch_happly_mfma(p, which, Vin, m, out, st);
  hipLaunchKernelGGL(happly_kernel, dim3(grid_of((size_t)p.nc * p.b * m)), dim3(256), 0, st, p,
                     which, Vin, m, out);
  return hipGetLastError();
}

// The projection's block partials and their sum, or the residuals' partial
// 1-norms, whichever is larger.
size_t hgram_partial_doubles(long long N, int m) {
  const size_t gram = 2 * (size_t)((N + kHGramRows - 1) / kHGramRows + 1) * m * m;
  const size_t resid = 3 * (size_t)m * ((N + kResRows - 1) / kResRows);
  return gram > resid ? gram : resid;
}

hipError_t launch_hgram(const double *X, const double *Vin, long long N, int m, double *partial,
                        double *G, hipStream_t st) {
  if (m < 1 || m > 64) return hipErrorInvalidValue;
  const int nblk = (int)((N + kHGramRows - 1) / kHGramRows);
  hipLaunchKernelGGL(hgram_kernel, dim3(nblk), dim3(kT), 0, st, X, Vin, N, m, partial);
  double *sum = partial + 2 * (size_t)nblk * m * m;
  hipLaunchKernelGGL(hgram_sum_kernel, dim3((m * m + 63) / 64), dim3(256), 0, st, partial, nblk, m,
                     sum);
  hipLaunchKernelGGL(hermitian_part_kernel, dim3((m * m + 255) / 256), dim3(256), 0, st,
                     (const double *)sum, m, G);
  return hipGetLastError();
}

hipError_t launch_hembed(const double *AQ, const double *BQ, int m, double *EA, double *EB,
                         hipStream_t st) {
  hipLaunchKernelGGL(hembed_kernel, dim3(grid_of((size_t)4 * m * m)), dim3(256), 0, st, AQ, BQ, m,
                     EA, EB);
  return hipGetLastError();
}

hipError_t launch_htridiag(const double *AQ, const double *BQ, int m, double *T, double *I,
                           double *Z, double *scratch, int *flag, hipStream_t st) {
  if (m < 1 || m > kRN) return hipErrorInvalidValue;
  const int shm = (int)sizeof(HTriLds);
  hipError_t e = hipFuncSetAttribute((const void *)htridiag_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(htridiag_kernel, dim3(1), dim3(kRThreads), shm, st, AQ, BQ, m, T, I, Z,
                     scratch, flag);
  return hipGetLastError();
}

hipError_t launch_hcombine(const double *Z, const double *VT, int m, double *Phi, hipStream_t st) {
  hipLaunchKernelGGL(hcombine_kernel, dim3((m * m + 255) / 256), dim3(256), 0, st, Z, VT, m, Phi);
  return hipGetLastError();
}

hipError_t launch_hextract(const double *eps2, const double *Phi2, int m, double *eps,
                           double *Phi, hipStream_t st) {
  hipLaunchKernelGGL(hextract_kernel, dim3(grid_of((size_t)m * m)), dim3(256), 0, st, eps2, Phi2,
                     m, eps, Phi);
  return hipGetLastError();
}

hipError_t launch_htall_gemm(const double *X, const double *G, long long N, int m, int m2,
                             double *T, hipStream_t st) {
  if (m < 1 || m > 64 || m2 < 1 || m2 > 64) return hipErrorInvalidValue;
  const int shm = (int)sizeof(TallLds);
  hipError_t e = hipFuncSetAttribute((const void *)htall_gemm_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, shm);
  if (e != hipSuccess) return e;
  const long long nblk = (N + kTallRows - 1) / kTallRows;
  hipLaunchKernelGGL(htall_gemm_kernel, dim3((unsigned)nblk), dim3(256), shm, st, X, G, N, m, m2,
                     T);
  return hipGetLastError();
}

hipError_t launch_hresiduals(const double *AX, const double *BX, const double *lam, long long N,
                             int m, double emin, double emax, double *partial, double *res,
                             hipStream_t st) {
  if (m < 1 || m > 64) return hipErrorInvalidValue;
  const int nblk = (int)((N + kResRows - 1) / kResRows);
  hipLaunchKernelGGL(hresidual_kernel, dim3(nblk), dim3(kT), 0, st, AX, BX, lam, N, m, partial);
  hipLaunchKernelGGL(hresidual_sum_kernel, dim3(1), dim3(1024), 0, st, (const double *)partial,
                     nblk, m, emin, emax, res);
  return hipGetLastError();
}

hipError_t launch_hgather(const double *in, const int *perm, long long N, int m, double *out,
                          hipStream_t st) {
  hipLaunchKernelGGL(hgather_kernel, dim3(grid_of((size_t)N * m)), dim3(256), 0, st, in, perm, N,
                     m, out);
  return hipGetLastError();
}

}  // namespace feast
