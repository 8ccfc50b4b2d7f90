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

// out[c] = D_c V_c + U_c V_{c+1} + U_{c-1}^T V_{c-1}; one wave per 16 rows
// and 16 columns of a cell.
template <int BP>
__global__ __launch_bounds__(BP * 4) void bt_multiply_kernel(const double *D, const double *U,
                                                             int nc, int b, const double *V,
                                                             int ld, double *out) {
  const int c = blockIdx.x, jt = blockIdx.y;
  const int l = lane_id(), w = wave_id();
  const int row = w * 16 + (l & 15);
  const int kl = l >> 4;
  const int col = jt * 16 + (l & 15);
  const size_t bb = (size_t)b * b;
  d4 acc0 = d4zero(), acc1 = d4zero();
  auto vrow = [&](int cell, int k) { return V[((size_t)cell * BP + k) * ld + col]; };
  {
    const double *Dc = D + c * bb;
    for (int k0 = 0; k0 < BP; k0 += 4) {
      const int k = k0 + kl;
      double a = (row < b && k < b) ? Dc[k * b + row] : 0.0;  // symmetric block
      acc0 = mfma(a, vrow(c, k), acc0);
    }
  }
  if (c + 1 < nc) {
    const double *Uc = U + c * bb;
    for (int k0 = 0; k0 < BP; k0 += 4) {
      const int k = k0 + kl;
      double a = (row < b && k < b) ? Uc[row * b + k] : 0.0;
      acc1 = mfma(a, vrow(c + 1, k), acc1);
    }
  }
  if (c > 0) {
    const double *Up = U + (c - 1) * bb;
    for (int k0 = 0; k0 < BP; k0 += 4) {
      const int k = k0 + kl;
      double a = (row < b && k < b) ? Up[k * b + row] : 0.0;
      acc0 = mfma(a, vrow(c - 1, k), acc0);
    }
  }
  d4 acc = acc0 + acc1;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int orow = w * 16 + acc_row(l, r);
    out[((size_t)c * BP + orow) * ld + jt * 16 + acc_col(l)] = acc[r];
  }
}

__global__ void sum_nodes_kernel(const double *P, int Ne, size_t count, double *Q) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int e = 0; e < Ne; ++e) s += P[(size_t)e * count + i];
    Q[i] = s;
  }
}

constexpr int kGramRows = 1024;  // rows per workgroup (256 per wave)

// partial[z][chunk] = Q(chunk rows)^T V_z(chunk rows), one 16x16 tile per
// workgroup; the four waves split the rows and are summed in wave order.
__global__ __launch_bounds__(256) void gram_kernel(const double *Q, const double *V1,
                                                   const double *V2, size_t rows, int m0p,
                                                   double *partial) {
  __shared__ double red[4][64][4];
  const int chunk = blockIdx.x;
  const int ntj = m0p / 16;
  const int ti = blockIdx.y / ntj, tj = blockIdx.y % ntj;
  const int z = blockIdx.z;
  const double *V = z ? V2 : V1;
  const int l = lane_id(), w = wave_id();
  const int kl = l >> 4;
  const size_t r0 = (size_t)chunk * kGramRows + (size_t)w * (kGramRows / 4);
  size_t r1 = r0 + kGramRows / 4;
  if (r1 > rows) r1 = rows;
  d4 acc0 = d4zero(), acc1 = d4zero();
  const int ci = ti * 16 + (l & 15), cj = tj * 16 + (l & 15);
  size_t r = r0;
  for (; r + 8 <= r1; r += 8) {
    const size_t ra = r + kl, rb = r + 4 + kl;
    acc0 = mfma(Q[ra * m0p + ci], V[ra * m0p + cj], acc0);
    acc1 = mfma(Q[rb * m0p + ci], V[rb * m0p + cj], acc1);
  }
  for (; r < r1; r += 4) {  // rows is a multiple of 16, so r1 - r is a multiple of 4
    const size_t ra = r + kl;
    acc0 = mfma(Q[ra * m0p + ci], V[ra * m0p + cj], acc0);
  }
  d4 acc = acc0 + acc1;
#pragma unroll
  for (int q = 0; q < 4; ++q) red[w][l][q] = acc[q];
  __syncthreads();
  if (w == 0) {
    const size_t nchunks = gridDim.x;
    double *out = partial + ((size_t)z * nchunks + chunk) * m0p * m0p;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double s = red[0][l][q] + red[1][l][q] + red[2][l][q] + red[3][l][q];
      out[(size_t)(ti * 16 + acc_row(l, q)) * m0p + tj * 16 + acc_col(l)] = s;
    }
  }
}

__global__ void gram_reduce_kernel(const double *partial, int nchunks, int m0p, int m0,
                                   double *G1, double *G2) {
  const int z = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m0 * m0) return;
  const int i = idx / m0, j = idx % m0;
  const double *p = partial + (size_t)z * nchunks * m0p * m0p;
  double s1 = 0.0, s2 = 0.0;
  for (int c = 0; c < nchunks; ++c) {
    s1 += p[((size_t)c * m0p + i) * m0p + j];
    s2 += p[((size_t)c * m0p + j) * m0p + i];
  }
  (z ? G2 : G1)[idx] = 0.5 * (s1 + s2);
}

// X[row][j] = sum_{k<m0} Q[row][k] Phi[k][j]; columns m0..m0p-1 are zero.
__global__ __launch_bounds__(256) void gemm_qphi_kernel(const double *Q, size_t rows, int m0p,
                                                        int m0, const double *Phi, double *X) {
  const int l = lane_id(), w = wave_id();
  const size_t rbase = (size_t)blockIdx.x * 64 + w * 16;
  if (rbase >= rows) return;
  const int jt = blockIdx.y;
  const int kl = l >> 4;
  const size_t row = rbase + (l & 15);
  const int col = jt * 16 + (l & 15);
  d4 acc0 = d4zero(), acc1 = d4zero();
  int k0 = 0;
  for (; k0 + 8 <= m0p; k0 += 8) {
    const int ka = k0 + kl, kb = k0 + 4 + kl;
    double a0 = Q[row * m0p + ka], a1 = Q[row * m0p + kb];
    double b0 = (ka < m0 && col < m0) ? Phi[(size_t)ka * m0 + col] : 0.0;
    double b1 = (kb < m0 && col < m0) ? Phi[(size_t)kb * m0 + col] : 0.0;
    acc0 = mfma(a0, b0, acc0);
    acc1 = mfma(a1, b1, acc1);
  }
  for (; k0 < m0p; k0 += 4) {
    const int ka = k0 + kl;
    double a0 = Q[row * m0p + ka];
    double b0 = (ka < m0 && col < m0) ? Phi[(size_t)ka * m0 + col] : 0.0;
    acc0 = mfma(a0, b0, acc0);
  }
  d4 acc = acc0 + acc1;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    X[(rbase + acc_row(l, r)) * m0p + jt * 16 + acc_col(l)] = acc[r];
}

constexpr int kResRows = 2048;

__global__ __launch_bounds__(256) void residual_kernel(const double *AX, const double *BX,
                                                       const double *lam, size_t rows, int m0p,
                                                       int m0, double *partial) {
  __shared__ double red[3][4][64];
  const int chunk = blockIdx.x;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int j = blockIdx.y * 64 + tx;
  double num = 0.0, na = 0.0, nb = 0.0;
  if (j < m0) {
    const double lj = lam[j];
    const size_t r0 = (size_t)chunk * kResRows;
    size_t r1 = r0 + kResRows;
    if (r1 > rows) r1 = rows;
    for (size_t r = r0 + ty; r < r1; r += 4) {
      const double ax = AX[r * m0p + j], bx = BX[r * m0p + j];
      num += fabs(ax - lj * bx);
      na += fabs(ax);
      nb += fabs(bx);
    }
  }
  red[0][ty][tx] = num;
  red[1][ty][tx] = na;
  red[2][ty][tx] = nb;
  __syncthreads();
  if (ty == 0 && j < m0p) {
    double *out = partial + (size_t)chunk * 3 * m0p;
#pragma unroll
    for (int q = 0; q < 3; ++q)
      out[q * m0p + j] = red[q][0][tx] + red[q][1][tx] + red[q][2][tx] + red[q][3][tx];
  }
}

__global__ void residual_reduce_kernel(const double *partial, int nchunks, int m0p, int m0,
                                       double emin, double emax, double *res) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m0) return;
  double num = 0.0, na = 0.0, nb = 0.0;
  for (int c = 0; c < nchunks; ++c) {
    const double *p = partial + (size_t)c * 3 * m0p;
    num += p[j];
    na += p[m0p + j];
    nb += p[2 * m0p + j];
  }
  const double r = 0.5 * (emax - emin);
  const double big = fmax(fmax(fabs(emin), fabs(emax)), r);
  const double den = (na < r * nb) ? nb * big : na;
  res[j] = num / den;
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

hipError_t launch_bt_multiply(const Pencil &p, int which, const double *V, int ld, double *out,
                              hipStream_t st) {
  const double *D = which ? p.Bd : p.Ad;
  const double *U = which ? p.Bu : p.Au;
  dim3 grid(p.nc, ld / 16);
  switch (p.bp) {
    case 16: hipLaunchKernelGGL(bt_multiply_kernel<16>, grid, dim3(64), 0, st, D, U, p.nc, p.b, V, ld, out); break;
    case 32: hipLaunchKernelGGL(bt_multiply_kernel<32>, grid, dim3(128), 0, st, D, U, p.nc, p.b, V, ld, out); break;
    case 48: hipLaunchKernelGGL(bt_multiply_kernel<48>, grid, dim3(192), 0, st, D, U, p.nc, p.b, V, ld, out); break;
    case 64: hipLaunchKernelGGL(bt_multiply_kernel<64>, grid, dim3(256), 0, st, D, U, p.nc, p.b, V, ld, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sum_nodes(const double *P, int Ne, size_t count, double *Q, hipStream_t st) {
  hipLaunchKernelGGL(sum_nodes_kernel, dim3(grid_for(count, 256)), dim3(256), 0, st, P, Ne, count,
                     Q);
  return hipGetLastError();
}

size_t gram_partial_doubles(size_t rows, int m0p) {
  size_t nchunks = (rows + kGramRows - 1) / kGramRows;
  return 2 * nchunks * (size_t)m0p * m0p;
}

hipError_t launch_gram2(const double *Q, const double *V1, const double *V2, size_t rows, int m0p,
                        int m0, double *partial, double *G1, double *G2, hipStream_t st) {
  const int nchunks = (int)((rows + kGramRows - 1) / kGramRows);
  const int nt = m0p / 16;
  hipLaunchKernelGGL(gram_kernel, dim3(nchunks, nt * nt, 2), dim3(256), 0, st, Q, V1, V2, rows,
                     m0p, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((m0 * m0 + 255) / 256, 2), dim3(256), 0, st,
                     partial, nchunks, m0p, m0, G1, G2);
  return hipGetLastError();
}

hipError_t launch_gemm_qphi(const double *Q, size_t rows, int m0p, int m0, const double *Phi,
                            double *X, hipStream_t st) {
  dim3 grid((unsigned)((rows + 63) / 64), m0p / 16);
  hipLaunchKernelGGL(gemm_qphi_kernel, grid, dim3(256), 0, st, Q, rows, m0p, m0, Phi, X);
  return hipGetLastError();
}

size_t residual_partial_doubles(size_t rows, int m0p) {
  return ((rows + kResRows - 1) / kResRows) * 3 * (size_t)m0p;
}

hipError_t launch_residuals(const double *AX, const double *BX, const double *lam, size_t rows,
                            int m0p, int m0, double emin, double emax, double *partial,
                            double *res, hipStream_t st) {
  const int nchunks = (int)((rows + kResRows - 1) / kResRows);
  hipLaunchKernelGGL(residual_kernel, dim3(nchunks, (m0p + 63) / 64), dim3(256), 0, st, AX, BX,
                     lam, rows, m0p, m0, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(residual_reduce_kernel, dim3((m0 + 127) / 128), dim3(128), 0, st, partial,
                     nchunks, m0p, m0, emin, emax, res);
  return hipGetLastError();
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

}  // namespace feast
