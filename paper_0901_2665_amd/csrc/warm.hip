// Learned warm start for a parameterised Hamiltonian family (the project's
// extension built on the subspace reuse of Sec. IV.C, Example III, where
// nearby problems start from a previous solution): kernels of the network
// that maps the family parameters to a start subspace Y, and the float64
// kernels that turn FEAST solutions into its training targets.
//
// Network: MLP d0 -> d1 -> d2 -> d3 with ReLU after the two hidden layers.
// Every product runs on the matrix cores in bfloat16 with float32
// accumulation (V_MFMA_F32_16X16X16_BF16): operands are rounded to bfloat16
// (round to nearest even), sums are float32.  Master weights, Adam moments
// and gradients are float32.
//
// Targets: for a member of the family with converged B-orthonormal
// eigenvectors X_in (the counted pairs) and a fixed start block Y_ref,
// T = X_in X_in^T B Y_ref (the first contour integration of an exact
// filter: gauge-free, unlike X_in itself).  Per cell c the rows T_c (b x m)
// are represented in a basis U_c (b x r) taken from the leading
// eigenvectors of sum_s T_c,s T_c,s^T over the training set:
// C_c = U_c^T T_c, and a start block is Y_c = U_c C_c.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace feast {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kGemmTile = 64;  // output tile of one workgroup (4 waves of 32 x 32)

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// C_partial[z][M][N] = sum over k in split z of A[m][k] B[n][k]; A [M][K] and
// B [N][K] bfloat16 row-major (k contiguous), K a multiple of 16.  Lane l of
// a 16x16x16 product holds A row l%16, k = 4(l/16)..+3 (likewise B), and
// accumulator element q at row 4(l/16)+q, column l%16.
__global__ __launch_bounds__(256) void gemm_nt_kernel(const uint16_t *A, const uint16_t *B, int M,
                                                      int N, int K, int kc, float *P) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int m0 = blockIdx.y * kGemmTile + (w >> 1) * 32;
  const int n0 = blockIdx.x * kGemmTile + (w & 1) * 32;
  const int kbeg = blockIdx.z * kc;
  const int kend = min(K, kbeg + kc);
  const int r = l & 15, kq = (l >> 4) * 4;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x4 zero = bf16x4{0, 0, 0, 0};
  for (int k = kbeg; k < kend; k += 16) {
    bf16x4 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = m0 + 16 * i + r;
      a[i] = row < M ? *reinterpret_cast<const bf16x4 *>(A + (size_t)row * K + k + kq) : zero;
      const int col = n0 + 16 * i + r;
      b[i] = col < N ? *reinterpret_cast<const bf16x4 *>(B + (size_t)col * K + k + kq) : zero;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
  }
  float *out = P + (size_t)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + 16 * j + r;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + 16 * i + kq + q;
        if (row < M && col < N) out[(size_t)row * N + col] = acc[i][j][q];
      }
    }
}

// Sum of the split partials in split order, then bias, ReLU or the ReLU
// derivative mask (mask[m][n] > 0 as bfloat16), and the requested outputs:
// float32 [M][N], bfloat16 [M][N], bfloat16 transposed [N][M].
__global__ void finish_kernel(const float *P, int splits, int M, int N, const float *bias,
                              int relu, const uint16_t *mask, float *outf, uint16_t *outb,
                              uint16_t *outbt) {
  const size_t total = (size_t)M * N;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    float s = P[i];
    for (int z = 1; z < splits; ++z) s += P[(size_t)z * total + i];
    const int m = (int)(i / N), n = (int)(i % N);
    if (bias) s += bias[n];
    if (relu) s = s > 0.f ? s : 0.f;
    if (mask && !(from_bf16(mask[i]) > 0.f)) s = 0.f;
    if (outf) outf[i] = s;
    const uint16_t h = to_bf16(s);
    if (outb) outb[i] = h;
    if (outbt) outbt[(size_t)n * M + m] = h;
  }
}

// bfloat16 copies of a float32 [M][N] matrix: row-major and transposed.
__global__ void cast_kernel(const float *x, int M, int N, uint16_t *xb, uint16_t *xbt) {
  const size_t total = (size_t)M * N;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const uint16_t h = to_bf16(x[i]);
    if (xb) xb[i] = h;
    if (xbt) xbt[(i % N) * M + i / N] = h;
  }
}

// Mean squared error of y against t over M x N entries: dy = 2 (y - t) / (M N)
// (float32, bfloat16, bfloat16 transposed) and per-block partial sums of
// (y - t)^2 in float64.
__global__ __launch_bounds__(256) void mse_kernel(const float *y, const float *t, int M, int N,
                                                  float *dyf, uint16_t *dyb, uint16_t *dybt,
                                                  double *partial) {
  __shared__ double red[256];
  const size_t total = (size_t)M * N;
  const float scale = 2.0f / (float)((double)M * N);
  double s = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const float d = y[i] - t[i];
    s += (double)d * d;
    const float g = scale * d;
    dyf[i] = g;
    const uint16_t h = to_bf16(g);
    dyb[i] = h;
    dybt[(i % N) * M + i / N] = h;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sum_kernel(const double *partial, int n, double scale, double *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    *out = s * scale;
  }
}

// out[n] = sum_m D[m][n] (m ascending): bias gradients.
__global__ void colsum_kernel(const float *D, int M, int N, float *out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += D[(size_t)m * N + n];
  out[n] = s;
}

// Adam (Kingma and Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
// p <- p - lr (m c1) / (sqrt(v c2) + eps) with the bias corrections
// c1 = 1/(1-b1^t), c2 = 1/(1-b2^t); for a weight matrix [rows][cols] also
// its bfloat16 copies (row-major and transposed).
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, size_t n, int rows,
                            int cols, float lr, float b1, float b2, float eps, float c1, float c2,
                            uint16_t *wb, uint16_t *wbt) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    if (wb) {
      const uint16_t h = to_bf16(pi);
      wb[i] = h;
      wbt[(i % cols) * rows + i / cols] = h;
    }
  }
}

// ---- float64 data kernels ----

constexpr int kGramRows = 256;  // rows of X and V per workgroup of the cross Gram product

// Partial[blk][i][j] = sum over rows of block blk of X[row][i] V[row][j],
// i < m, j < m2 (m, m2 <= 128).
__global__ __launch_bounds__(256) void cross_gram_kernel(const double *X, int ldx, const double *V,
                                                         int ldv, long long N, int m, int m2,
                                                         double *partial) {
  __shared__ double xs[16][129];
  __shared__ double vs[16][129];
  const long long r0 = (long long)blockIdx.x * kGramRows;
  const long long r1 = r0 + kGramRows < N ? r0 + kGramRows : N;
  const int nout = m * m2;
  double acc[64];
#pragma unroll
  for (int q = 0; q < 64; ++q) acc[q] = 0.0;
  for (long long rb = r0; rb < r1; rb += 16) {
    const int nr = (int)((r1 - rb) < 16 ? (r1 - rb) : 16);
    __syncthreads();
    for (int idx = threadIdx.x; idx < 16 * 128; idx += 256) {
      const int rr = idx / 128, c = idx % 128;
      xs[rr][c] = (rr < nr && c < m) ? X[(rb + rr) * ldx + c] : 0.0;
      vs[rr][c] = (rr < nr && c < m2) ? V[(rb + rr) * ldv + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 64; ++q) {
      const int o = threadIdx.x + 256 * q;
      if (o < nout) {
        const int i = o / m2, j = o % m2;
        double s = acc[q];
        for (int rr = 0; rr < nr; ++rr) s += xs[rr][i] * vs[rr][j];
        acc[q] = s;
      }
    }
  }
  double *out = partial + (size_t)blockIdx.x * nout;
#pragma unroll
  for (int q = 0; q < 64; ++q) {
    const int o = threadIdx.x + 256 * q;
    if (o < nout) out[o] = acc[q];
  }
}

__global__ void partial_sum_kernel(const double *partial, int nblk, int nout, double *G) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(size_t)b * nout + o];
  G[o] = s;
}

// T[row][j] = sum_i X[row][i] G[i][j]  (G [m][m2], read through the caches).
__global__ __launch_bounds__(256) void tall_gemm_kernel(const double *X, int ldx, const double *G,
                                                        long long N, int m, int m2, double *T) {
  const long long total = N * m2;
  for (long long o = blockIdx.x * 256LL + threadIdx.x; o < total; o += (long long)gridDim.x * 256) {
    const long long row = o / m2;
    const int j = (int)(o % m2);
    const double *x = X + row * ldx;
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += x[i] * G[i * m2 + j];
    T[o] = s;
  }
}

// Gc[c] += T_c T_c^T for the cell rows T_c = T[c b .. c b + b - 1][0 .. m-1]
// (b <= 64; the columns are staged through LDS 64 at a time).
__global__ __launch_bounds__(256) void cell_gram_kernel(const double *T, int b, int m, double *Gc) {
  __shared__ double ts[64][65];
  const int c = blockIdx.x;
  const double *Tc = T + (size_t)c * b * m;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int k0 = 0; k0 < m; k0 += 64) {
    const int nk = m - k0 < 64 ? m - k0 : 64;
    __syncthreads();
    for (int idx = threadIdx.x; idx < b * 64; idx += 256) {
      const int i = idx / 64, k = idx % 64;
      ts[i][k] = k < nk ? Tc[(size_t)i * m + k0 + k] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int o = threadIdx.x + 256 * q;
      if (o < b * b) {
        const int i = o / b, j = o % b;
        double s = acc[q];
        for (int k = 0; k < nk; ++k) s += ts[i][k] * ts[j][k];
        acc[q] = s;
      }
    }
  }
  double *g = Gc + (size_t)c * b * b;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int o = threadIdx.x + 256 * q;
    if (o < b * b) g[o] += acc[q];
  }
}

// C[c][k][j] = scale * sum_i U[c][i][k] T[c b + i][j]  (float32 out).
__global__ void basis_project_kernel(const double *U, const double *T, int nc, int b, int r, int m,
                                     double scale, float *C) {
  const size_t total = (size_t)nc * r * m;
  for (size_t o = blockIdx.x * (size_t)blockDim.x + threadIdx.x; o < total;
       o += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(o % m);
    const int k = (int)((o / m) % r);
    const size_t c = o / ((size_t)m * r);
    const double *u = U + c * b * r;
    const double *t = T + c * b * m;
    double s = 0.0;
    for (int i = 0; i < b; ++i) s += u[i * r + k] * t[(size_t)i * m + j];
    C[o] = (float)(scale * s);
  }
}

// Y[c b + i][j] = scale * sum_k U[c][i][k] C[c][k][j] + rscale * R[c b + i][j]
// (float64 out; R may be null).
__global__ void basis_expand_kernel(const double *U, const float *C, int nc, int b, int r, int m,
                                    double scale, const double *R, double rscale, double *Y) {
  const size_t total = (size_t)nc * b * m;
  for (size_t o = blockIdx.x * (size_t)blockDim.x + threadIdx.x; o < total;
       o += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(o % m);
    const size_t row = o / m;
    const size_t c = row / b;
    const int i = (int)(row % b);
    const double *u = U + (c * b + i) * r;
    const float *cc = C + c * r * m;
    double s = 0.0;
    for (int k = 0; k < r; ++k) s += u[k] * (double)cc[(size_t)k * m + j];
    Y[o] = scale * s + (R ? rscale * R[o] : 0.0);
  }
}

int blocks_for(size_t n, int threads) {
  size_t b = (n + threads - 1) / threads;
  return (int)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

}  // namespace

int gemm_splits(int K, int kc) { return (K + kc - 1) / kc; }

hipError_t launch_gemm_nt(const uint16_t *A, const uint16_t *B, int M, int N, int K, int kc,
                          float *P, hipStream_t st) {
  if (M < 1 || N < 1 || K < 16 || K % 16 || kc < 16 || kc % 16) return hipErrorInvalidValue;
  const int nz = gemm_splits(K, kc);
  dim3 grid((N + kGemmTile - 1) / kGemmTile, (M + kGemmTile - 1) / kGemmTile, nz);
  hipLaunchKernelGGL(gemm_nt_kernel, grid, dim3(256), 0, st, A, B, M, N, K, kc, P);
  return hipGetLastError();
}

hipError_t launch_finish(const float *P, int splits, int M, int N, const float *bias, int relu,
                         const uint16_t *mask, float *outf, uint16_t *outb, uint16_t *outbt,
                         hipStream_t st) {
  hipLaunchKernelGGL(finish_kernel, dim3(blocks_for((size_t)M * N, 256)), dim3(256), 0, st, P,
                     splits, M, N, bias, relu, mask, outf, outb, outbt);
  return hipGetLastError();
}

hipError_t launch_cast_bf16(const float *x, int M, int N, uint16_t *xb, uint16_t *xbt,
                            hipStream_t st) {
  hipLaunchKernelGGL(cast_kernel, dim3(blocks_for((size_t)M * N, 256)), dim3(256), 0, st, x, M, N,
                     xb, xbt);
  return hipGetLastError();
}

int mse_partials(int M, int N) { return blocks_for((size_t)M * N, 256) < 1024 ? blocks_for((size_t)M * N, 256) : 1024; }

hipError_t launch_mse(const float *y, const float *t, int M, int N, float *dyf, uint16_t *dyb,
                      uint16_t *dybt, double *partial, double *loss, hipStream_t st) {
  const int nb = mse_partials(M, N);
  hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, st, y, t, M, N, dyf, dyb, dybt, partial);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, st, partial, nb, 1.0 / ((double)M * N),
                     loss);
  return hipGetLastError();
}

hipError_t launch_colsum(const float *D, int M, int N, float *out, hipStream_t st) {
  hipLaunchKernelGGL(colsum_kernel, dim3((N + 255) / 256), dim3(256), 0, st, D, M, N, out);
  return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, size_t n, int rows, int cols,
                       float lr, float b1, float b2, float eps, float c1, float c2, uint16_t *wb,
                       uint16_t *wbt, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, g, m, v, n, rows,
                     cols, lr, b1, b2, eps, c1, c2, wb, wbt);
  return hipGetLastError();
}

size_t cross_gram_partial_doubles(long long N, int m, int m2) {
  return (size_t)((N + kGramRows - 1) / kGramRows) * m * m2;
}

hipError_t launch_cross_gram(const double *X, int ldx, const double *V, int ldv, long long N, int m,
                             int m2, double *partial, double *G, hipStream_t st) {
  if (m < 1 || m > 128 || m2 < 1 || m2 > 128 || N < 1) return hipErrorInvalidValue;
  const int nblk = (int)((N + kGramRows - 1) / kGramRows);
  hipLaunchKernelGGL(cross_gram_kernel, dim3(nblk), dim3(256), 0, st, X, ldx, V, ldv, N, m, m2,
                     partial);
  hipLaunchKernelGGL(partial_sum_kernel, dim3((m * m2 + 255) / 256), dim3(256), 0, st, partial,
                     nblk, m * m2, G);
  return hipGetLastError();
}

hipError_t launch_tall_gemm(const double *X, int ldx, const double *G, long long N, int m, int m2,
                            double *T, hipStream_t st) {
  if (m < 1 || m > 128 || m2 < 1 || m2 > 128 || N < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tall_gemm_kernel, dim3(blocks_for((size_t)N * m2, 256)), dim3(256), 0, st, X,
                     ldx, G, N, m, m2, T);
  return hipGetLastError();
}

hipError_t launch_cell_gram(const double *T, int nc, int b, int m, double *Gc, hipStream_t st) {
  if (b < 1 || b > 64 || m < 1 || m > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cell_gram_kernel, dim3(nc), dim3(256), 0, st, T, b, m, Gc);
  return hipGetLastError();
}

hipError_t launch_basis_project(const double *U, const double *T, int nc, int b, int r, int m,
                                double scale, float *C, hipStream_t st) {
  hipLaunchKernelGGL(basis_project_kernel, dim3(blocks_for((size_t)nc * r * m, 256)), dim3(256), 0,
                     st, U, T, nc, b, r, m, scale, C);
  return hipGetLastError();
}

hipError_t launch_basis_expand(const double *U, const float *C, int nc, int b, int r, int m,
                               double scale, const double *R, double rscale, double *Y,
                               hipStream_t st) {
  hipLaunchKernelGGL(basis_expand_kernel, dim3(blocks_for((size_t)nc * b * m, 256)), dim3(256), 0,
                     st, U, C, nc, b, r, m, scale, R, rscale, Y);
  return hipGetLastError();
}

}  // namespace feast
