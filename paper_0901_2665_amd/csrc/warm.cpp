// C ABI of the learned warm start: the MLP (forward, gradients, Adam steps
// on the matrix cores in bfloat16) and the float64 kernels that build its
// training targets from FEAST solutions.  Kernels in warm.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "../../include/feast.h"
#include "kernels.h"

namespace feast {
hipStream_t context_stream(const feast_ctx *ctx);
int context_device(const feast_ctx *ctx);
}  // namespace feast

using namespace feast;

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? 0 : -100 - (int)e; }

#define HIPCHK(x)                                \
  do {                                           \
    hipError_t _e = (x);                         \
    if (_e != hipSuccess) return hip_status(_e); \
  } while (0)

constexpr int kSplitK = 512;  // reduction length of one split of the long backward product
constexpr float kBeta1 = 0.9f, kBeta2 = 0.999f, kAdamEps = 1e-8f;

size_t align_up(size_t x) { return (x + 63) / 64 * 64; }  // elements (256 bytes of floats)

}  // namespace

struct feast_mlp {
  feast_ctx *ctx = nullptr;
  int d[4] = {0, 0, 0, 0};
  int max_batch = 0;
  size_t nparam = 0;
  size_t offW[3] = {0, 0, 0}, offb[3] = {0, 0, 0};
  void *mem = nullptr;          // one device allocation for everything below
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *wb[3] = {nullptr, nullptr, nullptr}, *wbt[3] = {nullptr, nullptr, nullptr};
  uint16_t *xb = nullptr, *xbt = nullptr, *h1b = nullptr, *h1bt = nullptr, *h2b = nullptr,
           *h2bt = nullptr;
  float *y = nullptr, *dyf = nullptr, *dz2f = nullptr, *dz1f = nullptr, *part = nullptr;
  uint16_t *dyb = nullptr, *dybt = nullptr, *dz2b = nullptr, *dz2bt = nullptr, *dz1b = nullptr,
           *dz1bt = nullptr;
  double *lpart = nullptr, *loss = nullptr, *h_loss = nullptr;
  int step = 0;
};

namespace {

int mlp_forward(feast_mlp *n, int B, const float *x, float *yout) {
  hipStream_t st = context_stream(n->ctx);
  const int d0 = n->d[0], d1 = n->d[1], d2 = n->d[2], d3 = n->d[3];
  HIPCHK(launch_cast_bf16(x, B, d0, n->xb, n->xbt, st));
  HIPCHK(launch_gemm_nt(n->xb, n->wb[0], B, d1, d0, d0, n->part, st));
  HIPCHK(launch_finish(n->part, 1, B, d1, n->p + n->offb[0], 1, nullptr, nullptr, n->h1b, n->h1bt,
                       st));
  HIPCHK(launch_gemm_nt(n->h1b, n->wb[1], B, d2, d1, d1, n->part, st));
  HIPCHK(launch_finish(n->part, 1, B, d2, n->p + n->offb[1], 1, nullptr, nullptr, n->h2b, n->h2bt,
                       st));
  HIPCHK(launch_gemm_nt(n->h2b, n->wb[2], B, d3, d2, d2, n->part, st));
  HIPCHK(launch_finish(n->part, 1, B, d3, n->p + n->offb[2], 0, nullptr, yout, nullptr, nullptr,
                       st));
  return 0;
}

// Gradients of the mean squared error into n->g (packed like the parameters).
int mlp_backward(feast_mlp *n, int B, const float *t) {
  hipStream_t st = context_stream(n->ctx);
  const int d0 = n->d[0], d1 = n->d[1], d2 = n->d[2], d3 = n->d[3];
  HIPCHK(launch_mse(n->y, t, B, d3, n->dyf, n->dyb, n->dybt, n->lpart, n->loss, st));
  // layer 3: dW3 = dy^T h2, db3 = sum_b dy, dh2 = dy W3 (split over d3)
  HIPCHK(launch_gemm_nt(n->dybt, n->h2bt, d3, d2, B, B, n->g + n->offW[2], st));
  HIPCHK(launch_colsum(n->dyf, B, d3, n->g + n->offb[2], st));
  HIPCHK(launch_gemm_nt(n->dyb, n->wbt[2], B, d2, d3, kSplitK, n->part, st));
  HIPCHK(launch_finish(n->part, gemm_splits(d3, kSplitK), B, d2, nullptr, 0, n->h2b, n->dz2f,
                       n->dz2b, n->dz2bt, st));
  // layer 2
  HIPCHK(launch_gemm_nt(n->dz2bt, n->h1bt, d2, d1, B, B, n->g + n->offW[1], st));
  HIPCHK(launch_colsum(n->dz2f, B, d2, n->g + n->offb[1], st));
  HIPCHK(launch_gemm_nt(n->dz2b, n->wbt[1], B, d1, d2, d2, n->part, st));
  HIPCHK(launch_finish(n->part, 1, B, d1, nullptr, 0, n->h1b, n->dz1f, n->dz1b, n->dz1bt, st));
  // layer 1
  HIPCHK(launch_gemm_nt(n->dz1bt, n->xbt, d1, d0, B, B, n->g + n->offW[0], st));
  HIPCHK(launch_colsum(n->dz1f, B, d1, n->g + n->offb[0], st));
  return 0;
}

int check_batch(const feast_mlp *n, int B, bool training) {
  if (B < 1 || B > n->max_batch) return -3;
  if (training && B % 16) return -3;
  return 0;
}

}  // namespace

namespace feast {
void mlp_free(feast_mlp *n);
}

extern "C" {

int feast_mlp_create(feast_ctx *ctx, const int32_t dims[4], int32_t max_batch,
                     const float *params, feast_mlp **out) {
  if (!ctx || !dims || !params || !out) return -5;
  *out = nullptr;
  for (int i = 0; i < 4; ++i)
    if (dims[i] < 16 || dims[i] % 16) return -1;
  if (max_batch < 16 || max_batch % 16) return -3;
  HIPCHK(hipSetDevice(context_device(ctx)));
  feast_mlp *n = new (std::nothrow) feast_mlp();
  if (!n) return -100 - (int)hipErrorOutOfMemory;
  n->ctx = ctx;
  for (int i = 0; i < 4; ++i) n->d[i] = dims[i];
  n->max_batch = max_batch;
  const size_t d0 = dims[0], d1 = dims[1], d2 = dims[2], d3 = dims[3], B = max_batch;
  const size_t wsz[3] = {d1 * d0, d2 * d1, d3 * d2}, bsz[3] = {d1, d2, d3};
  size_t off = 0;
  for (int l = 0; l < 3; ++l) {
    n->offW[l] = off;
    off += wsz[l];
    n->offb[l] = off;
    off += bsz[l];
  }
  n->nparam = off;
  // float32 arrays (in floats), then bfloat16 arrays (in halves of floats)
  const int splits = gemm_splits((int)d3, kSplitK);
  size_t part = B * d3;
  for (size_t c : {splits * B * d2, B * d1, B * d2})
    if (c > part) part = c;
  const size_t fsz[] = {align_up(n->nparam) * 4, align_up(B * d3), align_up(B * d3),
                        align_up(B * d2), align_up(B * d1), align_up(part)};
  size_t floats = 0;
  for (size_t s : fsz) floats += s;
  const size_t hsz[] = {align_up(wsz[0]), align_up(wsz[0]), align_up(wsz[1]), align_up(wsz[1]),
                        align_up(wsz[2]), align_up(wsz[2]), align_up(B * d0), align_up(B * d0),
                        align_up(B * d1), align_up(B * d1), align_up(B * d2), align_up(B * d2),
                        align_up(B * d3), align_up(B * d3), align_up(B * d2), align_up(B * d2),
                        align_up(B * d1), align_up(B * d1)};
  size_t halves = 0;
  for (size_t s : hsz) halves += s;
  const size_t nlp = (size_t)mse_partials((int)B, (int)d3);
  const size_t bytes = floats * 4 + halves * 2 + align_up(nlp + 1) * 8;
  hipError_t e = hipMalloc(&n->mem, bytes);
  if (e == hipSuccess) e = hipHostMalloc((void **)&n->h_loss, sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    mlp_free(n);
    return hip_status(e);
  }
  float *f = static_cast<float *>(n->mem);
  const size_t np = align_up(n->nparam);
  n->p = f;
  n->g = f + np;
  n->m = f + 2 * np;
  n->v = f + 3 * np;
  f += 4 * np;
  n->y = f;
  f += fsz[1];
  n->dyf = f;
  f += fsz[2];
  n->dz2f = f;
  f += fsz[3];
  n->dz1f = f;
  f += fsz[4];
  n->part = f;
  f += fsz[5];
  uint16_t *h = reinterpret_cast<uint16_t *>(f);
  uint16_t **hp[] = {&n->wb[0], &n->wbt[0], &n->wb[1], &n->wbt[1], &n->wb[2], &n->wbt[2],
                     &n->xb, &n->xbt, &n->h1b, &n->h1bt, &n->h2b, &n->h2bt,
                     &n->dyb, &n->dybt, &n->dz2b, &n->dz2bt, &n->dz1b, &n->dz1bt};
  for (size_t i = 0; i < sizeof(hsz) / sizeof(hsz[0]); ++i) {
    *hp[i] = h;
    h += hsz[i];
  }
  n->lpart = reinterpret_cast<double *>(h);
  n->loss = n->lpart + nlp;
  hipStream_t st = context_stream(ctx);
  e = hipMemcpyAsync(n->p, params, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(n->m, 0, 2 * np * sizeof(float), st);  // m and v
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    const int rows = (int)bsz[l], cols = (int)(wsz[l] / bsz[l]);
    e = launch_cast_bf16(n->p + n->offW[l], rows, cols, n->wb[l], n->wbt[l], st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    mlp_free(n);
    return hip_status(e);
  }
  *out = n;
  return 0;
}

int feast_mlp_destroy(feast_mlp *net) {
  if (!net) return 0;
  mlp_free(net);
  return 0;
}

int feast_mlp_params(feast_mlp *net, float *params) {
  if (!net || !params) return -5;
  HIPCHK(hipSetDevice(context_device(net->ctx)));
  hipStream_t st = context_stream(net->ctx);
  HIPCHK(hipMemcpyAsync(params, net->p, net->nparam * sizeof(float), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return 0;
}

int feast_mlp_forward(feast_mlp *net, int32_t batch, const float *x, float *y) {
  if (!net || !x || !y) return -5;
  int stc = check_batch(net, batch, false);
  if (stc) return stc;
  HIPCHK(hipSetDevice(context_device(net->ctx)));
  int s = mlp_forward(net, batch, x, y);
  if (s) return s;
  HIPCHK(hipStreamSynchronize(context_stream(net->ctx)));
  return 0;
}

int feast_mlp_gradients(feast_mlp *net, int32_t batch, const float *x, const float *target,
                        float *grads, double *loss) {
  if (!net || !x || !target || !grads) return -5;
  int stc = check_batch(net, batch, true);
  if (stc) return stc;
  HIPCHK(hipSetDevice(context_device(net->ctx)));
  hipStream_t st = context_stream(net->ctx);
  int s = mlp_forward(net, batch, x, net->y);
  if (!s) s = mlp_backward(net, batch, target);
  if (s) return s;
  HIPCHK(hipMemcpyAsync(grads, net->g, net->nparam * sizeof(float), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(net->h_loss, net->loss, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (loss) *loss = *net->h_loss;
  return 0;
}

int feast_mlp_train_step(feast_mlp *net, int32_t batch, const float *x, const float *target,
                         float lr, double *loss) {
  if (!net || !x || !target) return -5;
  int stc = check_batch(net, batch, true);
  if (stc) return stc;
  if (!(lr > 0.0f) || !std::isfinite(lr)) return -7;
  HIPCHK(hipSetDevice(context_device(net->ctx)));
  hipStream_t st = context_stream(net->ctx);
  int s = mlp_forward(net, batch, x, net->y);
  if (!s) s = mlp_backward(net, batch, target);
  if (s) return s;
  ++net->step;
  const float c1 = 1.0f / (1.0f - std::pow(kBeta1, (float)net->step));
  const float c2 = 1.0f / (1.0f - std::pow(kBeta2, (float)net->step));
  for (int l = 0; l < 3; ++l) {
    const int rows = net->d[l + 1], cols = net->d[l];
    const size_t ow = net->offW[l], ob = net->offb[l];
    HIPCHK(launch_adam(net->p + ow, net->g + ow, net->m + ow, net->v + ow, (size_t)rows * cols,
                       rows, cols, lr, kBeta1, kBeta2, kAdamEps, c1, c2, net->wb[l], net->wbt[l],
                       st));
    HIPCHK(launch_adam(net->p + ob, net->g + ob, net->m + ob, net->v + ob, (size_t)rows, rows, 1,
                       lr, kBeta1, kBeta2, kAdamEps, c1, c2, nullptr, nullptr, st));
  }
  if (loss) {
    HIPCHK(hipMemcpyAsync(net->h_loss, net->loss, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *loss = *net->h_loss;
  }
  return 0;
}

int feast_cross_gram(feast_ctx *ctx, int64_t N, int32_t m, int32_t m2, const double *X,
                     int32_t ldx, const double *V, int32_t ldv, double *workspace, double *G) {
  if (!ctx || !X || !V || !G || !workspace) return -5;
  if (N < 1 || m < 1 || m > 128 || m2 < 1 || m2 > 128 || ldx < m || ldv < m2) return -3;
  HIPCHK(hipSetDevice(context_device(ctx)));
  hipStream_t st = context_stream(ctx);
  HIPCHK(launch_cross_gram(X, ldx, V, ldv, N, m, m2, workspace, G, st));
  HIPCHK(hipStreamSynchronize(st));
  return 0;
}

int64_t feast_cross_gram_workspace(int64_t N, int32_t m, int32_t m2) {
  if (N < 1 || m < 1 || m2 < 1) return 0;
  return (int64_t)cross_gram_partial_doubles(N, m, m2);
}

int feast_tall_gemm(feast_ctx *ctx, int64_t N, int32_t m, int32_t m2, const double *X,
                    int32_t ldx, const double *G, double *T) {
  if (!ctx || !X || !G || !T) return -5;
  if (N < 1 || m < 1 || m > 128 || m2 < 1 || m2 > 128 || ldx < m) return -3;
  HIPCHK(hipSetDevice(context_device(ctx)));
  hipStream_t st = context_stream(ctx);
  HIPCHK(launch_tall_gemm(X, ldx, G, N, m, m2, T, st));
  HIPCHK(hipStreamSynchronize(st));
  return 0;
}

int feast_cell_gram_accumulate(feast_ctx *ctx, int32_t nc, int32_t b, int32_t m, const double *T,
                               double *Gc) {
  if (!ctx || !T || !Gc) return -5;
  if (nc < 1 || b < 1 || b > 64) return -1;
  if (m < 1 || m > 128) return -3;
  HIPCHK(hipSetDevice(context_device(ctx)));
  hipStream_t st = context_stream(ctx);
  HIPCHK(launch_cell_gram(T, nc, b, m, Gc, st));
  HIPCHK(hipStreamSynchronize(st));
  return 0;
}

int feast_basis_project(feast_ctx *ctx, int32_t nc, int32_t b, int32_t r, int32_t m,
                        const double *U, const double *T, double scale, float *C) {
  if (!ctx || !U || !T || !C) return -5;
  if (nc < 1 || b < 1 || r < 1 || r > b) return -1;
  if (m < 1) return -3;
  HIPCHK(hipSetDevice(context_device(ctx)));
  hipStream_t st = context_stream(ctx);
  HIPCHK(launch_basis_project(U, T, nc, b, r, m, scale, C, st));
  HIPCHK(hipStreamSynchronize(st));
  return 0;
}

int feast_basis_expand(feast_ctx *ctx, int32_t nc, int32_t b, int32_t r, int32_t m,
                       const double *U, const float *C, double scale, const double *R,
                       double rscale, double *Y) {
  if (!ctx || !U || !C || !Y) return -5;
  if (nc < 1 || b < 1 || r < 1 || r > b) return -1;
  if (m < 1) return -3;
  HIPCHK(hipSetDevice(context_device(ctx)));
  hipStream_t st = context_stream(ctx);
  HIPCHK(launch_basis_expand(U, C, nc, b, r, m, scale, R, rscale, Y, st));
  HIPCHK(hipStreamSynchronize(st));
  return 0;
}

}  // extern "C"

namespace feast {
void mlp_free(feast_mlp *n) {
  if (!n) return;
  (void)hipSetDevice(context_device(n->ctx));
  (void)hipStreamSynchronize(context_stream(n->ctx));
  if (n->mem) (void)hipFree(n->mem);
  if (n->h_loss) (void)hipHostFree(n->h_loss);
  delete n;
}
}  // namespace feast
