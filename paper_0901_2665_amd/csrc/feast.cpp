// Host driver and C ABI of the FEAST hot path (see include/feast.h).
//
// The host only validates arguments, computes the Gauss-Legendre rule and
// the contour (eqs. 13-14), launches the kernels in order on the context's
// stream and takes the loop decisions of Fig. 2 step 6 from the M0 Ritz
// values it copies back once per refinement loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

#include "../../include/feast.h"
#include "kernels.h"

using namespace feast;

namespace {

constexpr int kMaxB = 64;
constexpr int kMaxM0 = 128;
// convergence waits while the smallest residual of the uncounted in-interval
// Ritz pairs falls below this fraction of its previous-loop value
constexpr double kUncountedDrop = 0.5;
// Hermitian variant: block size and subspace limits (the fallback solves the
// reduced problem through its real embedding of size 2 M0 <= 128)
constexpr int kMaxHB = 96;
constexpr int kMaxHM0 = 64;

struct Buf {
  void *ptr = nullptr;
  size_t cap = 0;
};

enum Slot {
  S_SINV, S_W, S_WT, S_TW, S_G, S_TV, S_Y, S_R, S_P, S_Q, S_X, S_GRAMP, S_AQ, S_BQ,
  S_EPS, S_PHI, S_RRS, S_FLAG, S_RESP, S_RES, S_PERM, S_T0, S_T1, S_FWORK, S_CHAINS,
  S_SINV32, S_W32, S_WT32, S_G32, S_TV32, S_XC, S_RC, S_RPART, S_WORST,
  // Hermitian variant
  S_HSINV, S_HW, S_HV, S_HG, S_HY, S_HR, S_HQ, S_HX, S_HAX, S_HBX, S_HPART, S_HAQ, S_HBQ,
  S_HEA, S_HEB, S_HEPS2, S_HPHI2, S_HEPS, S_HPHI, S_HRES, S_HCOEF, S_HFWORK, S_HZ, S_CONV, S_COUNT
};

}  // namespace

namespace {
// Kernel classes timed by feast_timing / feast_timing_read.
enum Kind { K_FACTOR, K_FORWARD, K_BACK, K_BTMUL, K_SUM, K_GRAM, K_RR, K_RITZ, K_RESID,
            K_LAYOUT, K_ROUND, K_FWD32, K_BACK32, K_REFRES, K_HSWEEP, K_COUNT };
const char *kKindNames[K_COUNT] = {"factor",        "forward_sweep",   "back_sweep",
                                   "bt_multiply",   "sum_nodes",       "projection",
                                   "reduced_eig",   "ritz_gemm",       "residual",
                                   "layout",        "round_factors",   "forward_sweep32",
                                   "back_sweep32",  "refine_residual", "sweeps_hermitian"};
struct Timing {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, size_t>> recs;  // (kind, index of the start event)
};
}  // namespace

struct feast_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool owns_stream = false;          // workers of a batched call own theirs
  hipStream_t capture = nullptr;     // graph capture (the caller's stream may be
                                     // the null stream, which cannot capture)
  Buf buf[S_COUNT];
  double *h_eps = nullptr;  // pinned: eps[128] + res[128]
  int *h_flag = nullptr;    // pinned
  double *rr_static = nullptr;  // device address of the reduced eigensolver's static scratch
  int *rr_static_flag = nullptr;
  Timing timing;
  std::vector<feast_ctx *> workers;  // sub-contexts of feast_solve_batched
};

namespace feast {
hipStream_t context_stream(const feast_ctx *ctx) { return ctx->stream; }
int context_device(const feast_ctx *ctx) { return ctx->device; }
}  // namespace feast

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? 0 : -100 - (int)e; }

#define HIPCHK(x)                          \
  do {                                     \
    hipError_t _e = (x);                   \
    if (_e != hipSuccess) return hip_status(_e); \
  } while (0)

hipError_t ensure(feast_ctx *ctx, Slot s, size_t bytes, void **out) {
  Buf &b = ctx->buf[s];
  if (bytes == 0) bytes = 256;
  if (b.cap < bytes) {
    if (b.ptr) {
      hipError_t e = hipFree(b.ptr);
      if (e != hipSuccess) return e;
      b.ptr = nullptr;
      b.cap = 0;
    }
    hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) return e;
    b.cap = bytes;
  }
  *out = b.ptr;
  return hipSuccess;
}

template <typename T>
hipError_t ensure_t(feast_ctx *ctx, Slot s, size_t count, T **out) {
  void *p = nullptr;
  hipError_t e = ensure(ctx, s, count * sizeof(T), &p);
  *out = static_cast<T *>(p);
  return e;
}

int round16(int x) { return (x + 15) / 16 * 16; }

// Start/stop events around one launch when timing is on.
hipError_t tmark(feast_ctx *ctx, size_t *idx) {
  Timing &t = ctx->timing;
  if (!t.on) return hipSuccess;
  if (t.used == t.pool.size()) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    t.pool.push_back(ev);
  }
  *idx = t.used++;
  return hipEventRecord(t.pool[*idx], ctx->stream);
}

#define TIMED(kind, expr)                                   \
  do {                                                      \
    size_t _t0 = 0, _t1 = 0;                                \
    HIPCHK(tmark(ctx, &_t0));                               \
    HIPCHK(expr);                                           \
    HIPCHK(tmark(ctx, &_t1));                               \
    if (ctx->timing.on) ctx->timing.recs.push_back({(kind), _t0}); \
  } while (0)

// Gauss-Legendre rule on [-1, 1]: Newton on the roots of P_n with the
// three-term recurrence; weights 2 / ((1 - x^2) P_n'(x)^2).  Ascending nodes.
void gauss_legendre(int n, double *x, double *w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int k = 1; k <= n; ++k) {
        double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * k - 1.0) * z * p2 - (k - 1.0) * p3) / k;
      }
      dp = n * (z * p1 - p2) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // one more evaluation of the derivative at the converged node
        double q1 = 1.0, q2 = 0.0;
        for (int k = 1; k <= n; ++k) {
          double q3 = q2;
          q2 = q1;
          q1 = ((2.0 * k - 1.0) * z * q2 - (k - 1.0) * q3) / k;
        }
        dp = n * (z * q1 - q2) / (z * z - 1.0);
        break;
      }
    }
    // cos(...) for i = 0 is the largest root; store ascending
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

void make_shifts(int Ne, double emin, double emax, Shifts &s, double *xo = nullptr,
                 double *wo = nullptr) {
  double x[kMaxNe], w[kMaxNe];
  gauss_legendre(Ne, x, w);
  const double r = 0.5 * (emax - emin), c = 0.5 * (emax + emin);
  std::memset(&s, 0, sizeof(s));
  for (int e = 0; e < Ne; ++e) {
    const double th = -(M_PI / 2.0) * (x[e] - 1.0);
    s.zre[e] = c + r * std::cos(th);
    s.zim[e] = r * std::sin(th);
    s.kre[e] = -(w[e] / 2.0) * r * std::cos(th);
    s.kim[e] = -(w[e] / 2.0) * r * std::sin(th);
    if (xo) xo[e] = x[e];
    if (wo) wo[e] = w[e];
  }
}

int validate_matrix(const feast_bt_matrix *AB) {
  if (!AB) return -5;
  if (AB->nc < 1 || AB->b < 1 || AB->b > kMaxB) return -1;
  if (!AB->A_diag || !AB->B_diag) return -5;
  if (AB->nc > 1 && (!AB->A_up || !AB->B_up)) return -5;
  return 0;
}

Pencil make_pencil(const feast_bt_matrix *AB) {
  Pencil p;
  p.Ad = AB->A_diag;
  p.Au = AB->A_up;
  p.Bd = AB->B_diag;
  p.Bu = AB->B_up;
  p.nc = AB->nc;
  p.b = AB->b;
  p.bp = round16(AB->b);
  return p;
}

// Real pencils with 64 < b <= 96 run on the wide kernels: one top-down
// chain per node over all cells (factor.hip, sweep.hip), blocks padded to 96.
constexpr int kWideBP = 96;
bool is_wide(const feast_bt_matrix *AB) { return AB && AB->b > kMaxB && AB->b <= kWideBP; }

Pencil make_wide_pencil(const feast_bt_matrix *AB) {
  Pencil p = make_pencil(AB);
  p.bp = kWideBP;
  return p;
}

int validate_wide(const feast_bt_matrix *AB) {
  if (!AB) return -5;
  if (AB->nc < 1 || AB->b <= kMaxB || AB->b > kWideBP) return -1;
  if (!AB->A_diag || !AB->B_diag) return -5;
  if (AB->nc > 1 && (!AB->A_up || !AB->B_up)) return -5;
  return 0;
}

// Non-finite scan of the pencil (and optionally Y0); returns -6 on NaN/Inf.
int check_inputs(feast_ctx *ctx, const feast_bt_matrix *AB, const double *Y0, size_t ny) {
  int *flag = nullptr;
  HIPCHK(ensure_t(ctx, S_FLAG, 4, &flag));
  HIPCHK(hipMemsetAsync(flag, 0, 4 * sizeof(int), ctx->stream));
  const size_t bb = (size_t)AB->b * AB->b;
  HIPCHK(launch_check_finite(AB->A_diag, AB->nc * bb, flag, ctx->stream));
  HIPCHK(launch_check_finite(AB->B_diag, AB->nc * bb, flag, ctx->stream));
  if (AB->nc > 1) {
    HIPCHK(launch_check_finite(AB->A_up, (AB->nc - 1) * bb, flag, ctx->stream));
    HIPCHK(launch_check_finite(AB->B_up, (AB->nc - 1) * bb, flag, ctx->stream));
  }
  if (Y0) HIPCHK(launch_check_finite(Y0, ny, flag, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ctx->h_flag[0] ? -6 : 0;
}

struct Work {
  Pencil p;
  Factors f;
  SolveBufs sb;
  int Ne, m0, m0p, parts, gtiles;
  size_t rows;
  double *fwork;
  Chain *chains;
};

// Partitions per half chain of the factorisation: enough independent chains
// for every compute unit (2 Ne chains a partition), at least 8 cells each.
int choose_parts(int nc, int Ne, int requested) {
  const int half = nc / 2;  // cells of the shorter (bottom) half; no empty partitions
  if (requested > 0) return std::max(1, std::min(requested, half));
  const int by_len = half / 8;
  const int by_cus = std::max(1, 256 / (2 * Ne));
  return std::max(1, std::min(by_len, by_cus));
}

// Workspace for the factors and the sweeps of Ne shifts.
int prepare_factor(feast_ctx *ctx, const Pencil &p, int Ne, int m0p, int parts, Work &wk) {
  const size_t blk = 2 * (size_t)p.bp * p.bp;
  wk.p = p;
  wk.Ne = Ne;
  wk.m0p = m0p;
  wk.rows = (size_t)p.nc * p.bp;
  wk.f.m = p.nc - p.nc / 2;
  wk.parts = parts;
  wk.gtiles = std::max(m0p, p.bp) / kTile;
  HIPCHK(ensure_t(ctx, S_SINV, (size_t)Ne * p.nc * blk, &wk.f.Sinv));
  HIPCHK(ensure_t(ctx, S_W, (size_t)Ne * p.nc * blk, &wk.f.W));
  HIPCHK(ensure_t(ctx, S_WT, (size_t)Ne * p.nc * blk, &wk.f.WT));
  HIPCHK(ensure_t(ctx, S_TW, (size_t)Ne * blk, &wk.f.TW));
  HIPCHK(ensure_t(ctx, S_G, (size_t)Ne * wk.gtiles * wk.rows * kTile * 2, &wk.sb.G));
  HIPCHK(ensure_t(ctx, S_TV, (size_t)Ne * (m0p / kTile) * 4 * p.bp * kTile, &wk.sb.TV));
  HIPCHK(ensure_t(ctx, S_FWORK, factor_work_doubles(p, Ne, parts), &wk.fwork));
  HIPCHK(ensure_t(ctx, S_CHAINS, (size_t)3 * Ne * 2 * parts, &wk.chains));
  return 0;
}

hipError_t run_factor(feast_ctx *ctx, const Work &wk, const Shifts &s) {
  return launch_factor(wk.p, s, wk.Ne, wk.f, wk.parts, wk.fwork, wk.chains, wk.sb.G, wk.gtiles,
                       ctx->stream);
}

// Workspace of the wide kernels for Ne nodes and m0p padded columns (the
// slots of the twisted factorisation, which a wide solve does not use).
struct WideWork {
  Pencil p;
  Factors f;
  SolveBufs sb;
  double *cpl;
  int Ne, m0p;
  size_t rows;
};

int prepare_wide(feast_ctx *ctx, const Pencil &p, int Ne, int m0p, WideWork &ww) {
  const size_t blk = 2 * (size_t)kWideBP * kWideBP;
  ww.p = p;
  ww.Ne = Ne;
  ww.m0p = m0p;
  ww.rows = (size_t)p.nc * kWideBP;
  ww.f.m = p.nc;
  ww.f.TW = nullptr;
  HIPCHK(ensure_t(ctx, S_SINV, (size_t)Ne * p.nc * blk, &ww.f.Sinv));
  HIPCHK(ensure_t(ctx, S_W, (size_t)Ne * p.nc * blk, &ww.f.W));
  HIPCHK(ensure_t(ctx, S_WT, (size_t)Ne * p.nc * blk, &ww.f.WT));
  HIPCHK(ensure_t(ctx, S_G, (size_t)Ne * (m0p / kTile) * p.nc * 2 * kWideBP * kTile, &ww.sb.G));
  ww.sb.TV = nullptr;
  HIPCHK(ensure_t(ctx, S_FWORK, wide_pack_doubles(p), &ww.cpl));
  return 0;
}

// ---- mixed precision: float32 factors and sweeps, float64 refinement ----

// Refinement stops when every column j of every node has
//   ||R_j - (Z_e B - A) x_j||_2 <= kRefineTol (||R_j|| + |Z_e| ||B x_j|| + ||A x_j||),
// i.e. a residual 1e-12 of the size of the terms it is formed from: float64
// rounding in forming it is about 1e-16 of that size, so the test is
// reachable however ill-conditioned Z_e B - A is (a bound relative to ||R_j||
// alone is not: float64 solves themselves miss it once cond(Z_e B - A) u_64
// exceeds it).
constexpr double kRefineTol = 1e-12;
constexpr int kMaxRefine = 10;  // correction solves per contour integration

struct Mixed {
  Factors32 f;
  SolveBufs32 sb;
  double *xc;      // [Ne][2][rows][m0p] iterates
  double *rc;      // [Ne][2][rows][m0p] residuals
  double *part;    // shift_residual_partial_doubles
  double *worst;   // one double
  size_t plane;
};

int prepare_mixed(feast_ctx *ctx, const Work &wk, Mixed &mx) {
  const size_t blk = 2 * (size_t)wk.p.bp * wk.p.bp;
  const size_t nf = (size_t)wk.Ne * wk.p.nc * blk;
  mx.f.m = wk.f.m;
  mx.plane = wk.rows * wk.m0p;
  HIPCHK(ensure_t(ctx, S_SINV32, nf, &mx.f.Sinv));
  HIPCHK(ensure_t(ctx, S_W32, nf, &mx.f.W));
  HIPCHK(ensure_t(ctx, S_WT32, nf, &mx.f.WT));
  HIPCHK(ensure_t(ctx, S_G32, (size_t)wk.Ne * wk.rows * wk.m0p * 2, &mx.sb.G));
  HIPCHK(ensure_t(ctx, S_TV32, (size_t)wk.Ne * (wk.m0p / kTile) * 4 * wk.p.bp * kTile, &mx.sb.TV));
  HIPCHK(ensure_t(ctx, S_XC, (size_t)wk.Ne * 2 * mx.plane, &mx.xc));
  HIPCHK(ensure_t(ctx, S_RC, (size_t)wk.Ne * 2 * mx.plane, &mx.rc));
  HIPCHK(ensure_t(ctx, S_RPART, shift_residual_partial_doubles(wk.p.nc, wk.m0p, wk.Ne), &mx.part));
  HIPCHK(ensure_t(ctx, S_WORST, 1, &mx.worst));
  return 0;
}

// x_e = (Z_e B - A)^{-1} R for every node: a float32 solve, then float64
// residuals and float32 corrections until every column passes the kRefineTol
// test (or kMaxRefine corrections).  R: padded real right-hand side.  Returns
// the corrections made in *steps and the final worst residual ratio in
// *worst.
int mixed_solve(feast_ctx *ctx, const Work &wk, const Mixed &mx, const Shifts &s, const double *R,
                int m0, int *steps, double *worst) {
  hipStream_t sm = ctx->stream;
  const Pencil &p = wk.p;
  TIMED(K_FWD32, launch_sweeps32(p, wk.Ne, mx.f, mx.sb, R, 0, 0, wk.m0p, mx.xc, 0, 1, sm));
  TIMED(K_BACK32, launch_sweeps32(p, wk.Ne, mx.f, mx.sb, R, 0, 0, wk.m0p, mx.xc, 0, 2, sm));
  double *h_worst = ctx->h_eps + 3 * kMaxM0;
  *steps = 0;
  while (true) {
    TIMED(K_REFRES, launch_shift_residuals(p, s, wk.Ne, mx.xc, R, wk.m0p, m0, mx.rc, mx.part,
                                           mx.worst, sm));
    HIPCHK(hipMemcpyAsync(h_worst, mx.worst, sizeof(double), hipMemcpyDeviceToHost, sm));
    HIPCHK(hipStreamSynchronize(sm));
    *worst = *h_worst;
    if (*worst <= kRefineTol || *steps >= kMaxRefine) break;
    TIMED(K_FWD32, launch_sweeps32(p, wk.Ne, mx.f, mx.sb, mx.rc, 2 * mx.plane, 1, wk.m0p, mx.xc,
                                   1, 1, sm));
    TIMED(K_BACK32, launch_sweeps32(p, wk.Ne, mx.f, mx.sb, mx.rc, 2 * mx.plane, 1, wk.m0p, mx.xc,
                                    1, 2, sm));
    ++*steps;
  }
  return 0;
}

}  // namespace

// One captured loop of feast_solve: the graph is built from the launches of
// body(cs) on the capture stream cs (it records only; the graph then runs on
// the caller's stream); capture always ends, also when a launch fails.
struct GraphExec {
  hipGraphExec_t exec = nullptr;
  template <class Body>
  hipError_t capture(hipStream_t cs, Body &&body) {
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return e;
    const hipError_t eb = body(cs);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &g);
    e = eb != hipSuccess ? eb : ee;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
  }
  ~GraphExec() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

extern "C" {

void feast_default_opts(feast_opts *opts) {
  if (!opts) return;
  opts->tol = 1e-12;
  opts->max_loops = 20;
  opts->precision = 0;
  opts->partitions = 0;
  opts->graph = 0;
  opts->Y0 = nullptr;
  opts->seed = 0;
  opts->verbose = 0;
}

int feast_init(feast_ctx **ctx, int device, void *hip_stream) {
  if (!ctx) return -5;
  *ctx = nullptr;
  HIPCHK(hipSetDevice(device));
  feast_ctx *c = new feast_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipHostMalloc((void **)&c->h_eps, 4 * kMaxM0 * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->h_flag, 16 * sizeof(int), hipHostMallocDefault);
  // this device's copy of the static scratch (device `device` is current)
  if (e == hipSuccess) e = reduced_eig_static_scratch(&c->rr_static, &c->rr_static_flag);
  if (e != hipSuccess) {
    feast_destroy(c);
    return hip_status(e);
  }
  *ctx = c;
  return 0;
}

int feast_destroy(feast_ctx *ctx) {
  if (!ctx) return 0;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  for (auto &b : ctx->buf)
    if (b.ptr) (void)hipFree(b.ptr);
  for (auto ev : ctx->timing.pool) (void)hipEventDestroy(ev);
  if (ctx->h_eps) (void)hipHostFree(ctx->h_eps);
  if (ctx->h_flag) (void)hipHostFree(ctx->h_flag);
  for (feast_ctx *w : ctx->workers) feast_destroy(w);
  if (ctx->owns_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
  delete ctx;
  return 0;
}

const char *feast_strerror(int status) {
  switch (status) {
    case 0: return "success";
    case -1: return "bad block structure (nc < 1, b < 1, or b above the call's maximum: 96 or 64)";
    case -2: return "bad interval (emin >= emax or not finite)";
    case -3: return "bad subspace size (M0 < 1, M0 > N or M0 > 128)";
    case -4: return "bad number of contour points (Ne < 1 or Ne > 64)";
    case -5: return "NULL pointer argument";
    case -6: return "non-finite value in the input";
    case -7: return "bad option";
    case 1: return "not converged within max_loops";
    case 2: return "B_Q not positive definite; reduced problem solved on its range";
    case 3: return "no eigenvalue in the interval";
    case 4: return "subspace too small: M = M0";
    case 5: return "mixed-precision refinement stopped above its tolerance";
    default: return status <= -100 ? "HIP runtime error" : "unknown status";
  }
}

int feast_timing(feast_ctx *ctx, int32_t enable) {
  if (!ctx) return -5;
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->timing.on = enable != 0;
  ctx->timing.used = 0;
  ctx->timing.recs.clear();
  return 0;
}

int feast_timing_read(feast_ctx *ctx, int32_t kind, const char **name, double *total_ms,
                      int64_t *launches) {
  if (!ctx) return -5;
  if (kind < 0) return K_COUNT;
  if (kind >= K_COUNT) return -7;
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto &r : ctx->timing.recs) {
    if (r.first != kind) continue;
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->timing.pool[r.second], ctx->timing.pool[r.second + 1]));
    tot += ms;
    ++cnt;
  }
  if (name) *name = kKindNames[kind];
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  return 0;
}

int feast_contour(int32_t Ne, double emin, double emax, double *x, double *w, double *z_re,
                  double *z_im, double *k_re, double *k_im) {
  if (Ne < 1 || Ne > kMaxNe) return -4;
  if (!(emin < emax) || !std::isfinite(emin) || !std::isfinite(emax)) return -2;
  if (!x || !w || !z_re || !z_im || !k_re || !k_im) return -5;
  Shifts s;
  make_shifts(Ne, emin, emax, s, x, w);
  for (int e = 0; e < Ne; ++e) {
    z_re[e] = s.zre[e];
    z_im[e] = s.zim[e];
    k_re[e] = s.kre[e];
    k_im[e] = s.kim[e];
  }
  return 0;
}

int feast_bt_multiply(feast_ctx *ctx, const feast_bt_matrix *AB, int32_t which, int32_t m,
                      const double *V, double *out) {
  if (!ctx || !V || !out) return -5;
  int st = validate_matrix(AB);
  if (st) return st;
  if (m < 1 || m > kMaxM0) return -3;
  if (which != 0 && which != 1) return -7;
  HIPCHK(hipSetDevice(ctx->device));
  Pencil p = make_pencil(AB);
  const int mp = round16(m);
  const size_t rows = (size_t)p.nc * p.bp;
  double *vin, *vout;
  HIPCHK(ensure_t(ctx, S_T0, rows * mp, &vin));
  HIPCHK(ensure_t(ctx, S_T1, rows * mp, &vout));
  HIPCHK(launch_pack(V, p.nc, p.b, p.bp, m, mp, vin, ctx->stream));
  HIPCHK(launch_cell_apply(p, which, vin, mp, vout, ctx->stream));
  HIPCHK(launch_unpack(vout, p.nc, p.b, p.bp, m, mp, nullptr, out, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return 0;
}

int feast_shifted_solve(feast_ctx *ctx, const feast_bt_matrix *AB, double z_re, double z_im,
                        int32_t m, const double *R, double *X_re, double *X_im,
                        int32_t partitions) {
  if (!ctx || !R || !X_re || !X_im) return -5;
  if (is_wide(AB)) {  // one chain, no partitions
    if (!AB->A_diag || !AB->B_diag || (AB->nc > 1 && (!AB->A_up || !AB->B_up))) return -5;
    if (AB->nc < 1) return -1;
    if (m < 1 || m > kMaxM0) return -3;
    if (!(z_im > 0.0) || !std::isfinite(z_re) || !std::isfinite(z_im)) return -2;
    if (partitions < 0) return -7;
    HIPCHK(hipSetDevice(ctx->device));
    const Pencil p = make_wide_pencil(AB);
    const int mp = round16(m);
    WideWork ww;
    int st = prepare_wide(ctx, p, 1, mp, ww);
    if (st) return st;
    Shifts s;
    std::memset(&s, 0, sizeof(s));
    s.zre[0] = z_re;
    s.zim[0] = z_im;
    double *rin, *xr, *xi;
    HIPCHK(ensure_t(ctx, S_R, ww.rows * mp, &rin));
    HIPCHK(ensure_t(ctx, S_T0, ww.rows * mp, &xr));
    HIPCHK(ensure_t(ctx, S_T1, ww.rows * mp, &xi));
    HIPCHK(launch_factor_wide(p, s, 1, ww.f, ww.cpl, ctx->stream));
    HIPCHK(launch_pack(R, p.nc, p.b, p.bp, m, mp, rin, ctx->stream));
    HIPCHK(launch_sweeps_wide(p, s, 1, ww.f, ww.sb, rin, mp, xr, xi, 3, ctx->stream));
    HIPCHK(launch_unpack(xr, p.nc, p.b, p.bp, m, mp, nullptr, X_re, ctx->stream));
    HIPCHK(launch_unpack(xi, p.nc, p.b, p.bp, m, mp, nullptr, X_im, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return 0;
  }
  int st = validate_matrix(AB);
  if (st) return st;
  if (m < 1 || m > kMaxM0) return -3;
  if (!(z_im > 0.0) || !std::isfinite(z_re) || !std::isfinite(z_im)) return -2;
  if (partitions < 0) return -7;
  HIPCHK(hipSetDevice(ctx->device));
  Pencil p = make_pencil(AB);
  const int mp = round16(m);
  Work wk;
  st = prepare_factor(ctx, p, 1, mp, choose_parts(p.nc, 1, partitions), wk);
  if (st) return st;
  Shifts s;
  std::memset(&s, 0, sizeof(s));
  s.zre[0] = z_re;
  s.zim[0] = z_im;
  double *rin, *xr, *xi;
  HIPCHK(ensure_t(ctx, S_R, wk.rows * mp, &rin));
  HIPCHK(ensure_t(ctx, S_T0, wk.rows * mp, &xr));
  HIPCHK(ensure_t(ctx, S_T1, wk.rows * mp, &xi));
  HIPCHK(run_factor(ctx, wk, s));
  HIPCHK(launch_pack(R, p.nc, p.b, p.bp, m, mp, rin, ctx->stream));
  HIPCHK(launch_sweeps_complex(p, s, wk.f, wk.sb, rin, mp, xr, xi, ctx->stream));
  HIPCHK(launch_unpack(xr, p.nc, p.b, p.bp, m, mp, nullptr, X_re, ctx->stream));
  HIPCHK(launch_unpack(xi, p.nc, p.b, p.bp, m, mp, nullptr, X_im, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return 0;
}

int feast_shifted_solve_mixed(feast_ctx *ctx, const feast_bt_matrix *AB, double z_re,
                              double z_im, int32_t m, const double *R, double *X_re,
                              double *X_im, int32_t partitions, int32_t *steps,
                              double *rel_res) {
  if (!ctx || !R || !X_re || !X_im) return -5;
  int st = validate_matrix(AB);
  if (st) return st;
  if (m < 1 || m > kMaxM0) return -3;
  if (!(z_im > 0.0) || !std::isfinite(z_re) || !std::isfinite(z_im)) return -2;
  if (partitions < 0) return -7;
  HIPCHK(hipSetDevice(ctx->device));
  Pencil p = make_pencil(AB);
  const int mp = round16(m);
  Work wk;
  st = prepare_factor(ctx, p, 1, mp, choose_parts(p.nc, 1, partitions), wk);
  if (st) return st;
  Mixed mx;
  st = prepare_mixed(ctx, wk, mx);
  if (st) return st;
  Shifts s;
  std::memset(&s, 0, sizeof(s));
  s.zre[0] = z_re;
  s.zim[0] = z_im;
  double *rin;
  HIPCHK(ensure_t(ctx, S_R, wk.rows * mp, &rin));
  HIPCHK(run_factor(ctx, wk, s));
  HIPCHK(launch_round_factors(p, 1, wk.f, mx.f, ctx->stream));
  HIPCHK(launch_pack(R, p.nc, p.b, p.bp, m, mp, rin, ctx->stream));
  int k = 0;
  double worst = 0.0;
  st = mixed_solve(ctx, wk, mx, s, rin, m, &k, &worst);
  if (st) return st;
  HIPCHK(launch_unpack(mx.xc, p.nc, p.b, p.bp, m, mp, nullptr, X_re, ctx->stream));
  HIPCHK(launch_unpack(mx.xc + mx.plane, p.nc, p.b, p.bp, m, mp, nullptr, X_im, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (steps) *steps = k;
  if (rel_res) *rel_res = worst;
  return worst <= kRefineTol ? 0 : 5;
}

int feast_filter_mixed(feast_ctx *ctx, const feast_bt_matrix *AB, double emin, double emax,
                       int32_t M0, int32_t Ne, const double *Y, double *Q, int32_t *steps,
                       double *rel_res) {
  if (!ctx || !Y || !Q) return -5;
  int st = validate_matrix(AB);
  if (st) return st;
  if (!(emin < emax) || !std::isfinite(emin) || !std::isfinite(emax)) return -2;
  if (M0 < 1 || M0 > kMaxM0 || M0 > AB->nc * AB->b) return -3;
  if (Ne < 1 || Ne > kMaxNe) return -4;
  HIPCHK(hipSetDevice(ctx->device));
  Pencil p = make_pencil(AB);
  const int mp = round16(M0);
  Work wk;
  st = prepare_factor(ctx, p, Ne, mp, choose_parts(p.nc, Ne, 0), wk);
  if (st) return st;
  Mixed mx;
  st = prepare_mixed(ctx, wk, mx);
  if (st) return st;
  Shifts s;
  make_shifts(Ne, emin, emax, s);
  double *y, *r, *q;
  HIPCHK(ensure_t(ctx, S_Y, wk.rows * mp, &y));
  HIPCHK(ensure_t(ctx, S_R, wk.rows * mp, &r));
  HIPCHK(ensure_t(ctx, S_Q, wk.rows * mp, &q));
  HIPCHK(run_factor(ctx, wk, s));
  HIPCHK(launch_round_factors(p, Ne, wk.f, mx.f, ctx->stream));
  HIPCHK(launch_pack(Y, p.nc, p.b, p.bp, M0, mp, y, ctx->stream));
  HIPCHK(launch_cell_apply(p, 1, y, mp, r, ctx->stream));
  int k = 0;
  double worst = 0.0;
  st = mixed_solve(ctx, wk, mx, s, r, M0, &k, &worst);
  if (st) return st;
  HIPCHK(launch_sum_nodes_complex(s, Ne, mx.xc, mx.plane, q, ctx->stream));
  HIPCHK(launch_unpack(q, p.nc, p.b, p.bp, M0, mp, nullptr, Q, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (steps) *steps = k;
  if (rel_res) *rel_res = worst;
  return worst <= kRefineTol ? 0 : 5;
}

int feast_random_start(feast_ctx *ctx, uint64_t seed, int64_t N, int32_t M0, double *Y) {
  if (!ctx || !Y) return -5;
  if (N < 1 || N > INT32_MAX) return -1;
  if (M0 < 1 || M0 > kMaxM0 || M0 > N) return -3;
  HIPCHK(hipSetDevice(ctx->device));
  // the caller's [N][M0] layout is the packed layout with one cell of N rows
  HIPCHK(launch_random_start(seed, 1, (int)N, (int)N, M0, M0, Y, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return 0;
}

int feast_filter(feast_ctx *ctx, const feast_bt_matrix *AB, double emin, double emax,
                 int32_t M0, int32_t Ne, const double *Y, double *Q) {
  if (!ctx || !Y || !Q) return -5;
  int st = validate_matrix(AB);
  if (st) return st;
  if (!(emin < emax) || !std::isfinite(emin) || !std::isfinite(emax)) return -2;
  if (M0 < 1 || M0 > kMaxM0 || M0 > AB->nc * AB->b) return -3;
  if (Ne < 1 || Ne > kMaxNe) return -4;
  HIPCHK(hipSetDevice(ctx->device));
  Pencil p = make_pencil(AB);
  const int mp = round16(M0);
  Work wk;
  st = prepare_factor(ctx, p, Ne, mp, choose_parts(p.nc, Ne, 0), wk);
  if (st) return st;
  Shifts s;
  make_shifts(Ne, emin, emax, s);
  double *y, *r, *pp, *q;
  HIPCHK(ensure_t(ctx, S_Y, wk.rows * mp, &y));
  HIPCHK(ensure_t(ctx, S_R, wk.rows * mp, &r));
  HIPCHK(ensure_t(ctx, S_P, (size_t)Ne * wk.rows * mp, &pp));
  HIPCHK(ensure_t(ctx, S_Q, wk.rows * mp, &q));
  HIPCHK(run_factor(ctx, wk, s));
  HIPCHK(launch_pack(Y, p.nc, p.b, p.bp, M0, mp, y, ctx->stream));
  HIPCHK(launch_cell_apply(p, 1, y, mp, r, ctx->stream));
  HIPCHK(launch_sweeps(p, s, Ne, wk.f, wk.sb, r, mp, pp, 3, ctx->stream));
  HIPCHK(launch_sum_nodes(pp, Ne, wk.rows * mp, q, ctx->stream));
  HIPCHK(launch_unpack(q, p.nc, p.b, p.bp, M0, mp, nullptr, Q, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return 0;
}

int feast_project(feast_ctx *ctx, const feast_bt_matrix *AB, int32_t M0, const double *Q,
                  double *AQ, double *BQ) {
  if (!ctx || !Q || !AQ || !BQ) return -5;
  int st = validate_matrix(AB);
  if (st) return st;
  if (M0 < 1 || M0 > kMaxM0 || M0 > AB->nc * AB->b) return -3;
  HIPCHK(hipSetDevice(ctx->device));
  Pencil p = make_pencil(AB);
  const int mp = round16(M0);
  const size_t rows = (size_t)p.nc * p.bp;
  double *q, *gp;
  HIPCHK(ensure_t(ctx, S_Q, rows * mp, &q));
  HIPCHK(ensure_t(ctx, S_GRAMP, cell_partial_doubles(p.nc, mp), &gp));
  HIPCHK(launch_pack(Q, p.nc, p.b, p.bp, M0, mp, q, ctx->stream));
  HIPCHK(launch_cell_project(p, q, mp, M0, gp, AQ, BQ, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return 0;
}

int feast_reduced_eig(feast_ctx *ctx, int32_t M0, const double *AQ, const double *BQ,
                      double *eps, double *Phi, int32_t *fallback) {
  if (!ctx || !AQ || !BQ || !eps || !Phi) return -5;
  if (M0 < 1 || M0 > kMaxM0) return -3;
  HIPCHK(hipSetDevice(ctx->device));
  double *scr;
  int *flag;
  HIPCHK(ensure_t(ctx, S_RRS, reduced_eig_scratch_doubles(), &scr));
  HIPCHK(ensure_t(ctx, S_FLAG, 4, &flag));
  HIPCHK(launch_reduced_eig(AQ, BQ, M0, eps, Phi, scr, flag, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (fallback) *fallback = ctx->h_flag[0];
  return 0;
}

int feast_reduced_eig_noalloc(feast_ctx *ctx, int32_t M0, const double *AQ, const double *BQ,
                              double *eps, double *Phi, int32_t *fallback) {
  if (!ctx || !AQ || !BQ || !eps || !Phi) return -5;
  if (M0 < 1 || M0 > kMaxM0) return -3;
  if (!ctx->rr_static) return -5;
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(launch_reduced_eig(AQ, BQ, M0, eps, Phi, ctx->rr_static, ctx->rr_static_flag,
                            ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->h_flag, ctx->rr_static_flag, sizeof(int), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (fallback) *fallback = ctx->h_flag[0];
  return 0;
}


int feast_solve(feast_ctx *ctx, const feast_bt_matrix *AB, double emin, double emax, int32_t M0,
                int32_t Ne, const feast_opts *opts, double *lambda, double *X, double *res,
                feast_info *info) {
  if (!ctx || !lambda || !X || !res) return -5;
  // 64 < b <= 96: the wide kernels for the shifted systems and the products
  const bool wide = is_wide(AB);
  int st = wide ? validate_wide(AB) : validate_matrix(AB);
  if (st) return st;
  if (!(emin < emax) || !std::isfinite(emin) || !std::isfinite(emax)) return -2;
  const long long N = (long long)AB->nc * AB->b;
  if (M0 < 1 || M0 > kMaxM0 || M0 > N) return -3;
  if (Ne < 1 || Ne > kMaxNe) return -4;
  feast_opts o;
  feast_default_opts(&o);
  if (opts) o = *opts;
  if (!(o.tol > 0.0) || o.max_loops < 1 || o.precision < 0 || o.precision > 2 ||
      o.partitions < 0 || o.graph < 0 || o.graph > 2 || (o.graph == 2 && o.max_loops > 64) ||
      (wide && o.precision != 0))
    return -7;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t sm = ctx->stream;

  st = check_inputs(ctx, AB, o.Y0, (size_t)N * M0);
  if (st) return st;

  Pencil p = wide ? make_wide_pencil(AB) : make_pencil(AB);
  const int mp = round16(M0);
  Work wk{};
  WideWork ww{};
  if (wide)
    st = prepare_wide(ctx, p, Ne, mp, ww);
  else
    st = prepare_factor(ctx, p, Ne, mp, choose_parts(p.nc, Ne, o.partitions), wk);
  if (st) return st;
  const size_t rows = wide ? ww.rows : wk.rows;
  Shifts s;
  make_shifts(Ne, emin, emax, s);
  const double r = 0.5 * (emax - emin);

  double *y, *rr, *pp, *q, *x, *gp, *aq, *bq, *eps, *phi, *scr, *resp, *resi;
  int *flag, *perm;
  HIPCHK(ensure_t(ctx, S_Y, rows * mp, &y));
  HIPCHK(ensure_t(ctx, S_R, rows * mp, &rr));
  HIPCHK(ensure_t(ctx, S_P, (size_t)Ne * rows * mp, &pp));
  HIPCHK(ensure_t(ctx, S_Q, rows * mp, &q));
  HIPCHK(ensure_t(ctx, S_X, rows * mp, &x));
  HIPCHK(ensure_t(ctx, S_GRAMP,
                  wide ? cross_gram_partial_doubles((long long)rows, M0, M0)
                       : cell_partial_doubles(p.nc, mp),
                  &gp));
  HIPCHK(ensure_t(ctx, S_AQ, (size_t)M0 * M0, &aq));
  HIPCHK(ensure_t(ctx, S_BQ, (size_t)M0 * M0, &bq));
  HIPCHK(ensure_t(ctx, S_EPS, (size_t)M0, &eps));
  HIPCHK(ensure_t(ctx, S_PHI, (size_t)M0 * M0, &phi));
  HIPCHK(ensure_t(ctx, S_RRS, reduced_eig_scratch_doubles(), &scr));
  HIPCHK(ensure_t(ctx, S_FLAG, 4, &flag));
  HIPCHK(ensure_t(ctx, S_RESP,
                  wide ? wide_residual_partial_doubles(p.nc, mp) : cell_partial_doubles(p.nc, mp),
                  &resp));
  WidePack pk{};
  double *wtmp = nullptr;  // [rows][mp]: T Q of the wide projection
  if (wide) {
    pk = wide_pack_planes(p, ww.cpl);
    HIPCHK(ensure_t(ctx, S_T1, rows * mp, &wtmp));
  }
  // the products and sweeps of one loop, for the kernels of either block size
  auto bt_apply = [&](int which, const double *V, double *out, hipStream_t cs,
                      const int *skip) -> hipError_t {
    return wide ? launch_wide_apply(p, pk, which, V, mp, out, cs, skip)
                : launch_cell_apply(p, which, V, mp, out, cs, skip);
  };
  auto sweeps = [&](const double *R, double *P, int part, hipStream_t cs,
                    const int *skip) -> hipError_t {
    return wide ? launch_sweeps_wide(p, s, Ne, ww.f, ww.sb, R, mp, P, nullptr, part, cs, skip)
                : launch_sweeps(p, s, Ne, wk.f, wk.sb, R, mp, P, part, cs, skip);
  };
  auto project = [&](const double *Qm, hipStream_t cs, const int *skip) -> hipError_t {
    return wide ? launch_wide_project(p, pk, Qm, mp, M0, wtmp, gp, aq, bq, cs, skip)
                : launch_cell_project(p, Qm, mp, M0, gp, aq, bq, cs, skip);
  };
  auto residuals = [&](const double *Xm, hipStream_t cs, const int *skip) -> hipError_t {
    return wide ? launch_wide_residuals(p, pk, Xm, mp, eps, M0, emin, emax, resp, resi, cs, skip)
                : launch_cell_residuals(p, Xm, mp, eps, M0, emin, emax, resp, resi, cs, skip);
  };
  HIPCHK(ensure_t(ctx, S_RES, (size_t)M0, &resi));
  HIPCHK(ensure_t(ctx, S_PERM, (size_t)M0, &perm));

  // factor every shifted matrix once (Sec. V, parallelism (ii))
  if (wide)
    TIMED(K_FACTOR, launch_factor_wide(p, s, Ne, ww.f, ww.cpl, sm));
  else
    TIMED(K_FACTOR, run_factor(ctx, wk, s));
  const bool mixed = o.precision == 1;
  // precision 2: the first contour integration by one float32 solve per node
  // (no refinement; the random start carries no accuracy that a float32 solve
  // could lose), every later one in float64 from the same float64 factors
  const bool adaptive = o.precision == 2;
  Mixed mx;
  if (mixed || adaptive) {
    st = prepare_mixed(ctx, wk, mx);
    if (st) return st;
    TIMED(K_ROUND, launch_round_factors(p, Ne, wk.f, mx.f, sm));
  }
  if (o.Y0) {
    TIMED(K_LAYOUT, launch_pack(o.Y0, p.nc, p.b, p.bp, M0, mp, y, sm));
  } else {  // Fig. 2 step 1: M0 random vectors, seeded
    TIMED(K_LAYOUT, launch_random_start(o.seed, p.nc, p.b, p.bp, M0, mp, y, sm));
  }

  std::vector<double> traces;
  std::vector<int> counts;
  double trace_rel = INFINITY;
  bool converged = false;
  int fallback = 0;
  int rr_sweeps = 0;
  int refine_steps = 0;
  double solve_res = 0.0;
  double *h_eps = ctx->h_eps;
  double *h_res = ctx->h_eps + kMaxM0;
  const double res_gate = std::sqrt(o.tol);
  double prev_left_min = INFINITY;
  std::vector<char> is_counted(M0, 0);
  // graph = 1: loops 2, 3, ... replay one captured loop; it ends with a copy
  // Y <- X (in place of the pointer swap of the eager loop)
  const bool use_graph = o.graph == 1 && o.precision == 0;
  bool prev_f32 = false;  // the previous loop's Q came from float32 solves
  GraphExec gx;
  auto graph_body = [&](hipStream_t sm) -> hipError_t {
    hipError_t e;
    if ((e = bt_apply(1, y, rr, sm, nullptr)) != hipSuccess) return e;
    if ((e = sweeps(rr, pp, 1, sm, nullptr)) != hipSuccess) return e;
    if ((e = sweeps(rr, pp, 2, sm, nullptr)) != hipSuccess) return e;
    if ((e = launch_sum_nodes(pp, Ne, rows * mp, q, sm)) != hipSuccess) return e;
    if ((e = project(q, sm, nullptr)) != hipSuccess) return e;
    if ((e = launch_reduced_eig(aq, bq, M0, eps, phi, scr, flag, sm)) != hipSuccess) return e;
    if ((e = launch_gemm_qphi(q, rows, mp, M0, phi, x, sm)) != hipSuccess) return e;
    if ((e = residuals(x, sm, nullptr)) != hipSuccess) return e;
    return hipMemcpyAsync(y, x, rows * mp * sizeof(double), hipMemcpyDeviceToDevice, sm);
  };
  // graph = 2: the convergence decision on the device (launch_converge); the
  // loops are captured kChunk at a time into one graph whose kernels return at
  // once after convergence, and the host reads the decision once per chunk.
  // Y and X alternate between the two buffers (odd loops read y, write x).
  const bool dev_graph = o.graph == 2 && o.precision == 0;
  if (dev_graph) {
    constexpr int kChunk = 4;
    DevConv *cs_dev;
    HIPCHK(ensure_t(ctx, S_CONV, 1, &cs_dev));
    DevConv h{};
    h.trace_rel = INFINITY;
    h.prev_left_min = INFINITY;
    HIPCHK(hipMemcpyAsync(cs_dev, &h, sizeof(h), hipMemcpyHostToDevice, sm));
    HIPCHK(hipStreamSynchronize(sm));
    HIPCHK(reduced_eig_set_lds());
    const int *skip = &cs_dev->done;
    auto chunk = [&](hipStream_t cs) -> hipError_t {
      hipError_t e;
      for (int i = 0; i < kChunk; ++i) {
        const double *in = (i % 2 == 0) ? y : x;
        double *out = (i % 2 == 0) ? x : y;
        if ((e = bt_apply(1, in, rr, cs, skip)) != hipSuccess) return e;
        if ((e = sweeps(rr, pp, 1, cs, skip)) != hipSuccess) return e;
        if ((e = sweeps(rr, pp, 2, cs, skip)) != hipSuccess) return e;
        if ((e = launch_sum_nodes(pp, Ne, rows * mp, q, cs, skip)) != hipSuccess) return e;
        if ((e = project(q, cs, skip)) != hipSuccess) return e;
        if ((e = launch_reduced_eig(aq, bq, M0, eps, phi, scr, flag, cs, skip)) != hipSuccess)
          return e;
        if ((e = launch_gemm_qphi(q, rows, mp, M0, phi, out, cs, skip)) != hipSuccess) return e;
        if ((e = residuals(out, cs, skip)) != hipSuccess) return e;
        if ((e = launch_converge(eps, resi, flag, M0, emin, emax, res_gate, o.tol, r,
                                 kUncountedDrop, o.max_loops, cs_dev, cs)) != hipSuccess)
          return e;
      }
      return hipSuccess;
    };
    if (!ctx->capture)  // default priority
      HIPCHK(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
    HIPCHK(gx.capture(ctx->capture, chunk));
    for (int launched = 0;;) {
      HIPCHK(hipGraphLaunch(gx.exec, sm));
      launched += kChunk;
      HIPCHK(hipMemcpyAsync(&h, cs_dev, sizeof(h), hipMemcpyDeviceToHost, sm));
      HIPCHK(hipStreamSynchronize(sm));
      if (h.done || launched >= o.max_loops) break;
    }
    for (int i = 0; i < h.k && i < 64; ++i) {
      traces.push_back(h.traces[i]);
      counts.push_back(h.counts[i]);
      if (o.verbose)
        std::fprintf(stderr, "feast (device decision): loop %d  M %d  trace %.17g\n", i + 1,
                     h.counts[i], h.traces[i]);
    }
    converged = h.converged != 0;
    fallback = h.fallback;
    rr_sweeps = h.rr_sweeps;
    trace_rel = h.trace_rel;
    if (h.k % 2 == 0) std::swap(x, y);  // the last loop wrote y
    HIPCHK(hipMemcpyAsync(h_eps, eps, M0 * sizeof(double), hipMemcpyDeviceToHost, sm));
    HIPCHK(hipMemcpyAsync(h_res, resi, M0 * sizeof(double), hipMemcpyDeviceToHost, sm));
    HIPCHK(hipStreamSynchronize(sm));
    for (int j = 0; j < M0; ++j)
      is_counted[j] = h_eps[j] >= emin && h_eps[j] <= emax && h_res[j] <= res_gate;
  }
  for (int k = 1; k <= o.max_loops && !dev_graph; ++k) {
    if (use_graph && k >= 2) {
      if (!ctx->capture)  // default priority
        HIPCHK(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
      if (!gx.exec) HIPCHK(gx.capture(ctx->capture, graph_body));
      HIPCHK(hipGraphLaunch(gx.exec, sm));
    } else {
    TIMED(K_BTMUL, bt_apply(1, y, rr, sm, nullptr));                         // R = B Y
    const bool f32_loop = adaptive && k == 1;
    if (f32_loop) {  // Q_e by one float32 solve per node, then Q (eq. 15)
      TIMED(K_FWD32, launch_sweeps32(p, Ne, mx.f, mx.sb, rr, 0, 0, mp, mx.xc, 0, 1, sm));
      TIMED(K_BACK32, launch_sweeps32(p, Ne, mx.f, mx.sb, rr, 0, 0, mp, mx.xc, 0, 2, sm));
      TIMED(K_SUM, launch_sum_nodes_complex(s, Ne, mx.xc, mx.plane, q, sm));
      ++refine_steps;
    } else if (mixed) {  // Q_e by refined float32 solves, then Q (eq. 15)
      int steps = 0;
      double worst = 0.0;
      st = mixed_solve(ctx, wk, mx, s, rr, M0, &steps, &worst);
      if (st) return st;
      refine_steps += steps;
      solve_res = std::max(solve_res, worst);
      TIMED(K_SUM, launch_sum_nodes_complex(s, Ne, mx.xc, mx.plane, q, sm));
    } else {
      TIMED(K_FORWARD, sweeps(rr, pp, 1, sm, nullptr));                     // Q_e ...
      TIMED(K_BACK, sweeps(rr, pp, 2, sm, nullptr));                        // ... weighted
      TIMED(K_SUM, launch_sum_nodes(pp, Ne, rows * mp, q, sm));                 // Q (eq. 15)
    }
    TIMED(K_GRAM, project(q, sm, nullptr));                                // A_Q, B_Q (eq. 7)
    TIMED(K_RR, launch_reduced_eig(aq, bq, M0, eps, phi, scr, flag, sm));   // eq. 6
    TIMED(K_RITZ, launch_gemm_qphi(q, rows, mp, M0, phi, x, sm));           // X = Q Phi (eq. 9)
    // residuals of the Ritz pairs (Table I caption) decide which in-interval
    // pairs count as eigenvalue solutions (relative residual <= sqrt(tol))
    TIMED(K_RESID, residuals(x, sm, nullptr));
    }
    HIPCHK(hipMemcpyAsync(h_eps, eps, M0 * sizeof(double), hipMemcpyDeviceToHost, sm));
    HIPCHK(hipMemcpyAsync(h_res, resi, M0 * sizeof(double), hipMemcpyDeviceToHost, sm));
    HIPCHK(hipMemcpyAsync(ctx->h_flag, flag, 3 * sizeof(int), hipMemcpyDeviceToHost, sm));
    HIPCHK(hipStreamSynchronize(sm));
    fallback = ctx->h_flag[0];
    rr_sweeps += ctx->h_flag[1] + (fallback ? ctx->h_flag[2] : 0);
    int Mk = 0;
    double Tk = 0.0;
    double left_min = INFINITY;  // smallest residual of an uncounted in-interval pair
    for (int j = 0; j < M0; ++j) {
      const bool in = h_eps[j] >= emin && h_eps[j] <= emax;
      is_counted[j] = in && h_res[j] <= res_gate;
      if (is_counted[j]) {
        ++Mk;
        Tk += h_eps[j];
      } else if (in) {
        left_min = std::min(left_min, h_res[j]);
      }
    }
    // a true pair below the gate shrinks its residual every loop; a mixture of
    // eigenvectors from both sides of the interval does not
    const bool still_converging = left_min < kUncountedDrop * prev_left_min;
    prev_left_min = left_min;
    if (k >= 2) {
      if (Mk == 0 && counts.back() == 0)
        trace_rel = 0.0;
      else
        trace_rel = std::fabs(Tk - traces.back()) / std::max(std::fabs(Tk), Mk * r);
    }
    traces.push_back(Tk);
    counts.push_back(Mk);
    if (o.verbose)
      std::fprintf(stderr, "feast: loop %d  M %d  trace %.17g  trace change %.3e%s\n", k, Mk, Tk,
                   k >= 2 ? trace_rel : INFINITY, std::isfinite(left_min) ? "  (uncounted pairs inside)" : "");
    // (both traces of the test from float64 solves)
    const bool this_f32 = adaptive && k == 1;
    if (k >= 2 && Mk == counts[counts.size() - 2] && trace_rel < o.tol && !still_converging &&
        !prev_f32 && !this_f32) {
      converged = true;
      break;
    }
    prev_f32 = this_f32;
    if (k < o.max_loops && !use_graph) std::swap(y, x);  // Y <- X (Fig. 2 step 6)
    if (use_graph && k == 1)  // the graph's loops read Y from the same buffer
      HIPCHK(hipMemcpyAsync(y, x, rows * mp * sizeof(double), hipMemcpyDeviceToDevice, sm));
  }

  // order: counted pairs first (ascending), then the rest, NaN slots last
  std::vector<int> order;
  order.reserve(M0);
  for (int j = 0; j < M0; ++j)
    if (is_counted[j]) order.push_back(j);
  for (int j = 0; j < M0; ++j)
    if (std::isfinite(h_eps[j]) && !is_counted[j]) order.push_back(j);
  for (int j = 0; j < M0; ++j)
    if (!std::isfinite(h_eps[j])) order.push_back(j);
  int *h_perm = reinterpret_cast<int *>(ctx->h_eps + 2 * kMaxM0);
  for (int j = 0; j < M0; ++j) h_perm[j] = order[j];
  std::vector<double> res_sorted(M0);
  for (int j = 0; j < M0; ++j) res_sorted[j] = h_res[order[j]];
  HIPCHK(hipMemcpyAsync(perm, h_perm, M0 * sizeof(int), hipMemcpyHostToDevice, sm));
  TIMED(K_LAYOUT, launch_unpack(x, p.nc, p.b, p.bp, M0, mp, perm, X, sm));
  HIPCHK(launch_gather(eps, perm, M0, lambda, sm));
  HIPCHK(launch_gather(resi, perm, M0, res, sm));
  HIPCHK(hipStreamSynchronize(sm));

  const int M = counts.back();
  double max_res = 0.0;
  for (int j = 0; j < M; ++j) max_res = std::max(max_res, res_sorted[j]);
  int status;
  if (!converged) status = 1;
  else if (fallback) status = 2;
  else if (mixed && !(solve_res <= kRefineTol)) status = 5;
  else if (M == M0) status = 4;
  else if (M == 0) status = 3;
  else status = 0;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->loops = (int)traces.size();
    info->M = M;
    info->trace = traces.back();
    info->trace_rel = trace_rel;
    info->max_res = max_res;
    info->status = status;
    info->fallback = fallback;
    info->rr_sweeps = rr_sweeps;
    info->refine_steps = refine_steps;
    info->solve_res = solve_res;
    info->m0_small = 2 * M0 < 3 * M;  // M0 < 1.5 M
    for (size_t k = 0; k < traces.size() && k < 64; ++k) {
      info->trace_hist[k] = traces[k];
      info->count_hist[k] = counts[k];
    }
  }
  return status;
}


// ---- independent problems (Sec. V, parallelism level (i)) ----

namespace {

// Estimated device work of one problem (flops of the factorisation and of
// three refinement loops of sweeps), the key of the longest-first order.
double problem_cost(const feast_problem &q) {
  const double nc = q.AB.nc, b = q.AB.b;
  return q.Ne * nc * b * b * (b + 3.0 * q.M0);
}

}  // namespace

int feast_solve_batched(feast_ctx *ctx, feast_problem *probs, int32_t count,
                        const feast_opts *opts, int32_t workers) {
  if (!ctx || (!probs && count > 0)) return -5;
  if (count < 0 || workers < 0) return -7;
  if (count == 0) return 0;
  HIPCHK(hipSetDevice(ctx->device));
  // inputs produced on the caller's stream are complete before any worker starts
  HIPCHK(hipStreamSynchronize(ctx->stream));
  const int nw = std::max(1, std::min<int>(workers ? workers : 8, count));
  while ((int)ctx->workers.size() < nw) {
    hipStream_t st = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));  // default priority
    feast_ctx *w = nullptr;
    const int e = feast_init(&w, ctx->device, st);
    if (e) {
      (void)hipStreamDestroy(st);
      return e;
    }
    w->owns_stream = true;
    ctx->workers.push_back(w);
  }
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return problem_cost(probs[a]) > problem_cost(probs[b]);
  });
  feast_opts base;
  feast_default_opts(&base);
  if (opts) base = *opts;
  std::atomic<int> next{0};
  auto run = [&](feast_ctx *w) {
    (void)hipSetDevice(w->device);
    for (int k = next++; k < count; k = next++) {
      feast_problem &q = probs[order[k]];
      feast_opts o = base;
      o.Y0 = q.Y0;
      // automatic: one partition per half chain.  The problems fill the GPU
      // together, and the partitioned factorisation loses accuracy on some
      // problems with contour points close to the real axis: a partition cut
      // off from its neighbours can be nearly singular there, and its spike
      // columns, solved through its unpivoted local factorisation, carry the
      // error into the interface step (Ne = 16: residuals 1e-9 against 1e-12
      // with one partition)
      if (o.partitions == 0) o.partitions = 1;
      q.status = feast_solve(w, &q.AB, q.emin, q.emax, q.M0, q.Ne, &o, q.lambda, q.X, q.res,
                             q.info);
    }
  };
  std::vector<std::thread> threads;
  for (int t = 1; t < nw; ++t) threads.emplace_back(run, ctx->workers[t]);
  run(ctx->workers[0]);
  for (auto &t : threads) t.join();
  int worst_neg = 0, worst_pos = 0;
  for (int i = 0; i < count; ++i) {
    const int st = probs[i].status;
    if (st < 0 && worst_neg == 0) worst_neg = st;
    if (st > worst_pos) worst_pos = st;
  }
  return worst_neg ? worst_neg : worst_pos;
}

// ---- partition-count tuning ----

namespace {

// "nc b M0 Ne partitions ms" lines of a tuning cache; returns the cached
// partitions for the shape or 0.
int cache_lookup(const char *path, const char *arch, int nc, int b, int M0, int Ne) {
  if (!path) return 0;
  FILE *f = std::fopen(path, "r");
  if (!f) return 0;
  char a[64];
  int cnc, cb, cm, ce, cp;
  double ms;
  int found = 0;
  while (std::fscanf(f, "%63s %d %d %d %d %d %lf", a, &cnc, &cb, &cm, &ce, &cp, &ms) == 7)
    if (!std::strcmp(a, arch) && cnc == nc && cb == b && cm == M0 && ce == Ne) found = cp;
  std::fclose(f);
  return found;
}

}  // namespace

int feast_autotune_partitions(feast_ctx *ctx, const feast_bt_matrix *AB, double emin,
                              double emax, int32_t M0, int32_t Ne, const char *cache_path,
                              int32_t *partitions) {
  if (!ctx || !partitions) return -5;
  int st = validate_matrix(AB);
  if (st) return st;
  if (!(emin < emax) || !std::isfinite(emin) || !std::isfinite(emax)) return -2;
  if (M0 < 1 || M0 > kMaxM0 || M0 > (long long)AB->nc * AB->b) return -3;
  if (Ne < 1 || Ne > kMaxNe) return -4;
  HIPCHK(hipSetDevice(ctx->device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, ctx->device));
  char arch[64];
  std::snprintf(arch, sizeof(arch), "%s/%dcu", prop.gcnArchName, prop.multiProcessorCount);
  for (char *c = arch; *c; ++c)
    if (*c == ' ' || *c == ':') *c = '_';
  const int cached = cache_lookup(cache_path, arch, AB->nc, AB->b, M0, Ne);
  if (cached > 0) {
    *partitions = cached;
    return 0;
  }
  Pencil p = make_pencil(AB);
  const int mp = round16(M0);
  Shifts s;
  make_shifts(Ne, emin, emax, s);
  const int half = p.nc / 2;
  const int pmax = std::max(1, half / 8);  // at least 8 cells a partition
  std::vector<int> cand;
  for (int q = 1; q <= pmax; q *= 2) cand.push_back(q);
  if (cand.back() != pmax) cand.push_back(pmax);
  // accuracy probe: the contour point nearest the real axis (node 0; node
  // Ne-1 mirrors it), one shifted solve with a seeded random right-hand side
  Shifts s1;
  std::memset(&s1, 0, sizeof(s1));
  s1.zre[0] = s.zre[0];
  s1.zim[0] = s.zim[0];
  double ratio1 = 0.0;  // relative residual with one partition
  double *h_ratio = ctx->h_eps + 3 * kMaxM0;
  auto probe = [&](int q, double *ratio) -> int {
    Work w1;
    int st1 = prepare_factor(ctx, p, 1, mp, q, w1);
    if (st1) return st1;
    double *rin, *xc, *rc, *part, *worst;
    const size_t plane = w1.rows * mp;
    HIPCHK(ensure_t(ctx, S_R, plane, &rin));
    HIPCHK(ensure_t(ctx, S_XC, 2 * plane, &xc));
    HIPCHK(ensure_t(ctx, S_RC, 2 * plane, &rc));
    HIPCHK(ensure_t(ctx, S_RPART, shift_residual_partial_doubles(p.nc, mp, 1), &part));
    HIPCHK(ensure_t(ctx, S_WORST, 1, &worst));
    HIPCHK(launch_random_start(0, p.nc, p.b, p.bp, M0, mp, rin, ctx->stream));
    HIPCHK(run_factor(ctx, w1, s1));
    HIPCHK(launch_sweeps_complex(p, s1, w1.f, w1.sb, rin, mp, xc, xc + plane, ctx->stream));
    HIPCHK(launch_shift_residuals(p, s1, 1, xc, rin, mp, M0, rc, part, worst, ctx->stream));
    HIPCHK(hipMemcpyAsync(h_ratio, worst, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *ratio = *h_ratio;
    return 0;
  };
  hipEvent_t t0, t1;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  int best = 0;
  float best_ms = 0.0f;
  for (int q : cand) {
    double ratio = 0.0;
    st = probe(q, &ratio);
    if (st) break;
    if (q == 1) ratio1 = ratio;
    else if (!(ratio <= 10.0 * ratio1)) continue;  // loses accuracy near the axis
    Work wk;
    st = prepare_factor(ctx, p, Ne, mp, q, wk);
    if (st) break;
    double *r, *pp;
    hipError_t e = ensure_t(ctx, S_R, wk.rows * mp, &r);
    if (e == hipSuccess) e = ensure_t(ctx, S_P, (size_t)Ne * wk.rows * mp, &pp);
    if (e == hipSuccess) e = hipMemsetAsync(r, 0, wk.rows * mp * sizeof(double), ctx->stream);
    float ms = 0.0f;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {  // first run warms up
      if (e == hipSuccess) e = hipEventRecord(t0, ctx->stream);
      if (e == hipSuccess) e = run_factor(ctx, wk, s);
      if (e == hipSuccess) e = launch_sweeps(p, s, Ne, wk.f, wk.sb, r, mp, pp, 3, ctx->stream);
      if (e == hipSuccess) e = hipEventRecord(t1, ctx->stream);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float m = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&m, t0, t1);
      if (rep > 0) ms += m;
    }
    if (e != hipSuccess) {
      st = hip_status(e);
      break;
    }
    if (best == 0 || ms < best_ms) {
      best = q;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (st) return st;
  *partitions = best;
  if (cache_path) {
    FILE *f = std::fopen(cache_path, "a");
    if (f) {
      std::fprintf(f, "%s %d %d %d %d %d %.4f\n", arch, AB->nc, AB->b, M0, Ne, best,
                   best_ms / 2.0f);
      std::fclose(f);
    }
  }
  return 0;
}

}  // extern "C"


// ---- Hermitian A (Sec. III.B, eq. 12 and the changes listed after Fig. 2) ----

namespace {

int validate_hmatrix(const feast_zbt_matrix *AB) {
  if (!AB) return -5;
  if (AB->nc < 1 || AB->b < 1 || AB->b > kMaxHB) return -1;
  if (!AB->A_diag || !AB->B_diag) return -5;
  if (AB->nc > 1 && (!AB->A_up || !AB->B_up)) return -5;
  return 0;
}

HPencil make_hpencil(const feast_zbt_matrix *AB) {
  HPencil p;
  p.Ad = AB->A_diag;
  p.Au = AB->A_up;
  p.Bd = AB->B_diag;
  p.Bu = AB->B_up;
  p.nc = AB->nc;
  p.b = AB->b;
  return p;
}

int check_hinputs(feast_ctx *ctx, const feast_zbt_matrix *AB, const double *Y0, size_t ny) {
  int *flag = nullptr;
  HIPCHK(ensure_t(ctx, S_FLAG, 4, &flag));
  HIPCHK(hipMemsetAsync(flag, 0, 4 * sizeof(int), ctx->stream));
  const size_t bb = (size_t)AB->b * AB->b;
  HIPCHK(launch_check_finite(AB->A_diag, 2 * AB->nc * bb, flag, ctx->stream));
  HIPCHK(launch_check_finite(AB->B_diag, AB->nc * bb, flag, ctx->stream));
  if (AB->nc > 1) {
    HIPCHK(launch_check_finite(AB->A_up, 2 * (AB->nc - 1) * bb, flag, ctx->stream));
    HIPCHK(launch_check_finite(AB->B_up, (AB->nc - 1) * bb, flag, ctx->stream));
  }
  if (Y0) HIPCHK(launch_check_finite(Y0, ny, flag, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ctx->h_flag[0] ? -6 : 0;
}

// Factors of every node: Sinv, W, V (complex), and the partitions of the
// factorisation with their work area (b <= 64).
struct HFactors {
  double *Sinv, *W, *V, *work;
  int parts;
};

int prepare_hfactors(feast_ctx *ctx, const HPencil &p, int Ne, int partitions, HFactors &f) {
  const size_t bb2 = 2 * hfactor_block_elems(p.b);
  HIPCHK(ensure_t(ctx, S_HSINV, (size_t)Ne * p.nc * bb2, &f.Sinv));
  HIPCHK(ensure_t(ctx, S_HW, (size_t)Ne * p.nc * bb2, &f.W));
  HIPCHK(ensure_t(ctx, S_HV, (size_t)Ne * p.nc * bb2, &f.V));
  f.parts = p.b <= 64 ? choose_parts(p.nc, Ne, partitions) : 1;
  f.work = nullptr;
  if (f.parts > 1) HIPCHK(ensure_t(ctx, S_HFWORK, hfactor_work_doubles(p, Ne, f.parts), &f.work));
  return 0;
}

hipError_t run_hfactor(const HPencil &p, const Shifts &s, int Ne, const HFactors &f,
                       hipStream_t st) {
  return launch_hfactor(p, s, Ne, f.Sinv, f.W, f.V, f.parts, f.work, st);
}

// Eq. 12 for the complex right-hand side R [N][m]: Q [N][m].
int hfilter(feast_ctx *ctx, const HPencil &p, int Ne, const HFactors &f, const double *R, int m,
            const double *coef_dev, double *Q) {
  const size_t N = (size_t)p.nc * p.b;
  double *G;
  HIPCHK(ensure_t(ctx, S_HG, hsweep_work_doubles(p, Ne, m), &G));
  TIMED(K_HSWEEP, launch_hsweeps(p, Ne, f.Sinv, f.W, f.V, R, m, G, ctx->stream));
  TIMED(K_SUM, launch_haccumulate(G, Ne, N * m, coef_dev, coef_dev + kMaxNe, Q, ctx->stream));
  return 0;
}

// c_e = -(w_e / 4) r e^{i theta_e} = kappa_e / 2 (eq. 12), on the device.
int hcoefficients(feast_ctx *ctx, const Shifts &s, int Ne, double **coef) {
  HIPCHK(ensure_t(ctx, S_HCOEF, 2 * kMaxNe, coef));
  double h[2 * kMaxNe];
  for (int e = 0; e < Ne; ++e) {
    h[e] = 0.5 * s.kre[e];
    h[kMaxNe + e] = 0.5 * s.kim[e];
  }
  HIPCHK(hipMemcpyAsync(*coef, h, sizeof(h), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return 0;
}

}  // namespace

int feast_shifted_solve_hermitian(feast_ctx *ctx, const feast_zbt_matrix *AB, double z_re,
                                  double z_im, int32_t m, const double *R, int32_t adjoint,
                                  double *X, int32_t partitions) {
  if (!ctx || !R || !X) return -5;
  int st = validate_hmatrix(AB);
  if (st) return st;
  if (m < 1 || m > kMaxHM0) return -3;
  if (!(z_im > 0.0) || !std::isfinite(z_re) || !std::isfinite(z_im)) return -2;
  HIPCHK(hipSetDevice(ctx->device));
  HPencil p = make_hpencil(AB);
  const size_t N = (size_t)p.nc * p.b;
  Shifts s;
  std::memset(&s, 0, sizeof(s));
  s.zre[0] = z_re;
  s.zim[0] = z_im;
  HFactors f;
  if (partitions < 0) return -7;
  st = prepare_hfactors(ctx, p, 1, partitions, f);
  if (st) return st;
  double *G;
  HIPCHK(ensure_t(ctx, S_HG, hsweep_work_doubles(p, 1, m), &G));
  HIPCHK(run_hfactor(p, s, 1, f, ctx->stream));
  HIPCHK(launch_hsweeps(p, 1, f.Sinv, f.W, f.V, R, m, G, ctx->stream));
  HIPCHK(hipMemcpyAsync(X, G + (adjoint ? 2 * N * m : 0), 2 * N * m * sizeof(double),
                        hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return 0;
}

int feast_filter_hermitian(feast_ctx *ctx, const feast_zbt_matrix *AB, double emin, double emax,
                           int32_t M0, int32_t Ne, const double *Y, double *Q) {
  if (!ctx || !Y || !Q) return -5;
  int st = validate_hmatrix(AB);
  if (st) return st;
  if (!(emin < emax) || !std::isfinite(emin) || !std::isfinite(emax)) return -2;
  if (M0 < 1 || M0 > kMaxHM0) return -3;
  if (Ne < 1 || Ne > kMaxNe) return -4;
  HIPCHK(hipSetDevice(ctx->device));
  HPencil p = make_hpencil(AB);
  const size_t N = (size_t)p.nc * p.b;
  Shifts s;
  make_shifts(Ne, emin, emax, s);
  HFactors f;
  st = prepare_hfactors(ctx, p, Ne, 0, f);
  if (st) return st;
  double *coef, *R;
  st = hcoefficients(ctx, s, Ne, &coef);
  if (st) return st;
  HIPCHK(ensure_t(ctx, S_HR, N * M0 * 2, &R));
  HIPCHK(run_hfactor(p, s, Ne, f, ctx->stream));
  HIPCHK(launch_happly(p, 1, Y, M0, R, ctx->stream));  // R = B Y
  st = hfilter(ctx, p, Ne, f, R, M0, coef, Q);
  if (st) return st;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return 0;
}

namespace {

// FEAST loop on the complex kernels of herm.hip for a Hermitian A.  y0: the
// caller's complex start block or NULL for the seeded random start.
int generic_solve(feast_ctx *ctx, const HPencil &p, double emin, double emax, int M0, int Ne,
                  const feast_opts &o, const double *y0, double *lambda, double *X_out,
                  double *res, feast_info *info) {
  hipStream_t sm = ctx->stream;
  int st = 0;
  const long long N = (long long)p.nc * p.b;
  Shifts s;
  make_shifts(Ne, emin, emax, s);
  const double r = 0.5 * (emax - emin);
  HFactors f;
  st = prepare_hfactors(ctx, p, Ne, o.partitions, f);
  if (st) return st;
  double *coef;
  st = hcoefficients(ctx, s, Ne, &coef);
  if (st) return st;
  const size_t nm2 = (size_t)N * M0 * 2;
  const int n2 = 2 * M0;  // size of the real embedding of the reduced problem
  double *y, *rr, *q, *x, *ax, *bx, *part, *aq, *bq, *ea, *eb, *eps2, *phi2, *eps, *phi, *resi,
      *scr, *hz;
  int *flag, *perm;
  HIPCHK(ensure_t(ctx, S_HY, nm2, &y));
  HIPCHK(ensure_t(ctx, S_HR, nm2, &rr));
  HIPCHK(ensure_t(ctx, S_HQ, nm2, &q));
  HIPCHK(ensure_t(ctx, S_HX, nm2, &x));
  HIPCHK(ensure_t(ctx, S_HAX, nm2, &ax));
  HIPCHK(ensure_t(ctx, S_HBX, nm2, &bx));
  HIPCHK(ensure_t(ctx, S_HPART, hgram_partial_doubles(N, M0), &part));
  HIPCHK(ensure_t(ctx, S_HAQ, (size_t)M0 * M0 * 2, &aq));
  HIPCHK(ensure_t(ctx, S_HBQ, (size_t)M0 * M0 * 2, &bq));
  HIPCHK(ensure_t(ctx, S_HEA, (size_t)n2 * n2, &ea));
  HIPCHK(ensure_t(ctx, S_HEB, (size_t)n2 * n2, &eb));
  HIPCHK(ensure_t(ctx, S_HEPS2, (size_t)n2, &eps2));
  HIPCHK(ensure_t(ctx, S_HPHI2, (size_t)n2 * n2, &phi2));
  HIPCHK(ensure_t(ctx, S_HEPS, (size_t)M0, &eps));
  HIPCHK(ensure_t(ctx, S_HPHI, (size_t)M0 * M0 * 2, &phi));
  HIPCHK(ensure_t(ctx, S_HZ, (size_t)M0 * M0 * 2, &hz));
  HIPCHK(ensure_t(ctx, S_HRES, (size_t)M0, &resi));
  HIPCHK(ensure_t(ctx, S_RRS, reduced_eig_scratch_doubles(), &scr));
  HIPCHK(ensure_t(ctx, S_FLAG, 4, &flag));
  HIPCHK(ensure_t(ctx, S_PERM, (size_t)M0, &perm));

  TIMED(K_FACTOR, run_hfactor(p, s, Ne, f, sm));  // once (Sec. V, level (ii))
  if (y0) {
    HIPCHK(hipMemcpyAsync(y, y0, nm2 * sizeof(double), hipMemcpyDeviceToDevice, sm));
  } else {  // real and imaginary parts N(0, 1): the real draw of N x 2 M0
    HIPCHK(launch_random_start(o.seed, 1, (int)N, (int)N, 2 * M0, 2 * M0, y, sm));
  }
  std::vector<double> traces;
  std::vector<int> counts;
  double trace_rel = INFINITY;
  bool converged = false;
  int fallback = 0, rr_sweeps = 0;
  double *h_eps = ctx->h_eps;
  double *h_res = ctx->h_eps + kMaxM0;
  const double res_gate = std::sqrt(o.tol);
  double prev_left_min = INFINITY;
  std::vector<char> is_counted(M0, 0);
  for (int k = 1; k <= o.max_loops; ++k) {
    TIMED(K_BTMUL, launch_happly(p, 1, y, M0, rr, sm));                // R = B Y
    st = hfilter(ctx, p, Ne, f, rr, M0, coef, q);                      // Q (eq. 12)
    if (st) return st;
    TIMED(K_GRAM, launch_happly_pair(p, q, M0, ax, bx, sm));          // A Q, B Q
    TIMED(K_GRAM, launch_hgram(q, ax, N, M0, part, aq, sm));           // A_Q = Q^H A Q
    TIMED(K_GRAM, launch_hgram(q, bx, N, M0, part, bq, sm));           // B_Q = Q^H B Q
    // a real symmetric tridiagonal problem of size M0 for the real eigensolver
    TIMED(K_RR, launch_htridiag(aq, bq, M0, ea, eb, hz, scr, flag, sm));
    HIPCHK(hipMemcpyAsync(ctx->h_flag + 3, flag + 3, sizeof(int), hipMemcpyDeviceToHost, sm));
    HIPCHK(hipStreamSynchronize(sm));
    if (!ctx->h_flag[3]) {
      TIMED(K_RR, launch_reduced_eig(ea, eb, M0, eps, phi2, scr, flag, sm));
      TIMED(K_RR, launch_hcombine(hz, phi2, M0, phi, sm));
    } else {  // B_Q fails the Cholesky test: the real embedding and its fallback
      TIMED(K_RR, launch_hembed(aq, bq, M0, ea, eb, sm));
      TIMED(K_RR, launch_reduced_eig(ea, eb, n2, eps2, phi2, scr, flag, sm));
      TIMED(K_RR, launch_hextract(eps2, phi2, M0, eps, phi, sm));
    }
    TIMED(K_RITZ, launch_htall_gemm(q, phi, N, M0, M0, x, sm));       // X = Q Phi
    TIMED(K_RESID, launch_happly_pair(p, x, M0, ax, bx, sm));        // A X, B X
    TIMED(K_RESID, launch_hresiduals(ax, bx, eps, N, M0, emin, emax, part, resi, sm));
    HIPCHK(hipMemcpyAsync(h_eps, eps, M0 * sizeof(double), hipMemcpyDeviceToHost, sm));
    HIPCHK(hipMemcpyAsync(h_res, resi, M0 * sizeof(double), hipMemcpyDeviceToHost, sm));
    HIPCHK(hipMemcpyAsync(ctx->h_flag, flag, 3 * sizeof(int), hipMemcpyDeviceToHost, sm));
    HIPCHK(hipStreamSynchronize(sm));
    fallback = ctx->h_flag[0];
    rr_sweeps += ctx->h_flag[1] + (fallback ? ctx->h_flag[2] : 0);
    int Mk = 0;
    double Tk = 0.0, left_min = INFINITY;
    for (int j = 0; j < M0; ++j) {
      const bool in = h_eps[j] >= emin && h_eps[j] <= emax;
      is_counted[j] = in && h_res[j] <= res_gate;
      if (is_counted[j]) {
        ++Mk;
        Tk += h_eps[j];
      } else if (in) {
        left_min = std::min(left_min, h_res[j]);
      }
    }
    const bool still_converging = left_min < kUncountedDrop * prev_left_min;
    prev_left_min = left_min;
    if (k >= 2) {
      if (Mk == 0 && counts.back() == 0)
        trace_rel = 0.0;
      else
        trace_rel = std::fabs(Tk - traces.back()) / std::max(std::fabs(Tk), Mk * r);
    }
    traces.push_back(Tk);
    counts.push_back(Mk);
    if (o.verbose)
      std::fprintf(stderr, "feast (%s): loop %d  M %d  trace %.17g  trace change %.3e\n",
                   "Hermitian", k, Mk, Tk, k >= 2 ? trace_rel : INFINITY);
    if (k >= 2 && Mk == counts[counts.size() - 2] && trace_rel < o.tol && !still_converging) {
      converged = true;
      break;
    }
    if (k < o.max_loops) std::swap(y, x);  // Y <- X
  }
  std::vector<int> order;
  order.reserve(M0);
  for (int j = 0; j < M0; ++j)
    if (is_counted[j]) order.push_back(j);
  for (int j = 0; j < M0; ++j)
    if (std::isfinite(h_eps[j]) && !is_counted[j]) order.push_back(j);
  for (int j = 0; j < M0; ++j)
    if (!std::isfinite(h_eps[j])) order.push_back(j);
  int *h_perm = reinterpret_cast<int *>(ctx->h_eps + 2 * kMaxM0);
  for (int j = 0; j < M0; ++j) h_perm[j] = order[j];
  std::vector<double> res_sorted(M0);
  for (int j = 0; j < M0; ++j) res_sorted[j] = h_res[order[j]];
  HIPCHK(hipMemcpyAsync(perm, h_perm, M0 * sizeof(int), hipMemcpyHostToDevice, sm));
  HIPCHK(launch_hgather(x, perm, N, M0, X_out, sm));
  HIPCHK(launch_gather(eps, perm, M0, lambda, sm));
  HIPCHK(launch_gather(resi, perm, M0, res, sm));
  HIPCHK(hipStreamSynchronize(sm));
  const int M = counts.back();
  double max_res = 0.0;
  for (int j = 0; j < M; ++j) max_res = std::max(max_res, res_sorted[j]);
  int status;
  if (!converged) status = 1;
  else if (fallback) status = 2;
  else if (M == M0) status = 4;
  else if (M == 0) status = 3;
  else status = 0;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->loops = (int)traces.size();
    info->M = M;
    info->trace = traces.back();
    info->trace_rel = trace_rel;
    info->max_res = max_res;
    info->status = status;
    info->fallback = fallback;
    info->rr_sweeps = rr_sweeps;
    info->m0_small = 2 * M0 < 3 * M;  // M0 < 1.5 M
    for (size_t k = 0; k < traces.size() && k < 64; ++k) {
      info->trace_hist[k] = traces[k];
      info->count_hist[k] = counts[k];
    }
  }
  return status;
}

}  // namespace

int feast_solve_hermitian(feast_ctx *ctx, const feast_zbt_matrix *AB, double emin, double emax,
                          int32_t M0, int32_t Ne, const feast_opts *opts, double *lambda,
                          double *X, double *res, feast_info *info) {
  if (!ctx || !lambda || !X || !res) return -5;
  int st = validate_hmatrix(AB);
  if (st) return st;
  if (!(emin < emax) || !std::isfinite(emin) || !std::isfinite(emax)) return -2;
  const long long N = (long long)AB->nc * AB->b;
  if (M0 < 1 || M0 > kMaxHM0 || M0 > N) return -3;
  if (Ne < 1 || Ne > kMaxNe) return -4;
  feast_opts o;
  feast_default_opts(&o);
  if (opts) o = *opts;
  if (!(o.tol > 0.0) || o.max_loops < 1 || o.precision != 0 || o.partitions < 0) return -7;
  HIPCHK(hipSetDevice(ctx->device));
  st = check_hinputs(ctx, AB, o.Y0, (size_t)N * M0 * 2);
  if (st) return st;
  return generic_solve(ctx, make_hpencil(AB), emin, emax, M0, Ne, o, o.Y0, lambda, X, res, info);
}



