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
// fly from the real blocks.  The inverse of a complex symmetric block is
// complex symmetric, so every computed inverse is symmetrised and Sinv may be
// read transposed.  The factors are
// computed once per solve and reused by every refinement loop (Sec. V,
// parallelism (ii)).
#include <algorithm>
#include <vector>

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
};

// slot <- z*Bblk - Ablk (or its transpose), identity padding on the diagonal,
// by NTH threads (tid = 0 .. NTH-1).
template <int BP, int NTH = kThreads>
__device__ void form_block(double *slot, const double *Ablk, const double *Bblk, int b,
                           double zr, double zi, bool transpose, bool diag_pad,
                           int tid = threadIdx.x) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  constexpr int NE = (BP * BP + NTH - 1) / NTH;
  // all loads first (consecutive threads read consecutive memory; a
  // transposed block is transposed on the way into LDS), then the stores
  double av[NE], bv[NE];
#pragma unroll
  for (int t = 0; t < NE; ++t) {
    const int idx = tid + t * NTH;
    const int x = idx / BP, y = idx % BP;  // memory row x, column y
    const bool in = idx < BP * BP && x < b && y < b;
    av[t] = in ? Ablk[x * b + y] : 0.0;
    bv[t] = in ? Bblk[x * b + y] : 0.0;
  }
#pragma unroll
  for (int t = 0; t < NE; ++t) {
    const int idx = tid + t * NTH;
    if (idx < BP * BP) {
      const int x = idx / BP, y = idx % BP;
      const int r = transpose ? y : x, c = transpose ? x : y;
      const bool in = x < b && y < b;
      slot[r * LD + c] = in ? zr * bv[t] - av[t] : ((diag_pad && r == c) ? 1.0 : 0.0);
      slot[PLANE + r * LD + c] = in ? zi * bv[t] : 0.0;
    }
  }
}

// Real blocks staged in registers (issued early, consumed after the
// Gauss-Jordan elimination so that the loads overlap it).
template <int BP>
struct BlockRegs {
  static constexpr int NE = (BP * BP + kThreads - 1) / kThreads;
  double a[NE], b[NE];
};

template <int BP>
__device__ __forceinline__ void block_regs_load(BlockRegs<BP> &g, const double *Ablk,
                                                const double *Bblk, int b, bool transpose) {
#pragma unroll
  for (int i = 0; i < BlockRegs<BP>::NE; ++i) {
    const int idx = threadIdx.x + kThreads * i;
    const int r = idx / BP, c = idx % BP;
    double av = 0.0, bv = 0.0;
    if (idx < BP * BP && r < b && c < b) {
      const int src = transpose ? c * b + r : r * b + c;
      av = Ablk[src];
      bv = Bblk[src];
    }
    g.a[i] = av;
    g.b[i] = bv;
  }
}

// slot <- z*B - A from staged registers (coupling block: zero padding).
template <int BP>
__device__ __forceinline__ void block_regs_store(double *slot, const BlockRegs<BP> &g, double zr,
                                                 double zi) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
#pragma unroll
  for (int i = 0; i < BlockRegs<BP>::NE; ++i) {
    const int idx = threadIdx.x + kThreads * i;
    if (idx < BP * BP) {
      const int r = idx / BP, c = idx % BP;
      slot[r * LD + c] = zr * g.b[i] - g.a[i];
      slot[PLANE + r * LD + c] = zi * g.b[i];
    }
  }
}

// Diagonal block in the accumulator layout, staged in registers.
template <int BP>
struct DiagRegs {
  double a[BP / 16][4], b[BP / 16][4];
};

template <int BP>
__device__ __forceinline__ void diag_regs_load(DiagRegs<BP> &g, const double *Ablk,
                                               const double *Bblk, int b) {
  constexpr int NT = BP / 16;
  const int w = wave_id(), l = lane_id();
  if (w >= NT) return;
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + acc_row(l, r), col = tj * 16 + acc_col(l);
      const bool in = row < b && col < b;
      g.a[tj][r] = in ? Ablk[row * b + col] : 0.0;
      g.b[tj][r] = in ? Bblk[row * b + col] : 0.0;
    }
}

// Position of element (r, c) in a global block plane: row-major, or the
// factor layout fpos of the factorisation's own blocks (FL).
template <int BP, bool FL>
__device__ __forceinline__ int gpos(int r, int c) {
  if constexpr (FL) return fpos<BP>(r, c);
  else return r * BP + c;
}

// slot <- complex block from global planes [2][BP][BP].
template <int BP, bool FL, int NTH = kThreads>
__device__ void load_block(double *slot, const double *g) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  for (int idx = threadIdx.x; idx < BP * BP; idx += NTH) {
    int r = idx / BP, c = idx % BP;
    const int gi = gpos<BP, FL>(r, c);
    slot[r * LD + c] = g[gi];
    slot[PLANE + r * LD + c] = g[BP * BP + gi];
  }
}

// slot -> global block in the factor layout fpos, consecutive threads on
// consecutive addresses: element gi of a plane holds (i, j) with
// j = (gi / 2) % BP, R = (gi / 2) / BP, i = 8 (R / 4) + 4 (gi % 2) + R % 4.
template <int BP, int NTH = kThreads>
__device__ void store_block_fl(double *g, const double *slot, bool transpose) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  for (int gi = threadIdx.x; gi < BP * BP; gi += NTH) {
    const int j = (gi >> 1) % BP, R = (gi >> 1) / BP;
    const int i = ((R >> 2) << 3) + ((gi & 1) << 2) + (R & 3);
    const int s = transpose ? j * LD + i : i * LD + j;
    g[gi] = slot[s];
    g[BP * BP + gi] = slot[PLANE + s];
  }
}

template <int BP, bool FL>
__device__ void store_block(double *g, const double *slot, bool transpose) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  for (int idx = threadIdx.x; idx < BP * BP; idx += kThreads) {
    int r = idx / BP, c = idx % BP;
    int s = transpose ? c * LD + r : r * LD + c;
    const int gi = gpos<BP, FL>(r, c);
    g[gi] = slot[s];
    g[BP * BP + gi] = slot[PLANE + s];
  }
}

// In-place inverse of a 16x16 complex tile (LDS, planes re/im with row
// stride ld) by one wave: Gauss-Jordan elimination without pivoting, the
// tile held in registers (lane l: row l%16, columns 4(l/16)..4(l/16)+3).
// At step j the pivot row reaches every lane of a 16-lane row through the
// DPP broadcast of lane j (no LDS), the pivot through the scalar unit, and
// each row's column-j entry (held in another 16-lane row) through a lane
// shuffle of one complex value.  The division of a pivot row by its pivot
// is deferred to one scaling of every row at the end (row j keeps its values
// times a_jj; later steps act on rows linearly, so the scaling commutes with
// them), which leaves one complex multiply-add per element and step.
__device__ __forceinline__ double readlane_d(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

template <int J>
__device__ __forceinline__ double row_bcast_j(double x) {  // DPP row_newbcast:J
  return __builtin_amdgcn_mov_dpp(x, 0x150 + J, 0xF, 0xF, false);
}

// lane J of each 16-lane row, to the whole row (J a constant after unrolling)
__device__ __forceinline__ double row_bcast(double x, int j) {
  switch (j) {
    case 0: return row_bcast_j<0>(x);
    case 1: return row_bcast_j<1>(x);
    case 2: return row_bcast_j<2>(x);
    case 3: return row_bcast_j<3>(x);
    case 4: return row_bcast_j<4>(x);
    case 5: return row_bcast_j<5>(x);
    case 6: return row_bcast_j<6>(x);
    case 7: return row_bcast_j<7>(x);
    case 8: return row_bcast_j<8>(x);
    case 9: return row_bcast_j<9>(x);
    case 10: return row_bcast_j<10>(x);
    case 11: return row_bcast_j<11>(x);
    case 12: return row_bcast_j<12>(x);
    case 13: return row_bcast_j<13>(x);
    case 14: return row_bcast_j<14>(x);
    default: return row_bcast_j<15>(x);
  }
}

__device__ __forceinline__ void inv16_wave(double *Xr, double *Xi, int ld) {
  const int l = lane_id();
  const int r = l & 15, g = l >> 4, cb = 4 * g;
  double ar[4], ai[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    ar[v] = Xr[r * ld + cb + v];
    ai[v] = Xi[r * ld + cb + v];
  }
  cplx srow{1.0, 0.0};  // deferred scale of my row: 1 / its pivot
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int vj = j & 3, jg = j >> 2;
    const int pl = j + 16 * jg;                  // lane holding (j, j)
    const cplx piv = crecip_fast(cplx{readlane_d(ar[vj], pl), readlane_d(ai[vj], pl)});
    cplx rj[4];                                  // row j (unscaled), my columns
#pragma unroll
    for (int v = 0; v < 4; ++v) rj[v] = cplx{row_bcast(ar[v], j), row_bcast(ai[v], j)};
    const int cl = r + 16 * jg;                  // lane holding my row, column j
    const cplx cj{__shfl(ar[vj], cl), __shfl(ai[vj], cl)};
    const bool me = r == j;
    cplx m = cmul(cj, piv);                      // a_rj / a_jj; 0 for row j itself
    if (me) m = cplx{0.0, 0.0};
#pragma unroll
    for (int v = 0; v < 4; ++v) {  // a_rc -= (a_rj / a_jj) a_jc
      ar[v] = fma(m.im, rj[v].im, fma(-m.re, rj[v].re, ar[v]));
      ai[v] = fma(-m.im, rj[v].re, fma(-m.re, rj[v].im, ai[v]));
    }
    if (g == jg) {  // column j: -a_rj / a_jj, and 1 in row j (scaled at the end)
      ar[vj] = me ? 1.0 : -m.re;
      ai[vj] = me ? 0.0 : -m.im;
    }
    if (me) srow = piv;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const cplx x = cmul(cplx{ar[v], ai[v]}, srow);
    Xr[r * ld + cb + v] = x.re;
    Xi[r * ld + cb + v] = x.im;
  }
}

// One 16x16 complex tile on the matrix cores, operands in LDS:
//   acc += sign * X(16 x 16) * Y(16 x 16),
// X and Y point at the tile origins of their re planes (im plane at +PLANE).
template <int BP>
__device__ __forceinline__ void tile_cgemm16(d4 &accr, d4 &acci, const double *X, const double *Y,
                                             double sign) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  const int l = lane_id();
  const int row = l & 15, kl = l >> 4;
#pragma unroll
  for (int k0 = 0; k0 < 16; k0 += 4) {
    const int k = k0 + kl;
    const double xr = sign * X[row * LD + k], xi = sign * X[PLANE + row * LD + k];
    const double yr = Y[k * LD + row], yi = Y[PLANE + k * LD + row];
    accr = mfma(xr, yr, accr);
    accr = mfma(-xi, yi, accr);
    acci = mfma(xr, yi, acci);
    acci = mfma(xi, yr, acci);
  }
}

template <int BP>
__device__ __forceinline__ void tile_load(d4 &accr, d4 &acci, const double *T) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  const int l = lane_id();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    accr[r] = T[acc_row(l, r) * LD + acc_col(l)];
    acci[r] = T[PLANE + acc_row(l, r) * LD + acc_col(l)];
  }
}

template <int BP>
__device__ __forceinline__ void tile_store(double *T, const d4 &accr, const d4 &acci) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  const int l = lane_id();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    T[acc_row(l, r) * LD + acc_col(l)] = accr[r];
    T[PLANE + acc_row(l, r) * LD + acc_col(l)] = acci[r];
  }
}

// In-place inverse of the complex block in slot A by block Gauss-Jordan
// elimination with 16-wide panels, without pivoting (every leading principal
// minor of a complex symmetric matrix with positive definite imaginary part
// is non-zero, and so is every diagonal block of its Schur complements).
// For panel K with P = S_KK^{-1}:
//   S_KJ <- P S_KJ (J != K);  S_IJ <- S_IJ - S_IK S_KJ,  S_IK <- -S_IK P (I != K);
//   S_KK <- P.
// The diagonal inverse runs in one wave; the panel products on the matrix
// cores.  The result is left in slot A and, if gout != nullptr, written to
// global memory.  While wave 0 inverts the first diagonal tile, waves 1-3
// run side() (work that does not touch slot A).
struct NoSide {
  __device__ void operator()() const {}
};

// NW waves run the elimination (at least NB - 1 of them: the row panel has a
// wave per tile); the block sits in the LDS slot A.
template <int BP, int NW, class Side = NoSide>
__device__ __forceinline__ void gj_invert_slot(double *A, double *gout, Side side = Side(),
                                               bool symm = true) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE, NB = BP / 16;
  static_assert(NW >= NB - 1 && NW >= 2, "one wave per tile of the row panel");
  const int w = wave_id();
  auto tile = [&](int bi, int bj) { return A + (bi * 16) * LD + bj * 16; };
  // The next pivot tile (kb+1, kb+1) is updated first, by wave 0, which then
  // inverts it while waves 1-3 update the other tiles (look-ahead): the
  // one-wave inverse overlaps the panel update instead of idling three waves.
  if (w == 0)
    inv16_wave(tile(0, 0), tile(0, 0) + PLANE, LD);
  else
    side();
  auto panel = [&](int kb) {
    __syncthreads();
    if constexpr (NB > 1) {
      // row panel S_KJ <- P S_KJ
      d4 rr = d4zero(), ri = d4zero();
      int jb = -1;
      if (w < NB - 1) {
        jb = w < kb ? w : w + 1;
        tile_cgemm16<BP>(rr, ri, tile(kb, kb), tile(kb, jb), 1.0);
      }
      __syncthreads();
      if (jb >= 0) tile_store<BP>(tile(kb, jb), rr, ri);
      __syncthreads();
      // trailing tiles and column panel: tile t of the (NB-1) x NB tiles off
      // row kb (rows bi != kb in order, all columns)
      constexpr int NT = (NB - 1) * NB;
      const bool look = kb + 1 < NB;
      const int tnext = kb * NB + kb + 1;  // tile (kb+1, kb+1): row index kb (= kb+1 - 1)
      auto tile_of = [&](int t, int &bi, int &j0) {
        const int i0 = t / NB;
        j0 = t % NB;
        bi = i0 < kb ? i0 : i0 + 1;
      };
      auto update = [&](int bi, int j0, d4 &tr, d4 &ti) {
        if (j0 == kb) {
          tr = d4zero();
          ti = d4zero();
          tile_cgemm16<BP>(tr, ti, tile(bi, kb), tile(kb, kb), -1.0);
        } else {
          tile_load<BP>(tr, ti, tile(bi, j0));
          tile_cgemm16<BP>(tr, ti, tile(bi, kb), tile(kb, j0), -1.0);
        }
      };
      if (look && w == 0) {
        d4 tr, ti;
        update(kb + 1, kb + 1, tr, ti);
        tile_store<BP>(tile(kb + 1, kb + 1), tr, ti);
        // (no other tile of this phase reads tile (kb+1, kb+1))
        inv16_wave(tile(kb + 1, kb + 1), tile(kb + 1, kb + 1) + PLANE, LD);
      }
      // the other tiles over waves 1.. (look-ahead) or all waves
      constexpr int PER = NT > 0 ? (NT + NW - 2) / (NW - 1) : 1;
      d4 tr[PER], ti[PER];
      int ib[PER], jbb[PER];
      const int nw = look ? NW - 1 : NW, wi = look ? w - 1 : w;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        ib[q] = -1;
        if (wi < 0) continue;
        int t = wi + nw * q;
        if (look && t >= tnext) ++t;  // skip the look-ahead tile
        if (t < NT) {
          int bi, j0;
          tile_of(t, bi, j0);
          ib[q] = bi;
          jbb[q] = j0;
          update(bi, j0, tr[q], ti[q]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PER; ++q)
        if (ib[q] >= 0) tile_store<BP>(tile(ib[q], jbb[q]), tr[q], ti[q]);
    }
  };
  if constexpr (NW == 4) {
    for (int kb = 0; kb < NB; ++kb) panel(kb);
  } else {  // a rolled loop keeps the wide block's tile addresses out of registers
#pragma unroll 1
    for (int kb = 0; kb < NB; ++kb) panel(kb);
  }
  __syncthreads();
  // S <- (S + S^T) / 2 (the inverse of a complex symmetric block is complex
  // symmetric; the sweeps read Sinv U transposed as U^T Sinv, which holds
  // only to the asymmetry of the computed inverse, and that grows with its
  // condition number near the real axis)
  if (symm && (NW != 4 || BP > 64)) {  // by pairs (r < c), each pair by one thread
    for (int idx = threadIdx.x; idx < BP * BP; idx += 64 * NW) {
      const int r = idx / BP, c = idx % BP;
      if (r < c) {
        const double ar = 0.5 * (A[r * LD + c] + A[c * LD + r]);
        const double ai = 0.5 * (A[PLANE + r * LD + c] + A[PLANE + c * LD + r]);
        A[r * LD + c] = ar;
        A[c * LD + r] = ar;
        A[PLANE + r * LD + c] = ai;
        A[PLANE + c * LD + r] = ai;
      }
    }
    __syncthreads();
  } else if (symm) {  // by 4x4 patches, 256 threads
    const int t = threadIdx.x;
    const int pi = t >> 4, pj = t & 15;
    const bool act = (4 * pi < BP) && (4 * pj < BP);
    double ar[4][4], ai[4][4];
    if (act) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 4 * pi + u, c = 4 * pj + v;
          ar[u][v] = 0.5 * (A[r * LD + c] + A[c * LD + r]);
          ai[u][v] = 0.5 * (A[PLANE + r * LD + c] + A[PLANE + c * LD + r]);
        }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 4 * pi + u, c = 4 * pj + v;
          A[r * LD + c] = ar[u][v];
          A[PLANE + r * LD + c] = ai[u][v];
        }
    }
    __syncthreads();
  }
  if (gout) store_block_fl<BP, 64 * NW>(gout, A, false);  // a block of Sinv: factor layout
  __syncthreads();
}

template <int BP, class Side = NoSide>
__device__ __forceinline__ void gj_invert(Lds<BP> &s, double *gout, Side side = Side(),
                                          bool symm = true) {
  gj_invert_slot<BP, kThreads / 64>(s.A, gout, side, symm);
}

// Complex product on the matrix cores, operands in LDS slots:
//   acc (+)= sign * op(X) * op(Y),   op(Z) = Z or Z^T.
// Wave w (< BP/16) owns row block w and all column blocks; acc[tj] holds
// the re / im 16x16 tiles.  Three real products per complex one: with
// x = sign*X,  T1 = x_re (y_re + y_im),  T2 = y_im (x_re + x_im),
// T3 = y_re (x_im - x_re),  the product is (T1 - T2) + i (T1 + T3); T1 sits
// in an accumulator of its own and is added to both parts at the end.
template <int BP>
__device__ __forceinline__ void cgemm_lds(d4 (&accr)[BP / 16], d4 (&acci)[BP / 16], const double *X,
                                          bool transX, const double *Y, double sign,
                                          bool transY = false) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE, NT = BP / 16;
  const int w = wave_id(), l = lane_id();
  if (w >= NT) return;
  const int row = w * 16 + (l & 15);
  const int kl = l >> 4;
  d4 t1[NT];
#pragma unroll
  for (int tj = 0; tj < NT; ++tj) t1[tj] = d4zero();
#pragma unroll  // a rolled loop moves the accumulators between register files each trip
  for (int k0 = 0; k0 < BP; k0 += 4) {
    const int k = k0 + kl;
    const int xa = transX ? k * LD + row : row * LD + k;
    const double xr = sign * X[xa], xi = sign * X[PLANE + xa];
    const double xs = -(xr + xi), xd = xi - xr;
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) {
      const int yb = transY ? (tj * 16 + (l & 15)) * LD + k : k * LD + tj * 16 + (l & 15);
      const double yr = Y[yb], yi = Y[PLANE + yb];
      t1[tj] = mfma(xr, yr + yi, t1[tj]);
      accr[tj] = mfma(xs, yi, accr[tj]);
      acci[tj] = mfma(xd, yr, acci[tj]);
    }
  }
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      accr[tj][q] += t1[tj][q];
      acci[tj][q] += t1[tj][q];
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

template <int BP, bool FL>
__device__ void acc_to_global(double *g, const d4 (&accr)[BP / 16], const d4 (&acci)[BP / 16]) {
  constexpr int NT = BP / 16;
  const int w = wave_id(), l = lane_id();
  if (w >= NT) return;
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + acc_row(l, r), col = tj * 16 + acc_col(l);
      const int gi = gpos<BP, FL>(row, col);
      g[gi] = accr[tj][r];
      g[BP * BP + gi] = acci[tj][r];
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
__device__ __forceinline__ void acc_from_diag_regs(d4 (&accr)[BP / 16], d4 (&acci)[BP / 16],
                                                   const DiagRegs<BP> &g, int b, double zr,
                                                   double zi) {
  constexpr int NT = BP / 16;
  const int w = wave_id(), l = lane_id();
  if (w >= NT) return;
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + acc_row(l, r), col = tj * 16 + acc_col(l);
      const bool in = row < b && col < b;
      accr[tj][r] = in ? zr * g.b[tj][r] - g.a[tj][r] : (row == col ? 1.0 : 0.0);
      acci[tj][r] = in ? zi * g.b[tj][r] : 0.0;
    }
}

template <int BP, bool FL>
__device__ void acc_from_global(d4 (&accr)[BP / 16], d4 (&acci)[BP / 16], const double *g) {
  constexpr int NT = BP / 16;
  const int w = wave_id(), l = lane_id();
  if (w >= NT) return;
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + acc_row(l, r), col = tj * 16 + acc_col(l);
      const int gi = gpos<BP, FL>(row, col);
      accr[tj][r] = g[gi];
      acci[tj][r] = g[BP * BP + gi];
    }
}

// One chain of the factorisation per workgroup.  The first cell starts from
// S = D_start (- K_in); every cell is inverted, and every cell but the last
// (also the last one when end == 2) gets W = Sinv * Cpl and passes the Schur
// complement S_next = D_next - Cpl^T W on; end == 1 keeps the raw Schur
// complement of the last cell for the twist kernel.
template <int BP>
__global__ __launch_bounds__(kThreads) void factor_chain_kernel(Pencil p, Shifts sh, Factors f,
                                                                const Chain *chains,
                                                                const double *Kbuf) {
  extern __shared__ double smem_raw[];
  Lds<BP> &s = *reinterpret_cast<Lds<BP> *>(smem_raw);
  constexpr int NT = BP / 16, LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  const Chain ch = chains[blockIdx.x];
  const int e = ch.e, start = ch.start, dir = ch.dir, len = ch.len;
  if (len <= 0) return;
  const int nc = p.nc, b = p.b;
  const double zr = sh.zre[e], zi = sh.zim[e];
  const size_t blk = 2 * (size_t)BP * BP;
  const size_t bb = (size_t)b * b;
  double *Sinv = f.Sinv + (size_t)e * nc * blk;
  double *Wg = f.W + (size_t)e * nc * blk;
  double *WTg = f.WT + (size_t)e * nc * blk;

  form_block<BP>(s.A, p.Ad + start * bb, p.Bd + start * bb, b, zr, zi, false, true);
  if (ch.kin >= 0) {  // self-energy of the cells before this chain
    __syncthreads();
    const double *K = Kbuf + (size_t)ch.kin * blk;
    for (int idx = threadIdx.x; idx < BP * BP; idx += kThreads) {
      const int r = idx / BP, c = idx % BP;
      s.A[r * LD + c] -= K[idx];
      s.A[PLANE + r * LD + c] -= K[BP * BP + idx];
    }
  }
  __syncthreads();
  for (int j = 0; j < len; ++j) {
    const int c = start + dir * j;
    const bool last = (j == len - 1);
    if (last && ch.end == 1) {
      // raw Schur complement at the twist cell, finished by twist_kernel
      store_block<BP, false>(f.TW + (size_t)e * blk, s.A, false);
      break;
    }
    if (last && ch.end == 0) {
      gj_invert<BP>(s, Sinv + c * blk);
      break;
    }
    // coupling from c to the next cell in chain order, into slot B (free
    // here) by waves 1-3 while wave 0 inverts the first pivot tile
    auto coupling = [&]() {
      const int t = threadIdx.x - 64;
      if (dir > 0)
        form_block<BP, kThreads - 64>(s.B, p.Au + c * bb, p.Bu + c * bb, b, zr, zi, false, false, t);
      else
        form_block<BP, kThreads - 64>(s.B, p.Au + (c - 1) * bb, p.Bu + (c - 1) * bb, b, zr, zi,
                                      true, false, t);
    };
    gj_invert<BP>(s, Sinv + c * blk, coupling);  // slot A: Sinv (read until the next barrier)
    DiagRegs<BP> dn;  // next diagonal block, loaded under the W product
    if (!last) diag_regs_load<BP>(dn, p.Ad + (c + dir) * bb, p.Bd + (c + dir) * bb, b);
    __syncthreads();
    d4 wr[NT], wi[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) { wr[q] = d4zero(); wi[q] = d4zero(); }
    cgemm_lds<BP>(wr, wi, s.A, true, s.B, 1.0);  // W = Sinv * Cpl
    __syncthreads();
    acc_to_lds<BP>(s.A, wr, wi);
    __syncthreads();
    store_block_fl<BP>(Wg + c * blk, s.A, false);
    store_block_fl<BP>(WTg + c * blk, s.A, true);
    if (!last) {
      d4 sr[NT], si[NT];
      acc_from_diag_regs<BP>(sr, si, dn, b, zr, zi);
      cgemm_lds<BP>(sr, si, s.B, true, s.A, -1.0);  // S_next = D - Cpl^T W
      __syncthreads();
      acc_to_lds<BP>(s.A, sr, si);
      __syncthreads();
    }
  }
}

// Interface pass of the partitioned factorisation, one workgroup per
// (node, half), sequential over the partitions of the half.  For partition q
// with local matrix T (its own cells, no coupling to the cells before it) let
// G_11 = [T^-1]_{first,first}, G_L1 = [T^-1]_{last,first} and G_LL =
// [T^-1]_{last,last}.  With K the self-energy entering its first cell, the
// exact inverse Schur complement of its last cell is (Woodbury identity)
//   Sinv_last = G_LL + G_L1 K (I - G_11 K)^{-1} G_L1^T,
// and the next partition starts from D - K' with K' = C^T Sinv_last C, C the
// coupling from the last cell to the next one in chain order.
template <int BP>
__global__ __launch_bounds__(kThreads) void interface_kernel(Pencil p, Shifts sh, Factors f,
                                                             const Chain *chainsF1, int parts,
                                                             const double *G11, const double *GL1,
                                                             double *Kbuf) {
  extern __shared__ double smem_raw[];
  Lds<BP> &s = *reinterpret_cast<Lds<BP> *>(smem_raw);
  constexpr int NT = BP / 16;
  const int grp = blockIdx.x;  // e * 2 + half
  const int nc = p.nc, b = p.b;
  const size_t blk = 2 * (size_t)BP * BP;
  const size_t bb = (size_t)b * b;
  const Chain *ch0 = chainsF1 + (size_t)grp * (parts - 1);
  const int e = ch0->e;
  const double zr = sh.zre[e], zi = sh.zim[e];
  const double *Sinv = f.Sinv + (size_t)e * nc * blk;
  const int w = wave_id(), l = lane_id();
  d4 ar[NT], ai[NT];
  for (int q = 0; q < parts - 1; ++q) {
    const Chain ch = ch0[q];
    const int last = ch.start + ch.dir * (ch.len - 1);
    const size_t gi = ((size_t)grp * parts + q) * blk;
    if (q == 0) {
      load_block<BP, true>(s.A, Sinv + last * blk);  // K = 0: Sinv_last = G_LL
      __syncthreads();
    } else {
      // slot B holds K.  N = (I - G_11 K)^{-1}
      load_block<BP, false>(s.A, G11 + gi);
      __syncthreads();
      if (w < NT) {
#pragma unroll
        for (int tj = 0; tj < NT; ++tj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            ar[tj][r] = (w * 16 + acc_row(l, r) == tj * 16 + acc_col(l)) ? 1.0 : 0.0;
            ai[tj][r] = 0.0;
          }
      }
      cgemm_lds<BP>(ar, ai, s.A, false, s.B, -1.0);
      __syncthreads();
      acc_to_lds<BP>(s.A, ar, ai);
      __syncthreads();
      gj_invert<BP>(s, nullptr, NoSide(), false);
      // M3 = K N
#pragma unroll
      for (int t = 0; t < NT; ++t) { ar[t] = d4zero(); ai[t] = d4zero(); }
      cgemm_lds<BP>(ar, ai, s.B, false, s.A, 1.0);
      __syncthreads();
      acc_to_lds<BP>(s.B, ar, ai);
      load_block<BP, false>(s.A, GL1 + gi);
      __syncthreads();
      // M4 = G_L1 M3
#pragma unroll
      for (int t = 0; t < NT; ++t) { ar[t] = d4zero(); ai[t] = d4zero(); }
      cgemm_lds<BP>(ar, ai, s.A, false, s.B, 1.0);
      __syncthreads();
      acc_to_lds<BP>(s.B, ar, ai);
      __syncthreads();
      // Sinv_last = G_LL + M4 G_L1^T
      acc_from_global<BP, true>(ar, ai, Sinv + last * blk);
      cgemm_lds<BP>(ar, ai, s.B, false, s.A, 1.0, true);
      __syncthreads();
      acc_to_lds<BP>(s.A, ar, ai);
      __syncthreads();
    }
    // K' = C^T Sinv_last C
    if (ch.dir > 0)
      form_block<BP>(s.B, p.Au + last * bb, p.Bu + last * bb, b, zr, zi, false, false);
    else
      form_block<BP>(s.B, p.Au + (last - 1) * bb, p.Bu + (last - 1) * bb, b, zr, zi, true,
                     false);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT; ++t) { ar[t] = d4zero(); ai[t] = d4zero(); }
    cgemm_lds<BP>(ar, ai, s.A, false, s.B, 1.0);
    __syncthreads();
    acc_to_lds<BP>(s.A, ar, ai);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT; ++t) { ar[t] = d4zero(); ai[t] = d4zero(); }
    cgemm_lds<BP>(ar, ai, s.B, true, s.A, 1.0);
    __syncthreads();
    acc_to_global<BP, false>(Kbuf + ((size_t)grp * parts + q + 1) * blk, ar, ai);
    acc_to_lds<BP>(s.B, ar, ai);  // K for the next partition
    __syncthreads();
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
    load_block<BP, false>(s.A, TW);
    __syncthreads();
  } else {
    load_block<BP, true>(s.A, f.W + ((size_t)e * nc + m) * blk);
    form_block<BP>(s.B, p.Au + (m - 1) * bb, p.Bu + (m - 1) * bb, b, zr, zi, false, false);
    __syncthreads();
    d4 sr[NT], si[NT];
    acc_from_global<BP, false>(sr, si, TW);
    cgemm_lds<BP>(sr, si, s.B, false, s.A, -1.0);
    __syncthreads();
    acc_to_lds<BP>(s.A, sr, si);
    __syncthreads();
  }
  gj_invert<BP>(s, f.Sinv + ((size_t)e * nc + (m - 1)) * blk);
}

// ---- blocks of 64 < b <= 96 (BP = 96) ----
//
// One chain per contour point over all cells, top-down (no twist, no
// partitions), six waves.  The complex 96 x 96 block fits in LDS once only,
// so the slot holds S, then Sinv, then W, then the next S, and the coupling
// U_c = Z B_{c,c+1} - A_{c,c+1} enters the products as matrix-operand
// fragments of its real planes, packed once per solve in the layout fpos.
// Wave w holds the fragments of column block w of U_c: they are the B
// operand of column block w of W = Sinv U_c (every row block) and the A
// operand of row block w of U_c^T W (every column block).
constexpr int kWideBP = 96;
constexpr int kWideWaves = kWideBP / 16;
constexpr int kWideThreads = 64 * kWideWaves;

// Couplings Au, Bu (caller layout, b x b) -> cpl [nc-1][2][BP][BP], their
// transposes -> cplt [nc-1][2][BP][BP], and diagonal blocks Ad, Bd -> dia
// [nc][2][BP][BP], all in the layout fpos.  Padding: zero, but -1 in A on
// the diagonal of a diagonal block (so that Z B - A holds the identity there).
__global__ void pack_wide_kernel(Pencil p, WidePack w) {
  constexpr int BP = kWideBP;
  const size_t per = (size_t)BP * BP;
  const size_t ncpl = (size_t)(p.nc - 1) * per;
  const size_t total = 2 * ncpl + (size_t)p.nc * per;
  for (size_t o = blockIdx.x * (size_t)blockDim.x + threadIdx.x; o < total;
       o += (size_t)gridDim.x * blockDim.x) {
    const int region = o < ncpl ? 0 : (o < 2 * ncpl ? 1 : 2);  // cpl, cplt, dia
    const size_t q = region == 0 ? o : (region == 1 ? o - ncpl : o - 2 * ncpl);
    const int c = (int)(q / per), idx = (int)(q % per);
    const int i = idx / BP, j = idx % BP;
    const bool in = i < p.b && j < p.b;
    const size_t src = region == 1 ? ((size_t)c * p.b + j) * p.b + i : ((size_t)c * p.b + i) * p.b + j;
    const bool diag = region == 2;
    double *d = (region == 0 ? w.cpl : region == 1 ? w.cplt : w.dia) + (size_t)c * 2 * per;
    const int fp = fpos<BP>(i, j);
    const double pad_a = (diag && i == j) ? -1.0 : 0.0;
    d[fp] = in ? (diag ? p.Ad : p.Au)[src] : pad_a;
    d[per + fp] = in ? (diag ? p.Bd : p.Bu)[src] : 0.0;
  }
}

// Tile (rb, tj) of a packed real plane (layout fpos) in the accumulator
// layout: element r of lane l is M[rb*16 + l/16 + 4r][tj*16 + l%16]; rows
// l/16 and l/16 + 4 (and + 8, + 12) sit next to each other in fpos, so two
// sixteen-byte loads fetch the four.
template <int BP>
__device__ __forceinline__ d4 acc_plane_load(__amdgpu_buffer_rsrc_t rs, int soff, int rb, int tj) {
  const int l = threadIdx.x & 63;
  const int vo = fpos<BP>(rb * 16 + (l >> 4), tj * 16 + (l & 15)) * 8;
  const auto x = __builtin_amdgcn_raw_buffer_load_b128(rs, vo, soff, 0);
  const auto y = __builtin_amdgcn_raw_buffer_load_b128(rs, vo + 8 * BP * 8, soff, 0);
  return d4{__builtin_bit_cast(double, (u32x2){x[0], x[1]}),
            __builtin_bit_cast(double, (u32x2){x[2], x[3]}),
            __builtin_bit_cast(double, (u32x2){y[0], y[1]}),
            __builtin_bit_cast(double, (u32x2){y[2], y[3]})};
}

__global__ __launch_bounds__(kWideThreads) void factor_wide_kernel(Pencil p, Shifts sh, Factors f,
                                                                   const double *cpl,
                                                                   const double *dia) {
  constexpr int BP = kWideBP, NT = BP / 16, KS = BP / 4;
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  extern __shared__ double smem_raw[];
  double *S = smem_raw;
  const int e = blockIdx.x;
  const int nc = p.nc, b = p.b;
  const double zr = sh.zre[e], zi = sh.zim[e];
  const size_t blk = 2 * (size_t)BP * BP, per = (size_t)BP * BP;
  double *Sinv = f.Sinv + (size_t)e * nc * blk;
  double *Wg = f.W + (size_t)e * nc * blk;
  double *WTg = f.WT + (size_t)e * nc * blk;
  const int w = wave_id(), l = lane_id();
  const int kl = l >> 4, m = l & 15;

  form_block<BP, kWideThreads>(S, p.Ad, p.Bd, b, zr, zi, false, true);  // S_0 = D_0
  __syncthreads();
  for (int c = 0; c < nc; ++c) {
    gj_invert_slot<BP, kWideWaves>(S, Sinv + c * blk);  // S <- Sinv_c (also stored)
    if (c == nc - 1) break;
    double ua[KS], ub[KS];  // column block w of the real planes of U_c
    frag_plane_load<BP>(ua, cpl + c * 2 * per, w, true);
    frag_plane_load<BP>(ub, cpl + c * 2 * per + per, w, true);
    // column block w of W = Sinv U_c: tile (ib, w), A operand Sinv[ib rows][k]
    // read as Sinv[k][ib rows] (symmetric)
    d4 wr[NT], wi[NT];
#pragma unroll
    for (int ib = 0; ib < NT; ++ib) {
      d4 t1 = d4zero(), ar = d4zero(), ai = d4zero();
#pragma unroll 4
      for (int ks = 0; ks < KS; ++ks) {
        const int xa = (4 * ks + kl) * LD + ib * 16 + m;
        const double xr = S[xa], xi = S[PLANE + xa];
        const double yr = zr * ub[ks] - ua[ks], yi = zi * ub[ks];
        t1 = mfma(xr, yr + yi, t1);
        ar = mfma(-(xr + xi), yi, ar);
        ai = mfma(xi - xr, yr, ai);
      }
      wr[ib] = ar + t1;
      wi[ib] = ai + t1;
    }
    __syncthreads();  // every wave is done with Sinv
#pragma unroll
    for (int ib = 0; ib < NT; ++ib)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = ib * 16 + acc_row(l, r), col = w * 16 + acc_col(l);
        S[row * LD + col] = wr[ib][r];
        S[PLANE + row * LD + col] = wi[ib][r];
      }
    __syncthreads();
    store_block_fl<BP, kWideThreads>(Wg + c * blk, S, false);
    store_block_fl<BP, kWideThreads>(WTg + c * blk, S, true);
    // row block w of S_{c+1} = D_{c+1} - U_c^T W: A operand -U_c[k][w rows]
    const auto rd = buf_rsrc(dia, nc * 2 * BP * BP * 8);
    const int dsoff = (c + 1) * 2 * BP * BP * 8;
    d4 sr[NT], si[NT];
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) {
      const d4 av = acc_plane_load<BP>(rd, dsoff, w, tj);
      const d4 bv = acc_plane_load<BP>(rd, dsoff + BP * BP * 8, w, tj);
      sr[tj] = zr * bv - av;
      si[tj] = zi * bv;
      d4 t1 = d4zero();
#pragma unroll 4
      for (int ks = 0; ks < KS; ++ks) {
        const double xr = ua[ks] - zr * ub[ks], xi = -zi * ub[ks];
        const int yb = (4 * ks + kl) * LD + tj * 16 + m;
        const double yr = S[yb], yi = S[PLANE + yb];
        t1 = mfma(xr, yr + yi, t1);
        sr[tj] = mfma(-(xr + xi), yi, sr[tj]);
        si[tj] = mfma(xi - xr, yr, si[tj]);
      }
      sr[tj] += t1;
      si[tj] += t1;
    }
    __syncthreads();  // every wave is done with W
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = w * 16 + acc_row(l, r), col = tj * 16 + acc_col(l);
        S[row * LD + col] = sr[tj][r];
        S[PLANE + row * LD + col] = si[tj][r];
      }
    __syncthreads();
  }
}

template <int BP>
hipError_t set_lds(const void *fn) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)sizeof(Lds<BP>));
}

template <int BP>
hipError_t launch_factor_bp(const Pencil &p, const Shifts &s, int Ne, const Factors &f, int parts,
                            double *work, Chain *chains, double *G, int gtiles, hipStream_t st) {
  const size_t shm = sizeof(Lds<BP>);
  hipError_t err;
  if ((err = set_lds<BP>((const void *)factor_chain_kernel<BP>)) != hipSuccess) return err;
  if ((err = set_lds<BP>((const void *)twist_kernel<BP>)) != hipSuccess) return err;
  if ((err = set_lds<BP>((const void *)interface_kernel<BP>)) != hipSuccess) return err;
  const int nc = p.nc, m = f.m;
  // chain tables: F1 = local factorisation of every partition but the last
  // of each half, F3 = exact factorisation of every partition
  std::vector<Chain> host;
  const int nF1 = Ne * 2 * (parts - 1), nF3 = Ne * 2 * parts;
  host.reserve(nF1 + nF3);
  for (int pass = 0; pass < 2; ++pass)
    for (int e = 0; e < Ne; ++e)
      for (int h = 0; h < 2; ++h) {
        const int len = h == 0 ? m : nc - m;
        const int start = h == 0 ? 0 : nc - 1;
        const int dir = h == 0 ? 1 : -1;
        const int np = pass == 0 ? parts - 1 : parts;
        for (int q = 0; q < np; ++q) {
          const int a = (int)((long long)q * len / parts);
          const int z = (int)((long long)(q + 1) * len / parts);
          Chain c;
          c.e = e;
          c.start = start + dir * a;
          c.len = z - a;
          c.dir = dir;
          c.half = h;
          c.part = q;
          if (pass == 0) {
            c.end = 0;
            c.kin = -1;
          } else {
            c.end = (q < parts - 1) ? 2 : (h == 0 ? 1 : 2);
            c.kin = q > 0 ? (e * 2 + h) * parts + q : -1;
          }
          host.push_back(c);
        }
      }
  if ((err = hipMemcpyAsync(chains, host.data(), host.size() * sizeof(Chain),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
    return err;
  if ((err = hipStreamSynchronize(st)) != hipSuccess) return err;
  const size_t blk = 2 * (size_t)BP * BP;
  double *Kbuf = work;
  double *G11 = work + (size_t)Ne * 2 * parts * blk;
  double *GL1 = G11 + (size_t)Ne * 2 * parts * blk;
  if (parts > 1) {
    hipLaunchKernelGGL(factor_chain_kernel<BP>, dim3(nF1), dim3(kThreads), shm, st, p, s, f,
                       (const Chain *)chains, (const double *)Kbuf);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if ((err = launch_spikes(p, f, chains, nF1, parts, gtiles, G, G11, GL1, st)) != hipSuccess)
      return err;
    hipLaunchKernelGGL(interface_kernel<BP>, dim3(Ne * 2), dim3(kThreads), shm, st, p, s, f,
                       (const Chain *)chains, parts, (const double *)G11, (const double *)GL1,
                       Kbuf);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  hipLaunchKernelGGL(factor_chain_kernel<BP>, dim3(nF3), dim3(kThreads), shm, st, p, s, f,
                     (const Chain *)(chains + nF1), (const double *)Kbuf);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(twist_kernel<BP>, dim3(Ne), dim3(kThreads), shm, st, p, s, f);
  return hipGetLastError();
}

// ---- Hermitian A (eq. 12): block LU of the non-symmetric M = Z B - A ----
//
// With A complex Hermitian, M_e = Z_e B - A is neither symmetric nor
// Hermitian, so the factorisation keeps Sinv_c, W_c = Sinv_c C_c (upper
// coupling C_c = Z B_{c,c+1} - A_{c,c+1}) and V_c = L_c Sinv_c (lower
// coupling L_c = Z B_{c,c+1}^T - A_{c,c+1}^H), and S_{c+1} = D_{c+1} - L_c W_c.
// Every principal submatrix of M has the positive definite Hermitian part
// Im(Z) B in M - M^H = 2i Im(Z) B, so the blocked Gauss-Jordan inverse needs
// no pivoting; it is not symmetrised.  One workgroup per partition of a half
// chain, the blocks in the two LDS slots, the products on the matrix cores;
// the factors are stored in the 4 x 4 tiled layout of kernels.h, which the
// Hermitian sweeps read.

// slot <- one shifted block of the Hermitian pencil by NTH threads: kind 0
// D_cell (identity padding), 1 C_cell, 2 L_cell (zero padding).
template <int BP, int NTH = kThreads>
__device__ void hform_block(double *slot, const HPencil &p, int cell, int kind, double zr,
                            double zi, int tid = threadIdx.x) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  const int b = p.b;
  const size_t bb = (size_t)b * b;
  const double *Ac = (kind == 0 ? p.Ad : p.Au) + 2 * (size_t)cell * bb;
  const double *Br = (kind == 0 ? p.Bd : p.Bu) + (size_t)cell * bb;
  for (int idx = tid; idx < BP * BP; idx += NTH) {
    const int r = idx / BP, c = idx % BP;
    double re = (kind == 0 && r == c) ? 1.0 : 0.0, im = 0.0;
    if (r < b && c < b) {
      const int o = kind == 2 ? c * b + r : r * b + c;  // L: the transposed element
      const double bv = Br[o], ar = Ac[2 * o], ai = Ac[2 * o + 1];
      re = zr * bv - ar;
      im = kind == 2 ? zi * bv + ai : zi * bv - ai;  // L: conj(A_u) transposed
    }
    slot[r * LD + c] = re;
    slot[PLANE + r * LD + c] = im;
  }
}

// acc <- D_cell in the accumulator layout (identity padding).
template <int BP>
__device__ void acc_from_hdiag(d4 (&accr)[BP / 16], d4 (&acci)[BP / 16], const HPencil &p,
                               int cell, double zr, double zi) {
  constexpr int NT = BP / 16;
  const int w = wave_id(), l = lane_id();
  if (w >= NT) return;
  const int b = p.b;
  const size_t bb = (size_t)b * b;
  const double *Ac = p.Ad + 2 * (size_t)cell * bb;
  const double *Br = p.Bd + (size_t)cell * bb;
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + acc_row(l, r), col = tj * 16 + acc_col(l);
      double re = row == col ? 1.0 : 0.0, im = 0.0;
      if (row < b && col < b) {
        const int o = row * b + col;
        re = zr * Br[o] - Ac[2 * o];
        im = zi * Br[o] - Ac[2 * o + 1];
      }
      accr[tj][r] = re;
      acci[tj][r] = im;
    }
}

// Factor blocks in the tiled layout (kernels.h): tiled <- the slot, tiled <-
// this wave's accumulator tiles, slot <- tiled (zero outside b x b).
__device__ __forceinline__ int htile_off(int i, int j, int bt) {
  return ((i >> 2) * bt + (j >> 2)) * 16 + (i & 3) * 4 + (j & 3);
}

template <int BP>
__device__ void hstore_tiled(double *g, const double *slot, int b) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  const int t4 = htile_dim(b), bt = t4 / 4;
  for (int idx = threadIdx.x; idx < t4 * t4; idx += kThreads) {
    const int i = idx / t4, j = idx % t4;
    const int o = htile_off(i, j, bt);
    g[2 * o] = slot[i * LD + j];
    g[2 * o + 1] = slot[PLANE + i * LD + j];
  }
}

template <int BP>
__device__ void hacc_to_tiled(double *g, const d4 (&accr)[BP / 16], const d4 (&acci)[BP / 16],
                              int b) {
  constexpr int NT = BP / 16;
  const int w = wave_id(), l = lane_id();
  if (w >= NT) return;
  const int t4 = htile_dim(b), bt = t4 / 4;
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + acc_row(l, r), col = tj * 16 + acc_col(l);
      if (row < t4 && col < t4) {
        const int o = htile_off(row, col, bt);
        g[2 * o] = accr[tj][r];
        g[2 * o + 1] = acci[tj][r];
      }
    }
}

template <int BP>
__device__ void hload_tiled(double *slot, const double *g, int b) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  const int bt = htile_dim(b) / 4;
  for (int idx = threadIdx.x; idx < BP * BP; idx += kThreads) {
    const int r = idx / BP, c = idx % BP;
    const bool in = r < b && c < b;
    const int o = in ? htile_off(r, c, bt) : 0;
    slot[r * LD + c] = in ? g[2 * o] : 0.0;
    slot[PLANE + r * LD + c] = in ? g[2 * o + 1] : 0.0;
  }
}

// Operands of the Hermitian block products: an LDS slot, or a complex block
// in global memory in the 4 x 4 tiled layout, read as zero outside b x b.
template <int BP>
struct SlotOp {
  const double *s;
  __device__ __forceinline__ void ld(int r, int c, double &re, double &im) const {
    re = s[r * Lds<BP>::LD + c];
    im = s[Lds<BP>::PLANE + r * Lds<BP>::LD + c];
  }
};
struct GlobOp {  // a block in the 4 x 4 tiled layout
  const double *g;
  int b;
  __device__ __forceinline__ void ld(int r, int c, double &re, double &im) const {
    const bool in = r < b && c < b;
    const int o = in ? htile_off(r, c, htile_dim(b) >> 2) : 0;
    const double2 v = *reinterpret_cast<const double2 *>(g + 2 * o);
    re = in ? v.x : 0.0;
    im = in ? v.y : 0.0;
  }
};

// acc (+)= sign * X * Y with either operand in LDS or in global memory; the
// three-product form of cgemm_lds.
template <int BP, class OX, class OY>
__device__ __forceinline__ void cgemm_op(d4 (&accr)[BP / 16], d4 (&acci)[BP / 16], OX X, OY Y,
                                         double sign) {
  constexpr int NT = BP / 16;
  const int w = wave_id(), l = lane_id();
  if (w >= NT) return;
  const int row = w * 16 + (l & 15);
  const int kl = l >> 4;
  d4 t1[NT];
#pragma unroll
  for (int tj = 0; tj < NT; ++tj) t1[tj] = d4zero();
#pragma unroll 4  // fully unrolled, the hoisted global loads spill
  for (int k0 = 0; k0 < BP; k0 += 4) {
    const int k = k0 + kl;
    double xr, xi;
    X.ld(row, k, xr, xi);
    xr *= sign;
    xi *= sign;
    const double xs = -(xr + xi), xd = xi - xr;
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) {
      double yr, yi;
      Y.ld(k, tj * 16 + (l & 15), yr, yi);
      t1[tj] = mfma(xr, yr + yi, t1[tj]);
      accr[tj] = mfma(xs, yi, accr[tj]);
      acci[tj] = mfma(xd, yr, acci[tj]);
    }
  }
#pragma unroll
  for (int tj = 0; tj < NT; ++tj)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      accr[tj][q] += t1[tj][q];
      acci[tj][q] += t1[tj][q];
    }
}

template <int BP>
__device__ __forceinline__ void acc_fill(d4 (&accr)[BP / 16], d4 (&acci)[BP / 16], double diag) {
  const int l = lane_id(), w = wave_id();
#pragma unroll
  for (int tj = 0; tj < BP / 16; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      accr[tj][r] = (w * 16 + acc_row(l, r) == tj * 16 + acc_col(l)) ? diag : 0.0;
      acci[tj][r] = 0.0;
    }
}

// acc <- complex tiled block (zero outside b x b)
template <int BP>
__device__ void hacc_from_global(d4 (&accr)[BP / 16], d4 (&acci)[BP / 16], const double *g,
                                 int b) {
  const int w = wave_id(), l = lane_id();
  if (w >= BP / 16) return;
  const GlobOp G{g, b};
#pragma unroll
  for (int tj = 0; tj < BP / 16; ++tj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double re, im;
      G.ld(w * 16 + acc_row(l, r), tj * 16 + acc_col(l), re, im);
      accr[tj][r] = re;
      acci[tj][r] = im;
    }
}

template <int BP>
__device__ __forceinline__ void acc_negate(d4 (&accr)[BP / 16], d4 (&acci)[BP / 16]) {
#pragma unroll
  for (int tj = 0; tj < BP / 16; ++tj) {
    accr[tj] = -accr[tj];
    acci[tj] = -acci[tj];
  }
}

// slot -= K (complex tiled block) on the leading b x b block
template <int BP>
__device__ void hsub_block(double *slot, const double *K, int b) {
  constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
  const int bt = htile_dim(b) >> 2;
  for (int idx = threadIdx.x; idx < b * b; idx += kThreads) {
    const int r = idx / b, c = idx % b, o = htile_off(r, c, bt);
    slot[r * LD + c] -= K[2 * o];
    slot[PLANE + r * LD + c] -= K[2 * o + 1];
  }
}

// Blocks a (chain, partition) keeps in the factorisation's work area.
enum HWork { HW_K, HW_G11, HW_YH, HW_XH, HW_YGX, HW_P0, HW_P1, HW_Q, HW_T, HW_COUNT };

// Twisted: per contour point a top chain (cells 0..m-1, top-down) and a
// bottom chain (cells nc-1..m, bottom-up), m = nc - nc/2, joined at the twist
// cell m-1 by hfactor_twist_kernel.  Chain position j is cell j (top) or
// nc-1-j (bottom).  Per cell c of a chain, with X the coupling from c to the
// next cell in chain order and Y the one back (top: X = C_c, Y = L_c;
// bottom: X = L_{c-1}, Y = C_{c-1}):
//   Sinv_c = S_c^{-1},  W_c = Sinv_c X,  V_c = Y Sinv_c,  S_next = D_next - Y W_c,
// all stored at index c (W and V hold nc blocks a contour point).  The top
// chain leaves the raw Schur complement S_{m-1} in the unused W[m-1]; the
// bottom chain stops after W_m and V_m.
//
// hchain_final runs chain positions [jb, je) from S = D - K at jb (K: the
// self-energy of the part of the chain before jb, none for the first
// partition) and stores the factors.
template <int BP>
__device__ void hchain_final(Lds<BP> &s, const HPencil &p, double zr, double zi, bool top,
                             int len, int jb, int je, const double *K, double *Se, double *We,
                             double *Ve) {
  constexpr int NT = BP / 16;
  const int nc = p.nc, b = p.b, m = nc - nc / 2;
  const size_t bb = hfactor_block_elems(b);
  auto cell = [&](int j) { return top ? j : nc - 1 - j; };
  hform_block<BP>(s.A, p, cell(jb), 0, zr, zi);  // S = D_jb
  if (K) {
    __syncthreads();
    hsub_block<BP>(s.A, K, b);  // S = D_jb - K
  }
  __syncthreads();
  for (int j = jb; j < je; ++j) {
    const int c = cell(j);
    const bool chain_last = j == len - 1;
    if (top && chain_last && nc - m > 0) {  // raw S_{m-1} for the twist kernel
      hstore_tiled<BP>(We + 2 * (size_t)c * bb, s.A, b);
      break;
    }
    const bool more = !(top && chain_last);  // the bottom chain's last cell still gets W, V
    const int cc = top ? c : c - 1;          // cell of the couplings X, Y
    const int kx = top ? 1 : 2, ky = top ? 2 : 1;
    // X into slot B by waves 1-3 while wave 0 inverts the first pivot tile
    auto coupling = [&]() {
      if (more) hform_block<BP, kThreads - 64>(s.B, p, cc, kx, zr, zi, threadIdx.x - 64);
    };
    gj_invert<BP>(s, nullptr, coupling, false);  // slot A: Sinv_c
    hstore_tiled<BP>(Se + 2 * (size_t)c * bb, s.A, b);
    if (!more) break;
    d4 wr[NT], wi[NT], vr[NT], vi[NT], sr[NT], si[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      wr[t] = d4zero(); wi[t] = d4zero(); vr[t] = d4zero(); vi[t] = d4zero();
    }
    cgemm_lds<BP>(wr, wi, s.A, false, s.B, 1.0);  // W = Sinv X
    __syncthreads();
    hform_block<BP>(s.B, p, cc, ky, zr, zi);  // slot B: Y
    __syncthreads();
    cgemm_lds<BP>(vr, vi, s.B, false, s.A, 1.0);  // V = Y Sinv
    hacc_to_tiled<BP>(Ve + 2 * (size_t)c * bb, vr, vi, b);
    __syncthreads();
    acc_to_lds<BP>(s.A, wr, wi);  // slot A: W
    hacc_to_tiled<BP>(We + 2 * (size_t)c * bb, wr, wi, b);
    __syncthreads();
    if (j == je - 1) break;  // end of the partition (bottom chain: W_m and V_m, no S_{m-1})
    acc_from_hdiag<BP>(sr, si, p, cell(j + 1), zr, zi);
    cgemm_lds<BP>(sr, si, s.B, false, s.A, -1.0);  // S_next = D_next - Y W
    __syncthreads();
    acc_to_lds<BP>(s.A, sr, si);
    __syncthreads();
  }
}

// hchain_local factors chain positions [jb, je) on their own (from S = D_jb)
// for the corner blocks of the inverse G of that diagonal section: G11
// (first, first), GL1 (last, first), G1L (first, last), GLL (last, last).
// With the local factors Sinv'_t, W'_t, V'_t (t = 0..L-1) and
//   P_0 = Q_0 = I,  P_{t+1} = -V'_t P_t,  Q_{t+1} = -Q_t W'_t,
// the first block column of G ends in GL1 = Sinv'_L-1 P_L-1, the first block
// row in G1L = Q_L-1 Sinv'_L-1, and appending cell t to the section adds
// Q_t Sinv'_t P_t to G11 (Schur complement of the new cell).  With
// T_t = Sinv'_t P_t, P_{t+1} = -Y_t T_t, so V'_t is never formed.  With X, Y
// the couplings to the next partition it leaves G11, YH = Y GL1, XH = G1L X
// and YGX = Y GLL X.
template <int BP>
__device__ void hchain_local(Lds<BP> &s, const HPencil &p, double zr, double zi, bool top,
                             int jb, int je, double *wk) {
  constexpr int NT = BP / 16;
  const int nc = p.nc, b = p.b;
  const size_t bb2 = 2 * hfactor_block_elems(b);  // work blocks: tiled
  double *G11 = wk + HW_G11 * bb2, *YH = wk + HW_YH * bb2, *XH = wk + HW_XH * bb2;
  double *YGX = wk + HW_YGX * bb2, *Q = wk + HW_Q * bb2, *T = wk + HW_T * bb2;
  double *Pb[2] = {wk + HW_P0 * bb2, wk + HW_P1 * bb2};
  const int L = je - jb;
  auto cell = [&](int j) { return top ? j : nc - 1 - j; };
  hform_block<BP>(s.A, p, cell(jb), 0, zr, zi);  // S'_0 = D_jb
  __syncthreads();
  for (int t = 0; t < L; ++t) {
    const int c = cell(jb + t);
    const bool last = t == L - 1;
    const int cc = top ? c : c - 1;
    const int kx = top ? 1 : 2, ky = top ? 2 : 1;
    auto coupling = [&]() {
      hform_block<BP, kThreads - 64>(s.B, p, cc, kx, zr, zi, threadIdx.x - 64);
    };
    gj_invert<BP>(s, nullptr, coupling, false);  // slot A: Sinv'_t, slot B: X
    const double *Pc = Pb[t & 1];
    double *Pn = Pb[(t + 1) & 1];
    d4 ar[NT], ai[NT];
    if (t == 0) {  // P_0 = Q_0 = I
      hstore_tiled<BP>(G11, s.A, b);
      hstore_tiled<BP>(T, s.A, b);
    } else {
      acc_fill<BP>(ar, ai, 0.0);
      cgemm_op<BP>(ar, ai, SlotOp<BP>{s.A}, GlobOp{Pc, b}, 1.0);  // T_t = Sinv'_t P_t
      hacc_to_tiled<BP>(T, ar, ai, b);
      __syncthreads();
      hacc_from_global<BP>(ar, ai, G11, b);
      cgemm_op<BP>(ar, ai, GlobOp{Q, b}, GlobOp{T, b}, 1.0);  // G11 += Q_t T_t
      hacc_to_tiled<BP>(G11, ar, ai, b);
    }
    d4 wr[NT], wi[NT];
    acc_fill<BP>(wr, wi, 0.0);
    cgemm_lds<BP>(wr, wi, s.A, false, s.B, 1.0);  // W' = Sinv' X
    __syncthreads();
    hform_block<BP>(s.B, p, cc, ky, zr, zi);  // slot B: Y
    if (last) {  // XH = Q_t W', YGX = Y W', YH = Y GL1 (GL1 = T_t)
      acc_to_lds<BP>(s.A, wr, wi);
      if (t == 0) hacc_to_tiled<BP>(XH, wr, wi, b);
      __syncthreads();
      if (t > 0) {
        acc_fill<BP>(ar, ai, 0.0);
        cgemm_op<BP>(ar, ai, GlobOp{Q, b}, SlotOp<BP>{s.A}, 1.0);
        hacc_to_tiled<BP>(XH, ar, ai, b);
      }
      acc_fill<BP>(ar, ai, 0.0);
      cgemm_lds<BP>(ar, ai, s.B, false, s.A, 1.0);
      hacc_to_tiled<BP>(YGX, ar, ai, b);
      acc_fill<BP>(ar, ai, 0.0);
      cgemm_op<BP>(ar, ai, SlotOp<BP>{s.B}, GlobOp{T, b}, 1.0);
      hacc_to_tiled<BP>(YH, ar, ai, b);
      break;
    }
    __syncthreads();
    acc_fill<BP>(ar, ai, 0.0);
    cgemm_op<BP>(ar, ai, SlotOp<BP>{s.B}, GlobOp{T, b}, -1.0);  // P_{t+1} = -V'_t P_t = -Y T_t
    hacc_to_tiled<BP>(Pn, ar, ai, b);
    acc_to_lds<BP>(s.A, wr, wi);  // slot A: W'
    if (t == 0) {
      acc_negate<BP>(wr, wi);
      hacc_to_tiled<BP>(Q, wr, wi, b);  // Q_1 = -W'_0
    }
    __syncthreads();
    if (t > 0) {
      acc_fill<BP>(ar, ai, 0.0);
      cgemm_op<BP>(ar, ai, GlobOp{Q, b}, SlotOp<BP>{s.A}, -1.0);  // Q_{t+1} = -Q_t W'_t
      hacc_to_tiled<BP>(Q, ar, ai, b);  // in place: a wave reads and writes its own rows
    }
    acc_from_hdiag<BP>(ar, ai, p, cell(jb + t + 1), zr, zi);
    cgemm_lds<BP>(ar, ai, s.B, false, s.A, -1.0);  // S'_{t+1} = D - Y W'
    __syncthreads();
    acc_to_lds<BP>(s.A, ar, ai);
    __syncthreads();
  }
}

// First chain position of partition q of P over a chain of len positions.
// Partition 0 is factored exactly while the inner ones run their longer
// local pass (six products a cell against three), so it takes 1.8 shares of
// the chain to their 1; every partition is non-empty for P <= len.
__device__ __forceinline__ int hpart_start(int q, int len, int P) {
  if (q <= 0) return 0;
  if (q >= P) return len;
  return (int)((long long)len * (18 + 10 * (q - 1)) / (18 + 10 * (P - 1)));
}

// Partition q of a chain covers positions [hpart_start(q), hpart_start(q+1)).
// Phase 0: partition 0 exactly, partitions 1..P-2 locally; phase 1: the
// exact rerun of partitions 1..P-1 from the self-energies of
// hinterface_kernel.
template <int BP>
__global__ __launch_bounds__(kThreads) void hfactor_part_kernel(HPencil p, Shifts sh,
                                                                double *Sinv, double *W,
                                                                double *V, double *work,
                                                                int P, int phase) {
  extern __shared__ double smem_raw[];
  Lds<BP> &s = *reinterpret_cast<Lds<BP> *>(smem_raw);
  const int per = phase == 0 ? (P > 1 ? P - 1 : 1) : P - 1;
  const int ch = blockIdx.x / per, q = blockIdx.x % per + phase;
  const int e = ch >> 1;
  const bool top = (ch & 1) == 0;
  const int nc = p.nc, m = nc - nc / 2;
  const int len = top ? m : nc - m;
  if (len <= 0) return;
  const int jb = hpart_start(q, len, P), je = hpart_start(q + 1, len, P);
  const double zr = sh.zre[e], zi = sh.zim[e];
  const size_t bb2 = 2 * hfactor_block_elems(p.b);  // factor and work blocks: tiled
  double *Se = Sinv + (size_t)e * nc * bb2;
  double *We = W + (size_t)e * nc * bb2;
  double *Ve = V + (size_t)e * nc * bb2;
  double *wk = work + ((size_t)ch * P + q) * HW_COUNT * bb2;
  if (q == 0 || phase == 1)
    hchain_final<BP>(s, p, zr, zi, top, len, jb, je, q ? wk + HW_K * bb2 : nullptr, Se, We, Ve);
  else
    hchain_local<BP>(s, p, zr, zi, top, jb, je, wk);
}

// Twist cell m-1: Sinv_{m-1} = T = (S_{m-1} - C_{m-1} W_m)^{-1}, with S_{m-1}
// (raw, top chain) in W[m-1] and W_m = Sinv_m L_{m-1} of the bottom chain;
// nothing to do when the bottom chain is empty (nc = 1: the top chain
// inverted its last cell).
template <int BP>
__global__ __launch_bounds__(kThreads) void hfactor_twist_kernel(HPencil p, Shifts sh,
                                                                 double *Sinv, double *W) {
  extern __shared__ double smem_raw[];
  Lds<BP> &s = *reinterpret_cast<Lds<BP> *>(smem_raw);
  constexpr int NT = BP / 16;
  const int e = blockIdx.x;
  const int nc = p.nc, b = p.b, m = nc - nc / 2;
  if (nc - m == 0) return;
  const double zr = sh.zre[e], zi = sh.zim[e];
  const size_t fbb = hfactor_block_elems(b);
  double *We = W + 2 * (size_t)e * nc * fbb;
  hload_tiled<BP>(s.A, We + 2 * (size_t)(m - 1) * fbb, b);  // raw S_{m-1}
  __syncthreads();
  d4 tr[NT], ti[NT];
  {
    constexpr int LD = Lds<BP>::LD, PLANE = Lds<BP>::PLANE;
    const int w = wave_id(), l = lane_id();
    if (w < NT)
#pragma unroll
      for (int tj = 0; tj < NT; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = w * 16 + acc_row(l, r), col = tj * 16 + acc_col(l);
          // padding rows and columns of S_{m-1} hold the identity
          const bool in = row < b && col < b;
          tr[tj][r] = in ? s.A[row * LD + col] : (row == col ? 1.0 : 0.0);
          ti[tj][r] = in ? s.A[PLANE + row * LD + col] : 0.0;
        }
  }
  __syncthreads();
  hload_tiled<BP>(s.A, We + 2 * (size_t)m * fbb, b);  // W_m (bottom chain)
  hform_block<BP>(s.B, p, m - 1, 1, zr, zi);        // C_{m-1}
  __syncthreads();
  cgemm_lds<BP>(tr, ti, s.B, false, s.A, -1.0);  // S_{m-1} - C_{m-1} W_m
  __syncthreads();
  acc_to_lds<BP>(s.A, tr, ti);
  __syncthreads();
  gj_invert<BP>(s, nullptr, NoSide(), false);
  hstore_tiled<BP>(Sinv + 2 * ((size_t)e * nc + (m - 1)) * fbb, s.A, b);
}

// Self-energies across the partitions of a chain, one workgroup a chain, in
// chain order: partition q starts from D - K_q, K_q = Y Sinv_e X with X, Y
// the couplings between partitions q-1 and q and Sinv_e the exact inverse
// Schur complement at the last position of partition q-1.  K_1 = V X from
// the exact pass; otherwise partition q-1 started from D - K_{q-1}, and the
// Woodbury identity on its local inverse,
//   Sinv_e = GLL + GL1 K_{q-1} (I - G11 K_{q-1})^{-1} G1L,
// gives K_q = YGX + YH K_{q-1} (I - G11 K_{q-1})^{-1} XH.
template <int BP>
__global__ __launch_bounds__(kThreads) void hinterface_kernel(HPencil p, Shifts sh,
                                                              const double *V, double *work,
                                                              int P) {
  extern __shared__ double smem_raw[];
  Lds<BP> &s = *reinterpret_cast<Lds<BP> *>(smem_raw);
  constexpr int NT = BP / 16;
  const int ch = blockIdx.x, e = ch >> 1;
  const bool top = (ch & 1) == 0;
  const int nc = p.nc, b = p.b, m = nc - nc / 2;
  const int len = top ? m : nc - m;
  if (len <= 0 || P < 2) return;
  const double zr = sh.zre[e], zi = sh.zim[e];
  const size_t bb2 = 2 * hfactor_block_elems(b);  // work blocks: tiled
  double *wch = work + (size_t)ch * P * HW_COUNT * bb2;
  d4 ar[NT], ai[NT];
  {  // K_1 = V_c X at the last position of partition 0
    const int jl = hpart_start(1, len, P) - 1;
    const int c = top ? jl : nc - 1 - jl, cc = top ? c : c - 1;
    hload_tiled<BP>(s.A, V + ((size_t)e * nc + c) * bb2, b);
    hform_block<BP>(s.B, p, cc, top ? 1 : 2, zr, zi);
    __syncthreads();
    acc_fill<BP>(ar, ai, 0.0);
    cgemm_lds<BP>(ar, ai, s.A, false, s.B, 1.0);
    hacc_to_tiled<BP>(wch + ((size_t)HW_COUNT + HW_K) * bb2, ar, ai, b);
    __syncthreads();
  }
  for (int q = 2; q < P; ++q) {
    const double *wq = wch + (size_t)(q - 1) * HW_COUNT * bb2;
    hload_tiled<BP>(s.A, wq + HW_G11 * bb2, b);
    hload_tiled<BP>(s.B, wq + HW_K * bb2, b);
    __syncthreads();
    acc_fill<BP>(ar, ai, 1.0);
    cgemm_lds<BP>(ar, ai, s.A, false, s.B, -1.0);  // I - G11 K
    __syncthreads();
    acc_to_lds<BP>(s.A, ar, ai);
    __syncthreads();
    gj_invert<BP>(s, nullptr, NoSide(), false);
    acc_fill<BP>(ar, ai, 0.0);
    cgemm_lds<BP>(ar, ai, s.B, false, s.A, 1.0);  // U = K (I - G11 K)^{-1}
    __syncthreads();
    acc_to_lds<BP>(s.B, ar, ai);
    hload_tiled<BP>(s.A, wq + HW_YH * bb2, b);
    __syncthreads();
    acc_fill<BP>(ar, ai, 0.0);
    cgemm_lds<BP>(ar, ai, s.A, false, s.B, 1.0);  // YH U
    __syncthreads();
    acc_to_lds<BP>(s.A, ar, ai);
    hload_tiled<BP>(s.B, wq + HW_XH * bb2, b);
    __syncthreads();
    hacc_from_global<BP>(ar, ai, wq + HW_YGX * bb2, b);
    cgemm_lds<BP>(ar, ai, s.A, false, s.B, 1.0);  // K_q = YGX + YH U XH
    hacc_to_tiled<BP>(wch + ((size_t)q * HW_COUNT + HW_K) * bb2, ar, ai, b);
    __syncthreads();
  }
}

template <int BP>
hipError_t launch_hfactor_bp(const HPencil &p, const Shifts &s, int Ne, double *Sinv, double *W,
                             double *V, int P, double *work, hipStream_t st) {
  hipError_t err = set_lds<BP>((const void *)hfactor_part_kernel<BP>);
  if (err == hipSuccess) err = set_lds<BP>((const void *)hinterface_kernel<BP>);
  if (err == hipSuccess) err = set_lds<BP>((const void *)hfactor_twist_kernel<BP>);
  if (err != hipSuccess) return err;
  const size_t shm = sizeof(Lds<BP>);
  hipLaunchKernelGGL(hfactor_part_kernel<BP>, dim3(2 * Ne * (P > 1 ? P - 1 : 1)), dim3(kThreads),
                     shm, st, p, s, Sinv, W, V, work, P, 0);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if (P > 1) {
    hipLaunchKernelGGL(hinterface_kernel<BP>, dim3(2 * Ne), dim3(kThreads), shm, st, p, s,
                       (const double *)V, work, P);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(hfactor_part_kernel<BP>, dim3(2 * Ne * (P - 1)), dim3(kThreads), shm, st,
                       p, s, Sinv, W, V, work, P, 1);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  hipLaunchKernelGGL(hfactor_twist_kernel<BP>, dim3(Ne), dim3(kThreads), shm, st, p, s, Sinv, W);
  return hipGetLastError();
}

}  // namespace

size_t wide_pack_doubles(const Pencil &p) {
  return (size_t)(3 * p.nc - 2) * 2 * kWideBP * kWideBP;
}

WidePack wide_pack_planes(const Pencil &p, double *pack) {
  const size_t pair = 2 * (size_t)kWideBP * kWideBP;
  WidePack w;
  w.cpl = pack;
  w.cplt = pack + (size_t)(p.nc - 1) * pair;
  w.dia = pack + 2 * (size_t)(p.nc - 1) * pair;
  return w;
}

hipError_t launch_factor_wide(const Pencil &p, const Shifts &s, int Ne, const Factors &f,
                              double *pack, hipStream_t st) {
  if (p.bp != kWideBP || p.b > kWideBP || Ne < 1) return hipErrorInvalidValue;
  // the byte offsets of the packed diagonal blocks stay within 32 bits
  if ((size_t)p.nc * 2 * kWideBP * kWideBP * 8 > 0x7fffffffu) return hipErrorInvalidValue;
  const int shm = 2 * Lds<kWideBP>::PLANE * (int)sizeof(double);
  hipError_t err = hipFuncSetAttribute((const void *)factor_wide_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, shm);
  if (err != hipSuccess) return err;
  const WidePack w = wide_pack_planes(p, pack);
  const size_t total = (size_t)(3 * p.nc - 2) * kWideBP * kWideBP;
  const int grid = (int)std::min<size_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(pack_wide_kernel, dim3(grid), dim3(256), 0, st, p, w);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  hipLaunchKernelGGL(factor_wide_kernel, dim3(Ne), dim3(kWideThreads), shm, st, p, s, f,
                     (const double *)w.cpl, (const double *)w.dia);
  return hipGetLastError();
}

size_t hfactor_work_doubles(const HPencil &p, int Ne, int parts) {
  return parts > 1 ? (size_t)2 * Ne * parts * HW_COUNT * 2 * hfactor_block_elems(p.b) : 0;
}

hipError_t launch_hfactor_mfma(const HPencil &p, const Shifts &s, int Ne, double *Sinv,
                               double *W, double *V, int parts, double *work, hipStream_t st) {
  if (p.b < 1 || p.b > 64 || Ne < 1) return hipErrorInvalidValue;
  // every partition of both chains holds at least one cell
  if (parts < 1 || parts > std::max(1, p.nc / 2) || (parts > 1 && !work)) return hipErrorInvalidValue;
  switch ((p.b + 15) / 16 * 16) {
    case 16: return launch_hfactor_bp<16>(p, s, Ne, Sinv, W, V, parts, work, st);
    case 32: return launch_hfactor_bp<32>(p, s, Ne, Sinv, W, V, parts, work, st);
    case 48: return launch_hfactor_bp<48>(p, s, Ne, Sinv, W, V, parts, work, st);
    default: return launch_hfactor_bp<64>(p, s, Ne, Sinv, W, V, parts, work, st);
  }
}

size_t factor_work_doubles(const Pencil &p, int Ne, int parts) {
  return 3 * (size_t)Ne * 2 * parts * 2 * p.bp * p.bp;
}

hipError_t launch_factor(const Pencil &p, const Shifts &s, int Ne, const Factors &f, int parts,
                         double *work, Chain *chains, double *G, int gtiles, hipStream_t st) {
  if (parts < 1) return hipErrorInvalidValue;
  switch (p.bp) {
    case 16: return launch_factor_bp<16>(p, s, Ne, f, parts, work, chains, G, gtiles, st);
    case 32: return launch_factor_bp<32>(p, s, Ne, f, parts, work, chains, G, gtiles, st);
    case 48: return launch_factor_bp<48>(p, s, Ne, f, parts, work, chains, G, gtiles, st);
    case 64: return launch_factor_bp<64>(p, s, Ne, f, parts, work, chains, G, gtiles, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace feast
