// Host-side launchers of the FEAST kernels (implemented in *.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace feast {

constexpr int kMaxNe = 64;
constexpr int kTile = 8;  // complex right-hand sides per solve chain

// Contour data passed by value to the kernels that need it.
struct Shifts {
  double zre[kMaxNe], zim[kMaxNe];   // Z_e
  double kre[kMaxNe], kim[kMaxNe];   // kappa_e
};

struct Pencil {
  const double *Ad, *Au, *Bd, *Bu;   // caller blocks, row stride b
  int nc, b, bp;                     // bp = b rounded up to 16
};

// Twisted block factorisation of every (Z_e B - A): top chain 0..m-1
// top-down, bottom chain nc-1..m bottom-up, twist cell m-1.
struct Factors {
  double *Sinv, *W, *WT;   // [Ne][nc][2][bp][bp]
  double *TW;              // [Ne][2][bp][bp] raw Schur complement at the twist cell
  int m;                   // twist split
};

// One chain of cells processed by one workgroup of the factor kernels.
struct Chain {
  int e;      // node
  int start;  // first cell
  int len;    // number of cells
  int dir;    // +1 top-down, -1 bottom-up
  int end;    // last cell: 0 invert only, 1 keep raw S (twist cell), 2 invert + W
  int kin;    // incoming self-energy in Kbuf (-1: none): S_start = D_start - K
  int half;   // 0 top, 1 bottom
  int part;   // partition index within the half
};

// Partitioned exact factorisation (see factor.hip).  parts = partitions per
// half (1: one chain per half).  work: device workspace from
// factor_work_doubles(); chains: device buffer for 3 * Ne * 2 * parts Chain.
size_t factor_work_doubles(const Pencil &p, int Ne, int parts);
hipError_t launch_factor(const Pencil &p, const Shifts &s, int Ne, const Factors &f, int parts,
                         double *work, Chain *chains, double *G, int gtiles, hipStream_t st);

// Blocks of 64 < b <= 96 (bp = 96): one top-down chain per node over all
// cells (no twist: f.m unused, Sinv, W and W^T of every cell; W and W^T of
// the last cell unused).  pack: wide_pack_doubles() of workspace for the
// blocks of the pencil repacked in the operand layout (written by
// launch_factor_wide, read by the wide dense products below).
struct WidePack {
  double *cpl;   // [nc-1][2][96*96]: A_{c,c+1}, B_{c,c+1}
  double *cplt;  // [nc-1][2][96*96]: their transposes
  double *dia;   // [nc][2][96*96]: A_cc (identity padding as -1), B_cc
};
size_t wide_pack_doubles(const Pencil &p);
WidePack wide_pack_planes(const Pencil &p, double *pack);
hipError_t launch_factor_wide(const Pencil &p, const Shifts &s, int Ne, const Factors &f,
                              double *pack, hipStream_t st);

// Spike solves of the partitioned factorisation (sweep.hip): for every chain,
// the first and last block of T^{-1} E_1 where T is the chain's local matrix.
hipError_t launch_spikes(const Pencil &p, const Factors &f, const Chain *chains, int nchains,
                         int parts, int gtiles, double *G, double *G11, double *GL1,
                         hipStream_t st);

// Forward/back sweeps of all Ne shifts for right-hand side R (real,
// padded [nc][bp][m0p]); writes P[e] = Re(kappa_e x_e) (padded, per node).
struct SolveBufs {
  double *G;    // [Ne][ntiles][nc][2][bp][8]
  double *TV;   // [Ne][ntiles][2][2][bp][8]: twist vectors (h_{m-1}, c)
};
// part: 1 = forward sweep only, 2 = back sweep only, 3 = both.
// skip (here and in the launchers below): NULL, or a device flag that the
// kernels read first; non-zero makes them return at once (the loops of a
// captured solve after convergence).
hipError_t launch_sweeps(const Pencil &p, const Shifts &s, int Ne, const Factors &f,
                         const SolveBufs &sb, const double *R, int m0p, double *P, int part,
                         hipStream_t st, const int *skip = nullptr);
// The sweeps of the wide factorisation (launch_factor_wide): Xim == nullptr:
// P[e] = Re(kappa_e x_e) (padded, per node); else the complex solution of
// node 0 in P (real plane) and Xim.  sb.G as for launch_sweeps, sb.TV unused.
hipError_t launch_sweeps_wide(const Pencil &p, const Shifts &s, int Ne, const Factors &f,
                              const SolveBufs &sb, const double *R, int m0p, double *P,
                              double *Xim, int part, hipStream_t st, const int *skip = nullptr);
// Same sweeps, but the back sweep writes the complex solution of node 0
// (used by the single-shift entry point): X_re, X_im padded.
hipError_t launch_sweeps_complex(const Pencil &p, const Shifts &s, const Factors &f,
                                 const SolveBufs &sb, const double *R, int m0p,
                                 double *Xre, double *Xim, hipStream_t st);

// Mixed precision (sweep32.hip): the factor blocks rounded to float32 in
// the layout of the float32 sweeps, and the float32 sweeps for a complex
// right-hand side per node.
struct Factors32 {
  float *Sinv, *W, *WT;  // [Ne][nc][2][bp][bp]
  int m;                 // twist split
};
struct SolveBufs32 {
  float *G;   // [Ne][ntiles][nc][2][bp][8]
  float *TV;  // [Ne][ntiles][2][2][bp][8]
};
hipError_t launch_round_factors(const Pencil &p, int Ne, const Factors &f, const Factors32 &g,
                                hipStream_t st);
// Right-hand side of node e: real plane at R + e * rnode (padded
// [nc][bp][m0p], float64), imaginary plane one plane (nc*bp*m0p doubles)
// further when rcomplex.  X: node e's iterate, real plane at X + 2 e plane,
// imaginary plane after it; accumulate: X += solution, else X = solution.
hipError_t launch_sweeps32(const Pencil &p, int Ne, const Factors32 &f, const SolveBufs32 &sb,
                           const double *R, size_t rnode, int rcomplex, int m0p, double *X,
                           int accumulate, int part, hipStream_t st);

// Dense helpers (dense.hip).
// Fig. 2 step 1: seeded N(0,1) start block (Philox4x64-10 + Box-Muller),
// written in the packed layout of launch_pack (zero padding).
hipError_t launch_random_start(unsigned long long seed, int nc, int b, int bp, int m, int ldd,
                               double *dst, hipStream_t st);
hipError_t launch_pack(const double *src, int nc, int b, int bp, int m, int ldd,
                       double *dst, hipStream_t st);
hipError_t launch_unpack(const double *src, int nc, int b, int bp, int m, int lds,
                         const int *perm, double *dst, hipStream_t st);
hipError_t launch_sum_nodes(const double *P, int Ne, size_t count, double *Q,
                            hipStream_t st, const int *skip = nullptr);
hipError_t launch_gemm_qphi(const double *Q, size_t rows, int m0p, int m0,
                            const double *Phi, double *X, hipStream_t st,
                            const int *skip = nullptr);
hipError_t launch_check_finite(const double *x, size_t count, int *flag, hipStream_t st);
hipError_t launch_gather(const double *src, const int *perm, int m, double *dst,
                         hipStream_t st);

// Per-cell products (one workgroup walks a strided set of cells; ld <= 128,
// a multiple of 16).  partial: cell_partial_doubles(nc, ld) doubles, which
// also covers the 3 ld per group of the residual variant.
size_t cell_partial_doubles(int nc, int ld);
hipError_t launch_cell_apply(const Pencil &p, int which, const double *V, int ld, double *out,
                             hipStream_t st, const int *skip = nullptr);
hipError_t launch_cell_project(const Pencil &p, const double *Q, int ld, int m0, double *partial,
                               double *AQ, double *BQ, hipStream_t st,
                               const int *skip = nullptr);
hipError_t launch_cell_residuals(const Pencil &p, const double *X, int ld, const double *lam,
                                 int m0, double emin, double emax, double *partial, double *res,
                                 hipStream_t st, const int *skip = nullptr);

// The same products for 64 < b <= 96 (p.bp = 96) from the packed planes of
// launch_factor_wide: out = T V (which: 0 = A, 1 = B), the projection
// (tmp: [nc][96][ld] doubles, partial: cross_gram_partial_doubles(nc*96, m0,
// m0)) and the residuals (partial: wide_residual_partial_doubles()).
hipError_t launch_wide_apply(const Pencil &p, const WidePack &pk, int which, const double *V,
                             int ld, double *out, hipStream_t st, const int *skip = nullptr);
size_t wide_residual_partial_doubles(int nc, int ld);
hipError_t launch_wide_residuals(const Pencil &p, const WidePack &pk, const double *X, int ld,
                                 const double *lam, int m0, double emin, double emax,
                                 double *partial, double *res, hipStream_t st,
                                 const int *skip = nullptr);
hipError_t launch_wide_project(const Pencil &p, const WidePack &pk, const double *Q, int ld,
                               int m0, double *tmp, double *partial, double *AQ, double *BQ,
                               hipStream_t st, const int *skip = nullptr);

// Float64 residuals of the shifted systems for the mixed-precision solves:
// Rout_e = R - (Z_e B - A) x_e for every node (X and Rout: node e's real
// plane at + 2 e plane, imaginary plane after it; R real, shared), and
// worst = max over nodes and columns j < m0 of ||r_j|| / (||R_j|| +
// |Z_e| ||B x_j|| + ||A x_j||) in 2-norms (one double).  partial:
// shift_residual_partial_doubles().
size_t shift_residual_partial_doubles(int nc, int ld, int Ne);
hipError_t launch_shift_residuals(const Pencil &p, const Shifts &s, int Ne, const double *X,
                                  const double *R, int ld, int m0, double *Rout, double *partial,
                                  double *worst, hipStream_t st);
// Q = sum_e Re(kappa_e x_e) over the complex iterates (layout as above).
hipError_t launch_sum_nodes_complex(const Shifts &s, int Ne, const double *X, size_t plane,
                                    double *Q, hipStream_t st);

// Reduced eigenproblem (rr.hip): a few workgroups running the same Jacobi
// (each keeps a slice of the eigenvector rows), then a small kernel for Phi.
// scratch: reduced_eig_scratch_doubles().  eps, Phi outputs; flag[0] =
// fallback, flag[1] = Jacobi sweeps, flag[2] = sweeps of the fallback.
size_t reduced_eig_scratch_doubles();
// Device address (on the current device) of the reduced eigensolver's
// file-scope scratch array and of its flags, for the allocation-free entry
// point; called once per context at initialisation.
hipError_t reduced_eig_static_scratch(double **ptr, int **flag);
hipError_t launch_reduced_eig(const double *AQ, const double *BQ, int n, double *eps,
                              double *Phi, double *scratch, int *flag, hipStream_t st,
                              const int *skip = nullptr);
// Sets the reduced eigensolver's LDS limit (launch_reduced_eig does it
// itself, except while its stream is being captured).
hipError_t reduced_eig_set_lds();

// Convergence of one loop on the device (same decisions, in the same
// arithmetic, as the host loop of feast_solve): counts the in-interval pairs
// with residual <= gate, sums their Ritz values in index order, applies the
// trace test and the uncounted-pair wait, appends to the history in st and
// sets st->done once the solve has converged or reached max_loops.  Does
// nothing once done is set.  One thread.
struct DevConv {
  int k;            // loops done
  int done;         // converged or out of loops: later loop kernels skip
  int converged;
  int fallback;     // the last loop's B_Q fallback flag
  int rr_sweeps;    // Jacobi sweeps, all loops
  int counts[64];   // M_k (first 64 loops)
  double traces[64];
  double trace_rel;
  double prev_left_min;
  double last_trace;
  int last_count;
};
hipError_t launch_converge(const double *eps, const double *res, const int *flag, int m0,
                           double emin, double emax, double gate, double tol, double r,
                           double drop, int max_loops, DevConv *st_dev, hipStream_t st);


// Learned warm start (warm.hip).  bfloat16 values are stored as uint16_t.
// C_partial[z] = A B^T over split z of K (A [M][K], B [N][K], K and kc
// multiples of 16); gemm_splits(K, kc) partials of M*N floats.
int gemm_splits(int K, int kc);
hipError_t launch_gemm_nt(const uint16_t *A, const uint16_t *B, int M, int N, int K, int kc,
                          float *P, hipStream_t st);
// Sum of partials, bias, ReLU (relu) or ReLU-derivative mask, outputs
// float32 / bfloat16 / bfloat16 transposed (any may be null).
hipError_t launch_finish(const float *P, int splits, int M, int N, const float *bias, int relu,
                         const uint16_t *mask, float *outf, uint16_t *outb, uint16_t *outbt,
                         hipStream_t st);
hipError_t launch_cast_bf16(const float *x, int M, int N, uint16_t *xb, uint16_t *xbt,
                            hipStream_t st);
int mse_partials(int M, int N);
hipError_t launch_mse(const float *y, const float *t, int M, int N, float *dyf, uint16_t *dyb,
                      uint16_t *dybt, double *partial, double *loss, hipStream_t st);
hipError_t launch_colsum(const float *D, int M, int N, float *out, hipStream_t st);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, size_t n, int rows, int cols,
                       float lr, float b1, float b2, float eps, float c1, float c2, uint16_t *wb,
                       uint16_t *wbt, hipStream_t st);
size_t cross_gram_partial_doubles(long long N, int m, int m2);
hipError_t launch_cross_gram(const double *X, int ldx, const double *V, int ldv, long long N, int m,
                             int m2, double *partial, double *G, hipStream_t st);
hipError_t launch_tall_gemm(const double *X, int ldx, const double *G, long long N, int m, int m2,
                            double *T, hipStream_t st);
hipError_t launch_cell_gram(const double *T, int nc, int b, int m, double *Gc, hipStream_t st);
hipError_t launch_basis_project(const double *U, const double *T, int nc, int b, int r, int m,
                                double scale, float *C, hipStream_t st);
hipError_t launch_basis_expand(const double *U, const float *C, int nc, int b, int r, int m,
                               double scale, const double *R, double rscale, double *Y,
                               hipStream_t st);

// Hermitian variant (herm.hip).  Complex values are interleaved (re, im).
// Blocks up to kMaxHBlock (the factor kernel holds one complex b x (b+1)
// block in LDS: 149 KB at b = 96).
constexpr int kMaxHBlock = 96;
struct HPencil {
  const double *Ad, *Au;   // complex [nc][b][b], [nc-1][b][b] (A Hermitian)
  const double *Bd, *Bu;   // real, B s.p.d.
  int nc, b;
};
size_t hfactor_lds_bytes(int b);
// Blocks of the Hermitian factors for b <= 64 are stored as 4 x 4 tiles of
// complex elements, tiles row-major: element (i, j) at complex offset
// ((i/4) bt + j/4) 16 + (i%4) 4 + j%4, bt = ceil(b/4), so that both the
// sixteen-row fragments of M and those of M^H read whole tiles; a block holds
// (4 bt)^2 elements (entries outside b x b finite).  Blocks above 64 are
// plain [b][b].
__host__ __device__ inline int htile_dim(int b) { return (b + 3) / 4 * 4; }
__host__ __device__ inline size_t hfactor_block_elems(int b) {
  return b <= 64 ? (size_t)htile_dim(b) * htile_dim(b) : (size_t)b * b;
}
// Block LU of Z_e B - A for every node: Sinv, W and V [Ne][nc] blocks of
// hfactor_block_elems(b) complex elements (b > 64: W and V use the first
// max(nc-1,1) blocks of a node).
// For b <= 64 each half chain is cut into `parts` partitions (1 <= parts <=
// max(1, nc/2)) factored through their corner blocks and a sequential
// self-energy pass; work holds hfactor_work_doubles() doubles (none for one
// partition).  Blocks above 64 ignore parts and work.
hipError_t launch_hfactor(const HPencil &p, const Shifts &s, int Ne, double *Sinv, double *W,
                          double *V, int parts, double *work, hipStream_t st);
size_t hfactor_work_doubles(const HPencil &p, int Ne, int parts);
// The same factorisation for b <= 64 on the matrix cores (factor.hip), which
// launch_hfactor takes for those blocks.
hipError_t launch_hfactor_mfma(const HPencil &p, const Shifts &s, int Ne, double *Sinv,
                               double *W, double *V, int parts, double *work, hipStream_t st);
// Both solves of every node for the complex right-hand side R [N][m]:
// G [Ne][2][N][m] = (M_e^{-1} R, M_e^{-H} R), followed by the sweeps' twist
// slots; G holds hsweep_work_doubles() doubles.
size_t hsweep_work_doubles(const HPencil &p, int Ne, int m);
hipError_t launch_hsweeps(const HPencil &p, int Ne, const double *Sinv, const double *W,
                          const double *V, const double *R, int m, double *G, hipStream_t st);
// The same sweeps for b <= 64 on the matrix cores (sweep.hip), which
// launch_hsweeps takes for those blocks.
hipError_t launch_hsweeps_mfma(const HPencil &p, int Ne, const double *Sinv, const double *W,
                               const double *V, const double *R, int m, double *G,
                               hipStream_t st);
// Q = sum_e c_e x_e + conj(c_e) y_e over G (Nm = N*m complex entries per slot).
hipError_t launch_haccumulate(const double *G, int Ne, size_t Nm, const double *cre,
                              const double *cim, double *Q, hipStream_t st);
// out = A V (which 0) or B V (which 1), complex V and out [N][m].
hipError_t launch_happly(const HPencil &p, int which, const double *Vin, int m, double *out,
                         hipStream_t st);
// outA = A V and outB = B V in one pass over V where the blocks allow it.
hipError_t launch_happly_pair(const HPencil &p, const double *Vin, int m, double *outA,
                              double *outB, hipStream_t st);
// The same products for b <= 64 on the matrix cores (sweep.hip), which
// launch_happly and launch_happly_pair take for those blocks; which 2
// writes A V to out and B V to out2.
hipError_t launch_happly_mfma(const HPencil &p, int which, const double *V, int m, double *out,
                              hipStream_t st, double *out2 = nullptr);
size_t hgram_partial_doubles(long long N, int m);
// G = Hermitian part of X^H V (complex [m][m], m <= 64).
hipError_t launch_hgram(const double *X, const double *Vin, long long N, int m, double *partial,
                        double *G, hipStream_t st);
// The complex Hermitian-definite A_Q Phi = eps B_Q Phi (m <= 64) as a real
// symmetric tridiagonal T (with I, real [m][m]) for launch_reduced_eig, and
// Z (complex [m][m]) with Phi = Z V_T; scratch holds 2 (m+1)^2 doubles.
// flag[3] = 1 (nothing else written) when B_Q fails the Cholesky pivot
// test, else 0.
hipError_t launch_htridiag(const double *AQ, const double *BQ, int m, double *T, double *I,
                           double *Z, double *scratch, int *flag, hipStream_t st);
// Phi = Z VT (Z complex, VT real, [m][m]).
hipError_t launch_hcombine(const double *Z, const double *VT, int m, double *Phi, hipStream_t st);
hipError_t launch_hembed(const double *AQ, const double *BQ, int m, double *EA, double *EB,
                         hipStream_t st);
hipError_t launch_hextract(const double *eps2, const double *Phi2, int m, double *eps,
                           double *Phi, hipStream_t st);
hipError_t launch_htall_gemm(const double *X, const double *G, long long N, int m, int m2,
                             double *T, hipStream_t st);
// partial holds hgram_partial_doubles(N, m) doubles.
hipError_t launch_hresiduals(const double *AX, const double *BX, const double *lam, long long N,
                             int m, double emin, double emax, double *partial, double *res,
                             hipStream_t st);
hipError_t launch_hgather(const double *in, const int *perm, long long N, int m, double *out,
                          hipStream_t st);

}  // namespace feast
