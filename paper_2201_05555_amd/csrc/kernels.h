// Launch interface between the host orchestration and the HIP kernels.
#pragma once

#include <vector>
#include "common.h"

// Geometry of the particle-to-grid launches: nrb row blocks of rpb rows,
// parameter tiles of pt columns (pt * Nx doubles of LDS per table).
struct PicGeom {
  int nrb;
  int rpb;
  int pt;
};

// Up to eight N x k_s column blocks concatenated as one N x (sum k_s) matrix.
struct MatList {
  const cplx* ptr[8];
  int cols[8];
  int count;
};

// Up to eight real N x k column blocks.
struct RealList {
  const double* ptr[8];
  int count;
};

// gemm flags
enum { GEMM_B_REAL = 1, GEMM_A_REAL = 2, GEMM_NO_CONJ_A = 4, GEMM_SAME = 8 };  // SAME: internal

// Terms of a row-wise combination out = sum_s in_s M_s (in_s: N x k_s,
// M_s: k_s x m column-major with leading dimension ld[s], k_s when 0).
struct RowTerms {
  const cplx* in[4];
  const cplx* M[4];
  int k[4];
  int count;
  int ld[4];
};

// register width of the fused kernels: a count >= n, exact for the small
// ranks 2n = 10 and 14 (the position sums split into even and odd k, and the
// columns beyond n are zero, so every width gives the same cells)
inline int nc_even(int n) {
  if (n <= 4) return 4;
  if (n == 5) return 5;
  if (n <= 6) return 6;
  if (n == 7) return 7;
  if (n <= 8) return 8;
  if (n <= 12) return 12;
  return 16;
}
inline int nc_bucket(int n) {
  if (n <= 4) return 4;
  if (n <= 8) return 8;
  if (n <= 16) return 16;
  return 32;
}

// pic_kernels.hip
void launch_deposit_x(hipStream_t s, const double* X, int N, int p, int Nx, const PicGeom& g,
                      const double* factor, double* part);
// gate (nullable, device): when *gate == 0 the launch does nothing (the
// fixed point has converged: speculative iterations exit at once)
// fold (optional): the status words, given the end-of-step bookkeeping by
// one thread at the start (see fold_status_kernel)
// parameters per block of the reduced deposit on the matrix cores (n <= 16)
int deposit_tile_params(int Nx);
void launch_deposit_rom(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p, int Nx,
                        const PicGeom& g, const double* factor, const int* active, double* part,
                        const int* gate = nullptr,
                        int* fold = nullptr, int det = 0);
void launch_poisson(hipStream_t s, const double* part, int nrb, int p, int Nx, const double* qw,
                    const double* h, const double* mw, const int* active, double* rho,
                    double* phi, double* e, double* energy, const int* gate = nullptr);
// the Poisson solve followed, per parameter, by the DEIM gather of the
// sampled rows (gF, n x p) with the field just solved and, when counters is
// set, the fixed-point update of that column (see dense_fp_update_kernel;
// iter = the launch's ordinal in the solve, from 1)
void launch_poisson_deim(hipStream_t s, const double* part, int nrb, int p, int Nx,
                         const double* qw, const double* h, const double* mw, int* active,
                         double* rho, double* phi, double* e, double* energy, const int* gate,
                         const cplx* U, int N, int n, cplx* Z, const double* factor, double qm,
                         const int* idx, const double* w, int d, cplx* gF, const cplx* C12,
                         const cplx* Z0, cplx* ZG, cplx* k, double* prev, double dt, double tol,
                         double stall_tol, int fixed, int iter, int* counters);
void launch_fom_push(hipStream_t s, double* X, double* V, int N, int p, int Nx, const PicGeom& g,
                     const double* factor, const double* e, double qm, double ck, double cd,
                     double* part);
void launch_fom_velocity(hipStream_t s, const double* X, const double* V, int N, int p, int Nx,
                         const double* factor, const double* e, double qm, double c,
                         double* Vout);
void launch_cells(hipStream_t s, const double* X, int N, int p, int Nx, const double* factor,
                  int* cells);
void launch_colsumsq(hipStream_t s, const double* A, int N, int p, double sc, double* out,
                     double* scratch);  // scratch: 32 p doubles
void launch_vec_add(hipStream_t s, double* out, const double* in, int n);

// rom_kernels.hip
void launch_gather_rom(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p, int Nx,
                       const PicGeom& g, const double* factor, const double* e, double qm,
                       const int* active, bool full, void* out);
void launch_reconstruct(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p,
                        double* X, double* V, const int* rows = nullptr, int nrows = 0);
// cells j and scaled positions s = x N_x / L of every (particle, parameter)
// with the position arithmetic of the reduced deposit (cells: N x p int32;
// s: N x p, nullable)
void launch_rom_cells(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p, int Nx,
                      const double* factor, int* cells, double* sv);
void launch_gemm_ah_b(hipStream_t s, const MatList& A, int a, const MatList& B, int b, bool b_real,
                      int N, int nkb, cplx* part, cplx* C);
// C = op(A) B with flags (GEMM_*): real A / B inputs, A^T instead of A^*
void launch_gemm_flags(hipStream_t s, const MatList& A, int a, const MatList& B, int b, int flags,
                       int N, int nkb, cplx* part, cplx* C);
void launch_rowgemm(hipStream_t s, const RowTerms& T, int N, int m, cplx* out);
// the row combination and the Gram of [pre, out] ((kp + m) x (kp + m); pre
// optional, N x kp) in one pass over the rows; false (nothing launched) when
// m > 8, kp > 8 or the partials exceed part_cap
bool launch_rowgemm_gram(hipStream_t s, const RowTerms& T, int N, int m, cplx* out, cplx* part,
                         size_t part_cap, cplx* Gram, const cplx* pre = nullptr, int kp = 0);
// Fused gather + projection / basis velocity (G~ never stored); only for
// n with fused_gradient_ok(n).  launch_gather_project writes g (n x p) and,
// when want_colsq, |G~[:, c]|^2 into colsq; part holds part_cap complex.
// G12 = [U~^* U~, U~^T U~] of this U (the velocity part comes from them).
bool fused_gradient_ok(int n);
// Launch shape of the fused gather-projection: 16 cbn parameters per tile,
// their field rows in LDS (et_lds) or read from global memory, and at most
// nb_max row blocks.  launch_gather_project takes the shape set for (N, p,
// Nx, n) by set_gather_project_shape (process-wide), else a built-in rule.
struct GpShape {
  int cbn;
  bool et_lds;
  int nb_max;
};
std::vector<GpShape> gather_project_shapes(int N, int p, int Nx, int n, size_t part_cap);
void set_gather_project_shape(int N, int p, int Nx, int n, const GpShape* shape);
GpShape gather_project_shape(int N, int p, int Nx, int n, size_t part_cap);
void launch_gather_project(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p,
                           int Nx, const double* factor, const double* e, double qm,
                           const int* active, bool want_colsq, cplx* part, size_t part_cap,
                           cplx* g, double* colsq, const cplx* G12, const int* gate = nullptr);
// g (optional): the projection g~ (n x p); MU is then formed from g and Q
// inside the launch and the MU argument is not read
void launch_gather_xi(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p, int Nx,
                      const double* factor, const double* e, double qm, const cplx* Q,
                      const cplx* MU, double h, cplx* out, const cplx* g = nullptr);
// With start (and active == nullptr): also the DEIM reduced gradient
// k = -i (gF + (C1 Z - conj(C2) conj(Z)) / 2) (C12 = [C1, C2]), the first
// fixed-point iterate Zev = Z + h k, and the fixed-point start (prev = inf,
// all columns active, counters reset), each block for its own column.
struct DeimStartArgs {
  const cplx* C12;
  cplx* k;
  cplx* Zev;
  double h;
  double* prev;
  int* active;
  int* counters;
};
void launch_deim_gather(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, int p, int Nx,
                        const double* factor, const double* e, double qm, const int* idx,
                        const double* w, int d, const int* active, cplx* gF,
                        const int* gate = nullptr, const DeimStartArgs* start = nullptr);
void launch_snapshot(hipStream_t s, const cplx* U, int N, int n, const cplx* Z, const int* sub,
                     int psub, int Nx, const double* factor, const double* phi, double* Y,
                     const int* stop = nullptr);
// DEIM basis Psi = sum_s Y_s M_s with per-block column sums (psi_blocks(N)
// blocks, colpart[block][c]); fused greedy step k (per-block winners into
// bval, bidx from the previous pass pval, pidx); last index and weights.
int psi_blocks(int N);
void launch_psi_colsum(hipStream_t s, const double* const* in, int nin, int kin, int N,
                       const double* M, int ldM, int d, double* out, double* colpart);
void launch_deim_greedy(hipStream_t s, const double* Psi, int N, int k, int* idx,
                        const double* pval, const int* pidx, int nprev, int nblk, double* bval,
                        int* bidx, const double* Bprev, const double* uprev, double* Bnext,
                        double* cnext, int* flags, const int* forced = nullptr);
void launch_deim_weights(hipStream_t s, const double* Psi, int N, int d, int* idx,
                         const double* pval, const int* pidx, int nprev, const double* Bprev,
                         const double* uprev, const double* colpart, int ncp, double* w,
                         int* flags, const int* forced = nullptr);
// adaptive DEIM update: forced[k] = idx_old[k] for the positions kept, -1
// for the n_up positions whose basis vectors rotated most (part: psi_blocks(N)
// x d doubles of scratch)
void launch_deim_forced(hipStream_t s, const double* Pn, const double* Po, int N, int d, int n_up,
                        const int* idx_old, double* part, int* forced, const int* stop);

// dense_kernels.hip  (single-workgroup FP64 kernels on small matrices)
struct DenseCtl;  // device-resident control block, see dense_kernels.hip
void launch_dense_spinv(hipStream_t s, const cplx* Z, int n, int p, double rtol, cplx* Q,
                        double* sigma2, int* flags);
void launch_dense_xfinish(hipStream_t s, const cplx* g, const cplx* Q, int n, int p, double dt,
                          cplx* k1, cplx* MP, cplx* MU);
// chol: also one Cholesky-QR pass of the retraction's result from the 2n x 2n
// Gram alone (R^* R = its Gram): MU, MX returned times R^{-1}, Z <- R Z
void launch_dense_cayley(hipStream_t s, const cplx* Gram, int n, cplx* A_out, cplx* MU,
                         cplx* MX, int* flags, bool chol = false, cplx* Z = nullptr, int p = 0);
void launch_dense_tangent1(hipStream_t s, const cplx* A, const cplx* Gram2, int n, cplx* M1,
                           cplx* M2, cplx* M3, cplx* C0x_out, int* flags);
void launch_dense_tangent2(hipStream_t s, const cplx* Gram3, const cplx* C0x, int n, double dt,
                           cplx* M1, cplx* M2, int* flags);
// the whole tangent velocity from G4 = [U0, xi, Ux, X]^* [U0, xi, Ux, X] (4n x 4n):
// xi1 = X K1 + xi K2 + U0 K3 (n x n each)
void launch_dense_tangent(hipStream_t s, const cplx* G4, int n, double dt, cplx* K1, cplx* K2,
                          cplx* K3, int* flags);
// one Cholesky-QR pass: Gram = U~^* U~ = R^* R, U~ <- U~ R^{-1} (N rows), and
// Z~ <- R Z~ (n x p) when Z is given
void launch_cholqr_apply(hipStream_t s, const cplx* Gram, int n, cplx* U, int N, cplx* Z, int p,
                         int* flags);
void launch_dense_fp_update(hipStream_t s, const cplx* gF, const cplx* C12, int n, int p,
                            const cplx* Z0, cplx* Zeval, cplx* ZG, cplx* k, double* prev,
                            int* active, double dt, double tol, double stall_tol, int fixed,
                            int linear_part, int iter, int* counters);
void launch_dense_finish_z(hipStream_t s, const cplx* Z0, const cplx* k, int n, int p, double dt,
                           cplx* Z1);
void launch_fp_init(hipStream_t s, double* prev, int* active, int* counters, int p);
void launch_dense_herm_eig(hipStream_t s, cplx* A, int m, cplx* V, double* lam, int* flags);
void launch_fill_cplx(hipStream_t s, cplx* a, size_t n, cplx v);
void launch_copy_cplx(hipStream_t s, cplx* dst, const cplx* src, size_t n);
void launch_make_complex(hipStream_t s, const double* X, const double* V, size_t n, cplx* C);
void launch_split_complex(hipStream_t s, const cplx* C, size_t n, double* X, double* V);
void launch_ux_from_u(hipStream_t s, const cplx* U, int N, int n, double* UX);
void launch_u_from_ux(hipStream_t s, const double* UX, int N, int n, cplx* U);
void launch_z_from_real(hipStream_t s, const double* Z, int n, int p, cplx* Zc);
void launch_z_to_real(hipStream_t s, const cplx* Zc, int n, int p, double* Z);
void launch_dense_hh(hipStream_t s, cplx* Gp, const cplx* g, int n, int p, double* eps);
void launch_dense_grow_prep(hipStream_t s, const cplx* V, const double* lam, const cplx* g, int n,
                            int p, int k, cplx* W, cplx* T, int* flags);
void launch_colphase(hipStream_t s, cplx* U, int N, int col0, int k);
void launch_z_resize(hipStream_t s, const cplx* Zin, int nin, cplx* Zout, int nout, int p);
void launch_dense_shrink(hipStream_t s, const cplx* Z, int n, int p, cplx* V, cplx* Znew,
                         double* sig2);

void launch_dense_symeig(hipStream_t s, const cplx* G, int n, double* V, double* lam, int* flags);
void launch_dense_indicator(hipStream_t s, const double* colsq, const cplx* g, int n, int p,
                            double* eps);
// automatic shrink: *word = 0 when sigma_min(Z~) / sigma_max(Z~) > sqrt(c)
// is certified by a shifted Cholesky factor of Z~ Z~^*, else 1
void launch_dense_rank_cert(hipStream_t s, const cplx* Z, int n, int p, double c, int* word);
// singular values of Z~ (n x p) by one-sided Jacobi (work: n x p complex)
void launch_dense_zsvals(hipStream_t s, const cplx* Z, int n, int p, cplx* work, double* sig);
// Ik = I (k x k) and Cn = -C (n x k)
void launch_proj_mats(hipStream_t s, const cplx* C, int n, int k, cplx* Ik, cplx* Cn);
// Mc (optional, n x d): the DEIM basis coefficients V[:, c] / sqrt(lam_c)
void launch_dense_topeig(hipStream_t s, const double* G, int n, int d, double* V, double* lam,
                         int* flags, const int* stop = nullptr, double* Mc = nullptr);
// error-word bookkeeping at the end of a step with the DEIM chain
void launch_fold_status(hipStream_t s, int* status);
void launch_gram_block_real(hipStream_t s, const double* Ynew, const double* const* slots,
                            int nslots, int psub, int N, int r0, int nkb_cap, double* part,
                            double* S, const int* stop = nullptr);

// ensemble_kernels.hip (large ensembles)
// G[a0.., b0..] = blk (ac x bc) and its conjugate transpose at [b0.., a0..]
void launch_scatter_block(hipStream_t s, const cplx* blk, int ac, int bc, cplx* G, int p, int a0,
                          int b0);
// W = A V (A p x p, V p x m, ld p)
void launch_herm_mm(hipStream_t s, const cplx* A, const cplx* V, int p, int m, cplx* W);
// orthonormalise the m <= 64 columns of W (p x m, ld p) in place
void launch_cgs2(hipStream_t s, cplx* W, int p, int m);
// initial ensemble of a family (0 Landau, 1 two-stream) from eta (device,
// p x 4: alpha, k, v0, sigma) and shared uniforms ux, uv (device [N]):
// X, V (N x p, nullable) and/or C = X + i V (nullable)
void launch_load_family(hipStream_t s, int family, int N, int p, const double* eta,
                        const double* ux, const double* uv, double* X, double* V, cplx* C);

// dmd_kernels.hip (DMD-DEIM: Sec. 4.1, Sec. 4.2.1 Alg. 1, eq. grHDD, Alg. 2)
// subset of eq. pSampl: pstar column indices of Z~ (n x p) into S; dmin: p doubles
void launch_subset_select(hipStream_t s, const cplx* Z, int n, int p, int pstar, double* dmin,
                          int* S);
// radial basis weights beta (p x pstar, row i contiguous) of the subset
// nodes S for parameters eta (device, dim per parameter); member: p ints
void launch_rbf_weights(hipStream_t s, const double* eta, int dim, int p, const int* S, int pstar,
                        int* member, double* beta, int* flags);
// rows `cols` (or the first k) of a p x Nx grid into a k x Nx block
void launch_grid_rows(hipStream_t s, const double* src, const int* cols, int k, int Nx,
                      double* dst);
// columns S of Z~ (n x p) into a compact n x k block
void launch_gather_zcols(hipStream_t s, const cplx* Z, int n, const int* S, int k, cplx* out);

// buffers of the DMD of the subset potentials (all device)
struct DmdChainArgs {
  const double* ring;  // nslots blocks of pstar x Nx: the window levels
  int nslots, base;    // level t in slot (base + t) % nslots, t = 0 .. T
  int pstar, T, Nx;
  double tol;          // relative singular value cut of Alg. 1
  double *Y, *Yp, *W;  // Nx x P each (P = pstar T): data, shifted data, QR work
  double *sig, *V;     // P, P x P: singular values and right vectors (sorted)
  int* rdev;           // retained rank r
  double *B, *U, *A;   // Nx x P, Nx x P, P x P (r used)
  double* M;           // r x r: Re(W Lambda^{1/2} W^{-1})
  cplx* lam;           // r eigenvalues of A_tol
  double *Wb, *Wf;     // Nx x P, Nx x pstar: QR work for B^+
  double* C;           // r x pstar: subset coordinates B^+ Phi_{tau-1}
  double* BM;          // Nx x P: B M
  int* flags;
};
// window matrices, SVD, A_tol, its eigendecomposition and M, coordinates
void launch_dmd_operator(hipStream_t s, const DmdChainArgs& c);
// predicted field tables e0 (t_{tau-1}) and eh (t_{tau-1} + dt/2), p x Nx
void launch_dmd_tables(hipStream_t s, const DmdChainArgs& c, int p, const double* beta,
                       const double* h, double* e0, double* eh);

// the fixed point of the coefficients with the DMD-DEIM gradient, whole
struct DmdFpArgs {
  const cplx *U0, *Uh;  // bases at t_{tau-1} and at the half step (N x n)
  int N, n;
  const int* idx;       // d DEIM rows
  const double* w;      // d DEIM weights
  int d;
  const cplx* Z0;       // n x p
  const double* factor; // Nx / L per parameter
  const double *e0, *eh;  // p x Nx field tables
  int Nx;
  double qm;
  const cplx *C12a, *C12;  // [U~^* U~, U~^T U~] at U0 and at U_half
  double dt, tol, stall_tol;
  int max_iters, fixed;
  cplx *k, *ZG;
  double* prev;
  int* active;
  int* counters;        // [0] left, [1] stalled, [2] iterations, [6..7] stall max (zeroed first)
};
void launch_dmd_fp(hipStream_t s, const DmdFpArgs& a, int p);
