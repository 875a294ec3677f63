/*
 * symrom.h -- C ABI of the MI355X library for the dynamical symplectic
 * reduced model of the parametric particle-based 1D1V Vlasov-Poisson
 * system (Hesthaven, Pagliantini, Ripamonti, arXiv:2201.05555), and of the
 * particle-in-cell full-order model it is compared against.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All functions are extern "C" and return symrom_status (0 = OK,
 *   negative = error); the text of the last error of the calling thread is
 *   available from symrom_last_error().
 * - Array arguments are DEVICE pointers (memory of the current HIP device)
 *   unless the comment says "host".  Particle arrays are FP64, N x p,
 *   column-major (leading dimension N): column i belongs to parameter i.
 *   Positions are unwrapped; they are reduced modulo the domain length only
 *   inside the particle-to-cell lookup.
 * - The reduced basis crosses the boundary as U_X (N x 2n, column-major,
 *   ld = N), the position rows of the orthosymplectic U = [U_X; U_V]
 *   (Sec. 3.2); U_V = U_X J_2n is implied (the orthosymplectic structure
 *   forces U = [[A, -B], [B, A]]).  Coefficients Z are 2n x p, ld = 2n.
 * - Memory: the library never allocates device memory.  The caller passes a
 *   workspace `ws` of at least *_workspace_bytes() bytes, borrowed until the
 *   handle is destroyed.  Host arrays are read during the call only.
 * - Streams: all work is enqueued on the caller's `stream` (a hipStream_t,
 *   passed as void*).  Functions that return host data synchronise that
 *   stream; the others return once work is enqueued, except rom_step and
 *   fom_step, which read small device flags to drive the fixed point and so
 *   synchronise the stream at least once per step.
 * - A handle is used by one host thread at a time.
 * - Physical units: q = -1, m = 1 and the weight of the N macro-particles
 *   of parameter i is L_i / N, so that their charge cancels the uniform
 *   unit background on [0, L_i) (Sec. 2 background remark, Sec. 6.1).
 */
#ifndef SYMROM_H
#define SYMROM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t symrom_status;
enum {
  SYMROM_OK = 0,
  SYMROM_EINVAL = -1,     /* bad sizes, odd rank, null pointers, ...        */
  SYMROM_ENOMEM = -2,     /* workspace smaller than *_workspace_bytes()     */
  SYMROM_ESINGULAR = -3,  /* a small dense matrix could not be factorised   */
  SYMROM_ENOCONV = -4,    /* fixed point not converged within fp_max_iters  */
  SYMROM_EDEVICE = -5,    /* a HIP call failed                              */
  SYMROM_ESTATE = -6,     /* handle not initialised                          */
  SYMROM_ERANKCAP = -7    /* rank growth beyond two_n_max requested          */
};

enum { SYMROM_GALERKIN = 0, SYMROM_DEIM = 1, SYMROM_DMD_DEIM = 2 };

typedef struct {
  int32_t N;             /* particles                                        */
  int32_t p;             /* parameters of the ensemble                       */
  int32_t Nx;            /* grid cells (= nodes) of the periodic P1 mesh     */
  int32_t two_n;         /* reduced dimension 2n (even)                      */
  int32_t two_n_max;     /* capacity for rank growth (even, >= two_n, <= 60) */
  double dt;             /* time step                                        */
  double q, m;           /* charge and mass (-1 and 1 in the paper)          */
  int32_t projection;    /* SYMROM_GALERKIN, SYMROM_DEIM (exact potential) or */
                         /* SYMROM_DMD_DEIM (Alg. 2: DMD of the potential,  */
                         /* DEIM of Lambda^0 Phi_DMD, basis evolved on the  */
                         /* parameter subset of eq. pSampl)                 */
  int32_t deim_window;   /* T: DEIM snapshots of the last T+1 time levels    */
  double fp_tol;         /* fixed point: relative update threshold           */
  int32_t fp_max_iters;  /* fixed point: iteration cap (ENOCONV beyond)      */
  int32_t fp_fixed_iters;/* >0: run exactly this many iterations, no test    */
  double pinv_rtol;      /* S(Z)^+ drops eigenvalues < pinv_rtol * max       */
  int32_t reorth;        /* 1: FP64 re-orthonormalisation after each step    */
  int32_t rank_auto;     /* 1: apply the rank indicator after each step      */
  double rank_tol_up;    /* grow one pair when eps_perp exceeds this         */
  double fp_stall_tol;   /* a column whose relative update stops decreasing  */
                         /* is accepted only when the smaller of its last   */
                         /* two updates is below this (else it iterates on; */
                         /* ENOCONV at fp_max_iters); 0: 1e-3               */
  double rank_tol_down;  /* automatic shrink: drop the pairs whose singular  */
                         /* value of Z~ is below this times the largest     */
  int32_t deim_rows;     /* d, DEIM sample rows; 0: d = 2n (capped by the    */
                         /* snapshot count p*(T+1))                          */
  int32_t precision;     /* SYMROM_FP64 (the only arithmetic built)          */
  int32_t deterministic; /* 1: theta sums of the reduced deposit as 64-bit   */
                         /* integers in units of 2^-40, so the charge and    */
                         /* everything after it is bitwise reproducible      */
  int32_t deim_update_every; /* k_DEIM: the DEIM indices by the full greedy */
                         /* every k-th operator (0 or 1: every step)         */
  int32_t deim_update_rows;  /* n_DEIM: positions chosen again in between    */
                         /* (those of the most rotated basis vectors, eq.    */
                         /* indices_adaptive_DEIM); the others are inherited */
  int32_t p_star;        /* SYMROM_DMD_DEIM: size p* of the parameter subset */
                         /* (Sec. 4.1; 0: p); p*(T+1) <= 64, p* T <= 48      */
  int32_t reserved;
  double dmd_tol;        /* SYMROM_DMD_DEIM: relative singular value cut of  */
                         /* Alg. 1, step 1 (0: 1e-5, the value of Sec. 6.1)  */
} symrom_config;

enum { SYMROM_FP64 = 0 };

typedef struct {
  int32_t iters;          /* fixed-point iterations of the last step          */
  int32_t stalled;        /* columns accepted by the stagnation rule          */
  int32_t two_n;          /* rank after the call                              */
  int32_t deim_active;    /* 1 if the last step used the DEIM gradient        */
  double rank_indicator;  /* eps_perp of the last evaluation, -1 if none      */
  int32_t iters_total;    /* fixed-point iterations summed over the call      */
  int32_t deim_steps;     /* steps of the call that used the DEIM gradient    */
  double stall_rel;       /* largest relative update accepted by the          */
                          /* stagnation rule over the call (0 if none)        */
  int32_t stalled_total;  /* stagnation acceptances summed over the call      */
  int32_t shrunk;         /* pairs dropped by the automatic shrink, last step */
  double worst_rel;       /* on ENOCONV: the largest last relative update of  */
                          /* the columns still iterating (else 0)             */
  int32_t unconverged;    /* on ENOCONV: the number of those columns          */
  int32_t reserved;
} symrom_step_info;

typedef struct symrom_rom symrom_rom;
typedef struct symrom_fom symrom_fom;

/* ------------------------------------------------------------------------
 * Reduced model (Sec. 3.2 eq. UZred, time stepping Sec. 5 eq. discrete_dynROM)
 * ------------------------------------------------------------------------ */

/* Exact workspace bytes rom_init needs for this configuration; 0 when the
 * configuration is invalid. */
size_t rom_workspace_bytes(const symrom_config* cfg);

/* Create a reduced-model handle and initialise U, Z by the truncated complex
 * SVD of R_0 = [X0; V0] (Sec. 3.2, initial condition of eq. UZred):
 * U~ = leading n left singular vectors of X0 + i V0 (largest-modulus entry of
 * each made real positive, completed by Gram-Schmidt of e_1, e_2, ... when
 * n exceeds the numerical rank), Z~ = U~^* (X0 + i V0).
 *   cfg       host, copied.
 *   L         host [p]: domain length of each parameter (2 pi / k_i).
 *   X0, V0    device, N x p column-major, unwrapped initial states.
 *   ws        device workspace, >= rom_workspace_bytes(cfg) bytes.
 *   stream    hipStream_t.
 *   out       host: receives the handle.
 * Errors: EINVAL (config), ENOMEM (ws too small), EDEVICE. */
symrom_status rom_init(const symrom_config* cfg, const double* L, const double* X0,
                       const double* V0, void* ws, size_t ws_bytes, void* stream,
                       symrom_rom** out);

/* rom_init with the initial ensemble loaded on the device (Sec. 6.1: the
 * perturbed Maxwellian f0 = f_v(v) (1 + alpha cos kx) on [0, 2 pi / k) x
 * [-10, 10], sampled by inverse CDF with uniforms shared by every
 * parameter; see symrom_load_family), so that no N x p host array is ever
 * formed.  family: 0 Landau (f_v = N(0, sigma)), 1 two-stream
 * (f_v = (N(-v0, sigma) + N(v0, sigma)) / 2).  eta: host, p x 4 row-major
 * (alpha, k, v0, sigma) per parameter; L_i = 2 pi / k_i.  ux, uv: device [N]
 * uniforms in (0, 1).  Other arguments and errors as rom_init (EINVAL also
 * for k <= 0, sigma <= 0 or non-finite eta). */
symrom_status rom_init_family(const symrom_config* cfg, int32_t family, const double* eta,
                              const double* ux, const double* uv, void* ws, size_t ws_bytes,
                              void* stream, symrom_rom** out);

/* Advance the whole ensemble by nsteps steps of the order-2 partitioned
 * Runge-Kutta scheme (Sec. 5): implicit midpoint for Z solved by per-column
 * fixed point (relative update < fp_tol, Sec. 6.1), explicit midpoint for U
 * on the tangent space through the Cayley retraction, with the Galerkin or
 * DEIM (Sec. 4.2.2, eq. grHDD with the exact potential) gradient.  A column
 * whose relative update stops decreasing is accepted when the smaller of its
 * last two updates is below fp_stall_tol (a node crossing of the
 * piecewise-constant gathered force makes the iterates cycle between jumps
 * and contraction steps); the largest update so accepted is
 * info->stall_rel.  With
 * rank_auto the rank is updated after every step (see rom_adapt_rank, target
 * 0).  With SYMROM_DMD_DEIM (Alg. 2) the first T steps are the plain
 * reduced step, recording the snapshot and the potential of the subset S of
 * eq. pSampl at the start of each; from then on the basis evolves with the
 * exact gradient of S only (eq. UZredhyp), the coefficients of every
 * parameter with the DMD-DEIM gradient of eq. grHDD: the potential predicted
 * by the DMD of the last T+1 subset potentials (Alg. 1, eq.
 * DMD_approx_potential_subset, coordinates interpolated over the parameters
 * outside S), evaluated at the d DEIM particles (Sec. 4.2.2), at t_{tau-1}
 * for the start value and t_{tau-1} + dt/2 for the implicit midpoint stage.
 * info (host, nullable) describes the last step.  On ENOCONV the state
 * (U, Z and the snapshot and potential windows) is the one before the
 * failing step. */
symrom_status rom_step(symrom_rom* h, int32_t nsteps, symrom_step_info* info);

/* Replace the fixed-point controls of the following steps (fp_tol,
 * fp_max_iters, fp_fixed_iters as in symrom_config).  Host-only. */
symrom_status rom_set_fixed_point(symrom_rom* h, double fp_tol, int32_t fp_max_iters,
                                  int32_t fp_fixed_iters);

/* Change the rank.  target_two_n > current: append (target - current)/2
 * symplectic pairs, the leading left singular vectors of
 * (I - U~U~^*)(-i G~) at the current state (orthonormalised against the
 * basis and among themselves), with zero coefficient rows (R = U Z
 * unchanged).  target < current: rotate to the singular vectors of Z~ and
 * drop the trailing pairs.  target 0: grow one pair if the indicator
 * eps_perp = ||(I - U U^T) J G|| / ||G|| exceeds rank_tol_up and the cap
 * allows; otherwise drop the pairs whose singular value of Z~ is below
 * rank_tol_down times the largest (at least one pair stays).  (The paper
 * defers rank adaptation to future work, Sec. 6.4.)  new_two_n: host,
 * nullable.  Errors: ERANKCAP beyond two_n_max, EINVAL for odd targets,
 * ESINGULAR when the new directions cannot be formed (the state is then
 * unchanged). */
symrom_status rom_adapt_rank(symrom_rom* h, int32_t target_two_n, int32_t* new_two_n);

/* Copy the state out: U_X (N x 2n, ld N) and Z (2n x p, ld 2n), device;
 * two_n and step are host, nullable.  Synchronises the stream. */
symrom_status rom_get_state(symrom_rom* h, double* UX, double* Z, int32_t* two_n, int64_t* step);

/* Replace the state by (U_X, Z) of rank two_n (device, layouts as above).
 * U_X must be the position rows of an orthosymplectic basis.  Clears the
 * DEIM snapshot window. */
symrom_status rom_set_state(symrom_rom* h, int32_t two_n, const double* UX, const double* Z,
                            int64_t step);

/* R = U Z: positions X_r = U_X Z and velocities V_r = U_V Z (device, N x p). */
symrom_status rom_reconstruct(symrom_rom* h, double* X, double* V);

/* R = U Z on a subset of particle rows (Sec. 3.2, eq. UZred): rows (device
 * int32 [nrows]) lists the rows; X, V (device, nrows x p, column-major,
 * ld nrows; each nullable) receive X_r and V_r of those rows.  A row index
 * outside [0, N) gives NaN in its output row.  Synchronises the stream. */
symrom_status rom_reconstruct_rows(symrom_rom* h, const int32_t* rows, int32_t nrows, double* X,
                                   double* V);

/* The particle-to-cell map of the reduced model (Sec. 2.1, node index of
 * x = Re(U~ Z~) with the position arithmetic of the fused deposit, gather and
 * projection kernels): cells (device int32, N x p) and, nullable, the scaled
 * positions s = x N_x / L (device, N x p) whose floor gives the cell.  Z
 * (device, 2n x p, nullable) replaces the handle's coefficients for this call
 * only.  Synchronises the stream. */
symrom_status rom_cells(symrom_rom* h, const double* Z, int32_t* cells, double* s);

/* The DEIM operator of the last DEIM step (Sec. 4.2.2; with rank_auto it is
 * the one already built for the next step): the d sample indices in greedy
 * order (device int32, capacity >= d) and the weights w = (P^T Psi)^{-T}
 * Psi^T 1 of eq. grHDD (device, capacity >= d); d (host, nullable).
 * Errors: ESTATE when no DEIM operator has been built yet. */
symrom_status rom_deim_operator(symrom_rom* h, int32_t* idx, double* w, int32_t* d);

/* SYMROM_DMD_DEIM: the ensemble's parameters for the Gaussian radial basis
 * interpolation of the DMD coordinates over the parameters outside the
 * subset (Sec. 4.2.1): eta (host, p x dim row-major, dim <= 8; e.g. alpha,
 * k, v0, sigma).  Each coordinate is scaled to [0, 1] by its range over the
 * ensemble; the kernel width is the median distance between subset nodes.
 * rom_init_family sets them itself (dim 4); rom_init handles need this call
 * before their first DMD-DEIM step (else that step fails with ESTATE).
 * Errors: EINVAL (not a DMD-DEIM handle, dim, non-finite eta), ESINGULAR
 * (interpolation matrix not positive definite: coincident subset nodes). */
symrom_status rom_set_parameters(symrom_rom* h, const double* eta, int32_t dim);

/* SYMROM_DMD_DEIM: the subset S of eq. pSampl (host int32, capacity >= p*,
 * nullable) and p* (host, nullable); of the last DMD-DEIM step the DMD rank
 * r (host, nullable), the eigenvalues of A_tol (Alg. 1; host, 2 r doubles
 * re/im interleaved, nullable) and the predicted field tables e = (Phi_DMD
 * (x_{j+1}) - Phi_DMD(x_j)) / h of every parameter at t_{tau-1} (e0) and at
 * t_{tau-1} + dt/2 (eh) (device, p x Nx row-major, nullable).  Errors:
 * ESTATE (not a DMD-DEIM handle). */
symrom_status rom_dmd_state(symrom_rom* h, int32_t* S, int32_t* pstar, int32_t* rank, double* lam,
                            double* e0, double* eh);

/* Tile autotuning of the fused gather-projection (the dominant kernel of
 * the reduced step, eq. grads) for this handle's sizes (N, p, N_x, n): every
 * launch shape that fits (16, 32 or 64 parameters per tile, their field rows
 * in LDS or read from global memory, 256 to 1024 row blocks) is timed on the
 * handle's current state (three launches after one untimed), and the
 * fastest, when at least 3 % faster than the built-in rule, is kept for
 * every later launch of these sizes in the process (all handles).  Results
 * differ between shapes only by the rounding of the row-block partial sums.
 * Out (host, nullable): the shape kept and the time per launch of it and of
 * the rule (ms).  Errors: ESTATE for a deterministic handle (it keeps the
 * built-in shape, so that its results repeat bitwise across processes) or
 * for a rank beyond the fused kernels (2n > 32); EDEVICE if a timed launch
 * failed (the rule is kept). */
symrom_status rom_autotune(symrom_rom* h, int32_t* cbn, int32_t* et_lds, int32_t* nb_max,
                           double* best_ms, double* rule_ms);

/* Scratch bytes for rom_step_hamiltonian_split: U_{tau-1/2} (N x n_max
 * complex) and Z_tau (n_max x p complex), 256-byte aligned. */
size_t rom_hamiltonian_split_bytes(const symrom_rom* h);

/* One step as rom_step (without rank adaptation) that also returns the four
 * Hamiltonians of the splitting of the step's Hamiltonian change (Sec. 6.2,
 * eq. error_ham_tot), per parameter, in H4 (device, 4 x p row-major):
 * H(U_{tau-1} Z_{tau-1}), H(U_{tau-1/2} Z_{tau-1}), H(U_{tau-1/2} Z_tau),
 * H(U_tau Z_tau), with H(UZ) = |V_r|^2 / 2 + E(X_r) (eq. HamEEfull).  The
 * change |H_3 - H_0| is bounded by the two basis terms |H_3 - H_2| and
 * |H_1 - H_0| and the coefficient term |H_2 - H_1|.  Z_tau is taken before
 * the re-orthonormalisation (which rotates U_tau and Z_tau together and
 * leaves U_tau Z_tau unchanged).  scratch: device, at least
 * rom_hamiltonian_split_bytes(h) bytes, 256-byte aligned, caller-owned.
 * Every projection, DMD-DEIM steps included (H is the Hamiltonian of the
 * full model at the reconstructed state, not the DMD-DEIM approximation).
 * Errors as rom_step (on failure the state is the one before the step and
 * H4 is not written); EINVAL for a null pointer or a small or misaligned
 * scratch. */
symrom_status rom_step_hamiltonian_split(symrom_rom* h, void* scratch, size_t scratch_bytes,
                                         double* H4, symrom_step_info* info);

/* Singular values of the initial state C0 = X0 + i V0 (N x p) that
 * rom_init or rom_init_family decomposed (the complex SVD of the
 * initialisation, Sec. 6.1), in decreasing order, as the square roots of the
 * eigenvalues of C0^* C0: all p of them for p <= 64, the n = two_n/2
 * leading ones beyond.  With V0 = 0 they are the singular values of the
 * local snapshot matrix S_X = [X^1 ... X^p] of eq. local_snapshots, whose
 * count above tol * sigma_1 is the numerical rank of Sec. 6.1 (values below
 * about 1e-7 sigma_1 are not resolved through the Gram).  sig: host, up to
 * cap values written; *m: the number available.  Errors: EINVAL. */
symrom_status rom_init_singular_values(symrom_rom* h, double* sig, int32_t cap, int32_t* m);

/* Per-parameter electric energy E(X_r^i) (eq. HamEEfull) and Hamiltonian
 * H = 1/2 |V_r^i|^2 + E (device [p] each). */
symrom_status rom_diagnostics(symrom_rom* h, double* E, double* H);

/* Galerkin reduced gradient at (current U, Z): g = U^T G (eq. grads), device
 * 2n x p; and, nullable, rho, Phi, e (device, Nx x p) of the deposit
 * (eq. PoissonSystem plus background), the zero-mean potential and the cell
 * field (Phi_{j+1} - Phi_j)/h. */
symrom_status rom_gradient(symrom_rom* h, const double* Z, double* g, double* rho, double* Phi,
                           double* e);

/* Release the handle (the workspace is the caller's). */
void rom_destroy(symrom_rom* h);

/* ------------------------------------------------------------------------
 * Full-order particle-in-cell model (Sec. 2.1, Stormer-Verlet eq. sv_full_order)
 * ------------------------------------------------------------------------ */

size_t fom_workspace_bytes(int32_t N, int32_t p, int32_t Nx);

/* Create a full-order handle holding X, V (copied from X0, V0, device,
 * N x p) in its workspace. */
symrom_status fom_init(int32_t N, int32_t p, int32_t Nx, double dt, double q, double m,
                       const double* L, const double* X0, const double* V0, void* ws,
                       size_t ws_bytes, void* stream, symrom_fom** out);

/* fom_init with the initial ensemble loaded on the device: family, eta
 * (host, p x 4), ux, uv (device [N]) as in rom_init_family. */
symrom_status fom_init_family(int32_t N, int32_t p, int32_t Nx, double dt, double q, double m,
                              int32_t family, const double* eta, const double* ux,
                              const double* uv, void* ws, size_t ws_bytes, void* stream,
                              symrom_fom** out);

/* nsteps Stormer-Verlet steps for every parameter:
 * X+ = X + dt (V + dt/2 a(X)),  V+ = V + dt/2 (a(X) + a(X+)),
 * a = -(q/m) e_{j(X)} the acceleration of eq. VPHamEqn. */
symrom_status fom_step(symrom_fom* h, int32_t nsteps);

/* Copy X, V out (device, N x p). Synchronises the stream. */
symrom_status fom_get_state(symrom_fom* h, double* X, double* V);

/* Electric energy and Hamiltonian per parameter (device [p]). */
symrom_status fom_diagnostics(symrom_fom* h, double* E, double* H);

void fom_destroy(symrom_fom* h);

/* ------------------------------------------------------------------------
 * Stateless particle-to-grid pieces (Sec. 2.1), for tests and tools
 * ------------------------------------------------------------------------ */

/* Initial particle states of an ensemble (Sec. 6.1 loading): for particle l
 * and parameter i, x = F_x^{-1}(ux[l]) with F_x(x) = (x + (alpha_i / k_i)
 * sin k_i x) / L_i by Newton kept in [0, L_i], and v = F_v^{-1}(lo + uv[l]
 * (hi - lo)), lo, hi = F_v(-10), F_v(10), for the Gaussian (family 0) or the
 * two-beam mixture (family 1) of spread sigma_i (and drift v0_i), by the
 * inverse normal CDF (family 0) or bracketed Newton (family 1).  eta:
 * DEVICE, p x 4 row-major (alpha, k, v0, sigma); ux, uv: device [N]; X, V:
 * device N x p (column-major; each nullable).  Synchronises the stream. */
symrom_status symrom_load_family(int32_t family, int32_t N, int32_t p, const double* eta,
                                 const double* ux, const double* uv, double* X, double* V,
                                 void* stream);

/* Workspace bytes for deim_select; 0 unless 1 <= d <= 64 and d <= N. */
size_t deim_select_workspace_bytes(int32_t N, int32_t d);

/* Greedy DEIM selection (Sec. 4.2.2) on a given orthonormal basis Psi
 * (device, N x d, column-major): idx[0] = argmax |psi_1|, then for k >= 2
 * the index of the largest |r_k|, r_k = psi_k - Psi_{k-1} (P^T Psi_{k-1})^{-1}
 * P^T psi_k (ties to the smaller index); and the weights
 * w = (P^T Psi)^{-T} Psi^T 1 of eq. grHDD.  idx (device int32 [d]), w (device
 * [d]).  The kernels are those of the reduced step.  Errors: EINVAL, ENOMEM,
 * ESINGULAR when a residual vanishes everywhere (rank-deficient basis). */
symrom_status deim_select(int32_t N, int32_t d, const double* Psi, int32_t* idx, double* w,
                          void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for pic_fields. */
size_t pic_workspace_bytes(int32_t N, int32_t p, int32_t Nx);

/* For positions X (device, N x p): cell index j (device int32 N x p,
 * nullable; j = floor(x N_x / L) mod N_x with the factor N_x / L formed in
 * FP64), rho, Phi, e (device Nx x p, each nullable).  L host [p]. */
symrom_status pic_fields(int32_t N, int32_t p, int32_t Nx, const double* L, double q,
                         const double* X, int32_t* cells, double* rho, double* Phi, double* e,
                         void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): pic_fields without a workspace
 * and without any allocation.  L is a DEVICE array [p] here (no host memory
 * is touched); X, cells, rho, Phi, e as in pic_fields.  The deposit
 * partials, the per-parameter constants and the energies live in a
 * file-scope device array of SYMROM_NOALLOC_SCRATCH_BYTES per GPU, held
 * until the process ends; every word a call reads is written by that call
 * first.  Calls that overlap on one GPU share that array and race: issue
 * them one after another.  Errors: EINVAL for bad sizes and when p * Nx is
 * too large for the array (about 5e5 grid values); use pic_fields then.
 * Synchronises the stream. */
#define SYMROM_NOALLOC_SCRATCH_BYTES (8u << 20)
symrom_status pic_fields_noalloc(int32_t N, int32_t p, int32_t Nx, const double* L, double q,
                                 const double* X, int32_t* cells, double* rho, double* Phi,
                                 double* e, void* stream);

/* ------------------------------------------------------------------------
 * Serving: a request loop over ensembles of parameter queries
 * ------------------------------------------------------------------------
 * A request is one ensemble (family, eta of its p parameters, N shared
 * uniforms, a rank configuration) advanced by nsteps reduced steps from its
 * initial condition (rom_init_family, rom_step).  Requests arriving at any
 * time are admitted, in arrival order but without head-of-line blocking,
 * when one of `slots` worker threads is free and their device memory
 * (srv_request_bytes: the exact workspace, the uniforms, the results) fits
 * in the free space of the caller's pool; each runs on a stream of its own,
 * so admitted requests overlap on the device.  U and Z stay resident in the
 * request's workspace for all its steps.  Ensembles are never merged (U
 * depends on all parameters of its ensemble).  With cfg->deterministic = 1 a
 * request's results are bitwise the same alone and in any mix.  The pool
 * (device memory, borrowed until srv_destroy) is the only device memory the
 * server uses; host copies of the request's inputs are kept until it runs. */
typedef struct symrom_server symrom_server;
typedef struct {
  int32_t status;     /* 1 queued, 2 running, 0 done, negative: its error    */
  int32_t two_n;      /* rank at the end                                     */
  int64_t steps_done; /* nsteps when done, -1 on error                       */
  double t_arrival;   /* seconds on the server's clock: submission,          */
  double t_start;     /* admission to a worker,                              */
  double t_finish;    /* results ready                                       */
  double pp_steps;    /* N p nsteps                                          */
} symrom_request_info;

/* Device bytes a request holds while it runs (0 for an invalid config). */
size_t srv_request_bytes(const symrom_config* cfg, int32_t nrows);

/* Start a server with `slots` worker threads (1..64) on the current device;
 * pool: device memory of pool_bytes. */
symrom_status srv_create(int32_t slots, void* pool, size_t pool_bytes, symrom_server** out);

/* Queue a request: cfg (host, copied), family 0 Landau / 1 two-stream, eta
 * (host, p x 4: alpha, k, v0, sigma), ux, uv (HOST [N] uniforms, copied),
 * nsteps, and nrows particle rows (host int32, copied) whose X_r, V_r are
 * returned.  id: host.  Errors: EINVAL; ENOMEM when the request could never
 * fit the pool. */
symrom_status srv_submit(symrom_server* sv, const symrom_config* cfg, int32_t family,
                         const double* eta, const double* ux, const double* uv, int32_t nsteps,
                         int32_t nrows, const int32_t* rows, int64_t* id);

/* State and times of a request (host). */
symrom_status srv_info(symrom_server* sv, int64_t id, symrom_request_info* info);

/* Block until the request is done; returns its status. */
symrom_status srv_wait(symrom_server* sv, int64_t id);

/* Block until every queued request is done; peak_pool_bytes (host,
 * nullable) receives the largest pool occupancy so far. */
symrom_status srv_drain(symrom_server* sv, double* peak_pool_bytes);

/* Results of a finished request (host arrays, each nullable): the electric
 * energy and Hamiltonian per parameter (p each, eq. HamEEfull), X_r and V_r
 * of the requested rows (nrows x p, column-major).  ESTATE while it runs. */
symrom_status srv_result(symrom_server* sv, int64_t id, double* E, double* H, double* X,
                         double* V);

/* Finish the requests already admitted, drop the queued ones, stop. */
void srv_destroy(symrom_server* sv);

/* ------------------------------------------------------------------------ */
const char* symrom_status_string(symrom_status s);
const char* symrom_last_error(void);

/* Accumulated device time (ms) of the kernels the library launched on the
 * handle's stream since the last call, measured with HIP events around each
 * launch of the named kernel family when timing is enabled by
 * symrom_set_timing(1).  family: 0 = reconstruct-and-deposit, 1 = fused
 * gather-projection (g = U~^* G~), 2 = Poisson (histogram sum and solve),
 * 3 = FOM push, 4 = basis (tall-skinny Grams and row combines), 5 = dense
 * (small matrices, DEIM greedy), 6 = DEIM eigenpairs (top d of the snapshot
 * Gram), 7 = fused gather-basis-velocity (xi = -i h G~ Q + U~ M), 8 = the
 * rest of the DEIM chain on the second stream (snapshot, snapshot Gram block,
 * basis Psi, greedy passes, weights).  Counts launches in *launches (host,
 * nullable). */
void symrom_set_timing(int32_t on);
double symrom_kernel_ms(int32_t family, int64_t* launches);

/* Algorithmic work of the timed launches of a family since the last call:
 * flops and HBM bytes as counted by the operation definitions (not by
 * hardware counters).  Reconstruct-and-deposit: 4n flops per
 * particle-parameter (x = Re(U~ Z~), n complex products), bytes = U~ and Z~
 * read once plus the charge written (8 Nx per active parameter; the
 * per-row-block partial histograms are traffic of this design, not of the
 * operation).  Gather-projection: (8n + 4) flops per particle-parameter,
 * bytes = U~ and Z~ read and g written once.  Gather-basis-velocity: 8n flops per particle-parameter plus
 * 8n^2 per particle, bytes = U~ read and xi written.  DEIM eigenpairs:
 * 4P^3/3 + 2P^2 d + 2P d^2 flops for the tridiagonal reduction,
 * back-transform and orthonormalisation of a P x P Gram, no HBM bytes
 * beyond the matrix.  FOM push: 32 bytes per particle-parameter (read and
 * write X and V) plus the histograms.  flops, bytes: host, nullable. */
void symrom_kernel_work(int32_t family, double* flops, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* SYMROM_H */
