/* csipm — sparse 3D-DFT recovery by a matrix-free primal-dual interior-point
 * method on one AMD Instinct MI355X (gfx950).
 *
 * Method: Kuang, Rao, Montoison, Pacaud, Anitescu, "Recovering sparse DFT
 * from missing signals via interior point method on GPU" (arXiv 2502.04217).
 * The library solves
 *     beta* = argmin_beta 1/2 ||b - M_perp beta||^2 + lambda ||beta||_1
 * (paper, equation "realopt"), where M_perp are the observed rows of the real
 * orthogonal operator A = IDFT o B^H that maps the real parametrisation beta
 * of a conjugate-symmetric spectrum to a real 3D signal (section "Problem
 * formulation", equations "beta", "v", derivation "map").
 *
 * Conventions shared by every entry point
 *  - Grid: N1 x N2 x N3, each a product 2^a 3^b 5^c 7^d in [3, 1024] (the
 *    FFT passes have radix-2^k, -3, -5 and -7 stages: register-resident
 *    kernels for the powers of two, the paper's sizes 96, 192, 384, 560 and
 *    the small extents 12-70, 3-45 that have them; kernels holding the
 *    pencils in LDS, with a radix plan computed at launch, for the rest);
 *    N1 and N2 may also be 1 or 2, so a 2D problem is the grid 1 x N2 x N3
 *    and a 1D one 1 x 1 x N3.  Any axis may be odd (the odd-N case of the
 *    parametrisation, section "Problem formulation": no Nyquist index on
 *    that axis; an odd N3 runs the transforms on the whole spectrum, with
 *    twice the bytes of the half-spectrum passes, and when N1*N2*N3 is odd
 *    the library adds internally one coordinate with no data, a zero column
 *    of A, which the solution sets to 0).  n = N1*N2*N3.
 *    Other extents return CSIPM_EUNSUPPORTED.
 *  - Real-space arrays are row-major [N1][N2][N3] (index j3 fastest).
 *  - beta-space arrays ("external beta layout") are row-major [N1][N2][N3]
 *    indexed by the frequency k: beta[k] = v_k for self-conjugate k
 *    (k == -k mod N), and for the canonical member k of each pair {k, -k}
 *    beta[k] = sqrt2 Re v_k, beta[-k] = sqrt2 Im v_k, with v the unitary
 *    3D DFT.  k is canonical iff k3 in [1, N3/2), or k3 in {0, N3/2} and
 *    k2 in [1, N2/2), or k3, k2 in {0, N/2} and k1 in [1, N1/2).
 *  - All pointers named d_* are device pointers (HIP, the current device);
 *    all buffers are owned by the caller and must outlive the context.
 *  - Work is queued on the HIP stream given at creation.  Calls that return
 *    host scalars (csipm_lambda_rule, csipm_solve, csipm_get_residuals)
 *    synchronise that stream; all others are asynchronous.
 *  - Every call returns a csipm_status: 0 success, > 0 success with a
 *    warning (the result is usable), < 0 failure (no outputs written).
 *    csipm_last_error gives a message for the last failure on a context.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef CSIPM_H
#define CSIPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct csipm_ctx csipm_ctx;

typedef enum {
  CSIPM_OK = 0,
  CSIPM_NOT_CONVERGED = 1, /* iteration limit reached; iterate usable          */
  CSIPM_STALLED = 2,       /* the precision floor was reached: a step along
                              a Newton direction that missed its tolerance
                              raised rel_kkt (the iterate before that step
                              is returned), or rel_kkt rose above 10x its
                              best value; iterate usable                     */
  CSIPM_FELL_BACK = 3,     /* converged, but some Newton systems fell back to
                              the paper's preconditioner                       */
  CSIPM_EINVAL = -1,       /* bad argument (null pointer, size, lambda <= 0)   */
  CSIPM_ENOMEM = -2,       /* workspace too small                              */
  CSIPM_EHIP = -3,         /* a HIP runtime call failed                        */
  CSIPM_ENONFINITE = -4,   /* NaN/Inf in an observed sample or an iterate      */
  CSIPM_EUNSUPPORTED = -5, /* grid size not supported                          */
  CSIPM_ESTATE = -6        /* call out of order (e.g. solve before lambda)     */
} csipm_status;

typedef enum { CSIPM_FP64 = 0, CSIPM_FP32 = 1 } csipm_precision;
/* Preconditioner of the Newton systems (sec. "Krylov methods and
 * preconditioners"): the paper's P = [[I + L1, L2], [L2, L1]]; P with the
 * learned diagonal correction C = diag(c) in place of I; or the scaled
 * identity rho I in place of I (the variant the paper compares P with). */
typedef enum { CSIPM_PC_PLAIN = 0, CSIPM_PC_LEARNED = 1, CSIPM_PC_SCALED = 2 } csipm_pc;
/* Krylov method of the Newton systems (section "Krylov methods and
 * preconditioners" lists CG, CR and CAr for SPD systems): CG; conjugate
 * residuals (CR): alpha = (z.Kz)/(q.P^{-1}q), one K-apply per iteration,
 * residual minimised in the P^{-1} norm; conjugate A-residuals (CAr): CR
 * applied to the A-residual K z, ||K z|| minimised in the P^{-1} norm, one
 * K-apply per iteration after two at the start.  CAr's residual stops
 * decreasing near 1e-9 relative on ill-conditioned systems (late FP64
 * interior-point iterations at tight tolerances). */
typedef enum { CSIPM_KRYLOV_CG = 0, CSIPM_KRYLOV_CR = 1, CSIPM_KRYLOV_CAR = 2 } csipm_krylov;
typedef enum {
  CSIPM_BETA = 0, CSIPM_Z = 1, CSIPM_NU1 = 2, CSIPM_NU2 = 3,
  CSIPM_XI = 4,       /* M_perp^T b, fixed at creation                        */
  CSIPM_DIAG_H = 5,   /* diag(M_perp^T M_perp), fixed at creation             */
  CSIPM_PC_C = 6      /* current learned correction c (1 = paper's P)          */
} csipm_var;

/* Interior-point options (paper: "Primal-dual interior-point method"; the
 * barrier strategy is the library's, the paper leaves it to the IPM).       */
typedef struct {
  double tol;          /* stop at rel_kkt <= tol (default 1e-6)               */
  int max_iter;        /* interior-point iterations (default 200)             */
  int cg_max;          /* PCG iterations per Newton system (default 500)      */
  double cg_rtol;      /* relative PCG tolerance cap (default 1e-2); the
                          tolerance used is min(cg_rtol, 0.1 rel_kkt)          */
  double cg_atol;      /* absolute floor on the preconditioned residual norm
                          (default 0; 1e-12 with cg_rtol = 0 reproduces the
                          paper's rule)                                        */
  double sigma;        /* centring parameter (default 0.1)                    */
  double tau;          /* fraction to the boundary (default 0.99)             */
  int precision;       /* csipm_precision of the Krylov solves               */
  int pc;              /* csipm_pc                                           */
  int refine_max;      /* FP32: refinement steps per Newton system (def. 8)  */
  double refine_inner_rtol; /* FP32: tightest relative tolerance asked of one inner
                               PCG solve (default 1e-5); each inner solve aims at
                               half the remaining reduction, at most 1e-2     */
  double refine_trust; /* FP32: Newton systems whose tolerance min(cg_rtol,
                          0.1 rel_kkt) is at least this (default 2e-6) take
                          the FP32 solution (inner tolerance half of it)
                          without an FP64 residual pass; the residual of the
                          iterate then carries FP32-level error until it is
                          recomputed in FP64, which happens before every
                          stopping test and before the first system below
                          the threshold.  The first time the solve would
                          stall after such a step (a step that raised
                          rel_kkt, or rel_kkt 10x above its best), the
                          trust is revoked for the rest of the solve: the
                          step is undone where a snapshot holds the iterate
                          before it, and every later system is refined.
                          0 = always refine.                              */
  int pc_min_cg;       /* learned correction: applied to a Newton system only
                          when the previous system took at least this many
                          PCG iterations (default 2; the first system and
                          systems after a one-iteration solve use the paper's
                          P, which already makes them one-iteration solves);
                          0 = every system                                   */
  int krylov;          /* csipm_krylov (default CG); the learned
                          correction's training capture needs CG             */
  double pc_rho;       /* CSIPM_PC_SCALED: rho (default 0 = m/n, the
                          observed fraction: H = M_perp^T M_perp has mean
                          diagonal m/n)                                      */
  double pc_max_relevant; /* learned correction: applied only when at most
                          this fraction of the coefficients are relevant,
                          L1 / (L1 + 4 S1 S2) >= 1e-3 at the current
                          iterate (default 0.5).  Early iterates have every
                          coefficient relevant and need one or two PCG
                          iterations with the paper's P, so evaluating the
                          network on all n coefficients cannot pay; late
                          iterates have the relevant set near the support,
                          where the network runs on few chunks.  1 = no
                          limit.                                              */
  int mehrotra;        /* 1: Mehrotra predictor-corrector steps (default 0):
                          an affine direction (target 0) and its step to the
                          boundary give mu_a and sigma = (mu_a/mu)^3 (at
                          least 0.1 tol (1 + |xi|_inf) / mu); a second solve
                          with the same K, whose complementarity rows carry
                          the affine ds * dnu, gives the step.  Fewer
                          interior-point iterations, two Krylov solves each.
                          Not from the paper, which leaves the barrier update
                          to its solver; Mehrotra's scheme on the condensed K
                          (eq. condensedkkt) with the rows of eq. kktmu. */
  int build_next;      /* 1 (default): the iterate update of a standard CG
                          step also builds the next Newton system (Sigma,
                          h, r, p) from the new iterate, at the target sigma
                          mu+ formed from the step's sums, when that system's
                          precision and preconditioner can be foreseen; a
                          system the next iteration cannot use is rebuilt.
                          0: every system is built by its own pass.  Saves
                          a pass over the state per iteration; the result
                          differs from 0 only by rounding. */
  int graphs;          /* 1 (default): from a context's second solve on,
                          PCG chunks are recorded once per context as HIP
                          graphs and replayed (one launch per chunk of 2-16
                          iterations instead of about ten per iteration;
                          what small grids gain).  0: every kernel is
                          launched directly.  Not used while kernel timing
                          or sample capture is on.  Same kernels and
                          arguments, so the same results. */
  double pc_min_missing; /* learned correction: used only when at least this
                          fraction of the samples is missing (default 0.01,
                          the least in the training family of the shipped
                          parameters: lattice period 32, cubes of half-width
                          3, 1.05 %).  Below it the paper's P is nearly K
                          itself and the network would act outside the range
                          it was trained on, so the solve runs with the
                          paper's P, exactly as CSIPM_PC_PLAIN.  0 = no limit.
                          A policy capture (csipm_capture mode 2) follows the
                          same rule. */
} csipm_options;

typedef struct {
  int status;
  int ipm_iters;
  int cg_iters_max;         /* largest PCG count of one Newton system          */
  long long cg_iters_total; /* sum over Newton systems (inner FP32 + FP64)     */
  int refine_steps_total;
  int fallbacks;            /* learned -> plain preconditioner restarts        */
  double rel_kkt;           /* max(|F_beta|_inf, |F_z|_inf, max s.nu)/(1+|xi|_inf) */
  double res_beta_inf, res_z_inf, compl_max;
  double mu;
  double lambda;
  double xi_inf;
  double solve_seconds;
  /* LASSO certificate of the returned beta (equation "realopt" and its
   * dual max b^T theta - 1/2 ||theta||^2 s.t. ||M_perp^T theta||_inf <=
   * lambda), from g = M_perp^T (b - M_perp beta) = xi - H beta evaluated by
   * an FP64 apply of H; M_perp^T is an isometry on the observed samples,
   * so ||b - M_perp beta|| = ||g||:
   *   objective     P = 1/2 ||b - M_perp beta||^2 + lambda ||beta||_1
   *   dual_objective D = s b^T r - s^2 ||r||^2 / 2 at theta = s r,
   *                 r = b - M_perp beta, s = min(1, lambda / ||g||_inf)
   *   rel_dual_gap  (P - D) / |P|, with P - D summed termwise as
   *                 (1 - s)^2 ||r||^2 / 2 + sum_i (lambda |beta_i| -
   *                 s beta_i g_i)
   *   natural_residual ||beta - soft(beta + g, lambda)||_inf / max(1,
   *                 ||beta||_inf)  (0 exactly at the LASSO solution)
   *   g_inf         ||g||_inf  (<= lambda at the solution)            */
  double objective;
  double dual_objective;
  double rel_dual_gap;
  double natural_residual;
  double g_inf;
  double setup_seconds;     /* wall time of csipm_create for this context  */
} csipm_info;

/* One record per interior-point iteration (csipm_get_log). */
typedef struct {
  int iter, cg_iters, refine_steps, fell_back;
  int learned;   /* 1 when the learned correction was applied to this system */
  double mu, rel_kkt, alpha;
  double relevant; /* learned form: fraction of coefficients where the
                      correction can matter at this iterate (see
                      pc_max_relevant); -1 in the other forms            */
} csipm_iter_log;

/* Fills `o` with the defaults listed in csipm_options. */
void csipm_default_options(csipm_options* o);

/* Device workspace bytes needed for a grid (all precisions and the learned
 * preconditioner included).  Returns 0 for an unsupported grid. */
size_t csipm_workspace_bytes(int n1, int n2, int n3);

/* Creates a problem (paper: "Matrix-free operators", equation "xi").
 *   d_signal    : n doubles, real space; values at missing samples ignored
 *   d_observed  : n bytes, 1 = observed, 0 = missing; at least one observed
 *   d_workspace : csipm_workspace_bytes(...) bytes, 256-byte aligned
 *   hip_stream  : hipStream_t to queue all work on (NULL = default stream)
 * Computes xi = M_perp^T b (zero-filled signal, r2c 3D DFT, real map) and
 * diag(M_perp^T M_perp).  Errors: EINVAL, EUNSUPPORTED, ENOMEM,
 * ENONFINITE (non-finite observed sample), EHIP. */
csipm_status csipm_create(csipm_ctx** out, int n1, int n2, int n3, const double* d_signal,
                          const uint8_t* d_observed, void* d_workspace, size_t workspace_bytes,
                          void* hip_stream);

/* Sets the penalty lambda > 0 (EINVAL otherwise). */
csipm_status csipm_set_lambda(csipm_ctx* ctx, double lambda);
/* Sets lambda = frac * ||M_perp^T b||_inf and returns it (frac > 0). */
csipm_status csipm_lambda_rule(csipm_ctx* ctx, double frac, double* lambda_out);

/* Runs the primal-dual interior-point method (paper: section "Primal-dual
 * interior-point method", the KKT system of equation "kkt", Newton steps on
 * equation "kktmu" condensed to equation "condensedkkt" and solved by a
 * Krylov method with the preconditioner of equation "precond1") from the
 * standard starting point (beta = 0, z = ||xi||_inf, nu1 = nu2 =
 * lambda/2) until rel_kkt <= opts->tol.  The iterate stays in the
 * context's workspace (csipm_get_iterate).  `info` may be NULL; it also
 * receives the LASSO certificate of the returned beta (one more FP64 pass
 * over beta and H beta).  Returns OK, NOT_CONVERGED, STALLED or FELL_BACK,
 * or an error (EINVAL bad options, ESTATE no lambda or no parameters for
 * the learned form, ENONFINITE non-finite iterate, EHIP). */
csipm_status csipm_solve(csipm_ctx* ctx, const csipm_options* opts, csipm_info* info);

/* Solves `count` independent problems concurrently (the "next" item of
 * batches of small problems: one 16^3-64^3 problem leaves most of the GPU
 * idle).  Each context's csipm_solve runs on one of up to `max_threads`
 * host threads (<= 0: min(count, 8)), on the device and stream the context
 * was created with; kernels of different contexts overlap when their
 * streams differ.  The contexts must be distinct.  statuses[i] receives
 * context i's status and infos[i] its info (infos may be NULL).  Returns
 * EINVAL for a bad argument (nothing run), else the first negative status
 * in context order, else OK. */
csipm_status csipm_solve_batch(csipm_ctx* const* ctxs, int count, const csipm_options* opts, csipm_info* infos,
                               int* statuses, int max_threads);

/* Batches of small problems in one launch (the learned correction's
 * training throughput; no context, no host round trip until the batch is
 * done).  `count` problems of one N1 x N2 x N3 grid, each extent in
 * [1, 64] (any length, odd or even; n = N1*N2*N3), are solved by one kernel,
 * one workgroup per problem, each to rel_kkt <= opts->tol with the standard
 * interior-point steps in FP64 and PCG with the paper's preconditioner
 * (section "Primal-dual interior-point method", equations "kkt", "kktmu",
 * "condensedkkt", "invprecond1"; the readings of csipm_solve: starting
 * point, fixed centring sigma, step tau, PCG tolerance min(cg_rtol,
 * 0.1 rel_kkt) with floor cg_atol).  H beta is recomputed at every iterate.
 *   d_signals   [count][n] doubles, d_observed [count][n] bytes (0 missing)
 *   d_lambdas   [count] doubles > 0, or NULL: lambda = lambda_frac *
 *               ||M_perp^T b||_inf per problem (lambda_frac > 0)
 *   d_beta_out  [count][n] doubles, the solutions (external beta layout)
 *   d_info      [count][CSIPM_SMALL_INFO] doubles: status (0 converged,
 *               1 iteration limit, -2 non-finite iterate), interior-point
 *               iterations, PCG iterations, rel_kkt, mu, lambda
 *   d_workspace csipm_small_workspace_bytes(n1, n2, n3, count) bytes,
 *               256-byte aligned, owned by the caller
 * Reads tol, max_iter, cg_max, cg_rtol, cg_atol, sigma, tau of opts (the
 * others are ignored).  A problem's result does not depend on the rest of
 * its batch.  Copies the twiddle tables into the workspace and
 * synchronises hip_stream once before the launch; the solve itself is
 * asynchronous on it.  Errors: EINVAL, EUNSUPPORTED (an extent outside
 * [1, 64]), ENOMEM (workspace too small), EHIP. */
#define CSIPM_SMALL_INFO 6
size_t csipm_small_workspace_bytes(int n1, int n2, int n3, int count);
csipm_status csipm_solve_small_batch(int n1, int n2, int n3, int count, const double* d_signals,
                                     const uint8_t* d_observed, const double* d_lambdas, double lambda_frac,
                                     const csipm_options* opts, double* d_beta_out, double* d_info,
                                     void* d_workspace, size_t workspace_bytes, void* hip_stream);

/* Copies an iterate or a fixed vector to d_dst (n doubles, external beta
 * layout). */
csipm_status csipm_get_iterate(csipm_ctx* ctx, int which, double* d_dst);

/* KKT residual parts of the current iterate (paper, equation "kkt": the
 * rows F_beta = H beta - xi - nu1 + nu2 and F_z = lambda - nu1 - nu2 and
 * the complementarity s_j nu_j, with the slacks s1 = z + beta, s2 = z -
 * beta eliminated) from one FP64 apply of H, and the LASSO certificate of
 * beta (the certificate fields of csipm_info); solve_seconds and the
 * iteration counts are 0.  Synchronises.  Errors: EINVAL, ESTATE (no
 * lambda), EHIP. */
csipm_status csipm_get_residuals(csipm_ctx* ctx, csipm_info* out);

/* Copies up to max_records per-iteration records of the last solve. */
csipm_status csipm_get_log(csipm_ctx* ctx, csipm_iter_log* host_buf, int max_records, int* n_records);

/* Single operator applies, for parity tests and external Krylov drivers.
 * Inputs and outputs are device arrays of n values in the precision given
 * (double for CSIPM_FP64, float for CSIPM_FP32), beta-space ones in the
 * external beta layout.  Outputs may not alias inputs.
 *   apply_A    : x = A beta                     (derivation "map")
 *   apply_At   : beta = A^T x = B DFT(x)          (adjoint of A)
 *   apply_H    : y = M_perp^T M_perp beta = A^T D A beta
 *   apply_K    : [qb; qz] = K [pb; pz], K = [[H + L1, L2], [L2, L1]],
 *                L1 = S1 + S2, L2 = S1 - S2 (equation "condensedkkt"),
 *                with the barrier diagonals of csipm_set_barrier
 *   apply_Pinv : [zb; zz] = P^{-1} [rb; rz], P = [[I + L1, L2], [L2, L1]]
 *                (equation "invprecond1": the paper's preconditioner,
 *                whatever correction or scaling the last solve used) */
csipm_status csipm_apply_A(csipm_ctx* ctx, const void* d_beta, void* d_x, int precision);
csipm_status csipm_apply_At(csipm_ctx* ctx, const void* d_x, void* d_beta, int precision);
csipm_status csipm_apply_H(csipm_ctx* ctx, const void* d_beta, void* d_y, int precision);
csipm_status csipm_apply_K(csipm_ctx* ctx, const void* d_pb, const void* d_pz, void* d_qb, void* d_qz,
                           int precision);
csipm_status csipm_apply_Pinv(csipm_ctx* ctx, const void* d_rb, const void* d_rz, void* d_zb, void* d_zz,
                              int precision);

/* Sets the barrier diagonals Sigma_1, Sigma_2 (n doubles each, > 0, external
 * beta layout) used by apply_K / apply_Pinv (paper, equation "defsigma"). */
csipm_status csipm_set_barrier(csipm_ctx* ctx, const double* d_sigma1, const double* d_sigma2);

/* Learned preconditioner correction (not in the paper): parameters of the
 * 4-32-32-1 network, float32, flat layout W1[32][4], b1[32], W2[32][32],
 * b2[32], w3[32], b3 (1249 values).  Used by csipm_solve when
 * opts.pc = CSIPM_PC_LEARNED. */
csipm_status csipm_set_pc_params(csipm_ctx* ctx, const float* d_params, int n_params);

#define CSIPM_MLP_PARAMS 1249

/* Network kernels (stateless; queued on hip_stream; no allocation):
 *   forward  : c[i] = softplus(MLP(feat[i][0..3])) + 1e-6, i < n_rec
 *   backward : grad += d/dparams sum_i dc[i] c[i]
 *   loss_grad: loss_out[0] = sum_i w_i (L1_i^2 + L2_i^2)(u_i - c_i p_i)^2 /
 *              (L1_i + S12_i)^2 (the i-th block of P^{-1}(K - P_c)p squared,
 *              P the paper's preconditioner) and grad = its parameter gradient
 *              (overwritten), records rec[i] = {u, p, L1, L2, S12, w}
 *              (6 floats each)
 *   adam     : one Adam step (beta1 0.9, beta2 0.999, eps 1e-8; t counted
 *              from 1) on params with moments m, v (1249 floats each)
 * feat is [n_rec][4] float; d_scratch must hold csipm_mlp_scratch_bytes(n_rec)
 * bytes (8-byte aligned); per-record work is reduced in a fixed order, so
 * results are bitwise reproducible. */
size_t csipm_mlp_scratch_bytes(int n_rec);
csipm_status csipm_mlp_forward(const float* d_params, const float* d_feat, float* d_c, int n_rec,
                               void* hip_stream);
csipm_status csipm_mlp_backward(const float* d_params, const float* d_feat, const float* d_dc, float* d_grad,
                                int n_rec, void* d_scratch, size_t scratch_bytes, void* hip_stream);
csipm_status csipm_mlp_loss_grad(const float* d_params, const float* d_feat, const float* d_rec, int n_rec,
                                 double* d_loss_out, float* d_grad, void* d_scratch, size_t scratch_bytes,
                                 void* hip_stream);
csipm_status csipm_mlp_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, int t, float lr,
                            void* hip_stream);
/* One training step of the network on n_rec records: loss_grad at the
 * current parameters (loss to d_loss_out, gradient to d_grad), then adam
 * with step count t on d_params, d_m, d_v; the same kernels as those two
 * calls, queued in that order.  The moments are two arrays (m, v) and the
 * step count is the caller's; d_scratch is as for loss_grad. */
csipm_status csipm_mlp_train_step(float* d_params, float* d_m, float* d_v, int t, float lr, const float* d_feat,
                                  const float* d_rec, int n_rec, double* d_loss_out, float* d_grad, void* d_scratch,
                                  size_t scratch_bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training loops, hosts that forbid allocation):
 * csipm_mlp_loss_grad without the workspace.  The gradient partials live in
 * a fixed device array of the library, sized for CSIPM_MLP_NOALLOC_MAX_REC
 * records (9.8 MiB), that every GPU the library runs on keeps until the
 * process ends; the call itself allocates nothing.  n_rec above the maximum
 * returns ENOMEM and queues nothing.  Calls that overlap on one GPU share
 * the array and race.  The kernels and their reduction order are those of
 * csipm_mlp_loss_grad, so the results are the same bit for bit.
 * Errors: EINVAL, ENOMEM, EHIP; csipm_last_error(NULL) gives the message of
 * the last failed call on the calling thread. */
#define CSIPM_MLP_NOALLOC_MAX_REC 65536
csipm_status csipm_mlp_loss_grad_noalloc(const float* d_params, const float* d_feat, const float* d_rec, int n_rec,
                                         double* d_loss_out, float* d_grad, void* hip_stream);

/* Training-record capture during csipm_solve with the paper's
 * preconditioner.  At every interior-point iteration (up to max_iters), the
 * first Krylov direction p = P^{-1} r_0 of the Newton solve and q = K p are
 * reduced to n_per_iter records at coefficients
 * idx_j = splitmix64(seed + it * n_per_iter + j) mod n, j < n_per_iter:
 * d_feat gets [max_iters][n_per_iter][4] features, d_rec gets
 * [max_iters][n_per_iter][6] records {u = (H p_beta)_i, p_beta_i, L1, L2,
 * 4 S1 S2, w}, with w = (PCG iterations of that Newton system) /
 * sum_j (p_beta_j^2 + p_z_j^2).  enable = 0 turns capture off.
 * enable = 2 captures as the learned correction is used: only at the
 * iterations where the learned form would apply it (the previous Newton
 * system needed at least opts->pc_min_cg PCG iterations, at most
 * opts->pc_max_relevant of the coefficients are relevant, and at least one
 * is), and with idx_j = a[splitmix64(seed + it * n_per_iter + j) mod m],
 * where a lists in increasing order the m coefficients at which
 * L1 / (L1 + 4 S1 S2) >= 1e-3 (where c can act on P_c^{-1}).  Other values
 * of enable return CSIPM_EINVAL.
 * csipm_captured returns how many iterations were captured by the last solve
 * and their PCG counts (cg_counts_host may be NULL). */
csipm_status csipm_capture(csipm_ctx* ctx, int enable, float* d_feat, float* d_rec, int n_per_iter,
                           int max_iters, unsigned long long seed);
csipm_status csipm_captured(csipm_ctx* ctx, int* n_iters, int* cg_counts_host, int max_iters);

/* Features of the current iterate and barrier diagonals, [n][4] float,
 * coefficients in the external beta layout order. */
csipm_status csipm_features(csipm_ctx* ctx, float* d_feat);

/* The correction c the solver would apply at the current iterate
 * (n doubles, external beta layout): the network is evaluated on the
 * iterate's features where L1/(L1 + 4 S1 S2) >= 1e-3 (there c can act on
 * P_c^{-1}), and c = 1 elsewhere.  Needs parameters (ESTATE otherwise). */
csipm_status csipm_pc_correction(csipm_ctx* ctx, double* d_c);

/* Instrumentation: runs `reps` K-applies (apply_K's kernels on the
 * internal vectors, with the current barrier diagonals) and returns in
 * ms_out[0..4] the average duration of each of its five kernels, timed with
 * HIP events on the context's stream around each kernel, in launch order:
 * axis-1 inverse (with the m = 0 plane's mixing), axis-2 inverse, axis-3
 * c2r/mask/r2c, axis-2 forward, axis-1 forward with the m = 0 unmixing and
 * the K epilogue; in ms_out[5] the average time of one K-apply over `reps`
 * more applies replayed from one HIP graph between a single event pair (as
 * a solve launches its PCG iterations; the direct-launch time when the
 * graph cannot be recorded), and in ms_out[6] the same with the applies
 * launched directly.  ms_out holds CSIPM_KAPPLY_PASSES + 2 values.
 * Synchronises.  CSIPM_EUNSUPPORTED for an odd N3 (whose K-apply
 * is the full-spectrum transforms). */
#define CSIPM_KAPPLY_PASSES 5
csipm_status csipm_profile_kapply(csipm_ctx* ctx, int precision, int reps, double* ms_out);

/* Instrumentation: per-kernel timing of everything the context launches.
 * csipm_timing(ctx, 1) clears earlier records and starts recording a HIP
 * event pair around each kernel launch (launchers that also queue a
 * one-workgroup finalize kernel are timed as one record, named "...+fin");
 * csipm_timing(ctx, 0) stops.  csipm_timing_report synchronises the stream
 * and aggregates the records by kernel name: calls, total duration, and the
 * calls (and their duration) that took at least min_us microseconds, which
 * separates real work from the launches of a queued Krylov batch that
 * return at once after convergence.  Up to max_records entries are written
 * to out (host memory); *n_records receives the number of distinct names.
 * At most 1,000,000 launches are recorded; later ones are counted in
 * `dropped` of the first entry.  Recording adds host work per launch and is
 * meant for measurement runs only. */
typedef struct {
  char name[48];
  int calls;
  int working_calls;
  double total_ms;
  double working_ms;
  long long dropped;
} csipm_kernel_time;
csipm_status csipm_timing(csipm_ctx* ctx, int enable);
csipm_status csipm_timing_report(csipm_ctx* ctx, double min_us, csipm_kernel_time* out, int max_records,
                                 int* n_records);

csipm_status csipm_destroy(csipm_ctx* ctx);
const char* csipm_status_string(int status);
/* Message of the last failure on ctx; with ctx NULL, that of the last
 * failed call without a context on this thread (csipm_create,
 * csipm_mlp_loss_grad_noalloc). */
const char* csipm_last_error(const csipm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* CSIPM_H */
