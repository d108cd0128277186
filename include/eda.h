/*
 * eda.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot path
 * of a randomized-preconditioned ensemble of incremental 4D-Var assimilations
 * (Dauzickaite, Gurol, Destouches, Berre, Weaver: "Accelerating an ensemble of
 * variational data assimilations with randomized preconditioning").
 *
 * Problem (incremental 4D-Var with the control-variable transform, the
 * system_with_CVT equation): every ensemble member j = 0..L (0 = control)
 * solves   (I + A_j) dz_j = b_j,   A_j = U_B^T G_j^T R^-1 G_j U_B,
 *          b_j = U_B^T G_j^T R^-1 d_j,
 * where G_j is the Lorenz-96 RK4 tangent-linear model linearised about member
 * j's own background trajectory followed by direct observation, R = sigma_o^2 I
 * and B = U_B U_B.  A here is the paper's low-rank part; the system matrix is
 * I + A.
 *
 * Conventions for every call:
 *  - Matrices are column-major: column c of an n x nb matrix X starts at
 *    X + c * ldx, with ldx >= n.  A contiguous torch tensor of shape [nb, n]
 *    passes as is with ldx = n.
 *  - Pointers named d_* are device pointers on the GPU that is current when the
 *    context is created; h_* are host pointers.  The caller owns every buffer
 *    it passes, including the workspace; the library never allocates device
 *    memory on its own (it allocates small host structures only).
 *  - All work is enqueued on the stream given to eda_setup (a hipStream_t,
 *    passed as void*).  Calls that return values through h_* pointers
 *    synchronise that stream before they return; the others are asynchronous.
 *  - Return value: EDA_OK (0), a negative error code, or a positive warning.
 *    No C++ exception crosses the ABI.  eda_strerror maps a code to static
 *    text.  A context is bound to one stream and is not thread-safe.
 */
#ifndef EDA_H
#define EDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define EDA_OK                  0
#define EDA_ERR_INVALID_ARG    -1  /* a size, pointer, leading dimension or option is invalid */
#define EDA_ERR_WORKSPACE      -2  /* workspace smaller than eda_workspace_bytes reports      */
#define EDA_ERR_HIP            -3  /* a HIP runtime call failed                                */
#define EDA_ERR_NOT_SPD        -4  /* Cholesky of Phi^T A Phi failed even after the shift      */
#define EDA_ERR_ORDER          -5  /* LMP requested before eda_sketch_evd built one            */
#define EDA_ERR_UNSUPPORTED    -6  /* option not supported by the library (sizes, modes)        */
#define EDA_ERR_SYNC           -7  /* a bounded wait between the pieces of a column (or the   */
                                   /* LMP's tiles) gave up, or the device placed workgroups     */
                                   /* unlike the exchange form expects (eda_set_exchange)       */
#define EDA_WARN_NOT_CONVERGED  1  /* eda_pcg_solve: some member hit maxit or broke down      */

/* ---- per-member PCG outcome (h_status of eda_pcg_solve) ---- */
#define EDA_MEMBER_CONVERGED      0
#define EDA_MEMBER_NOT_CONVERGED  1
#define EDA_MEMBER_BREAKDOWN      2  /* p^T (I+A) p <= 0, r^T z <= 0 or a non-finite value */

/* ---- options ---- */
#define EDA_UB_DENSE   0   /* U_B products as dense FP64 MFMA GEMMs (n x n matrix stored)   */
#define EDA_UB_BANDED  1   /* U_B products as a cyclic banded convolution over the taps of  */
                           /* U_B's first row that exceed 2^-60 |r(0)| (for the diffusion B: */
                           /* those of the unbounded line's kernel)                           */

#define EDA_B_GAUSS      0  /* B = sigma_b^2 C, C the cyclic Gaussian correlation (len_b)       */
#define EDA_B_DIFFUSION  1  /* B = sigma_b^2 C_B, C_B the diffusion-based correlation with Daley */
                            /* length-scale len_b and diff_steps implicit diffusion steps        */

#define EDA_HV_ADD_IDENTITY  1u  /* eda_hessvec returns (I + A) X instead of A X           */
#define EDA_HV_MIXED         2u  /* reduced precision (sketch products): FP32 TL/AD runs; the  */
                                 /* dense U_B products on the matrix cores with FP32 operands */
                                 /* and FP32 accumulation                                      */
#define EDA_HV_BF16          4u  /* as EDA_HV_MIXED, the dense U_B products with BF16 operands */

#define EDA_SKETCH_RHS_DIFF  0   /* Phi = Gamma = [b_1 - b_0, ..., b_ell - b_0] (Gamma eq.) */
#define EDA_SKETCH_USER      1   /* Phi = d_phi (e.g. a Gaussian Psi drawn by the caller)   */
#define EDA_SKETCH_B_PSI     2   /* Phi = U_B^T U_B Psi = B Psi, Psi = d_phi                */
#define EDA_SKETCH_UBT_PSI   3   /* Phi = U_B^T Psi, Psi = d_phi                            */

#define EDA_METHOD_NYSTROM   0   /* Algorithm 1 (q-pass Nystrom)                            */
#define EDA_METHOD_REVD      1   /* Rayleigh-Ritz REVD: Q = orth(A Phi), eig(Q^T A Q)        */

#define EDA_THETA_MID   0        /* theta = (lambda_k(I+A) + 1) / 2                          */
#define EDA_THETA_LAMK  1        /* theta = lambda_k(I+A)                                    */
#define EDA_THETA_ONE   2        /* theta = 1                                                */

#define EDA_XCH_OFF   0          /* eda_set_exchange: independent ring pieces (full halos)     */
#define EDA_XCH_ON    1          /* eda_set_exchange: wave pieces with halo exchange whenever  */
                                 /* a launch shape exists for the running columns             */
#define EDA_XCH_OBS   2          /* eda_set_exchange: ring pieces that share the observed      */
                                 /* increments: shorter halos, one wait per iteration         */
                                 /* (default)                                                 */

#define EDA_LMP_P  0             /* apply P_theta                                            */
#define EDA_LMP_U  1             /* apply the symmetric factor U_theta                       */

#define EDA_LMP_FORM_TWO 0       /* eda_set_lmp_form: projection and expansion, two launches    */
                                 /* (default)                                                   */
#define EDA_LMP_FORM_ONE 1       /* eda_set_lmp_form: one launch with tile barriers             */

/* ---- problem description ----
 * Lorenz-96 (numerical-experiments section): 4 <= n <= 4096 cyclic variables
 * (a whole column's ring fits one workgroup's registers), forcing F,
 * RK4 step dt, window of nsteps steps.  Observations (direct, R = sigma_o^2 I)
 * at steps s = obs_dt, 2 obs_dt, ..., <= nsteps (time 0 is not observed) of the
 * variables i = obs_x0 + q obs_dx < n.
 * Background-error covariance B (b_kind), U_B symmetric with B = U_B U_B:
 *  - EDA_B_GAUSS: B = sigma_b^2 C, C the cyclic Gaussian correlation
 *    exp(-d^2 / (2 len_b^2)); U_B is its symmetric root in closed form, the
 *    cyclic Gaussian r(d) = sigma_b (2/pi)^(1/4) len_b^(-1/2) exp(-d^2/len_b^2)
 *    (U_B U_B = B to 5e-9 relative for len_b >= 2, which is required);
 *  - EDA_B_DIFFUSION: the diffusion-based correlation of the experiments
 *    section (the paper names it, with a Daley length-scale D and a number M of
 *    diffusion steps, without defining it; this is the reading taken):
 *    C_B = g^2 (I - kappa Lap)^-M on the ring, Lap the second difference,
 *    kappa = D^2 / (2M - 3) (the Daley length-scale of the spectrum
 *    (1 + kappa k^2)^-M), g normalising diag(C_B) to one; U_B =
 *    sigma_b g (I - kappa Lap)^(-M/2), built by M/2 implicit diffusion steps
 *    applied to a unit impulse.  len_b = D > 0, diff_steps = M even, 2..64.
 * Truth: spin-up of `spinup` RK4 steps from F * 1 with spin_pert_std * z added
 * to variable 0.  members = L perturbed members (identical-twin set-up of the
 * experiments).  max_cols bounds the number of columns of one eda_hessvec call
 * and of one eda_pcg_solve call (0 selects max(L + 1, 2 * max_ell)); max_ell
 * bounds the sketch width (<= 128). */
typedef struct {
    int32_t n;
    int32_t nsteps;
    double  F;
    double  dt;
    int32_t spinup;
    double  spin_pert_std;
    int32_t obs_dt, obs_dx, obs_x0;
    double  sigma_o;
    double  sigma_b, len_b;
    int32_t members;
    int32_t max_ell;
    int32_t max_cols;
    int32_t ub_mode;     /* EDA_UB_DENSE or EDA_UB_BANDED  */
    int32_t b_kind;      /* EDA_B_GAUSS or EDA_B_DIFFUSION */
    int32_t diff_steps;  /* M (EDA_B_DIFFUSION only)       */
} eda_config;

typedef struct eda_ctx eda_ctx;

/* Bytes of device workspace a context for `cfg` needs (256-byte aligned
 * sub-buffers).  Errors: EDA_ERR_INVALID_ARG for an invalid configuration. */
int eda_workspace_bytes(const eda_config *cfg, size_t *bytes);

/* Number of standard normals eda_setup consumes: 1 + (L+1)(n+p), p the number
 * of observations. */
int eda_normals_count(const eda_config *cfg, int64_t *count);

/* Build one EDA problem on the device (ensemble-formulation section and the
 * experiment set-up):
 *   truth x^t: spin-up, then the window trajectory;
 *   observations y = H x^t + sigma_o eta_0, member j: y_j = y + sigma_o eta_j;
 *   backgrounds x^b = x^t_0 + U_B xi_0, x^b_j = x^b + U_B xi_j;
 *   member trajectories X_j[s], s = 0..N (the linearisation states of G_j);
 *   innovations d_j = y_j - H(X_j), right-hand sides b_j = U_B^T G_j^T R^-1 d_j;
 *   cost constants c_j = 1/2 d_j^T R^-1 d_j.
 * d_normals: device array of eda_normals_count doubles laid out as
 *   [z][xi_0 .. xi_L (n each)][eta_0 .. eta_L (p each)].
 * d_ws / ws_bytes: caller-owned device workspace of at least
 * eda_workspace_bytes; it must outlive the context.  stream: hipStream_t.
 * Synchronises the stream.  On success *out receives the context. */
int eda_setup(const eda_config *cfg, const double *d_normals, void *d_ws, size_t ws_bytes,
              void *stream, eda_ctx **out);

/* Batched Hessian products (the system_with_CVT equation): column c of
 * Y is A_m x_c, or (I + A_m) x_c with EDA_HV_ADD_IDENTITY, where m =
 * d_col_member[c] (device int32 array of nb entries, 0 <= m <= L) selects the
 * linearisation trajectory.  A_m x = U_B^T G_m^T R^-1 G_m U_B x: a U_B product,
 * a TL run over the window writing the observed increments, an AD run forced
 * by them, and a U_B^T product.  nb <= max_cols; X and Y must not overlap.
 * EDA_HV_MIXED runs the TL/AD in FP32 and, with the dense U_B, the U_B products
 * with FP32 operands (relative error of order 1e-6 against FP64); EDA_HV_BF16
 * takes BF16 operands for the dense U_B products (relative error of order 1e-3).
 * Both are meant for sketch products only; with the banded U_B the U_B products
 * stay FP64.  With the banded U_B, when few columns are given the columns run
 * on pieces (eda_set_split); the results are the same bit for bit.  With
 * EDA_XCH_OBS (eda_set_exchange, the default) those pieces share the observed
 * increments and wait for each other, bounded: a wait that gives up (only
 * when other work holds the device's compute units) leaves NaN in that
 * piece's rows of the column's product (the call does not synchronise, so
 * this is how the failure shows; eda_sketch_evd reports EDA_ERR_SYNC for the
 * waits of its own products). */
int eda_hessvec(eda_ctx *ctx, const int32_t *d_col_member, int32_t nb,
                const double *d_X, int64_t ldx, double *d_Y, int64_t ldy, uint32_t flags);

/* Randomized eigendecomposition of the control member's A (preconditioning
 * with randomized algorithms section) and the spectral LMP built from it.
 * kind: EDA_SKETCH_* (d_phi, ldphi: the n x ell user matrix or Psi; ignored for
 * EDA_SKETCH_RHS_DIFF, which uses the first ell perturbed members' RHS
 * differences, ell <= L).  method EDA_METHOD_NYSTROM runs Algorithm 1 with q
 * passes (sketch Y = A Phi, CholQR2 of Y, W = Phi^T Y, Cholesky W = C^T C with
 * the shift nu = u ||Y||_F on breakdown, u the unit roundoff of the sketch
 * products (2^-52 in FP64, 2^-24 with EDA_HV_MIXED, 2^-8 with EDA_HV_BF16),
 * T = R_Y C^-1, SVD T = U Sigma V^T, S = Q_Y U, D = Sigma^2 - nu, truncation
 * to k).  Its last pass runs unshifted with no host round trip; if one of its
 * Choleskys fails, one workgroup repeats the pass on the device with the shifts
 * (CholQR3 with the trace shift, then nu), the same kernel the batch runs.
 * EDA_METHOD_REVD runs
 * Q = orth(A Phi), T = Q^T A Q, T = V D V^T, S = Q V (q ignored).
 * theta_rule: EDA_THETA_*.  flags: 0, EDA_HV_MIXED or EDA_HV_BF16 for the
 * sketch products (with BF16 operands the Cholesky of an ill-conditioned
 * sketch can fail: EDA_ERR_NOT_SPD).
 * The context keeps S_k, D_k and theta for eda_lmp_apply / eda_pcg_solve.
 * h_eig (k doubles, may be NULL): D_k, descending; h_theta (may be NULL).
 * 1 <= k <= ell <= max_ell, q >= 1.  Synchronises the stream.
 * Errors: EDA_ERR_NOT_SPD if the shifted Cholesky fails too; EDA_ERR_SYNC if
 * a wait between the pieces of its products gave up (eda_hessvec), and then
 * the context holds no LMP. */
int eda_sketch_evd(eda_ctx *ctx, int32_t kind, const double *d_phi, int64_t ldphi,
                   int32_t ell, int32_t k, int32_t q, int32_t method, int32_t theta_rule,
                   uint32_t flags, double *h_eig, double *h_theta);

/* Spectral LMP (the spectral LMP subsection and the lmp equation):
 * which = EDA_LMP_P:  Y = P_theta X = X + S_k (theta (D_k + I)^-1 - I) S_k^T X;
 * which = EDA_LMP_U:  Y = U_theta X = X + S_k (sqrt(theta) (D_k + I)^-1/2 - I) S_k^T X.
 * nb <= max_cols; X and Y must not overlap.  EDA_ERR_ORDER before a sketch. */
int eda_lmp_apply(eda_ctx *ctx, int32_t which, int32_t nb, const double *d_X, int64_t ldx,
                  double *d_Y, int64_t ldy);

/* Allocation-free variant of eda_lmp_apply, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same operation, arguments, kernels and bits as
 * eda_lmp_apply; the row-block partial projections S_b^T X_b, which
 * eda_lmp_apply keeps in the context's workspace, go to a fixed device buffer
 * of EDA_LMP_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs
 * on (one per device, kept until the process ends; no call allocates or frees
 * anything).  The partials of a call need ceil(n / 256) * k * (16 ceil(nb / 16))
 * doubles; larger requests return EDA_ERR_UNSUPPORTED before anything is
 * enqueued.  Every call on one GPU shares that GPU's buffer: calls that overlap
 * in time on one GPU (other streams, other threads, other contexts) race and
 * must be serialised by the caller.  Each call writes every partial it reads
 * before reading it, so nothing needs to start at zero.  EDA_ERR_ORDER before a
 * sketch; other errors as eda_lmp_apply. */
#define EDA_LMP_NOALLOC_SCRATCH_BYTES 4194304
int eda_lmp_apply_noalloc(eda_ctx *ctx, int32_t which, int32_t nb, const double *d_X, int64_t ldx,
                          double *d_Y, int64_t ldy);

/* Batched PCG (solving-linear-systems section) for members h_members[0..nm-1]
 * (host array, each in 0..L, nm <= max_cols), from dz = 0, preconditioned by
 * the context's P_theta when use_lmp != 0 (EDA_ERR_ORDER if none was built) or
 * by the identity.  Member c stops when ||r||_2 <= rtol ||b||_2 (recurrence
 * residual) or after maxit iterations (rtol = 0 runs exactly maxit unless a
 * breakdown occurs).  Solutions go to column c of d_DZ (n x nm, ldz).
 * h_iters, h_relres, h_status: nm entries each (required).  h_cost_hist: NULL
 * or nm * (maxit + 1) doubles, row c holding J_i - c_m = -1/2 x_i^T (b + r_i)
 * for i = 0..iters (the quadratic cost of the incremental problem minus its
 * constant), NaN after the last iteration.  Synchronises the stream.
 * Returns EDA_WARN_NOT_CONVERGED if any member did not converge.  With the
 * banded U_B, the pieces of a split iteration wait for each other
 * (eda_set_exchange): they assume that the launch has the device to itself,
 * so a solve whose kernels overlap other work on the device (other streams
 * or contexts) may see a wait give up (EDA_ERR_SYNC); such callers set
 * EDA_XCH_OFF, whose pieces never wait.  Admission (banded U_B with the LMP,
 * automatic pieces, EDA_XCH_OBS): when nm exceeds half the device's compute
 * units (each running column then takes at least two pieces), only that many
 * columns start; the control member's columns wait first, then the last ones,
 * and waiting columns start, in column order with the control's last, as
 * running ones stop.  A column's iteration count and cost history are its
 * own; one that starts at loop iteration s has maxit - s + 1 iterations left,
 * and one that never starts ends EDA_MEMBER_NOT_CONVERGED after 0. */
int eda_pcg_solve(eda_ctx *ctx, const int32_t *h_members, int32_t nm, double rtol, int32_t maxit,
                  int32_t use_lmp, double *d_DZ, int64_t ldz, int32_t *h_iters, double *h_relres,
                  int32_t *h_status, double *h_cost_hist);

/* Read-only views of what eda_setup and eda_sketch_evd stored in the
 * workspace: byte offset into d_ws and element count (doubles).
 *   EDA_FIELD_TRUTH  (N+1) x n truth trajectory, step-major
 *   EDA_FIELD_XB     n x (L+1) backgrounds
 *   EDA_FIELD_TRAJ   (L+1) x (N+1) x n member trajectories
 *   EDA_FIELD_Y      p x (L+1) observations (time-major within a column)
 *   EDA_FIELD_D      p x (L+1) innovations
 *   EDA_FIELD_B      n x (L+1) right-hand sides
 *   EDA_FIELD_COSTC  L+1 cost constants
 *   EDA_FIELD_UBROW  n, first row of U_B
 *   EDA_FIELD_S      n x k eigenvector estimates of the last sketch
 *   EDA_FIELD_EIG    k eigenvalue estimates of the last sketch
 *   EDA_FIELD_SKETCH_INFO  6 int32 (not doubles) of the last Nystrom sketch
 *                    (eda_sketch_evd or a batch solve with LMP): the outcomes
 *                    of its three unshifted Choleskys (Y^T Y, Q1^T Q1, W; 0 or
 *                    the failing pivot + 1; the second is defined only when
 *                    the first is 0), 1 if the device-side pass with the
 *                    shifts ran, 1 if that failed (no LMP), and the shifts it
 *                    took (bit 0: the trace shift of CholQR3, bit 1: the
 *                    Nystrom shift) */
#define EDA_FIELD_TRUTH  0
#define EDA_FIELD_XB     1
#define EDA_FIELD_TRAJ   2
#define EDA_FIELD_Y      3
#define EDA_FIELD_D      4
#define EDA_FIELD_B      5
#define EDA_FIELD_COSTC  6
#define EDA_FIELD_UBROW  7
#define EDA_FIELD_S      8
#define EDA_FIELD_EIG    9
#define EDA_FIELD_SKETCH_INFO 10
int eda_field(const eda_ctx *ctx, int32_t field, size_t *byte_offset, int64_t *count);

/* Opt-in timing of the tangent-linear/adjoint kernel launched by
 * eda_pcg_solve (the fused PCG-iteration kernel with the banded U_B, the TL/AD
 * kernel between the U_B GEMMs with the dense U_B), with HIP events recorded
 * on the context's stream around its launches.  eda_profile(ctx, every)
 * starts (and clears) the accounting, timing every `every`-th launch
 * (every = 1: each launch; a larger period keeps the event records, which sit
 * between kernels on the stream, out of most iterations); eda_profile(ctx, 0)
 * stops it.  eda_profile_read synchronises and returns the number of timed
 * launches, the number of all such launches since eda_profile, and the timed
 * launches' summed duration in milliseconds.  every < 0: EDA_ERR_INVALID_ARG. */
int eda_profile(eda_ctx *ctx, int32_t every);
int eda_profile_read(eda_ctx *ctx, int64_t *timed, int64_t *launches, double *timed_ms);

/* Which launches eda_profile times: EDA_PROF_TLAD (default) the kernels
 * described above; EDA_PROF_UB_GEMM every U_B GEMM of the dense form (the
 * first-level preconditioning product, FP64 MFMA, or FP32 / BF16 operands in
 * reduced-precision sketch products), in any call; EDA_PROF_TLAD_ALL every
 * TL/AD launch in any call (with the dense U_B, the TL/AD core of a Hessian
 * product without its U_B GEMMs).  Takes effect at the next eda_profile.
 * Errors: EDA_ERR_INVALID_ARG for other kinds. */
#define EDA_PROF_TLAD     0
#define EDA_PROF_UB_GEMM  1
#define EDA_PROF_TLAD_ALL 2
int eda_profile_select(eda_ctx *ctx, int32_t kind);

/* ---- learned sketch ----
 * A small MLP maps the control member's right-hand side to k sketch directions
 * (there is no such component in the paper; it learns what its Nystrom finds):
 *   x = b_0 / ||b_0|| sqrt(n),  h1 = gelu(W1 x + b1),  h2 = gelu(W2 h1 + b2),
 *   o = W3 h2 + b3,  Z[:, j] = o[j n : (j + 1) n]  (Z: n x k),
 * gelu(t) = t Phi(t) (erf form).  Training pairs: inputs x and Ritz pairs
 * (S, D) of the control A computed by the q-pass Nystrom algorithm, S
 * orthonormal n x k; loss = ||Z Z^T - S diag(D) S^T||_F^2 / ||D||^2 averaged
 * over the batch.  Parameters: one flat FP32 array, column-major
 * W1 (h x n), b1 (h), W2 (h x h), b2 (h), W3 (k n x h), b3 (k n).
 * Batches are column-major: X n x B (FP32), S n x k x B, D k x B. */
typedef struct {
    int32_t n;       /* state size (input length), 4..4096 */
    int32_t hidden;  /* width of both hidden layers         */
    int32_t k;       /* directions produced, 1..32          */
} eda_mlp_dims;

int eda_mlp_param_count(const eda_mlp_dims *dims, int64_t *count);
/* Device workspace of eda_mlp_forward / eda_mlp_loss_grad for `batch` samples. */
int eda_mlp_workspace_bytes(const eda_mlp_dims *dims, int32_t batch, size_t *bytes);
/* He initialisation: weights = d_normals * sqrt(2 / fan_in), biases 0
 * (d_normals: one standard normal per parameter). */
int eda_mlp_init(const eda_mlp_dims *dims, const float *d_normals, float *d_params, void *stream);
/* FP32 forward pass: d_O (k n x batch) = outputs o of the batch d_X (n x batch). */
int eda_mlp_forward(const eda_mlp_dims *dims, int32_t batch, const float *d_params, const float *d_X, float *d_O,
                    void *d_ws, size_t ws_bytes, void *stream);
/* FP32 forward pass, loss (mean over the batch, to *h_loss) and, if d_grad is
 * not NULL, the gradient of that mean with respect to every parameter (same
 * layout as the parameters).  Synchronises the stream. */
int eda_mlp_loss_grad(const eda_mlp_dims *dims, int32_t batch, const float *d_params, const float *d_X,
                      const float *d_S, const float *d_D, float *d_grad, void *d_ws, size_t ws_bytes, void *stream,
                      double *h_loss);
/* Adam (Kingma and Ba), step counted from 1: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, theta -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). */
int eda_mlp_adam(int64_t count, float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t step, float lr,
                 float beta1, float beta2, float eps, void *stream);
/* The network input of this problem, x = b_0 / ||b_0|| sqrt(n) in FP32 (n
 * floats at d_x), enqueued on the context's stream. */
int eda_mlp_input(eda_ctx *ctx, float *d_x);
/* BF16 copy of the parameters (round to nearest even) for inference. */
int eda_mlp_to_bf16(int64_t count, const float *d_params, uint16_t *d_params16, void *stream);
/* BF16 inference on this problem's control right-hand side: d_Z (n x k, FP64)
 * = Z; BF16 weights and inputs, FP32 accumulation, FP64 epilogues.  dims->n
 * must equal the problem's n. */
int eda_mlp_infer(eda_ctx *ctx, const eda_mlp_dims *dims, const uint16_t *d_params16, double *d_Z);
/* The learned sketch: Phi = CholQR2(Z) with Z from eda_mlp_infer, then the
 * single-pass Nystrom approximation with that Phi (ell = dims->k), truncation
 * to k and theta, as eda_sketch_evd(EDA_SKETCH_USER, ...).  If that breaks down
 * (a Cholesky fails or an eigenvalue is not finite) the right-hand-side
 * difference sketch of the same size is used instead; *h_used (may be NULL)
 * receives 1 for the learned sketch, 0 for the fallback. */
int eda_sketch_learned(eda_ctx *ctx, const eda_mlp_dims *dims, const uint16_t *d_params16, int32_t k,
                       int32_t theta_rule, double *h_eig, double *h_theta, int32_t *h_used);

/* Launch geometry of this context's TL/AD kernels (eda_hessvec, the sketch
 * products and eda_pcg_solve): waves per workgroup (1, 2, 4 or 8; 0 = the
 * default for n) and time-block length (1 .. the maximum the window allows;
 * 0 = that maximum).  Results do not depend on it (the products are computed
 * point by point in the same order), only speed; the batch autotuner chooses
 * among these.  Errors: EDA_ERR_UNSUPPORTED for a geometry n does not admit. */
int eda_set_geometry(eda_ctx *ctx, int32_t waves, int32_t tb);

/* Pieces per column in the iterations of eda_pcg_solve with the banded U_B and
 * the LMP, and in eda_hessvec calls with the banded U_B.  The Hessian part
 * of such an iteration, or such a product, runs on P pieces of every running
 * column, one workgroup each: a piece integrates its share of the n states
 * plus halos covering the reach of the TL/AD runs over the window and of U_B
 * (w its half-width), so its own outputs are exact: 12 N + 2 w states on each
 * side for independent pieces, 12 N + 2 w in all for pieces that share the
 * observed increments (eda_set_exchange); the pieces' partial sums of
 * p^T (I + A) p are added in piece order.  pieces = 0 (the default): of 1, 2,
 * 3, 4 and 8 with P x (members still running at a recent convergence check,
 * or columns of the product) <= the device's compute units, the P whose ring
 * is shortest (with the admission of eda_pcg_solve); 1 to 8: that P in
 * every iteration and product, every column from the start.  Solutions
 * agree with P = 1 to rounding; Hessian products are bit-identical.  Errors:
 * EDA_ERR_UNSUPPORTED if the context is not banded, or P > 1 pieces fit
 * neither form (rings longer than n, pieces shorter than 8 N + w for the
 * shared form, or windows wider than the kernel supports); a forced P that
 * only the shared form fits makes a call that cannot share (EDA_XCH_OFF, or
 * more pieces than compute units) return EDA_ERR_UNSUPPORTED;
 * EDA_ERR_INVALID_ARG for other values. */
int eda_set_split(eda_ctx *ctx, int32_t pieces);

/* How the pieces of a member column exchange data in the split iterations of
 * eda_pcg_solve (banded U_B with the LMP, n >= 512; the integrations of the
 * tangent linear and adjoint models over the assimilation window, cost model
 * of the Nystrom subsection).  mode:
 *  EDA_XCH_OBS (default): ring pieces (eda_set_split) that share the
 *    column's observed increments R^-1 H dx (also in the Hessian products of
 *    eda_hessvec and the sketches): each piece computes those of its
 *    own states, then waits (bounded) for its two neighbours' before its AD
 *    run, so its rings carry ceil(n / P) + 12 N + 2 w states instead of
 *    ceil(n / P) + 24 N + 4 w (w: the U_B band half-width).  Used when every
 *    piece of the launch is co-resident (pieces x running columns <= compute
 *    units) and every piece has at least 8 N + w states; otherwise the
 *    independent ring pieces run.
 *  EDA_XCH_OFF: independent ring pieces (no waits).
 *  EDA_XCH_ON: wave pieces with halo exchange, pieces = 0 in eda_set_split
 *    only.  Every wave of a launch owns one segment of one running column;
 *    the segments of a column exchange the edges of their TL and AD states
 *    through device memory at every time-block boundary, so a column is
 *    spread over many compute units with no recomputed halo.  The launch
 *    takes one workgroup per compute unit, all co-resident.  On MI355X the
 *    ring pieces are faster at the sizes measured.
 * All waits are bounded.  spin_limit:
 * polls of one wait before it gives up; < 0 restores the default (about a
 * second); 0 makes every wait give up at once (to exercise the error path).
 * The limit also bounds the tile barriers of the single-launch LMP
 * (eda_set_lmp_form).  A wait that gives up stops its member with
 * EDA_MEMBER_BREAKDOWN (pieces) or voids the call's results (LMP) and makes
 * eda_pcg_solve return EDA_ERR_SYNC; so does a workgroup placed on an XCD other
 * than the one the layout assumes.  Solutions agree with the other forms to
 * rounding.  Errors: EDA_ERR_INVALID_ARG for other modes. */
int eda_set_exchange(eda_ctx *ctx, int32_t mode, int64_t spin_limit);

/* Form of the LMP inside eda_pcg_solve (the spectral LMP subsection: z = r +
 * S_k diag(c) S_k^T r for every running member).  EDA_LMP_FORM_TWO (default):
 * a projection launch and an expansion launch.  EDA_LMP_FORM_ONE: one launch,
 * a workgroup per (256-row block, 16-column tile) computes its partial
 * projection, the workgroups of a tile meet at a barrier in device memory
 * (bounded wait, see eda_set_exchange), then each expands its rows -- used
 * when the launch's workgroups fit the compute units at once (one each), else
 * the two-launch form.  Both forms give the same bits; on MI355X the
 * two-launch form is the faster one at the sizes measured (the barrier costs
 * more than the launch boundary it replaces).  eda_lmp_apply always takes the
 * two-launch form.  Errors: EDA_ERR_INVALID_ARG for other forms. */
int eda_set_lmp_form(eda_ctx *ctx, int32_t form);

/* Free the context's host structures (the workspace stays the caller's). */
int eda_destroy(eda_ctx *ctx);

/* ---- batches of independent problems ----
 * Many EDA problems of uneven n, window length and ensemble size solved
 * together: for every problem the RHS-difference sketch (Gamma of the
 * structure-of-the-EDA subsection, ell = min(k_cap, L, max_ell) columns), the
 * single-pass Nystrom approximation (the q-pass Nystrom algorithm with q = 1),
 * the spectral LMP with theta = (lambda_k(I+A) + 1)/2 and LMP-PCG of all members
 * 0..L from dz = 0 (the system_with_CVT equation), i.e. per problem exactly
 * what eda_sketch_evd(RHS_DIFF, ell, ell, 1, NYSTROM, MID) followed by
 * eda_pcg_solve(0..L) computes, up to rounding order.
 * Problems with equal n form a class.  One persistent launch computes the
 * sketch columns of every problem, (problem, column) tasks taken from one
 * list; the workgroup that finishes a problem's last column runs that
 * problem's last Nystrom pass on the device -- unshifted CholQR2 and Cholesky
 * first, and where one of them fails the shifts of eda_sketch_evd (shifted
 * CholQR3, the Nystrom shift), with the same routine and bits as
 * eda_sketch_evd's shifted pass.  A second persistent launch then solves the
 * members of every problem: its workgroups take member columns from work
 * queues (one per XCD, whole problems each) and iterate each to its final
 * status without host round trips.  Both are one captured graph; later calls
 * with the same parameters replay it.  The first call also tunes, per class,
 * the TL/AD geometry (waves per workgroup, time-block length) by timing a
 * sketch launch of the class, and the solve geometry for one common number of
 * waves, which the sketch launch uses too.
 * Every context must use the banded U_B (EDA_UB_BANDED), be set up and not be
 * used concurrently by other calls while the batch exists; a context appears
 * at most once.  The batch reuses each context's workspace for its sketch and
 * PCG state and writes each problem's solutions to that problem's PCG state
 * (read them with eda_batch_result). */
typedef struct eda_batch eda_batch;

/* Device workspace the batch needs for np problems (argument blocks, task
 * lists and queue counters; 256-byte aligned). */
int eda_batch_workspace_bytes(eda_ctx *const *ctxs, int32_t np, size_t *bytes);

/* Create a batch over ctxs[0..np).  d_ws: >= eda_batch_workspace_bytes, owned
 * by the caller, 256-byte aligned.  stream: the caller's stream; work already
 * enqueued on it (the problems' set-up) is ordered before the batch's work, and
 * the batch runs on a stream of its own.  Errors: EDA_ERR_INVALID_ARG (null or
 * repeated context, misaligned workspace), EDA_ERR_UNSUPPORTED (dense U_B),
 * EDA_ERR_WORKSPACE, EDA_ERR_HIP. */
int eda_batch_create(eda_ctx *const *ctxs, int32_t np, void *d_ws, size_t ws_bytes, void *stream,
                     eda_batch **out);

/* Sketch, Nystrom and LMP-PCG of every member of every problem (see above);
 * returns after the work is done.  rtol, maxit: the PCG stopping rule of
 * eda_pcg_solve.  use_lmp = 0 skips the sketch and runs plain CG.  A call
 * makes no host round trip between its sketch and its solve.  A problem whose
 * shifted sketch fails (Phi numerically rank-deficient, e.g. ell close to n)
 * has its members solved by plain CG.  h_fallbacks (optional, 2 entries)
 * receives the number of problems whose last Nystrom pass took a shift and,
 * of those, the number solved without LMP.  Returns
 * EDA_OK, EDA_WARN_NOT_CONVERGED if any member of any problem did not converge
 * (maxit or breakdown), or a negative error. */
int eda_batch_solve(eda_batch *batch, int32_t k_cap, double rtol, int32_t maxit, int32_t use_lmp,
                    int32_t *h_fallbacks);

/* Results of problem p of the last eda_batch_solve: d_DZ (optional, n x
 * (L+1), ldz >= n) receives dz of members 0..L; h_iters, h_relres, h_status
 * (L+1 entries each) as in eda_pcg_solve.  Returns EDA_OK or
 * EDA_WARN_NOT_CONVERGED. */
int eda_batch_result(eda_batch *batch, int32_t p, double *d_DZ, int64_t ldz, int32_t *h_iters, double *h_relres,
                     int32_t *h_status);

/* Tuning outcome of class cls (classes in increasing n), valid after the first
 * eda_batch_solve: h_out[11] = {n, problems, solve waves per workgroup, solve
 * points per lane, solve time-block length (the geometry both persistent
 * launches run the class with), persistent solve grid (the same for every
 * class), member columns, and the class's fastest timed geometry for its
 * sketch columns alone: its launch time in microseconds, waves, points per
 * lane, time-block length}.  Returns the number of classes. */
int eda_batch_tuning(eda_batch *batch, int32_t cls, int32_t *h_out);

/* GPU times of the last eda_batch_solve's graph in milliseconds, from clock
 * stamps taken inside the graph: h_ms[0] the sketch launch (products and
 * Nystrom passes), h_ms[1] the prelude (Gamma of every problem), h_ms[2] the
 * solve launch. */
int eda_batch_timing(eda_batch *batch, double *h_ms);

/* Free the batch's host structures and its graph and stream. */
int eda_batch_destroy(eda_batch *batch);

/* Static description of a status code. */
const char *eda_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* EDA_H */
