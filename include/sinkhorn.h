/*
 * sinkhorn.h - C ABI of the MI355X (gfx950) library for linear-time Sinkhorn
 * divergences with positive features (Scetbon & Cuturi, "Linear Time
 * Sinkhorn Divergences using Positive Features").
 *
 * The library computes, for two discrete measures mu = sum_i a_i delta_{x_i}
 * and nu = sum_j b_j delta_{y_j} (Sec. 2, Eq. reg-sdiv / reg-ot):
 *   1. positive Gaussian features phi_theta (Lemma 1, Sec. 3.2; Eq. general)
 *      so that K_theta = Phi_x Phi_y^T (Sec. 3.1),
 *   2. the Sinkhorn scalings (u, v) of Algorithm 1 (Sec. 2) applied to the
 *      factored kernel in r(n+m) operations per iteration (Sec. 3.1),
 *   3. the L1 marginal-error stopping test of Algorithm 1,
 *   4. the dual estimate eps (a^T log u + b^T log v) (Eq. dual-estimate) and
 *      the debiased divergence W(mu,nu) - (W(mu,mu) + W(nu,nu)) / 2,
 *   5. gradients with respect to point locations and weights through the
 *      envelope gradient -eps u v^T of Prop. 3.2 and the chain rule of
 *      Sec. 3.3.
 *
 * Conventions for every entry point:
 *   - Pointers named without a _host suffix are DEVICE pointers (memory of
 *     the current HIP device, e.g. from hipMalloc or a torch CUDA tensor).
 *     All device buffers are owned by the caller; the library never
 *     allocates device memory inside these calls and never frees caller
 *     memory.
 *   - Matrices are row-major and contiguous: X is n x d (row i = x_i),
 *     U is r x d (row k = anchor u_k), Phi is n x r (row i = phi(x_i)).
 *   - Floating point arrays are float32 unless named otherwise; results of
 *     the final reductions are float64.
 *   - Calls are asynchronous and stream-ordered on `stream` (a hipStream_t;
 *     NULL means the default stream).  Argument errors are detected on the
 *     host before anything is enqueued and returned synchronously; numerical
 *     outcomes are written to device-resident sk_solve_info records and are
 *     readable after the stream has been synchronised.
 *   - Return value: SK_OK or one of the error codes below.  Nothing is
 *     enqueued when a call returns an error.
 *   - Concurrency: the solver launches persistent kernels whose workgroups
 *     wait on each other.  Launches from this library must not overlap with
 *     each other on different streams of the same device (use one stream);
 *     every wait is bounded, and a wait that exceeds its bound ends the
 *     launch with status SK_ETIMEOUT instead of hanging.
 */
#ifndef PAPER_2006_07057_AMD_SINKHORN_H
#define PAPER_2006_07057_AMD_SINKHORN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* sk_stream_t; /* a hipStream_t */

/* Status codes (returned, or written to sk_solve_info.status). */
enum {
  SK_OK = 0,
  SK_EINVAL = 1,    /* invalid argument (size, pointer, eps, tol, weights) */
  SK_ENOMEM = 2,    /* workspace or state buffer too small */
  SK_ERANGE = 3,    /* a Sinkhorn division met a zero or non-finite value */
  SK_ENOTCONV = 4,  /* max_iter reached before the tolerance */
  SK_EHIP = 5,      /* a HIP runtime call failed */
  SK_ETIMEOUT = 6,  /* a device-side wait exceeded its bound */
  SK_ENOTSUP = 7    /* unsupported shape (see the entry point) */
};

/* Largest number of features per point supported by the solver. */
#define SK_MAX_R 4096

/* Numeric domain of the scaling loop (sk_solve_opts.range).
 *   SK_RANGE_EXTENDED (default): features are stored as log2 values
 *     L = log2(Phi) and every scaling / r-vector entry as a pair
 *     (E, M) meaning M * 2^E (E integer-valued, M a float32 mantissa),
 *     stored as two halves [E(len) | M(len)].  Relative precision is that
 *     of float32 arithmetic; the range covers scalings far beyond float32
 *     (well-separated clouds, small eps).
 *   SK_RANGE_LINEAR: plain float32 features, scalings and r-vectors.
 *     Faster, but fails with SK_ERANGE when the scalings leave the float32
 *     range. */
#define SK_RANGE_EXTENDED 0
#define SK_RANGE_LINEAR 1

/* Options of Algorithm 1 (Sec. 2).
 *   tol        stop after the first iteration whose column marginal error
 *              ||v o K^T u - b||_1 (computed in float64) is below tol;
 *   max_iter   at most this many iterations (one iteration = the v-update
 *              followed by the u-update);
 *   fixed_iter if > 0, exactly this many iterations and no stopping test
 *              (the final error is still measured and reported);
 *   warm_start if nonzero, the u buffer passed to sinkhorn_solve holds the
 *              starting (positive) scaling; otherwise u starts at 1.  Any
 *              positive start is allowed by Sec. 2;
 *   range      numeric domain, see SK_RANGE_EXTENDED / SK_RANGE_LINEAR. */
typedef struct {
  double tol;
  int32_t max_iter;
  int32_t fixed_iter;
  int32_t warm_start;
  int32_t range;      /* SK_RANGE_EXTENDED (0) or SK_RANGE_LINEAR (1) */
} sk_solve_opts;

/* Outcome of one run of Algorithm 1, written by the device.
 *   iters     iterations whose (u, v) are returned;
 *   status    SK_OK, SK_ENOTCONV, SK_ERANGE, SK_ETIMEOUT, or SK_EINVAL for
 *             weights outside the simplex (see sinkhorn_solve);
 *   err       ||v o K^T u - b||_1 of the returned pair (float64);
 *   w_hat     dual estimate eps (a^T log u + b^T log v) of Eq.
 *             (dual-estimate) for the kernel the solver was given, taken
 *             as eps (a^T log u + b^T log v - (u^T K v - sum(a))): the same
 *             value where the last u-update is exact (u^T K v = sum(a)),
 *             stationary in (u, v) like the objective of Eq. (eval-dual),
 *             so the float32 rounding of the scalings enters it at second
 *             order; every sum in float64. */
typedef struct {
  int32_t iters;
  int32_t status;
  double err;
  double w_hat;
} sk_solve_info;

/* ------------------------------------------------------------------ (a1) */
/* Bandwidth of the Gaussian feature map, Lemma 1 (Sec. 3.2):
 *   q = R^2 / (2 eps d W0(R^2 / (eps d))),  W0 = principal Lambert branch,
 * for points in the ball of radius R.  Anchors are then drawn i.i.d. from
 * N(0, sigma^2 I_d) with sigma^2 = q eps / 4.  Host-only; writes *q_host.
 * SK_EINVAL if R <= 0, eps <= 0, d <= 0 or q_host is NULL. */
int sinkhorn_gaussian_q(double R, double eps, int64_t d, double* q_host);

/* Anchors of the Gaussian feature map (Lemma 1): u_k ~ N(0, sigma^2 I_d)
 * i.i.d. with sigma^2 = q eps / 4, written as U = sigma Z from standard
 * normal draws Z supplied by the caller (its own seeded generator), so the
 * randomness stays an input.  Host-only.
 *   Z_host   r x d float64 standard normal draws (row-major, read only);
 *   sigma2   if > 0: the anchor variance itself, and q = 4 sigma2 / eps;
 *            otherwise q is Lemma 1's Lambert bandwidth for points in the
 *            ball of radius R (as sinkhorn_gaussian_q) and sigma2 = q eps / 4;
 *   U_host   r x d float32 output, U = (float)(sqrt(sigma2) Z);
 *   q_host   receives q (pass it to sinkhorn_features / sk_problem.q).
 * SK_EINVAL for null pointers, r < 1, d < 1, eps <= 0, a non-finite
 * sigma2, or (sigma2 <= 0) an invalid R. */
int sinkhorn_gaussian_anchors(const double* Z_host, int64_t r, int64_t d, double eps,
                              double sigma2, double R, float* U_host, double* q_host);

/* ------------------------------------------------------------------ (a2) */
/* Positive Gaussian features, row-scaled.  For each point x_i (row of X)
 * and anchor u_k (row of U) the log-feature of Lemma 1 / Eq. (general) is
 *   E_ik = -log(r)/2 + (d/4) log(2q) - (2/eps)||x_i - u_k||^2
 *          + ||u_k||^2 / (eps q),
 * so phi_theta(x_i)_k = exp(E_ik).  The call writes
 *   logscale[i] = s_i = max_k E_ik                   (n floats)
 *   Phi[i*r+k]  = exp(E_ik - s_i) in (0, 1]          (SK_RANGE_LINEAR)
 *              or (E_ik - s_i) log2(e) <= 0          (SK_RANGE_EXTENDED)
 * i.e. Phi_theta = diag(exp(s)) Phi (Phi = 2^L in the extended range).  The
 * factor exp(s) is absorbed exactly by the Sinkhorn scalings
 * (u = u~ exp(-s)).
 * Arguments: X (n x d), U (r x d) device float32; eps > 0; q > 1/2;
 * 1 <= r <= SK_MAX_R, d >= 1, n >= 1.  Phi and logscale must not overlap X
 * or U.  Errors: SK_EINVAL for bad sizes/pointers/eps/q. */
int sinkhorn_features(const float* X, int64_t n, int64_t d, const float* U,
                      int64_t r, double eps, double q, int32_t range,
                      float* Phi, float* logscale, sk_stream_t stream);

/* Row-scaled features of the perturbed arc-cosine kernel k_s + kappa
 * (Sec. 3.2, "Arc-cosine kernels", and the decomposition lemma of the
 * appendix).  For anchors u_k (rows of U, drawn from N(0, sigma^2 I),
 * sigma > 1) and Theta_s(w) = sqrt(2) max(0, w)^s:
 *   phi_k(x) = r^{-1/2} sigma^{d/2} Theta_s(u_k.x) exp(-||u_k||^2 (1 - 1/sigma^2)/4),
 *   phi_r(x) = sqrt(kappa)            (one constant feature, index r),
 * so the call writes r + 1 columns: Phi (n x (r+1)) = exp(log phi - s_i) in
 * [0, 1] (linear domain; rectified features are exact zeros) and
 * logscale[i] = s_i = max_k log phi_k(x_i).  Use the result with
 * SK_RANGE_LINEAR solves (the kernel is >= kappa > 0, well conditioned);
 * the solver needs (r + 1) % 4 == 0.  max(0, w)^0 is 1 for w > 0, else 0.
 * Errors: SK_EINVAL (sizes, pointers, s outside 0..8, sigma <= 1,
 * kappa <= 0), SK_ENOTSUP (r + 1 > SK_MAX_R). */
int sinkhorn_features_arccos(const float* X, int64_t n, int64_t d, const float* U,
                             int64_t r, int32_t s, double sigma, double kappa,
                             float* Phi, float* logscale, sk_stream_t stream);

/* ------------------------------------------------------------- (a3)(a4) */
/* Workspace bytes needed by sinkhorn_solve for these sizes (host). */
size_t sinkhorn_solve_workspace_size(int64_t n, int64_t m, int64_t r);

/* Algorithm 1 on the factored kernel K = Phix Phiy^T (Sec. 3.1), each
 * iteration v <- b / (Phiy (Phix^T u)), u <- a / (Phix (Phiy^T v)) done as
 * two fused passes that read each feature row once, until the float64 L1
 * column-marginal error drops below opts->tol (or per opts->fixed_iter).
 * Inputs:  Phix (n x r), Phiy (m x r) positive features (log2 features in
 *          the extended range); a (n), b (m) positive weights.
 *          r % 4 == 0, r <= SK_MAX_R.
 * Outputs: u (n), v (m) scalings; w = Phiy^T v (r), z = Phix^T u (r)
 *          (the r-vectors the adjoint needs); *info (device).  In the
 *          extended range every one of them is a pair array [E | M] of
 *          twice the length (2n, 2m, 2r, 2r floats).
 *          u is read as the starting point when opts->warm_start != 0.
 * ws:      device workspace of at least sinkhorn_solve_workspace_size bytes,
 *          used as scratch (contents on entry are ignored).
 * Weights: a and b must be probability vectors with positive entries (a in
 *          the simplex, Sec. 2).  The solver checks them on the device in
 *          float64 before iterating; an entry that is not positive and
 *          finite, or a sum farther than 1e-5 from 1, ends the solve at
 *          once with info->status = SK_EINVAL (iters 0, w_hat NaN).  The
 *          same holds for every entry point that runs Algorithm 1.
 * Errors:  SK_EINVAL (sizes, pointers, tol < 0, max_iter < 1),
 *          SK_ENOMEM (ws too small), SK_ENOTSUP (r % 4 != 0 or r > 4096). */
int sinkhorn_solve(const float* Phix, int64_t n, const float* Phiy, int64_t m,
                   int64_t r, const float* a, const float* b,
                   const sk_solve_opts* opts, float* u, float* v, float* w,
                   float* z, sk_solve_info* info, void* ws, size_t ws_bytes,
                   sk_stream_t stream);

/* Allocation-free variant of sinkhorn_solve, for callers that cannot
 * allocate device memory or pass a workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).
 * Arguments, outputs and results are those of sinkhorn_solve (the same
 * kernels run with the same launch plan, so results are identical); the
 * scratch space comes from a static device array of
 * SK_NOALLOC_SCRATCH_BYTES held by each device the library runs on until
 * the process ends, and the call allocates nothing.  Sizes whose workspace
 * (sinkhorn_solve_workspace_size) exceeds it are rejected with SK_ENOMEM:
 * with n = m, r <= 1024 fits up to about 6.2e6 points per side, r = 2048
 * up to 4.1e6, r = 4096 only up to 3.2e4.  Every call on one device shares that
 * device's array: calls that overlap on one device (two streams, two host
 * threads) race and must not be issued.
 * Errors: as sinkhorn_solve, plus SK_ENOMEM (scratch too small), SK_EHIP
 * (the array's device address could not be obtained), SK_ENOTSUP (device
 * index >= 64). */
#define SK_NOALLOC_SCRATCH_BYTES (64u << 20)
int sinkhorn_solve_noalloc(const float* Phix, int64_t n, const float* Phiy, int64_t m,
                           int64_t r, const float* a, const float* b,
                           const sk_solve_opts* opts, float* u, float* v, float* w,
                           float* z, sk_solve_info* info, sk_stream_t stream);

/* ------------------------------------------------------------------ (a5) */
/* One divergence problem: points, weights and the feature map. */
typedef struct {
  const float* X;  /* n x d */
  const float* Y;  /* m x d */
  const float* a;  /* n, positive, sums to 1 */
  const float* b;  /* m, positive, sums to 1 */
  const float* U;  /* r x d anchors */
  int64_t n, m, d, r;
  double eps;      /* entropic regularisation, > 0 */
  double q;        /* feature bandwidth parameter of Lemma 1, > 1/2 */
} sk_problem;

/* Byte offsets of the pieces of a divergence state buffer (all 256-byte
 * aligned).  The state holds everything the backward pass needs, so the
 * scaling loop never has to be replayed (Sec. 4, "Optimisation"). */
typedef struct {
  size_t phix, phiy;      /* float n x r, m x r   row-scaled features */
  size_t sx, sy;          /* float n, m           row log-scales */
  size_t u[3], v[3];      /* scalings of the (x,y), (x,x), (y,y) solves */
  size_t w[3], z[3];      /* r-vectors: w = Phi_col^T v, z = Phi_row^T u */
                          /* (each sized for the [E | M] pair layout) */
  size_t info;            /* sk_solve_info[3] */
  size_t out;             /* double[4]: W_bar, W_xy, W_xx, W_yy */
  size_t meta;            /* int32[4]: [0] = numeric domain used; [1..3] =
                             gradient evaluations of the three accelerated
                             solves (sinkhorn_divergence_accelerated), else 0 */
  size_t total;           /* total bytes */
} sk_state_layout;

/* Fill *layout for a problem of this size (host). */
int sinkhorn_state_layout(int64_t n, int64_t m, int64_t r,
                          sk_state_layout* layout);

/* Workspace bytes for sinkhorn_divergence / _backward (host). */
size_t sinkhorn_divergence_workspace_size(const sk_problem* p);

/* Debiased Sinkhorn divergence of Eq. (reg-sdiv):
 *   W_bar = W(mu,nu) - (W(mu,mu) + W(nu,nu)) / 2,
 * each term the dual estimate (Eq. dual-estimate) of one run of Algorithm 1
 * on K_theta.  Computes the features of X and Y, runs the three solves in
 * one persistent launch and reduces in float64.
 * out:   device double[4] = {W_bar, W_xy, W_xx, W_yy}.
 * state: device buffer of sinkhorn_state_layout().total bytes; on return it
 *        holds the features, scalings and infos (layout above).
 * ws:    device workspace of sinkhorn_divergence_workspace_size bytes.
 * Errors: SK_EINVAL, SK_ENOMEM, SK_ENOTSUP as for the calls it makes. */
int sinkhorn_divergence(const sk_problem* p, const sk_solve_opts* opts,
                        double* out, void* state, size_t state_bytes,
                        void* ws, size_t ws_bytes, sk_stream_t stream);

/* Debiased divergence on the perturbed arc-cosine features of
 * sinkhorn_features_arccos: the
 * cost is -eps log k_{s,kappa}, K = Phi_x Phi_y^T with r + 1 columns, and
 * W_bar = W(mu,nu) - (W(mu,mu) + W(nu,nu)) / 2 (Eq. reg-sdiv) with each term
 * the dual estimate of one run of Algorithm 1 in the linear domain.
 *   p      problem; p->q is not used, p->r anchors (r + 1 feature columns:
 *          (r + 1) % 4 == 0 and r + 1 <= SK_MAX_R);
 *   opts   opts->range must be SK_RANGE_LINEAR;
 *   out    device double[4] = {W_bar, W_xy, W_xx, W_yy};
 *   state  device buffer of sinkhorn_state_layout(n, m, r + 1).total bytes
 *          (features with r + 1 columns, scalings, infos);
 *   ws     sinkhorn_divergence_arccos_workspace_size(p) bytes.
 * The gradient entry points (which differentiate the Gaussian map) do not
 * apply to this state.  Errors: SK_EINVAL (pointers, sizes, eps, s outside
 * 0..8, sigma <= 1, kappa <= 0, opts), SK_ENOTSUP (column count, range),
 * SK_ENOMEM (state or workspace too small). */
size_t sinkhorn_divergence_arccos_workspace_size(const sk_problem* p);
int sinkhorn_divergence_arccos(const sk_problem* p, int32_t s, double sigma,
                               double kappa, const sk_solve_opts* opts, double* out,
                               void* state, size_t state_bytes, void* ws, size_t ws_bytes,
                               sk_stream_t stream);

/* W_bar = W_xy - (W_xx + W_yy) / 2 (Eq. reg-sdiv) in float64 from the dual
 * estimates of device-resident solve records, for divergences whose three
 * solves were run by sinkhorn_solve_batched (e.g. a serving loop).
 *   infos  device array of 3 * count records, (xy, xx, yy) per problem;
 *   out    device double[4 * count]: {W_bar, W_xy, W_xx, W_yy} per problem.
 * A failed solve's NaN estimate propagates into W_bar.  Stream-ordered.
 * Errors: SK_EINVAL (null pointer, count < 1), SK_EHIP. */
int sinkhorn_divergence_assemble(const sk_solve_info* infos, int32_t count, double* out,
                                 sk_stream_t stream);

/* ------------------------------------------------------------------ (a6) */
/* Workspace bytes for a batch of `count` problems (host). */
size_t sinkhorn_batched_workspace_size(const sk_problem* problems,
                                       int32_t count);

/* `count` independent divergences (the mini-batch objective of Sec. 4 is
 * an average of such terms).  problems: HOST array of count descriptors
 * (their pointers are device pointers).  states: HOST array of count device
 * state buffers, each sized by sinkhorn_state_layout for its problem.
 * out: device double[4*count] (W_bar, W_xy, W_xx, W_yy per problem).
 * Features of every problem are computed in batched launches, then all
 * 3*count solves run in persistent launches that pack problems of uneven
 * size (grouped by feature-count class), each solve on its own group of
 * workgroups.  Results equal those of sinkhorn_divergence on each problem
 * alone.  Errors as sinkhorn_divergence. */
int sinkhorn_divergence_batched(const sk_problem* problems, int32_t count,
                                const sk_solve_opts* opts, double* out,
                                void* const* states, void* ws,
                                size_t ws_bytes, sk_stream_t stream);

/* One run of Algorithm 1 inside sinkhorn_solve_batched, on the factored
 * kernel K = Prow Pcol^T (Sec. 3.1).  All pointers are device pointers:
 *   Prow (n x r), Pcol (m x r)  features in the layout opts->range selects
 *                               (as written by sinkhorn_features);
 *   a (n), b (m)                positive weights (row and column marginals);
 *   srow (n), scol (m)          row log-scales of Prow / Pcol, or NULL: when
 *                               given, w_hat is reported for the unscaled
 *                               features, eps(a^T log u + b^T log v) with
 *                               u = u~ e^(-srow) (the row-scaling identity);
 *   u (n), v (m), w (r), z (r)  scalings and r-vectors, 8 bytes per entry
 *                               (pair layout [E | M] in the extended range,
 *                               first half used in the linear one); u is
 *                               read as the starting scaling when
 *                               opts->warm_start is set; all four are
 *                               written (w = Pcol^T v, z = Prow^T u);
 *   info                        device record written at the end;
 *   eps                         the regularisation, only scales w_hat. */
typedef struct {
  const float* Prow;
  const float* Pcol;
  const float* a;
  const float* b;
  const float* srow;
  const float* scol;
  float* u;
  float* v;
  float* w;
  float* z;
  sk_solve_info* info;
  int64_t n, m, r;
  double eps;
} sk_solve_spec;

/* Workspace bytes for sinkhorn_solve_batched on these specs (host); 0 if a
 * spec is invalid. */
size_t sinkhorn_solve_batched_workspace_size(const sk_solve_spec* specs,
                                             int32_t count);

/* `count` independent runs of Algorithm 1 (specs: HOST array) in persistent
 * launches that pack solves of uneven size, one launch per feature-count
 * class, each solve on its own group of workgroups.  With
 * opts->warm_start, each solve continues from the scaling in its u buffer:
 * running K iterations and then K' more from the returned u gives the
 * iterates of K + K' iterations (up to rounding), which is how a serving
 * loop advances live requests in epochs.  Buffers of different specs must
 * not overlap, except that features, weights and log-scales may be shared.
 * Errors: SK_EINVAL (null pointer, n, m, r < 1, eps <= 0, count < 1, bad
 * opts), SK_ENOTSUP (r > SK_MAX_R or r % 4 != 0), SK_ENOMEM (workspace). */
int sinkhorn_solve_batched(const sk_solve_spec* specs, int32_t count,
                           const sk_solve_opts* opts, void* ws,
                           size_t ws_bytes, sk_stream_t stream);

/* ------------------------------------------------------------------ (a8) */
/* Adjoint of the feature map for the envelope gradient (Prop. 3.2 and the
 * point-location gradient of Sec. 3.3).  For one side of one solve with
 * scaling p (n) and r-vector g (w for the row side, z for the column side):
 *   dX[i] (+)= coef * 4 p_i ( x_i (Phi_i . g) - sum_k Phi_ik g_k u_k )
 * with Phi the row-scaled features of X (so p is the matching scaled
 * scaling).  accumulate != 0 adds to dX, otherwise overwrites it.  range
 * gives the layout of Phi, p and g (as written by sinkhorn_features and
 * sinkhorn_solve with that range).
 * Errors: SK_EINVAL, SK_ENOTSUP (r % 4 != 0). */
int sinkhorn_features_backward(const float* X, int64_t n, int64_t d,
                               const float* U, int64_t r, const float* Phi,
                               const float* p, const float* g, float coef,
                               int32_t accumulate, int32_t range, float* dX,
                               sk_stream_t stream);

/* Gradient of the divergence computed by sinkhorn_divergence (same problem
 * and state) with respect to X, a, Y and b, scaled by *grad_out (a device
 * float, NULL = 1):
 *   dX = G_row(xy) - (G_row(xx) + G_col(xx)) / 2,   G from the call above;
 *   da = eps (log u_xy - (log u_xx + log v_xx) / 2), centred (mean removed:
 *        the dual optimum is unique only up to a constant, App. B);
 * and symmetrically for dY, db.  Any of dX, da, dY, db may be NULL.  The
 * numeric domain is the one recorded in the state by the forward call.
 * ws: sinkhorn_divergence_workspace_size bytes.  Errors: SK_EINVAL. */
int sinkhorn_divergence_backward(const sk_problem* p, const void* state,
                                 const float* grad_out, float* dX, float* da,
                                 float* dY, float* db, void* ws,
                                 size_t ws_bytes, sk_stream_t stream);

/* Gradient of the divergence computed by sinkhorn_divergence (same problem
 * and state) with respect to the anchors U (r x d), q held fixed: from
 * Prop. 3.2 (dW/dK = -eps u v^T) and the Lemma 1 log-feature,
 * d log phi_k(z)/d u_k = (4/eps)(z - u_k) + (2/(eps q)) u_k, one solve gives
 *   dW/du_k = -4 [ sum_i u_i phi_k(x_i) w_k x_i + sum_j v_j phi_k(y_j) z_k y_j ]
 *             + 4 (2 - 1/q) z_k w_k u_k,
 * combined as dW(x,y) - (dW(x,x) + dW(y,y)) / 2 and scaled by *grad_out (a
 * device float, or 1 if NULL).  dU: device r x d floats (overwritten).
 * ws: sinkhorn_divergence_backward_anchors_workspace_size bytes (partial
 * sums: about 2.2e4 r floats for d < 8, and for d >= 8 one r x d float
 * block per slice of the points, at most 64 slices; the reduction is
 * deterministic).  Errors: SK_EINVAL, SK_ENOMEM. */
size_t sinkhorn_divergence_backward_anchors_workspace_size(const sk_problem* p);
int sinkhorn_divergence_backward_anchors(const sk_problem* p, const void* state,
                                         const float* grad_out, float* dU,
                                         void* ws, size_t ws_bytes,
                                         sk_stream_t stream);

/* ------------------------------------------------- accelerated Sinkhorn */
/* Workspace bytes for sinkhorn_solve_accelerated on this spec (host); 0 if
 * the spec is invalid. */
size_t sinkhorn_solve_accelerated_workspace_size(const sk_solve_spec* spec);

/* Accelerated Sinkhorn (the acceleration remark of Sec. 3.1 and the
 * accelerated algorithm of the appendix) on the factored kernel
 * K = Prow Pcol^T: accelerated alternating minimisation of
 *   phi(eta1, eta2) = log <e^eta1, K e^eta2> - <eta1, a> - <eta2, b>
 * (minus the dual of Eq. dual-smooth divided by eps).  Every step tries
 * the Lipschitz estimate L_k / 2 and doubles it until
 * phi(eta') <= phi(lambda) - ||grad phi(lambda)||^2 / (2L); with
 * a = 1/(2L) + sqrt(1/(4L^2) + A/L) and tau = a/(A + a), the momentum point
 * is lambda = tau zeta + (1 - tau) eta, eta' minimises phi exactly over the
 * block of lambda with the larger gradient norm (a Sinkhorn half-step) and
 * an accepted step sets zeta -= a grad phi(lambda), eta = eta', A += a.
 * The iteration runs on the kernel it is given, the row-scaled
 * Prow Pcol^T, from eta = zeta = 0 (the unscaled kernel from
 * eta = -(srow, scol)); one gradient evaluation reads each feature matrix
 * twice.
 *   spec   one solve, fields as for sinkhorn_solve_batched; the features
 *          must be in the linear layout (float32 values, not log2), and
 *          srow / scol (or NULL) are their row log-scales;
 *   opts   range must be SK_RANGE_LINEAR and warm_start 0.  tol: stop at
 *          the first momentum point whose gradient L1 norm (the marginal
 *          error of the normalised plan there) is below tol and return the
 *          block minimiser from it; max_iter: at most that many accepted
 *          steps (SK_ENOTCONV after); fixed_iter > 0: exactly that many
 *          accepted steps, no stopping test;
 *   L0     starting Lipschitz estimate (> 0, finite; the first step tries
 *          L0 / 2; the dual's gradient is 2-Lipschitz, so 1 is natural);
 *   trials device int32 (or NULL): gradient evaluations made (line-search
 *          trials, each one pass over both matrices for the r-vectors and
 *          one for the row sums).
 * Results (device): u (n), v (m) float32 scalings of the returned dual
 * point, balanced by a common factor; w = Pcol^T v, z = Prow^T u; info:
 * iters = accepted steps, status, err = L1 error of both marginals of
 * diag(u) K diag(v), w_hat = eps (a^T log u + b^T log v - log u^T K v) for
 * the unscaled kernel (the dual F at the returned point).  Features are
 * read as float32; per-point state, r-vectors and every sum are float64
 * (w, z and the scalings are returned rounded to float32).  Runs as one
 * persistent launch whose workgroups wait on each other (bounded:
 * SK_ETIMEOUT).
 * ws: device workspace of sinkhorn_solve_accelerated_workspace_size bytes.
 * Errors: SK_EINVAL (null pointer, n, m, r < 1, eps <= 0, tol < 0, bad
 * iteration counts, L0 <= 0), SK_ENOTSUP (extended range, warm start,
 * r % 4 != 0, r > SK_MAX_R), SK_ENOMEM (ws too small), SK_EHIP. */
int sinkhorn_solve_accelerated(const sk_solve_spec* spec, const sk_solve_opts* opts,
                               double L0, int32_t* trials, void* ws,
                               size_t ws_bytes, sk_stream_t stream);

/* Workspace bytes for sinkhorn_divergence_accelerated (host); 0 if the
 * problem is invalid. */
size_t sinkhorn_divergence_accelerated_workspace_size(const sk_problem* p);

/* The debiased divergence of sinkhorn_divergence with each of its three
 * terms solved by accelerated Sinkhorn (sinkhorn_solve_accelerated, one
 * launch per term, same opts and L0) on linear-layout features: opts->range
 * must be SK_RANGE_LINEAR.  Each term is the dual F at the returned point,
 * eps (a^T log u + b^T log v - log u^T K v).  The state is filled as by
 * sinkhorn_divergence (so sinkhorn_divergence_backward and
 * sinkhorn_divergence_backward_anchors apply to it), and meta[1..3] hold
 * the three solves' gradient-evaluation counts.
 * Errors: as sinkhorn_divergence and sinkhorn_solve_accelerated. */
int sinkhorn_divergence_accelerated(const sk_problem* p, const sk_solve_opts* opts,
                                    double L0, double* out, void* state,
                                    size_t state_bytes, void* ws, size_t ws_bytes,
                                    sk_stream_t stream);

/* ------------------------------------------------------------ tuning (a6) */
/* Per-process launch-planning table used by every solve of the feature
 * count class that serves r (classes: 4, 8, 16, ..., 4096).  A solve of
 * shape (n, m, r) runs on g = ceil(max(n, m) r 4 / target) workgroups
 * (capped by the device's co-resident grid), so `target_bytes` is the
 * feature bytes each workgroup streams per half-step: smaller targets mean
 * more workgroups (more bandwidth, costlier barriers, fewer rows summed per
 * lane).  target_bytes = 0 restores the built-in default (256 KiB).
 * Written by the autotuner (host-only, not thread-safe against concurrent
 * launches).  Errors: SK_EINVAL (r outside 1..SK_MAX_R, target < 0). */
int sinkhorn_tune_set(int64_t r, int64_t target_bytes);

/* Current target of the class serving r (the default if none was set), or
 * a negative value for an invalid r. */
int64_t sinkhorn_tune_get(int64_t r);

/* Lane layouts compiled for the solver class that serves r: writes up to
 * `max` entries of four int32 (G lanes per feature row, C float4 chunks per
 * lane with 4 G C the class's largest r, U rows per lane and batch, W waves
 * per SIMD the kernels are compiled for) to out (host memory, may be NULL
 * when max = 0) and returns the number of layouts of the class (variant 0,
 * the default, first), or SK_EINVAL (negative) for r outside 1..SK_MAX_R.
 * The layouts group the same sums differently: results differ by float32
 * rounding only.  Host-only. */
int32_t sinkhorn_solver_layouts(int64_t r, int32_t* out, int32_t max);

/* Select lane layout `variant` (an index into sinkhorn_solver_layouts) for
 * every later solve of the class serving r, in this process; 0 restores
 * the default.  Written by the autotuner (host-only, not thread-safe
 * against concurrent launches).  Errors: SK_EINVAL (r outside 1..SK_MAX_R,
 * or no such variant). */
int sinkhorn_tune_set_layout(int64_t r, int32_t variant);

/* Layout variant in use for the class serving r, or a negative value for an
 * invalid r. */
int32_t sinkhorn_tune_get_layout(int64_t r);

/* ------------------------------------------------------- instrumentation */
/* Launch timing for measurement: with enable != 0, every later launch of
 * the solver (kind 0), feature (kind 1) and adjoint (kind 2) kernels is
 * bracketed by two HIP events recorded on the launch's own stream.  Calling
 * it again clears the records.  Not for use under graph capture.
 * Returns SK_OK. */
int sinkhorn_profile(int32_t enable);

/* Sum (*total_ms), count (*launches) and maximum (*max_ms, may be NULL) of
 * the recorded launch durations of one kind; waits for the recorded events.
 * Errors: SK_EINVAL (NULL outputs), SK_EHIP. */
int sinkhorn_profile_read(int32_t kind, double* total_ms, int64_t* launches,
                          double* max_ms);

/* Human-readable name of a status code (static string). */
const char* sinkhorn_strerror(int status);

/* Library version string (static). */
const char* sinkhorn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_2006_07057_AMD_SINKHORN_H */
