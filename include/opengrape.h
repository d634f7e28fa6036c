/*
 * opengrape.h -- C ABI of the exponential-free open-GRAPE library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, for a batch of B independent control arrays, the
 * performance index and its gradient of open GRAPE without matrix
 * exponentials (Boutin et al., "Resonator reset in circuit QED by optimal
 * control for large open quantum systems", Sec. III):
 *
 *   H_j   = H0 + sum_k u[j,k] H_k                               Sec. II.A, Eq. (1)
 *   drho/dt = -i[H_j, rho] + sum_m gamma_m D[c_m] rho,
 *   D[c] rho = c rho c^dag - {c^dag c, rho}/2                    Sec. II.B, Eqs. (3)-(4)
 *   rho_{j+1} = RK4 integration of slice j (n_sub steps of dt/n_sub)
 *                                                                Sec. III, Eq. (14)
 *   Phi   = Tr(sigma rho_{N_t})                                  Sec. II.B, Eq. (8)
 *   lambda_{N_t} = sigma, lambda_j = RK4 integration of L_j^dag  Sec. II.B, Eq. (11);
 *                                                                Sec. III, Eq. (15)
 *   dPhi/du[j,k] = -i dt Tr(lambda_{j+1} [H_k, rho_{j+1}])       Sec. II.B, Eq. (13)
 *                  (OG_GRAD_GRAPE1), or the exact derivative of the
 *                  RK4-discretised Phi (OG_GRAD_EXACT, the higher-order
 *                  gradient mentioned after Eq. (12)).
 *
 * No d^2 x d^2 superoperator and no matrix exponential is ever formed.
 *
 * Conventions shared by every entry point
 *  - Complex arrays are interleaved (re, im) float64 pairs, row-major, i.e.
 *    the memory layout of numpy / torch complex128.  Control, cost and
 *    gradient arrays are float64.  Internally the library computes in the
 *    precision chosen at og_create (og_prec).
 *  - "host" pointers are read during the call only.  "device" pointers are
 *    HIP device memory owned by the caller; the library never frees them.
 *  - Every call that takes a stream enqueues its GPU work on that
 *    hipStream_t (NULL = the default stream) and returns without waiting,
 *    except where stated.  Argument and launch errors are reported by the
 *    return code; og_last_error() gives a text for the calling thread.
 *  - Call order per evaluation: og_forward -> og_cost -> og_adjoint ->
 *    og_gradient.  og_cost and og_adjoint may be skipped/repeated only as
 *    stated; a call out of order returns OG_ERR_ORDER.
 *  - One context must not be used from two host threads at once.  Contexts
 *    are independent of each other.
 */
#ifndef OPENGRAPE_H
#define OPENGRAPE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct og_ctx og_ctx;

typedef enum {
    OG_OK = 0,
    OG_ERR_ARG = -1,           /* NULL pointer, bad size or option            */
    OG_ERR_SHAPE = -2,         /* size limits exceeded / operator structure   */
    OG_ERR_NOT_HERMITIAN = -3, /* H0, H_k not Hermitian (validate = 1)         */
    OG_ERR_UNSTABLE_DT = -4,   /* dt / n_sub outside the RK4 stability bound  */
    OG_ERR_WORKSPACE = -5,     /* workspace NULL or smaller than required     */
    OG_ERR_ORDER = -6,         /* call out of order                          */
    OG_ERR_NONFINITE = -7,     /* a propagated state became non-finite        */
    OG_ERR_DEVICE = -8         /* HIP runtime error (allocation, launch)      */
} og_status;

typedef enum {
    OG_F64 = 0,                /* float64 states and arithmetic                */
    OG_F32 = 1,                /* float32 arithmetic; states carried as a
                                  float32 hi part plus a compensation term
                                  (two bfloat16 per element); cost, trace
                                  and gradient sums in float64               */
    OG_F32_SPLIT_BF16 = 2,     /* as OG_F32, but the dense-path GEMMs split
                                  every float32 operand into two bfloat16
                                  parts and use three bfloat16 matrix-core
                                  products with float32 accumulation
                                  (~16 significant bits per product)         */
    OG_F32_SPLIT_F16 = 3       /* as OG_F32_SPLIT_BF16 with float16 parts
                                  (~22 bits); operands are scaled by 2^8
                                  internally, so operator and state entries
                                  must stay below 2^7 in magnitude (larger
                                  ones overflow and are reported as
                                  OG_ERR_NONFINITE).  The banded path runs
                                  the split precisions as OG_F32.            */
} og_prec;

typedef enum {
    OG_GRAD_GRAPE1 = 0,        /* first-order gradient, Eq. (13)              */
    OG_GRAD_EXACT = 1          /* exact derivative of the RK4-discretised Phi */
} og_gmode;

typedef enum {
    OG_PATH_AUTO = 0,          /* banded if every operator has few diagonals  */
    OG_PATH_DENSE = 1,         /* dense complex GEMMs on the matrix cores     */
    OG_PATH_BANDED = 2         /* diagonal-storage stencil (HBM-bound)        */
} og_path;

typedef struct {
    int prec;         /* og_prec                                                */
    int gmode;        /* og_gmode                                               */
    int path;         /* og_path                                                */
    int n_sub;        /* RK4 steps per slice, >= 1 (h = dt / n_sub)             */
    int ckpt_stride;  /* slices between stored forward states; 0 = ceil(sqrt(N_t)) */
    int validate;     /* 1: check Hermiticity at create, RK4 stability and
                         non-finite states per evaluation (one stream sync in
                         og_forward and one in og_gradient)                    */
} og_options;

/* Fill *opt with the defaults: OG_F64, OG_GRAD_GRAPE1, OG_PATH_AUTO,
 * n_sub = 1, ckpt_stride = 0, validate = 1. */
void og_default_options(og_options *opt);

/*
 * Create a context for one operator set (Eq. (1), Eq. (4)).
 *   d              Hilbert-space dimension, 1 <= d <= 4096.
 *   K              number of control Hamiltonians, 0 <= K <= 16.
 *   J              number of collapse operators, 0 <= J <= 16.
 *   H0             host, complex128 d x d, Hermitian.
 *   Hk             host, complex128 K x d x d, each Hermitian (NULL if K = 0).
 *   c_ops          host, complex128 J x d x d (NULL if J = 0).
 *   gamma          host, float64 J rates, each >= 0 (NULL if J = 0).
 *   opt            host, options (NULL = defaults).
 * The context owns device copies of the operators in the working precision
 * (dense matrices or diagonal storage, per og_path).  Allocates device
 * memory; synchronous.  Returns OG_ERR_SHAPE if OG_PATH_BANDED is forced
 * and an operator has too many diagonals (more than 16 per operator set).
 */
og_status og_create(og_ctx **out, int d, int K, int J,
                    const void *H0, const void *Hk, const void *c_ops,
                    const double *gamma, const og_options *opt);

/*
 * As og_create, with every operator given in diagonal storage on one shared
 * offset list (the structure of ladder operators of coupled modes, Sec. IV):
 *   n_diag         number of diagonals, 1 <= n_diag <= 2 d - 1.
 *   offsets        host, n_diag distinct ints in (-d, d); diagonal t holds
 *                  the entries (i, i + offsets[t]).
 *   H0_diags       host, complex128 n_diag x d: H0_diags[t][i] = H0[i, i + offsets[t]].
 *   Hk_diags       host, complex128 K x n_diag x d (NULL if K = 0).
 *   c_diags        host, complex128 J x n_diag x d (NULL if J = 0).
 *   gamma, opt     as og_create.
 * Entries whose column i + offsets[t] falls outside [0, d) are ignored.
 * The operators are expanded on the host and the context is created as by
 * og_create (same validation, path choice and errors); repeated offsets
 * return OG_ERR_ARG.
 */
og_status og_create_banded(og_ctx **out, int d, int K, int J, int n_diag, const int *offsets,
                           const void *H0_diags, const void *Hk_diags, const void *c_diags,
                           const double *gamma, const og_options *opt);

/*
 * Adaptive steps (the adaptive Runge-Kutta integration of every slice,
 * Sec. III.A): with rtol > 0 every slice of the forward sweep, of its
 * checkpoint recompute and of the adjoint sweep is integrated by the
 * embedded Dormand-Prince 5(4) pair with step-size control per problem:
 * an attempt of size h' = min(h, time left in the slice) is accepted when
 * sqrt(mean_c (e_c / (atol + rtol max(|y_c|, |y5_c|)))^2) <= 1 over the real
 * and imaginary parts c of all matrix elements (e: difference of the order-5
 * and order-4 solutions, y5: the order-5 solution), and the next proposal is
 * h' min(fmax, max(0.2, 0.9 err^(-1/5))) with fmax = 1 after a rejection, 5
 * otherwise (h' max(0.2, 0.9 err^(-1/5)) after a rejection).  The first
 * slice of a sweep starts with h = dt; the proposal carries over between
 * slices.  n_sub and the fixed-step stability check are then not used.
 * rtol = 0 returns to fixed RK4 steps.  Only OG_GRAD_GRAPE1 contexts
 * (OG_ERR_ARG otherwise); servers refuse requests while it is on.
 * og_workspace_bytes grows by 9 state matrices per problem; query it after
 * this call.  Each attempt ends with one stream synchronization (the host
 * learns whether any problem is still inside the slice).
 */
og_status og_set_adaptive(og_ctx *ctx, double rtol, double atol);

/*
 * Resident final states (device memory for recomputation, the trade-off of
 * the checkpointed backward sweep that stores the forward states rho_j the
 * gradient of Eq. (13) needs): the last n_slices slices of the forward sweep
 * keep their states in the workspace, so that the backward sweep recomputes
 * only the slices before them from checkpoints (every ckpt_stride slices of
 * those, default ceil(sqrt(N_t - n_slices))).  n_slices = 0 (the default)
 * keeps none; values above N_t keep all.  og_workspace_bytes grows by
 * (min(n_slices, N_t) + 1) states per problem (working precision, no
 * compensation term): with the first-order gradient and fused steps in
 * both directions (og_fused_used) each is the packed Hermitian half of
 * rho_j, d (d + 1) / 2 elements, else a full d x d matrix; query it after
 * this call (the packed half can make the workspace with every slice
 * resident smaller than the one with checkpoints).  Results are bitwise
 * those without resident states.  Used with fixed steps, and for
 * OG_GRAD_EXACT only with n_sub = 1 (ignored otherwise).  Servers keep the
 * last min(n_slices, n_t) states of each request the same way (packed
 * halves only: with the first-order gradient and fused steps in both
 * directions, else they refuse requests while it is set).  OG_ERR_ARG for
 * n_slices < 0 or a NULL ctx.
 */
og_status og_set_resident(og_ctx *ctx, int n_slices);

/*
 * Fused Runge-Kutta steps (the Runge-Kutta integration of Sec. III,
 * Eq. (14), evaluated four stages per launch).  When the banded operators
 * have the structure of a multi-level system coupled to an oscillator
 * (Sec. IV): d = nq N, index q N + n, diagonals of the generator at offsets
 * 0, +-1 (no coupling between blocks of N) and +-N, dissipator taps
 * (0, 0), (s, s) and (s N, s N) with one sign s = +-1 and real factors
 * gamma c[i, i + p], nq <= 4 and nq (T + 6) <= 64 for a tile edge T >= 2 --
 * every fixed RK4 step of the forward sweep, its recompute
 * and the first-order adjoint sweep runs as one kernel that keeps a tile of
 * the state with a halo of four in on-chip memory through the four nested
 * stages, instead of four stage kernels that each read and write the whole
 * state.  The results agree to rounding (the stage inputs are not made
 * Hermitian in between).  enable = 1 (the default) uses it where the
 * structure allows; 0 always runs the four stage kernels.  OG_ERR_ORDER
 * while a server has requests in flight; invalidates a preceding og_forward.
 * og_fused_used returns 1 when the context's fixed steps run fused (both
 * directions), else 0.
 */
og_status og_set_fused(og_ctx *ctx, int enable);
int og_fused_used(const og_ctx *ctx);

/*
 * Step counts of the last evaluation, per problem: counts (host, long
 * B x 4) = [accepted forward, rejected forward, accepted adjoint, rejected
 * adjoint] (the checkpoint recompute repeats the forward steps and is not
 * counted).  Synchronous.  OG_ERR_ORDER before og_adjoint or without
 * adaptive steps.
 */
og_status og_adaptive_stats(og_ctx *ctx, long *counts);

/* Free the context and its device memory (synchronizes the device). */
og_status og_destroy(og_ctx *ctx);

/* The path the context runs (OG_PATH_DENSE or OG_PATH_BANDED). */
int og_path_used(const og_ctx *ctx);

/*
 * Device workspace (bytes) that og_forward needs for a batch of B problems
 * of N_t slices: working stage buffers, the stored forward states every
 * ckpt_stride slices, one segment of recomputed states for the backward
 * sweep, the resident final states (og_set_resident) and the float64
 * gradient.  Without resident states memory grows as O(sqrt(N_t) d^2) per
 * problem, not O(N_t d^2).  Returns 0 for invalid arguments.
 */
size_t og_workspace_bytes(const og_ctx *ctx, int B, int n_t);

/*
 * Forward sweep (Eqs. (10), (14)).
 *   B, n_t    batch size (>= 1) and number of slices (>= 1).
 *   dt        slice length (> 0).
 *   u         device, float64 B x n_t x K, row-major (u[b][j][k]).
 *   rho0      device, complex128 B x d x d initial states (Hermitian).
 *   rhoT      device, complex128 B x d x d output rho_{N_t}, or NULL.
 *   ws        device workspace of ws_bytes >= og_workspace_bytes(ctx, B, n_t),
 *             256-byte aligned; it must stay allocated and untouched until
 *             og_gradient returns.  u must stay unchanged until then too.
 * With validate = 1, reads max|u| back to the host (one stream sync) and
 * returns OG_ERR_UNSTABLE_DT if the RK4 step is outside the stability
 * bound of the Gershgorin estimate of the Hamiltonian's spectral span.
 */
og_status og_forward(og_ctx *ctx, int B, int n_t, double dt,
                     const double *u, const void *rho0, void *rhoT,
                     void *ws, size_t ws_bytes, void *stream);

/*
 * Number of successful og_forward calls on ctx so far (0 before the first).
 * og_cost, og_adjoint and og_gradient always work on the last forward sweep;
 * a caller that keeps several evaluations in flight on one context (an
 * autograd graph holding two applications of the same cost) records this
 * value after its og_forward and compares it before og_adjoint: a different
 * value means another forward sweep has replaced its own in the workspace,
 * which must then be run again.
 */
unsigned long long og_generation(const og_ctx *ctx);

/*
 * Performance index (Eq. (8)): phi[b] = Re Tr(sigma rho_{N_t}[b]), summed
 * in float64 in a fixed order.
 *   sigma     device, complex128 d x d, Hermitian, shared by the batch.
 *   phi       device, float64 B.
 * Requires a preceding og_forward.
 */
og_status og_cost(og_ctx *ctx, const void *sigma, double *phi, void *stream);

/*
 * Backward sweep (Eqs. (11), (13), (15)): lambda starts at sigma and is
 * integrated with L_j^dag slice by slice; forward states are recomputed one
 * segment at a time from the stored ones; the per-slice gradient
 * (GRAPE1 or EXACT, og_gmode) is written into the workspace.
 *   sigma     device, complex128 d x d, Hermitian (the same as for og_cost).
 * Requires a preceding og_forward.
 */
og_status og_adjoint(og_ctx *ctx, const void *sigma, void *stream);

/*
 * Copy the gradient dPhi/du to grad (device, float64 B x n_t x K) and, with
 * validate = 1, synchronize the stream and report OG_ERR_NONFINITE if a
 * state became non-finite during forward or adjoint.  Requires og_adjoint.
 */
og_status og_gradient(og_ctx *ctx, double *grad, void *stream);

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: one whole
 * evaluation (og_forward, og_cost, og_adjoint, og_gradient in that order,
 * same arguments and results: phi device float64 B, grad device float64
 * B x n_t x K) whose workspace is a buffer of the library instead of the
 * caller's: a device array of OG_STATIC_WS_BYTES (256 MiB) per GPU, created
 * with the library's code on every GPU it runs on and held until the
 * process ends (its address is resolved at og_create).  Allocates nothing
 * and never synchronizes: no stability check and no read-back of the
 * non-finite flag, whatever the context's validate option (check phi and
 * grad instead).  Returns OG_ERR_WORKSPACE, with nothing enqueued, when
 * og_workspace_bytes(ctx, B, n_t) exceeds OG_STATIC_WS_BYTES, and OG_ERR_ARG
 * with adaptive steps on (they read every attempt back).  Every call on one
 * GPU shares that GPU's buffer, which keeps the last call's contents: calls
 * in stream order are safe, calls that overlap on one GPU (two streams, two
 * host threads) race.  Afterwards the context is in the state of a finished
 * og_gradient (og_cost / og_gradient may be called again; the workspace is
 * the shared buffer, so only until the next og_evaluate_static).
 */
#define OG_STATIC_WS_BYTES (256u << 20)
og_status og_evaluate_static(og_ctx *ctx, int B, int n_t, double dt, const double *u, const void *rho0,
                             const void *sigma, double *phi, double *grad, void *stream);

/*
 * Multi-state index (Eq. (22), Sec. IV.B): with the B problems of the batch
 * being the input states rho_i(0) of one control array (u repeated for every
 * b), Phi = sum_i Tr(sigma rho_i(T)) and its gradient is the sum over the
 * batch.  og_gradient_sum writes (accumulate = 0) or adds (accumulate = 1)
 * sum_b dPhi_b/du to grad (device, float64 n_t x K), summed batch-major in a
 * fixed order; adding lets the states of different operator sets (the
 * qubit-conditioned resonator problems of Sec. IV.B) be combined from several
 * contexts.  Requires og_adjoint; with validate = 1 syncs like og_gradient.
 */
og_status og_gradient_sum(og_ctx *ctx, double *grad, int accumulate, void *stream);

/*
 * Observable penalty (Eqs. (24)-(25), App. B):
 *   Phi = Tr(sigma rho_{N_t}) - beta * sum_{n=0}^{N_t} dt Tr(A rho_n),
 * with A = a^dag a for the photon-number penalty of the paper.  The forward
 * sweep records Tr(A rho_n) after every slice, og_cost subtracts the sum, and
 * the backward sweep runs the combined adjoint lambda_{N_t} = sigma - beta dt A,
 * lambda_n = (propagated lambda_{n+1}) - beta dt A, so that one forward and one
 * backward sweep give the gradient of the penalised index (both gradient
 * modes).  A: host complex128 d x d, Hermitian (validate = 1 checks it).
 * beta = 0 or A = NULL removes the penalty.  Synchronous; set it before
 * og_forward: the call invalidates a preceding og_forward (og_cost,
 * og_adjoint, og_gradient then return OG_ERR_ORDER until the next
 * og_forward).  Not supported by the server.
 */
og_status og_set_penalty(og_ctx *ctx, const void *A, double beta);

/*
 * Gaussian control filter (App. A, Eqs. (A1)-(A4)): N piecewise-constant
 * controls u_k(j) of length dtu map to M subpixel controls of length dts,
 *   s[b][n][k] = sum_j T[n][j] u[b][j][k],
 *   T[n][j] = ( erf(w0 (n dts - j dtu) / 2) - erf(w0 (n dts - (j+1) dtu) / 2) ) / 2
 * (0-based n, j; the subpixel start time as printed), w0 = omega0 the
 * filter's reference bandwidth (omega_B / 0.5887 for a 3 dB bandwidth
 * omega_B).  og_filter_grad applies the chain rule (Eq. (A2)):
 *   g_u[b][j][k] = sum_n T[n][j] g_s[b][n][k],
 * and with fix_ends = 1 returns 0 for the first and last control, which are
 * held fixed (Fig. 1).  Arrays: device float64, row-major; 1 <= K <= 16.
 * Run the propagation on the subpixel grid (og_forward with M slices of
 * dts) between the two calls.
 */
og_status og_filter_apply(int B, int N, int M, int K, double dtu, double dts, double omega0,
                          const double *u, double *s, void *stream);
og_status og_filter_grad(int B, int N, int M, int K, double dtu, double dts, double omega0,
                         int fix_ends, const double *g_s, double *g_u, void *stream);

/*
 * Continuous batching (serving).  A server accepts independent requests
 * (one control array each, any N_t, on the context's operator set) while
 * others are in flight, and advances all of them together: every
 * og_server_step moves each active request by up to max_slices slice
 * operations (forward slices, then per checkpoint segment the recompute and
 * the adjoint slices with their first-order gradient, Eq. (13)), launching
 * one batched kernel per Runge-Kutta stage for all requests at the same
 * kind of operation.  The result of a request is identical to evaluating it
 * alone with og_forward / og_cost / og_adjoint / og_gradient (the kernels
 * and the reduction order are the same).  Banded path only; gradient mode
 * GRAPE1 (the context's gmode is ignored).  One server per context; the
 * server borrows the context, which must outlive it.
 */
typedef struct og_server og_server;

typedef struct {
    int n_t;            /* slices, >= 1                                        */
    double dt;          /* slice length, > 0                                   */
    const double *u;    /* device, float64 n_t x K                             */
    const void *rho0;   /* device, complex128 d x d                            */
    const void *sigma;  /* device, complex128 d x d (Hermitian)                */
    double *phi;        /* device, 1 float64: Phi (written at completion)      */
    double *grad;       /* device, float64 n_t x K: dPhi/du (at completion)    */
    void *ws;           /* device workspace, 256-byte aligned                  */
    size_t ws_bytes;    /* >= og_workspace_bytes(ctx, 1, n_t)                  */
    long tag;           /* caller's identifier, reported at completion         */
} og_request;

/* Create a server for ctx admitting at most max_active requests at a time
 * (1 <= max_active <= 65536).  The HBM budget is the caller's: every request
 * brings its own workspace. */
og_status og_server_create(og_server **out, og_ctx *ctx, int max_active);

/* Admit a request.  Returns OG_ERR_WORKSPACE when max_active requests are
 * in flight (nothing is enqueued), OG_ERR_ARG / OG_ERR_UNSTABLE_DT for bad
 * arguments (with validate = 1 the stability check reads max|u| back, one
 * sync of `stream`).  All pointers must stay valid until the tag is
 * reported by og_server_completed. */
og_status og_server_submit(og_server *s, const og_request *req, void *stream);

/* Enqueue up to max_slices slice operations for every active request on
 * `stream` (asynchronous).  Requests that finish during the call are
 * retired; their tags become available from og_server_completed and their
 * results are valid once the enqueued work has completed on the stream. */
og_status og_server_step(og_server *s, int max_slices, void *stream);

/* Number of requests in flight. */
int og_server_active(const og_server *s);

/* Move up to max_tags tags of retired requests (oldest first) to tags;
 * returns how many. */
int og_server_completed(og_server *s, long *tags, int max_tags);

/* Destroy the server (requests still in flight are dropped). */
og_status og_server_destroy(og_server *s);

/*
 * Kernel timing (tracing aid, off by default).  With every > 0, one launch in
 * `every` of the context's right-hand-side kernel (the banded stencil stage
 * kernel, or on the dense path the first GEMM of each stage) is bracketed by
 * a pair of HIP events on the stream it is launched on; at most 65536
 * launches are sampled.  every = 0 stops sampling.  og_profile_read waits
 * for the sampled events, returns the mean device duration in microseconds
 * and the number of samples, and clears the samples.
 */
og_status og_profile(og_ctx *ctx, int every);
og_status og_profile_read(og_ctx *ctx, double *mean_us, long *count);

/* Static text for a status code. */
const char *og_status_string(og_status s);

/* Detail of the last failing call on this host thread ("" if none). */
const char *og_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* OPENGRAPE_H */
