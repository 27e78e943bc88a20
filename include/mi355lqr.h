/*
 * mi355lqr.h -- C ABI of the MI355X (gfx950) parallel Riccati LQR solver.
 *
 * Problem solved (Laine & Tomlin, "The Parallelization of Riccati Recursion",
 * arXiv:1809.06360, Sec. II, problem (opt:globalwords) with the costs of
 * eq. (costtform) and the dynamics of eq. (dynamicsform)):
 *
 *   minimise  sum_{t<T} [ 1/2 x_t'Q_t x_t + u_t'S_t x_t + 1/2 u_t'R_t u_t
 *                          + q_t'x_t + r_t'u_t ]  +  1/2 x_T'Q_T x_T + q_T'x_T
 *   s.t.      x_{t+1} = A_t x_t + B_t u_t + c_t,   x_0 = x0.
 *
 * (Paper symbols: Q_xx = Q, Q_ux = S, Q_uu = R, q_x1 = q, q_u1 = r, F_x = A,
 * F_u = B, f_1 = c.) The un-halved objective sum x'Qx + u'Ru + 2q'x + 2r'u is
 * twice this one and has the same minimiser. The problem must be strictly
 * convex: R_t positive definite and Q_t - S_t'R_t^{-1}S_t positive
 * semidefinite (the assumption stated after eq. dynamicsform).
 *
 * Outputs are the serial-Riccati feedback policy u_t = K_t x_t + k_t (the sign
 * of eq. controlpolicy), the value function 1/2 x'P_t x + p_t'x (cost-to-go,
 * eq. costtogo without the x_term block), the optimal trajectory (x_t, u_t)
 * and, optionally, the costate lam_t = P_t x_t + p_t (minus the paper's
 * multiplier lambda_t of eq. KKT). The parallel algorithm splits the horizon
 * into J segments (Sec. II-A), solves every segment as an affine function of
 * its unknown end state, solves the small system linking the segments
 * (Sec. II-A, link equation, and its J-segment generalisation) and rebuilds
 * the per-stage results; all results equal the serial recursion's up to
 * rounding (Sec. III-A).
 *
 * Conventions for every entry point:
 *  - Arrays are row-major and time-major. Pointers inside lqr_problem_t and
 *    lqr_grad_t are DEVICE pointers (HBM of the current HIP device); the
 *    structs themselves and the arrays of structs are HOST memory and may be
 *    reused as soon as the call returns.
 *  - Element type is double for LQR_PREC_FP64 and LQR_PREC_MIXED and float for
 *    LQR_PREC_FP32.
 *  - The caller owns every buffer, including the workspace. The library
 *    allocates no device memory, never synchronises the stream, prints
 *    nothing, and lets no C++ exception cross the ABI.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream)
 *    and runs asynchronously. Argument errors are returned synchronously;
 *    numerical failures are written asynchronously to the instance's `info`.
 *  - Calls that share a workspace must be ordered on one stream.
 *  - Workspace regions (see lqr_workspace_layout): lqr_backward's plan, then
 *    lqr_solve_batched's plan, then scratch. The plans of a problem set (the
 *    same batch, n, m, T and segments per instance) sit in disjoint regions, so
 *    one workspace can serve a batched forward call and lqr_backward on the same
 *    problem set, eagerly or as captured graphs replayed in any order. A call
 *    on a different problem set writes over those regions: it invalidates every
 *    graph captured on the workspace, and a later capture there is rejected
 *    until an uncaptured call has uploaded its plan again.
 */
#ifndef MI355LQR_H
#define MI355LQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LQR_SUCCESS = 0,
    LQR_ERR_INVALID_ARG = 1,      /* bad size, NULL required pointer, segments out of range */
    LQR_ERR_NOT_PD = 2,           /* reserved for callers that turn `info` into a status */
    LQR_ERR_SINGULAR_COUPLING = 3,/* reserved, as above */
    LQR_ERR_NONFINITE = 4,        /* reserved, as above */
    LQR_ERR_WORKSPACE = 5,        /* workspace NULL or smaller than lqr_workspace_size */
    LQR_ERR_HIP = 6,              /* a HIP runtime call failed (launch, copy) */
    LQR_ERR_UNSUPPORTED = 7       /* valid problem the library cannot run: n above 128 or m
                                     above 64; an instance with more than 64 states in a
                                     batch of several; LDS footprint above 160 KiB; mode */
} lqr_status_t;

typedef enum {
    LQR_PREC_FP64 = 0,   /* everything in double */
    LQR_PREC_MIXED = 1,  /* double I/O; the bulk products of the segment sweeps
                            (P[B|A|c], B'P[B|A|c], A'PA, B'Gamma, Gamma and Psi updates)
                            in float on matrix cores with float accumulation, their
                            results widened to double; the input Hessian R + B'PB is
                            assembled and Cholesky-factored in double, the gains and
                            the linking solve are double. lqr_backward computes in
                            double. Instances with n <= 16 and m <= 16 run the
                            small-size kernels, which compute everything in double
                            whatever the precision (at that size float products save
                            no time). */
    LQR_PREC_FP32 = 2    /* float inputs and outputs (every array of lqr_problem_t
                            and lqr_grad_t). The call converts them to a double
                            staging area in the workspace, solves as LQR_PREC_MIXED
                            does (float matrix-core products, double factorizations,
                            gains and linking solve) and rounds the results back to
                            float; lqr_backward computes the adjoint in double from the
                            staged arrays. lqr_solve_phase returns LQR_ERR_UNSUPPORTED
                            for this precision. */
} lqr_precision_t;

typedef enum {
    LQR_ALGO_PARALLEL = 0, /* segment sweeps, linking solve, per-segment rebuild (Sec. II-A) */
    LQR_ALGO_SERIAL = 1    /* one plain Riccati recursion over the whole horizon per instance */
} lqr_algo_t;

/* info codes (per instance, device int32, written asynchronously):
 *   0                         success
 *   t + 1  (1 <= info <= T)   the input Hessian R_t + B_t'P B_t (+ terms) of
 *                             stage t is not positive definite (a finite pivot
 *                             of its Cholesky factorization was not positive);
 *                             when several stages fail, the largest such t is
 *                             reported. The instance's outputs are then NaN
 *                             from that stage on.
 *   LQR_INFO_COUPLING + j     the linking system at segment boundary j had a
 *                             zero or non-finite pivot.
 *   LQR_INFO_QUEUE            internal error of the persistent batched launch:
 *                             a task waited about ten seconds for a dependency
 *                             and gave up (outputs invalid).
 *   LQR_INFO_NONFINITE (< 0)  a non-finite value (NaN or infinity, normally from
 *                             non-finite input data) reached a pivot of an input
 *                             Hessian's factorization, a value gradient p_t, a
 *                             state, an input or a costate; the outputs are not
 *                             valid. Reported only when no positive code applies
 *                             (lqr_backward does not report it).               */
#define LQR_INFO_COUPLING 0x40000000
#define LQR_INFO_QUEUE 0x20000000
#define LQR_INFO_NONFINITE (-1)

/* One LQR instance. */
typedef struct {
    int32_t n, m, T;       /* state dim, input dim, horizon; all >= 1 */
    int32_t segments;      /* J, 1 <= J <= T; 0 = let the planner choose */
    const void *A;         /* [T][n][n]   dynamics, state                                 */
    const void *B;         /* [T][n][m]   dynamics, input                                 */
    const void *c;         /* [T][n]      dynamics, offset                                */
    const void *Q;         /* [T+1][n][n] state cost; index T is the terminal cost        */
    const void *q;         /* [T+1][n]    linear state cost; index T terminal             */
    const void *R;         /* [T][m][m]   input cost (symmetric positive definite)        */
    const void *r;         /* [T][m]      linear input cost                               */
    const void *S;         /* [T][m][n]   cross cost u'S x, or NULL for zero             */
    const void *x0;        /* [n]         initial state                                   */
    void *K;               /* [T][m][n]   out: feedback gains                     (required) */
    void *k;               /* [T][m]      out: feedforward terms                  (required) */
    void *P;               /* [T+1][n][n] out: value Hessians       (NULL = not written) */
    void *p;               /* [T+1][n]    out: value gradients      (NULL = not written) */
    void *x;               /* [T+1][n]    out: optimal states                     (required) */
    void *u;               /* [T][m]      out: optimal inputs                     (required) */
    void *lam;             /* [T+1][n]    out: costates P_t x_t + p_t (NULL = not written) */
    void *chol;            /* [T][m][m]   out: lower Cholesky factor of each stage's input
                                          Hessian, zero above the diagonal (NULL = not
                                          written); lqr_backward needs it              */
    int32_t *info;         /* [1] device int32, see the info codes above          (required) */
} lqr_problem_t;

/* Option flags (lqr_options_t.flags). */
#define LQR_FLAG_PHASED 0x1u   /* lqr_solve_batched: run the parallel algorithm as three
                                  launches, one per phase, instead of one persistent
                                  launch (same results; for comparison and timing) */
#define LQR_FLAG_SMOOTHED 0x2u /* lqr_solve, lqr_solve_phase, lqr_solve_noalloc with
                                  LQR_ALGO_PARALLEL, n <= 64: output the paper's smoothed
                                  policies (Sec. III-A) instead of the serial-exact ones.
                                  Segment j < J-2 is re-solved from segment j+1's
                                  cost-to-go at its start with that segment's end fixed at
                                  its link point, 1/2 x'(P0 + Gam Psi^{-1} Gam')x +
                                  (pbar + Gam Psi^{-1}(psi - x_link))'x; segment J-2 from
                                  the exact value. K, k, P, p are the smoothed policies and
                                  values; x and u are still the optimal trajectory. Every
                                  inner segment must reach any link point (Psi invertible;
                                  otherwise info LQR_INFO_COUPLING + j). Rejected with
                                  LQR_ERR_INVALID_ARG under LQR_ALGO_SERIAL and
                                  LQR_ERR_UNSUPPORTED for batched and adjoint calls and
                                  n above 64. */

typedef struct {
    lqr_precision_t precision;
    lqr_algo_t algo;
    uint32_t flags;        /* LQR_FLAG_PHASED, LQR_FLAG_SMOOTHED or 0; other bits are invalid */
} lqr_options_t;

/* Upstream gradients and gradient outputs of lqr_backward (device pointers). */
typedef struct {
    const void *dl_dx;     /* [T+1][n] dloss/dx_t   (required) */
    const void *dl_du;     /* [T][m]   dloss/du_t   (required) */
    void *dA, *dB, *dc;    /* shapes of A, B, c; NULL = not written */
    void *dQ, *dq;         /* shapes of Q, q (symmetric-form gradient for Q) */
    void *dR, *dr;         /* shapes of R, r (symmetric-form gradient for R) */
    void *dS;              /* shape of S ([T][m][n]) */
    void *dx0;             /* [n] */
} lqr_grad_t;

/* Bytes of device workspace that lqr_solve / lqr_solve_batched / lqr_backward
 * need for these problems and options (probs: HOST array of `batch`
 * descriptors; only n, m, T and segments are read). The same size serves all
 * three calls. Writes the size to *bytes (host). */
lqr_status_t lqr_workspace_size(const lqr_problem_t *probs, int32_t batch,
                                const lqr_options_t *opts, size_t *bytes);

/* Solve one instance (prob: HOST pointer to one descriptor). `ws` is a device
 * buffer of at least lqr_workspace_size bytes, 256-byte aligned; its contents
 * need no initialisation and are overwritten. */
lqr_status_t lqr_solve(const lqr_problem_t *prob, const lqr_options_t *opts,
                       void *ws, size_t ws_bytes, void *stream);

/* Run one launch of lqr_solve's sequence: phase 1 (segment sweeps), 2
 * (linking solve) or 3 (rebuild and forward simulation). Calling phases 1, 2,
 * 3 in order on one stream with the same arguments and workspace is exactly
 * lqr_solve; this exists so that callers can time or interleave the phases.
 * With LQR_ALGO_SERIAL, phase 1 is the whole solve and phases 2, 3 do nothing.
 * Returns LQR_ERR_INVALID_ARG for a phase outside 1..3. */
lqr_status_t lqr_solve_phase(const lqr_problem_t *prob, const lqr_options_t *opts, int32_t phase,
                             void *ws, size_t ws_bytes, void *stream);

/* Segment counts the planner picks for these instances (probs: HOST array;
 * only n, m, T and segments are read; instances with segments > 0 keep theirs)
 * and, if est_us is not NULL, the predicted makespan in microseconds of the
 * persistent batched launch (0 for LQR_ALGO_SERIAL). segments: HOST int32
 * array of `batch` entries. The planner picks every J_i of a batch together:
 * it minimises a bound on the batch's makespan on the device's resident
 * workgroups, max(total work / slots, longest instance critical path), under
 * a per-stage cost model of the kernels measured on MI355X, then checks the
 * best few candidates with a list-scheduling simulation (Sec. II-A fixes the
 * split, not how many segments to use; the choice trades the longer segment
 * sweeps of a small J against the serial linking chain of a large one). */
lqr_status_t lqr_plan_segments(const lqr_problem_t *probs, int32_t batch,
                               const lqr_options_t *opts, int32_t *segments, double *est_us);

/* Solve `batch` independent instances of possibly different n, m, T.
 * With LQR_ALGO_PARALLEL (and no LQR_FLAG_PHASED) this is ONE persistent
 * launch (after a small kernel that clears its counters; when every instance
 * has one segment, the same plain one-workgroup-per-instance launch as
 * LQR_ALGO_SERIAL, which that case reduces to): resident
 * workgroups take tasks -- segment sweeps, linking solves, rebuilds -- from a
 * queue in an order fixed by the planner, and per-instance counters in the
 * workspace make each linking solve wait for its instance's sweeps and each
 * rebuild for its linking solve. With LQR_ALGO_SERIAL it is one workgroup per
 * instance running the plain recursion (on the small-size kernel when every
 * instance has n <= 16 and m <= 16, as for one-segment batches; lqr_solve
 * uses the small-size kernels for all three phases of such an instance).
 * The execution plan (segment counts,
 * descriptor and task tables) is built on the host and copied into the
 * workspace; when a call is made while `stream` is being captured into a HIP
 * graph, the plan for exactly these descriptors must already be in this
 * workspace from an earlier, uncaptured call (else LQR_ERR_INVALID_ARG), and
 * the call then only launches kernels (no memset nodes: the counters are
 * cleared by a kernel, so graph replays are valid). */
lqr_status_t lqr_solve_batched(const lqr_problem_t *probs, int32_t batch,
                               const lqr_options_t *opts, void *ws, size_t ws_bytes,
                               void *stream);

/* Gradient of a scalar loss l(x, u) of the solution with respect to the
 * problem data, by implicit differentiation of the KKT system (eq. KKT): the
 * same LQR is re-solved with linear terms -dl/dx, -dl/du, zero offsets and a
 * zero initial state (the KKT matrix is symmetric, so its transpose is
 * itself), reusing the forward gains and factorizations, and the gradients
 * are outer products of the two solutions. probs[i] must hold the forward
 * data and the forward outputs K, P, x, u, lam and chol of the same call
 * sequence; grads[i] the upstream gradients and the outputs. */
lqr_status_t lqr_backward(const lqr_problem_t *probs, int32_t batch,
                          const lqr_grad_t *grads, const lqr_options_t *opts,
                          void *ws, size_t ws_bytes, void *stream);

/* Byte regions of the workspace of these problems (HOST array of `batch`
 * descriptors; only n, m, T and segments are read) under these options:
 * out[0], out[1]  offset and size of the region holding lqr_backward's plan,
 * out[2], out[3]  offset and size of the region holding lqr_solve_batched's plan,
 * out[4]          offset of the scratch region (everything after it may be
 *                 overwritten by any call),
 * out[5]          bytes of lqr_backward's plan, out[6] bytes of
 *                 lqr_solve_batched's plan (each at most its region's size),
 * out[7]          lqr_workspace_size of the same arguments.
 * Host only; `out` is a HOST array of 8 entries. */
lqr_status_t lqr_workspace_layout(const lqr_problem_t *probs, int32_t batch,
                                  const lqr_options_t *opts, size_t *out);

/* Bytes of the scratch array lqr_solve_noalloc uses on each device. */
#define LQR_NOALLOC_SCRATCH_BYTES (32u << 20)

/* lqr_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc. Same
 * problem, options, kernels and results as lqr_solve, but instead of a
 * workspace argument the call uses a scratch array of
 * LQR_NOALLOC_SCRATCH_BYTES that the library holds on each device (placed
 * there when the runtime loads the library's device code; it stays allocated
 * until the process ends). The call itself allocates nothing (no hipMalloc,
 * hipFree or allocating library routine); its first call on a device looks up
 * that device's copy of the array. Returns LQR_ERR_WORKSPACE if the problem
 * needs more scratch than that (it needs at most lqr_workspace_size of the
 * single problem), else as lqr_solve. Nothing in the array needs
 * clearing between calls: every call writes what it reads. All calls on one
 * device share its array, so calls that may overlap on one device (other
 * streams, other host threads) race and must not be issued; ordering them
 * on one stream is enough. */
lqr_status_t lqr_solve_noalloc(const lqr_problem_t *prob, const lqr_options_t *opts, void *stream);

/* Link multipliers of a solved instance (Sec. II-A: the multiplier of each
 * segment's end-point constraint x_{t_{j+1}} = x_term, matched across the link
 * equation; Sec. II-B, eq. mu): mu_j = P_{t_{j+1}} x_{t_{j+1}} + p_{t_{j+1}},
 * j = 0..J-2, the value gradient at the link point t_{j+1} = (j+1) floor(T/J)
 * + min(j+1, T mod J) (the segment split lqr_solve uses). In the paper's sign
 * convention the segment's dynamics multipliers are the negated costates, and
 * mu_j is the costate at the link point itself. prob: HOST descriptor whose
 * outputs P, p and x hold a finished solve of this instance, read on the
 * device (P, p and x must not be NULL); segments: the J of that solve (the
 * descriptor's, or lqr_plan_segments' choice when it was 0), 1 <= J <= T; mu:
 * DEVICE [J-1][n] output in the outputs' precision (FP32 with
 * LQR_PREC_FP32, else FP64); nothing is written for J = 1. One workgroup per
 * link point, stream-ordered after the solve on `stream`. Returns
 * LQR_ERR_INVALID_ARG for NULL pointers, J outside 1..T or n above 128,
 * LQR_ERR_HIP if the launch fails. */
lqr_status_t lqr_link_multipliers(const lqr_problem_t *prob, const lqr_options_t *opts,
                                  int32_t segments, void *mu, void *stream);

/* Static description of a status code. */
const char *lqr_status_string(lqr_status_t status);

#ifdef __cplusplus
}
#endif

#endif /* MI355LQR_H */
