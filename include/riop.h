/*
 * riop.h -- C interface of the MI355X (gfx950) library for the SDMM
 * radio-interferometric imaging hot path of Carrillo, McEwen & Wiaux,
 * "PURIFY: a new approach to radio-interferometric imaging" (arXiv:1307.4370).
 *
 * The library solves (Sec. 3.3, eq. delta; Sec. 4.3, eq. cvx2)
 *
 *     min ||W Psi^dagger x||_1  subject to  ||y - Phi x||_2 <= eps,  x >= 0
 *
 * with SDMM (Sec. 4.4, Algorithm 1), and exposes the linear operators it is
 * built from:
 *
 *   Phi         = G F D Z        measurement operator (Sec. 5, eq. opmodel; B = I)
 *   Phi^dagger  = Z^T D F^dagger G^T
 *   Psi^dagger  SARA analysis: Dirac plus Daubechies Db1..Db8 (Sec. 3.3), scaled
 *               by 1/sqrt(q) so that Psi Psi^dagger = I (Parseval, Sec. 4.4)
 *   Psi         SARA synthesis
 *
 * Conventions shared by every call
 *   - Data pointers are device pointers (hipMalloc'd or torch CUDA/HIP tensors)
 *     unless a comment says "host".  The caller owns every data buffer and must
 *     keep it alive until the work queued on `stream` has finished.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.  All
 *     calls only enqueue work on `stream` and return, except where noted.
 *   - Complex numbers are interleaved (re, im) pairs of the plan's real type:
 *     float for RIOP_F32 (8 bytes per complex), double for RIOP_F64 (16 bytes).
 *   - An image x is n x n, row-major: x[p * n + q].  Pixel p sits at offset
 *     p - n/2 from the image centre; u pairs with the row index p, v with q.
 *   - Visibilities are in the caller's order (the order of `uv` at plan
 *     creation) unless an entry point says "plan order".
 *   - (u, v) are continuous coordinates in radians per pixel in [-pi, pi]
 *     (pi * (spatial frequency) / (Nyquist frequency)); the oversampled grid
 *     coordinate is g = u K / (2 pi) with K = 2n.
 *   - Coefficients alpha of Psi^dagger are q planes of n x n (q = number of bits
 *     set in dict_mask), in increasing basis order (Dirac, Db1, ..., Db8); a
 *     wavelet plane holds the L-level periodised 2-D DWT in the Mallat layout
 *     (low-low in the top-left corner).
 *   - A plan is not re-entrant: calls on one plan must not overlap in time
 *     (use one plan per stream).  Plans on different devices are independent;
 *     a plan is bound to the device current at its creation.
 *   - Errors: functions return a riop_status.  On failure nothing has been
 *     enqueued that writes caller buffers, no memory is leaked, and
 *     riop_last_error() returns a message for the calling thread.  Errors
 *     raised by the GPU itself (e.g. a device fault) surface as RIOP_EDEVICE
 *     from the next call that synchronises.
 *   - Non-finite inputs: every call checks the caller data it reads (x, y,
 *     alpha, b, x0, weights, a resumed state) on the device.  A NaN or Inf
 *     sets the plan's sticky non-finite flag.  Calls that synchronise
 *     (riop_sdmm, riop_sdmm_finish, riop_gamma, riop_cg with an output
 *     pointer, riop_plan_sync) then return RIOP_ENONFINITE and clear the flag;
 *     the asynchronous operator calls return RIOP_OK and leave the flag for
 *     the next synchronising call (their outputs are then unspecified).
 *     riop_sdmm checks its inputs before the first iteration.
 *   - Device memory: the environment variable RIOP_DEVICE_MEMORY_LIMIT
 *     (bytes, read at each allocation) caps what the library holds in this
 *     process; an allocation past it fails with RIOP_ENOMEM, as a failed
 *     hipMalloc does (riop_device_bytes reports what is held).
 */
#ifndef RIOP_H
#define RIOP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct riop_plan riop_plan;

typedef enum {
    RIOP_OK = 0,
    RIOP_EINVAL = -1,     /* bad argument value (NULL, out-of-range uv, ...) */
    RIOP_ESHAPE = -2,     /* inconsistent sizes */
    RIOP_ENOMEM = -3,     /* device allocation failed */
    RIOP_EDEVICE = -4,    /* HIP runtime error */
    RIOP_ENOTSUP = -5,    /* valid but unsupported configuration */
    RIOP_ENONFINITE = -6  /* a NaN or Inf reached a norm or the input */
} riop_status;

enum { RIOP_F32 = 1, RIOP_F64 = 2 };

/* Plan description.
 *   n          image side; even, 8 <= n <= 3072, divisible by 2^levels, with
 *              K = 2n = 2^a 3^b (2^a >= 8); the FFT passes take K <= 2048
 *              for powers of two and K <= 6144 with factors of 3
 *              (RIOP_ENOTSUP beyond)
 *   oversample grid oversampling per axis (k of Sec. 5); must be 2
 *   M          number of visibilities, 0 <= M < 2^31
 *   J          Kaiser-Bessel kernel width in grid cells; even, 2 <= J <= 16;
 *              single-precision plans need J >= 6 (narrower kernels miss the
 *              1e-7 bound of the weight polynomials: RIOP_ENOTSUP)
 *   levels     wavelet levels, 1 <= levels
 *   dict_mask  bit 0 Dirac, bit k Daubechies k (k = 1..8); nonzero, < 2^9
 *   prec       RIOP_F32: float storage and arithmetic with double-precision
 *              norms, dot products and CG scalars; RIOP_F64: double throughout
 *   tile       gridding tile side in grid cells (power of two, 8..64, dividing
 *              K = 2n); 0 selects the library's choice
 * The tile changes speed only: results do not depend on it beyond
 * floating-point summation order.
 */
typedef struct {
    int32_t n;
    int32_t oversample;
    int64_t M;
    int32_t J;
    int32_t levels;
    uint32_t dict_mask;
    int32_t prec;
    int32_t tile;
    int32_t reserved[7];  /* must be zero */
} riop_desc;

/* Read-only facts about a plan, filled by riop_plan_info. */
typedef struct {
    int32_t n, K, J, levels, q, prec;
    int64_t M;
    int32_t tile;           /* tile side in grid cells */
    int32_t ntiles;         /* (K / tile)^2 */
    int32_t nunits;         /* gridding work units (tile, visibility chunk) */
    int32_t kernel_degree;  /* degree of the per-tap kernel polynomial */
    double kb_beta;         /* Kaiser-Bessel shape parameter */
    double kernel_fit_err;  /* max |polynomial - kernel| found at plan time */
    int64_t device_bytes;   /* device memory held by the plan */
} riop_info;

/* Create a plan for one coverage.
 *   desc    plan description (host)
 *   uv      device, M x 2 reals of the plan's type: (u_m, v_m) pairs
 *   stream  queue for the set-up kernels; the call synchronises `stream`
 *           before returning (it reads back validation flags and bin sizes)
 *   out     receives the plan (host)
 * Builds G's sparsity pattern on the device (Sec. 5: "G is highly sparse"):
 * every visibility's J x J window, binned by the grid cell of its first tap
 * (cells numbered tile by tile) with a stable radix sort, O(M) work for any
 * coverage.  uv outside [-pi, pi] or non-finite -> RIOP_EINVAL. */
riop_status riop_plan_create(const riop_desc *desc, const void *uv, void *stream,
                             riop_plan **out);

/* Free a plan and everything it owns.  Waits for the work the plan's last
 * uncaptured call enqueued (not for the whole device; replays of graphs the
 * caller captured are the caller's to wait for).  NULL is a no-op. */
riop_status riop_plan_destroy(riop_plan *plan);

/* Synchronise `stream` and report the plan's non-finite flag: RIOP_ENONFINITE
 * (flag cleared) if an input of an earlier call on the plan held a NaN or Inf
 * since the last report, RIOP_OK otherwise. */
riop_status riop_plan_sync(riop_plan *plan, void *stream);

/* Device bytes held by the library's allocations in this process (all plans,
 * batches and workspaces). */
int64_t riop_device_bytes(void);

/* The l2 bound eps of the data constraint for M visibilities with complex
 * Gaussian noise of variance sigma^2 (sigma^2 / 2 per real part), Sec. 6:
 * ||n||^2 / (sigma^2/2) is chi^2 with 2M degrees of freedom, and eps is set
 * two standard deviations above its mean, eps^2 = (2M + 4 sqrt(M)) sigma^2 / 2.
 * Host function; NaN for M < 0 or sigma < 0. */
double riop_noise_bound(int64_t M, double sigma);

riop_status riop_plan_info(const riop_plan *plan, riop_info *info /* host */);

/* Plan-order layout of the visibilities (for tests of the binning).
 *   perm        device int32[M]: perm[i] = caller index of the i-th visibility
 *               in plan order (sorted by tile, then by first window cell
 *               inside the tile, row-major, then by caller index)
 *   cell        device uint32[M]: first window cell of the i-th visibility,
 *               a0 | (b0 << 16) with a0, b0 in [0, K)
 *   tile_start  device int32[ntiles + 1]: plan-order offset of each tile
 * Any pointer may be NULL. */
riop_status riop_plan_layout(const riop_plan *plan, int32_t *perm, uint32_t *cell,
                             int32_t *tile_start, void *stream);

/* y = Phi x  (Sec. 5, eq. opmodel, B = I).
 *   x  device, n*n complex;  y  device, M complex (caller order).  x, y must not alias. */
riop_status riop_phi(riop_plan *plan, const void *x, void *y, void *stream);

/* Precomputed Gram operator G^T G (Sec. 4.5 and Sec. 7: storing G^T G lets
 * the CG x-update skip the M-length vector G F D Z p of every iteration).
 * riop_gram_build computes H = G^T G for the plan's coverage, with the plan's
 * own kernel weights, and stores it banded: one K x K plane of the plan's real
 * type per offset (da, db) of the half set (da = 0, 0 <= db < J, and
 * 0 < da < J, |db| < J; J + (J - 1)(2J - 1) planes, 113 for J = 8), the other
 * half by symmetry.  From then on every application of Phi^dagger Phi inside
 * the plan (riop_apply_q, riop_cg, riop_cg_noalloc, the SDMM x-update) applies
 * H to the oversampled spectrum instead of degridding and gridding; riop_phi
 * and riop_phi_adj are unchanged.  Memory: planes x K^2 x (4 or 8) bytes
 * (1.9 GB at 1024^2, J = 8, FP32), plus the same in doubles while building.
 * It pays off when M is several times K^2; at M ~ K^2 degridding and
 * gridding are faster.  Both synchronise; riop_gram_release frees H and
 * returns the plan to degridding and gridding. */
riop_status riop_gram_build(riop_plan *plan, void *stream);
riop_status riop_gram_release(riop_plan *plan);

/* x = Phi^dagger y, the exact adjoint of riop_phi (up to rounding).
 *   y  device, M complex (caller order);  x  device, n*n complex. */
riop_status riop_phi_adj(riop_plan *plan, const void *y, void *x, void *stream);

/* Plan-order variants of riop_phi / riop_phi_adj: y is indexed by plan order
 * (see riop_plan_layout), which avoids the scatter/gather through perm. */
riop_status riop_phi_sorted(riop_plan *plan, const void *x, void *y, void *stream);
riop_status riop_phi_adj_sorted(riop_plan *plan, const void *y, void *x, void *stream);

/* out = Q x = Phi^dagger Phi x + 2 x, the x-update matrix of Sec. 4.4 for a
 * Parseval Psi.  x, out device n*n complex; must not alias. */
riop_status riop_apply_q(riop_plan *plan, const void *x, void *out, void *stream);

/* alpha = Psi^dagger x (Sec. 3.3).  x device n*n complex; alpha device q*n*n complex. */
riop_status riop_psi_adj(riop_plan *plan, const void *x, void *alpha, void *stream);

/* x = Psi alpha.  alpha device q*n*n complex; x device n*n complex. */
riop_status riop_psi(riop_plan *plan, const void *alpha, void *x, void *stream);

/* Conjugate gradient for Q x = b (Sec. 4.4, step 5 of Algorithm 1), Hestenes-
 * Stiefel with complex inner product <a, b> = sum conj(a) b, at most n_iter
 * iterations.  Scalars alpha, beta and all inner products are double
 * precision on the device.  The iteration stops (the iterate no longer
 * changes) once ||r_k|| <= tol ||r_0||, r_0 = b - Q x_in the initial
 * residual; tol = 0 runs exactly n_iter iterations.  An exactly zero residual
 * always stops.  The launch sequence is the same either way (no host round
 * trip), so the call can be captured in a graph.
 *   b          device n*n complex
 *   x          device n*n complex: initial guess in, solution out
 *   tol        relative residual tolerance, >= 0
 *   rr_out     host, nullable: final <r, r>
 *   iters_out  host, nullable: iterations that changed the iterate
 * With rr_out or iters_out the call synchronises (and reports non-finite
 * inputs). */
riop_status riop_cg(riop_plan *plan, const void *b, void *x, int32_t n_iter, double tol,
                    double *rr_out, int32_t *iters_out, void *stream);

/* riop_cg without device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as riop_cg, but CG's
 * workspace (residual, direction, Q times the direction: 3 n^2 complex, plus
 * about 29 KB of reduction slots) lives in a static 64 MiB device array, one
 * per GPU the library runs on, held until the process ends, instead of the
 * plan's SDMM workspace (which riop_cg allocates on first use).  Plans whose
 * workspace does not fit (image sides above about 1180 in FP64 and 1670 in
 * FP32) get RIOP_ENOTSUP.  The call allocates nothing; it uses
 * only the buffers the plan allocated at creation.  All calls on one GPU
 * share that GPU's array: calls that overlap in time on one GPU (on
 * different streams or host threads) race and give wrong results. */
riop_status riop_cg_noalloc(riop_plan *plan, const void *b, void *x, int32_t n_iter, double tol,
                            double *rr_out, int32_t *iters_out, void *stream);

/* gamma = beta * ||Psi^dagger Phi^dagger y||_inf (Sec. 4.4).  Synchronises.
 *   y  device M complex (caller order);  gamma host.
 * Like the other operator calls, it leaves an SDMM state held by the plan
 * (riop_sdmm_init / riop_sdmm_step) unchanged. */
riop_status riop_gamma(riop_plan *plan, const void *y, double beta, double *gamma,
                       void *stream);

/* SDMM parameters (Algorithm 1 with S = 3, L1 = Psi^dagger, L2 = Phi, L3 = I). */
typedef struct {
    int32_t T;            /* SDMM iterations (upper bound when early_stop) */
    int32_t n_cg;         /* CG iterations per x-update */
    double gamma;         /* penalty; <= 0 selects beta * ||Psi^dagger Phi^dagger y||_inf */
    double beta;          /* used when gamma <= 0 (paper: 1e-3) */
    double xi;            /* halting bound on the relative change of f1 (paper: 1e-3) */
    double tau;           /* halting tolerance on ||y - Phi x||/eps (paper: 0.1) */
    int32_t early_stop;   /* 0: run T iterations; 1: stop when the halting rule holds
                             (checked on the host after every iteration) */
    int32_t resume;       /* 0: start from Algorithm 1 steps 1-3 with x^(0) = x_inout
                             (or 0 if x_inout is NULL); 1: continue from the state in
                             x_inout, z1, z2, z3, rhs and f1_prev */
    double f1_prev;       /* resume only: f1 of the previous iterate */
    const void *weights;  /* nullable device, q*n*n reals: diagonal of W in the
                             coefficient layout; NULL means W = I */
    void *z1;             /* nullable device q*n*n complex: dual variable of L1 (in/out) */
    void *z2;             /* nullable device M complex, caller order: dual of L2 (in/out) */
    void *z3;             /* nullable device n*n complex: dual of L3 (in/out) */
    void *rhs;            /* nullable device n*n complex: sum_i x_i (in/out) */
    double *history;      /* nullable host, 5*T doubles: per iteration f1, zeta, nu,
                             final CG <r, r>, CG iterations used */
    double cg_tol;        /* CG stops once ||r_k|| <= cg_tol ||r_0|| (see riop_cg);
                             0: always n_cg iterations */
} riop_sdmm_params;

typedef struct {
    int32_t iters;        /* iterations run */
    double gamma;         /* penalty used */
    double f1;            /* f1(Psi^dagger x) at the last iterate */
    double zeta;          /* relative change of f1 (+inf while the previous f1 is 0) */
    double nu;            /* ||y - Phi x|| / eps */
    int32_t status_iter;  /* 1-based iteration that decided the outcome: the first
                             iteration whose f1 or nu was not finite (the call
                             returns RIOP_ENONFINITE), else the iteration at which
                             the halting rule held (early_stop), else 0 */
    int32_t cg_iters;     /* CG iterations that changed x in the last iteration */
} riop_sdmm_stats;

/* Run SDMM (Algorithm 1).  Everything runs on `stream` with no host round trip
 * inside an iteration unless early_stop is set; the call synchronises once at
 * the end to fill `stats` and `history`.
 *   y        device M complex (caller order)
 *   eps      l2 bound of the data term (> 0)
 *   x_inout  device n*n complex, nullable unless resume: x^(0) in, x^(T) out
 *            (if NULL the final iterate is not returned)
 *   stats    host, nullable
 * The printed l2-ball projection (eq. prox2) is read as the projection onto the
 * ball of radius eps centred at y (the set B of Sec. 4.3). */
riop_status riop_sdmm(riop_plan *plan, const void *y, double eps,
                      const riop_sdmm_params *params, void *x_inout,
                      riop_sdmm_stats *stats, void *stream);

/* Block SDMM (Sec. 4.5, eqs. blocks, dbp1, dbp2): the visibilities are split
 * into R blocks, each with its own data constraint ||y_i - Phi_i x|| <= eps_i,
 * and Algorithm 1 runs with S = R + 2 terms: L1 = Psi^dagger (l1), L2 = I
 * (positivity), L_{i+2} = Phi_i (the l2 ball of block i).  Q is unchanged,
 * since sum_i Phi_i^dagger Phi_i = Phi^dagger Phi; the blocks' steps 7-9 run
 * together and sum_i Phi_i^dagger (r_i - z_i) is one Phi^dagger of the
 * concatenated values.  This is the one-GPU form of the paper's distributed
 * split (each block's data and duals would live on its own node).
 *   y         device M complex (caller order)
 *   nblocks   R, 1 <= R <= 1024
 *   block_of  device int32[M], caller order: the block of each visibility;
 *             a value outside [0, R) -> RIOP_EINVAL (synchronises to check)
 *   eps       host double[R], each > 0
 *   params    as riop_sdmm (T, n_cg, gamma/beta, cg_tol, weights, early_stop,
 *             history, state outputs z1/z2/z3/rhs); resume must be 0
 *   x_inout   nullable device n*n complex: x^(0) in (NULL: 0), x^(T) out
 *   stats     host, nullable; stats->nu and the history's nu are the largest
 *             ||y_i - Phi_i x|| / eps_i over the blocks
 *   nu_out    host, nullable, R doubles: every block's ratio at the last
 *             iteration
 * The halting rule (early_stop) uses the largest ratio.  Synchronises. */
riop_status riop_sdmm_blocks(riop_plan *plan, const void *y, int32_t nblocks, const int32_t *block_of,
                             const double *eps, const riop_sdmm_params *params, void *x_inout,
                             riop_sdmm_stats *stats, double *nu_out, void *stream);

/* Reweighted l1 (Sec. 3.3: SARA replaces the l0 prior by a sequence of
 * weighted l1 problems of eq. delta whose weights are essentially the
 * inverse of the previous solution's coefficients; RWBP and RWBPDb8 of Sec. 6
 * with a one-basis dictionary).
 *   pass 0       Algorithm 1 with W = I from x^(0) = x_inout
 *   pass k >= 1  Algorithm 1 restarted (duals zero) from the previous solution
 *                with w_j = delta_k / (delta_k + |alpha_j|), alpha = Psi^dagger
 *                x_hat^(k-1), and the penalty gamma of pass 0
 *   delta_1      delta0 if > 0, else the root mean square of |alpha| after
 *                pass 0 (1 if that is 0); delta_{k+1} = max(rho delta_k, delta_min)
 *   stop         after `outer` reweighted passes, or once
 *                ||x_k - x_{k-1}|| <= tol ||x_k|| (tol > 0)
 * The regularised inverse and the delta schedule are this library's reading:
 * the paper defers them to its SARA reference. */
typedef struct {
    int32_t outer;     /* reweighted passes after the unweighted one, >= 0 */
    double delta0;     /* delta of the first reweighting; <= 0: RMS of |alpha| */
    double rho;        /* geometric decrease of delta, 0 < rho <= 1 */
    double delta_min;  /* floor of delta, >= 0 */
    double tol;        /* relative change of x that ends the passes; 0: never */
} riop_reweight_params;

/* Run the reweighted passes (synchronises).
 *   params       T, n_cg, gamma/beta, cg_tol, xi, tau, early_stop of every pass;
 *                weights, resume, state and history pointers must be zero
 *   x_inout      device n*n complex, required: x^(0) in, final solution out
 *   weights_out  nullable device q*n*n reals: the weights of the last pass
 *                (all ones if only pass 0 ran)
 *   stats        host, nullable: the last pass's statistics
 *   passes       host, nullable: SDMM runs made (1 + reweighted passes)
 * Allocates the weights and the previous solution (q n^2 reals, n^2 complex)
 * in the plan on first use. */
riop_status riop_sdmm_reweighted(riop_plan *plan, const void *y, double eps, const riop_sdmm_params *params,
                                 const riop_reweight_params *rw, void *x_inout, void *weights_out,
                                 riop_sdmm_stats *stats, int32_t *passes, void *stream);

/* Weighted TV problems (Sec. 3.3 eq. tvproblem; Sec. 5: weighted TV
 * ||W grad x||_1 with its prox computed by the fast iterative method of Beck
 * and Teboulle; Sec. 6: TV with positivity, TV and RWTV):
 *     min ||W grad x||_1  subject to  ||y - Phi x||_2 <= eps,  x >= 0
 * by Algorithm 1 with S = 3: L1 = I (prox of gamma ||W grad .||_1 by n_inner
 * iterations of fast gradient projection on the dual, started at zero, step
 * 1/(8 gamma)), L2 = Phi, L3 = I; Q = Phi^dagger Phi + 2 I as for SARA.  The
 * gradient is the forward difference, zero across the last row and column;
 * complex images count as real vectors of twice the length (gradient
 * magnitude sqrt(|dx|^2 + |dy|^2)); gamma <= 0 selects beta ||Phi^dagger y||_inf.
 *   params       as riop_sdmm; params->weights (nullable) are n*n reals, one
 *                per pixel's gradient magnitude; z1 (state) is n*n complex
 *   n_inner      dual iterations per prox (>= 0; 0 makes the prox the identity)
 *   rw           NULL: one run with params->weights (TV, or weighted TV).
 *                Non-NULL: the reweighted passes of riop_sdmm_reweighted
 *                (RWTV) with w_ij = delta / (delta + |(grad x)_ij|), delta_1 the
 *                RMS of the gradient magnitudes unless given; x_inout then
 *                required, params->weights and state pointers zero
 *   weights_out  nullable device n*n reals (reweighted runs only): the last
 *                pass's weights
 *   passes       host, nullable: SDMM runs made
 * Synchronises. */
riop_status riop_sdmm_tv(riop_plan *plan, const void *y, double eps, const riop_sdmm_params *params,
                         int32_t n_inner, const riop_reweight_params *rw, void *x_inout, void *weights_out,
                         riop_sdmm_stats *stats, int32_t *passes, void *stream);

/* The same run in three phases, for callers that capture the iterations in a
 * HIP graph or interleave several plans.
 *   riop_sdmm_init    Algorithm 1 steps 1-3 (or a resumed state), the penalty
 *                     gamma and y in plan order; allocates the plan's SDMM
 *                     workspace on first use.  params->T sets how many
 *                     iterations the per-iteration history keeps.  Asynchronous.
 *   riop_sdmm_step    enqueue `iterations` iterations (steps 5-9 and the halting
 *                     quantities).  No allocation, no host synchronisation:
 *                     may be captured in a HIP graph and the graph replayed; the
 *                     iteration counter lives on the device.  A captured graph
 *                     stays valid across later riop_sdmm_init calls as long as
 *                     T does not exceed the largest T the plan has been
 *                     initialised with (the history buffer only grows) and
 *                     n_cg, cg_tol and the weights pointer are unchanged;
 *                     otherwise capture again.
 *   riop_sdmm_finish  copy x (x_out, nullable) and, if params is non-NULL, the
 *                     state (params->z1, z2, z3, rhs) and history out; fills
 *                     stats.  Synchronises `stream`.
 * No early stopping in this form. */
riop_status riop_sdmm_init(riop_plan *plan, const void *y, double eps,
                           const riop_sdmm_params *params, const void *x0, void *stream);
riop_status riop_sdmm_step(riop_plan *plan, int32_t iterations, void *stream);
riop_status riop_sdmm_finish(riop_plan *plan, const riop_sdmm_params *params, void *x_out,
                             riop_sdmm_stats *stats, void *stream);

/* ---------------------------------------------------------------------------
 * Batched SDMM over channels of uneven sizes (many frequency channels or
 * observations solved independently, each its own instance of Algorithm 1).
 *
 * riop_batch_create   one plan per channel: descs[c] and device uv[c] as for
 *                     riop_plan_create.  autotune != 0 picks each channel's
 *                     gridding tile by timing Phi / Phi^dagger pairs for every
 *                     admissible tile (desc.tile is then ignored).  Synchronises.
 * riop_batch_sdmm     run params->T iterations of every channel from x^(0) = 0.
 *                     The iterations are captured once into a HIP graph (one
 *                     branch per channel, default-priority streams owned by the
 *                     batch) holding iters_per_graph iterations, and the graph is
 *                     replayed; a remainder runs without the graph.  y[c] device
 *                     M_c complex (caller order), eps[c] > 0, x_out[c] device
 *                     n_c^2 complex (nullable array or entries), stats array of
 *                     nchannels (nullable).  params: shared T, n_cg, gamma/beta;
 *                     resume, early_stop, weights, state and history pointers
 *                     must be zero.  Synchronises.
 * riop_batch_plan     borrow channel c's plan (owned by the batch).
 * riop_batch_tile     channel c's tile and the measured ms per pair for tiles
 *                     8, 16, 32, 64 (negative where not tried or not tuned).
 * riop_autotune_tile  the tile search alone for one description. */
typedef struct riop_batch riop_batch;
riop_status riop_batch_create(const riop_desc *descs, int32_t nchannels, const void *const *uv,
                              int32_t autotune, void *stream, riop_batch **out);
riop_status riop_batch_sdmm(riop_batch *batch, const void *const *y, const double *eps,
                            const riop_sdmm_params *params, int32_t iters_per_graph,
                            void *const *x_out, riop_sdmm_stats *stats, void *stream);
riop_status riop_batch_plan(riop_batch *batch, int32_t channel, riop_plan **plan);
riop_status riop_batch_tile(const riop_batch *batch, int32_t channel, int32_t *tile, double *pair_ms);
riop_status riop_batch_destroy(riop_batch *batch);
riop_status riop_autotune_tile(const riop_desc *desc, const void *uv, int32_t reps, void *stream,
                               int32_t *best_tile, double *pair_ms);

/* Kernel timing with HIP events (for benchmarks).  When enabled, every kernel
 * launch of the plan is bracketed by a pair of events recorded on the launch
 * stream and attributed to a kernel kind (see riop_timing_name).  Enabling
 * resets the accumulators; disabling stops recording.  No effect on results. */
riop_status riop_timing_enable(riop_plan *plan, int32_t on);

/* Total time (ms) and number of launches of one kernel kind since the last
 * enable.  Synchronises with the recorded events.  kind in [0, riop_timing_kinds()). */
riop_status riop_timing_read(riop_plan *plan, int32_t kind, double *total_ms, int64_t *launches);

/* Number of kernel kinds and the name of one ("degrid", "grid", ...). */
int32_t riop_timing_kinds(void);
const char *riop_timing_name(int32_t kind);

/* Message for the last failure on the calling thread ("" if none). */
const char *riop_last_error(void);

/* Library version, e.g. "riop 0.1.0 gfx950". */
const char *riop_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RIOP_H */
