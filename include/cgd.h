/*
 * cgd.h -- coarse-grained (binned) photon-number distributions of Gaussian
 * states on one AMD Instinct MI355X (gfx950).  C ABI, C99.
 *
 * What is computed (arXiv:2412.17742):
 *   For a Gaussian state of M external modes, each carrying K internal
 *   (Schmidt) modes, measured by detectors grouped into L bins, the
 *   probability generating function of the bin counts is
 *       G(w) = sum_b Pr(b) prod_l w_l^{b_l} = Pr(0) q(A, gamma, w)
 *   (Eq. Lamb_lhaf_master times the vacuum probability, Eq. vacuum_probability;
 *   q in closed form, Eq. q_d).  The library evaluates G at every point of the
 *   roots-of-unity grid w_l = exp(2 pi i k_l / G_l) -- one complex determinant
 *   det[I - D(w) X A] with the square-root branch continuous from w = 0, times
 *   the displacement exponential -- and inverts the grid with an L-dimensional
 *   DFT (the finite-difference sieve of Sec. V with roots-of-unity nodes).
 *   The result is the wrapped distribution
 *       P(b) = sum_{m >= 0} Pr(b + m o G),   b_l in [0, cutoff_l],
 *   which equals the exact binned probability Pr(b) of Eq. coarse_grained_prob
 *   when the probability mass beyond the grid is negligible; choose G_l large
 *   enough for that, or accept the wrap.
 *
 * State model (Sec. II, Sec. VI B, Sec. VIII A):
 *   input j, internal mode k is a single-mode squeezed vacuum with squeezing
 *   r_jk, where tanh^2 r_jk = (lambda_k / lambda_0) tanh^2 r_j (the two-mode
 *   relation Eq. relation_between_sqz_par generalised to K modes), displaced
 *   by alpha_j on internal mode 0 only; the interferometer a_out = T a_in acts
 *   identically on every internal mode; internal modes never interfere.
 *
 * Conventions common to every call:
 *   - complex numbers are interleaved (re, im) pairs of double;
 *   - matrices are row-major;
 *   - host pointers are read only during the call; the caller keeps ownership;
 *   - device pointers are plain HIP device allocations owned by the caller
 *     (e.g. torch tensor data_ptr()); work is enqueued on the context's stream
 *     and is asynchronous with respect to the host;
 *   - no call throws or exits; each returns a cgd_status and, on failure,
 *     cgd_last_error() describes it.
 */
#ifndef CGD_H
#define CGD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cgd_ctx cgd_ctx; /* opaque; owned by the library */

typedef enum {
    CGD_OK = 0,
    CGD_ERR_ARG = 1,         /* invalid argument (sizes, indices, NULLs, unsupported shape) */
    CGD_ERR_NONPHYSICAL = 2, /* ||T||_2 > 1, r < 0, bad Schmidt weights: not a valid state  */
    CGD_ERR_NUMERIC = 3,     /* a pivot left the right half-plane or a value was not finite  */
    CGD_ERR_DEVICE = 4,      /* a HIP runtime call failed                                    */
    CGD_ERR_NOMEM = 5,       /* host or device allocation failed                             */
    CGD_ERR_STATE = 6        /* call order violated (e.g. grad before eval)                  */
} cgd_status;

typedef enum {
    CGD_PREC_FP64 = 0,  /* complex128 factorisations everywhere                          */
    CGD_PREC_MIXED = 1  /* complex64 factorisations at every grid point, then a complex128
                           re-factorisation of the points with the largest |G| until the
                           error bound of the points left in FP32 is within tol
                           (see cgd_create) */
} cgd_precision;

/* cgd_create flags */
#define CGD_FLAG_DENSE_INTERNAL 1u /* keep all K internal modes in one 2MK x 2MK matrix
                                      instead of K independent 2M x 2M blocks (the two
                                      give the same determinant; for testing/measurement) */
#define CGD_FLAG_NO_SCHUR 2u       /* evaluate every grid point with a full factorisation
                                      instead of reusing the first bin's eigenbasis */
#define CGD_FLAG_HESSENBERG 8u     /* Hessenberg route, forced: when the rows left after
                                      eliminating the first bin all lie in one bin B (order
                                      <= 144, no displacement border), reduce every Schur
                                      matrix C(w_A) once to Hessenberg form so that each point
                                      costs O(n^2) instead of a full factorisation.  When they
                                      lie in two bins P and B (order <= 480, bin B <= 144),
                                      the pair route first eliminates the rows of P for every
                                      (w_A, w_P) by a partial LU and reduces what is left.
                                      FP64 in both precisions.  Without either Hessenberg flag
                                      the library takes these routes for those blocks when its
                                      estimate of the time is lower (many points per
                                      reduction). */
#define CGD_FLAG_NO_HESSENBERG 16u /* never take the Hessenberg route                        */
#define CGD_FLAG_GRAD 4u           /* prepare cgd_grad (keeps each internal block's full
                                      matrix on the device); needs 2M(+1) <= 481 per block
                                      (above 96: a blocked inverse with an HBM workspace
                                      of up to 512 x order^2 x 16 bytes) */
#define CGD_FLAG_MOMENTS 64u       /* cgd_eval writes, per instance and in the layout of the
                                      probabilities, the coarse-grained joint moments
                                      E[prod_l b_l^{p_l}] for p_l in [0, cutoff_l] (Sec. VI C,
                                      Eq. CGmom) instead of probabilities; see below       */
#define CGD_FLAG_CUMULANTS 128u    /* as CGD_FLAG_MOMENTS, with the joint cumulants
                                      <<prod_l b_l^{p_l}>> (Eq. CGmom2; p = 0 gives 0)
   Moments and cumulants are the Taylor coefficients of the moment generating
   function M(t) = G(e^t) (Eq. M) and of log M(t) times p!: G (or log G, on the
   continuous branch) is evaluated on a polydisk t_l = rho exp(2 pi i k / G_l)
   and inverted with the same DFT (the finite-difference sieve with a shared
   variable per bin, nodes on a circle).  rho is a quarter of the distance
   log(1 / ||H||_2) to the nearest singularity, where I - D(e^t) H stays
   accretive; G_l defaults to max(24, 2 (cutoff_l + 1)) points (grid NULL or 0),
   so the aliasing of the coefficients scales as 4^-G_l (cgd_bounds reports it
   as wrap_bound) and rounding grows as (4 / log(1/||H||))^{|p|} p!.  FP64 only,
   no CGD_FLAG_GRAD. */
#define CGD_FLAG_NO_LOWRANK 256u   /* factorise low-rank blocks like the others (see
                                      "Low-rank blocks"; for tests)                        */
#define CGD_FLAG_NO_AUTOTUNE 32u   /* skip the autotuner of cgd_create: default kernel shape
                                      per size class, FP32 pass for every eligible class on
                                      the mixed path (see cgd_tuning)                      */

/* One instance (a Gaussian state plus its binning).  Sec. VI A (set partition
 * Lambda, coarse pattern b), Sec. VI B (internal modes). */
typedef struct {
    int32_t M;               /* external modes, >= 1; M*K <= 4096 (M <= 512 if distinguishable) */
    int32_t K;               /* internal (Schmidt) modes per external mode, >= 1              */
    int32_t L;               /* bins, 1..8                                                    */
    const double *T;         /* M*M complex: a_out[i] = sum_j T[i*M+j] a_in[j]; ||T||_2 <= 1  */
    const double *r;         /* M squeezing parameters >= 0 (internal mode 0)                 */
    const double *alpha;     /* M complex displacements of internal mode 0, or NULL (zero)    */
    const double *schmidt;   /* K weights > 0 summing to 1, lambda_k <= lambda_0; NULL iff K==1 */
    const int32_t *bin_of;   /* per mode: bin index in [0, L), -1 (not measured: traced out) or
                                CGD_KEEP (-2: kept, see "Heralded density matrices" below); M
                                entries (external modes; a kept external mode keeps all its K
                                internal modes) or M*K entries (index i*K+k) if
                                resolve_internal != 0                                          */
    int32_t resolve_internal;/* 0: detectors see external modes; 1: bins over (i, k) pairs     */
    const int32_t *cutoff;   /* L entries N_l >= 0: output box b_l in [0, N_l]                */
    const int32_t *grid;     /* L entries G_l >= N_l + 1, or NULL for G_l = N_l + 1; an entry 0
                                asks for the smallest G_l >= N_l + 1 whose tail bound
                                Pr(b_l >= G_l) (see cgd_bounds) is at most tol / (10 L), so
                                that the wrapped distribution is within tol / 10 of the exact
                                binned probabilities (needs a finite tol > 0; G_l <= 4096)    */
    int32_t fock_cutoff;     /* with kept modes: Fock cutoff N >= 0 of every kept mode; ignored
                                otherwise                                                      */
    int32_t distinguishable; /* 1: fully distinguishable inputs (App. D): input j carries its
                                squeezing r_j in its own internal mode j and vacuum in the
                                others, so K must equal M; schmidt and alpha must be NULL.
                                Each internal block then has rank 2 (see "Low-rank blocks")    */
} cgd_instance;

#define CGD_KEEP (-2)

/* Heralded density matrices (Sec. VII, Eq. heralded_state_internal).  An
 * instance with g >= 1 kept modes returns, for every heralding pattern b~ of
 * its L bins in the box, the unnormalised state of the kept modes conditioned
 * on b~:
 *     rho(b~)[v][u] = <v| rho_G(b~) |u> = sum_{n~ in K(b~)} <n~, v| rho |n~, u>,
 * u, v Fock patterns of the kept modes with entries in [0, fock_cutoff]; modes
 * with bin -1 are traced out.  Its trace over all u is Pr(b~).  Like the
 * probabilities, the output is the wrapped sum over b~ + m o G; each element
 * is within cgd_bounds' wrap_bound of the exact one.
 * Layout of the instance's output: 2 D^2 prod_l (N_l + 1) doubles (interleaved
 * complex), [b~][v][u], D = (fock_cutoff + 1)^g, the multi-indices u and v
 * row-major over the kept modes in mode order (last kept mode fastest); the
 * instance's offset from cgd_layout is even.
 * Method: per grid point, the kept modes' rows and columns of A and their
 * loop-vector entries border the heralding block, whose elimination leaves
 * the quadratic form of the generating function
 *     sum_{u,v} <v| rho_G(w) |u> x^u y^v / sqrt(u! v!)
 *         = G_H(w) exp(l(w)^T c + 1/2 c^T Q(w) c),  c = (y, x)
 * (the master theorem, Eq. lhaf_master, with a loop vector that depends on the
 * kept modes' variables); a recurrence expands it into the D^2 elements, and
 * the inverse DFT over the heralding grid runs for each of them.  The
 * permutation trick of Sec. VII (a larger matrix per (u, v)) is not used.
 * Restrictions: CGD_PREC_FP64; no CGD_FLAG_GRAD, CGD_FLAG_MOMENTS,
 * CGD_FLAG_CUMULANTS; 2 g <= 16; D^2 <= 2^22; every internal block of order
 * <= 144 (heralding rows left after eliminating one bin, plus 2 g_k + 1 border
 * rows); at most 2^31 values per instance (grid points times D^2). */

/* Low-rank blocks (App. D; Sec. VI B for the internal-mode blocks).  An
 * internal block in which q inputs are squeezed has Sigma - I, and so
 * H = I - Sigma^-1, of rank at most 2q: every block of an instance with
 * distinguishable != 0 has rank 2 (its one squeezed input), and a K = 1
 * instance with one or two squeezed inputs has rank 2 or 4.  When the rank
 * r = 2q is at most 4 and at most half the block's order, the block has no
 * displacement, no kept mode and CGD_FLAG_GRAD is off, cgd_create writes
 * Sigma - I = Y C Y^H (Y: 2M x r from the squeezed inputs' columns of T, C:
 * their sinh^2 and sinh cosh), takes H = V diag(lambda) V^H from the order-r
 * matrix |Y| C |Y| (Woodbury; O(M r^2) work per block, no matrix of order 2M;
 * a numerically rank-deficient Y sends the block to the general route) and
 * keeps the (L + 1) matrices G_g = diag(lambda) V^H E_g V of order r
 * (E_g: the rows of bin g; one more for the traced rows).  Per grid point
 * det(I - D(w) H) = det(I_r - G_t - sum_l w_l G_l) (Sylvester's identity), an
 * r x r unpivoted LU in FP64 on both precision paths; the pivots lie in the
 * right half-plane (I_r - C is a diagonal similarity transform of an
 * accretive matrix), so the sum of their principal logarithms is the same
 * continuous branch as the factorisation's.  CGD_FLAG_NO_LOWRANK sends these
 * blocks through the general factorisation instead (results agree to
 * rounding).  cgd_tuning's lowrank_blocks counts the blocks taken this way. */

/* Assemble the states (FP64, host) and upload everything the evaluation
 * needs.  n_inst instances are evaluated together by cgd_eval.
 *   prec        CGD_PREC_FP64 or CGD_PREC_MIXED
 *   tol         absolute error budget per probability for the mixed path (e.g.
 *               1e-9).  A point's FP32 value of G is taken to carry a relative
 *               error of at most tau (2 (n+1) 2^-24 summed over its blocks of
 *               order n) and enters every probability as c_k |G_k| tau / prod G
 *               (c_k = 1 or 2 on the Hermitian half grid).  Per instance, the
 *               points are ranked by |G| (quarter-octave buckets); the smallest
 *               ones stay in FP32 as long as their summed c_k |G_k| tau / prod G
 *               is at most tol, the others are factorised again in FP64;
 *               ignored for FP64
 *   flags       0 or CGD_FLAG_* bits
 *   hip_stream  hipStream_t to enqueue on, or NULL for the null stream
 * Errors: CGD_ERR_ARG / CGD_ERR_NONPHYSICAL synchronously, before any launch.
 * On failure *out is set to NULL. */
cgd_status cgd_create(cgd_ctx **out, const cgd_instance *inst, int32_t n_inst,
                      cgd_precision prec, double tol, uint32_t flags, void *hip_stream);

/* Sizes of the outputs, in doubles.  n_probs_total = sum_i of prod_l (N_l + 1)
 * (2 D^2 prod_l (N_l + 1) for an instance with kept modes, after one double of
 * padding if needed to keep its offset even); prob_offsets (n_inst + 1
 * entries, may be NULL) gives each instance's first double; n_grid_total (may
 * be NULL) is the number of grid points whose values are produced
 * (sum_i prod_l G_l).  Probabilities are row-major over (b_1, ..., b_L) with
 * b_L fastest. */
cgd_status cgd_layout(const cgd_ctx *ctx, int64_t *n_probs_total, int64_t *prob_offsets,
                      int64_t *n_grid_total);

/* Evaluate the wrapped distributions (density matrices for instances with
 * kept modes) of all instances into d_probs (device, n_probs_total doubles).  d_err_bound (device, n_inst doubles, or NULL)
 * receives, per instance, a bound on the absolute error added by the mixed
 * path to every probability: (1/prod G) sum over the points kept in FP32 of
 * c_k |G_k| tau, with tau the modelled relative error of an FP32 value of G
 * (0 on the FP64 path; +inf after a numeric failure).  A numeric failure
 * detected on the device is reported by the next call as CGD_ERR_NUMERIC. */
cgd_status cgd_eval(cgd_ctx *ctx, double *d_probs, double *d_err_bound);

/* Evaluation that allocates nothing, for callers that cannot allocate device
 * memory: code under HIP stream capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, result and error behaviour as cgd_eval,
 * bit for bit, but the launches are enqueued directly on the context's stream
 * (no HIP graph is instantiated, no per-stage timing) and the per-evaluation
 * buffers (per-point contributions, log G, the DFT passes, the mixed path's
 * FP32 values, bucket sums and re-factorisation lists, the Hessenberg route's
 * tables) live in a static device array of 128 MiB per GPU, held by each GPU
 * the library runs on until the process ends.  The context's own allocations
 * from cgd_create (state, matrix pool, blocked-LU workspace, status word) are
 * used as by cgd_eval.
 *   Errors: CGD_ERR_ARG if the context needs more than 128 MiB of these
 *   buffers (the message gives the size) or the current device is not the one
 *   the context was created on; the other errors as for cgd_eval.
 *   Every call on one GPU shares that GPU's array and keeps the last call's
 *   contents: calls that overlap on one GPU (other streams, other host
 *   threads) race and must be serialised by the caller.  cgd_grid_values,
 *   cgd_grad and cgd_mixed_stats need a cgd_eval after it (CGD_ERR_STATE). */
cgd_status cgd_eval_static(cgd_ctx *ctx, double *d_probs, double *d_err_bound);

/* Diagnostic: after cgd_eval, copy log G(w) (complex) at the evaluated grid
 * points into d_logg (device, 2 * cgd_points(ctx) doubles).  Points are
 * instance by instance; within an instance k_1 runs over [0, G_1/2] (the other
 * half follows from G(conj w) = conj G(w)) and k_2..k_L over [0, G_l), row-major
 * with k_L fastest. */
int64_t    cgd_points(const cgd_ctx *ctx);
cgd_status cgd_grid_values(cgd_ctx *ctx, double *d_logg);

/* Gradient of a real loss with respect to the inputs, given dLoss/dP (device,
 * n_probs_total doubles, same layout as the probabilities).  Requires a
 * context created with CGD_FLAG_GRAD and a preceding cgd_eval (CGD_ERR_STATE
 * otherwise).  Outputs (device, may be NULL each; instances concatenated):
 *   d_dr        sum_i M_i doubles               dLoss/dr
 *   d_dT        sum_i M_i*M_i complex            dLoss/dRe T + i dLoss/dIm T
 *   d_dalpha    sum_i M_i complex                dLoss/dRe alpha + i dLoss/dIm alpha
 *   d_dschmidt  sum_i K_i doubles                dLoss/dlambda_k, each Schmidt weight
 *               taken as a free variable (the state depends on lambda_k / lambda_0
 *               only, through tanh^2 r_jk = (lambda_k / lambda_0) tanh^2 r_j, so
 *               sum_k lambda_k dLoss/dlambda_k = 0; 0 for K = 1)
 * Per grid point and internal block, S' (bordered) is inverted in FP64 on the
 * GPU (d log det S = tr(S^-1 dS)); the sums over the grid are reduced in a
 * fixed order (bitwise reproducible); the chain rule from H = I - Sigma^-1,
 * gamma and log Pr(0) to (r, T, alpha, lambda) runs on the host in FP64.  The
 * call waits for the device (the host chain rule needs the reduced sums). */
cgd_status cgd_grad(cgd_ctx *ctx, const double *d_dprobs, double *d_dr, double *d_dT, double *d_dalpha,
                    double *d_dschmidt);

/* Profiling.  The evaluation is a fixed sequence of launch stages:
 *   CGD_STAGE_SCHUR      Schur matrices of the bins left after eliminating one bin
 *   CGD_STAGE_LU_REG0..4 register-resident factorisations, orders <= 32, 64, 96, 128, 144
 *                        (mixed path: the FP32 MFMA kernels of the same orders)
 *   CGD_STAGE_LU_BIG     blocked FP64 factorisations, orders 145..480 (mixed path:
 *                        the FP32 MFMA kernel for orders 145..192, FP64 above)
 *   CGD_STAGE_COMBINE    log G per point and G = exp(log G)
 *   CGD_STAGE_DFT        all axis passes of the inverse DFT
 *   CGD_STAGE_HESS       Hessenberg route: reduction of each C(w_A)
 *   CGD_STAGE_HESS_DET   Hessenberg route: the O(n^2) factorisation of every
 *                        (w_A, w_B) pair, copy to the points
 *   CGD_STAGE_PAIR       pair route: partial LU of every (w_A, w_P) pair, which
 *                        leaves the matrix the Hessenberg stages reduce
 *   CGD_STAGE_FIX        mixed path: selection of the points whose FP32 value can
 *                        matter, their FP64 re-factorisation and the second combine
 *   CGD_STAGE_DENSITY    density mode: expansion of every point's generating function
 *                        into matrix elements, and rho = R + R^H after the DFT
 * With timing enabled, cgd_eval runs eagerly and records a HIP event pair on
 * the context's stream around every launch of a stage; cgd_stage_times waits
 * for the last evaluation and returns, per stage, the sum of its launches'
 * durations in ms (-1 for stages with no work).
 * cgd_stage_work returns each stage's algorithmic work per evaluation:
 * flops (complex LU of order n: 8 sum_m m^2 + 6 sum_m m, m = n-1..0, i.e.
 * about 8n^3/3 real flops; Schur build: 8 nA nB^2 per eliminated-bin value;
 * pair route: the nP pivots of a partial LU as for the LU; Hessenberg
 * reduction of order n: step k (m = n - k - 1 rows below the
 * diagonal) 2 m (m + 1) + 2 n m complex multiply-adds; Hessenberg
 * factorisation: 2 (n - k - 1) per pivot k; DFT: 8 flops per complex
 * multiply-add) and bytes (DFT: each grid value read once, each
 * probability written once, 16 and 8 bytes). */
enum {
    CGD_STAGE_SCHUR = 0,
    CGD_STAGE_LU_REG0 = 1,
    CGD_STAGE_LU_BIG = 6,
    CGD_STAGE_COMBINE = 7,
    CGD_STAGE_DFT = 8,
    CGD_STAGE_FIX = 9,
    CGD_STAGE_HESS = 10,
    CGD_STAGE_HESS_DET = 11,
    CGD_STAGE_PAIR = 12,
    CGD_STAGE_DENSITY = 13,
    CGD_NSTAGES = 14
};
cgd_status cgd_set_timing(cgd_ctx *ctx, int32_t enable);
cgd_status cgd_stage_times(cgd_ctx *ctx, double *ms /* CGD_NSTAGES */);
cgd_status cgd_stage_work(const cgd_ctx *ctx, double *flops /* CGD_NSTAGES */, double *bytes /* CGD_NSTAGES */);

/* Mixed path: number of (internal block, grid point) factorisations that the
 * last cgd_eval repeated in FP64, and the total number of factorisations per
 * evaluation.  Waits for the last evaluation.  CGD_ERR_STATE on the FP64 path
 * or before the first evaluation. */
cgd_status cgd_mixed_stats(cgd_ctx *ctx, int64_t *n_refactored, int64_t *n_total);

/* Grid and wrap bound of every instance (host outputs, may be NULL each):
 *   grid        sum_i L_i entries: the grid extents G_l in use (automatic
 *               entries resolved), instances concatenated
 *   wrap_bound  n_inst entries: sum_l B_l with B_l >= Pr(b_l >= G_l), so that
 *               0 <= P(b) - Pr(b) <= wrap_bound for every b in the box, P the
 *               wrapped distribution on the grid and Pr(b) the exact binned
 *               probability (Eq. coarse_grained_prob).
 * B_l is the Chernoff bound min_{s > 1} E[s^{b_l}] / s^{G_l} with the marginal
 * moment generating function of bin l in closed form (Sec. VI C, Eq. M, the
 * other bins' variables at t = 0): per internal block, with R the bin's rows
 * and columns of Sigma^(s=1) and zbar its means,
 *   E[s^b] = exp(1/2 (s-1) zbar^H (I - (s-1) R)^-1 zbar) / sqrt(det(I - (s-1) R)),
 * evaluated exactly (FP64) from a tridiagonal form of R, and minimised over s
 * up to the edge of convergence.  With the Hermitian half grid the library
 * sums, the output has no imaginary part to report. */
cgd_status cgd_bounds(const cgd_ctx *ctx, int32_t *grid, double *wrap_bound);

/* Autotuner report (JSON text, valid until cgd_destroy; NULL if ctx is NULL).
 * cgd_create times, for every size class of per-point factorisations in the
 * context, each candidate kernel shape on a sample of up to 8192 of the
 * class's own (block, grid point) items: the thread grids of the FP64 register
 * kernel and, on the mixed path, the wave layouts of the FP32 MFMA kernel, and
 * keeps, of each kind, the first shape within 2% of the fastest (so that
 * shapes that time alike do not flip between runs).  On the mixed path a class whose best FP32
 * pass is not below 0.5 of its best FP64 time is evaluated directly in FP64
 * (no FP32 error, nothing to factorise again).  On the sample the tuner also
 * compares each FP32 item with its FP64 value: fp32_err_ratio_max is the largest
 * difference in units of the assumed FP32 error of the block, and where it
 * exceeds 0.5 the assumed error of the class's blocks is scaled up by
 * ratio / 0.5 (the error bound only grows).  Per class: every time (ms),
 * the chosen kernels, the precision and that ratio.  lowrank_blocks counts
 * the internal blocks evaluated by the low-rank route (no factorisation). */
const char *cgd_tuning(const cgd_ctx *ctx);

/* Pin the kernel shape of a size class (0..4: orders <= 32, 64, 96, 128, 144),
 * overriding the autotuner: fp64_shape indexes the class's FP64 shapes in the
 * order of the report's "fp64_ms" (register-kernel thread grids first, then
 * FP64 MFMA wave layouts), fp32_shape its FP32 MFMA shapes ("fp32_ms"); -1
 * keeps the current one.  For tests, profiling (the same kernel in every
 * run) and callers that want reproducible launch shapes; results differ only
 * by rounding.  Precision choices (which classes run an FP32 pass) are not
 * changed.  Errors: CGD_ERR_ARG for a shape out of range, an FP32 shape for a
 * class without an FP32 pass, or an FP64 MFMA shape for a class with kept
 * modes (density mode needs the register kernel). */
cgd_status cgd_set_kernel_shape(cgd_ctx *ctx, int32_t size_class, int32_t fp64_shape, int32_t fp32_shape);

void cgd_destroy(cgd_ctx *ctx);

/* Message of the last failure on this thread (valid until the next call). */
const char *cgd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CGD_H */
