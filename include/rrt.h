/*
 * rrt.h -- C ABI of the MI355X reverse ray tracer (librrt.so).
 *
 * The library computes the self-shielded hydrogen photoionisation rate and the
 * equilibrium neutral fraction of every SPH gas particle by reverse ray tracing
 * (Altay & Theuns, "URCHIN: A Reverse Ray Tracer for Astrophysical
 * Applications", Sec. 3.3 and Sec. 4):
 *
 *   1. every particle casts n_ray rays of length l_ray (HEALPix directions,
 *      Sec. 3.3) -- the directions are an input array;
 *   2. each ray's HI column is the sum, over every particle whose kernel sphere
 *      the segment enters, of mu_j x_j times the line integral of the truncated
 *      Gaussian kernel G_t along the part of the chord inside the segment
 *      (Sec. 4.1.1, eq. colden and eq. Gt, closed form I(h,b,z1,z2));
 *   3. Gamma = (1/n_ray) sum_k sum_b w_b sigma_b exp(-sigma_b N_k)
 *      (Sec. 3.3, eq. gamma_shld, frequency integral done over bins with
 *      w_b = 4 pi J_b dnu_b / (h nu_b));
 *   4. x = x_-(Gamma, n_H, T), the physical root of the equilibrium quadratic
 *      (Appendix C.3, eq. xroots, y = 0);
 *   5. steps 2-4 repeat to a fixed point; every particle is updated from the
 *      same previous state (the order-independent update of Sec. 4).
 *
 * Units: positions and h in kpc; mu = hydrogen atoms / (kpc in cm)^2, so that
 * mu * x * (kernel line integral in kpc^-2) is a column in cm^-2; n_H in
 * cm^-3; T in K; sigma in cm^2; w in photons cm^-2 s^-1; Gamma in s^-1.
 *
 * Conventions for every entry point:
 *  - Return value: RRT_OK (0) on success, a negative RRT_E_* code on error,
 *    RRT_NOT_CONVERGED (> 0) as a warning.  rrt_last_error() gives text.
 *    No C++ exception crosses the ABI.
 *  - Pointers marked "device" are caller-owned device memory on the GPU the
 *    context was created on; "host" pointers are caller-owned host memory.
 *    The library copies what it keeps; it never frees caller memory.
 *  - Work is enqueued on the stream given to rrt_create (NULL = the null
 *    stream).  Calls that return a scalar to the host synchronise that stream.
 *  - The library allocates its own device buffers (tree, sorted particle
 *    arrays, columns, scratch) with hipMalloc, sized by the particle count,
 *    and releases them in rrt_destroy.
 *  - A context is not thread-safe; use one context per host thread.
 */
#ifndef RRT_H
#define RRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RRT_OK = 0,
    RRT_NOT_CONVERGED = 1,    /* warning: max_iter reached before tolerance   */
    RRT_E_ARG = -1,           /* invalid argument (null, size, range)          */
    RRT_E_HIP = -2,           /* HIP runtime error                             */
    RRT_E_INPUT = -3,         /* non-finite or out-of-range particle data      */
    RRT_E_STATE = -4,         /* call out of order (e.g. columns before tree)  */
    RRT_E_NOMEM = -5,         /* device allocation failed                      */
    RRT_E_CAPACITY = -6       /* caller buffer too small                       */
};

typedef struct rrt_ctx rrt_ctx;

typedef struct {
    double l_ray;          /* ray length in kpc, >= 0 (Sec. 3.3: l_ray)              */
    double box;            /* periodic box side in kpc; 0 = isolated (no images)    */
    int64_t path_budget;   /* bytes the recorded ray paths may take; 0 = half of the
                              free device memory at the time of recording           */
    int32_t leaf_size;     /* max particles per tree leaf, 1..8 (0 = default 8)     */
    int32_t block_size;    /* threads per block of the traversal: 0 (= 128) or a
                              multiple of 64 up to 256                               */
    int32_t record_paths;  /* -1 = record when within path_budget (default),
                              0 = traverse every iteration, 1 = require recording   */
    int32_t traversal;     /* 0 = wave-cooperative walk (default), 1 = one
                              independent walk per lane; identical results          */
    int32_t reserved[2];   /* must be zero                                           */
} rrt_params;

/* Ray paths.  The geometry of every ray (which particles it intersects and the
 * kernel chord factor K/h^2 of each) does not depend on x, because the column
 * is linear in the neutral fractions (Sec. 4.1.1, eq. colden).  With path
 * recording the first column evaluation after a tree build traverses the tree
 * and records 8 bytes per intersection (particle index and factor), in one
 * walk or in a counting walk and a recording walk (RRT_TUNE_ONE_PASS); every
 * evaluation then forms N = sum (mu x)_j * factor_j by a
 * streaming product over the recorded paths.  Without it, every evaluation
 * traverses the tree.  Both give the same intersections and terms; the two
 * sums differ only in summation order. */

/* Library version as major*10000 + minor*100 + patch. */
int rrt_version(void);

/* Create a context on the current HIP device.  stream: a hipStream_t (may be
 * NULL).  *out receives the context; on failure *out is NULL. */
int rrt_create(rrt_ctx** out, const rrt_params* params, void* stream);

/* Release every device buffer the context owns. Safe on NULL. */
void rrt_destroy(rrt_ctx* ctx);

/* Text of the last error on this context (or of the last failed create when
 * ctx is NULL).  Valid until the next call on the context. */
const char* rrt_last_error(const rrt_ctx* ctx);

/* Particle data (Sec. 4.1.1, eq. nhi: m_i, x_i, h_i; plus n_H and T for the
 * rates of Appendix C.3).  All device pointers, n entries each:
 *   pos  float[n][3]  positions in kpc
 *   h    float[n]     smoothing length in kpc, > 0 (kernel support radius)
 *   mu   float[n]     hydrogen atoms / kpc_cm^2, >= 0
 *   n_H  float[n]     hydrogen density in cm^-3, > 0
 *   T    float[n]     temperature in K, > 0
 * x_init: device double[n] initial neutral fractions, or NULL for the optically
 * thin state x_thin = x_-(Gamma_thin) (Sec. 4).  Copied; validated by
 * rrt_build_tree, which must follow. n >= 1. */
int rrt_set_particles(rrt_ctx* ctx, int64_t n, const float* pos, const float* h,
                      const float* mu, const float* n_H, const float* T,
                      const double* x_init);

/* Independent problems in one context: particles [offsets[h], offsets[h+1])
 * form halo h, and a halo's rays see only its own particles.  host int64
 * offsets[n_halo + 1], 0 = offsets[0] < ... < offsets[n_halo] = n, n_halo
 * 1..4096.  Call after rrt_set_particles (which resets to one halo) and before
 * rrt_build_tree.  The tree keeps each halo in its own subtree. */
int rrt_set_halos(rrt_ctx* ctx, int32_t n_halo, const int64_t* offsets);

/* Ray directions (Sec. 3.3: HEALPix pixel centres): host double[n_ray][3] unit
 * vectors, 1 <= n_ray <= 3072.  Every particle casts the same directions. */
int rrt_set_rays(rrt_ctx* ctx, int32_t n_ray, const double* dirs);

/* HEALPix RING-order pixel-centre directions for n_side (1..16): writes
 * 12 n_side^2 unit vectors into host double[12 n_side^2][3]. */
int rrt_healpix_dirs(int32_t n_side, double* dirs_out);

/* Binned optically thin spectrum (Sec. 2 eq. gamma; Sec. 3.3 eq. gamma_shld):
 * host double sigma[n_bins] (cm^2, > 0) and w[n_bins] (>= 0) with
 * Gamma_thin = sum_b w_b sigma_b > 0.  1 <= n_bins <= 4096. */
int rrt_set_spectrum(rrt_ctx* ctx, int32_t n_bins, const double* sigma, const double* w);

/* Build the bounding-volume tree over the particles: scene bounds, 63-bit
 * Morton keys, radix sort by (key, index), binary radix tree, box refit,
 * depth-first layout with skip links; gathers particle data into tree order,
 * evaluates the per-particle rates and sets the initial state.  Synchronises
 * (the key quantisation needs the scene bounds on the host). */
int rrt_build_tree(rrt_ctx* ctx);

/* Columns for the current state x (Sec. 4.1.1, eq. colden): N[p][k] in cm^-2.
 * N_out: device double[n][n_ray] in input particle order, or NULL to keep the
 * columns internal.  n_hits_out: host, total ray-particle intersections of this
 * call (counting each periodic image separately), or NULL (then no sync). */
int rrt_compute_columns(rrt_ctx* ctx, double* N_out, int64_t* n_hits_out);

/* Shielded rate from the current columns (Sec. 3.3, eq. gamma_shld):
 * ln Gamma, Gamma and tau_eff = ln Gamma_thin - ln Gamma per particle.
 * Device outputs in input order, each nullable: double lnG[n], double G[n],
 * float tau[n]. */
int rrt_compute_gamma(rrt_ctx* ctx, double* lnG_out, double* G_out, float* tau_out);

/* One equilibrium update from the current Gamma (Appendix C.3, physical root
 * x_-): x <- x_-(Gamma, n_H, T) with case A rates, for every particle
 * (the update rule below applies to rrt_iterate_equilibrium only).
 * x_out: device double[n] (nullable); max_dx_out: host max |x_new - x_old|
 * (nullable, syncs). */
int rrt_update_equilibrium(rrt_ctx* ctx, double* x_out, double* max_dx_out);

/* The paper's stable scheme for SPH (Sec. 4.1.2).  near_far = 1: the
 * particles a ray from source i intersects are split into near ones (their
 * kernel contains i, so they contribute to i's density in the scatter form of
 * eq. nhi; |d|^2 < h^2 in FP64 with d as in the hit predicate) and far ones.
 * Per ray the far HI column attenuates the radiation reaching a uniform slab
 * that stands for the near particles: density n_H and temperature of i, total
 * hydrogen column = the near particles' column with every x = 1.  The ray's
 * rate is the rate at the bottom of that slab (eq. gammashldk): for one bin
 * the monochromatic slab solution of Appendix C.4; for several bins the slab
 * in equilibrium at every depth under the far-attenuated binned spectrum,
 * solved per ray (the bottom is where the hydrogen column, the integral of
 * 1/x over the HI column, reaches the near column; 6-point Gauss-Legendre
 * steps and Newton's method, with the spectrum's attenuation tabulated once
 * per spectrum), in place of the paper's 4-D table of the same function.
 * Weighting (eq. gammashld, 4 pi inside w): with near_far = 1 each ray's slab
 * is lit by the ray's share, 1/n_ray of the far-attenuated spectrum, and
 * Gamma = sum_k Gamma_k (exact for a plane-parallel beam, Sec. 5.1-5.2);
 * near_far = 2 is a variant that lights each slab with the whole
 * far-attenuated spectrum and takes Gamma = (1/n_ray) sum_k Gamma_k (exact
 * when light arrives alike from every direction).  Recorded paths are dropped
 * when the split is switched on or off, not between 1 and 2.  While a near/far
 * scheme is set, rrt_forward, rrt_backward, rrt_iterate_halos and update rules
 * other than the default return RRT_E_STATE.  0 (default): the plain scheme. */
int rrt_set_scheme(rrt_ctx* ctx, int32_t near_far);

/* Near total-hydrogen columns of the last rrt_compute_columns under the
 * near/far scheme (the far columns are what rrt_compute_columns returns):
 * device double out[n][n_ray], input order, cm^-2.  Synchronises. */
int rrt_get_near_columns(rrt_ctx* ctx, double* out);

/* Non-equilibrium evolution (Appendix C.3, time-dependent solution of eq.
 * dxdt with y = 0): n_steps steps of length dt seconds; each step takes the
 * columns and Gamma of the current state and advances every particle by dt
 * with the closed-form solution at that constant Gamma (case A rates, the
 * current scheme).  dt = 0 leaves x unchanged; a very long dt gives the
 * equilibrium update.  x_out: device double[n] (nullable, syncs).  Needs the
 * default update rule (RRT_E_STATE otherwise). */
int rrt_evolve(rrt_ctx* ctx, double dt, int32_t n_steps, double* x_out);

/* The update rule of rrt_iterate_equilibrium, after the paper's own scheme
 * (Sec. 4, implementation details).  Defaults (0, +inf, 0, 1) give the
 * order-independent case A update that every other entry point assumes.
 *   tau_skip    >= 0: particles whose first shielded rate of the solve gives
 *               tau_eff < tau_skip keep their starting state for good and cast
 *               no rays afterwards (0 = none are frozen);
 *   tau_case_b  > 0: case B recombination (Hui & Gnedin 1997) for particles
 *               with tau_eff >= tau_case_b, case A below (+inf = case A only);
 *   relative    1: convergence on max |dx| / x instead of max |dx|;
 *   n_blocks    1..2^20: each sweep visits the particles from high to low
 *               n_H (ties: lower input index first) in n_blocks blocks of
 *               ceil(n / n_blocks); a block's rates see every update of the
 *               blocks before it (1 = every particle from the same state).
 * tau_eff decisions are taken in FP64 from ln Gamma.  While a rule other than
 * the default is set, rrt_forward, rrt_backward and rrt_iterate_halos return
 * RRT_E_STATE.  Intersections are not counted for sweeps that skip rays over
 * recorded paths (rrt_get_counters reports -1 for the last sweep). */
int rrt_set_update_rule(rrt_ctx* ctx, double tau_skip, double tau_case_b, int32_t relative,
                        int32_t n_blocks);

/* The fixed point (Sec. 3.3, Sec. 4): repeat columns -> Gamma -> x until the
 * largest change of a sweep is below tol or max_iter sweeps, under the update
 * rule above.  x_out: device double[n] (nullable).  iters_done, max_dx_out:
 * host (nullable).  Returns RRT_NOT_CONVERGED if max_iter was reached without
 * convergence.  Synchronises once per sweep (16 bytes) for the convergence
 * test; the first call of rrt_set_update_rule's density order also copies
 * n_H to the host once. */
int rrt_iterate_equilibrium(rrt_ctx* ctx, int32_t max_iter, double tol, double* x_out,
                            int32_t* iters_done, double* max_dx_out);

/* ---- reverse mode ------------------------------------------------------
 * The differentiated map is K unrolled order-independent iterations from the
 * optically thin state: x^0 = x_-(Gamma_thin), then K times columns -> Gamma ->
 * x.  Parameters: the bin weights w (rrt_set_spectrum) and the particle
 * densities n_H; a particle's hydrogen content scales with its density at
 * fixed smoothing length, mu_j = mu_j(input) * n_H,j / n_H,j(input).  Outputs:
 * ln Gamma of the last iteration and x^K. */

/* New densities without a new tree (geometry and recorded paths are kept):
 * n_H device float[n] in input order, > 0. */
int rrt_set_density(rrt_ctx* ctx, const float* n_H);

/* Exactly K iterations from the optically thin state, keeping every iterate
 * for rrt_backward (K+1 device vectors of n doubles).  Outputs (device, input
 * order, nullable): lnG_out double[n] = ln Gamma^K, x_out double[n] = x^K. */
int rrt_forward(rrt_ctx* ctx, int32_t K, double* lnG_out, double* x_out);

/* Gradients of a scalar loss through the last rrt_forward, given its
 * derivatives with respect to the outputs (device, input order, nullable =
 * zero): dL_dlnG double[n], dL_dx double[n].  RRT_E_STATE unless rrt_forward
 * ran after the last change of spectrum, rays, tree or densities.  Writes
 * dL_dw (host double[n_bins], the spectrum as given; every w_b must be > 0)
 * and dL_dnH (device double[n], input order).  The transposed column product uses the recorded
 * paths, or re-traverses the tree when they are not recorded; it accumulates
 * with FP64 atomics, so dL_dnH can differ between runs in the last bits. */
int rrt_backward(rrt_ctx* ctx, const double* dL_dlnG, const double* dL_dx, double* dL_dw,
                 double* dL_dnH);

/* The fixed point of every halo at once: each halo iterates until its own
 * max|dx| < tol or max_iter iterations, then keeps its state while the others
 * continue (per-halo masks on the device).  After a first eager iteration
 * (which records the ray paths when they fit), the iterations run as replays
 * of a HIP graph of per_launch (1..256) iterations captured once per geometry
 * and parameters, on a stream the library owns (ordered after the context's
 * stream by events); the host reads 8 bytes after each replay.  x_out: device
 * double[n], input order (nullable).  halo_iters_out: host int32[n_halo]
 * iterations of each halo (nullable).  Returns RRT_NOT_CONVERGED if a halo
 * reached max_iter.  Works with one halo too. */
int rrt_iterate_halos(rrt_ctx* ctx, int32_t max_iter, double tol, int32_t per_launch,
                      double* x_out, int32_t* halo_iters_out);

/* Launch knobs for the autotuner (results never change, only speed):
 *   RRT_TUNE_TRACE_BLOCK  threads per block of the traversal (64, 128, 192, 256)
 *   RRT_TUNE_PACKET       rays walking one node sequence: 64 (a wave-cooperative
 *                         packet, default) or 1 (independent lanes)
 *   RRT_TUNE_PATH_GROUP   lanes per ray in the recorded-path product: 8, 16, 32,
 *                         64, or 0 = chosen from the mean intersections per ray
 *   RRT_TUNE_LEAF         particles per tree leaf (1..8), from the next build
 *   RRT_TUNE_ADJOINT      transposed column product of rrt_backward over
 *                         recorded paths: 0 (default) = gather over paths
 *                         transposed once per geometry when memory allows
 *                         (deterministic), else per row tile in LDS with one
 *                         atomic add per distinct particle of a tile (when the
 *                         tiles fit), else one atomic add per intersection;
 *                         1 = always one atomic add per intersection;
 *                         2 = always per row tile (when the tiles fit)
 *   RRT_TUNE_TILES        0 (default): columns from the recorded paths as
 *                         recorded.  1: after a few column evaluations over the
 *                         same recorded paths (and before the graph of a
 *                         batched solve is captured), group consecutive rays
 *                         into tiles whose particle values are staged in LDS,
 *                         so each intersection streams 6 bytes instead of 8 and
 *                         needs no global gather; the columns agree to FP64
 *                         summation order.  The one-time build costs about as
 *                         much as a hundred evaluations save on long rays, so
 *                         it pays for long solves with short rays only.
 *   RRT_TUNE_KEEP_COLUMNS 1 (default): rrt_forward keeps every iteration's
 *                         columns for rrt_backward when they take at most an
 *                         eighth of the free device memory (8 n n_ray K
 *                         bytes); 0: rrt_backward recomputes them from the
 *                         kept states.  The same columns either way.
 *   RRT_TUNE_ONE_PASS     1 (default): with the wave-cooperative walk and an
 *                         automatic path budget, record the paths in one walk
 *                         that appends each ray's entries to 32-entry chunks
 *                         of a pool and counts them, then compact the chunks
 *                         into rows; when the pool runs short, record in a
 *                         second walk as with 0.  The pool is sized from the
 *                         context's previous recording (so its first
 *                         recording takes two walks): 5/4 of its entries plus
 *                         half a chunk per ray, in 1024 slices with a counter
 *                         each, at most 45% of the free memory.  It is kept
 *                         between recordings, and released with the particle
 *                         buffers, at rrt_destroy, when this knob is set, or
 *                         when the paths would not fit beside it.  0: a
 *                         counting walk, then a recording walk.  n > 1: one
 *                         pass with a pool of about n chunks, also on a first
 *                         recording.  The same paths either way. */
enum { RRT_TUNE_TRACE_BLOCK = 1, RRT_TUNE_PACKET = 2, RRT_TUNE_PATH_GROUP = 3, RRT_TUNE_LEAF = 4,
       RRT_TUNE_ADJOINT = 5, RRT_TUNE_TILES = 6, RRT_TUNE_KEEP_COLUMNS = 7,
       RRT_TUNE_ONE_PASS = 8 };
int rrt_set_tuning(rrt_ctx* ctx, int32_t key, int32_t value);

/* Replace the state: x device double[n] in input order (checkpoint / resume,
 * or a given iterate); NULL resets to x_thin. */
int rrt_set_state(rrt_ctx* ctx, const double* x);

/* Read the state: device outputs in input order, each nullable. */
int rrt_get_state(rrt_ctx* ctx, double* x_out, double* lnG_out, double* G_out,
                  float* tau_out);

/* Tree export for inspection (host outputs).  Node i of the depth-first layout:
 * box lo[i][3], hi[i][3] (exact FP32 min/max of r -/+ h over its particles),
 * skip[i] (first node after its subtree), first[i] (first particle in tree
 * order), count[i] (particles in a leaf, 0 for internal nodes).  perm[n]: tree
 * order -> input index; codes[n]: sorted 63-bit Morton keys.  cap: capacity
 * in nodes; *n_nodes receives the node count (RRT_E_CAPACITY if cap is too
 * small).  Any output may be NULL. */
int rrt_get_tree(rrt_ctx* ctx, int64_t cap, int64_t* n_nodes, float* lo, float* hi,
                 int32_t* skip, int32_t* first, int32_t* count, int32_t* perm,
                 uint64_t* codes);

/* Hit lists for the current geometry (host outputs): the intersections of ray
 * (p, k) are hit_j[row_off[p*n_ray+k] .. row_off[p*n_ray+k+1]) as input
 * particle indices, with the periodic image of each in hit_img as
 * (sx+8) | (sy+8)<<4 | (sz+8)<<8 (the image of particle j sits at r_j + s*box).
 * row_off: int64[n*n_ray + 1].  cap: capacity of hit_j/hit_img; if the total
 * exceeds it, row_off is still filled and RRT_E_CAPACITY is returned. */
int rrt_get_hits(rrt_ctx* ctx, int64_t cap, int64_t* row_off, int32_t* hit_j,
                 int32_t* hit_img);

/* Accumulated device time (ms, HIP events on the context's stream) since the
 * last rrt_reset_timing, per phase, into host double out12[12]:
 *   [0] traversal + column launches      [1] rate + equilibrium
 *   [2] tree builds                      [3] number of traversal launches
 *   [4] path recording (count + record traversals)
 *   [5] columns from recorded paths      [6] number of those launches
 *   [7] intersections held in the recorded paths (-1 when none are valid)
 *   [8] columns from row tiles           [9] number of those launches
 *   [10] row-tile builds                 [11] distinct particles summed over
 *                                             the row tiles (-1 when none)
 * Timing is recorded only after rrt_enable_timing(ctx, 1): a pair of events
 * on the context's stream around each timed phase, resolved (and the stream
 * synchronised) by rrt_get_timing, so timing adds no synchronisation between
 * launches.  Phases of a batched solve replayed from a graph are not timed. */
int rrt_enable_timing(rrt_ctx* ctx, int32_t on);
int rrt_get_timing(rrt_ctx* ctx, double* out12);
int rrt_reset_timing(rrt_ctx* ctx);

/* Intersection counters (host): out2[0] = intersections of the last iteration
 * of rrt_iterate_equilibrium, out2[1] = intersections summed over every
 * iteration since the last rrt_reset_timing. */
int rrt_get_counters(rrt_ctx* ctx, int64_t* out2);

#ifdef __cplusplus
}
#endif
#endif /* RRT_H */
