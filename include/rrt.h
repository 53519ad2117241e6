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
 *  - Device memory: the library never allocates device memory.  Every device
 *    buffer of a context (particle arrays in tree order, tree, columns,
 *    reductions, scratch, the reverse mode's iterates) is carved from the
 *    workspace the caller gives with rrt_set_workspace, sized by
 *    rrt_workspace_size; the recorded ray paths, and what is derived from
 *    them, from the path buffer given with rrt_set_path_buffer, sized by
 *    rrt_count_paths.  A call that finds too little room returns
 *    RRT_E_WORKSPACE before it changes any state, and rrt_workspace_info
 *    says how much it asked for.  Both regions stay referenced until they are
 *    replaced or the context is destroyed.  (The one exception is
 *    rrt_get_hits_rows_noalloc, which stages in a fixed device array inside
 *    the library.)  Pinned host memory of a few bytes is allocated for
 *    reductions.
 *  - Work is enqueued on the stream given to rrt_create (NULL = the null
 *    stream).  Calls that return a scalar to the host synchronise that stream.
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
    RRT_E_WORKSPACE = -5,     /* no workspace or path buffer, or too little room */
    RRT_E_CAPACITY = -6       /* caller output buffer too small                */
};

typedef struct rrt_ctx rrt_ctx;

typedef struct {
    double l_ray;          /* ray length in kpc, >= 0 (Sec. 3.3: l_ray)              */
    double box;            /* periodic box side in kpc; 0 = isolated (no images)    */
    int32_t leaf_size;     /* max particles per tree leaf, 1..16 (0 = default 16)   */
    int32_t block_size;    /* threads per block of the traversal: 0 (= 128) or a
                              multiple of 64 up to 256                               */
    int32_t record_paths;  /* -1 = record when they fit in the path buffer
                              (default), 0 = traverse every iteration, 1 = require
                              recording (RRT_E_WORKSPACE when they do not fit)       */
    int32_t traversal;     /* 0 = wave-cooperative walk (default), 1 = one
                              independent walk per lane; identical results          */
    int32_t reserved[2];   /* must be zero                                           */
} rrt_params;

/* Ray paths.  The geometry of every ray (which particles it intersects and the
 * kernel chord factor K/h^2 of each) does not depend on x, because the column
 * is linear in the neutral fractions (Sec. 4.1.1, eq. colden).  With path
 * recording the first column evaluation after a tree build traverses the tree
 * and records 8 bytes per intersection (particle index and factor) into the
 * path buffer; every evaluation then forms N = sum (mu x)_j * factor_j by a
 * streaming product over the recorded paths.  Without it, every evaluation
 * traverses the tree.  Both give the same intersections and terms; the two
 * sums differ only in summation order.  The recording takes
 *   - one recording walk, when rrt_count_paths counted the current tree;
 *   - else, when the path buffer has room for the paths and a pool of chunks
 *     beside them (RRT_TUNE_ONE_PASS), one walk that appends each ray's
 *     entries to 32-entry chunks of the pool and counts them, and a copy of
 *     the chunks into rows; if the pool runs short, a second, recording walk
 *     with the counts the first one took;
 *   - else a counting walk and a recording walk. */

/* Library version as major*10000 + minor*100 + patch. */
int rrt_version(void);

/* Create a context on the current HIP device.  stream: a hipStream_t (may be
 * NULL).  *out receives the context; on failure *out is NULL.  Allocates no
 * device memory: give it a workspace before any call that needs one. */
int rrt_create(rrt_ctx** out, const rrt_params* params, void* stream);

/* Release the context.  The caller's workspace and path buffer are not freed
 * (the caller owns them); they are no longer referenced afterwards. Safe on
 * NULL. */
void rrt_destroy(rrt_ctx* ctx);

/* ---- device memory -----------------------------------------------------
 * The problem statement of the method (Sec. 4, implementation details: the
 * spectrum, N_ray, l_ray, the update criterion; the particle fields of
 * Sec. 4.1.1, eq. nhi) fixes what a context holds, so its fixed buffers are
 * known from the sizes alone. */

/* Bytes of workspace for a problem of n particles, n_ray rays, n_bins
 * frequency bins and n_halo independent halos (1 = one problem), under the
 * context's current scheme (rrt_set_scheme adds the near columns), plus the
 * reverse mode's buffers for K iterations (reverse_K = 0: none).  Includes
 * the largest scratch any call takes, except the staging of the inspection
 * calls' hit lists (rrt_get_hits: 8 bytes per ray plus 8 per intersection).
 * host size_t* bytes.  No device work. */
int rrt_workspace_size(const rrt_ctx* ctx, int64_t n, int32_t n_ray, int32_t n_bins,
                       int32_t n_halo, int32_t reverse_K, size_t* bytes);

/* Give the context its workspace: device memory of `bytes` bytes, 256-byte
 * aligned, owned by the caller, not overlapping the previous workspace or the
 * path buffer.  The context's buffers are carved from it.  When a workspace
 * was set before, every live buffer moves into the new one (a device copy;
 * synchronises the stream), so a context can grow its workspace at any time
 * without losing state; the old memory is no longer referenced when the call
 * returns.  RRT_E_WORKSPACE if the live buffers do not fit. */
int rrt_set_workspace(rrt_ctx* ctx, void* dev, size_t bytes);

/* Usage of the context's device memory, host size_t out[6]: workspace bytes
 * in use and its size, path-buffer bytes in use and its size, and the size
 * and region (0 = workspace, 1 = path buffer) of the last request that found
 * no room (0 and -1 if none). */
int rrt_workspace_info(const rrt_ctx* ctx, size_t* out6);

/* Recorded paths, first step: a counting walk over the current tree (Sec.
 * 4.1.1, eq. colden: which particles each ray intersects).  Host outputs,
 * each nullable: *n_hits, the intersections of every ray (each periodic
 * image separately); *bytes_paths, the path buffer the recorded paths need
 * (8 bytes per intersection and a little padding); *bytes_one_walk, the size
 * with which a later recording of a geometry with up to this many
 * intersections takes one walk (the paths and the chunk pool beside them).
 * The counts are kept, so the next column evaluation records with one walk.
 * Synchronises. */
int rrt_count_paths(rrt_ctx* ctx, int64_t* n_hits, size_t* bytes_paths, size_t* bytes_one_walk);

/* Recorded paths, second step: the device memory they are recorded into,
 * owned by the caller, 256-byte aligned (NULL and 0: none).  Besides the
 * paths, the library uses the rest of it for the one-walk chunk pool while
 * recording, and, room permitting, for the reverse mode's transposed paths
 * and kept columns and for row tiles; each of these is optional and has a
 * slower form that needs no memory.  Replacing the buffer drops the recorded
 * paths and everything in the old buffer (synchronises the stream first). */
int rrt_set_path_buffer(rrt_ctx* ctx, void* dev, size_t bytes);

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
 * thin state x_thin = x_-(Gamma_thin) (Sec. 4).  Copied into the workspace
 * (rrt_workspace_size with this n); validated by rrt_build_tree, which must
 * follow and returns RRT_E_INPUT for non-finite or out-of-range values
 * (x_init outside [0, 1] included).  1 <= n <= 2^27 (RRT_E_ARG otherwise). */
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
 * Ray k of source p meets particle j (and each periodic image s of it) when,
 * with d = (r_j - r_p) + s B, s_par = d.u, t = clamp(s_par, 0, l_ray) and
 * c = d - t u, |c|^2 < h_j^2 strictly; FP64, the two dot products as the x
 * product followed by fused multiply-adds of y and z, each component of c one
 * fused multiply-add, nothing else contracted, so the hit sets are exact.
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
 * Each ray's slab is lit by the ray's share, 1/n_ray of the far-attenuated
 * spectrum, and Gamma = sum_k Gamma_k (eq. gammashld with 4 pi inside w; the
 * weighting the paper's two-sided slab discussion of Sec. 5.3 implies).
 * Recorded paths are dropped when the scheme changes; the near columns take
 * 8 bytes per ray more workspace.  While the near/far scheme is set,
 * rrt_forward, rrt_backward, rrt_iterate_halos and update rules other than
 * the default return RRT_E_STATE.  0 (default): the plain scheme. */
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
 * convergence.  Synchronises once per sweep (64 bytes: the largest change,
 * intersections, the convergence counts of rrt_get_convergence and the input
 * flags) for the convergence test; the first call of rrt_set_update_rule's
 * density order also copies n_H to the host once.  RRT_E_INPUT when a given
 * state or density was out of range, or an update left a neutral fraction
 * outside [0, 1]. */
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
 * n_H device float[n] in input order, > 0 and finite; other values raise the
 * device flag of rrt_set_state (RRT_E_INPUT at the next synchronising call). */
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
 * (which records the ray paths when they fit in the path buffer; when the
 * whole batch's do not, the halos are solved in groups whose paths fit, after
 * one counting walk, which takes 8 more bytes per ray of workspace; a halo
 * too large alone traverses), the iterations run as replays
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
 *                         64, or 0 (default): a full sweep of the plain product
 *                         streams the path array by blocks of rows, and the
 *                         other products (near/far split, halos that stopped,
 *                         per-block source lists) take lanes per ray from the
 *                         mean intersections per ray
 *   RRT_TUNE_LEAF         particles per tree leaf (1..16), from the next build
 *   RRT_TUNE_ADJOINT      transposed column product of rrt_backward over
 *                         recorded paths: 0 (default) = gather over paths
 *                         transposed once per geometry when they fit in the
 *                         path buffer (32 bytes per intersection while they are
 *                         built; deterministic), else per row tile in LDS with one
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
 *                         columns for rrt_backward when they fit in the path
 *                         buffer beside the paths (8 n n_ray K bytes); 0:
 *                         rrt_backward recomputes them from the kept states.
 *                         The same columns either way.
 *   RRT_TUNE_ONE_PASS     1 (default): with the wave-cooperative walk,
 *                         record the paths in one walk that appends each
 *                         ray's entries to 32-entry chunks of a pool in the
 *                         path buffer and counts them, then copy the chunks
 *                         into rows; when the pool runs short, record in a
 *                         second walk as with 0.  The pool is sized from the
 *                         context's previous recording or count (so a
 *                         context's first recording takes two walks unless
 *                         rrt_count_paths ran): 5/4 of its entries plus half
 *                         a chunk per ray, in 1024 slices with a counter
 *                         each; after a recording that ran short, half as
 *                         large again (up to 4x).  It is used only when the
 *                         path buffer holds it beside the paths, and freed
 *                         once the paths are in rows.  0: a counting walk,
 *                         then a recording walk.  n > 1: one pass with a pool
 *                         of about n chunks, also on a first recording.  The
 *                         same paths either way.
 *   RRT_TUNE_PACKET_QUEUE 1 (default): the wave-cooperative walk runs as a
 *                         persistent grid of the blocks the device holds at
 *                         once, whose waves take packets (64 sources of one
 *                         direction, over every halo) from one global counter
 *                         until none is left; 0: one wave per packet, the
 *                         hardware scheduling them.  The same results either
 *                         way (measured on MI355X: the queue is 5% faster on
 *                         the 64-halo batch's column walk, 2-3% on the
 *                         recording walks of the field and the halo). */
enum { RRT_TUNE_TRACE_BLOCK = 1, RRT_TUNE_PACKET = 2, RRT_TUNE_PATH_GROUP = 3, RRT_TUNE_LEAF = 4,
       RRT_TUNE_ADJOINT = 5, RRT_TUNE_TILES = 6, RRT_TUNE_KEEP_COLUMNS = 7,
       RRT_TUNE_ONE_PASS = 8, RRT_TUNE_PACKET_QUEUE = 9 };
int rrt_set_tuning(rrt_ctx* ctx, int32_t key, int32_t value);

/* Replace the state: x device double[n] in input order (checkpoint / resume,
 * or a given iterate); NULL resets to x_thin.  Values outside [0, 1] (NaN
 * included) raise a device flag that the next call which synchronises
 * reports as RRT_E_INPUT (and clears). */
int rrt_set_state(rrt_ctx* ctx, const double* x);

/* Read the state: device outputs in input order, each nullable. */
int rrt_get_state(rrt_ctx* ctx, double* x_out, double* lnG_out, double* G_out,
                  float* tau_out);

/* Convergence history of the last rrt_iterate_equilibrium (Sec. 4: the paper
 * reports the fraction of particles whose neutral fraction has converged
 * after each iteration).  For sweep s < min(cap, sweeps): max_dx[s], the
 * largest change (relative when the update rule says so); n_abs[s] and
 * n_rel[s], the particles updated in that sweep whose change |dx| was below
 * the solve's tol, and whose |dx| / x_old was below tol (with tol = 0, a
 * fixed number of sweeps, below the paper's 1e-3).  Host outputs, each
 * nullable; *n_sweeps receives the number of sweeps. */
int rrt_get_convergence(rrt_ctx* ctx, int32_t cap, int32_t* n_sweeps, double* max_dx,
                        int64_t* n_abs, int64_t* n_rel);

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

/* Each halo's subtree (rrt_set_halos): nodes [root[h], end[h]) of the
 * depth-first layout hold exactly halo h's particles (host int32 outputs,
 * n_halo each; one problem: the whole tree). */
int rrt_get_halo_roots(rrt_ctx* ctx, int32_t* root, int32_t* end);

/* Hit lists of the rays of some sources, from the wave-cooperative walk the
 * column evaluations and the path recording run (Sec. 4.1.1, eq. colden:
 * which particles each ray intersects, and the kernel chord factor of each).
 * src: host int64[n_src] input indices of distinct source particles, 1 <=
 * n_src <= 4096.  Host outputs: row_off int64[n_src * n_ray + 1], the hits of
 * ray k of source src[i] are entries row_off[i*n_ray+k] ..
 * row_off[i*n_ray+k+1]) of hit_j (input index of the particle), hit_img (its
 * periodic image, coded as in rrt_get_hits) and hit_fac (K/h^2 in kpc^-2,
 * FP32; nullable).  cap: capacity of the entry arrays; with too little
 * capacity (or null hit_j), row_off is filled and RRT_E_CAPACITY returned
 * (RRT_OK for null arrays).  Staging comes from the workspace (12 bytes per
 * hit plus 8 per ray).  Synchronises. */
int rrt_get_hits_rows(rrt_ctx* ctx, int32_t n_src, const int64_t* src, int64_t cap,
                      int64_t* row_off, int32_t* hit_j, int32_t* hit_img, float* hit_fac);

/* rrt_get_hits_rows for callers that cannot allocate, or grow the workspace,
 * at that point (under graph capture, in serving loops, under harnesses that
 * forbid allocation): the same arguments and results, with the device
 * staging in a fixed array inside the library (about 25 MiB, one per GPU,
 * held until the process ends) instead of the workspace.  At most 1024
 * sources, 65536 rays and 2^21 hits per call (RRT_E_CAPACITY beyond).  Calls
 * on one GPU share the array: calls that overlap on one GPU race. */
int rrt_get_hits_rows_noalloc(rrt_ctx* ctx, int32_t n_src, const int64_t* src, int64_t cap,
                              int64_t* row_off, int32_t* hit_j, int32_t* hit_img,
                              float* hit_fac);

/* The recorded paths of the rays of some sources, as the streaming product
 * sums them: same arguments and layout as rrt_get_hits_rows, with hit_j the
 * input index of each recorded particle and hit_fac its factor.  The order
 * within a ray is the order of the walk.  RRT_E_STATE when no paths are
 * recorded.  Synchronises. */
int rrt_get_path_rows(rrt_ctx* ctx, int32_t n_src, const int64_t* src, int64_t cap,
                      int64_t* row_off, int32_t* hit_j, float* hit_fac);

/* Hit lists for the current geometry (host outputs): the intersections of ray
 * (p, k) are hit_j[row_off[p*n_ray+k] .. row_off[p*n_ray+k+1]) as input
 * particle indices, with the periodic image of each in hit_img as
 * (sx+8) | (sy+8)<<4 | (sz+8)<<8 (the image of particle j sits at r_j + s*box).
 * row_off: int64[n*n_ray + 1].  cap: capacity of hit_j/hit_img; with null
 * hit_j or hit_img only row_off is filled (RRT_OK); if the total exceeds cap,
 * row_off is still filled and RRT_E_CAPACITY is returned.
 * Staging comes from the workspace: 8 bytes per ray, plus 8 per intersection
 * when the lists are written. */
int rrt_get_hits(rrt_ctx* ctx, int64_t cap, int64_t* row_off, int32_t* hit_j,
                 int32_t* hit_img);

/* Accumulated device time (ms, HIP events on the context's stream) since the
 * last rrt_reset_timing, per phase, into host double out[n_out] (up to
 * RRT_N_TIMING entries):
 *   [0] traversal + column launches      [1] rate + equilibrium
 *   [2] tree builds                      [3] number of traversal launches
 *   [4] path recording (count + record traversals)
 *   [5] columns from recorded paths      [6] number of those launches
 *   [7] intersections held in the recorded paths (-1 when none are valid)
 *   [8] columns from row tiles           [9] number of those launches
 *   [10] row-tile builds                 [11] distinct particles summed over
 *                                             the row tiles (-1 when none)
 *   [12] one-walk chunk walks (inside [4])  [13] number of those walks
 *   [14] chunk compaction (inside [4])   [15] counting and recording walks
 *                                             (inside [4])
 * Timing is recorded only after rrt_enable_timing(ctx, 1): a pair of events
 * on the context's stream around each timed phase, resolved (and the stream
 * synchronised) by rrt_get_timing, so timing adds no synchronisation between
 * launches.  Phases of a batched solve replayed from a graph are not timed. */
enum { RRT_N_TIMING = 16 };
int rrt_enable_timing(rrt_ctx* ctx, int32_t on);
int rrt_get_timing(rrt_ctx* ctx, double* out, int32_t n_out);
int rrt_reset_timing(rrt_ctx* ctx);

/* Intersection counters (host): out2[0] = intersections of the last iteration
 * of rrt_iterate_equilibrium, out2[1] = intersections summed over every
 * iteration since the last rrt_reset_timing. */
int rrt_get_counters(rrt_ctx* ctx, int64_t* out2);

/* Path recordings since rrt_create, host int64 out[n_out] (up to
 * RRT_N_REC_STATS entries): [0] in one walk into the chunk pool, [1] one walk
 * whose pool ran short, finished by a second, recording walk, [2] one
 * recording walk after rrt_count_paths, [3] a counting and a recording walk,
 * [4] recordings that did not fit the path buffer (traversal instead). */
enum { RRT_N_REC_STATS = 5 };
int rrt_get_recording_stats(rrt_ctx* ctx, int64_t* out, int32_t n_out);

/* The work of the walk (diagnostics): one counting pass of the
 * wave-cooperative walk over every ray of the current tree that also tallies
 * host int64 out6 = [rays, node visits of the 64-ray packets, node visits of
 * single rays (box tests passed), leaf visits of the packets, particle pair
 * tests, intersections].  Synchronises. */
int rrt_trace_stats(rrt_ctx* ctx, int64_t* out6);

#ifdef __cplusplus
}
#endif
#endif /* RRT_H */
