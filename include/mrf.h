/*
 * mrf.h -- C ABI of the MI355X ray-MRF belief-propagation library (libmrf.so).
 *
 * The library infers per-voxel occupancy marginals from depth images with the
 * ray Markov random field of MRFMap (Shankar & Michael, arXiv 2006.03512):
 * binary occupancy o_v per voxel with a Bernoulli prior factor
 * (Sec. III-A, Eq. prior_potential), one ray depth potential per depth pixel
 * that rewards the first occupied voxel along the ray with the forward sensor
 * model nu(d) = N(Z; d, sigma(d)) (Eqs. depth_potential, noise), and loopy
 * sum-product belief propagation (Sec. III-B) with the linear-time ray
 * messages of Eqs. pos and neg.  A reverse pass (not in the paper) gives the
 * gradient of any loss of the marginal log-odds with respect to the per-voxel
 * prior log-odds and the 64-bin sigma table (and the 64-bin depth-bias table of
 * the sensor model, Sec. IV-C).  mrf_accuracy evaluates a map with the
 * accuracy metric of Sec. III-D.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns MRF_OK (0) or a negative MRF_E* code; no C++ exception
 *   crosses this boundary.  mrf_strerror() names a code; mrf_last_error()
 *   gives the message of the last failure on the calling thread.
 * - All array arguments are DEVICE pointers (hipMalloc'ed or torch CUDA
 *   tensors on the current device) unless stated otherwise.  The caller owns
 *   them and keeps them valid until the call's work on `stream` completes.
 *   The context owns everything it allocates; mrf_destroy frees it.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Calls enqueue work asynchronously on it; the only host synchronisation is
 *   inside mrf_build (it reads the edge count back to size its buffers).
 * - A context is not thread-safe: use one context per host thread.
 * - Ray r of scene s is global ray ray_base(s) + (f H + v) W + u (frame f,
 *   pixel row v, column u).  Voxel (i, j, k) of scene s is global voxel
 *   voxel_base(s) + i + nx (j + ny k).  Scenes are concatenated in call order.
 * - Edge = one (ray, voxel) incidence, numbered by ray then by distance along
 *   the ray (the order the 3D-DDA visits voxels).
 */
#ifndef MRF_H
#define MRF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MRF_OK = 0,
    MRF_EINVAL = -1,   /* bad argument: null pointer, bad shape or parameter */
    MRF_ENOMEM = -2,   /* device allocation failed */
    MRF_EHIP = -3,     /* a HIP runtime call failed */
    MRF_ESTATE = -4,   /* call out of order (e.g. backward without checkpoints) */
    MRF_ERANGE = -5    /* a size exceeds an index type (E >= 2^32, ray > 2048 voxels) */
};

typedef struct mrf_ctx mrf_ctx;

/* Pinhole camera: pixel (u, v) looks along R ((u - cx)/fx, (v - cy)/fy, 1),
 * so the ray parameter is z-depth (Sec. III: one distance per ray). */
typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
} mrf_intrinsics;

/* Dense voxel grid: voxel (i, j, k) covers [o + i h, o + (i+1) h) x ... */
typedef struct {
    int32_t nx, ny, nz, reserved;
    double voxel;
    double origin[3];
} mrf_grid;

/* One scene: n_frames depth images of one camera model into one grid. */
typedef struct {
    int32_t n_frames, reserved;
    const float* depth;     /* host or device, n_frames*H*W z-depth [m]; 0 or NaN = no return */
    const double* T_wc;     /* host or device, n_frames*16 row-major camera->world (OpenCV axes) */
    mrf_intrinsics K;
    mrf_grid grid;
} mrf_scene;

/* Graph construction parameters (Sec. IV-B: rays stop 3 sigma past the
 * measured depth).  A pixel is used iff z_min <= Z <= z_max and Z lies inside
 * the grid; its ray is walked from the grid entry to
 * min(Z + trunc_nsigma * sigma_tr(Z), grid exit) with
 * sigma_tr(Z) = max(trunc_c0 + trunc_c2 Z^2, trunc_min), frozen at build so
 * the incidence never depends on learnable parameters.  Rays that cross fewer
 * than min_ray_voxels voxels (>= 2, since a one-voxel ray factor forces its
 * voxel occupied with infinite log-odds) are dropped.  The sigma table has 64
 * bins of width table_dmax/64 indexed by the voxel's depth.
 * Sparse grid (Sec. IV-B: storage only in 8^3-voxel bricks allocated around
 * the reprojected depth points, rays skip the rest): with sparse_bricks != 0
 * a brick (voxels [8b, 8b + 8) per axis from the grid origin) is allocated
 * iff the measured point c + Z w of a usable pixel of any frame of the scene
 * lies in a grid voxel whose brick is within brick_radius bricks of it on
 * every axis; a ray then keeps only its voxels in allocated bricks (same
 * chords), and min_ray_voxels applies to those.  Voxels of other bricks take
 * part in no ray factor and keep their prior.  With skip_empty_bricks the
 * traversal steps over unallocated bricks a brick at a time (the rays skip
 * empty space) instead of voxel by voxel; the incidence is identical bit for
 * bit either way, and which is faster depends on the scene (the voxel walk
 * keeps the lanes of a wave in step).
 * Per-keyframe averaged messages (Sec. IV-A): with keyframe_average != 0 the
 * build also prepares mrf_infer_keyframe_avg: every frame is a keyframe, and
 * each (keyframe, voxel) pair crossed by at least one of the keyframe's rays
 * gets the chord-length weights of its rays and one slot in a per-keyframe
 * message buffer (4 bytes per voxel of the frame's scene and frame, plus
 * 4 bytes per edge and 12 per pair). */
typedef struct {
    double z_min, z_max;
    double trunc_nsigma, trunc_c0, trunc_c2, trunc_min;
    double table_dmax;
    int32_t min_ray_voxels;
    int32_t keep_chords;    /* nonzero: keep f64 chord entry/exit per edge for export */
    int32_t sparse_bricks;  /* nonzero: sparse grid (Sec. IV-B), see below; 0: dense */
    int32_t brick_radius;   /* sparse grid: bricks allocated around a point's brick, 0..64 */
    int32_t keyframe_average;  /* nonzero: prepare per-keyframe averaged messages (Sec. IV-A) */
    int32_t skip_empty_bricks; /* sparse grid: nonzero steps over unallocated bricks brick by brick */
    int32_t reserve_frames;    /* >= 0: buffers sized for this many more frames of the last scene
                                  (mrf_add_frames), per-edge ones at 1.25 times the batch's mean
                                  edge slots per frame */
    int32_t group_slots_log2;  /* 0 (= 32) or 12..32: a group of scenes holds fewer than 2^this
                                  edge slots (see below); smaller values only for testing */
} mrf_build_params;

typedef struct {
    int64_t n_scenes, n_rays, n_edges, n_voxels;
    int64_t n_kept_rays, n_touched_voxels, max_ray_len, max_voxel_degree;
    int64_t ray_len_hist[16];       /* rays with length in [2^i, 2^(i+1)) */
    int64_t voxel_degree_hist[24];  /* touched voxels with degree in [2^i, 2^(i+1)) */
    double fwd_bytes_per_sweep;     /* algorithmic HBM bytes of one forward sweep */
    int32_t sweeps_done, have_checkpoints;
    int64_t n_slots;                /* edge slots in memory: edges plus tile padding */
    int64_t n_tiles;                /* 4x4-pixel ray tiles */
    int64_t n_keyframe_pairs;       /* (keyframe, voxel) pairs (builds with keyframe_average) */
    int64_t n_slot_groups;          /* groups of scenes under 2^32 edge slots each (see mrf_build) */
} mrf_stats_t;

/* Create an empty context on the current HIP device.  *out receives it. */
int mrf_create(mrf_ctx** out);

/* Build (or rebuild, reusing buffers when they are large enough) the ray MRF
 * of n_scenes scenes: 3D-DDA traversal of every kept ray (Amanatides-Woo, the
 * traversal named in Sec. IV-A), ray->voxel CSR in edge order, voxel->ray CSR
 * by a stable device radix sort (edges ascending inside a voxel), per-edge
 * voxel depth (chord midpoint) and sigma-table bin.  Depth and pose arrays
 * may be device memory or host memory (queried with hipPointerGetAttributes):
 * device arrays and pinned, mapped host arrays are read in place and must stay
 * valid while the build is in use (mrf_accuracy and rebuilds read them);
 * pageable host arrays are copied into the context, which keeps the copies
 * until the next mrf_build, and need only stay valid until the call returns.
 * Edge slots (edges plus tile padding) and list positions are 64-bit; the
 * voxel -> ray lists hold 32-bit slot ids relative to a group of whole
 * scenes: the scenes in order form groups of fewer than 2^32 slots each (at
 * most 8 groups), so a batch may hold more than 2^32 slots while every scene
 * holds fewer (mrf_stats reports the groups).  Errors: MRF_EINVAL (bad shapes,
 * min_ray_voxels < 2, more than 65535 frames), MRF_ERANGE (a scene of 2^32 or
 * more edge slots, more than 8 groups, a ray longer than 2048 voxels; with
 * keyframe_average, 2^32 or more slots in the batch or per-keyframe message
 * buffers of 2^32 or more entries), MRF_ENOMEM, MRF_EHIP. */
int mrf_build(mrf_ctx* ctx, const mrf_scene* scenes, int32_t n_scenes,
              const mrf_build_params* params, void* stream);

/* Add keyframes to the last scene of the built batch (Sec. V: the online use
 * adds an image, then re-infers every keyframe): the result is the graph
 * mrf_build makes with these frames appended to that scene, bit for bit
 * (same ray ids, slots and voxel -> ray lists), but only the new frames are
 * traversed and sorted; their entries are merged behind each voxel's existing
 * ones.  depth: n_frames * H * W floats and T_wc: n_frames * 16 doubles
 * (host or device, as in mrf_build), the last scene's camera model.  The last inference is
 * discarded.  Errors: MRF_ESTATE before mrf_build, MRF_EINVAL for a sparse grid
 * (its bricks depend on every frame: rebuild) or more than 65535 frames,
 * MRF_ERANGE, MRF_ENOMEM, MRF_EHIP. */
int mrf_add_frames(mrf_ctx* ctx, int32_t n_frames, const float* depth, const double* T_wc, void* stream);

/* The count pass of mrf_build alone (the traversal of Sec. IV-A counts each
 * ray's voxels; no incidence, potentials or message arrays are made): for
 * every frame of the batch, scenes in order and their frames in order, the
 * edge slots it would occupy (edges plus the padding of its 4 x 4 tiles:
 * per-edge memory is proportional to slots) and its edges.  frame_slots and
 * frame_edges are host arrays of the batch's total frame count (either may be
 * NULL, not both).  A caller sizes a batch to its memory with it before
 * building.  Arguments and errors as mrf_build; the context is left without a
 * graph (mrf_infer needs a new mrf_build). */
int mrf_count(mrf_ctx* ctx, const mrf_scene* scenes, int32_t n_scenes, const mrf_build_params* params,
              int64_t* frame_slots, int64_t* frame_edges, void* stream);

/* Run `sweeps` flooding sweeps of loopy sum-product BP (Sec. III-B/C, IV-A)
 * from uniform ray messages.  One sweep sends every voxel->ray message
 * (Eq. node_to_factor: the prior times every other ray's message, formed as
 * the voxel's total log-odds less the receiving ray's own message) and then
 * every ray->voxel message (Eqs. pos and neg, computed in the log domain
 * with prefix products of mu(o=0) and the division-free suffix form of
 * Eq. neg).  prior_logit: V floats, log(gamma_v / (1 - gamma_v)) per voxel
 * (copied).  sigma_table: 64 floats > 0, the learnt depth-indexed Gaussian
 * sigma of Eq. noise (copied); after mrf_set_sensor_cells with cell_px > 0,
 * 64 floats per pixel region (n_cells rows).  keep_checkpoints != 0 stores, for
 * mrf_backward, the ray->voxel messages of sweeps 1..K-1 ((sweeps - 1) * E
 * floats) and the voxel totals of sweeps 2..K ((sweeps - 1) * V FP32 pairs),
 * which together give every sweep's voxel->ray messages.  Errors: MRF_ESTATE
 * before mrf_build, MRF_EINVAL for sweeps < 1, MRF_ENOMEM. */
int mrf_infer(mrf_ctx* ctx, const float* prior_logit, const float* sigma_table,
              int32_t sweeps, int32_t keep_checkpoints, void* stream);

/* mrf_infer with the learnt sensor bias of Sec. IV-C: the bias b(d) at a
 * traversed depth d gives the predicted mean measurement d + b(d), so the
 * forward sensor model of Eq. noise becomes nu = N(Z; d + b(d), sigma(d)).
 * bias_table: 64 floats [m] on the same depth bins as sigma_table (device,
 * copied; one row per pixel region like sigma_table), or NULL for b = 0, which is mrf_infer exactly.  The incidence
 * (truncation of every ray 3 sigma past its measurement) is fixed at build
 * and does not depend on either table.  Errors as mrf_infer. */
int mrf_infer_sensor(mrf_ctx* ctx, const float* prior_logit, const float* sigma_table,
                     const float* bias_table, int32_t sweeps, int32_t keep_checkpoints,
                     void* stream);

/* Loopy BP with the memory approximation of Sec. IV-A: the rays of one
 * keyframe that cross a voxel are taken to send it the same message, their
 * average weighted by the length each ray travels in the voxel (Euclidean
 * chord length), so a voxel's belief is theta_v plus ONE averaged message per
 * keyframe, and the voxel -> ray message into a ray of keyframe f is theta_v
 * plus the averages of the OTHER keyframes (the receiving ray's keyframe is
 * left out as a whole, as Eq. node_to_factor leaves out the receiving
 * factor).  Ray -> voxel messages are Eqs. pos and neg as in mrf_infer, and
 * ray messages start uniform, so the first sweep's voxel -> ray message is
 * theta.  After K sweeps mrf_marginals returns theta plus every keyframe's
 * average of the last sweep; mrf_export_edges gives the last sweep's messages.
 * Averages are FP64 sums of weight * message in a fixed order; each
 * keyframe's message is one FP32 rounding of its FP64 value.  Tables and
 * arguments as mrf_infer_sensor (bias_table may be NULL).  keep_checkpoints
 * != 0 keeps the pair averages of sweeps 2..K ((sweeps - 1) * n_keyframe_pairs
 * doubles, instead of the per-edge messages mrf_infer keeps), from which
 * mrf_backward* rebuild every sweep's keyframe messages: the reverse pass then
 * differentiates this scheme (the derivative reaching a pair's average is
 * shared by its edges in proportion to their weights).  Errors: MRF_ESTATE
 * before mrf_build or when the build did not set keyframe_average,
 * MRF_EINVAL for sweeps < 1, MRF_ENOMEM. */
int mrf_infer_keyframe_avg(mrf_ctx* ctx, const float* prior_logit, const float* sigma_table,
                           const float* bias_table, int32_t sweeps, int32_t keep_checkpoints, void* stream);

/* Marginals of the last mrf_infer (Sec. III-B: normalised product of all
 * factor messages into the voxel): logit_v = theta_v + sum of ray messages,
 * p_v = sigmoid(logit_v).  Either output may be NULL.  V floats each.
 * Errors: MRF_ESTATE before mrf_infer. */
int mrf_marginals(mrf_ctx* ctx, float* p, float* logit, void* stream);

/* Reverse pass through the K sweeps of the last mrf_infer, mrf_infer_sensor or
 * mrf_infer_keyframe_avg (which must have kept checkpoints).  dloss_dlogit: V floats, the gradient with respect to
 * the marginal log-odds (for BCE with logits: (p - y) / V).  Outputs
 * dprior_logit (V floats) and dsigma_table (the sigma table's size: 64
 * floats, or 64 per pixel region); either may be NULL.
 * Deterministic: no floating-point atomics.  Errors: MRF_ESTATE. */
int mrf_backward(mrf_ctx* ctx, const float* dloss_dlogit, float* dprior_logit,
                 float* dsigma_table, void* stream);

/* mrf_backward that also returns dbias_table (the bias table's size, device;
 * may be NULL), the gradient with respect to the bias table of the last inference
 * (zero table after plain mrf_infer).  With r = Z - d - b the residual about
 * the predicted mean, d g / d b = r / sigma^2 and d g / d sigma = r^2 / sigma^3
 * - 1 / sigma, g = log nu.  Deterministic like mrf_backward; dprior_logit and
 * dsigma_table are bit-identical to mrf_backward's.  Errors: MRF_ESTATE. */
int mrf_backward_sensor(mrf_ctx* ctx, const float* dloss_dlogit, float* dprior_logit,
                        float* dsigma_table, float* dbias_table, void* stream);

/* Generation of the context's last inference: a counter that every
 * successful mrf_infer / mrf_infer_sensor increments and every mrf_build
 * increments too (a build discards the inference).  A caller that keeps
 * results of one inference for a later reverse pass (an autograd node)
 * records it and passes it to mrf_backward_gen.  Errors: MRF_EINVAL. */
int mrf_generation(const mrf_ctx* ctx, uint64_t* out);

/* mrf_backward_sensor for the inference of the given generation: returns
 * MRF_ESTATE, with nothing enqueued, when the context's last inference is not
 * that one (a later mrf_infer or mrf_build replaced its checkpoints), instead
 * of differentiating the later inference.  dbias_table may be NULL.
 * Errors: as mrf_backward_sensor, and MRF_ESTATE on a generation mismatch. */
int mrf_backward_gen(mrf_ctx* ctx, uint64_t generation, const float* dloss_dlogit, float* dprior_logit,
                     float* dsigma_table, float* dbias_table, void* stream);

/* The accuracy metric of Sec. III-D for a map: every pixel of the scenes of
 * the last mrf_build with a usable measurement (z_min <= Z <= z_max) whose ray
 * meets the grid is walked through the whole grid (3D-DDA, no truncation).
 * A voxel is a region of constant occlusion density alpha = -ln(1 - p) / h
 * (= softplus(logit) / h: crossing one voxel side blocks the ray with the
 * voxel's occupancy probability p); along the ray vis(s) = exp(-integral of
 * alpha ds) and the generating surface has density omega = alpha vis, largest
 * at the entry of the voxel maximising alpha_n vis_n (the first on ties).
 * The ray is accurate iff its measurement lies in that voxel's chord, or, when
 * the visibility at the grid exit is still at least vis_min (the map does not
 * block the ray enough), iff the measurement lies beyond the exit.  All of it
 * in FP64.
 *   logit: V floats, the map's log-odds (NULL: the last mrf_infer's marginals).
 *   vis_min: in (0, 1] (0.5: the surface is more likely beyond the map).
 *   ray_code: R int8 (ray id as in mrf_build: frame-major, then row-major
 *     pixels), 1 accurate, 0 not, -1 not evaluated; may be NULL.
 *   surface_depth: R doubles, z-depth of the chosen voxel's entry, +inf for a
 *     surface beyond the map, NaN if not evaluated; may be NULL.
 *   counts: 2 int64 per scene (evaluated rays, accurate rays); may be NULL.
 * Reads the depth images and poses passed to mrf_build, which must still be
 * valid.  Allocates 16 V bytes of scratch in the context on first use.
 * Errors: MRF_ESTATE (before mrf_build, or logit NULL before mrf_infer),
 * MRF_EINVAL (vis_min out of range). */
int mrf_accuracy(mrf_ctx* ctx, const float* logit, double vis_min, int8_t* ray_code,
                 double* surface_depth, int64_t* counts, void* stream);

/* mrf_accuracy with the paper's evaluation options (Sec. V).  ref_depth: R
 * floats (device, ray order as in mrf_build), the image each ray is scored
 * against instead of its measurement, e.g. noise-free depth rendered from the
 * same poses or a held-out image (0 or NaN: not evaluated); NULL scores
 * against the measurements.  tol_nsigma > 0: a ray whose map does not leave
 * it visible is accurate iff the most likely generating surface (the chosen
 * voxel's entry, z-depth) lies within tol_nsigma sigma(Z) of the depth Z it is
 * scored against, sigma(Z) = max(trunc_c0 + trunc_c2 Z^2, trunc_min) the
 * build's sensor noise (the paper uses 1.5); 0 keeps the voxel-chord rule of
 * mrf_accuracy.  The beyond-the-map rule is unchanged.  Outputs and errors as
 * mrf_accuracy, and MRF_EINVAL for a negative tol_nsigma. */
int mrf_accuracy_ex(mrf_ctx* ctx, const float* logit, double vis_min, const float* ref_depth,
                    double tol_nsigma, int8_t* ray_code, double* surface_depth, int64_t* counts,
                    void* stream);

/* The ray factors' messages to their depth variables (Eq. depth_message,
 * Sec. III-C) after the last inference: the measurement of ray r came from
 * the depth of its i-th voxel with weight nu(d_i) mu(o_i = 1) prod_{k<i}
 * mu(o_k = 0), mu the voxel -> ray messages of the last sweep (of
 * mrf_infer, or the keyframe messages of mrf_infer_keyframe_avg), normalised
 * over the ray's voxels (the all-empty configuration has potential zero).
 *   prob: E floats in canonical edge order (as mrf_export_edges), the
 *     probability of each voxel's depth; may be NULL.
 *   mode_step: R int32, the step (0-based along the ray) of the most probable
 *     depth, the first on ties, -1 for rays without voxels; may be NULL.
 *   mean_depth: R floats, the expected z-depth sum_i prob_i d_i (chord
 *     midpoints), NaN for rays without voxels; may be NULL.
 * Weights are formed in base-2 logs with the visibility summed in FP64.
 * Errors: MRF_ESTATE before an inference. */
int mrf_depth_distribution(mrf_ctx* ctx, float* prob, int32_t* mode_step, float* mean_depth,
                           void* stream);

/* mrf_accuracy for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same computation and outputs, bit for bit, but the 16 V bytes of per-voxel
 * scratch come from a device array inside the library (one per GPU, held
 * until the process ends) instead of a context allocation; the call makes no
 * allocation.  Limit: V <= 2^21 = 2,097,152 voxels over the built scenes, else
 * MRF_ERANGE with nothing enqueued.  Every call on one GPU shares that GPU's
 * array (every entry read is written first in the same call): calls that
 * overlap on one GPU (other streams, other threads, other contexts) race.
 * Errors: as mrf_accuracy, MRF_ERANGE, MRF_EHIP if the array could not be
 * located on this device. */
int mrf_accuracy_static(mrf_ctx* ctx, const float* logit, double vis_min, int8_t* ray_code,
                        double* surface_depth, int64_t* counts, void* stream);

/* Sizes and histograms of the built graph (host struct). */
int mrf_stats(const mrf_ctx* ctx, mrf_stats_t* out);

/* Copy the incidence out in canonical order (for parity checks): edge id
 * = row_ptr[ray] + step along the ray, voxel id = linear id.  row_ptr (R+1
 * int64), col (E int32 voxel ids), t_in / t_out (E f64 chord entry/exit
 * z-depths; only if built with keep_chords, else must be NULL), vptr (V+1
 * int64), vedge (E uint32 edge ids ascending inside each voxel).  Any pointer
 * may be NULL.  The library stores edges in its own tiled order; producing
 * the canonical vedge re-sorts on the device and allocates 20 E bytes of
 * temporaries kept by the context. */
int mrf_export_incidence(const mrf_ctx* ctx, int64_t* row_ptr, int32_t* col,
                         double* t_in, double* t_out, int64_t* vptr, uint32_t* vedge,
                         void* stream);

/* Copy per-edge data out in canonical edge order: delta = Z - d (f32),
 * bin (u8), g = log nu (f32), lam = last voxel->ray log-odds, ell = last
 * ray->voxel log-odds (f32).  Any pointer may be NULL. */
int mrf_export_edges(const mrf_ctx* ctx, float* delta, uint8_t* bin, float* g,
                     float* lam, float* ell, void* stream);

/* Execution schedule of the sweeps:
 *   MRF_SCHED_PLAIN  eager launches, no graph: one launch per phase and ray
 *                    class, per frame for the ray phase, every ray class
 *                    with the fixed untuned shape of one 64-lane wave per
 *                    ray (16 lanes for rays of at most 16 voxels);
 *   MRF_SCHED_GRAPH  all sweeps captured once into a hipGraph and replayed
 *                    (default), with tuned launch shapes. */
enum { MRF_SCHED_PLAIN = 0, MRF_SCHED_GRAPH = 1 };
int mrf_set_schedule(mrf_ctx* ctx, int32_t schedule);

/* Per-pixel-region sensor tables (Sec. IV-C learns bias and noise for every
 * 20 x 20 pixel neighbourhood and depth).  cell_px = 0 (the default): one
 * 64-bin sigma table and one bias table serve every pixel.  cell_px > 0, a
 * multiple of 4 (a 4 x 4 ray tile then lies in one region): the tables of
 * mrf_infer, mrf_infer_sensor and mrf_infer_keyframe_avg, and the gradients of
 * mrf_backward*, hold n_cells rows of 64 bins, row-major; pixel (u, v) of a
 * W-wide image uses row (v / cell_px) * ceil(W / cell_px) + u / cell_px, and
 * n_cells is the largest ceil(W / cell_px) * ceil(H / cell_px) over the built
 * scenes (rows past a smaller image's regions are unused).  The setting stays
 * across rebuilds; changing it discards the last inference.  *n_cells (may be
 * NULL) receives the rows for the built scenes, 0 before a build.  The
 * accuracy metric and the traversal's truncation use the build's analytic
 * sigma and do not read the tables.  Errors: MRF_EINVAL for a negative
 * cell_px or one that is not a multiple of 4, MRF_ERANGE when the tables
 * would exceed 2^31 entries. */
int mrf_set_sensor_cells(mrf_ctx* ctx, int32_t cell_px, int64_t* n_cells);

/* The current region size (0: one table) and table rows (0 before a build);
 * either pointer may be NULL. */
int mrf_sensor_cells(const mrf_ctx* ctx, int32_t* cell_px, int64_t* n_cells);

/* Diagnostic timing of the sweep kernels (not part of the method).  Runs
 * `reps` eager forward sweeps (voxel phase, then ray phase) on the messages
 * of the last mrf_infer, and with include_backward != 0 also `reps` reverse
 * sweeps, recording a HIP event pair around every kernel launch on `stream`
 * (the stream the kernels run on).  Writes only scratch buffers that
 * mrf_backward initialises, so the last inference (messages, checkpoints,
 * marginals) is kept.  Writes up to max_out entries, one per kernel that ran, and
 * the count to *n_out.  bytes_per_launch is the kernel's algorithmic HBM
 * traffic per launch (each per-edge and per-item array read or written once).
 * Errors: MRF_ESTATE before mrf_infer. */
typedef struct {
    char name[40];
    int32_t launches;
    int32_t reserved;
    double total_ms;
    double bytes_per_launch;
    int64_t edges_per_launch;
} mrf_kernel_time_t;
int mrf_profile_sweeps(mrf_ctx* ctx, int32_t reps, int32_t include_backward,
                       mrf_kernel_time_t* out, int32_t max_out, int32_t* n_out, void* stream);

/* Launch shapes of the ray-length classes (the ray-segment length and the
 * lanes per ray the ray kernels use).  Rays are grouped in 4x4-pixel
 * tiles and tiles in classes by their longest ray (cap[q] steps).  A class
 * has fwd_candidates shapes for the ray phase (Eqs. pos and neg) and
 * adj_candidates for the reverse pass; a shape is the lanes per ray (16, 32 or
 * 64; steps per lane = cap / lanes) and, in the reverse pass, the rays a lane
 * group walks in turn (1 or 2).  *_sel is the selected candidate, 0 the
 * built-in default.  MRF_MAX_RAY_CLASSES bounds n_classes. */
#define MRF_MAX_RAY_CLASSES 32
typedef struct {
    int32_t n_classes;
    int32_t cap[MRF_MAX_RAY_CLASSES];
    int32_t fwd_candidates[MRF_MAX_RAY_CLASSES], fwd_sel[MRF_MAX_RAY_CLASSES], fwd_lanes[MRF_MAX_RAY_CLASSES];
    int32_t adj_candidates[MRF_MAX_RAY_CLASSES], adj_sel[MRF_MAX_RAY_CLASSES], adj_lanes[MRF_MAX_RAY_CLASSES];
    int32_t adj_rays[MRF_MAX_RAY_CLASSES];
} mrf_tuning_t;

/* Current launch shapes (host struct).  Errors: MRF_EINVAL for NULL. */
int mrf_get_tuning(const mrf_ctx* ctx, mrf_tuning_t* out);

/* Select launch shapes: fwd_sel / adj_sel hold n_classes candidate indices
 * (host arrays); NULL leaves that pass unchanged.  Every shape computes the
 * same messages up to FP32 rounding order.  Errors: MRF_EINVAL for an index
 * out of range (nothing changed). */
int mrf_set_tuning(mrf_ctx* ctx, const int32_t* fwd_sel, const int32_t* adj_sel);

/* Autotuner: time every candidate shape of every populated class on the
 * built graph (one warm-up and reps timed launches per candidate, HIP events
 * on `stream`) and select the fastest per class and pass.  Needs a preceding
 * mrf_infer (it reads the last sweep's messages; it writes only buffers that
 * mrf_backward initialises, so marginals and checkpoints are kept).
 * Synchronises `stream`.  Errors: MRF_EINVAL (reps < 1), MRF_ESTATE, MRF_EHIP. */
int mrf_autotune(mrf_ctx* ctx, int32_t reps, void* stream);

void mrf_destroy(mrf_ctx* ctx);
const char* mrf_strerror(int code);
const char* mrf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MRF_H */
