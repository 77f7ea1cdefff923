/*
 * FP64 CPU oracle for ray-MRF loopy sum-product belief propagation
 * (MRFMap, Shankar & Michael, arXiv 2006.03512).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  It shares no code,
 * header, table or constant generator with the HIP library; it is written from
 * the paper's equations in the paper's order, with plain sequential loops in
 * double precision and OpenMP only across independent rays or voxels (every
 * output has exactly one writer and every sum runs in fixed CSR order, so the
 * result does not depend on the thread count).
 *
 * Pieces, each with the passage it follows:
 *   or_trace_count / or_trace_emit  -- the ray of each depth pixel clipped to
 *       the grid and truncated 3 sigma past the measurement (Sec. IV-B), walked
 *       voxel by voxel with the 3D-DDA of Amanatides and Woo (Sec. IV-A).
 *   or_brick_mask                   -- sparse grid (Sec. IV-B): the 8^3 bricks
 *       allocated around the reprojected depth points; with a mask, the walk
 *       emits only voxels of allocated bricks.
 *   or_incidence                    -- voxel -> ray incidence: the rays that
 *       share a voxel (Sec. III-A, Fig. "graphical model"), a stable counting
 *       sort of edges by voxel.
 *   or_potentials                   -- log of the forward sensor model
 *       nu(d_i) = N(Z; d_i + b(d_i), sigma(d_i)) (Eq. noise with the learnt
 *       bias of Sec. IV-C: the bias at the traversed depth gives the predicted
 *       mean measurement, the noise its spread), sigma and b from 64-bin
 *       depth-indexed tables (b = 0 when no bias table is given), or from one
 *       such table per pixel region (Sec. IV-C learns the model per 20 x 20
 *       pixel neighbourhood): the caller passes each edge's table entry.
 *   or_infer                        -- flooding schedule of K sweeps; each
 *       sweep sends variable->factor messages (Eq. node_to_factor, including
 *       the prior factor, Eq. prior_potential) and then the ray-factor ->
 *       variable messages of Eqs. pos and neg, in the log domain with the
 *       division-free form of the second sum of Eq. neg (supplement, Sec. II-C,
 *       the sum over j > i of the product over k < j, k != i).  Marginals are
 *       the normalised product of all incoming factor messages (Sec. III-B).
 *   or_accuracy                     -- the accuracy metric of a map
 *       (Sec. III-D): visibility and generating-surface density along each
 *       depth ray through voxels of constant occlusion density, the
 *       measurement checked against the most likely surface.
 *   or_depth_distribution           -- the ray factor's message to its depth
 *       variable (Eq. depth_message, Sec. III-C): where along each ray the
 *       measurement was generated, given the voxel -> ray messages.
 *   or_infer_f32_storage            -- the same sweeps with the messages
 *       stored at single precision: a conditioning measure, not the method.
 *   or_infer_keyframe_avg           -- the same sweeps with the paper's
 *       memory approximation (Sec. IV-A): one length-weighted average message
 *       per keyframe and voxel.
 *   or_backward                     -- reverse-mode derivative of the K
 *       unrolled sweeps (not in the paper: a project extension), written from
 *       the chain rule on the forward steps above.
 *   or_backward_keyframe_avg        -- the same for the sweeps with per-keyframe
 *       averaged messages.
 *
 * Messages to a binary variable are carried as log-odds
 *   lambda = log mu(o=1) - log mu(o=0)      (voxel -> ray, per edge)
 *   ell    = log mu(o=1) - log mu(o=0)      (ray -> voxel, per edge)
 * which makes every incoming message normalised (supplement, Sec. II-A):
 *   mu(o=1) = sigmoid(lambda), mu(o=0) = sigmoid(-lambda).
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ------------------------------------------------------------------ */
/* scalar helpers                                                      */
/* ------------------------------------------------------------------ */

/* log(exp(a) + exp(b)) with log(0 + 0) = -inf */
static double or_lse(double a, double b)
{
    double hi = a > b ? a : b;
    double lo = a > b ? b : a;
    if (hi == -INFINITY) return -INFINITY;
    return hi + log1p(exp(lo - hi));
}

/* log(1 + exp(x)) */
static double or_softplus(double x)
{
    return (x > 0.0 ? x : 0.0) + log1p(exp(-fabs(x)));
}

/* ------------------------------------------------------------------ */
/* rays and 3D-DDA                                                     */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
    int32_t nx, ny, nz;
    double h;
    double origin[3];
    double z_min, z_max;
    double trunc_nsigma, trunc_c0, trunc_c2, trunc_min;
    double table_dmax;
    int32_t min_ray_voxels;
    const uint8_t* bricks;   /* allocated 8^3 bricks (or_brick_mask), NULL: dense grid */
} or_cfg;

typedef struct {
    double c[3], w[3];
    double Z, ts, te;
} or_ray;

/* The ray of pixel (u, v) of frame f: origin = camera centre, direction =
 * R (x_n, y_n, 1) so the ray parameter is z-depth, clipped to the grid box:
 * [*ts, *texit].  Returns 0 when the pixel carries no usable measurement or
 * the ray misses the grid. */
static int or_clip_ray(const or_cfg* g, const float* depth, const double* T,
                       int v, int u, or_ray* r, double* ts_out, double* texit_out)
{
    double Z = (double)depth[(int64_t)v * g->width + u];
    if (!isfinite(Z) || Z < g->z_min || Z > g->z_max) return 0;
    double xn = ((double)u - g->cx) / g->fx;
    double yn = ((double)v - g->cy) / g->fy;
    const int n[3] = {g->nx, g->ny, g->nz};
    double ts = 0.0, texit = INFINITY;
    for (int a = 0; a < 3; ++a) {
        r->c[a] = T[4 * a + 3];
        double wa = T[4 * a + 0] * xn;
        wa = wa + T[4 * a + 1] * yn;
        wa = wa + T[4 * a + 2];
        r->w[a] = wa;
        if (!isfinite(wa) || !isfinite(r->c[a])) return 0;   /* unusable pose */
        double lo = g->origin[a];
        double hi = g->origin[a] + (double)n[a] * g->h;
        if (wa != 0.0) {
            double t0 = (lo - r->c[a]) / wa;
            double t1 = (hi - r->c[a]) / wa;
            double tmin = t0 < t1 ? t0 : t1;
            double tmax = t0 < t1 ? t1 : t0;
            if (tmin > ts) ts = tmin;
            if (tmax < texit) texit = tmax;
        } else if (r->c[a] < lo || r->c[a] >= hi) {
            return 0;
        }
    }
    r->Z = Z;
    *ts_out = ts;
    *texit_out = texit;
    return 1;
}

/* The graph's ray of a pixel: the clipped ray, kept only when the surface
 * lies inside the grid, walked from the grid entry to 3 sigma_tr past the
 * measurement (Sec. IV-B) or the grid exit. */
static int or_make_ray(const or_cfg* g, const float* depth, const double* T,
                       int v, int u, or_ray* r)
{
    double ts, texit;
    if (!or_clip_ray(g, depth, T, v, u, r, &ts, &texit)) return 0;
    double Z = r->Z;
    /* the surface must lie inside the grid */
    if (Z >= texit) return 0;
    double sig = g->trunc_c2 * Z;
    sig = sig * Z;
    sig = g->trunc_c0 + sig;
    if (sig < g->trunc_min) sig = g->trunc_min;
    double te = Z + g->trunc_nsigma * sig;
    if (te > texit) te = texit;
    if (te <= ts) return 0;
    r->ts = ts;
    r->te = te;
    return 1;
}

static double or_face(const or_cfg* g, int a, int idx)
{
    return g->origin[a] + (double)idx * g->h;
}

/* Sparse bricks (Sec. IV-B): storage exists only in 8^3-voxel bricks
 * allocated around the reprojected depth points, and rays skip the rest.
 * A brick is allocated when the measured surface point c + Z w of a pixel
 * with a usable measurement (any frame) lies in a voxel of the grid whose
 * brick is within `radius` bricks of it along every axis.  mask: one byte per
 * brick, brick (bi, bj, bk) at bi + nbx (bj + nby bk), nb = ceil(n / 8). */
void or_brick_mask(const or_cfg* g, int32_t n_frames, const float* depth, const double* T_wc,
                   int32_t radius, uint8_t* mask)
{
    const int n[3] = {g->nx, g->ny, g->nz};
    int nb[3];
    for (int a = 0; a < 3; ++a) nb[a] = (n[a] + 7) / 8;
    memset(mask, 0, (size_t)nb[0] * nb[1] * nb[2]);
    const int64_t HW = (int64_t)g->width * g->height;
    for (int32_t f = 0; f < n_frames; ++f) {
        const double* T = T_wc + 16 * f;
        for (int64_t pix = 0; pix < HW; ++pix) {
            int v = (int)(pix / g->width), u = (int)(pix % g->width);
            double Z = (double)depth[f * HW + pix];
            if (!isfinite(Z) || Z < g->z_min || Z > g->z_max) continue;
            double xn = ((double)u - g->cx) / g->fx;
            double yn = ((double)v - g->cy) / g->fy;
            int b[3], ok = 1;
            for (int a = 0; a < 3 && ok; ++a) {
                double wa = T[4 * a + 0] * xn;
                wa = wa + T[4 * a + 1] * yn;
                wa = wa + T[4 * a + 2];
                double pa = T[4 * a + 3] + Z * wa;
                double q = floor((pa - g->origin[a]) / g->h);
                if (!(q >= 0.0 && q < (double)n[a])) ok = 0;
                else b[a] = (int)q / 8;
            }
            if (!ok) continue;
            for (int dk = -radius; dk <= radius; ++dk)
                for (int dj = -radius; dj <= radius; ++dj)
                    for (int di = -radius; di <= radius; ++di) {
                        int bi = b[0] + di, bj = b[1] + dj, bk = b[2] + dk;
                        if (bi < 0 || bj < 0 || bk < 0 || bi >= nb[0] || bj >= nb[1] || bk >= nb[2]) continue;
                        mask[bi + (int64_t)nb[0] * (bj + (int64_t)nb[1] * bk)] = 1;
                    }
        }
    }
}

/* whether the voxel idx lies in an allocated brick (always, for a dense grid) */
static int or_allocated(const or_cfg* g, const int idx[3])
{
    if (!g->bricks) return 1;
    const int nbx = (g->nx + 7) / 8, nby = (g->ny + 7) / 8;
    return g->bricks[idx[0] / 8 + (int64_t)nbx * (idx[1] / 8 + (int64_t)nby * (idx[2] / 8))];
}

typedef void (*or_emit_fn)(void* ud, int64_t k, int32_t id, double tin, double tout);

/* Amanatides-Woo walk from t_s to t_e; calls emit for every voxel crossed
 * with a chord of positive length (in an allocated brick, when the grid is
 * sparse).  Ties between axes step the lowest axis first.  Returns the number
 * of voxels emitted. */
static int64_t or_walk(const or_cfg* g, const or_ray* r, or_emit_fn emit, void* ud)
{
    const int n[3] = {g->nx, g->ny, g->nz};
    int idx[3];
    double tmax[3];
    for (int a = 0; a < 3; ++a) {
        double p = r->c[a] + r->ts * r->w[a];
        double q = floor((p - g->origin[a]) / g->h);
        if (q < 0.0) q = 0.0;
        if (q > (double)(n[a] - 1)) q = (double)(n[a] - 1);
        idx[a] = (int)q;
    }
    for (int a = 0; a < 3; ++a) {
        if (r->w[a] > 0.0)
            tmax[a] = (or_face(g, a, idx[a] + 1) - r->c[a]) / r->w[a];
        else if (r->w[a] < 0.0)
            tmax[a] = (or_face(g, a, idx[a]) - r->c[a]) / r->w[a];
        else
            tmax[a] = INFINITY;
    }
    double tin = r->ts;
    int64_t k = 0;
    for (;;) {
        int a = (tmax[0] <= tmax[1] && tmax[0] <= tmax[2]) ? 0 : (tmax[1] <= tmax[2] ? 1 : 2);
        double tm = tmax[a];
        double tout = tm < r->te ? tm : r->te;
        if (tout > tin && or_allocated(g, idx)) {
            int32_t id = idx[0] + g->nx * (idx[1] + g->ny * idx[2]);
            if (emit) emit(ud, k, id, tin, tout);
            ++k;
        }
        if (tm >= r->te) break;
        if (tm > tin) tin = tm;
        idx[a] += r->w[a] > 0.0 ? 1 : -1;
        if (idx[a] < 0 || idx[a] >= n[a]) break;
        if (r->w[a] > 0.0)
            tmax[a] = (or_face(g, a, idx[a] + 1) - r->c[a]) / r->w[a];
        else
            tmax[a] = (or_face(g, a, idx[a]) - r->c[a]) / r->w[a];
    }
    return k;
}

/* Per-ray voxel counts for every pixel of every frame, in the order
 * r = (f H + v) W + u.  Rays shorter than min_ray_voxels get 0. */
void or_trace_count(const or_cfg* g, int32_t n_frames, const float* depth,
                    const double* T_wc, int64_t* counts)
{
    const int64_t HW = (int64_t)g->width * g->height;
    const int64_t R = HW * n_frames;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < R; ++r) {
        int64_t f = r / HW, pix = r % HW;
        int v = (int)(pix / g->width), u = (int)(pix % g->width);
        or_ray ray;
        int64_t m = 0;
        if (or_make_ray(g, depth + f * HW, T_wc + 16 * f, v, u, &ray))
            m = or_walk(g, &ray, NULL, NULL);
        counts[r] = m >= g->min_ray_voxels ? m : 0;
    }
}

typedef struct {
    int32_t* col;
    double *tin, *tout, *delta;
    int32_t* bin;
    int64_t base;
    double Z, dbin;
} or_emit_ud;

static void or_emit(void* p, int64_t k, int32_t id, double tin, double tout)
{
    or_emit_ud* e = (or_emit_ud*)p;
    int64_t at = e->base + k;
    double d = (tin + tout) * 0.5;          /* depth of the voxel: chord midpoint */
    double q = floor(d / e->dbin);
    if (q < 0.0) q = 0.0;
    if (q > 63.0) q = 63.0;
    e->col[at] = id;
    e->tin[at] = tin;
    e->tout[at] = tout;
    e->delta[at] = e->Z - d;
    e->bin[at] = (int32_t)q;
}

/* Edges of every kept ray at row_ptr[r] .. row_ptr[r+1]: voxel id, chord
 * entry/exit, measurement minus voxel depth, and sigma-table bin. */
void or_trace_emit(const or_cfg* g, int32_t n_frames, const float* depth,
                   const double* T_wc, const int64_t* row_ptr, int32_t* col,
                   double* tin, double* tout, double* delta, int32_t* bin)
{
    const int64_t HW = (int64_t)g->width * g->height;
    const int64_t R = HW * n_frames;
    const double dbin = g->table_dmax / 64.0;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < R; ++r) {
        if (row_ptr[r + 1] == row_ptr[r]) continue;
        int64_t f = r / HW, pix = r % HW;
        int v = (int)(pix / g->width), u = (int)(pix % g->width);
        or_ray ray;
        or_make_ray(g, depth + f * HW, T_wc + 16 * f, v, u, &ray);
        or_emit_ud ud = {col, tin, tout, delta, bin, row_ptr[r], ray.Z, dbin};
        or_walk(g, &ray, or_emit, &ud);
    }
}

/* Stable counting sort of edges by voxel: vptr[V+1], vedge[E] with edge ids
 * ascending inside every voxel. */
void or_incidence(const int32_t* col, int64_t E, int64_t V, int64_t* vptr, int64_t* vedge)
{
    memset(vptr, 0, sizeof(int64_t) * (size_t)(V + 1));
    for (int64_t e = 0; e < E; ++e) vptr[col[e] + 1] += 1;
    for (int64_t v = 0; v < V; ++v) vptr[v + 1] += vptr[v];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(V > 0 ? V : 1));
    memcpy(fill, vptr, sizeof(int64_t) * (size_t)V);
    for (int64_t e = 0; e < E; ++e) vedge[fill[col[e]]++] = e;
    free(fill);
}

/* g_e = log N(Z; d_e + mu_b, sigma_b) = -((delta - mu_b)/sigma_b)^2/2 - log sigma_b
 * - log(2 pi)/2 with delta = Z - d_e; bias (mu) may be NULL for mu = 0.  bin[e]
 * indexes the tables: the depth bin, or, with per-pixel-region tables (Sec. IV-C),
 * the region's row times 64 plus the depth bin. */
void or_potentials(const double* delta, const int32_t* bin, int64_t E,
                   const double* sigma, const double* bias, double* g)
{
    const double half_log_2pi = 0.5 * log(2.0 * M_PI);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        double s = sigma[bin[e]];
        double mu = bias ? bias[bin[e]] : 0.0;
        double x = (delta[e] - mu) / s;
        g[e] = -0.5 * x * x - log(s) - half_log_2pi;
    }
}

/* ------------------------------------------------------------------ */
/* message passing                                                     */
/* ------------------------------------------------------------------ */

/* Variable -> factor messages (Eq. node_to_factor): the voxel's prior factor
 * times every other ray factor's message.  In log-odds: theta_v plus the sum
 * of ell over the voxel's other edges, taken as (theta + sum before) + sum
 * after, never as a difference. */
static void or_voxel_phase(const int64_t* vptr, const int64_t* vedge, int64_t V,
                           const double* base, const double* ell, double* lam)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < V; ++v) {
        int64_t s = vptr[v], e = vptr[v + 1];
        double after = 0.0;
        for (int64_t j = e - 1; j >= s; --j) {   /* suffix sums, parked in lam */
            lam[vedge[j]] = after;
            after += ell[vedge[j]];
        }
        double before = 0.0;
        for (int64_t j = s; j < e; ++j) {
            double b0 = base ? base[v] : 0.0;
            lam[vedge[j]] = (b0 + before) + lam[vedge[j]];
            before += ell[vedge[j]];
        }
    }
}

/* Ray-factor -> variable messages for one ray (Eqs. pos and neg).
 *
 * With a_k = mu(o_k=0), b_k = mu(o_k=1), nu_k = exp(g_k) and 1-based i:
 *   m1_i = sum_{j<i} b_j nu_j prod_{k<j} a_k  +  nu_i prod_{k<i} a_k
 *   m0_i = sum_{j<i} b_j nu_j prod_{k<j} a_k  +  sum_{j>i} b_j nu_j prod_{k<j,k!=i} a_k
 * In logs, with P_i = sum_{k<i} log a_k (visibility up to voxel i):
 *   first term   F_i = LSE_{j<i} (log b_j + g_j + P_j)       (Eq. depth_message summed)
 *   second sum   P_i + T_i with T_i = log sum_{j>i} b_j nu_j prod_{i<k<j} a_k,
 *                T_i = LSE(log b_{i+1} + g_{i+1}, log a_{i+1} + T_{i+1}), T_N = -inf
 *   ell_i = LSE(F_i, g_i + P_i) - LSE(F_i, P_i + T_i).
 * Scratch arrays hold n doubles each. */
static void or_ray_messages(int64_t n, const double* lam, const double* g, double* ell,
                            double* la, double* lb, double* P, double* F, double* T)
{
    for (int64_t i = 0; i < n; ++i) {
        la[i] = -or_softplus(lam[i]);    /* log mu(o=0) = log sigmoid(-lambda) */
        lb[i] = -or_softplus(-lam[i]);   /* log mu(o=1) = log sigmoid(lambda)  */
    }
    double acc = 0.0, f = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        P[i] = acc;
        F[i] = f;
        f = or_lse(f, lb[i] + g[i] + P[i]);
        acc += la[i];
    }
    T[n - 1] = -INFINITY;
    for (int64_t i = n - 2; i >= 0; --i)
        T[i] = or_lse(lb[i + 1] + g[i + 1], la[i + 1] + T[i + 1]);
    for (int64_t i = 0; i < n; ++i) {
        double m1 = or_lse(F[i], g[i] + P[i]);
        double m0 = or_lse(F[i], P[i] + T[i]);
        ell[i] = m1 - m0;
    }
}

static int64_t or_max_len(const int64_t* row_ptr, int64_t R)
{
    int64_t m = 1;
    for (int64_t r = 0; r < R; ++r)
        if (row_ptr[r + 1] - row_ptr[r] > m) m = row_ptr[r + 1] - row_ptr[r];
    return m;
}

static void or_ray_phase(const int64_t* row_ptr, int64_t R, const double* lam,
                         const double* g, double* ell)
{
    int64_t mx = or_max_len(row_ptr, R);
#pragma omp parallel
    {
        double* scratch = (double*)malloc(sizeof(double) * 5 * (size_t)mx);
#pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < R; ++r) {
            int64_t s = row_ptr[r], n = row_ptr[r + 1] - s;
            if (n == 0) continue;
            or_ray_messages(n, lam + s, g + s, ell + s, scratch, scratch + mx,
                            scratch + 2 * mx, scratch + 3 * mx, scratch + 4 * mx);
        }
        free(scratch);
    }
}

/* Belief of every voxel: L_v = theta_v + sum of all incoming ray messages. */
static void or_beliefs(const int64_t* vptr, const int64_t* vedge, int64_t V,
                       const double* theta, const double* ell, double* L)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < V; ++v) {
        double s = theta[v];
        for (int64_t j = vptr[v]; j < vptr[v + 1]; ++j) s += ell[vedge[j]];
        L[v] = s;
    }
}

/* K sweeps of the flooding schedule starting from uniform ray messages
 * (ell = 0).  lam_hist (K*E, optional) keeps lambda of every sweep for the
 * reverse pass; ell_out (E) and lam_out (E) hold the last sweep's messages;
 * L (V) the marginal log-odds. */
void or_infer(const int64_t* row_ptr, int64_t R, const int64_t* vptr, const int64_t* vedge,
              int64_t V, int64_t E, const double* theta, const double* g, int32_t K,
              double* lam_hist, double* lam_out, double* ell_out, double* L)
{
    double* ell = ell_out;
    memset(ell, 0, sizeof(double) * (size_t)E);
    for (int32_t k = 0; k < K; ++k) {
        or_voxel_phase(vptr, vedge, V, theta, ell, lam_out);
        if (lam_hist) memcpy(lam_hist + (int64_t)k * E, lam_out, sizeof(double) * (size_t)E);
        or_ray_phase(row_ptr, R, lam_out, g, ell);
    }
    or_beliefs(vptr, vedge, V, theta, ell, L);
}

/* The same K sweeps with every message stored at single precision: after
 * each voxel phase every lambda, and after each ray phase every ell, is
 * replaced by a nearby float32 value, all arithmetic staying in FP64.  This
 * does not change the method; it measures how far the exact answer moves when
 * the messages carry a relative error of 2^-24 -- the conditioning of the
 * iteration, which bounds what any implementation with float32 message
 * arrays can reach.  mode 1 rounds to the nearest float32; mode 2 takes the
 * float32 neighbour below or above, chosen by a counter-based hash of
 * (sweep, edge) (splitmix64): a second, independent rounding pattern. */
static uint64_t or_splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static void or_store_f32(double* a, int64_t E, int mode, uint64_t salt)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        float f = (float)a[e];
        if (mode == 2 && isfinite(f) && (double)f != a[e]) {
            /* the float32 neighbours lo < a[e] < hi; the hash picks one */
            float lo = (double)f < a[e] ? f : nextafterf(f, -INFINITY);
            float hi = (double)f > a[e] ? f : nextafterf(f, INFINITY);
            f = (or_splitmix64(salt * 0x100000001B3ull + (uint64_t)e) >> 63) ? hi : lo;
        }
        a[e] = (double)f;
    }
}

void or_infer_f32_storage(const int64_t* row_ptr, int64_t R, const int64_t* vptr, const int64_t* vedge,
                          int64_t V, int64_t E, const double* theta, const double* g, int32_t K, int32_t mode,
                          double* lam_out, double* ell_out, double* L)
{
    double* ell = ell_out;
    memset(ell, 0, sizeof(double) * (size_t)E);
    for (int32_t k = 0; k < K; ++k) {
        or_voxel_phase(vptr, vedge, V, theta, ell, lam_out);
        or_store_f32(lam_out, E, mode, 2u * (uint64_t)k + 1u);
        or_ray_phase(row_ptr, R, lam_out, g, ell);
        or_store_f32(ell, E, mode, 2u * (uint64_t)k + 2u);
    }
    or_beliefs(vptr, vedge, V, theta, ell, L);
}

/* Per-keyframe averaged messages (Sec. IV-A): storing every incoming message
 * of a voxel is avoided by assuming that the rays of one keyframe crossing a
 * voxel send the same message, their average weighted by the length each ray
 * travels in the voxel.  Read here as: each keyframe f contributes ONE message
 * m_f,v = sum w_e ell_e / sum w_e (over its edges e in voxel v) to the voxel's
 * belief, and the voxel -> ray message of an edge of keyframe f is the prior
 * plus the averages of the OTHER keyframes (the receiving ray's keyframe is
 * excluded as a whole).  key: keyframe of every edge, non-decreasing along
 * every voxel's edge list (edge ids are keyframe-major); w: weight per edge.
 * Sums over keyframes are taken as (theta + before) + after, never as a
 * difference.  Returns 0, or -1 when key is not grouped per voxel. */
static int or_voxel_phase_kf(const int64_t* vptr, const int64_t* vedge, int64_t V, const double* theta,
                             const double* ell, const int32_t* key, const double* w, double* lam, double* L)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : bad)
    for (int64_t v = 0; v < V; ++v) {
        int64_t s = vptr[v], e = vptr[v + 1];
        /* run averages, parked per edge in lam as the run's mean, then replaced */
        double after = 0.0;
        for (int64_t j = s; j < e;) {
            int32_t f = key[vedge[j]];
            double sw = 0.0, sm = 0.0;
            int64_t q = j;
            for (; q < e && key[vedge[q]] == f; ++q) {
                sw += w[vedge[q]];
                sm += w[vedge[q]] * ell[vedge[q]];
            }
            if (q < e && key[vedge[q]] < f) bad = 1;
            for (int64_t r = j; r < q; ++r) lam[vedge[r]] = sm / sw;
            j = q;
        }
        /* suffix sums over the runs after each run */
        for (int64_t j = e - 1; j >= s;) {
            int32_t f = key[vedge[j]];
            double m = lam[vedge[j]];
            int64_t q = j;
            for (; q >= s && key[vedge[q]] == f; --q) lam[vedge[q]] = after;
            after += m;
            j = q;
        }
        /* (theta + runs before) + runs after */
        double before = 0.0;
        for (int64_t j = s; j < e;) {
            int32_t f = key[vedge[j]];
            int64_t q = j;
            double m = 0.0, sw = 0.0;
            for (; q < e && key[vedge[q]] == f; ++q) {
                sw += w[vedge[q]];
                m += w[vedge[q]] * ell[vedge[q]];
            }
            for (int64_t r = j; r < q; ++r) lam[vedge[r]] = (theta[v] + before) + lam[vedge[r]];
            before += m / sw;
            j = q;
        }
        if (L) L[v] = theta[v] + before;
    }
    return bad ? -1 : 0;
}

/* K sweeps of the flooding schedule with per-keyframe averaged messages;
 * ell = 0 initially, so the first sweep's lambda is theta.  Outputs as
 * or_infer: the last sweep's lambda and ell (E) and the beliefs L (V): the
 * prior plus one averaged message per keyframe; lam_hist (K*E, or NULL)
 * receives every sweep's lambda.  Returns 0 or -1 (key). */
int or_infer_keyframe_avg(const int64_t* row_ptr, int64_t R, const int64_t* vptr, const int64_t* vedge,
                          int64_t V, int64_t E, const double* theta, const double* g, int32_t K,
                          const int32_t* key, const double* w, double* lam_out, double* ell_out, double* L,
                          double* lam_hist)
{
    memset(ell_out, 0, sizeof(double) * (size_t)E);
    for (int32_t k = 0; k < K; ++k) {
        if (or_voxel_phase_kf(vptr, vedge, V, theta, ell_out, key, w, lam_out, NULL)) return -1;
        if (lam_hist) memcpy(lam_hist + (int64_t)k * E, lam_out, sizeof(double) * (size_t)E);
        or_ray_phase(row_ptr, R, lam_out, g, ell_out);
    }
    double* tmp = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    int rc = or_voxel_phase_kf(vptr, vedge, V, theta, ell_out, key, w, tmp, L);
    free(tmp);
    return rc;
}

/* ------------------------------------------------------------------ */
/* reverse mode (project extension)                                    */
/* ------------------------------------------------------------------ */

/* Adjoint of or_ray_messages for one ray: given d loss / d ell_i, returns
 * d loss / d lambda_i and adds d loss / d g_i into gbar.  Follows the forward
 * recurrences backwards:
 *   ell_i = M1_i - M0_i, M1_i = LSE(F_i, A_i), M0_i = LSE(F_i, B_i),
 *   A_i = g_i + P_i, B_i = P_i + T_i,
 *   F_{i+1} = LSE(F_i, W_i), W_i = log b_i + g_i + P_i,
 *   T_i = LSE(c_{i+1}, log a_{i+1} + T_{i+1}), c_j = log b_j + g_j,
 *   P_{i+1} = P_i + log a_i,
 *   d log a / d lambda = -b,  d log b / d lambda = a. */
static void or_ray_adjoint(int64_t n, const double* lam, const double* g, const double* ellbar,
                           double* lambar, double* gbar, double* w)
{
    double *la = w, *lb = w + n, *P = w + 2 * n, *F = w + 3 * n, *T = w + 4 * n;
    double *M1 = w + 5 * n, *M0 = w + 6 * n, *Pb = w + 7 * n, *lab = w + 8 * n, *lbb = w + 9 * n;
    double *Fb = w + 10 * n, *Tb = w + 11 * n;
    for (int64_t i = 0; i < n; ++i) {
        la[i] = -or_softplus(lam[i]);
        lb[i] = -or_softplus(-lam[i]);
    }
    double acc = 0.0, f = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        P[i] = acc;
        F[i] = f;
        f = or_lse(f, lb[i] + g[i] + P[i]);
        acc += la[i];
    }
    T[n - 1] = -INFINITY;
    for (int64_t i = n - 2; i >= 0; --i)
        T[i] = or_lse(lb[i + 1] + g[i + 1], la[i + 1] + T[i + 1]);
    for (int64_t i = 0; i < n; ++i) {
        M1[i] = or_lse(F[i], g[i] + P[i]);
        M0[i] = or_lse(F[i], P[i] + T[i]);
        Pb[i] = lab[i] = lbb[i] = 0.0;
    }
    /* direct partials of ell_i */
    for (int64_t i = 0; i < n; ++i) {
        double eb = ellbar[i];
        Fb[i] = eb * (exp(F[i] - M1[i]) - exp(F[i] - M0[i]));
        double Ab = eb * exp(g[i] + P[i] - M1[i]);
        double Bb = -eb * exp(P[i] + T[i] - M0[i]);
        gbar[i] += Ab;
        Pb[i] += Ab + Bb;
        Tb[i] = Bb;
    }
    /* T runs right-to-left, so its adjoint runs left-to-right */
    for (int64_t i = 0; i + 1 < n; ++i) {
        double cj = lb[i + 1] + g[i + 1];
        double wc = exp(cj - T[i]);
        double wt = exp(la[i + 1] + T[i + 1] - T[i]);
        lbb[i + 1] += Tb[i] * wc;
        gbar[i + 1] += Tb[i] * wc;
        lab[i + 1] += Tb[i] * wt;
        Tb[i + 1] += Tb[i] * wt;
    }
    /* F runs left-to-right, so its adjoint runs right-to-left */
    for (int64_t i = n - 1; i >= 1; --i) {
        /* F_i = LSE(F_{i-1}, W_{i-1}) */
        double Wm = lb[i - 1] + g[i - 1] + P[i - 1];
        double wf = exp(F[i - 1] - F[i]);
        double ww = exp(Wm - F[i]);
        Fb[i - 1] += Fb[i] * wf;
        lbb[i - 1] += Fb[i] * ww;
        gbar[i - 1] += Fb[i] * ww;
        Pb[i - 1] += Fb[i] * ww;
    }
    /* P_i = sum_{k<i} log a_k */
    double suf = 0.0;
    for (int64_t k = n - 1; k >= 0; --k) {
        lab[k] += suf;
        suf += Pb[k];
    }
    for (int64_t i = 0; i < n; ++i) {
        double a = exp(la[i]), b = exp(lb[i]);
        lambar[i] = -b * lab[i] + a * lbb[i];
    }
}

/* Reverse pass over K sweeps.  Inputs: the forward's lambda of every sweep
 * (lam_hist, K*E), g (E), and Lbar = d loss / d L (V).  Outputs:
 * d loss / d theta (V), d loss / d g accumulated over sweeps (gbar, E), and
 * d loss / d sigma_b and d loss / d mu_b (n_tab entries each: 64 depth bins,
 * or 64 per pixel region; bin[e] indexes them as in or_potentials) through
 * g_e = log N(Z; d_e + mu_b, sigma_b), with r = Z - d_e - mu_b:
 *   d g / d sigma = r^2 / sigma^3 - 1 / sigma,   d g / d mu = r / sigma^2.
 * bias may be NULL (mu = 0); bias_bar may be NULL (not wanted). */
void or_backward(const int64_t* row_ptr, int64_t R, const int64_t* vptr, const int64_t* vedge,
                 int64_t V, int64_t E, const double* g, int32_t K, const double* lam_hist,
                 const double* Lbar, const double* delta, const int32_t* bin,
                 const double* sigma, const double* bias, int32_t n_tab, double* theta_bar, double* gbar,
                 double* sigma_bar, double* bias_bar)
{
    double* ellbar = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    double* lambar = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    memset(gbar, 0, sizeof(double) * (size_t)E);
    for (int64_t v = 0; v < V; ++v) {
        theta_bar[v] = Lbar[v];
        for (int64_t j = vptr[v]; j < vptr[v + 1]; ++j) ellbar[vedge[j]] = Lbar[v];
    }
    int64_t mx = or_max_len(row_ptr, R);
    for (int32_t k = K - 1; k >= 0; --k) {
        const double* lam = lam_hist + (int64_t)k * E;
#pragma omp parallel
        {
            double* w = (double*)malloc(sizeof(double) * 12 * (size_t)mx);
#pragma omp for schedule(dynamic, 256)
            for (int64_t r = 0; r < R; ++r) {
                int64_t s = row_ptr[r], n = row_ptr[r + 1] - s;
                if (n == 0) continue;
                or_ray_adjoint(n, lam + s, g + s, ellbar + s, lambar + s, gbar + s, w);
            }
            free(w);
        }
        /* lambda_e = theta_v + sum_{e' in v, e' != e} ell_e' */
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t v = 0; v < V; ++v) {
            double tot = 0.0;
            for (int64_t j = vptr[v]; j < vptr[v + 1]; ++j) tot += lambar[vedge[j]];
            theta_bar[v] += tot;
        }
        if (k > 0) or_voxel_phase(vptr, vedge, V, NULL, lambar, ellbar);
    }
    for (int32_t b = 0; b < n_tab; ++b) {
        sigma_bar[b] = 0.0;
        if (bias_bar) bias_bar[b] = 0.0;
    }
    for (int64_t e = 0; e < E; ++e) {
        double s = sigma[bin[e]];
        double r = delta[e] - (bias ? bias[bin[e]] : 0.0);
        sigma_bar[bin[e]] += gbar[e] * (r * r / (s * s * s) - 1.0 / s);
        if (bias_bar) bias_bar[bin[e]] += gbar[e] * (r / (s * s));
    }
    free(ellbar);
    free(lambar);
}

/* Reverse pass through K sweeps with per-keyframe averaged messages
 * (or_infer_keyframe_avg, with lam_hist).  The chain rule on its steps:
 *   L_v = theta_v + sum over runs r of v of A_r(ell of the last sweep),
 *   A_r = sum_{q in r} w_q ell_q / sum_{q in r} w_q  (the run's average),
 *   lambda_e = theta_v + sum over the runs of v other than e's own of A_r,
 * so with s_r = sum_{e in r} d/d lambda_e, the derivative reaching ell_q of
 * the previous sweep is w_q / sum_r w times the sum of s over the OTHER runs
 * of q's voxel (taken as before + after, never as a difference), every sweep
 * adds sum_{e in v} d/d lambda_e to d/d theta_v, and the last sweep's ell_q
 * receives w_q / sum_r w times d/d L_v.  The ray adjoint and the sensor-table
 * gradients are those of or_backward (same arguments). */
void or_backward_keyframe_avg(const int64_t* row_ptr, int64_t R, const int64_t* vptr, const int64_t* vedge,
                              int64_t V, int64_t E, const double* g, int32_t K, const double* lam_hist,
                              const double* Lbar, const double* delta, const int32_t* bin, const double* sigma,
                              const double* bias, int32_t n_tab, const int32_t* key, const double* w,
                              double* theta_bar, double* gbar, double* sigma_bar, double* bias_bar)
{
    double* ellbar = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    double* lambar = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    memset(gbar, 0, sizeof(double) * (size_t)E);
    /* the last sweep's ell reaches L through its run averages */
    for (int64_t v = 0; v < V; ++v) {
        theta_bar[v] = Lbar[v];
        for (int64_t j = vptr[v]; j < vptr[v + 1];) {
            int32_t f = key[vedge[j]];
            int64_t q = j;
            double sw = 0.0;
            for (; q < vptr[v + 1] && key[vedge[q]] == f; ++q) sw += w[vedge[q]];
            for (int64_t r = j; r < q; ++r) ellbar[vedge[r]] = w[vedge[r]] / sw * Lbar[v];
            j = q;
        }
    }
    int64_t mx = or_max_len(row_ptr, R);
    for (int32_t k = K - 1; k >= 0; --k) {
        const double* lam = lam_hist + (int64_t)k * E;
#pragma omp parallel
        {
            double* wk = (double*)malloc(sizeof(double) * 12 * (size_t)mx);
#pragma omp for schedule(dynamic, 256)
            for (int64_t r = 0; r < R; ++r) {
                int64_t s = row_ptr[r], n = row_ptr[r + 1] - s;
                if (n == 0) continue;
                or_ray_adjoint(n, lam + s, g + s, ellbar + s, lambar + s, gbar + s, wk);
            }
            free(wk);
        }
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t v = 0; v < V; ++v) {
            int64_t s = vptr[v], e = vptr[v + 1];
            double tot = 0.0;
            for (int64_t j = s; j < e; ++j) tot += lambar[vedge[j]];
            theta_bar[v] += tot;
            if (k == 0) continue;
            /* ell of the previous sweep: w_q / sum w times the other runs' sums */
            double after = 0.0;
            for (int64_t j = e - 1; j >= s;) {   /* after-sums parked in ellbar */
                int32_t f = key[vedge[j]];
                int64_t q = j;
                double sr = 0.0;
                for (; q >= s && key[vedge[q]] == f; --q) sr += lambar[vedge[q]];
                for (int64_t r = j; r > q; --r) ellbar[vedge[r]] = after;
                after += sr;
                j = q;
            }
            double before = 0.0;
            for (int64_t j = s; j < e;) {
                int32_t f = key[vedge[j]];
                int64_t q = j;
                double sr = 0.0, sw = 0.0;
                for (; q < e && key[vedge[q]] == f; ++q) {
                    sr += lambar[vedge[q]];
                    sw += w[vedge[q]];
                }
                for (int64_t r = j; r < q; ++r) ellbar[vedge[r]] = w[vedge[r]] / sw * (before + ellbar[vedge[r]]);
                before += sr;
                j = q;
            }
        }
    }
    for (int32_t b = 0; b < n_tab; ++b) {
        sigma_bar[b] = 0.0;
        if (bias_bar) bias_bar[b] = 0.0;
    }
    for (int64_t e = 0; e < E; ++e) {
        double s = sigma[bin[e]];
        double r = delta[e] - (bias ? bias[bin[e]] : 0.0);
        sigma_bar[bin[e]] += gbar[e] * (r * r / (s * s * s) - 1.0 / s);
        if (bias_bar) bias_bar[bin[e]] += gbar[e] * (r / (s * s));
    }
    free(ellbar);
    free(lambar);
}

/* ------------------------------------------------------------------ */
/* accuracy metric of a map (Sec. III-D)                               */
/* ------------------------------------------------------------------ */

/* Each voxel is a region of constant occlusion density alpha; a ray that
 * crosses the voxel's side h is blocked with the voxel's occupancy
 * probability p, so alpha = -ln(1 - p) / h = softplus(L) / h for log-odds L.
 * Along the ray (Euclidean distance s) vis(s) = exp(-integral of alpha) and
 * the density of the generating surface is omega(s) = alpha(s) vis(s); inside
 * a voxel it decays, so its maximum over the ray is at the entry of the voxel
 * maximising log alpha_n - sum_{i<n} alpha_i l_i (the first such voxel on
 * ties). */
typedef struct {
    const double* L;
    double inv_h, wn;
    double acc;              /* sum of alpha_i l_i over the voxels walked */
    double best, second;     /* largest and second largest log omega at an entry */
    double btin, btout;      /* chord of the best voxel (z-depth) */
} or_metric_ud;

static void or_metric_emit(void* p, int64_t k, int32_t id, double tin, double tout)
{
    (void)k;
    or_metric_ud* m = (or_metric_ud*)p;
    double alpha = or_softplus(m->L[id]) * m->inv_h;
    double lw = log(alpha) - m->acc;
    if (lw > m->best) {
        m->second = m->best;
        m->best = lw;
        m->btin = tin;
        m->btout = tout;
    } else if (lw > m->second) {
        m->second = lw;
    }
    m->acc += alpha * ((tout - tin) * m->wn);
}

/* Accuracy of every depth ray of one scene against the map L (V log-odds,
 * scene-local ids).  A ray is walked over the whole grid (no truncation; the
 * surface may lie beyond it).  When the visibility at the grid exit is at
 * least vis_min the map has not blocked the ray enough and the ray counts as
 * accurate iff its measurement lies beyond the exit (Z > exit z-depth);
 * otherwise iff the measurement lies inside the chord of the voxel where the
 * most likely generating surface is.  Per ray (r = (f H + v) W + u):
 *   code   1 accurate, 0 not, -1 not evaluated (no usable measurement, or the
 *          ray misses the grid);
 *   tin, tout  chord of the chosen voxel, or (exit, +inf) for the beyond rule;
 *   lvis   log visibility at the grid exit;
 *   margin distance of the decision from a tie: the smaller of (best - second
 *          best log omega) and |lvis - log vis_min| (+inf when neither exists). */
/* tol_nsigma > 0 selects the paper's evaluation rule (Sec. V) instead: the ray
 * is accurate iff the most likely generating surface (the chosen voxel's
 * entry, z-depth) lies within tol_nsigma sigma(Z) of Z, sigma(Z) =
 * max(trunc_c0 + trunc_c2 Z^2, trunc_min) the sensor's noise; the beyond rule
 * is unchanged.  `depth` is the image the rays are scored against (the
 * measurement, or a reference such as noise-free depth from the same poses). */
void or_accuracy(const or_cfg* g, int32_t n_frames, const float* depth, const double* T_wc,
                 const double* L, double vis_min, double tol_nsigma, int8_t* code, double* tin, double* tout,
                 double* lvis, double* margin)
{
    const int64_t HW = (int64_t)g->width * g->height;
    const int64_t R = HW * n_frames;
    const double lvmin = log(vis_min);
    or_cfg dense = *g;          /* the metric walks the whole grid */
    dense.bricks = NULL;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < R; ++r) {
        int64_t f = r / HW, pix = r % HW;
        int v = (int)(pix / g->width), u = (int)(pix % g->width);
        or_ray ray;
        double ts, texit;
        code[r] = -1;
        tin[r] = tout[r] = lvis[r] = margin[r] = NAN;
        if (!or_clip_ray(g, depth + f * HW, T_wc + 16 * f, v, u, &ray, &ts, &texit)) continue;
        if (!(ts < texit)) continue;
        ray.ts = ts;
        ray.te = texit;
        or_metric_ud m;
        m.L = L;
        m.inv_h = 1.0 / g->h;
        m.wn = sqrt(ray.w[0] * ray.w[0] + ray.w[1] * ray.w[1] + ray.w[2] * ray.w[2]);
        m.acc = 0.0;
        m.best = m.second = -INFINITY;
        m.btin = m.btout = NAN;
        or_walk(&dense, &ray, or_metric_emit, &m);
        double lv = -m.acc;
        double gap = m.best > -INFINITY && m.second > -INFINITY ? m.best - m.second : INFINITY;
        double vgap = fabs(lv - lvmin);
        lvis[r] = lv;
        margin[r] = gap < vgap ? gap : vgap;
        if (lv >= lvmin) {
            code[r] = ray.Z > texit ? 1 : 0;
            tin[r] = texit;
            tout[r] = INFINITY;
        } else if (tol_nsigma > 0.0) {
            double sig = g->trunc_c2 * ray.Z;
            sig = sig * ray.Z;
            sig = g->trunc_c0 + sig;
            if (sig < g->trunc_min) sig = g->trunc_min;
            code[r] = fabs(m.btin - ray.Z) <= tol_nsigma * sig ? 1 : 0;
            tin[r] = m.btin;
            tout[r] = m.btout;
        } else {
            code[r] = (m.btin <= ray.Z && ray.Z < m.btout) ? 1 : 0;
            tin[r] = m.btin;
            tout[r] = m.btout;
        }
    }
}

/* ------------------------------------------------------------------ */
/* ray depth potential -> depth variable (Eq. depth_message)           */
/* ------------------------------------------------------------------ */

/* The message of each ray factor to its depth variable (Sec. III-C): the
 * measurement was generated at voxel i's depth with weight
 *   nu(d_i) mu(o_i = 1) prod_{k<i} mu(o_k = 0),
 * the incoming messages being the voxel -> ray messages lam (log-odds) of a
 * sweep.  Normalised over the ray's voxels (the all-empty configuration has
 * potential zero), per edge q = the probability of the depth d_i; per ray
 * mode = the step of the most probable depth (the first on ties), -1 for a
 * ray without voxels. */
void or_depth_distribution(const int64_t* row_ptr, int64_t R, const double* lam, const double* g,
                           double* q, int32_t* mode)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < R; ++r) {
        int64_t s = row_ptr[r], n = row_ptr[r + 1] - s;
        mode[r] = -1;
        if (n == 0) continue;
        double P = 0.0, best = -INFINITY, tot = -INFINITY;
        for (int64_t i = 0; i < n; ++i) {
            double w = -or_softplus(-lam[s + i]) + g[s + i] + P;   /* log of the weight of depth d_i */
            q[s + i] = w;
            tot = or_lse(tot, w);
            if (w > best) {
                best = w;
                mode[r] = (int32_t)i;
            }
            P += -or_softplus(lam[s + i]);
        }
        for (int64_t i = 0; i < n; ++i) q[s + i] = exp(q[s + i] - tot);
    }
}

/* ------------------------------------------------------------------ */
/* small exports for tests                                             */
/* ------------------------------------------------------------------ */

/* Messages of a single ray factor, exposed for the brute-force checks. */
void or_single_ray(int64_t n, const double* lam, const double* g, double* ell)
{
    double* s = (double*)malloc(sizeof(double) * 5 * (size_t)n);
    or_ray_messages(n, lam, g, ell, s, s + n, s + 2 * n, s + 3 * n, s + 4 * n);
    free(s);
}

void or_single_ray_adjoint(int64_t n, const double* lam, const double* g, const double* ellbar,
                           double* lambar, double* gbar)
{
    double* w = (double*)malloc(sizeof(double) * 12 * (size_t)n);
    for (int64_t i = 0; i < n; ++i) gbar[i] = 0.0;
    or_ray_adjoint(n, lam, g, ellbar, lambar, gbar, w);
    free(w);
}

int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_threads(int n) { omp_set_num_threads(n); }
