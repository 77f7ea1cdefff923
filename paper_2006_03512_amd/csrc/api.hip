// C ABI of libmrf (declared in include/mrf.h): context lifetime, graph
// construction, the sweep schedule (eager launches or one captured hipGraph),
// marginals, the reverse pass, stats and exports.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mrf_internal.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (!g_err.empty() && e == hipErrorInvalidConfiguration) m = g_err;
    g_err = m;
    return e == hipErrorOutOfMemory ? MRF_ENOMEM : MRF_EHIP;
}

#define HCK(expr, what)                                  \
    do {                                                 \
        hipError_t _e = (expr);                          \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

void drop_graph(mrf_ctx* c)
{
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->g_K = c->g_ckpt = -1;
    c->g_key.clear();
}

// Everything a captured forward graph bakes in: launch shapes and addresses.
std::vector<uint64_t> graph_key(const mrf_ctx* c, int K, int keep)
{
    std::vector<uint64_t> k = {(uint64_t)K, (uint64_t)keep, (uint64_t)c->E, (uint64_t)c->R, (uint64_t)c->V,
                               (uint64_t)c->Vk, (uint64_t)c->S, (uint64_t)c->T};
    for (int i = 0; i < mrf::kRayClasses; ++i) k.push_back((uint64_t)c->ray_cnt[i]);
    for (int i = 0; i < mrf::kVoxClasses; ++i) k.push_back((uint64_t)c->vox_cnt[i]);
    for (int i = 0; i < mrf::kRayClasses; ++i) k.push_back((uint64_t)c->fwd_sel[i]);
    const mrf::DevBuf* bufs[] = {&c->b_rowptr, &c->b_col,   &c->b_delta, &c->b_bin,  &c->b_g,    &c->b_lam,
                                 &c->b_ell,    &c->b_vedge, &c->b_vptr,  &c->b_theta, &c->b_L,   &c->b_sigma, &c->b_bias,
                                 &c->b_ckpt,   &c->b_tsum,  &c->b_tbar,  &c->b_tiles, &c->b_counts, &c->b_theta2,
                                 &c->b_kfw,    &c->b_pair_m, &c->b_pair_x, &c->b_kfx, &c->b_kfxb, &c->b_kf_vox};
    for (const mrf::DevBuf* b : bufs) k.push_back((uint64_t)(uintptr_t)b->p);
    for (const auto& b : c->b_ray_list) k.push_back((uint64_t)(uintptr_t)b.p);
    for (const auto& b : c->b_vox_list) k.push_back((uint64_t)(uintptr_t)b.p);
    for (const auto& b : c->b_vox_desc) k.push_back((uint64_t)(uintptr_t)b.p);
    for (const auto& b : c->b_pair_desc) k.push_back((uint64_t)(uintptr_t)b.p);
    for (int i = 0; i < mrf::kVoxClasses; ++i) k.push_back((uint64_t)c->pair_cnt[i]);
    k.push_back((uint64_t)c->n_kf_vox);
    k.push_back((uint64_t)c->cell_px);
    k.push_back((uint64_t)c->n_cells);
    k.push_back((uint64_t)c->sg.n);
    for (int g = 0; g < mrf::kMaxSlotGroups; ++g) {
        k.push_back((uint64_t)c->sg.slot[g]);
        k.push_back((uint64_t)c->sg.pos[g]);
    }
    k.push_back((uint64_t)(uintptr_t)c->b_frames.p);
    k.push_back((uint64_t)(uintptr_t)c->b_scenes.p);
    return k;
}

int bits_for(int64_t maxval)
{
    int b = 1;
    while (b < 63 && (int64_t(1) << b) <= maxval) ++b;
    return b;
}

}  // namespace

namespace mrf {

void set_error(const std::string& msg) { g_err = msg; }

// Set while mrf_add_frames runs: a buffer that ensure() has to grow then gets
// room for four more growths of the same size (at most doubling it), so that
// frames added one at a time reallocate rarely.
static thread_local int g_grow_room = 0;

static size_t with_room(size_t need, size_t prev)
{
    const size_t step = need > prev ? need - prev : 0;
    return step < need / 4 ? need + 4 * step : 2 * need;
}

hipError_t ensure(DevBuf& b, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (b.p && b.cap >= bytes) return hipSuccess;
    const size_t old = b.p ? b.cap : 0;
    if (b.p) hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    const size_t want = g_grow_room && old > 0 ? with_room(bytes, old) : bytes;
    hipError_t e = hipMalloc(&b.p, want);
    if (e == hipSuccess) {
        b.cap = want;
        return e;
    }
    b.p = nullptr;
    hipGetLastError();
    if (want == bytes) return e;
    e = hipMalloc(&b.p, bytes);   // without the room
    if (e != hipSuccess) {
        b.p = nullptr;
        hipGetLastError();
        return e;
    }
    b.cap = bytes;
    return hipSuccess;
}

// ------------------------------------------------------------ sweeps

// ray->voxel messages of sweep k (1..K): the last in b_ell; with checkpoints
// the earlier ones in b_ckpt (the reverse pass needs each), otherwise
// alternating between b_lam and b_ell so that sweep K-1's survive
static float* ell_slot(const mrf_ctx* c, int K, int k, bool keep)
{
    if (k == K) return (float*)c->b_ell.p;
    if (keep) return (float*)c->b_ckpt.p + (size_t)(k - 1) * (size_t)c->S;
    return ((K - k) & 1) ? (float*)c->b_lam.p : (float*)c->b_ell.p;
}

// voxel total pairs that sweep k (2..K) reads: theta plus the ray messages of sweep k-1
static float2* tot_slot(const mrf_ctx* c, int k, bool keep)
{
    return (float2*)c->b_tsum.p + (keep ? (size_t)(k - 2) * (size_t)c->V : 0);
}

// the voxel->ray messages of sweep k (1..K): lambda_e = tot[col_e] - own_e
static ExclSrc lam_src(const mrf_ctx* c, int K, int k, bool keep)
{
    if (k == 1) return ExclSrc{(const float2*)c->b_theta2.p, nullptr};   // no incoming message yet
    return ExclSrc{tot_slot(c, k, keep), ell_slot(c, K, k - 1, keep)};
}

// Everything mrf_infer enqueues after the parameter copies; capturable.
static hipError_t enqueue_forward(mrf_ctx* c, int K, int keep, bool plain, hipStream_t s)
{
    hipError_t e;
    const float* theta = (const float*)c->b_theta.p;
    if ((e = launch_pair(theta, (float2*)c->b_theta2.p, c->V, s)) != hipSuccess) return e;
    if ((e = launch_potentials(c, s)) != hipSuccess) return e;
    for (int k = 1; k <= K; ++k) {
        if (k > 1 && (e = launch_voxel_phase(c, ell_slot(c, K, k - 1, keep),
                                             VoxOut{theta, tot_slot(c, k, keep), nullptr, nullptr}, s)) != hipSuccess)
            return e;
        if ((e = launch_ray_phase(c, lam_src(c, K, k, keep), ell_slot(c, K, k, keep), plain, s)) != hipSuccess)
            return e;
    }
    if ((e = launch_copy((float*)c->b_L.p, theta, c->V, s)) != hipSuccess) return e;
    return launch_voxel_phase(c, ell_slot(c, K, K, keep), VoxOut{theta, nullptr, (float*)c->b_L.p, nullptr}, s);
}

// Per-keyframe averaged messages (Sec. IV-A): the first sweep's lambda is the
// prior (no incoming message yet); sweep k > 1 forms every keyframe's average
// of the previous sweep's ray messages per voxel (pair phase) and from them each
// keyframe's voxel -> ray message (theta plus the OTHER keyframes' averages);
// after the last sweep the beliefs L = theta plus every keyframe's average.
// ell alternates between b_lam and b_ell so that the last sweep's ends in b_ell.
// keep: the pair averages of sweeps 2..K go to b_ckpt ((K - 1) * n_pairs doubles),
// from which the reverse pass rebuilds every sweep's keyframe messages.
static hipError_t enqueue_forward_kf(mrf_ctx* c, int K, int keep, bool plain, hipStream_t s)
{
    hipError_t e;
    const float* theta = (const float*)c->b_theta.p;
    const float* w = (const float*)c->b_kfw.p;
    double* Mlast = (double*)c->b_pair_m.p;
    float* x = (float*)c->b_kfx.p;
    const KfSrc kf{x, (const int64_t*)c->b_kfxb.p};
    if ((e = launch_pair(theta, (float2*)c->b_theta2.p, c->V, s)) != hipSuccess) return e;
    if ((e = launch_potentials(c, s)) != hipSuccess) return e;
    for (int k = 1; k <= K; ++k) {
        float* ell = ell_slot(c, K, k, false);
        if (k == 1) {
            e = launch_ray_phase(c, ExclSrc{(const float2*)c->b_theta2.p, nullptr}, ell, plain, s);
        } else {
            double* M = keep ? (double*)c->b_ckpt.p + (size_t)(k - 2) * (size_t)c->n_pairs : Mlast;
            e = launch_pair_phase(c, ell_slot(c, K, k - 1, false), w, M, s);
            if (e == hipSuccess) e = launch_kf_voxel(c, M, theta, x, nullptr, s);
            if (e == hipSuccess) e = launch_ray_phase_kf(c, kf, ell, plain, s);
        }
        if (e != hipSuccess) return e;
    }
    if ((e = launch_copy((float*)c->b_L.p, theta, c->V, s)) != hipSuccess) return e;
    if ((e = launch_pair_phase(c, (const float*)c->b_ell.p, w, Mlast, s)) != hipSuccess) return e;
    return launch_kf_voxel(c, Mlast, theta, nullptr, (float*)c->b_L.p, s);
}

static const float* final_ell(const mrf_ctx* c) { return c->inferred ? (const float*)c->b_ell.p : nullptr; }

// the last sweep's voxel->ray messages
static ExclSrc final_lam(const mrf_ctx* c) { return lam_src(c, c->K, c->K, c->have_ckpt != 0); }

}  // namespace mrf

using namespace mrf;

extern "C" {

const char* mrf_strerror(int code)
{
    switch (code) {
        case MRF_OK: return "ok";
        case MRF_EINVAL: return "invalid argument";
        case MRF_ENOMEM: return "out of device memory";
        case MRF_EHIP: return "HIP runtime error";
        case MRF_ESTATE: return "call out of order";
        case MRF_ERANGE: return "size exceeds an index type";
        default: return "unknown error";
    }
}

const char* mrf_last_error(void) { return g_err.c_str(); }

int mrf_create(mrf_ctx** out)
{
    if (!out) return fail(MRF_EINVAL, "mrf_create: out is NULL");
    *out = nullptr;
    mrf_ctx* c = new (std::nothrow) mrf_ctx();
    if (!c) return fail(MRF_ENOMEM, "mrf_create: host allocation failed");
    hipError_t e = hipGetDevice(&c->device);
    // the static scratch of mrf_accuracy_static on this device: looked up once per
    // device with the device current (a failed lookup only disables that call)
    if (e == hipSuccess) static_scratch_init(c->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming);
    if (e != hipSuccess) {
        int rc = hip_fail(e, "mrf_create");
        mrf_destroy(c);
        return rc;
    }
    *out = c;
    return MRF_OK;
}

static void free_buf(DevBuf& b)
{
    if (b.p) hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

void mrf_destroy(mrf_ctx* c)
{
    if (!c) return;
    drop_graph(c);
    DevBuf* all[] = {&c->b_scenes, &c->b_frames, &c->b_counts, &c->b_rowptr, &c->b_col, &c->b_delta,
                     &c->b_bin, &c->b_tin, &c->b_tout, &c->b_g, &c->b_lam, &c->b_ell, &c->b_vedge,
                     &c->b_vptr, &c->b_theta, &c->b_theta2, &c->b_L, &c->b_thetabar, &c->b_sigma, &c->b_bias,
                     &c->b_ckpt, &c->b_tsum, &c->b_tbar, &c->b_metric, &c->b_bricks,
                     &c->b_ellbar, &c->b_lambar, &c->b_gsum, &c->b_tmp64, &c->b_cls, &c->b_sigpart,
                     &c->b_misc, &c->b_frame_list, &c->b_tiles, &c->b_tbase, &c->b_export,
                     &c->b_kfw, &c->b_kflen, &c->b_pair_m, &c->b_pair_x, &c->b_kfx, &c->b_kfxb, &c->b_kf_vox,
                     &c->b_kfxr, &c->b_kfy, &c->b_kfws};
    for (DevBuf* b : all) free_buf(*b);
    for (auto& b : c->b_host_in) free_buf(b);
    for (auto& b : c->b_pair_desc) free_buf(b);
    for (auto& b : c->b_ray_list) free_buf(b);
    for (auto& b : c->b_vox_list) free_buf(b);
    for (auto& b : c->b_vox_desc) free_buf(b);
    if (c->ev_in) hipEventDestroy(c->ev_in);
    if (c->ev_out) hipEventDestroy(c->ev_out);
    if (c->aux) hipStreamDestroy(c->aux);
    delete c;
}

int mrf_set_schedule(mrf_ctx* c, int32_t schedule)
{
    if (!c || (schedule != MRF_SCHED_PLAIN && schedule != MRF_SCHED_GRAPH))
        return fail(MRF_EINVAL, "mrf_set_schedule: bad context or schedule");
    c->schedule = schedule;
    return MRF_OK;
}

static void update_stats(mrf_ctx* c);
static int64_t sensor_cells(const std::vector<SceneDev>& scenes, int cp);
static hipError_t alloc_tables(mrf_ctx* c);

int mrf_set_sensor_cells(mrf_ctx* c, int32_t cell_px, int64_t* n_cells)
{
    if (!c || cell_px < 0 || cell_px % kTileW != 0)
        return fail(MRF_EINVAL, "mrf_set_sensor_cells: cell_px must be 0 or a positive multiple of 4");
    HCK(hipSetDevice(c->device), "mrf_set_sensor_cells: hipSetDevice");
    const int64_t n = sensor_cells(c->scenes_h, cell_px);
    if (n * kBins >= (int64_t(1) << 31)) return fail(MRF_ERANGE, "mrf_set_sensor_cells: too many regions");
    if (cell_px != c->cell_px) {
        drop_graph(c);   // the captured potentials launch depends on the table layout
        c->cell_px = cell_px;
        c->inferred = c->have_ckpt = c->kf_inferred = 0;   // the next inference reads the new layout
    }
    c->n_cells = n;
    if (!c->scenes_h.empty()) HCK(alloc_tables(c), "mrf_set_sensor_cells: alloc sensor tables");
    if (n_cells) *n_cells = c->scenes_h.empty() ? 0 : n;
    return MRF_OK;
}

int mrf_sensor_cells(const mrf_ctx* c, int32_t* cell_px, int64_t* n_cells)
{
    if (!c) return fail(MRF_EINVAL, "mrf_sensor_cells: null context");
    if (cell_px) *cell_px = c->cell_px;
    if (n_cells) *n_cells = c->scenes_h.empty() ? 0 : c->n_cells;
    return MRF_OK;
}

// Rows of the sensor tables: 1, or with per-region tables the most regions of any
// scene's image.
static int64_t sensor_cells(const std::vector<SceneDev>& scenes, int cp)
{
    if (cp <= 0) return 1;
    int64_t n = 1;
    for (const SceneDev& d : scenes) {
        const int64_t k = (int64_t)((d.W + cp - 1) / cp) * ((d.H + cp - 1) / cp);
        if (k > n) n = k;
    }
    return n;
}

// sigma and bias tables, their gradient accumulators and a scratch output table
static hipError_t alloc_tables(mrf_ctx* c)
{
    const size_t n = (size_t)table_entries(c);
    hipError_t e = ensure(c->b_sigma, sizeof(float) * n);
    if (e == hipSuccess) e = ensure(c->b_bias, sizeof(float) * n);
    if (e == hipSuccess) e = ensure(c->b_sigpart, sigpart_bytes(c) + sizeof(float) * n);
    return e;
}

// Device address of an input array of `bytes` bytes: the array itself when it is
// device memory (or host memory the device can address), otherwise a copy the
// context keeps (in b_host_in, until the next mrf_build).
static hipError_t device_view(mrf_ctx* c, const void* p, size_t bytes, const void** out, hipStream_t s)
{
    hipPointerAttribute_t a{};
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e == hipSuccess && a.type == hipMemoryTypeDevice) {
        *out = p;
        return hipSuccess;
    }
    if (e == hipSuccess && a.type == hipMemoryTypeHost && a.devicePointer) {
        *out = a.devicePointer;   // pinned and mapped
        return hipSuccess;
    }
    hipGetLastError();   // pageable host memory is not known to HIP
    DevBuf b;
    e = ensure(b, bytes);
    if (e == hipSuccess) e = hipMemcpyAsync(b.p, p, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        free_buf(b);
        return e;
    }
    c->b_host_in.push_back(b);
    *out = b.p;
    return hipSuccess;
}

// mrf_build, or with frame_slots / frame_edges (host, one entry per frame) its
// count pass alone: the per-frame slot and edge counts, and no graph.
static int build_impl(mrf_ctx* c, const mrf_scene* scenes, int32_t n_scenes, const mrf_build_params* p,
                      void* stream, int64_t* frame_slots, int64_t* frame_edges)
{
    if (!c || !scenes || !p || n_scenes < 1) return fail(MRF_EINVAL, "mrf_build: null argument or no scenes");
    if (p->min_ray_voxels < 2) return fail(MRF_EINVAL, "mrf_build: min_ray_voxels must be >= 2");
    if (!(p->table_dmax > 0.0) || !(p->z_max >= p->z_min) || !(p->trunc_nsigma >= 0.0))
        return fail(MRF_EINVAL, "mrf_build: bad depth window, truncation or table range");
    hipStream_t s = (hipStream_t)stream;
    HCK(hipSetDevice(c->device), "mrf_build: hipSetDevice");
    c->built = c->inferred = c->have_ckpt = c->kf_inferred = 0;   // a cached graph is revalidated by mrf_infer
    ++c->gen;

    c->scenes_h.clear();
    c->frames_h.clear();
    // copies of host inputs of the previous build, once this one has stopped using them
    HCK(hipStreamSynchronize(s), "mrf_build: sync");
    for (auto& b : c->b_host_in) free_buf(b);
    c->b_host_in.clear();
    c->n_scenes = n_scenes;
    int64_t R = 0, V = 0, Vk = 0, Tn = 0, NB = 0;
    if (p->sparse_bricks && (p->brick_radius < 0 || p->brick_radius > 64))
        return fail(MRF_EINVAL, "mrf_build: brick_radius must lie in [0, 64]");
    int max_hw = 0, max_tpf = 0;
    for (int i = 0; i < n_scenes; ++i) {
        const mrf_scene& sc = scenes[i];
        if (sc.n_frames < 1 || !sc.depth || !sc.T_wc) return fail(MRF_EINVAL, "mrf_build: scene without frames");
        if (sc.K.width < 1 || sc.K.height < 1 || sc.K.fx == 0.0 || sc.K.fy == 0.0)
            return fail(MRF_EINVAL, "mrf_build: bad intrinsics");
        if (sc.grid.nx < 1 || sc.grid.ny < 1 || sc.grid.nz < 1 || !(sc.grid.voxel > 0.0))
            return fail(MRF_EINVAL, "mrf_build: bad grid");
        SceneDev d{};
        d.W = sc.K.width;
        d.H = sc.K.height;
        d.fx = sc.K.fx;
        d.fy = sc.K.fy;
        d.cx = sc.K.cx;
        d.cy = sc.K.cy;
        d.n[0] = sc.grid.nx;
        d.n[1] = sc.grid.ny;
        d.n[2] = sc.grid.nz;
        d.h = sc.grid.voxel;
        for (int a = 0; a < 3; ++a) d.o[a] = sc.grid.origin[a];
        d.voxel_base = V;
        d.ray_base = R;
        for (int a = 0; a < 3; ++a) d.nb[a] = (d.n[a] + kBrick - 1) / kBrick;
        d.key_base = Vk;
        Vk += (int64_t)d.nb[0] * d.nb[1] * d.nb[2] * kBrick * kBrick * kBrick;
        d.brick_off = NB;
        NB += (int64_t)d.nb[0] * d.nb[1] * d.nb[2];
        const int64_t hw = (int64_t)d.W * d.H;
        if (hw > (int64_t(1) << 30)) return fail(MRF_ERANGE, "mrf_build: image too large");
        const void* dv = nullptr;
        const void* tv = nullptr;
        HCK(device_view(c, sc.depth, sizeof(float) * (size_t)hw * sc.n_frames, &dv, s), "mrf_build: depth input");
        HCK(device_view(c, sc.T_wc, sizeof(double) * 16 * (size_t)sc.n_frames, &tv, s), "mrf_build: pose input");
        if (hw > max_hw) max_hw = (int)hw;
        const int ntx = (d.W + kTileW - 1) / kTileW, nty = (d.H + kTileW - 1) / kTileW;
        if (ntx * nty > max_tpf) max_tpf = ntx * nty;
        for (int f = 0; f < sc.n_frames; ++f) {
            FrameDev fr{};
            fr.depth = (const float*)dv + (size_t)f * hw;
            fr.T = (const double*)tv + (size_t)f * 16;
            fr.scene = i;
            fr.ntx = ntx;
            fr.ray_base = R + (int64_t)f * hw;
            fr.tile_base = Tn + (int64_t)f * ntx * nty;
            c->frames_h.push_back(fr);
        }
        Tn += (int64_t)ntx * nty * sc.n_frames;
        R += hw * sc.n_frames;
        V += (int64_t)sc.grid.nx * sc.grid.ny * sc.grid.nz;
        c->scenes_h.push_back(d);
    }
    if (c->frames_h.size() > 65535) return fail(MRF_EINVAL, "mrf_build: more than 65535 frames");
    if (V >= (int64_t(1) << 31) || Vk >= (int64_t(1) << 32) - 1 || R >= (int64_t(1) << 31))
        return fail(MRF_ERANGE, "mrf_build: too many voxels or rays (>= 2^31)");
    c->R = R;
    c->V = V;
    c->Vk = Vk;
    c->T = Tn;
    c->n_frames = (int)c->frames_h.size();
    c->max_hw = max_hw;
    c->max_tpf = max_tpf;
    c->bp.z_min = p->z_min;
    c->bp.z_max = p->z_max;
    c->bp.nsig = p->trunc_nsigma;
    c->bp.c0 = p->trunc_c0;
    c->bp.c2 = p->trunc_c2;
    c->bp.smin = p->trunc_min;
    c->bp.dmax = p->table_dmax;
    c->bp.min_vox = p->min_ray_voxels;
    c->bp.radius = p->sparse_bricks ? p->brick_radius : 0;
    c->bp.bricks = nullptr;
    c->bp.skip = p->sparse_bricks && p->skip_empty_bricks ? 1 : 0;
    c->n_bricks = NB;
    c->keep_chords = p->keep_chords ? 1 : 0;
    c->kf = p->keyframe_average ? 1 : 0;
    c->kfws_ready = 0;
    if (p->group_slots_log2 != 0 && (p->group_slots_log2 < 12 || p->group_slots_log2 > 32))
        return fail(MRF_EINVAL, "mrf_build: group_slots_log2 must be 0 or lie in [12, 32]");
    c->group_log2 = p->group_slots_log2 ? p->group_slots_log2 : 32;
    c->n_pairs = c->n_kfx = c->n_kf_vox = 0;
    for (int k = 0; k < kVoxClasses; ++k) c->pair_cnt[k] = 0;
    c->n_cells = sensor_cells(c->scenes_h, c->cell_px);

    HCK(ensure(c->b_scenes, sizeof(SceneDev) * c->scenes_h.size()), "mrf_build: alloc");
    HCK(ensure(c->b_frames, sizeof(FrameDev) * c->frames_h.size()), "mrf_build: alloc");
    HCK(hipMemcpyAsync(c->b_scenes.p, c->scenes_h.data(), sizeof(SceneDev) * c->scenes_h.size(),
                       hipMemcpyHostToDevice, s),
        "mrf_build: upload");
    HCK(hipMemcpyAsync(c->b_frames.p, c->frames_h.data(), sizeof(FrameDev) * c->frames_h.size(),
                       hipMemcpyHostToDevice, s),
        "mrf_build: upload");
    // room for reserve_frames more frames of the last scene (mrf_add_frames)
    const int64_t reserve = p->reserve_frames > 0 ? p->reserve_frames : 0;
    const SceneDev& sl = c->scenes_h.back();
    const int64_t Rcap = R + reserve * (int64_t)sl.W * sl.H;
    const int64_t Tcap = Tn + reserve * (int64_t)((sl.W + kTileW - 1) / kTileW) * ((sl.H + kTileW - 1) / kTileW);
    HCK(ensure(c->b_counts, sizeof(int32_t) * (size_t)Rcap), "mrf_build: alloc counts");
    HCK(ensure(c->b_rowptr, sizeof(int64_t) * (size_t)(Rcap + 1)), "mrf_build: alloc row_ptr");
    const size_t sbytes = scan_tmp_bytes(R + 1);
    HCK(ensure(c->b_misc, sbytes), "mrf_build: alloc scan");
    if (p->sparse_bricks) {
        HCK(ensure(c->b_bricks, (size_t)((NB + 3) / 4) * 4), "mrf_build: alloc brick mask");
        c->bp.bricks = (const uint8_t*)c->b_bricks.p;
        HCK(launch_brick_mask(c, s), "mrf_build: brick mask");
    }
    HCK(launch_trace_count(c, s), "mrf_build: trace count");
    HCK(scan_exclusive_i32((const int32_t*)c->b_counts.p, (int64_t*)c->b_rowptr.p, R, c->b_misc.p, sbytes, s),
        "mrf_build: scan");
    int64_t E = 0;
    HCK(hipMemcpyAsync(&E, (int64_t*)c->b_rowptr.p + R, sizeof(int64_t), hipMemcpyDeviceToHost, s),
        "mrf_build: read E");
    HCK(hipStreamSynchronize(s), "mrf_build: sync");
    c->E = E;

    // tiles of 4x4 rays, slot bases = exclusive scan of 16 * longest ray
    const int64_t T = c->T;
    HCK(ensure(c->b_tiles, sizeof(TileDev) * (size_t)Tcap), "mrf_build: alloc tiles");
    HCK(ensure(c->b_tbase, sizeof(int64_t) * (size_t)(Tcap + 1)), "mrf_build: alloc tile bases");
    HCK(ensure(c->b_tmp64, sizeof(int32_t) * (size_t)(T + 1)), "mrf_build: alloc");
    const size_t tbytes = scan_tmp_bytes(T + 1);
    HCK(ensure(c->b_misc, tbytes > sbytes ? tbytes : sbytes), "mrf_build: alloc scan");
    HCK(launch_tiles(c, (int32_t*)c->b_tmp64.p, s), "mrf_build: tiles");
    HCK(scan_exclusive_i32((const int32_t*)c->b_tmp64.p, (int64_t*)c->b_tbase.p, T, c->b_misc.p, c->b_misc.cap, s),
        "mrf_build: tile scan");
    HCK(launch_tile_bases(c, s), "mrf_build: tile bases");
    int64_t S = 0;
    HCK(hipMemcpyAsync(&S, (int64_t*)c->b_tbase.p + T, sizeof(int64_t), hipMemcpyDeviceToHost, s),
        "mrf_build: read S");
    HCK(hipStreamSynchronize(s), "mrf_build: sync");
    if (frame_slots || frame_edges) {
        // count only: per-frame slots and edges, and the context keeps no graph
        c->S = S;
        const size_t nf = c->frames_h.size();
        HCK(ensure(c->b_export, 2 * sizeof(int64_t) * nf), "mrf_count: alloc");
        HCK(launch_frame_counts(c, (int64_t*)c->b_export.p, s), "mrf_count: per-frame counts");
        std::vector<int64_t> h(2 * nf);
        HCK(hipMemcpyAsync(h.data(), c->b_export.p, 2 * sizeof(int64_t) * nf, hipMemcpyDeviceToHost, s),
            "mrf_count: read counts");
        HCK(hipStreamSynchronize(s), "mrf_count: sync");
        for (size_t f = 0; f < nf; ++f) {
            if (frame_slots) frame_slots[f] = h[2 * f];
            if (frame_edges) frame_edges[f] = h[2 * f + 1];
        }
        return MRF_OK;
    }
    c->S = S;
    {
        // slot groups: runs of whole scenes with fewer than 2^group_log2 slots each; a
        // voxel's list entries hold slots relative to their group's first slot
        const size_t nf = c->frames_h.size();
        HCK(ensure(c->b_export, 2 * sizeof(int64_t) * nf), "mrf_build: alloc");
        HCK(launch_frame_counts(c, (int64_t*)c->b_export.p, s), "mrf_build: per-frame counts");
        std::vector<int64_t> h(2 * nf);
        HCK(hipMemcpyAsync(h.data(), c->b_export.p, 2 * sizeof(int64_t) * nf, hipMemcpyDeviceToHost, s),
            "mrf_build: read counts");
        HCK(hipStreamSynchronize(s), "mrf_build: sync");
        std::vector<int64_t> scene_slots(c->n_scenes, 0);
        for (size_t f = 0; f < nf; ++f) scene_slots[c->frames_h[f].scene] += h[2 * f];
        const int64_t limit = int64_t(1) << c->group_log2;
        SlotGroups g{};
        c->group_scene.assign(1, 0);
        int64_t acc = 0, first = 0;
        for (int i = 0; i < c->n_scenes; ++i) {
            if (scene_slots[i] >= limit)
                return fail(MRF_ERANGE, "mrf_build: a scene with 2^" + std::to_string(c->group_log2) +
                                            " or more edge slots");
            if (acc + scene_slots[i] >= limit) {
                if (g.n == kMaxSlotGroups)
                    return fail(MRF_ERANGE, "mrf_build: more than " + std::to_string(kMaxSlotGroups) +
                                                " groups of scenes under 2^" + std::to_string(c->group_log2) +
                                                " edge slots");
                g.slot[g.n] = first;
                c->group_scene.push_back(i);
                ++g.n;
                acc = 0;
            }
            acc += scene_slots[i];
            first += scene_slots[i];
        }
        if (c->kf && g.n > 1)
            return fail(MRF_ERANGE, "mrf_build: per-keyframe averages need fewer than 2^" +
                                        std::to_string(c->group_log2) + " edge slots");
        c->sg = g;
    }

    // per-slot arrays, with room for the reserved frames at 1.25 times the batch's mean
    // slots per frame
    const int64_t Scap = S + (5 * reserve * S + 4 * c->n_frames - 1) / (4 * c->n_frames);
    const size_t e1 = (size_t)(Scap > 0 ? Scap : 1);
    const size_t e4 = sizeof(float) * e1;
    HCK(ensure(c->b_col, e4), "mrf_build: alloc col");
    HCK(ensure(c->b_delta, e4), "mrf_build: alloc delta");
    HCK(ensure(c->b_bin, e1), "mrf_build: alloc bin");
    HCK(ensure(c->b_g, e4), "mrf_build: alloc g");
    // one entry more: the keyframe-pair build keeps an exclusive count of E + 1 entries in each
    HCK(ensure(c->b_lam, e4 + 16), "mrf_build: alloc lam");
    HCK(ensure(c->b_ell, e4 + 16), "mrf_build: alloc ell");
    HCK(ensure(c->b_vedge, e4 + 16), "mrf_build: alloc vedge");
    HCK(ensure(c->b_ellbar, e4), "mrf_build: alloc ellbar");
    HCK(ensure(c->b_lambar, e4), "mrf_build: alloc lambar");
    HCK(ensure(c->b_gsum, e4), "mrf_build: alloc gsum");
    if (c->kf) HCK(ensure(c->b_kflen, e4), "mrf_build: alloc chord lengths");
    if (c->keep_chords) {
        HCK(ensure(c->b_tin, 2 * e4), "mrf_build: alloc t_in");
        HCK(ensure(c->b_tout, 2 * e4), "mrf_build: alloc t_out");
    }
    HCK(ensure(c->b_vptr, sizeof(int64_t) * (size_t)(Vk + 1)), "mrf_build: alloc vptr");
    const size_t vb = sizeof(float) * (size_t)V;
    HCK(ensure(c->b_theta, vb), "mrf_build: alloc theta");
    HCK(ensure(c->b_L, vb), "mrf_build: alloc L");
    HCK(ensure(c->b_thetabar, vb), "mrf_build: alloc thetabar");
    HCK(ensure(c->b_theta2, 2 * vb), "mrf_build: alloc theta pairs");
    HCK(ensure(c->b_tbar, 3 * 2 * vb), "mrf_build: alloc voxel sums");
    HCK(alloc_tables(c), "mrf_build: alloc sensor tables");

    // every slot is written: edges by the traversal, the rest as padding (no voxel,
    // no bin, sort key past every voxel)
    HCK(launch_trace_emit(c, s), "mrf_build: trace emit");

    // voxel -> ray incidence by a stable LSD radix sort of (brick-major voxel key,
    // slot); the emit pass left the keys in the potentials buffer, and the
    // message buffers are free during build and hold the sort's ping-pong
    const int64_t nh = (int64_t)radix_hist_entries(S);
    HCK(ensure(c->b_tmp64, sizeof(int64_t) * (size_t)(nh + 1) + sizeof(int32_t) * (size_t)nh),
        "mrf_build: alloc sort tables");
    int64_t* offs = (int64_t*)c->b_tmp64.p;
    int32_t* hist = (int32_t*)(offs + nh + 1);
    const size_t sb2 = radix_tmp_bytes(S);
    HCK(ensure(c->b_misc, sb2 > c->b_misc.cap ? sb2 : c->b_misc.cap), "mrf_build: alloc sort scan");
    HCK(radix_sort_pairs((const uint32_t*)c->b_g.p, (uint32_t*)c->b_lam.p, (uint32_t*)c->b_ell.p,
                         (uint32_t*)c->b_ellbar.p, (uint32_t*)c->b_gsum.p, (uint32_t*)c->b_lambar.p,
                         (uint32_t*)c->b_vedge.p, S, bits_for(Vk), hist, offs, c->b_misc.p, c->b_misc.cap, s, c->sg),
        "mrf_build: radix sort");
    HCK(launch_vptr_from_sorted((const uint32_t*)c->b_lambar.p, S, Vk, (int64_t*)c->b_vptr.p, s),
        "mrf_build: vptr");
    for (int g = 1; g < c->sg.n; ++g) {   // list position of each group's first key
        const int64_t k0 = c->scenes_h[c->group_scene[g]].key_base;
        HCK(hipMemcpyAsync(&c->sg.pos[g], (const int64_t*)c->b_vptr.p + k0, sizeof(int64_t), hipMemcpyDeviceToHost,
                           s),
            "mrf_build: group positions");
    }
    HCK(hipStreamSynchronize(s), "mrf_build: sync");
    {
        hipError_t e = build_classes(c, s);
        if (e == hipErrorInvalidConfiguration) return fail(MRF_ERANGE, "mrf_build: " + g_err);
        HCK(e, "mrf_build: work lists");
    }
    if (c->kf) {
        hipError_t e = build_keyframe_pairs(c, s);
        if (e == hipErrorInvalidConfiguration) return fail(MRF_ERANGE, "mrf_build: " + g_err);
        HCK(e, "mrf_build: keyframe pairs");
    }
    HCK(hipStreamSynchronize(s), "mrf_build: sync");

    update_stats(c);
    c->built = 1;
    return MRF_OK;
}

// sizes, histograms (set by build_classes) and bytes per sweep of the built graph
static void update_stats(mrf_ctx* c)
{
    mrf_stats_t& st = c->stats;
    const int64_t E = c->E;
    st.n_scenes = c->n_scenes;
    st.n_rays = c->R;
    st.n_edges = E;
    st.n_voxels = c->V;
    st.n_kept_rays = 0;
    for (int k = 0; k < kRayClasses; ++k) st.n_kept_rays += c->ray_cls_rays[k];
    st.n_slots = c->S;
    st.n_slot_groups = c->sg.n;
    st.n_tiles = c->T;
    st.n_touched_voxels = 0;
    for (int k = 0; k < kVoxClasses; ++k) st.n_touched_voxels += c->vox_cnt[k];
    // voxel phase: vedge 4 + gathered ell 4 per edge, descriptor 16 + theta 4 + total 4 per
    // touched voxel; ray phase: col 4 + own ell 4 + g 4 + ell 4 per edge, total 4 per touched
    // voxel, count 4 per kept ray, list 4 + descriptor 32 per tile
    st.fwd_bytes_per_sweep =
        24.0 * (double)E + 28.0 * (double)st.n_touched_voxels + 4.0 * (double)st.n_kept_rays + 36.0 * (double)c->T;
    st.sweeps_done = 0;
    st.have_checkpoints = 0;
    st.n_keyframe_pairs = c->n_pairs;
}

int mrf_build(mrf_ctx* c, const mrf_scene* scenes, int32_t n_scenes, const mrf_build_params* p, void* stream)
{
    return build_impl(c, scenes, n_scenes, p, stream, nullptr, nullptr);
}

int mrf_count(mrf_ctx* c, const mrf_scene* scenes, int32_t n_scenes, const mrf_build_params* p,
              int64_t* frame_slots, int64_t* frame_edges, void* stream)
{
    if (!frame_slots && !frame_edges) return fail(MRF_EINVAL, "mrf_count: no output");
    return build_impl(c, scenes, n_scenes, p, stream, frame_slots, frame_edges);
}

// Grows b to hold `need` bytes, keeping its first `keep` bytes; a buffer that has
// to move gets room for four more additions of the same size (at most doubling
// it), so that frames added one at a time reallocate rarely.
static hipError_t grow_keep(DevBuf& b, size_t need, size_t keep, hipStream_t s)
{
    if (need == 0) need = 16;
    if (b.p && b.cap >= need) return hipSuccess;
    const size_t grown = with_room(need, keep);
    void* p = nullptr;
    size_t got = grown;
    hipError_t e = hipMalloc(&p, grown);
    if (e != hipSuccess) {   // without the extra room
        hipGetLastError();
        got = need;
        e = hipMalloc(&p, need);
    }
    if (e != hipSuccess) {
        hipGetLastError();
        return e;
    }
    if (b.p && keep > 0) e = hipMemcpyAsync(p, b.p, keep < b.cap ? keep : b.cap, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        hipFree(p);
        return e;
    }
    if (b.p) hipFree(b.p);
    b.p = p;
    b.cap = got;
    return hipSuccess;
}

int mrf_add_frames(mrf_ctx* c, int32_t n_frames, const float* depth, const double* T_wc, void* stream)
{
    if (!c || n_frames < 1 || !depth || !T_wc) return fail(MRF_EINVAL, "mrf_add_frames: null argument or no frames");
    if (!c->built) return fail(MRF_ESTATE, "mrf_add_frames: call mrf_build first");
    if (c->bp.bricks)
        return fail(MRF_EINVAL, "mrf_add_frames: a sparse grid's bricks depend on every frame; rebuild instead");
    if (c->frames_h.size() + (size_t)n_frames > 65535) return fail(MRF_EINVAL, "mrf_add_frames: more than 65535 frames");
    struct GrowRoom {
        GrowRoom() { g_grow_room = 1; }
        ~GrowRoom() { g_grow_room = 0; }
    } grow_room;
    hipStream_t s = (hipStream_t)stream;
    HCK(hipSetDevice(c->device), "mrf_add_frames: hipSetDevice");
    drop_graph(c);
    c->built = c->inferred = c->have_ckpt = c->kf_inferred = 0;
    c->kfws_ready = 0;
    ++c->gen;

    const int last = c->n_scenes - 1;
    const SceneDev& sd = c->scenes_h[last];
    const int64_t hw = (int64_t)sd.W * sd.H;
    const int ntx = (sd.W + kTileW - 1) / kTileW, nty = (sd.H + kTileW - 1) / kTileW;
    const int f0 = c->n_frames;
    const int64_t R0 = c->R, T0 = c->T, S0 = c->S, E0 = c->E;
    const int64_t R1 = R0 + hw * n_frames, T1 = T0 + (int64_t)ntx * nty * n_frames;
    if (R1 >= (int64_t(1) << 31)) return fail(MRF_ERANGE, "mrf_add_frames: too many rays (>= 2^31)");
    const void* dv = nullptr;
    const void* tv = nullptr;
    HCK(device_view(c, depth, sizeof(float) * (size_t)hw * n_frames, &dv, s), "mrf_add_frames: depth input");
    HCK(device_view(c, T_wc, sizeof(double) * 16 * (size_t)n_frames, &tv, s), "mrf_add_frames: pose input");
    for (int f = 0; f < n_frames; ++f) {
        FrameDev fr{};
        fr.depth = (const float*)dv + (size_t)f * hw;
        fr.T = (const double*)tv + (size_t)f * 16;
        fr.scene = last;
        fr.ntx = ntx;
        fr.ray_base = R0 + (int64_t)f * hw;
        fr.tile_base = T0 + (int64_t)f * ntx * nty;
        c->frames_h.push_back(fr);
    }
    c->n_frames = (int)c->frames_h.size();
    c->R = R1;
    c->T = T1;
    HCK(grow_keep(c->b_frames, sizeof(FrameDev) * c->frames_h.size(), 0, s), "mrf_add_frames: alloc frames");
    HCK(hipMemcpyAsync(c->b_frames.p, c->frames_h.data(), sizeof(FrameDev) * c->frames_h.size(),
                       hipMemcpyHostToDevice, s),
        "mrf_add_frames: upload");

    // rays of the new frames: counts, then row_ptr[R0..R1] = E0 + their exclusive scan
    HCK(grow_keep(c->b_counts, sizeof(int32_t) * (size_t)R1, sizeof(int32_t) * (size_t)R0, s), "mrf_add_frames: alloc");
    HCK(grow_keep(c->b_rowptr, sizeof(int64_t) * (size_t)(R1 + 1), sizeof(int64_t) * (size_t)(R0 + 1), s),
        "mrf_add_frames: alloc");
    size_t sb = scan_tmp_bytes(R1 - R0 + 1);
    HCK(ensure(c->b_misc, sb > c->b_misc.cap ? sb : c->b_misc.cap), "mrf_add_frames: alloc scan");
    HCK(launch_trace_count(c, s, f0, n_frames), "mrf_add_frames: trace count");
    HCK(scan_exclusive_i32((const int32_t*)c->b_counts.p + R0, (int64_t*)c->b_rowptr.p + R0, R1 - R0, c->b_misc.p,
                           c->b_misc.cap, s),
        "mrf_add_frames: scan");
    HCK(launch_add_i64((int64_t*)c->b_rowptr.p + R0, E0, R1 - R0 + 1, s), "mrf_add_frames: scan");
    int64_t E1 = 0;
    HCK(hipMemcpyAsync(&E1, (int64_t*)c->b_rowptr.p + R1, sizeof(int64_t), hipMemcpyDeviceToHost, s), "read E");
    HCK(hipStreamSynchronize(s), "mrf_add_frames: sync");
    c->E = E1;

    // tiles of the new frames, slot bases after every existing slot
    HCK(grow_keep(c->b_tiles, sizeof(TileDev) * (size_t)T1, sizeof(TileDev) * (size_t)T0, s), "mrf_add_frames: alloc");
    HCK(grow_keep(c->b_tbase, sizeof(int64_t) * (size_t)(T1 + 1), sizeof(int64_t) * (size_t)(T0 + 1), s),
        "mrf_add_frames: alloc");
    HCK(ensure(c->b_tmp64, sizeof(int32_t) * (size_t)(T1 - T0 + 1)), "mrf_add_frames: alloc");
    sb = scan_tmp_bytes(T1 - T0 + 1);
    HCK(ensure(c->b_misc, sb > c->b_misc.cap ? sb : c->b_misc.cap), "mrf_add_frames: alloc scan");
    HCK(launch_tiles(c, (int32_t*)c->b_tmp64.p, s, f0, n_frames), "mrf_add_frames: tiles");
    HCK(scan_exclusive_i32((const int32_t*)c->b_tmp64.p, (int64_t*)c->b_tbase.p + T0, T1 - T0, c->b_misc.p,
                           c->b_misc.cap, s),
        "mrf_add_frames: tile scan");
    HCK(launch_add_i64((int64_t*)c->b_tbase.p + T0, S0, T1 - T0 + 1, s), "mrf_add_frames: tile scan");
    HCK(launch_tile_bases(c, s, T0), "mrf_add_frames: tile bases");
    int64_t S1 = 0;
    HCK(hipMemcpyAsync(&S1, (int64_t*)c->b_tbase.p + T1, sizeof(int64_t), hipMemcpyDeviceToHost, s), "read S");
    HCK(hipStreamSynchronize(s), "mrf_add_frames: sync");
    const int64_t gb = c->sg.slot[c->sg.n - 1];   // the last scene's group
    if (S1 - gb >= (int64_t(1) << c->group_log2))
        return fail(MRF_ERANGE, "mrf_add_frames: the last scene's group would reach 2^" +
                                    std::to_string(c->group_log2) + " edge slots");
    c->S = S1;

    // per-slot arrays: the existing slots are kept, the new ones written by the emit pass
    const size_t k4 = sizeof(float) * (size_t)S0, e4 = sizeof(float) * (size_t)S1;
    HCK(grow_keep(c->b_col, e4, k4, s), "mrf_add_frames: alloc col");
    HCK(grow_keep(c->b_delta, e4, k4, s), "mrf_add_frames: alloc delta");
    HCK(grow_keep(c->b_bin, (size_t)S1, (size_t)S0, s), "mrf_add_frames: alloc bin");
    if (c->keep_chords) {
        HCK(grow_keep(c->b_tin, 2 * e4, 2 * k4, s), "mrf_add_frames: alloc t_in");
        HCK(grow_keep(c->b_tout, 2 * e4, 2 * k4, s), "mrf_add_frames: alloc t_out");
    }
    if (c->kf) HCK(grow_keep(c->b_kflen, e4, k4, s), "mrf_add_frames: alloc chord lengths");
    HCK(grow_keep(c->b_vedge, e4 + 16, sizeof(uint32_t) * (size_t)E0, s), "mrf_add_frames: alloc vedge");
    // message and scratch arrays: the old messages are stale once frames are added
    HCK(ensure(c->b_g, e4), "mrf_add_frames: alloc");
    HCK(ensure(c->b_lam, e4 + 16), "mrf_add_frames: alloc");
    HCK(ensure(c->b_ell, e4 + 16), "mrf_add_frames: alloc");
    HCK(ensure(c->b_ellbar, e4), "mrf_add_frames: alloc");
    HCK(ensure(c->b_lambar, e4), "mrf_add_frames: alloc");
    HCK(ensure(c->b_gsum, e4), "mrf_add_frames: alloc");
    HCK(launch_trace_emit(c, s, f0, n_frames), "mrf_add_frames: trace emit");

    // the new slots sorted by voxel key on their own (keys were left in b_g), then merged
    // behind each voxel's existing entries
    const int64_t n1 = S1 - S0;
    const int64_t nh = (int64_t)radix_hist_entries(n1);
    HCK(ensure(c->b_tmp64, sizeof(int64_t) * (size_t)(nh + 1) + sizeof(int32_t) * (size_t)nh),
        "mrf_add_frames: alloc sort tables");
    int64_t* offs = (int64_t*)c->b_tmp64.p;
    int32_t* hist = (int32_t*)(offs + nh + 1);
    sb = radix_tmp_bytes(n1);
    HCK(ensure(c->b_misc, sb > c->b_misc.cap ? sb : c->b_misc.cap), "mrf_add_frames: alloc sort scan");
    uint32_t* nkeys = (uint32_t*)c->b_lambar.p;   // sorted new keys
    uint32_t* nvals = (uint32_t*)c->b_gsum.p;     // their slots less S0
    // temporaries in b_export: the new keys' vptr (Vk + 1 int64), then the sort's spare values
    const size_t vpb = sizeof(int64_t) * (size_t)(c->Vk + 1);
    hipError_t e = ensure(c->b_export, vpb + sizeof(uint32_t) * (size_t)n1 + 64);
    int64_t* nvptr = (int64_t*)c->b_export.p;
    uint32_t* vals_b = (uint32_t*)((char*)c->b_export.p + (vpb + 63) / 64 * 64);
    if (e == hipSuccess)
        e = radix_sort_pairs((const uint32_t*)c->b_g.p + S0, (uint32_t*)c->b_lam.p, (uint32_t*)c->b_ell.p,
                             (uint32_t*)c->b_ellbar.p, vals_b, nkeys, nvals, n1, bits_for(c->Vk), hist, offs,
                             c->b_misc.p, c->b_misc.cap, s);
    if (e == hipSuccess) e = launch_vptr_from_sorted(nkeys, n1, c->Vk, nvptr, s);
    uint32_t* okeys = (uint32_t*)c->b_ell.p;      // keys of the existing entries
    uint32_t* merged = (uint32_t*)c->b_lam.p;
    if (e == hipSuccess) e = launch_entry_keys(c, (const uint32_t*)c->b_vedge.p, E0, okeys, s);
    if (e == hipSuccess)
        e = launch_merge_incidence((const uint32_t*)c->b_vedge.p, okeys, E0, nvals, nkeys, E1 - E0,
                                   (uint32_t)(S0 - gb), (int64_t*)c->b_vptr.p, nvptr, c->Vk + 1, merged, s);
    HCK(e, "mrf_add_frames: sort and merge");
    std::swap(c->b_vedge, c->b_lam);
    // padding entries past E (their key is past every voxel) keep the list's tail defined
    HCK(launch_fill_u32((uint32_t*)c->b_vedge.p + E1, 0u, S1 - E1, s), "mrf_add_frames: fill");
    {
        hipError_t e2 = build_classes(c, s);
        if (e2 == hipErrorInvalidConfiguration) return fail(MRF_ERANGE, "mrf_add_frames: " + g_err);
        HCK(e2, "mrf_add_frames: work lists");
    }
    if (c->kf) {
        HCK(launch_entry_keys(c, (const uint32_t*)c->b_vedge.p, E1, (uint32_t*)c->b_lambar.p, s),
            "mrf_add_frames: keys");
        hipError_t e2 = build_keyframe_pairs(c, s);
        if (e2 == hipErrorInvalidConfiguration) return fail(MRF_ERANGE, "mrf_add_frames: " + g_err);
        HCK(e2, "mrf_add_frames: keyframe pairs");
    }
    HCK(hipStreamSynchronize(s), "mrf_add_frames: sync");
    update_stats(c);
    c->built = 1;
    return MRF_OK;
}

int mrf_infer(mrf_ctx* c, const float* prior_logit, const float* sigma_table, int32_t sweeps,
              int32_t keep_checkpoints, void* stream)
{
    return mrf_infer_sensor(c, prior_logit, sigma_table, nullptr, sweeps, keep_checkpoints, stream);
}

int mrf_infer_sensor(mrf_ctx* c, const float* prior_logit, const float* sigma_table, const float* bias_table,
                     int32_t sweeps, int32_t keep_checkpoints, void* stream)
{
    if (!c || !prior_logit || !sigma_table) return fail(MRF_EINVAL, "mrf_infer: null argument");
    if (!c->built) return fail(MRF_ESTATE, "mrf_infer: call mrf_build first");
    if (sweeps < 1) return fail(MRF_EINVAL, "mrf_infer: sweeps must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    HCK(hipSetDevice(c->device), "mrf_infer: hipSetDevice");
    const int keep = keep_checkpoints ? 1 : 0;
    {
        // checkpoints: ell of sweeps 1..K-1 and the voxel total pairs of sweeps 2..K
        const size_t need_ell = keep ? sizeof(float) * (size_t)(sweeps - 1) * (size_t)c->S : 0;
        const size_t need_tot = sizeof(float2) * (size_t)(keep && sweeps > 2 ? sweeps - 1 : 1) * (size_t)c->V;
        if (c->b_ckpt.cap < need_ell || c->b_tsum.cap < need_tot) {
            drop_graph(c);   // the graph holds the old addresses
            HCK(ensure(c->b_ckpt, need_ell), "mrf_infer: alloc checkpoints");
            HCK(ensure(c->b_tsum, need_tot), "mrf_infer: alloc voxel totals");
        }
    }
    HCK(launch_copy((float*)c->b_theta.p, prior_logit, c->V, s), "mrf_infer: copy prior");
    HCK(launch_copy((float*)c->b_sigma.p, sigma_table, table_entries(c), s), "mrf_infer: copy sigma");
    if (bias_table)
        HCK(launch_copy((float*)c->b_bias.p, bias_table, table_entries(c), s), "mrf_infer: copy bias");
    else
        HCK(launch_fill((float*)c->b_bias.p, 0.0f, table_entries(c), s), "mrf_infer: zero bias");
    if (c->schedule == MRF_SCHED_PLAIN) {
        HCK(enqueue_forward(c, sweeps, keep, true, s), "mrf_infer: sweeps");
    } else {
        std::vector<uint64_t> key = graph_key(c, sweeps, keep);
        if (!c->gexec || key != c->g_key) {
            drop_graph(c);
            hipGraph_t g = nullptr;
            HCK(hipStreamBeginCapture(c->aux, hipStreamCaptureModeThreadLocal), "mrf_infer: begin capture");
            hipError_t e = enqueue_forward(c, sweeps, keep, false, c->aux);
            hipError_t e2 = hipStreamEndCapture(c->aux, &g);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
            if (g) hipGraphDestroy(g);
            if (e != hipSuccess) {
                c->gexec = nullptr;
                return hip_fail(e, "mrf_infer: graph capture");
            }
            c->g_K = sweeps;
            c->g_ckpt = keep;
            c->g_key = key;
        }
        HCK(hipEventRecord(c->ev_in, s), "mrf_infer: event");
        HCK(hipStreamWaitEvent(c->aux, c->ev_in, 0), "mrf_infer: wait");
        HCK(hipGraphLaunch(c->gexec, c->aux), "mrf_infer: graph launch");
        HCK(hipEventRecord(c->ev_out, c->aux), "mrf_infer: event");
        HCK(hipStreamWaitEvent(s, c->ev_out, 0), "mrf_infer: wait");
    }
    c->inferred = 1;
    c->kf_inferred = 0;
    ++c->gen;
    c->K = sweeps;
    c->have_ckpt = keep;
    c->stats.sweeps_done = sweeps;
    c->stats.have_checkpoints = keep;
    return MRF_OK;
}

int mrf_infer_keyframe_avg(mrf_ctx* c, const float* prior_logit, const float* sigma_table, const float* bias_table,
                           int32_t sweeps, int32_t keep_checkpoints, void* stream)
{
    if (!c || !prior_logit || !sigma_table) return fail(MRF_EINVAL, "mrf_infer_keyframe_avg: null argument");
    if (!c->built) return fail(MRF_ESTATE, "mrf_infer_keyframe_avg: call mrf_build first");
    if (!c->kf)
        return fail(MRF_ESTATE, "mrf_infer_keyframe_avg: the graph was built without keyframe_average");
    if (sweeps < 1) return fail(MRF_EINVAL, "mrf_infer_keyframe_avg: sweeps must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    HCK(hipSetDevice(c->device), "mrf_infer_keyframe_avg: hipSetDevice");
    const int keep = keep_checkpoints ? 1 : 0;
    if (keep) {   // the pair averages of sweeps 2..K
        const size_t need = sizeof(double) * (size_t)(sweeps > 1 ? sweeps - 1 : 1) * (size_t)c->n_pairs;
        if (c->b_ckpt.cap < need) {
            drop_graph(c);   // the graph holds the old address
            HCK(ensure(c->b_ckpt, need), "mrf_infer_keyframe_avg: alloc checkpoints");
        }
    }
    HCK(launch_copy((float*)c->b_theta.p, prior_logit, c->V, s), "mrf_infer_keyframe_avg: copy prior");
    HCK(launch_copy((float*)c->b_sigma.p, sigma_table, table_entries(c), s), "mrf_infer_keyframe_avg: copy sigma");
    if (bias_table)
        HCK(launch_copy((float*)c->b_bias.p, bias_table, table_entries(c), s), "mrf_infer_keyframe_avg: copy bias");
    else
        HCK(launch_fill((float*)c->b_bias.p, 0.0f, table_entries(c), s), "mrf_infer_keyframe_avg: zero bias");
    if (c->schedule == MRF_SCHED_PLAIN) {
        HCK(enqueue_forward_kf(c, sweeps, keep, true, s), "mrf_infer_keyframe_avg: sweeps");
    } else {
        std::vector<uint64_t> key = graph_key(c, sweeps, keep);
        key.push_back(0x6b66);   // the keyframe-average schedule
        if (!c->gexec || key != c->g_key) {
            drop_graph(c);
            hipGraph_t g = nullptr;
            HCK(hipStreamBeginCapture(c->aux, hipStreamCaptureModeThreadLocal),
                "mrf_infer_keyframe_avg: begin capture");
            hipError_t e = enqueue_forward_kf(c, sweeps, keep, false, c->aux);
            hipError_t e2 = hipStreamEndCapture(c->aux, &g);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
            if (g) hipGraphDestroy(g);
            if (e != hipSuccess) {
                c->gexec = nullptr;
                return hip_fail(e, "mrf_infer_keyframe_avg: graph capture");
            }
            c->g_K = sweeps;
            c->g_ckpt = keep;
            c->g_key = key;
        }
        HCK(hipEventRecord(c->ev_in, s), "mrf_infer_keyframe_avg: event");
        HCK(hipStreamWaitEvent(c->aux, c->ev_in, 0), "mrf_infer_keyframe_avg: wait");
        HCK(hipGraphLaunch(c->gexec, c->aux), "mrf_infer_keyframe_avg: graph launch");
        HCK(hipEventRecord(c->ev_out, c->aux), "mrf_infer_keyframe_avg: event");
        HCK(hipStreamWaitEvent(s, c->ev_out, 0), "mrf_infer_keyframe_avg: wait");
    }
    c->inferred = 1;
    c->kf_inferred = 1;
    ++c->gen;
    c->K = sweeps;
    c->have_ckpt = keep;
    c->stats.sweeps_done = sweeps;
    c->stats.have_checkpoints = keep;
    return MRF_OK;
}

int mrf_marginals(mrf_ctx* c, float* p, float* logit, void* stream)
{
    if (!c) return fail(MRF_EINVAL, "mrf_marginals: null context");
    if (!c->inferred) return fail(MRF_ESTATE, "mrf_marginals: call mrf_infer first");
    hipStream_t s = (hipStream_t)stream;
    if (p) HCK(launch_sigmoid((const float*)c->b_L.p, p, c->V, s), "mrf_marginals");
    if (logit) HCK(launch_copy(logit, (const float*)c->b_L.p, c->V, s), "mrf_marginals");
    return MRF_OK;
}

// Reverse pass through K sweeps with per-keyframe averaged messages (as in the
// oracle's or_backward_keyframe_avg): y holds, per (keyframe, voxel) pair, the
// derivative reaching the pair's average (seed: d/d L_v), an edge's d/d ell is
// its share of the pair's weight times y, and each sweep rebuilds its keyframe
// messages from the checkpointed pair averages.  d/d theta accumulates in
// b_thetabar, d/d g in b_gsum.
static hipError_t backward_kf(mrf_ctx* c, const float* dlogit, hipStream_t s)
{
    const int K = c->K;
    const size_t nx = (size_t)(c->n_kfx > 0 ? c->n_kfx : 1);
    hipError_t e = ensure(c->b_kfxr, sizeof(float) * nx);
    if (e == hipSuccess) e = ensure(c->b_kfy, sizeof(float) * nx);
    if (e == hipSuccess && !c->kfws_ready) {   // per-slot pair weights, once per build
        e = ensure(c->b_kfws, sizeof(float) * (size_t)(c->S > 0 ? c->S : 1));
        if (e == hipSuccess) e = launch_fill((float*)c->b_kfws.p, 0.0f, c->S, s);
        if (e == hipSuccess)
            e = launch_scatter_by_slot((const uint32_t*)c->b_vedge.p, (const float*)c->b_kfw.p, c->E,
                                       (float*)c->b_kfws.p, s);
        if (e == hipSuccess) c->kfws_ready = 1;
    }
    if (e != hipSuccess) return e;
    float* thetabar = (float*)c->b_thetabar.p;
    float* xr = (float*)c->b_kfxr.p;
    float* y = (float*)c->b_kfy.p;
    double* sp = (double*)c->b_pair_m.p;   // pair sums of d/d lambda (scratch)
    const int64_t* xb = (const int64_t*)c->b_kfxb.p;
    const float* theta = (const float*)c->b_theta.p;
    if ((e = launch_copy(thetabar, dlogit, c->V, s)) != hipSuccess) return e;
    // seed: the last sweep's messages reach L_v through their pair averages
    if ((e = launch_kf_voxel(c, nullptr, dlogit, y, nullptr, s)) != hipSuccess) return e;
    for (int k = K; k >= 1 && e == hipSuccess; --k) {
        const double* M = k >= 2 ? (const double*)c->b_ckpt.p + (size_t)(k - 2) * (size_t)c->n_pairs : nullptr;
        e = launch_kf_voxel(c, M, theta, xr, nullptr, s);   // the keyframe messages of sweep k
        if (e == hipSuccess)
            e = launch_ray_adjoint_kf(c, AdjKf{KfSrc{xr, xb}, y, (const float*)c->b_kfws.p}, (float*)c->b_lambar.p,
                                      (float*)c->b_gsum.p, k == K, s);
        if (e == hipSuccess) e = launch_pair_phase(c, (const float*)c->b_lambar.p, nullptr, sp, s);
        if (e == hipSuccess) e = launch_kf_voxel_rev(c, sp, thetabar, k > 1 ? y : nullptr, s);
    }
    return e;
}

int mrf_backward(mrf_ctx* c, const float* dlogit, float* dprior, float* dsigma, void* stream)
{
    return mrf_backward_sensor(c, dlogit, dprior, dsigma, nullptr, stream);
}

int mrf_backward_sensor(mrf_ctx* c, const float* dlogit, float* dprior, float* dsigma, float* dbias, void* stream)
{
    if (!c || !dlogit) return fail(MRF_EINVAL, "mrf_backward: null argument");
    if (!c->inferred || !c->have_ckpt)
        return fail(MRF_ESTATE, "mrf_backward: needs a preceding mrf_infer with keep_checkpoints");
    hipStream_t s = (hipStream_t)stream;
    HCK(hipSetDevice(c->device), "mrf_backward: hipSetDevice");
    if (c->kf_inferred) {
        HCK(backward_kf(c, dlogit, s), "mrf_backward: reverse sweeps with keyframe averages");
        if (dsigma || dbias) HCK(launch_sigma_grad(c, dsigma, dbias, s), "mrf_backward: sensor-table gradients");
        if (dprior) HCK(launch_copy(dprior, (const float*)c->b_thetabar.p, c->V, s), "mrf_backward: copy");
        return MRF_OK;
    }
    const int K = c->K;
    float* gsum = (float*)c->b_gsum.p;
    float* thetabar = (float*)c->b_thetabar.p;
    float2* tbar = (float2*)c->b_tbar.p;
    float2* seed = tbar + c->V;
    float* lbuf[2] = {(float*)c->b_lambar.p, (float*)c->b_ellbar.p};
    // d loss / d theta starts at d loss / d L; d loss / d ell^(K)_e = d loss / d L_v(e)
    HCK(launch_copy(thetabar, dlogit, c->V, s), "mrf_backward: seed");
    HCK(launch_pair(dlogit, seed, c->V, s), "mrf_backward: seed");
    ExclSrc eb{seed, nullptr};
    hipError_t e = hipSuccess;
    for (int k = K; k >= 1 && e == hipSuccess; --k) {
        // sweep k: d/d lambda^(k) from the ray adjoint, then its per-voxel sums, which
        // give d/d theta and (less the edge's own) d/d ell^(k-1)
        float* lb = lbuf[(K - k) & 1];
        e = launch_ray_adjoint(c, lam_src(c, K, k, true), eb, lb, gsum, k == K, s);
        if (e == hipSuccess) e = launch_voxel_phase(c, lb, VoxOut{nullptr, k > 1 ? tbar : nullptr, nullptr, thetabar}, s);
        eb = ExclSrc{tbar, lb};
    }
    HCK(e, "mrf_backward: sweeps");
    if (dsigma || dbias) HCK(launch_sigma_grad(c, dsigma, dbias, s), "mrf_backward: sensor-table gradients");
    if (dprior) HCK(launch_copy(dprior, thetabar, c->V, s), "mrf_backward: copy");
    return MRF_OK;
}

int mrf_generation(const mrf_ctx* c, uint64_t* out)
{
    if (!c || !out) return fail(MRF_EINVAL, "mrf_generation: null argument");
    *out = c->gen;
    return MRF_OK;
}

int mrf_backward_gen(mrf_ctx* c, uint64_t generation, const float* dlogit, float* dprior, float* dsigma,
                     float* dbias, void* stream)
{
    if (!c) return fail(MRF_EINVAL, "mrf_backward_gen: null context");
    if (generation != c->gen)
        return fail(MRF_ESTATE, "mrf_backward_gen: the inference to differentiate was replaced by a later "
                                "mrf_infer or mrf_build on this context");
    return mrf_backward_sensor(c, dlogit, dprior, dsigma, dbias, stream);
}

int mrf_accuracy(mrf_ctx* c, const float* logit, double vis_min, int8_t* ray_code, double* surface_depth,
                 int64_t* counts, void* stream)
{
    if (!c) return fail(MRF_EINVAL, "mrf_accuracy: null context");
    if (!c->built) return fail(MRF_ESTATE, "mrf_accuracy: call mrf_build first");
    if (!(vis_min > 0.0 && vis_min <= 1.0)) return fail(MRF_EINVAL, "mrf_accuracy: vis_min must lie in (0, 1]");
    if (!logit) {
        if (!c->inferred) return fail(MRF_ESTATE, "mrf_accuracy: no map given and no mrf_infer yet");
        logit = (const float*)c->b_L.p;
    }
    hipStream_t s = (hipStream_t)stream;
    HCK(hipSetDevice(c->device), "mrf_accuracy: hipSetDevice");
    HCK(ensure(c->b_metric, 2 * sizeof(double) * (size_t)c->V), "mrf_accuracy: alloc");
    HCK(launch_accuracy(c, logit, vis_min, nullptr, 0.0, ray_code, surface_depth, counts, (double*)c->b_metric.p, s),
        "mrf_accuracy");
    return MRF_OK;
}

int mrf_accuracy_ex(mrf_ctx* c, const float* logit, double vis_min, const float* ref_depth, double tol_nsigma,
                    int8_t* ray_code, double* surface_depth, int64_t* counts, void* stream)
{
    if (!c) return fail(MRF_EINVAL, "mrf_accuracy_ex: null context");
    if (!c->built) return fail(MRF_ESTATE, "mrf_accuracy_ex: call mrf_build first");
    if (!(vis_min > 0.0 && vis_min <= 1.0)) return fail(MRF_EINVAL, "mrf_accuracy_ex: vis_min must lie in (0, 1]");
    if (!(tol_nsigma >= 0.0)) return fail(MRF_EINVAL, "mrf_accuracy_ex: tol_nsigma must be >= 0");
    if (!logit) {
        if (!c->inferred) return fail(MRF_ESTATE, "mrf_accuracy_ex: no map given and no mrf_infer yet");
        logit = (const float*)c->b_L.p;
    }
    hipStream_t s = (hipStream_t)stream;
    HCK(hipSetDevice(c->device), "mrf_accuracy_ex: hipSetDevice");
    HCK(ensure(c->b_metric, 2 * sizeof(double) * (size_t)c->V), "mrf_accuracy_ex: alloc");
    HCK(launch_accuracy(c, logit, vis_min, ref_depth, tol_nsigma, ray_code, surface_depth, counts,
                        (double*)c->b_metric.p, s),
        "mrf_accuracy_ex");
    return MRF_OK;
}

int mrf_depth_distribution(mrf_ctx* c, float* prob, int32_t* mode_step, float* mean_depth, void* stream)
{
    if (!c) return fail(MRF_EINVAL, "mrf_depth_distribution: null context");
    if (!c->inferred) return fail(MRF_ESTATE, "mrf_depth_distribution: call mrf_infer first");
    hipStream_t s = (hipStream_t)stream;
    HCK(hipSetDevice(c->device), "mrf_depth_distribution: hipSetDevice");
    float* q = prob ? (float*)c->b_ellbar.p : nullptr;   // slot order, then canonical edge order
    const KfSrc kfs{(const float*)c->b_kfx.p, (const int64_t*)c->b_kfxb.p};
    ExclSrc lam = final_lam(c);
    if (c->kf_inferred) lam = ExclSrc{(const float2*)c->b_theta2.p, nullptr};   // one sweep: the prior
    HCK(launch_depth_distribution(c, lam, c->kf_inferred && c->K > 1 ? &kfs : nullptr, q, mode_step, mean_depth, s),
        "mrf_depth_distribution");
    if (prob) HCK(export_canonical_edges(c, q, prob, 4, s), "mrf_depth_distribution: export");
    return MRF_OK;
}

int mrf_accuracy_static(mrf_ctx* c, const float* logit, double vis_min, int8_t* ray_code, double* surface_depth,
                        int64_t* counts, void* stream)
{
    if (!c) return fail(MRF_EINVAL, "mrf_accuracy_static: null context");
    if (!c->built) return fail(MRF_ESTATE, "mrf_accuracy_static: call mrf_build first");
    if (!(vis_min > 0.0 && vis_min <= 1.0))
        return fail(MRF_EINVAL, "mrf_accuracy_static: vis_min must lie in (0, 1]");
    if (c->V > kStaticMetricVoxels)
        return fail(MRF_ERANGE, "mrf_accuracy_static: the scenes hold " + std::to_string(c->V) +
                                    " voxels, more than the static scratch's " +
                                    std::to_string(kStaticMetricVoxels));
    if (!logit) {
        if (!c->inferred) return fail(MRF_ESTATE, "mrf_accuracy_static: no map given and no mrf_infer yet");
        logit = (const float*)c->b_L.p;
    }
    hipStream_t s = (hipStream_t)stream;
    double* work = nullptr;
    HCK(static_scratch(c->device, &work), "mrf_accuracy_static: static scratch of this device");
    HCK(hipSetDevice(c->device), "mrf_accuracy_static: hipSetDevice");
    HCK(launch_accuracy(c, logit, vis_min, nullptr, 0.0, ray_code, surface_depth, counts, work, s),
        "mrf_accuracy_static");
    return MRF_OK;
}

int mrf_stats(const mrf_ctx* c, mrf_stats_t* out)
{
    if (!c || !out) return fail(MRF_EINVAL, "mrf_stats: null argument");
    if (!c->built) return fail(MRF_ESTATE, "mrf_stats: call mrf_build first");
    *out = c->stats;
    return MRF_OK;
}

int mrf_export_incidence(const mrf_ctx* c, int64_t* row_ptr, int32_t* col, double* t_in, double* t_out,
                         int64_t* vptr, uint32_t* vedge, void* stream)
{
    if (!c) return fail(MRF_EINVAL, "mrf_export_incidence: null context");
    if (!c->built) return fail(MRF_ESTATE, "mrf_export_incidence: call mrf_build first");
    if ((t_in || t_out) && !c->keep_chords)
        return fail(MRF_ESTATE, "mrf_export_incidence: chords were not kept (keep_chords = 0)");
    hipStream_t s = (hipStream_t)stream;
    if (row_ptr)
        HCK(hipMemcpyAsync(row_ptr, c->b_rowptr.p, 8 * (size_t)(c->R + 1), hipMemcpyDeviceToDevice, s), "export");
    if (col) HCK(export_canonical_edges(c, c->b_col.p, col, 4, s), "export");
    if (t_in) HCK(export_canonical_edges(c, c->b_tin.p, t_in, 8, s), "export");
    if (t_out) HCK(export_canonical_edges(c, c->b_tout.p, t_out, 8, s), "export");
    if (vptr || vedge) HCK(export_canonical_incidence(c, vptr, vedge, s), "export");
    return MRF_OK;
}

int mrf_export_edges(const mrf_ctx* c, float* delta, uint8_t* bin, float* g, float* lam, float* ell, void* stream)
{
    if (!c) return fail(MRF_EINVAL, "mrf_export_edges: null context");
    if (!c->built) return fail(MRF_ESTATE, "mrf_export_edges: call mrf_build first");
    if ((g || lam || ell) && !c->inferred) return fail(MRF_ESTATE, "mrf_export_edges: call mrf_infer first");
    hipStream_t s = (hipStream_t)stream;
    if (delta) HCK(export_canonical_edges(c, c->b_delta.p, delta, 4, s), "export");
    if (bin) HCK(export_canonical_edges(c, c->b_bin.p, bin, 1, s), "export");
    if (g) HCK(export_canonical_edges(c, c->b_g.p, g, 4, s), "export");
    if (lam) {   // materialised into a scratch edge array first
        float* tmp = (float*)c->b_ellbar.p;
        if (c->kf_inferred && c->K > 1)
            HCK(launch_excl_kf(c, KfSrc{(const float*)c->b_kfx.p, (const int64_t*)c->b_kfxb.p}, tmp, s), "export");
        else if (c->kf_inferred)   // one sweep: the prior was every incoming message
            HCK(launch_excl(c, ExclSrc{(const float2*)c->b_theta2.p, nullptr}, tmp, s), "export");
        else
            HCK(launch_excl(c, final_lam(c), tmp, s), "export");
        HCK(export_canonical_edges(c, tmp, lam, 4, s), "export");
    }
    if (ell) HCK(export_canonical_edges(c, final_ell(c), ell, 4, s), "export");
    return MRF_OK;
}

}  // extern "C"

extern "C" {

static std::string kid_name(const mrf_ctx* c, int k)
{
    if (k >= KID_VOX0 && k < KID_VOX0 + kVoxClasses) {
        const int q = k - KID_VOX0;
        if (q == kVoxClasses - 1) return "voxel_chunked_k";
        if (kVoxNW[q] == 0)
            return "voxel_small_k<" + std::to_string(kVoxCap[q]) + "," + std::to_string(kVoxVPW[q]) + ">";
        return "voxel_k<" + std::to_string(kVoxNW[q]) + "," + std::to_string(kVoxCap[q] / (64 * kVoxNW[q])) + "," +
               std::to_string(kVoxVPW[q]) + ">";
    }
    auto ray_name = [](const char* direct, const char* lds, int q, RayShape sh, bool adj) {
        std::string n = std::string(ray_class_lds(q) ? lds : direct) + "<" + std::to_string(sh.g) + "," +
                        std::to_string(kRayCap[q] / sh.g);
        if (adj && ray_class_lds(q)) n += "," + std::to_string(sh.rpw);
        return n + ">";
    };
    if (k >= KID_RAY0 && k < KID_RAY0 + kRayClasses) {
        const int q = k - KID_RAY0;
        return ray_name("ray_k", "ray_lds_k", q, kFwdShapes[q][c->fwd_sel[q]], false);
    }
    if (k >= KID_ADJ0 && k < KID_ADJ0 + kRayClasses) {
        const int q = k - KID_ADJ0;
        return ray_name("ray_adj_k", "ray_adj_lds_k", q, kAdjShapes[q][c->adj_sel[q]], true);
    }
    if (k == KID_PAIR) return "keyframe pair averages";
    if (k == KID_KFVOX) return "kf_voxel_k";
    if (k == KID_POT) return "potentials_k";
    if (k == KID_SIGMA) return "sigma_grad_k<false>";   // the profile asks for no bias gradient
    return "?";
}

// algorithmic bytes and edges of one launch of kernel k (steady-state sweep)
static void kid_bytes(const mrf_ctx* c, int k, double* bytes, int64_t* edges)
{
    *bytes = 0.0;
    *edges = 0;
    if (k >= KID_VOX0 && k < KID_VOX0 + kVoxClasses) {
        const int q = k - KID_VOX0;
        // per edge: vedge 4 + gathered message 4; per voxel: descriptor 16 + base 4 + total 4
        *edges = c->vox_cls_edges[q];
        *bytes = 8.0 * (double)*edges + 24.0 * (double)c->vox_cnt[q];
    } else if (k >= KID_RAY0 && k < KID_RAY0 + kRayClasses) {
        const int q = k - KID_RAY0;
        // per edge: col 4 + own ell 4 + g 4 + ell 4 (voxel totals: counted once per voxel
        // in the sweep figure; with per-keyframe messages no own ell, and the keyframe's
        // message counted once per pair); per ray: count 4; per tile: list 4 + descriptor 32
        *edges = c->ray_cls_edges[q];
        *bytes = (c->kf_inferred ? 12.0 : 16.0) * (double)*edges + 4.0 * (double)c->ray_cls_rays[q] +
                 36.0 * (double)c->ray_cnt[q];
    } else if (k == KID_PAIR) {
        // per edge: vedge 4 + weight 4 + gathered ell 4; per pair: descriptor 16 + average 8
        *edges = c->E;
        *bytes = 12.0 * (double)c->E + 24.0 * (double)c->n_pairs;
    } else if (k == KID_KFVOX) {
        // per pair: average 8 + message index 4 + message 4; per voxel: descriptor 16 + theta 4
        *edges = c->E;
        *bytes = 16.0 * (double)c->n_pairs + 20.0 * (double)c->n_kf_vox;
    } else if (k >= KID_ADJ0 && k < KID_ADJ0 + kRayClasses) {
        const int q = k - KID_ADJ0;
        // per edge: col 4 + own ell 4 + g 4 + own lambar of the later sweep 4 + lambar 4 +
        // gsum read 4 + write 4
        *edges = c->ray_cls_edges[q];
        *bytes = 28.0 * (double)*edges + 4.0 * (double)c->ray_cls_rays[q] + 36.0 * (double)c->ray_cnt[q];
    } else if (k == KID_POT || k == KID_SIGMA) {
        *edges = c->E;
        *bytes = 9.0 * (double)c->S;
    }
}

int mrf_profile_sweeps(mrf_ctx* c, int32_t reps, int32_t include_backward, mrf_kernel_time_t* out, int32_t max_out,
                       int32_t* n_out, void* stream)
{
    if (!c || !out || !n_out || reps < 1) return fail(MRF_EINVAL, "mrf_profile_sweeps: bad argument");
    if (!c->inferred) return fail(MRF_ESTATE, "mrf_profile_sweeps: call mrf_infer first");
    hipStream_t s = (hipStream_t)stream;
    Profiler P;
    c->prof = &P;
    hipError_t e = hipSuccess;
    // inputs: the last sweep's messages; outputs go to scratch buffers, so the
    // inference state stays untouched
    const float* theta = (const float*)c->b_theta.p;
    const float* ell_in = final_ell(c);
    float2* vt = (float2*)c->b_tbar.p;
    float* ell = (float*)c->b_ellbar.p;
    if (c->kf_inferred) {
        // per-keyframe sweeps from the last sweep's messages: the pair averages are
        // rewritten with the values the inference left, the keyframe messages go to
        // scratch (b_export), the ray messages to b_ellbar
        e = ensure(c->b_export, sizeof(float) * (size_t)(c->n_kfx > 0 ? c->n_kfx : 1));
        float* xs = (float*)c->b_export.p;
        const KfSrc kf{xs, (const int64_t*)c->b_kfxb.p};
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            e = launch_pair_phase(c, ell_in, (const float*)c->b_kfw.p, (double*)c->b_pair_m.p, s);
            if (e == hipSuccess) e = launch_kf_voxel(c, (const double*)c->b_pair_m.p, theta, xs, nullptr, s);
            if (e == hipSuccess) e = launch_ray_phase_kf(c, kf, ell, false, s);
        }
        include_backward = 0;
    }
    for (int r = 0; r < reps && e == hipSuccess && !c->kf_inferred; ++r) {
        e = launch_voxel_phase(c, ell_in, VoxOut{theta, vt, nullptr, nullptr}, s);
        if (e == hipSuccess) e = launch_ray_phase(c, ExclSrc{vt, ell_in}, ell, false, s);
    }
    if (include_backward) {
        float* lambar = (float*)c->b_lambar.p;
        float* gsum = (float*)c->b_gsum.p;
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            e = launch_ray_adjoint(c, ExclSrc{vt, ell_in}, ExclSrc{vt, ell}, lambar, gsum, r == 0, s);
            if (e == hipSuccess)
                e = launch_voxel_phase(c, lambar, VoxOut{nullptr, vt + 2 * c->V, nullptr, (float*)c->b_thetabar.p},
                                       s);
        }
        if (e == hipSuccess)
            e = launch_sigma_grad(c, (float*)((char*)c->b_sigpart.p + sigpart_bytes(c)), nullptr, s);
    }
    c->prof = nullptr;
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        for (hipEvent_t ev : P.pool) hipEventDestroy(ev);
        return hip_fail(e, "mrf_profile_sweeps");
    }
    double tot[KID_COUNT] = {0};
    int cnt[KID_COUNT] = {0};
    for (auto& rec : P.recs) {
        float ms = 0.0f;
        hipEventElapsedTime(&ms, P.pool[rec.second], P.pool[rec.second + 1]);
        tot[rec.first] += ms;
        cnt[rec.first] += 1;
    }
    for (hipEvent_t ev : P.pool) hipEventDestroy(ev);
    int n = 0;
    for (int k = 0; k < KID_COUNT; ++k) {
        if (!cnt[k]) continue;
        if (n < max_out) {
            mrf_kernel_time_t& o = out[n];
            memset(&o, 0, sizeof(o));
            strncpy(o.name, kid_name(c, k).c_str(), sizeof(o.name) - 1);
            o.launches = cnt[k];
            o.total_ms = tot[k];
            kid_bytes(c, k, &o.bytes_per_launch, &o.edges_per_launch);
        }
        ++n;
    }
    *n_out = n < max_out ? n : max_out;
    return MRF_OK;
}


int mrf_get_tuning(const mrf_ctx* c, mrf_tuning_t* out)
{
    if (!c || !out) return fail(MRF_EINVAL, "mrf_get_tuning: null argument");
    memset(out, 0, sizeof(*out));
    out->n_classes = kRayClasses;
    for (int q = 0; q < kRayClasses; ++q) {
        out->cap[q] = kRayCap[q];
        out->fwd_candidates[q] = ray_shape_count(q, false);
        out->fwd_sel[q] = c->fwd_sel[q];
        out->fwd_lanes[q] = kFwdShapes[q][c->fwd_sel[q]].g;
        out->adj_candidates[q] = ray_shape_count(q, true);
        out->adj_sel[q] = c->adj_sel[q];
        out->adj_lanes[q] = kAdjShapes[q][c->adj_sel[q]].g;
        out->adj_rays[q] = kAdjShapes[q][c->adj_sel[q]].rpw;
    }
    return MRF_OK;
}

int mrf_set_tuning(mrf_ctx* c, const int32_t* fwd_sel, const int32_t* adj_sel)
{
    if (!c) return fail(MRF_EINVAL, "mrf_set_tuning: null context");
    for (int q = 0; q < kRayClasses; ++q) {
        if (fwd_sel && (fwd_sel[q] < 0 || fwd_sel[q] >= ray_shape_count(q, false)))
            return fail(MRF_EINVAL, "mrf_set_tuning: ray-phase shape index out of range");
        if (adj_sel && (adj_sel[q] < 0 || adj_sel[q] >= ray_shape_count(q, true)))
            return fail(MRF_EINVAL, "mrf_set_tuning: reverse-pass shape index out of range");
    }
    for (int q = 0; q < kRayClasses; ++q) {
        if (fwd_sel) c->fwd_sel[q] = fwd_sel[q];
        if (adj_sel) c->adj_sel[q] = adj_sel[q];
    }
    return MRF_OK;   // a cached forward graph is revalidated by mrf_infer (its key holds the shapes)
}

int mrf_autotune(mrf_ctx* c, int32_t reps, void* stream)
{
    if (!c || reps < 1) return fail(MRF_EINVAL, "mrf_autotune: bad argument");
    if (!c->inferred) return fail(MRF_ESTATE, "mrf_autotune: call mrf_infer first");
    hipStream_t s = (hipStream_t)stream;
    HCK(hipSetDevice(c->device), "mrf_autotune: hipSetDevice");
    // inputs: the last sweep's messages; outputs go to buffers the reverse pass
    // initialises before use, so the inference state stays untouched.  The
    // reverse kernels run in the form of every reverse sweep after the first:
    // an own term in their d/d ell input (any per-voxel pairs and any slot
    // array serve for timing) and the running g-bar sum read and accumulated.
    const ExclSrc lam = final_lam(c);
    const ExclSrc eb{(const float2*)c->b_theta2.p, (const float*)c->b_ellbar.p};
    float* ell_out = (float*)c->b_ellbar.p;
    float* lambar = (float*)c->b_lambar.p;
    float* gsum = (float*)c->b_gsum.p;
    hipEvent_t ev[2] = {nullptr, nullptr};
    HCK(hipEventCreate(&ev[0]), "mrf_autotune: event");
    hipError_t e = hipEventCreate(&ev[1]);
    // after per-keyframe averaged sweeps: their ray phase only (the reverse
    // shapes are tuned on the exact scheme's sweeps)
    const bool kf = c->kf_inferred != 0;
    const KfSrc kfs{(const float*)c->b_kfx.p, (const int64_t*)c->b_kfxb.p};
    for (int adj = 0; adj < (kf ? 1 : 2) && e == hipSuccess; ++adj) {
        for (int q = 0; q < kRayClasses && e == hipSuccess; ++q) {
            const int ns = ray_shape_count(q, adj == 1);
            if (c->ray_cnt[q] <= 0 || ns < 2) continue;
            int best = 0;
            float best_ms = 0.0f;
            for (int i = 0; i < ns && e == hipSuccess; ++i) {
                auto run = [&]() {
                    if (kf) return launch_ray_class_shape_kf(c, q, i, kfs, ell_out, s);
                    return adj ? launch_adj_class_shape(c, q, i, lam, eb, lambar, gsum, 0, s)
                               : launch_ray_class_shape(c, q, i, lam, ell_out, s);
                };
                e = run();   // warm-up
                if (e == hipSuccess) e = hipEventRecord(ev[0], s);
                for (int r = 0; r < reps && e == hipSuccess; ++r) e = run();
                if (e == hipSuccess) e = hipEventRecord(ev[1], s);
                if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
                if (e == hipSuccess && (i == 0 || ms < best_ms)) {
                    best = i;
                    best_ms = ms;
                }
            }
            if (adj)
                c->adj_sel[q] = best;
            else
                c->fwd_sel[q] = best;
        }
    }
    hipEventDestroy(ev[0]);
    if (ev[1]) hipEventDestroy(ev[1]);
    if (e != hipSuccess) return hip_fail(e, "mrf_autotune");
    return MRF_OK;
}

}  // extern "C"
