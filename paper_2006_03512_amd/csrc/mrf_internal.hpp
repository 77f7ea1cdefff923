// Internal declarations of libmrf: device-side descriptors, the context, and
// the host launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mrf.h"

namespace mrf {

// ---------------------------------------------------------------- limits
constexpr int kBins = 64;
constexpr int kMaxRayLen = 2048;      // longest ray factor a group can hold

// Ray-length classes by tile length (longest ray of the tile), capacity cap.
// A ray is held by a group of G lanes (16, 32 or 64), each holding IPL = cap / G
// consecutive steps; in the reverse pass a group may walk RPW = 2 rays in turn.
// Class 0 (cap 16) is G = 16 reading the tile directly; classes up to
// kLdsMaxCap stage the tile through LDS; longer classes are G = 64, direct.
constexpr int kRayClasses = 13;
constexpr int kRayCap[kRayClasses] = {16, 64, 128, 192, 256, 320, 384, 512, 640, 768, 1024, 1536, 2048};
constexpr int kLdsMaxCap = 512;
constexpr bool ray_class_lds(int q) { return q > 0 && kRayCap[q] <= kLdsMaxCap; }

// Candidate launch shapes of every class; the first is the default (fastest
// on the 30-keyframe batch), mrf_autotune times them all on the built graph
// and keeps the fastest per class.  A zero G ends a list.
struct RayShape {
    int g, rpw;
};
constexpr int kNShapes = 5;
constexpr RayShape kFwdShapes[kRayClasses][kNShapes] = {
    {{16, 1}},
    {{16, 1}, {32, 1}, {64, 1}},
    {{16, 1}, {32, 1}, {64, 1}},
    {{16, 1}, {32, 1}, {64, 1}},
    {{32, 1}, {16, 1}, {64, 1}},
    {{32, 1}, {64, 1}, {16, 1}},
    {{32, 1}, {64, 1}},
    {{64, 1}, {32, 1}},
    {{64, 1}}, {{64, 1}}, {{64, 1}}, {{64, 1}}, {{64, 1}},
};
constexpr RayShape kAdjShapes[kRayClasses][kNShapes] = {
    {{16, 1}},
    {{16, 1}, {32, 1}, {64, 1}},
    {{16, 1}, {32, 1}, {64, 1}, {64, 2}},
    {{16, 1}, {32, 1}, {64, 1}, {64, 2}},
    {{32, 2}, {32, 1}, {64, 1}, {64, 2}},
    {{64, 2}, {64, 1}, {32, 1}, {32, 2}},
    {{64, 2}, {64, 1}, {32, 1}},
    {{64, 1}, {64, 2}},
    {{64, 1}}, {{64, 1}}, {{64, 1}}, {{64, 1}}, {{64, 1}},
};
constexpr int ray_shape_count(int q, bool adj)
{
    int n = 0;
    while (n < kNShapes && (adj ? kAdjShapes[q][n].g : kFwdShapes[q][n].g) != 0) ++n;
    return n;
}
constexpr bool ray_shapes_valid()
{
    for (int q = 0; q < kRayClasses; ++q)
        for (int a = 0; a < 2; ++a)
            for (int i = 0; i < ray_shape_count(q, a == 1); ++i) {
                const RayShape sh = a ? kAdjShapes[q][i] : kFwdShapes[q][i];
                if ((sh.g != 16 && sh.g != 32 && sh.g != 64) || kRayCap[q] % sh.g != 0) return false;
                if (sh.rpw != 1 && !(a == 1 && sh.rpw == 2 && ray_class_lds(q))) return false;
                if (!ray_class_lds(q) && !(sh.g == 64 || kRayCap[q] == sh.g)) return false;   // direct kernels
            }
    return true;
}
static_assert(ray_shapes_valid(), "ray shapes: 16, 32 or 64 lanes dividing the capacity; 2 rays per group only "
                                  "in reverse LDS classes; direct classes hold a ray in one group");

// Edges are stored in tiles of 4x4 pixels, step-major: slot of (ray lane i,
// step k) = tile_base + 16 k + i.  Rays of one camera reach a voxel after the
// same number of 3D-DDA steps, so the edges a voxel receives from one tile
// share a 64-byte line.
constexpr int kTileW = 4;
constexpr int kTile = kTileW * kTileW;

// Voxel work classes by degree: (waves per voxel NW, items per lane IPL =
// capacity / (64 NW), voxels per wave VPW); each wave owns 64*IPL consecutive
// edges of a voxel, and a one-wave class (NW = 1) walks VPW voxels per wave
// (a packed class, NW = 0: VPW voxels per lane group) with every load issued
// first.  Above the last class a 1024-thread block walks the voxel in
// 1024-edge pieces.
#ifndef MRF_VOX_CAPS
#define MRF_VOX_CAPS 16, 32, 64, 128, 256, 1024, 4096, 16384, 32768
#define MRF_VOX_NW 0, 0, 1, 1, 1, 1, 4, 16, 16
#define MRF_VOX_VPW 4, 4, 8, 4, 4, 1, 1, 1, 1
#endif
// Degree capacity of each single-pass class and its waves per voxel; NW = 0
// packs 64 / cap voxels into a wave (cap = 16 or 32 lanes per voxel, one edge
// per lane).
constexpr int kVoxCap[] = {MRF_VOX_CAPS};
constexpr int kVoxNW[] = {MRF_VOX_NW};
constexpr int kVoxVPW[] = {MRF_VOX_VPW};
constexpr int kVoxClasses = (int)(sizeof(kVoxCap) / sizeof(int)) + 1;   // + the chunked class
static_assert(sizeof(kVoxNW) == sizeof(kVoxCap) && sizeof(kVoxVPW) == sizeof(kVoxCap),
              "one wave count and one voxels-per-wave count per voxel class");
constexpr bool vox_classes_valid()
{
    for (int k = 0; k + 1 < kVoxClasses; ++k) {
        if (kVoxNW[k] == 0) {
            if (kVoxCap[k] != 16 && kVoxCap[k] != 32) return false;
        } else if (kVoxCap[k] % (64 * kVoxNW[k]) != 0 || kVoxCap[k] / (64 * kVoxNW[k]) > 32 || kVoxNW[k] > 16) {
            return false;
        }
        if (kVoxVPW[k] < 1 || kVoxVPW[k] > 32 || (kVoxNW[k] > 1 && kVoxVPW[k] != 1)) return false;
        if (kVoxNW[k] == 1 && kVoxVPW[k] * (kVoxCap[k] / 64) > 32) return false;
        if (k > 0 && kVoxCap[k] <= kVoxCap[k - 1]) return false;
    }
    return true;
}
static_assert(vox_classes_valid(), "voxel classes: increasing capacities; 16 or 32 lanes per packed voxel, or "
                                   "64 NW IPL edges with IPL <= 32, NW <= 16; several voxels per wave or "
                                   "group only with NW <= 1, at most 32 items per lane in all");
constexpr int kVoxChunk = 1024;   // piece of a hub voxel (16 items per lane)

// Voxels are keyed brick-major (8^3 bricks) for the voxel -> ray incidence so
// that one brick's voxels, which share most of their rays, are adjacent.
constexpr int kBrick = 8;

struct SceneDev {
    int32_t W, H;
    double fx, fy, cx, cy;
    int32_t n[3];
    int32_t pad;
    double h;
    double o[3];
    int64_t voxel_base;
    int64_t ray_base;
    int32_t nb[3];        // bricks per axis
    int32_t pad2;
    int64_t key_base;     // first brick-major key of this scene
    int64_t brick_off;    // the scene's first byte in the brick allocation mask
};

struct FrameDev {
    const float* depth;   // H*W
    const double* T;      // 16
    int32_t scene;
    int32_t ntx;          // tiles per image row
    int64_t ray_base;     // global id of pixel (0, 0)
    int64_t tile_base;    // global id of the frame's first tile
};

// One 4x4-pixel tile: its slots are [base, base + 16 len).
struct TileDev {
    int64_t base;
    int32_t ray0;         // global ray id of the tile's top-left pixel
    int32_t W;            // image width (ray id stride between tile rows)
    int32_t nu, nv;       // pixels of the tile inside the image
    int32_t len;          // longest ray of the tile (steps)
    int32_t frame;        // global frame (keyframe) index
};

// Per-edge voxel -> ray messages (forward) or d/d ell (reverse) in the form the
// ray kernels read them: value_e = tot[col_e] - own_e, tot a per-voxel total
// (linear voxel id) and own_e the edge's own term in it (own null: 0).  A total
// is the FP32 pair (hi, lo) of its FP64 sum, and the value is formed as
// (hi - own) + lo: when own is most of the total, hi - own is exact and the
// remainder keeps the accuracy of the FP64 sum instead of losing itself in the
// rounding of a total of magnitude |own|.
struct ExclSrc {
    const float2* tot;
    const float* own;
};

// The kernel-side form: own always points at a readable per-slot array (the
// potentials g when absent), with has_own telling whether to use it.
struct ExclDev {
    const float2* tot;
    const float* own;
    int has_own;
};

// Voxel -> ray messages with per-keyframe averaged messages (Sec. IV-A): the
// message into a ray of keyframe f from voxel v is x[xb[f] + v], one value
// per (keyframe, voxel) pair (xb[f] = the keyframe's first entry less the
// first linear voxel id of its scene).
struct KfSrc {
    const float* x;
    const int64_t* xb;
};

// Reverse pass with per-keyframe averaged messages: lambda_e as in KfSrc
// (x, the sweep's messages), and d/d ell_e = w_e y[xb[f] + col_e], w_e the
// edge's share of its pair's weight (per slot) and y the derivative reaching
// the pair's average (same layout as x).
struct AdjKf {
    KfSrc x;
    const float* y;
    const float* w;
};

// Outputs of a voxel-phase reduction of sum_v (the FP64 sum of a per-edge
// array over voxel v's edges), each optional: tot2[v] = pair(base[v] + sum_v),
// totf[v] = fl(base[v] + sum_v), acc[v] += fl(sum_v); base null reads as 0.
struct VoxOut {
    const float* base;
    float2* tot2;
    float* totf;
    float* acc;
    double* dsum = nullptr;   // dsum[v] = sum_v (FP64)
};

// Work item of the voxel kernels: one voxel's edge list vedge[start, start + m)
// and its linear id.
struct VoxDev {
    int64_t start;
    int32_t m;
    uint32_t v;
};

struct BuildDev {
    double z_min, z_max, nsig, c0, c2, smin, dmax;
    int32_t min_vox;
    int32_t radius;            // sparse grid: bricks allocated around a measured point's brick
    const uint8_t* bricks;     // sparse grid: allocation mask (SceneDev::brick_off); null: dense
    int32_t skip;              // sparse grid: step over unallocated bricks brick by brick
};

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

// Edge slots in groups of whole scenes with fewer than 2^32 slots each (one group
// unless the batch has 2^32 slots or more): a voxel's list entry holds its slot
// less the first slot of its group, in 32 bits, and the entries of group g take
// the list positions [pos[g], pos[g + 1]).  slot[0] = pos[0] = 0.
constexpr int kMaxSlotGroups = 8;
struct SlotGroups {
    int32_t n = 1;
    int64_t slot[kMaxSlotGroups] = {0};
    int64_t pos[kMaxSlotGroups] = {0};
};

// First slot of the group of list position j (constant indices only, so the
// table stays in kernel arguments).
__host__ __device__ __forceinline__ int64_t group_slot_base(const SlotGroups& g, int64_t j)
{
    int64_t b = 0;
#pragma unroll
    for (int k = 1; k < kMaxSlotGroups; ++k)
        if (k < g.n && j >= g.pos[k]) b = g.slot[k];
    return b;
}

// First slot of the group holding slot x.
__host__ __device__ __forceinline__ int64_t group_slot_base_of_slot(const SlotGroups& g, int64_t x)
{
    int64_t b = 0;
#pragma unroll
    for (int k = 1; k < kMaxSlotGroups; ++k)
        if (k < g.n && x >= g.slot[k]) b = g.slot[k];
    return b;
}

// Kernel launches that the profiler can time individually.
enum KernelId {
    KID_VOX0 = 0,
    KID_RAY0 = KID_VOX0 + kVoxClasses, KID_ADJ0 = KID_RAY0 + kRayClasses,
    KID_POT = KID_ADJ0 + kRayClasses, KID_SIGMA, KID_PAIR, KID_KFVOX, KID_COUNT
};

// HIP events recorded around launches on the stream they run on.
struct Profiler {
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<std::pair<int, size_t>> recs;   // (kernel id, index of its start event)
    hipEvent_t next()
    {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            hipEventCreate(&e);
            pool.push_back(e);
        }
        return pool[used++];
    }
};

}  // namespace mrf

struct mrf_ctx {
    int device = 0;
    hipStream_t aux = nullptr;    // internal stream used for graph capture/launch
    hipEvent_t ev_in = nullptr, ev_out = nullptr;

    // graph description
    int32_t n_scenes = 0;
    int64_t R = 0, E = 0, V = 0;
    int64_t S = 0;                        // edge slots (E plus tile padding)
    int64_t T = 0;                        // tiles
    int64_t Vk = 0;                       // brick-major key space (>= V, padded bricks)
    int32_t n_frames = 0, max_hw = 0, max_tpf = 0;   // most pixels / tiles in one frame
    std::vector<mrf::SceneDev> scenes_h;
    std::vector<mrf::FrameDev> frames_h;
    std::vector<int32_t> frame_hw;
    mrf::BuildDev bp{};
    int keep_chords = 0;

    // sensor tables (Sec. IV-C): one 64-bin row, or with cell_px > 0 one row per
    // cell_px x cell_px pixel region of the frame (n_cells rows)
    int32_t cell_px = 0;
    int64_t n_cells = 1;

    mrf::SlotGroups sg{};     // edge-slot groups of the voxel -> ray lists
    int32_t group_log2 = 32;  // a group holds fewer than 2^group_log2 slots
    std::vector<int> group_scene;   // first scene of each group

    // buffers (raw device pointers into `bufs`)
    mrf::DevBuf b_scenes, b_frames, b_counts, b_rowptr, b_col, b_delta, b_bin, b_tin, b_tout,
        b_g, b_lam, b_ell, b_vedge, b_vptr, b_theta, b_L, b_thetabar, b_sigma, b_bias, b_ckpt,
        b_ellbar, b_lambar, b_gsum, b_tmp64, b_cls, b_sigpart, b_misc;
    mrf::DevBuf b_tiles, b_tbase;
    mrf::DevBuf b_tsum;   // per-voxel totals of the sweeps (theta + incoming ray messages), float2 pairs
    mrf::DevBuf b_theta2; // the prior log-odds as total pairs (theta, 0): the first sweep's lambda
    mrf::DevBuf b_metric; // accuracy metric: per-voxel alpha and log alpha (2 V doubles)
    mrf::DevBuf b_bricks; // sparse grid: one byte per 8^3 brick of every scene
    int64_t n_bricks = 0;
    mrf::DevBuf b_tbar;   // reverse pass, float2 pairs: per-voxel sums of d/d lambda, the seed d/d L, a spare
    mrf::DevBuf b_export;     // temporaries of the canonical incidence export
    std::vector<mrf::DevBuf> b_host_in;   // device copies of depth and pose arrays given in host memory

    // per-keyframe averaged messages (Sec. IV-A), built when requested
    int kf = 0;                   // the build made the pair structures
    int kf_inferred = 0;          // the last inference used them
    int64_t n_pairs = 0;          // (keyframe, voxel) pairs with at least one edge
    int64_t n_kfx = 0;            // entries of the per-keyframe message buffers
    mrf::DevBuf b_kflen;          // per edge slot: chord length (Euclidean) of the edge
    mrf::DevBuf b_kfw;            // per vedge entry: chord length / the pair's summed chord length
    mrf::DevBuf b_pair_m;         // per pair: FP64 average message of the keyframe into the voxel
    mrf::DevBuf b_pair_x;         // per pair: index of its entry in b_kfx
    mrf::DevBuf b_kfx;            // per-keyframe voxel -> ray messages
    mrf::DevBuf b_kfxb;           // per frame: b_kfx base less its scene's first voxel id
    mrf::DevBuf b_kfxr, b_kfy;    // reverse pass: a sweep's rebuilt keyframe messages, the pair derivatives
    mrf::DevBuf b_kfws;           // reverse pass: per edge slot, the edge's share of its pair's weight
    int kfws_ready = 0;           // b_kfws holds the current build's weights
    mrf::DevBuf b_kf_vox;         // per touched voxel: VoxDev over its pairs (start, count, voxel id)
    mrf::DevBuf b_pair_desc[mrf::kVoxClasses];   // pairs by edge-count class: VoxDev (start, m, pair id)
    int64_t pair_cnt[mrf::kVoxClasses] = {0};
    int64_t n_kf_vox = 0;
    mrf::DevBuf b_ray_list[mrf::kRayClasses];     // tile ids by tile length class
    mrf::DevBuf b_vox_list[mrf::kVoxClasses];     // brick-major keys
    mrf::DevBuf b_vox_desc[mrf::kVoxClasses];     // matching VoxDev descriptors
    mrf::DevBuf b_frame_list;     // per-frame ray lists for the plain schedule

    int64_t ray_cnt[mrf::kRayClasses] = {0};       // tiles per class
    int64_t vox_cnt[mrf::kVoxClasses] = {0};
    int64_t ray_cls_edges[mrf::kRayClasses] = {0};
    int64_t vox_cls_edges[mrf::kVoxClasses] = {0};
    std::vector<int64_t> frame_ray_off;   // plain schedule: tiles of frame f at [off[f], off[f+1])
    int64_t ray_cls_rays[mrf::kRayClasses] = {0};

    // stats
    mrf_stats_t stats{};

    // state
    int built = 0, inferred = 0, K = 0, have_ckpt = 0;
    uint64_t gen = 0;   // bumped by every build and every successful inference
    int schedule = MRF_SCHED_GRAPH;

    // graph cache
    hipGraphExec_t gexec = nullptr;
    int g_K = -1, g_ckpt = -1;
    std::vector<uint64_t> g_key;   // sizes and buffer addresses the captured graph depends on

    mrf::Profiler* prof = nullptr;   // non-null while mrf_profile_sweeps records

    // selected launch shape (index into kFwdShapes / kAdjShapes) of every ray class
    int fwd_sel[mrf::kRayClasses] = {0};
    int adj_sel[mrf::kRayClasses] = {0};
};

namespace mrf {

void set_error(const std::string& msg);

// Records start/stop events around one launch when the context is profiling.
struct ProfScope {
    Profiler* p;
    hipStream_t s;
    ProfScope(const mrf_ctx* c, int kid, hipStream_t st) : p(c->prof), s(st)
    {
        if (p) {
            p->recs.push_back({kid, p->used});
            hipEventRecord(p->next(), s);
        }
    }
    ~ProfScope()
    {
        if (p) hipEventRecord(p->next(), s);
    }
};
hipError_t ensure(DevBuf& b, size_t bytes);

// every launcher returns hipSuccess or the first error
// build_kernels.hip
// the count and emit passes over frames [f0, f0 + nf) (nf < 0: to the last frame)
hipError_t launch_trace_count(mrf_ctx* c, hipStream_t s, int f0 = 0, int nf = -1);
hipError_t launch_trace_emit(mrf_ctx* c, hipStream_t s, int f0 = 0, int nf = -1);
// per frame f: out[2 f] = its edge slots, out[2 f + 1] = its edges (after the count
// pass and the tile bases)
hipError_t launch_frame_counts(const mrf_ctx* c, int64_t* out, hipStream_t s);
hipError_t scan_exclusive_i32(const int32_t* in, int64_t* out, int64_t n, void* tmp, size_t tmp_bytes,
                              hipStream_t s);
size_t scan_tmp_bytes(int64_t n);
// Stable LSD sort of (key, value) pairs; the values are the items' indices less
// the first slot of their group under `groups` (one group: the indices).
hipError_t radix_sort_pairs(const uint32_t* keys_in, uint32_t* keys_a, uint32_t* vals_a,
                            uint32_t* keys_b, uint32_t* vals_b, uint32_t* keys_out,
                            uint32_t* vals_out, int64_t n, int key_bits, int32_t* hist,
                            int64_t* offs, void* tmp, size_t tmp_bytes, hipStream_t s,
                            const SlotGroups& groups = SlotGroups{});
size_t radix_hist_entries(int64_t n);
size_t radix_tmp_bytes(int64_t n);   // tmp bytes radix_sort_pairs needs for n items
hipError_t launch_vptr_from_sorted(const uint32_t* sorted_keys, int64_t n, int64_t V, int64_t* vptr,
                                   hipStream_t s);
hipError_t build_classes(mrf_ctx* c, hipStream_t s);
// canonical (linear voxel id, edge id = row_ptr[ray] + step) incidence
hipError_t export_canonical_incidence(const mrf_ctx* c, int64_t* vptr, uint32_t* vedge, hipStream_t s);
// per-edge array from slot order to canonical edge order
hipError_t export_canonical_edges(const mrf_ctx* c, const void* in_slots, void* out, int elem_bytes, hipStream_t s);
// tile descriptors of frames [f0, f0 + nf); slots16[t - first tile of f0] = 16 * longest ray
hipError_t launch_tiles(mrf_ctx* c, int32_t* slots16, hipStream_t s, int f0 = 0, int nf = -1);
hipError_t launch_tile_bases(mrf_ctx* c, hipStream_t s, int64_t t0 = 0);
hipError_t launch_add_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s);
// keys[j] = brick-major key of the voxel of list entry j
hipError_t launch_entry_keys(const mrf_ctx* c, const uint32_t* vedge, int64_t n, uint32_t* keys, hipStream_t s);
// merged voxel -> ray list of the old entries (sorted, keys_old per entry) and the new
// slots sorted on their own (vals relative to s_new0); vptr += new_vptr
hipError_t launch_merge_incidence(const uint32_t* vedge_old, const uint32_t* keys_old, int64_t n_old,
                                  const uint32_t* vals_new, const uint32_t* keys_new, int64_t n_new,
                                  uint32_t s_new0, int64_t* vptr, int64_t* new_vptr, int64_t nkeys, uint32_t* out,
                                  hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
// out[slot[j]] = in[j] for j < n (list order to slot order)
hipError_t launch_scatter_by_slot(const uint32_t* slot, const float* in, int64_t n, float* out, hipStream_t s);
// per-keyframe averaged messages: (keyframe, voxel) pairs of the built graph,
// their weights, work classes and message-buffer indices (after build_classes,
// with the sorted voxel keys still in b_lambar and chord lengths in b_kfw)
hipError_t build_keyframe_pairs(mrf_ctx* c, hipStream_t s);

inline ExclDev excl_dev(const mrf_ctx* c, ExclSrc x)
{
    return ExclDev{x.tot, x.own ? x.own : (const float*)c->b_g.p, x.own ? 1 : 0};
}

// sweep_kernels.hip
hipError_t launch_potentials(mrf_ctx* c, hipStream_t s);
hipError_t launch_fill(float* p, float v, int64_t n, hipStream_t s);
hipError_t launch_copy(float* dst, const float* src, int64_t n, hipStream_t s);
// voxel phase: per touched voxel v, sum_v = FP64 sum of in over its edges,
// written as VoxOut describes
hipError_t launch_voxel_phase(mrf_ctx* c, const float* in, VoxOut out, hipStream_t s);
// out[v] = (in[v], 0): a per-voxel array as a total pair
hipError_t launch_pair(const float* in, float2* out, int64_t n, hipStream_t s);
hipError_t launch_ray_phase(mrf_ctx* c, ExclSrc lam, float* ell, bool plain, hipStream_t s);
// one class of the ray phase / reverse pass with launch shape `sel` (autotuner)
hipError_t launch_ray_class_shape(const mrf_ctx* c, int q, int sel, ExclSrc lam, float* ell, hipStream_t s);
hipError_t launch_adj_class_shape(const mrf_ctx* c, int q, int sel, ExclSrc lam, ExclSrc ellbar, float* lambar,
                                  float* gsum, int first, hipStream_t s);
// out_e = tot[col_e] - own_e on every edge slot (0 on padding)
hipError_t launch_excl(const mrf_ctx* c, ExclSrc x, float* out, hipStream_t s);
// per-keyframe averaged messages: the ray phase reading x[xb[frame] + col]
hipError_t launch_ray_phase_kf(mrf_ctx* c, KfSrc lam, float* ell, bool plain, hipStream_t s);
hipError_t launch_ray_class_shape_kf(const mrf_ctx* c, int q, int sel, KfSrc lam, float* ell, hipStream_t s);
// M[p] = FP64 sum over pair p's list entries j of w[j] in[vedge[j]] (w null: 1)
hipError_t launch_pair_phase(mrf_ctx* c, const float* in, const float* w, double* M, hipStream_t s);
// per touched voxel: T = theta + sum of its pairs' M (M null: 0); x[pair_x[p]] =
// fl(T - M[p]) for every pair when x is not null; L[v] = fl(T) when L is not null
hipError_t launch_kf_voxel(mrf_ctx* c, const double* M, const float* theta, float* x, float* L, hipStream_t s);
// reverse: S = sum of the voxel's pair values sp; acc[v] += fl(S); y[pair_x[p]] =
// fl(S - sp[p]) when y is not null
hipError_t launch_kf_voxel_rev(mrf_ctx* c, const double* sp, float* acc, float* y, hipStream_t s);
// out_e = x[xb[frame of e] + col_e] on every edge slot (0 on padding)
hipError_t launch_excl_kf(const mrf_ctx* c, KfSrc x, float* out, hipStream_t s);
hipError_t launch_sigmoid(const float* L, float* p, int64_t n, hipStream_t s);

// adjoint_kernels.hip
// the reverse ray phase with per-keyframe averaged messages
hipError_t launch_ray_adjoint_kf(mrf_ctx* c, AdjKf kf, float* lambar, float* gsum, bool first, hipStream_t s);
hipError_t launch_ray_adjoint(mrf_ctx* c, ExclSrc lam, ExclSrc ellbar, float* lambar, float* gsum, bool first,
                              hipStream_t s);
// d loss / d sigma and, when dbias is not null, d loss / d bias (a table entry
// each, table_entries(c)) from the accumulated d loss / d g; b_sigpart holds
// the 2 x 2 x entries fixed-point accumulators (sigpart_bytes), scratch past
// them is free for callers.
inline int64_t table_entries(const mrf_ctx* c) { return c->n_cells * kBins; }
inline size_t sigpart_bytes(const mrf_ctx* c) { return sizeof(double) * 4 * (size_t)table_entries(c); }
hipError_t launch_sigma_grad(mrf_ctx* c, float* dsigma, float* dbias, hipStream_t s);
// Accuracy metric (Sec. III-D) of the map `logit` over every pixel of the built
// scenes; counts: 2 per scene (evaluated, accurate), zeroed here.  Needs
// b_metric of 2 V doubles.
// Sparse grid (Sec. IV-B): zero the allocation mask and mark the bricks around
// every measured point (c->bp.bricks, c->bp.radius).
hipError_t launch_brick_mask(mrf_ctx* c, hipStream_t s);
hipError_t launch_accuracy(mrf_ctx* c, const float* logit, double vis_min, const float* ref, double tol,
                           int8_t* code, double* surf, int64_t* counts, double* work, hipStream_t s);
// the ray factors' messages to their depth variables (Eq. depth_message) from
// the last inference's voxel -> ray messages: per slot the probability of the
// voxel's depth (q, slot order), per ray the most probable step and the mean depth
hipError_t launch_depth_distribution(const mrf_ctx* c, ExclSrc lam, const KfSrc* kf, float* q, int32_t* mode,
                                     float* mean, hipStream_t s);
// Device-resident scratch of mrf_accuracy_static: 2 kStaticMetricVoxels doubles
// per GPU.  static_scratch_init looks up the current device's copy (once per
// device); static_scratch returns it (hipErrorNotInitialized before init).
constexpr int64_t kStaticMetricVoxels = int64_t(1) << 21;
hipError_t static_scratch_init(int device);
hipError_t static_scratch(int device, double** out);

}  // namespace mrf
