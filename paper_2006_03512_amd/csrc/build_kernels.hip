// Graph construction on gfx950: ray clipping and 3D-DDA traversal
// (Amanatides-Woo, the traversal Sec. IV-A names; truncation 3 sigma past the
// measurement, Sec. IV-B), device exclusive scans, a stable LSD radix sort
// for the voxel->ray incidence, and the work lists of the message kernels.
//
// The traversal is FP64 and compiled with -ffp-contract=off: every rounding
// step is an IEEE-754 operation on doubles in a fixed order, so the voxel
// ids and chord end points are reproducible bit for bit by any FP64
// implementation that performs the same operations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "dev_common.hpp"
#include "mrf_internal.hpp"

namespace mrf {

// ============================================================== traversal

struct Ray {
    double c[3], w[3];
    double Z, ts, te;
};

// Ray of pixel (u, v): centre c, direction R (x_n, y_n, 1) (t is z-depth),
// clipped to the grid box: [ts, texit].  False when the pixel has no usable
// measurement or the ray misses the grid.
__device__ bool clip_ray(const SceneDev& sd, const BuildDev& bp, const double* T, float zf, int v, int u,
                         Ray& r, double& ts_out, double& texit_out)
{
    const double Z = (double)zf;
    if (!isfinite(Z) || Z < bp.z_min || Z > bp.z_max) return false;
    const double xn = ((double)u - sd.cx) / sd.fx;
    const double yn = ((double)v - sd.cy) / sd.fy;
    double ts = 0.0, texit = __builtin_huge_val();
    for (int a = 0; a < 3; ++a) {
        r.c[a] = T[4 * a + 3];
        double wa = T[4 * a + 0] * xn;
        wa = wa + T[4 * a + 1] * yn;
        wa = wa + T[4 * a + 2];
        r.w[a] = wa;
        if (!isfinite(wa) || !isfinite(r.c[a])) return false;   // unusable pose
        const double lo = sd.o[a];
        const double hi = sd.o[a] + (double)sd.n[a] * sd.h;
        if (wa != 0.0) {
            const double t0 = (lo - r.c[a]) / wa;
            const double t1 = (hi - r.c[a]) / wa;
            const double tmn = t0 < t1 ? t0 : t1;
            const double tmx = t0 < t1 ? t1 : t0;
            if (tmn > ts) ts = tmn;
            if (tmx < texit) texit = tmx;
        } else if (r.c[a] < lo || r.c[a] >= hi) {
            return false;
        }
    }
    r.Z = Z;
    ts_out = ts;
    texit_out = texit;
    return true;
}

// The graph's ray: the clipped ray of a surface inside the grid, walked to
// Z + nsig * sigma_tr(Z) or the grid exit.
__device__ bool setup_ray(const SceneDev& sd, const BuildDev& bp, const double* T, float zf,
                          int v, int u, Ray& r)
{
    double ts, texit;
    if (!clip_ray(sd, bp, T, zf, v, u, r, ts, texit)) return false;
    const double Z = r.Z;
    if (Z >= texit) return false;   // surface outside the grid
    double sig = bp.c2 * Z;
    sig = sig * Z;
    sig = bp.c0 + sig;
    if (sig < bp.smin) sig = bp.smin;
    double te = Z + bp.nsig * sig;
    if (te > texit) te = texit;
    if (te <= ts) return false;
    r.ts = ts;
    r.te = te;
    return true;
}

__device__ __forceinline__ double face(const SceneDev& sd, int a, int idx)
{
    return sd.o[a] + (double)idx * sd.h;
}

// Boundary time of voxel index i along axis a in the walk's direction (the
// face the ray leaves voxel i through), +inf when the ray is parallel to it.
__device__ __forceinline__ double tmax_at(const SceneDev& sd, const Ray& r, int a, int i)
{
    if (r.w[a] > 0.0) return (face(sd, a, i + 1) - r.c[a]) / r.w[a];
    if (r.w[a] < 0.0) return (face(sd, a, i) - r.c[a]) / r.w[a];
    return __builtin_huge_val();
}

// The last voxel along axis a inside brick b in the walk's direction (the
// grid's last voxel for a partial brick); cur when the ray is parallel to a.
__device__ __forceinline__ int brick_last(const SceneDev& sd, const Ray& r, int a, int b, int cur)
{
    if (r.w[a] > 0.0) return min(b * kBrick + kBrick - 1, sd.n[a] - 1);
    if (r.w[a] < 0.0) return b * kBrick;
    return cur;
}

// Walk voxels from ts to te; emit(k, i, j, kz, tin, tout) for each chord of
// positive length (voxel (i, j, kz)) in an allocated brick (every brick when
// bricks is null); ties between axes step the lowest axis.  Returns count.
//
// Empty-space skip (Sec. IV-B: rays skip unallocated bricks), when skip is
// set: from a voxel of an unallocated brick the walk steps brick by brick.  The ray leaves a brick
// along an axis at the boundary time of its last voxel there (the expression
// the voxel walk evaluates at that voxel), so stepping the axis with the
// earliest such time (ties: lowest axis) visits the bricks in the voxel walk's
// order.  On entering an allocated brick across axis a at time t, every other
// axis has crossed exactly the voxel boundaries earlier than t (and one at t
// if it is the lower axis); its index is estimated from the entry point and
// settled by those comparisons.  The state then -- indices, boundary times,
// entry time -- is bit for bit the one the voxel-by-voxel walk reaches, so the
// emitted chords are unchanged.
template <class Emit>
__device__ int walk(const SceneDev& sd, const Ray& r, const uint8_t* bricks, Emit&& emit, bool skip = false)
{
    int idx[3];
    double tmax[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double p = r.c[a] + r.ts * r.w[a];
        double q = floor((p - sd.o[a]) / sd.h);
        if (q < 0.0) q = 0.0;
        if (q > (double)(sd.n[a] - 1)) q = (double)(sd.n[a] - 1);
        idx[a] = (int)q;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (r.w[a] > 0.0)
            tmax[a] = (face(sd, a, idx[a] + 1) - r.c[a]) / r.w[a];
        else if (r.w[a] < 0.0)
            tmax[a] = (face(sd, a, idx[a]) - r.c[a]) / r.w[a];
        else
            tmax[a] = __builtin_huge_val();
    }
    double tin = r.ts;
    const double inv_h = 1.0 / sd.h;
    int k = 0;
    for (;;) {
        const bool unalloc = bricks && !bricks[(idx[0] >> 3) + sd.nb[0] * ((idx[1] >> 3) + sd.nb[1] * (idx[2] >> 3))];
        if (unalloc && skip) {
            // walk brick by brick until an allocated brick, the ray's end or the grid's exit
            int bi[3], last[3];
            double tb[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                bi[a] = idx[a] >> 3;
                last[a] = brick_last(sd, r, a, bi[a], idx[a]);
                tb[a] = last[a] == idx[a] ? tmax[a] : tmax_at(sd, r, a, last[a]);
            }
            int a;
            double tm;
            bool stop = false;
            for (;;) {
                a = (tb[0] <= tb[1] && tb[0] <= tb[2]) ? 0 : (tb[1] <= tb[2] ? 1 : 2);
                tm = tb[a];
                if (tm >= r.te) {   // the ray ends in unallocated space
                    stop = true;
                    break;
                }
                bi[a] += r.w[a] > 0.0 ? 1 : -1;
                if (bi[a] < 0 || bi[a] >= sd.nb[a]) {   // it leaves the grid
                    stop = true;
                    break;
                }
                if (bricks[bi[0] + sd.nb[0] * (bi[1] + sd.nb[1] * bi[2])]) break;
                last[a] = brick_last(sd, r, a, bi[a], -1);
                tb[a] = tmax_at(sd, r, a, last[a]);
            }
            if (stop) break;
            // the voxel walk's state as it enters brick bi across axis a at time tm
            idx[a] = r.w[a] > 0.0 ? bi[a] * kBrick : min(bi[a] * kBrick + kBrick - 1, sd.n[a] - 1);
            tmax[a] = tmax_at(sd, r, a, idx[a]);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (b == a || r.w[b] == 0.0) continue;
                const int sg = r.w[b] > 0.0 ? 1 : -1;
                // b has crossed every boundary earlier than tm, and one at tm if it is the lower axis
                auto stepped = [&](double t) { return t < tm || (t == tm && b < a); };
                const int blo = bi[b] * kBrick, bhi = min(blo + kBrick - 1, sd.n[b] - 1);
                int first = sg > 0 ? blo : bhi;
                if ((idx[b] >> 3) == bi[b]) first = idx[b];   // still in the brick it started in
                const int lastb = sg > 0 ? bhi : blo;
                const double q = floor((r.c[b] + tm * r.w[b] - sd.o[b]) * inv_h);   // estimate only
                const int lo = min(first, lastb), hi = max(first, lastb);
                int i = (int)fmin(fmax(q, (double)lo), (double)hi);
                double ti = tmax_at(sd, r, b, i);
                while (i != lastb && stepped(ti)) {
                    i += sg;
                    ti = tmax_at(sd, r, b, i);
                }
                while (i != first) {
                    const double tp = tmax_at(sd, r, b, i - sg);
                    if (stepped(tp)) break;
                    i -= sg;
                    ti = tp;
                }
                idx[b] = i;
                tmax[b] = ti;   // the first boundary of b not yet crossed
            }
            if (tm > tin) tin = tm;
            continue;
        }
        const int a = (tmax[0] <= tmax[1] && tmax[0] <= tmax[2]) ? 0 : (tmax[1] <= tmax[2] ? 1 : 2);
        const double tm = tmax[a];
        const double tout = tm < r.te ? tm : r.te;
        if (tout > tin && !unalloc) {
            emit(k, idx[0], idx[1], idx[2], tin, tout);
            ++k;
        }
        if (tm >= r.te) break;
        if (tm > tin) tin = tm;
        idx[a] += r.w[a] > 0.0 ? 1 : -1;
        if (idx[a] < 0 || idx[a] >= sd.n[a]) break;
        if (r.w[a] > 0.0)
            tmax[a] = (face(sd, a, idx[a] + 1) - r.c[a]) / r.w[a];
        else
            tmax[a] = (face(sd, a, idx[a]) - r.c[a]) / r.w[a];
    }
    return k;
}

__device__ __forceinline__ const uint8_t* scene_bricks(const BuildDev& bp, const SceneDev& sd)
{
    return bp.bricks ? bp.bricks + sd.brick_off : nullptr;
}

// Sparse grid (Sec. IV-B: bricks are allocated around the reprojected depth
// points): one thread per pixel of one frame (blockIdx.y).  The measured
// surface point c + Z w of a usable measurement marks every brick within
// bp.radius bricks (per axis) of the brick of its voxel; points outside the
// grid mark nothing.  Bytes are only ever set to 1, so the mask does not
// depend on the order of the stores.
__global__ __launch_bounds__(256) void brick_mark_k(const SceneDev* __restrict__ scenes,
                                                    const FrameDev* __restrict__ frames, BuildDev bp,
                                                    uint8_t* __restrict__ bricks)
{
    const FrameDev fr = frames[blockIdx.y];
    const SceneDev& sd = scenes[fr.scene];
    const int pix = blockIdx.x * 256 + threadIdx.x;
    if (pix >= sd.W * sd.H) return;
    const int v = pix / sd.W, u = pix - v * sd.W;
    const double Z = (double)fr.depth[pix];
    if (!isfinite(Z) || Z < bp.z_min || Z > bp.z_max) return;
    const double xn = ((double)u - sd.cx) / sd.fx;
    const double yn = ((double)v - sd.cy) / sd.fy;
    const double* T = fr.T;
    int b[3];
    for (int a = 0; a < 3; ++a) {
        double wa = T[4 * a + 0] * xn;
        wa = wa + T[4 * a + 1] * yn;
        wa = wa + T[4 * a + 2];
        const double pa = T[4 * a + 3] + Z * wa;
        const double q = floor((pa - sd.o[a]) / sd.h);
        if (!(q >= 0.0 && q < (double)sd.n[a])) return;
        b[a] = (int)q / kBrick;
    }
    const int r = bp.radius;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = max(b[a] - r, 0);
        hi[a] = min(b[a] + r, sd.nb[a] - 1);
    }
    uint8_t* m = bricks + sd.brick_off;
    for (int bk = lo[2]; bk <= hi[2]; ++bk)
        for (int bj = lo[1]; bj <= hi[1]; ++bj)
            for (int bi = lo[0]; bi <= hi[0]; ++bi) m[bi + (int64_t)sd.nb[0] * (bj + (int64_t)sd.nb[1] * bk)] = 1;
}

struct NoEmit {
    __device__ void operator()(int, int, int, int, double, double) const {}
};

__global__ __launch_bounds__(256) void trace_count_k(const SceneDev* __restrict__ scenes,
                                                     const FrameDev* __restrict__ frames,
                                                     BuildDev bp, int32_t* __restrict__ counts)
{
    const FrameDev fr = frames[blockIdx.y];
    const SceneDev& sd = scenes[fr.scene];
    const int pix = blockIdx.x * 256 + threadIdx.x;
    if (pix >= sd.W * sd.H) return;
    const int v = pix / sd.W, u = pix - v * sd.W;
    Ray r;
    int m = 0;
    if (setup_ray(sd, bp, fr.T, fr.depth[pix], v, u, r)) m = walk(sd, r, scene_bricks(bp, sd), NoEmit{}, bp.skip);
    counts[fr.ray_base + pix] = m >= bp.min_vox ? m : 0;
}

// brick-major key of voxel (i, j, k) of a scene
__device__ __forceinline__ uint32_t brick_key(const SceneDev& sd, int i, int j, int k)
{
    const int64_t brick = ((int64_t)(k >> 3) * sd.nb[1] + (j >> 3)) * sd.nb[0] + (i >> 3);
    return (uint32_t)(sd.key_base + brick * 512 + ((k & 7) * 8 + (j & 7)) * 8 + (i & 7));
}

struct EdgeEmit {
    int32_t* col;
    uint32_t* key;
    float* delta;
    uint8_t* bin;
    double* tin;
    double* tout;
    float* wlen;          // chord length per edge (per-keyframe averaging), or null
    const SceneDev* sd;
    int64_t base;
    int32_t vbase;
    double Z, dbin;
    double wn;            // |w| of the ray: chord length = (t_out - t_in) |w|
    double rbin;          // 1 / dbin, correctly rounded
    // The bin is floor(d / dbin) with the quotient rounded once, as in the
    // oracle.  y = d * rbin is within about 2^-51 |d / dbin| of that quotient
    // (under 4e-10 below 2^20), so wherever y is more than 1e-9 from an integer
    // the two have the same floor; next to a bin boundary the division decides.
    // Quotients of 2^20 and more clamp to the last bin either way.
    __device__ double bin_of(double d) const
    {
        const double y = d * rbin;
        double q = floor(y);
        const double f = y - q;   // exact for y >= 0 (chord midpoints are)
        if (f < 1e-9 || f > 1.0 - 1e-9) q = floor(d / dbin);
        return q;
    }
    __device__ void operator()(int k, int vi, int vj, int vk, double ti, double to) const
    {
        const int64_t e = base + (int64_t)kTile * k;   // step k of this ray's tile lane
        const double d = (ti + to) * 0.5;   // voxel depth: chord midpoint
        double q = bin_of(d);
        if (q < 0.0) q = 0.0;
        if (q > 63.0) q = 63.0;
        col[e] = vbase + vi + sd->n[0] * (vj + sd->n[1] * vk);
        key[e] = brick_key(*sd, vi, vj, vk);
        delta[e] = (float)(Z - d);
        bin[e] = (uint8_t)q;
        if (tin) {
            tin[e] = ti;
            tout[e] = to;
        }
        if (wlen) wlen[e] = (float)((to - ti) * wn);
    }
};

// Threads are grouped by tile: the 16 lanes 16t..16t+15 of a block trace the 16 pixels
// of tile t, so at every traversal step they write one whole 64-byte line of each
// per-slot array (a row-major pixel order would write 16-byte pieces of 16 lines).
// Each lane then marks its column's slots past its ray, up to the tile's length, as
// padding (no voxel, no bin, sort key pad_key past every voxel); lanes of pixels
// outside the image pad their whole column.
__global__ __launch_bounds__(256) void trace_emit_k(const SceneDev* __restrict__ scenes,
                                                    const FrameDev* __restrict__ frames, BuildDev bp,
                                                    const int32_t* __restrict__ counts,
                                                    const int64_t* __restrict__ tbase,
                                                    const TileDev* __restrict__ tiles, uint32_t pad_key,
                                                    int32_t* col, uint32_t* key, float* delta, uint8_t* bin,
                                                    double* tin, double* tout, float* wlen)
{
    const FrameDev fr = frames[blockIdx.y];
    const SceneDev& sd = scenes[fr.scene];
    const int nty = (sd.H + kTileW - 1) / kTileW;
    const int lt = blockIdx.x * (256 / kTile) + (int)threadIdx.x / kTile;
    if (lt >= fr.ntx * nty) return;
    const int ty = lt / fr.ntx, tx = lt - ty * fr.ntx;
    const int q = (int)threadIdx.x % kTile;
    const int v = ty * kTileW + q / kTileW, u = tx * kTileW + q % kTileW;
    const int64_t t = fr.tile_base + lt;
    const int64_t slot0 = tbase[t] + q;
    const int len = tiles[t].len;
    int m = 0;
    if (v < sd.H && u < sd.W) {
        const int pix = v * sd.W + u;
        m = counts[fr.ray_base + pix];
        if (m > 0) {
            Ray ray;
            setup_ray(sd, bp, fr.T, fr.depth[pix], v, u, ray);
            double wn = ray.w[0] * ray.w[0];
            wn = wn + ray.w[1] * ray.w[1];
            wn = wn + ray.w[2] * ray.w[2];
            const double dbin = bp.dmax / 64.0;
            EdgeEmit em{col,   key,   delta, bin, tin, tout, wlen, &sd, slot0, (int32_t)sd.voxel_base, ray.Z,
                        dbin,  sqrt(wn), 1.0 / dbin};
            walk(sd, ray, scene_bricks(bp, sd), em, bp.skip);
        }
    }
    for (int k = m; k < len; ++k) {
        const int64_t e = slot0 + (int64_t)kTile * k;
        col[e] = -1;
        key[e] = pad_key;
        delta[e] = 0.0f;
        bin[e] = 255;
    }
}

// One thread per tile: its rays, extent inside the image and longest ray.
__global__ void tile_init_k(const SceneDev* __restrict__ scenes, const FrameDev* __restrict__ frames, int f0,
                            const int32_t* __restrict__ counts, TileDev* __restrict__ tiles,
                            int32_t* __restrict__ slots16, int64_t t0)
{
    const FrameDev fr = frames[f0 + blockIdx.y];
    const SceneDev& sd = scenes[fr.scene];
    const int nty = (sd.H + kTileW - 1) / kTileW;
    const int lt = blockIdx.x * blockDim.x + threadIdx.x;
    if (lt >= fr.ntx * nty) return;
    const int ty = lt / fr.ntx, tx = lt - ty * fr.ntx;
    TileDev td;
    td.ray0 = (int32_t)(fr.ray_base + (int64_t)(ty * kTileW) * sd.W + tx * kTileW);
    td.W = sd.W;
    td.nu = min(kTileW, sd.W - tx * kTileW);
    td.nv = min(kTileW, sd.H - ty * kTileW);
    int len = 0;
    for (int a = 0; a < td.nv; ++a)
        for (int b = 0; b < td.nu; ++b) len = max(len, counts[td.ray0 + a * sd.W + b]);
    td.len = len;
    td.base = 0;
    td.frame = f0 + (int32_t)blockIdx.y;
    tiles[fr.tile_base + lt] = td;
    slots16[fr.tile_base + lt - t0] = kTile * len;
}

__global__ void tile_base_k(TileDev* __restrict__ tiles, const int64_t* __restrict__ tbase, int64_t T)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < T) tiles[t].base = tbase[t];
}

__global__ void fill_u32_k(uint32_t* __restrict__ p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_brick_mask(mrf_ctx* c, hipStream_t s)
{
    hipError_t e = launch_fill_u32((uint32_t*)c->b_bricks.p, 0u, (c->n_bricks + 3) / 4, s);
    if (e != hipSuccess) return e;
    dim3 grid((c->max_hw + 255) / 256, c->n_frames);
    hipLaunchKernelGGL(brick_mark_k, grid, dim3(256), 0, s, (const SceneDev*)c->b_scenes.p,
                       (const FrameDev*)c->b_frames.p, c->bp, (uint8_t*)c->b_bricks.p);
    return hipGetLastError();
}

hipError_t launch_trace_count(mrf_ctx* c, hipStream_t s, int f0, int nf)
{
    if (nf < 0) nf = c->n_frames - f0;
    if (nf <= 0) return hipSuccess;
    dim3 grid((c->max_hw + 255) / 256, nf);
    hipLaunchKernelGGL(trace_count_k, grid, dim3(256), 0, s, (const SceneDev*)c->b_scenes.p,
                       (const FrameDev*)c->b_frames.p + f0, c->bp, (int32_t*)c->b_counts.p);
    return hipGetLastError();
}

hipError_t launch_tiles(mrf_ctx* c, int32_t* slots16, hipStream_t s, int f0, int nf)
{
    if (nf < 0) nf = c->n_frames - f0;
    if (nf <= 0) return hipSuccess;
    int max_tiles = 0;
    for (const auto& sd : c->scenes_h)
        max_tiles = std::max(max_tiles, ((sd.W + kTileW - 1) / kTileW) * ((sd.H + kTileW - 1) / kTileW));
    dim3 grid((max_tiles + 255) / 256, nf);
    hipLaunchKernelGGL(tile_init_k, grid, dim3(256), 0, s, (const SceneDev*)c->b_scenes.p,
                       (const FrameDev*)c->b_frames.p, f0, (const int32_t*)c->b_counts.p, (TileDev*)c->b_tiles.p,
                       slots16, c->frames_h[f0].tile_base);
    return hipGetLastError();
}

hipError_t launch_tile_bases(mrf_ctx* c, hipStream_t s, int64_t t0)
{
    if (c->T > t0)
        hipLaunchKernelGGL(tile_base_k, dim3((unsigned)((c->T - t0 + 255) / 256)), dim3(256), 0, s,
                           (TileDev*)c->b_tiles.p + t0, (const int64_t*)c->b_tbase.p + t0, c->T - t0);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    hipLaunchKernelGGL(fill_u32_k, dim3((unsigned)b), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

__global__ void scatter_by_slot_k(const uint32_t* __restrict__ slot, const float* __restrict__ in, int64_t n,
                                  float* __restrict__ out)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        out[slot[j]] = in[j];
}

hipError_t launch_scatter_by_slot(const uint32_t* slot, const float* in, int64_t n, float* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    hipLaunchKernelGGL(scatter_by_slot_k, dim3((unsigned)b), dim3(256), 0, s, slot, in, n, out);
    return hipGetLastError();
}

hipError_t launch_trace_emit(mrf_ctx* c, hipStream_t s, int f0, int nf)
{
    if (nf < 0) nf = c->n_frames - f0;
    if (nf <= 0) return hipSuccess;
    dim3 grid((unsigned)((c->max_tpf + 256 / kTile - 1) / (256 / kTile)), nf);
    hipLaunchKernelGGL(trace_emit_k, grid, dim3(256), 0, s, (const SceneDev*)c->b_scenes.p,
                       (const FrameDev*)c->b_frames.p + f0, c->bp, (const int32_t*)c->b_counts.p,
                       (const int64_t*)c->b_tbase.p, (const TileDev*)c->b_tiles.p, (uint32_t)c->Vk,
                       (int32_t*)c->b_col.p, (uint32_t*)c->b_g.p, (float*)c->b_delta.p, (uint8_t*)c->b_bin.p,
                       c->keep_chords ? (double*)c->b_tin.p : nullptr,
                       c->keep_chords ? (double*)c->b_tout.p : nullptr, c->kf ? (float*)c->b_kflen.p : nullptr);
    return hipGetLastError();
}

// ============================================================== scans

constexpr int SC_T = 256, SC_IPT = 8, SC_TILE = SC_T * SC_IPT;

struct LoadI32 {
    const int32_t* p;
    __device__ int64_t operator()(int64_t i) const { return p[i]; }
};
struct LoadI64 {
    const int64_t* p;
    __device__ int64_t operator()(int64_t i) const { return p[i]; }
};
struct LoadEqU8 {
    const uint8_t* p;
    uint8_t c;
    __device__ int64_t operator()(int64_t i) const { return p[i] == c ? 1 : 0; }
};

__device__ int64_t block_excl_scan_i64(int64_t x, int64_t* total)
{
    __shared__ int64_t wsum[SC_T / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < SC_T / 64; ++i) {
        if (i < w) off += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return off + incl - x;
}

template <class Load>
__global__ __launch_bounds__(SC_T) void scan_reduce_k(Load ld, int64_t n, int64_t* __restrict__ bsum)
{
    const int64_t base = (int64_t)blockIdx.x * SC_TILE;
    int64_t acc = 0;
#pragma unroll
    for (int k = 0; k < SC_IPT; ++k) {
        const int64_t i = base + k * SC_T + threadIdx.x;
        if (i < n) acc += ld(i);
    }
    int64_t tot;
    block_excl_scan_i64(acc, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

template <class Load, class Out>
__global__ __launch_bounds__(SC_T) void scan_apply_k(Load ld, int64_t n, const int64_t* __restrict__ boff,
                                                     Out* __restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_IPT;
    int64_t v[SC_IPT];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SC_IPT; ++k) {
        const int64_t i = base + k;
        v[k] = i < n ? ld(i) : 0;
        s += v[k];
    }
    int64_t tot;
    int64_t ex = block_excl_scan_i64(s, &tot) + (boff ? boff[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < SC_IPT; ++k) {
        const int64_t i = base + k;
        if (i < n) out[i] = (Out)ex;
        ex += v[k];
        if (i == n - 1) out[n] = (Out)ex;
    }
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

size_t scan_tmp_bytes(int64_t n)
{
    size_t words = 0;
    int64_t m = n;
    while (cdiv(m, SC_TILE) > 1) {
        const int64_t nb = cdiv(m, SC_TILE);
        words += 2 * nb + 1;
        m = nb;
    }
    return (words + 8) * sizeof(int64_t);
}

template <class Out>
__global__ void zero_k(Out* p) { *p = 0; }

// Exclusive scan of ld(0..n-1) into out[0..n] (out[n] = the total), written as
// Out (the caller guarantees the total fits); tmp holds scan_tmp_bytes(n).
template <class Load, class Out = int64_t>
static hipError_t scan_rec(Load ld, int64_t n, Out* out, int64_t* tmp, hipStream_t s)
{
    if (n == 0) {
        hipLaunchKernelGGL(zero_k<Out>, dim3(1), dim3(1), 0, s, out);
        return hipGetLastError();
    }
    const int64_t nb = cdiv(n, SC_TILE);
    if (nb == 1) {
        hipLaunchKernelGGL((scan_apply_k<Load, Out>), dim3(1), dim3(SC_T), 0, s, ld, n, (const int64_t*)nullptr,
                           out);
        return hipGetLastError();
    }
    int64_t* bsum = tmp;
    int64_t* boff = tmp + nb;
    hipLaunchKernelGGL(scan_reduce_k<Load>, dim3((unsigned)nb), dim3(SC_T), 0, s, ld, n, bsum);
    hipError_t e = scan_rec(LoadI64{bsum}, nb, boff, tmp + 2 * nb + 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((scan_apply_k<Load, Out>), dim3((unsigned)nb), dim3(SC_T), 0, s, ld, n, (const int64_t*)boff,
                       out);
    return hipGetLastError();
}

hipError_t scan_exclusive_i32(const int32_t* in, int64_t* out, int64_t n, void* tmp, size_t tmp_bytes,
                              hipStream_t s)
{
    if (tmp_bytes < scan_tmp_bytes(n)) return hipErrorInvalidValue;
    return scan_rec(LoadI32{in}, n, out, (int64_t*)tmp, s);
}

// ============================================================== radix sort

#ifndef MRF_RS_T
#define MRF_RS_T 256
#define MRF_RS_IPT 16
#endif
constexpr int RS_T = MRF_RS_T, RS_IPT = MRF_RS_IPT, RS_TILE = RS_T * RS_IPT;
static_assert(RS_T == 256 && RS_IPT % 4 == 0, "radix tile shape: one thread per digit");

constexpr int RS_CB = 256;   // tiles per chunk of the digit-offset scan

size_t radix_hist_entries(int64_t n) { return (size_t)256 * (size_t)cdiv(n > 0 ? n : 1, RS_TILE); }

size_t radix_tmp_bytes(int64_t n)
{
    const int64_t nch = cdiv(cdiv(n > 0 ? n : 1, RS_TILE), RS_CB);
    return sizeof(int64_t) * (size_t)(2 * 256 * nch + 256);
}

// Lanes of a wave holding digit d (of valid items): 8 ballots.  Per bit, with
// s the bit sign-extended (all ones when set, 0 when clear) and m the lanes
// whose bit is set, the lanes that agree with this lane are ~(m ^ s); each
// 32-bit half is updated with one three-input bit operation, p & ~(m ^ s)
// (truth table 0x90 over (p, m, s)), instead of a select of the 64-bit mask.
__device__ __forceinline__ uint64_t rs_peers(int d, bool valid)
{
    const uint64_t v = __ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint32_t sb = (uint32_t)((int32_t)((uint32_t)d << (31 - b)) >> 31);   // 0 or all ones
        const uint64_t m = __ballot(sb != 0u);
        lo = __builtin_amdgcn_bitop3_b32(lo, (uint32_t)m, sb, 0x90);
        hi = __builtin_amdgcn_bitop3_b32(hi, (uint32_t)(m >> 32), sb, 0x90);
    }
    return ((uint64_t)hi << 32) | lo;
}

// Digit counts of one tile of RS_TILE keys.  Thread t takes RS_IPT
// consecutive keys (vector loads) and adds each run of equal digits with one
// LDS atomic: keys in slot order come in runs (the rays of a tile cross the
// same voxels at the same step), which would otherwise serialise the atomics
// of a wave on a few addresses.  RS_TILE is a multiple of 16 and n of 4 is
// not assumed: the tile's tail is read key by key.
__global__ __launch_bounds__(RS_T) void rs_hist_k(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                  int32_t* __restrict__ hist, int64_t nblocks)
{
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    const int64_t i0 = (int64_t)blockIdx.x * RS_TILE + (int64_t)threadIdx.x * RS_IPT;
    uint32_t kr[RS_IPT];
    if (i0 + RS_IPT <= n) {
        const uint4* p = (const uint4*)(keys + i0);   // keys and RS_IPT * 4 bytes: 16-byte aligned
#pragma unroll
        for (int q = 0; q < RS_IPT / 4; ++q) {
            const uint4 w = p[q];
            kr[4 * q] = w.x;
            kr[4 * q + 1] = w.y;
            kr[4 * q + 2] = w.z;
            kr[4 * q + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < RS_IPT; ++j) kr[j] = i0 + j < n ? keys[i0 + j] : 0u;
    }
    const int nv = (int)(n - i0 < RS_IPT ? (n - i0 > 0 ? n - i0 : 0) : RS_IPT);
    __syncthreads();
    if (nv > 0) {
        int cur = (kr[0] >> shift) & 255, cnt = 1;
#pragma unroll
        for (int j = 1; j < RS_IPT; ++j) {
            const int d = (kr[j] >> shift) & 255;
            if (j < nv) {
                if (d == cur) {
                    ++cnt;
                } else {
                    atomicAdd(&h[cur], cnt);
                    cur = d;
                    cnt = 1;
                }
            }
        }
        atomicAdd(&h[cur], cnt);
    }
    __syncthreads();
    hist[(int64_t)blockIdx.x * 256 + threadIdx.x] = h[threadIdx.x];
}

// Digit offsets from the tile-major (tile, digit) counts, in three steps:
// per-chunk column sums (coalesced rows), an exclusive scan of each digit's
// chunk sums (one block per digit), and per-tile running sums inside each
// chunk on top of the digit's base (the exclusive scan of the digit totals).
__global__ __launch_bounds__(256) void rs_colsum_k(const int32_t* __restrict__ hist, int64_t nb,
                                                   int64_t* __restrict__ csum)
{
    const int64_t b0 = (int64_t)blockIdx.x * RS_CB;
    const int64_t b1 = b0 + RS_CB < nb ? b0 + RS_CB : nb;
    int64_t acc = 0;
#pragma unroll 8
    for (int64_t b = b0; b < b1; ++b) acc += hist[b * 256 + threadIdx.x];
    csum[(int64_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

// block d: coff[c][d] = items of digit d in chunks < c; dtot[d] = all of them
__global__ __launch_bounds__(256) void rs_colscan_k(const int64_t* __restrict__ csum, int64_t nch,
                                                    int64_t* __restrict__ coff, int64_t* __restrict__ dtot)
{
    const int d = blockIdx.x;
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nch; c0 += 256) {
        const int64_t c = c0 + threadIdx.x;
        const int64_t x = c < nch ? csum[c * 256 + d] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan_i64(x, &tot);
        if (c < nch) coff[c * 256 + d] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) dtot[d] = carry;
}

// offs[b][d]: output position of tile b's first item of digit d
__global__ __launch_bounds__(256) void rs_offsets_k(const int32_t* __restrict__ hist, int64_t nb,
                                                    const int64_t* __restrict__ coff,
                                                    const int64_t* __restrict__ dtot, int64_t* __restrict__ offs)
{
    const int64_t b0 = (int64_t)blockIdx.x * RS_CB;
    const int64_t b1 = b0 + RS_CB < nb ? b0 + RS_CB : nb;
    int64_t total;
    const int64_t base = block_excl_scan_i64(dtot[threadIdx.x], &total);
    int64_t run = base + coff[(int64_t)blockIdx.x * 256 + threadIdx.x];
    for (int64_t b = b0; b < b1; ++b) {
        offs[b * 256 + threadIdx.x] = run;
        run += hist[b * 256 + threadIdx.x];
    }
}

// Stable scatter of one tile of RS_TILE items.  Wave w owns items
// [w RS_IPT 64, (w + 1) RS_IPT 64) of the tile, RS_IPT rounds of 64; equal
// digits inside a round are matched with wave ballots.  A first walk counts
// each wave's digits, the per-wave bases follow in digit-major, wave-minor
// order (index order, hence stable), and a second walk places every item in
// an LDS copy of the tile grouped by digit: two barriers in all.  The copy is
// then written out as contiguous runs, one per digit, at the digit's global
// offset for this tile (coalesced stores in place of scattered words).  Tile
// t's run of a digit ends where tile t+1's begins, so consecutive tiles run on
// one XCD (block remap) and their shared lines merge in its L2.  hist
// and offs hold the tile's digit counts and output offsets (tile-major rows
// of 256).
__global__ __launch_bounds__(RS_T) void rs_scatter_k(const uint32_t* __restrict__ keys_in,
                                                     const uint32_t* __restrict__ vals_in, int64_t n,
                                                     int shift, const int32_t* __restrict__ hist,
                                                     const int64_t* __restrict__ offs,
                                                     uint32_t* __restrict__ keys_out,
                                                     uint32_t* __restrict__ vals_out, const SlotGroups groups)
{
    constexpr int NW = RS_T / 64;
    constexpr int WI = RS_IPT * 64;   // items per wave
    __shared__ uint32_t lk[RS_TILE];
    __shared__ uint32_t lv[RS_TILE];
    __shared__ int64_t boff[256];
    __shared__ int32_t dstart[256];
    __shared__ int32_t wcnt[NW][256];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform across the wave
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);   // neighbouring tiles on one XCD
    const int64_t start = tile * RS_TILE;
    const int64_t wstart = start + (int64_t)w * WI;
    // items of this wave below n: item r * 64 + lane is valid iff it is < nvw
    const int64_t rem = n - wstart;
    const int nvw = rem <= 0 ? 0 : (rem < WI ? (int)rem : WI);
    uint32_t kr[RS_IPT], vr[RS_IPT];
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r) {
        const int64_t i = wstart + r * 64 + lane;
        const int64_t ic = i < n ? i : n - 1;
        kr[r] = keys_in[ic];
        if (vals_in) vr[r] = vals_in[ic];
    }
    if (!vals_in) {   // first pass: the values are the slots, relative to their group's first slot
        if (groups.n > 1) {
#pragma unroll
            for (int r = 0; r < RS_IPT; ++r) {
                const int64_t i = wstart + r * 64 + lane;
                vr[r] = (uint32_t)(i - group_slot_base_of_slot(groups, i));
            }
        } else {
#pragma unroll
            for (int r = 0; r < RS_IPT; ++r) vr[r] = (uint32_t)(wstart + r * 64 + lane);
        }
    }
    const int64_t o0 = offs[tile * 256 + tid];
    const int64_t cnt = hist[tile * 256 + tid];
    boff[tid] = o0;
#pragma unroll
    for (int q = 0; q < NW; ++q) wcnt[q][tid] = 0;
    int64_t total;
    dstart[tid] = (int32_t)block_excl_scan_i64(cnt, &total);   // synchronises the block
    const uint64_t below = lane ? ((~0ull) >> (64 - lane)) : 0ull;
    // walk 1: digit counts of this wave (the lowest lane of each digit adds;
    // the digits of one round are distinct, so no two lanes share an address).
    // Each item keeps its rank among equal digits of its round and their
    // count, packed as rank | count << 8 (both <= 64).
    int rc[RS_IPT];
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r) {
        const bool valid = r * 64 + lane < nvw;
        const int d = (kr[r] >> shift) & 255;
        const uint64_t peers = rs_peers(d, valid);
        const int rank = __popcll(peers & below), num = __popcll(peers);
        rc[r] = rank | (num << 8);
        if (valid && rank == 0) wcnt[w][d] += num;
    }
    __syncthreads();
    {   // thread = digit: wave bases inside the tile's LDS copy
        int acc = dstart[tid];
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const int t = wcnt[q][tid];
            wcnt[q][tid] = acc;
            acc += t;
        }
    }
    __syncthreads();
    // walk 2: place the items; a round's lanes read their digit's base before
    // the lowest lane of each digit advances it (LDS operations of a wave
    // complete in order)
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r) {
        const bool valid = r * 64 + lane < nvw;
        const int d = (kr[r] >> shift) & 255;
        const int rank = rc[r] & 255;
        const int b = wcnt[w][d];
        if (valid) {
            lk[b + rank] = kr[r];
            lv[b + rank] = vr[r];
        }
        if (valid && rank == 0) wcnt[w][d] = b + (rc[r] >> 8);
    }
    __syncthreads();
    const int tn = (int)(n - start < RS_TILE ? n - start : RS_TILE);
    for (int j = tid; j < tn; j += RS_T) {
        const uint32_t key = lk[j];
        const int d = (key >> shift) & 255;
        const int64_t pos = boff[d] + (j - dstart[d]);
        keys_out[pos] = key;
        vals_out[pos] = lv[j];
    }
}

hipError_t radix_sort_pairs(const uint32_t* keys_in, uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                            uint32_t* vals_b, uint32_t* keys_out, uint32_t* vals_out, int64_t n,
                            int key_bits, int32_t* hist, int64_t* offs, void* tmp, size_t tmp_bytes,
                            hipStream_t s, const SlotGroups& groups)
{
    if (n == 0) return hipSuccess;
    const int passes = key_bits <= 8 ? 1 : (key_bits + 7) / 8;
    const int64_t nb = cdiv(n, RS_TILE);
    const int64_t nch = cdiv(nb, RS_CB);
    if (tmp_bytes < radix_tmp_bytes(n)) return hipErrorInvalidValue;
    for (const uint32_t* k : {keys_in, (const uint32_t*)keys_a, (const uint32_t*)keys_b})   // rs_hist_k's 16-byte loads
        if ((uintptr_t)k % 16 != 0) return hipErrorInvalidValue;
    int64_t* csum = (int64_t*)tmp;
    int64_t* coff = csum + 256 * nch;
    int64_t* dtot = coff + 256 * nch;
    const uint32_t* sk = keys_in;
    const uint32_t* sv = nullptr;
    for (int p = 0; p < passes; ++p) {
        uint32_t* dk = (p == passes - 1) ? keys_out : ((p & 1) ? keys_b : keys_a);
        uint32_t* dv = (p == passes - 1) ? vals_out : ((p & 1) ? vals_b : vals_a);
        hipLaunchKernelGGL(rs_hist_k, dim3((unsigned)nb), dim3(RS_T), 0, s, sk, n, 8 * p, hist, nb);
        hipLaunchKernelGGL(rs_colsum_k, dim3((unsigned)nch), dim3(256), 0, s, (const int32_t*)hist, nb, csum);
        hipLaunchKernelGGL(rs_colscan_k, dim3(256), dim3(256), 0, s, (const int64_t*)csum, nch, coff, dtot);
        hipLaunchKernelGGL(rs_offsets_k, dim3((unsigned)nch), dim3(256), 0, s, (const int32_t*)hist, nb,
                           (const int64_t*)coff, (const int64_t*)dtot, offs);
        hipLaunchKernelGGL(rs_scatter_k, dim3((unsigned)nb), dim3(RS_T), 0, s, sk, sv, n, 8 * p,
                           (const int32_t*)hist, (const int64_t*)offs, dk, dv, groups);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        sk = dk;
        sv = dv;
    }
    return hipSuccess;
}

// vptr[v] = first position whose key >= v (binary search), v in [0, V]
__global__ void vptr_k(const uint32_t* __restrict__ keys, int64_t n, int64_t V, int64_t* __restrict__ vptr)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > V) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)keys[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    vptr[v] = lo;
}

hipError_t launch_vptr_from_sorted(const uint32_t* sorted_keys, int64_t n, int64_t V, int64_t* vptr,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(vptr_k, dim3((unsigned)cdiv(V + 1, 256)), dim3(256), 0, s, sorted_keys, n, V, vptr);
    return hipGetLastError();
}

// ============================================================== work lists

// length class of every tile (255: no edges)
__global__ void tile_class_k(const TileDev* __restrict__ tiles, int64_t T, uint8_t* __restrict__ cls)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const int n = tiles[t].len;
    uint8_t c = 255;
    if (n > 0) {
        c = kRayClasses;   // too long: reported as an error by the host
        for (int k = 0; k < kRayClasses; ++k)
            if (n <= kRayCap[k]) {
                c = (uint8_t)k;
                break;
            }
    }
    cls[t] = c;
}

// degree class of every brick-major key (kVoxClasses: too large, 255: empty)
__global__ void vox_class_k(const int64_t* __restrict__ vptr, int64_t Vk, uint8_t* __restrict__ cls)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= Vk) return;
    const int64_t m = vptr[v + 1] - vptr[v];
    uint8_t c = 255;
    if (m > 0) {
        c = kVoxClasses - 1;
        for (int k = 0; k < kVoxClasses - 1; ++k)
            if (m <= kVoxCap[k]) {
                c = (uint8_t)k;
                break;
            }
        if (m > 2147483647LL) c = kVoxClasses;
    }
    cls[v] = c;
}

// linear voxel id of a brick-major key (keys of padding voxels never appear)
__device__ uint32_t key_to_voxel(const SceneDev* __restrict__ scenes, int ns, uint32_t key)
{
    int sc = 0;
    while (sc + 1 < ns && (int64_t)key >= scenes[sc + 1].key_base) ++sc;
    const SceneDev& sd = scenes[sc];
    const int64_t local = (int64_t)key - sd.key_base;
    const int64_t brick = local >> 9;
    const int l = (int)(local & 511);
    const int bx = (int)(brick % sd.nb[0]);
    const int by = (int)((brick / sd.nb[0]) % sd.nb[1]);
    const int bz = (int)(brick / ((int64_t)sd.nb[0] * sd.nb[1]));
    const int i = bx * 8 + (l & 7), j = by * 8 + ((l >> 3) & 7), k = bz * 8 + (l >> 6);
    return (uint32_t)(sd.voxel_base + i + (int64_t)sd.n[0] * (j + (int64_t)sd.n[1] * k));
}

__global__ void vox_desc_k(const SceneDev* __restrict__ scenes, int ns, const uint32_t* __restrict__ keys, int64_t n,
                           const int64_t* __restrict__ vptr, VoxDev* __restrict__ desc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t key = keys[i];
    VoxDev d;
    d.start = vptr[key];
    d.m = (int32_t)(vptr[key + 1] - d.start);
    d.v = key_to_voxel(scenes, ns, key);
    desc[i] = d;
}

// brick-major key of a linear voxel id
__device__ uint32_t voxel_to_key(const SceneDev* __restrict__ scenes, int ns, int64_t v)
{
    int sc = 0;
    while (sc + 1 < ns && v >= scenes[sc + 1].voxel_base) ++sc;
    const SceneDev& sd = scenes[sc];
    const int64_t local = v - sd.voxel_base;
    const int64_t nxy = (int64_t)sd.n[0] * sd.n[1];
    const int k = (int)(local / nxy);
    const int64_t rem = local - k * nxy;
    const int j = (int)(rem / sd.n[0]), i = (int)(rem - (int64_t)j * sd.n[0]);
    return brick_key(sd, i, j, k);
}

// canonical incidence: degree per linear voxel, then each voxel's edge list
__global__ void canon_degree_k(const SceneDev* __restrict__ scenes, int ns, const int64_t* __restrict__ vptr,
                               int64_t V, int32_t* __restrict__ deg)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const uint32_t k = voxel_to_key(scenes, ns, v);
    deg[v] = (int32_t)(vptr[k + 1] - vptr[k]);
}

// first slot of ray r (its tile's base plus its lane)
__device__ int64_t ray_slot0(const FrameDev* __restrict__ frames, int nf, const SceneDev* __restrict__ scenes,
                             const int64_t* __restrict__ tbase, int64_t r)
{
    int lo = 0, hi = nf;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (frames[mid].ray_base <= r)
            lo = mid;
        else
            hi = mid;
    }
    const FrameDev fr = frames[lo];
    const int W = scenes[fr.scene].W;
    const int64_t pix = r - fr.ray_base;
    const int v = (int)(pix / W), u = (int)(pix - (int64_t)v * W);
    return tbase[fr.tile_base + (int64_t)(v / kTileW) * fr.ntx + u / kTileW] + (v % kTileW) * kTileW + u % kTileW;
}

template <class T>
__global__ void canon_edges_k(const FrameDev* __restrict__ frames, int nf, const SceneDev* __restrict__ scenes,
                              const int64_t* __restrict__ tbase, const int64_t* __restrict__ row_ptr, int64_t R,
                              const T* __restrict__ in, T* __restrict__ out)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const int64_t d = row_ptr[r], m = row_ptr[r + 1] - d;
    if (m == 0) return;
    const int64_t s0 = ray_slot0(frames, nf, scenes, tbase, r);
    for (int64_t k = 0; k < m; ++k) out[d + k] = in[s0 + kTile * k];
}

__global__ void compact_k(const uint8_t* __restrict__ cls, int64_t n, uint8_t c,
                          const int64_t* __restrict__ pos, uint32_t* __restrict__ list)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && cls[i] == c) list[pos[i]] = (uint32_t)i;
}

}  // namespace mrf

namespace mrf {

// lower_bound of every frame's first ray id in every class list
__global__ void frame_offsets_k(const uint32_t* const* __restrict__ lists, const int64_t* __restrict__ cnt,
                                const int64_t* __restrict__ fbase, int32_t nf, int64_t* __restrict__ out)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (f > nf) return;
    const uint32_t* L = lists[c];
    int64_t lo = 0, hi = cnt[c];
    const int64_t key = fbase[f];
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)L[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    out[(int64_t)c * (nf + 1) + f] = lo;
}

// log2 histograms of ray lengths and voxel degrees (integer atomics only)
__global__ void hist_k(const int32_t* __restrict__ counts, int64_t R, const int64_t* __restrict__ vptr,
                       int64_t V, unsigned long long* __restrict__ h)
{
    __shared__ unsigned long long loc[16 + 24 + 2];
    for (int i = threadIdx.x; i < 42; i += blockDim.x) loc[i] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < R) {
        const int n = counts[i];
        if (n > 0) {
            const int b = min(15, 31 - __clz(n));
            atomicAdd(&loc[b], 1ull);
            atomicMax(&loc[40], (unsigned long long)n);
        }
    }
    if (i < V) {
        const int64_t m = vptr[i + 1] - vptr[i];
        if (m > 0) {
            const int b = min(23, 63 - __clzll(m));
            atomicAdd(&loc[16 + b], 1ull);
            atomicMax(&loc[41], (unsigned long long)m);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 42; k += blockDim.x) {
        if (loc[k] == 0) continue;
        if (k >= 40)
            atomicMax(&h[k], loc[k]);
        else
            atomicAdd(&h[k], loc[k]);
    }
}

// total edges and rays of the tiles of one class list (integer atomics: exact)
__global__ void tile_class_edges_k(const uint32_t* __restrict__ list, int64_t n, const TileDev* __restrict__ tiles,
                                   const int32_t* __restrict__ counts, unsigned long long* __restrict__ out_e,
                                   unsigned long long* __restrict__ out_r)
{
    __shared__ unsigned long long acc, accr;
    if (threadIdx.x == 0) acc = accr = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const TileDev td = tiles[list[i]];
        unsigned long long sum = 0, nr = 0;
        for (int a = 0; a < td.nv; ++a)
            for (int b = 0; b < td.nu; ++b) {
                const int x = counts[td.ray0 + a * td.W + b];
                sum += (unsigned long long)x;
                nr += x > 0;
            }
        atomicAdd(&acc, sum);
        atomicAdd(&accr, nr);
    }
    __syncthreads();
    if (threadIdx.x == 0 && acc) {
        atomicAdd(out_e, acc);
        atomicAdd(out_r, accr);
    }
}

// total edges of the items of one class list (integer atomics: exact)
__global__ void class_edges_k(const uint32_t* __restrict__ list, int64_t n, const int64_t* __restrict__ ptr,
                              unsigned long long* __restrict__ out)
{
    __shared__ unsigned long long acc;
    if (threadIdx.x == 0) acc = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const uint32_t x = list[i];
        atomicAdd(&acc, (unsigned long long)(ptr[x + 1] - ptr[x]));
    }
    __syncthreads();
    if (threadIdx.x == 0 && acc) atomicAdd(out, acc);
}

static hipError_t partition(const uint8_t* cls, int64_t n, uint8_t c, int64_t* pos, void* tmp,
                            size_t tmp_bytes, DevBuf& list, int64_t* count, hipStream_t s)
{
    if (tmp_bytes < scan_tmp_bytes(n)) return hipErrorInvalidValue;
    hipError_t e = scan_rec(LoadEqU8{cls, c}, n, pos, (int64_t*)tmp, s);
    if (e != hipSuccess) return e;
    int64_t total = 0;
    if ((e = hipMemcpyAsync(&total, pos + n, sizeof(int64_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    *count = total;
    if ((e = ensure(list, (size_t)(total > 0 ? total : 1) * sizeof(uint32_t))) != hipSuccess) return e;
    if (total > 0)
        hipLaunchKernelGGL(compact_k, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, cls, n, c,
                           (const int64_t*)pos, (uint32_t*)list.p);
    return hipGetLastError();
}

hipError_t build_classes(mrf_ctx* c, hipStream_t s)
{
    hipError_t e;
    const int64_t nmax = std::max(c->R, std::max(c->Vk, c->T));
    if ((e = ensure(c->b_cls, (size_t)(nmax + 1))) != hipSuccess) return e;
    if ((e = ensure(c->b_tmp64, (size_t)(nmax + 2) * sizeof(int64_t))) != hipSuccess) return e;
    const size_t sbytes = scan_tmp_bytes(nmax + 1);
    if ((e = ensure(c->b_misc, sbytes)) != hipSuccess) return e;
    uint8_t* cls = (uint8_t*)c->b_cls.p;
    int64_t* pos = (int64_t*)c->b_tmp64.p;

    // tiles of rays, by their longest ray
    if (c->T > 0)
        hipLaunchKernelGGL(tile_class_k, dim3((unsigned)cdiv(c->T, 256)), dim3(256), 0, s,
                           (const TileDev*)c->b_tiles.p, c->T, cls);
    for (int k = 0; k < kRayClasses; ++k)
        if ((e = partition(cls, c->T, (uint8_t)k, pos, c->b_misc.p, sbytes, c->b_ray_list[k], &c->ray_cnt[k], s)) !=
            hipSuccess)
            return e;
    {
        DevBuf tmp;
        int64_t too_long = 0;
        e = partition(cls, c->T, (uint8_t)kRayClasses, pos, c->b_misc.p, sbytes, tmp, &too_long, s);
        hipFree(tmp.p);
        if (e != hipSuccess) return e;
        if (too_long > 0) {
            set_error("a ray crosses more than 2048 voxels");
            return hipErrorInvalidConfiguration;
        }
    }
    // voxels, by brick-major key
    if (c->Vk > 0)
        hipLaunchKernelGGL(vox_class_k, dim3((unsigned)cdiv(c->Vk, 256)), dim3(256), 0, s,
                           (const int64_t*)c->b_vptr.p, c->Vk, cls);
    for (int k = 0; k < kVoxClasses; ++k) {
        if ((e = partition(cls, c->Vk, (uint8_t)k, pos, c->b_misc.p, sbytes, c->b_vox_list[k], &c->vox_cnt[k], s)) !=
            hipSuccess)
            return e;
        const int64_t n = c->vox_cnt[k];
        if ((e = ensure(c->b_vox_desc[k], (size_t)(n > 0 ? n : 1) * sizeof(VoxDev))) != hipSuccess) return e;
        if (n > 0)
            hipLaunchKernelGGL(vox_desc_k, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s,
                               (const SceneDev*)c->b_scenes.p, c->n_scenes, (const uint32_t*)c->b_vox_list[k].p, n,
                               (const int64_t*)c->b_vptr.p, (VoxDev*)c->b_vox_desc[k].p);
    }
    {
        DevBuf tmp;
        int64_t too_big = 0;
        e = partition(cls, c->Vk, (uint8_t)kVoxClasses, pos, c->b_misc.p, sbytes, tmp, &too_big, s);
        hipFree(tmp.p);
        if (e != hipSuccess) return e;
        if (too_big > 0) {
            set_error("a voxel is crossed by more than 2^31 - 1 rays");
            return hipErrorInvalidConfiguration;
        }
    }

    // per-frame offsets of every ray class list (plain schedule)
    {
        const int nf = c->n_frames;
        std::vector<int64_t> fbase(nf + 1);
        for (int f = 0; f < nf; ++f) fbase[f] = c->frames_h[f].tile_base;
        fbase[nf] = c->T;
        std::vector<const uint32_t*> lists(kRayClasses);
        for (int k = 0; k < kRayClasses; ++k) lists[k] = (const uint32_t*)c->b_ray_list[k].p;
        // fbase (nf+1) | counts (classes) | offsets ((nf+1) * classes) | list pointers (classes)
        const size_t need = sizeof(int64_t) * ((size_t)(nf + 1) * (kRayClasses + 1) + kRayClasses) +
                            sizeof(void*) * kRayClasses;
        if ((e = ensure(c->b_frame_list, need)) != hipSuccess) return e;
        char* base = (char*)c->b_frame_list.p;
        int64_t* d_fbase = (int64_t*)base;
        int64_t* d_cnt = d_fbase + (nf + 1);
        int64_t* d_out = d_cnt + kRayClasses;
        const uint32_t** d_lists = (const uint32_t**)(d_out + (size_t)(nf + 1) * kRayClasses);
        hipMemcpyAsync(d_fbase, fbase.data(), sizeof(int64_t) * (nf + 1), hipMemcpyHostToDevice, s);
        hipMemcpyAsync(d_cnt, c->ray_cnt, sizeof(int64_t) * kRayClasses, hipMemcpyHostToDevice, s);
        hipMemcpyAsync(d_lists, lists.data(), sizeof(void*) * kRayClasses, hipMemcpyHostToDevice, s);
        hipLaunchKernelGGL(frame_offsets_k, dim3((unsigned)cdiv(nf + 1, 64), kRayClasses), dim3(64), 0, s,
                           d_lists, (const int64_t*)d_cnt, (const int64_t*)d_fbase, nf, d_out);
        c->frame_ray_off.assign((size_t)(nf + 1) * kRayClasses, 0);
        if ((e = hipMemcpyAsync(c->frame_ray_off.data(), d_out, sizeof(int64_t) * (nf + 1) * kRayClasses,
                                hipMemcpyDeviceToHost, s)) != hipSuccess)
            return e;
        // the host arrays above are read by the copies: finish before they go away
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    }
    // edges per work class (for the profiler's byte counts)
    {
        if ((e = ensure(c->b_sigpart, 64 * sizeof(double) * 4096)) != hipSuccess) return e;
        unsigned long long* d = (unsigned long long*)c->b_sigpart.p + 64;
        const int nc = 2 * kRayClasses + kVoxClasses;
        hipMemsetAsync(d, 0, nc * sizeof(unsigned long long), s);
        for (int k = 0; k < kRayClasses; ++k)
            if (c->ray_cnt[k] > 0)
                hipLaunchKernelGGL(tile_class_edges_k, dim3((unsigned)cdiv(c->ray_cnt[k], 256)), dim3(256), 0, s,
                                   (const uint32_t*)c->b_ray_list[k].p, c->ray_cnt[k], (const TileDev*)c->b_tiles.p,
                                   (const int32_t*)c->b_counts.p, d + k, d + kRayClasses + kVoxClasses + k);
        for (int k = 0; k < kVoxClasses; ++k) {
            const int64_t n = c->vox_cnt[k];
            if (n > 0)
                hipLaunchKernelGGL(class_edges_k, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s,
                                   (const uint32_t*)c->b_vox_list[k].p, n, (const int64_t*)c->b_vptr.p,
                                   d + kRayClasses + k);
        }
        unsigned long long hh[2 * kRayClasses + kVoxClasses];
        if ((e = hipMemcpyAsync(hh, d, sizeof(hh), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        for (int k = 0; k < kRayClasses; ++k) c->ray_cls_edges[k] = (int64_t)hh[k];
        for (int k = 0; k < kVoxClasses; ++k) c->vox_cls_edges[k] = (int64_t)hh[kRayClasses + k];
        for (int k = 0; k < kRayClasses; ++k) c->ray_cls_rays[k] = (int64_t)hh[kRayClasses + kVoxClasses + k];
    }
    // histograms
    {
        unsigned long long* d_h = (unsigned long long*)c->b_sigpart.p;
        if ((e = ensure(c->b_sigpart, 64 * sizeof(double) * 4096)) != hipSuccess) return e;
        d_h = (unsigned long long*)c->b_sigpart.p;
        hipMemsetAsync(d_h, 0, 42 * sizeof(unsigned long long), s);
        const int64_t nmx = c->R > c->Vk ? c->R : c->Vk;
        if (nmx > 0)
            hipLaunchKernelGGL(hist_k, dim3((unsigned)cdiv(nmx, 256)), dim3(256), 0, s,
                               (const int32_t*)c->b_counts.p, c->R, (const int64_t*)c->b_vptr.p, c->Vk, d_h);
        unsigned long long hh[42];
        if ((e = hipMemcpyAsync(hh, d_h, sizeof(hh), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        for (int i = 0; i < 16; ++i) c->stats.ray_len_hist[i] = (int64_t)hh[i];
        for (int i = 0; i < 24; ++i) c->stats.voxel_degree_hist[i] = (int64_t)hh[16 + i];
        c->stats.max_ray_len = (int64_t)hh[40];
        c->stats.max_voxel_degree = (int64_t)hh[41];
    }
    return hipGetLastError();
}

// ============================================================== adding keyframes
//
// Frames appended to the last scene add tiles and slots after every existing
// one, so within a voxel's edge list (slots ascending) the existing entries come
// first: with the new slots sorted by voxel key on their own, the merged list of
// key k is the old list of k followed by the new one, at merged offset
// old_vptr[k] + new_vptr[k].

// brick-major key of the voxel of list entry j (col of its slot)
__global__ void entry_keys_k(const SceneDev* __restrict__ scenes, int ns, const uint32_t* __restrict__ vedge,
                             const int32_t* __restrict__ col, int64_t n, uint32_t* __restrict__ keys,
                             const SlotGroups sg)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        keys[j] = voxel_to_key(scenes, ns, col[group_slot_base(sg, j) + vedge[j]]);
}

// old entry j of key k moves to j + new_vptr[k]; new entry i (slot s_new0 + vals[i],
// key keys_new[i] < Vk) to old_vptr[keys_new[i] + 1] + i
__global__ void merge_old_k(const uint32_t* __restrict__ vedge_old, const uint32_t* __restrict__ keys_old, int64_t n,
                            const int64_t* __restrict__ new_vptr, uint32_t* __restrict__ out)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        out[j + new_vptr[keys_old[j]]] = vedge_old[j];
}

__global__ void merge_new_k(const uint32_t* __restrict__ vals, const uint32_t* __restrict__ keys_new, int64_t n,
                            uint32_t s_new0, const int64_t* __restrict__ old_vptr, uint32_t* __restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[old_vptr[keys_new[i] + 1] + i] = s_new0 + vals[i];
}

// vptr_old[k] += new_vptr[k] over every key (k <= Vk)
__global__ void add_vptr_k(int64_t* __restrict__ vptr, const int64_t* __restrict__ add, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        vptr[k] += add[k];
}

__global__ void add_i64_k(int64_t* __restrict__ p, int64_t v, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] += v;
}

static unsigned grid_of(int64_t n)
{
    int64_t b = cdiv(n, 256);
    if (b > 65536) b = 65536;
    return (unsigned)(b > 0 ? b : 1);
}

hipError_t launch_add_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(add_i64_k, dim3(grid_of(n)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_entry_keys(const mrf_ctx* c, const uint32_t* vedge, int64_t n, uint32_t* keys, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(entry_keys_k, dim3(grid_of(n)), dim3(256), 0, s, (const SceneDev*)c->b_scenes.p, c->n_scenes,
                       vedge, (const int32_t*)c->b_col.p, n, keys, c->sg);
    return hipGetLastError();
}

hipError_t launch_merge_incidence(const uint32_t* vedge_old, const uint32_t* keys_old, int64_t n_old,
                                  const uint32_t* vals_new, const uint32_t* keys_new, int64_t n_new,
                                  uint32_t s_new0, int64_t* vptr, int64_t* new_vptr, int64_t nkeys, uint32_t* out,
                                  hipStream_t s)
{
    if (n_old > 0)
        hipLaunchKernelGGL(merge_old_k, dim3(grid_of(n_old)), dim3(256), 0, s, vedge_old, keys_old, n_old,
                           (const int64_t*)new_vptr, out);
    if (n_new > 0)
        hipLaunchKernelGGL(merge_new_k, dim3(grid_of(n_new)), dim3(256), 0, s, vals_new, keys_new, n_new, s_new0,
                           (const int64_t*)vptr, out);
    hipLaunchKernelGGL(add_vptr_k, dim3(grid_of(nkeys)), dim3(256), 0, s, vptr, (const int64_t*)new_vptr, nkeys);
    return hipGetLastError();
}

// ============================================================== keyframe pairs
//
// Per-keyframe averaged messages (Sec. IV-A): the rays of one keyframe that
// cross a voxel send it one message, the average of theirs weighted by the
// length each travels in the voxel.  A voxel's edge list (slots ascending) is
// grouped by keyframe, since slots are frame-major; each run of one keyframe
// inside one voxel's list is a (keyframe, voxel) pair.

// first slot of every frame (frames occupy consecutive slot ranges in order);
// fs[nf] = S
__global__ void frame_slots_k(const FrameDev* __restrict__ frames, int nf, const int64_t* __restrict__ tbase,
                              int64_t T, int64_t* __restrict__ fs)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < nf) fs[f] = tbase[frames[f].tile_base];
    if (f == nf) fs[nf] = tbase[T];
}

// frame holding slot x: the last f with fs[f] <= x (frames without edges
// share their successor's first slot and are skipped)
__device__ __forceinline__ int slot_frame(const int64_t* __restrict__ fs, int nf, uint32_t x)
{
    int lo = 0, hi = nf;   // fs[lo] <= x < fs[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (fs[mid] <= (int64_t)x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// the frame (keyframe) of every entry of the voxel -> ray list
__global__ void entry_frame_k(const uint32_t* __restrict__ vedge, int64_t n, const int64_t* __restrict__ fs, int nf,
                              uint16_t* __restrict__ fr)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        fr[j] = (uint16_t)slot_frame(fs, nf, vedge[j]);
}

// 1 where entry j of the voxel -> ray list starts a (keyframe, voxel) run
struct LoadPairStart {
    const uint16_t* fr;     // frame of each entry
    const uint32_t* keys;   // sorted voxel keys, aligned with the list
    __device__ int64_t operator()(int64_t j) const
    {
        if (j == 0) return 1;
        if (keys[j] != keys[j - 1]) return 1;
        return fr[j] != fr[j - 1] ? 1 : 0;
    }
};

// pair p (starting at entry j): its first entry and the index of its message
// in the per-keyframe buffers, xb[f] + linear voxel id
__global__ void pair_init_k(const LoadPairStart ld, int64_t E, const uint32_t* __restrict__ pos,
                            const SceneDev* __restrict__ scenes, int ns, const int64_t* __restrict__ xb,
                            uint32_t* __restrict__ pstart, uint32_t* __restrict__ px)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > E) return;
    if (j == E) {
        pstart[pos[E]] = (uint32_t)E;
        return;
    }
    if (!ld(j)) return;
    const uint32_t p = pos[j];
    pstart[p] = (uint32_t)j;
    const int f = ld.fr[j];
    px[p] = (uint32_t)(xb[f] + (int64_t)key_to_voxel(scenes, ns, ld.keys[j]));
}

// edge-count class of every pair (as the voxel classes)
__global__ void pair_class_k(const uint32_t* __restrict__ pstart, int64_t P, uint8_t* __restrict__ cls)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t m = (int64_t)pstart[p + 1] - pstart[p];
    uint8_t c = kVoxClasses - 1;
    for (int k = 0; k < kVoxClasses - 1; ++k)
        if (m <= kVoxCap[k]) {
            c = (uint8_t)k;
            break;
        }
    cls[p] = c;
}

__global__ void pair_desc_k(const uint32_t* __restrict__ list, int64_t n, const uint32_t* __restrict__ pstart,
                            VoxDev* __restrict__ desc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = list[i];
    desc[i] = VoxDev{(int64_t)pstart[p], (int32_t)(pstart[p + 1] - pstart[p]), p};
}

// the pairs of every touched voxel of one class list: [pos[vptr[key]], pos[vptr[key + 1]])
__global__ void kf_vox_k(const SceneDev* __restrict__ scenes, int ns, const uint32_t* __restrict__ keys, int64_t n,
                         const int64_t* __restrict__ vptr, const uint32_t* __restrict__ pos,
                         VoxDev* __restrict__ desc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t key = keys[i];
    const uint32_t p0 = pos[vptr[key]], p1 = pos[vptr[key + 1]];
    desc[i] = VoxDev{(int64_t)p0, (int32_t)(p1 - p0), key_to_voxel(scenes, ns, key)};
}

// weight of entry j = chord length / its pair's summed chord length (equal
// weights should every chord of the pair have rounded to zero length)
__global__ void pair_weight_k(const uint32_t* __restrict__ vedge, const uint32_t* __restrict__ pos, int64_t E,
                              const uint32_t* __restrict__ pstart, const float* __restrict__ wlen,
                              const double* __restrict__ wsum, float* __restrict__ w)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < E; j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = pos[j + 1] - 1;   // inclusive count of pair starts, less one
        const double sw = wsum[p];
        w[j] = sw > 0.0 ? (float)((double)wlen[vedge[j]] / sw) : (float)(1.0 / (double)(pstart[p + 1] - pstart[p]));
    }
}

hipError_t build_keyframe_pairs(mrf_ctx* c, hipStream_t s)
{
    hipError_t e;
    const int64_t E = c->E;
    const int nf = c->n_frames;
    // per-keyframe message buffers: frame f's entries follow the frames before it
    std::vector<int64_t> xb(nf);
    int64_t nx = 0;
    for (int f = 0; f < nf; ++f) {
        const SceneDev& sd = c->scenes_h[c->frames_h[f].scene];
        xb[f] = nx - sd.voxel_base;
        nx += (int64_t)sd.n[0] * sd.n[1] * sd.n[2];
    }
    if (nx >= (int64_t(1) << 32)) {
        set_error("per-keyframe message buffers of 2^32 or more entries");
        return hipErrorInvalidConfiguration;
    }
    c->n_kfx = nx;
    if ((e = ensure(c->b_kfxb, sizeof(int64_t) * (size_t)(nf + 1) * 2)) != hipSuccess) return e;
    int64_t* d_xb = (int64_t*)c->b_kfxb.p;
    int64_t* d_fs = d_xb + nf + 1;
    if ((e = hipMemcpyAsync(d_xb, xb.data(), sizeof(int64_t) * nf, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(frame_slots_k, dim3((unsigned)cdiv(nf + 1, 64)), dim3(64), 0, s,
                       (const FrameDev*)c->b_frames.p, nf, (const int64_t*)c->b_tbase.p, c->T, d_fs);
    if ((e = ensure(c->b_kfx, sizeof(float) * (size_t)(nx > 0 ? nx : 1))) != hipSuccess) return e;

    // pair starts: exclusive count over the voxel -> ray list (b_lam, E + 1 entries),
    // keys sorted in b_lambar from the radix sort, each entry's frame in b_gsum
    const uint32_t* vedge = (const uint32_t*)c->b_vedge.p;
    uint16_t* fr = (uint16_t*)c->b_gsum.p;   // 2 E bytes of a per-slot array free during the build
    if (E > 0) {
        int64_t b = cdiv(E, 256);
        if (b > 65536) b = 65536;
        hipLaunchKernelGGL(entry_frame_k, dim3((unsigned)b), dim3(256), 0, s, vedge, E, (const int64_t*)d_fs, nf, fr);
    }
    const LoadPairStart ld{fr, (const uint32_t*)c->b_lambar.p};
    uint32_t* pos = (uint32_t*)c->b_lam.p;
    const size_t sb = scan_tmp_bytes(E);
    if ((e = ensure(c->b_misc, sb > c->b_misc.cap ? sb : c->b_misc.cap)) != hipSuccess) return e;
    if ((e = scan_rec(ld, E, pos, (int64_t*)c->b_misc.p, s)) != hipSuccess) return e;
    uint32_t P32 = 0;
    if ((e = hipMemcpyAsync(&P32, pos + E, sizeof(uint32_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const int64_t P = P32;
    c->n_pairs = P;
    uint32_t* pstart = (uint32_t*)c->b_ell.p;   // P + 1 <= E + 1 entries
    if ((e = ensure(c->b_pair_x, sizeof(uint32_t) * (size_t)(P > 0 ? P : 1))) != hipSuccess) return e;
    if ((e = ensure(c->b_pair_m, sizeof(double) * (size_t)(P > 0 ? P : 1))) != hipSuccess) return e;
    hipLaunchKernelGGL(pair_init_k, dim3((unsigned)cdiv(E + 1, 256)), dim3(256), 0, s, ld, E, (const uint32_t*)pos,
                       (const SceneDev*)c->b_scenes.p, c->n_scenes, (const int64_t*)d_xb, pstart,
                       (uint32_t*)c->b_pair_x.p);

    // pairs by edge count, as VoxDev work items of the voxel-phase kernels
    if ((e = ensure(c->b_cls, (size_t)(P + 1))) != hipSuccess) return e;
    if ((e = ensure(c->b_tmp64, (size_t)(P + 2) * sizeof(int64_t))) != hipSuccess) return e;
    const size_t pb = scan_tmp_bytes(P + 1);
    if ((e = ensure(c->b_misc, pb > c->b_misc.cap ? pb : c->b_misc.cap)) != hipSuccess) return e;
    uint8_t* cls = (uint8_t*)c->b_cls.p;
    if (P > 0)
        hipLaunchKernelGGL(pair_class_k, dim3((unsigned)cdiv(P, 256)), dim3(256), 0, s, (const uint32_t*)pstart, P,
                           cls);
    DevBuf list;
    for (int k = 0; k < kVoxClasses; ++k) {
        e = partition(cls, P, (uint8_t)k, (int64_t*)c->b_tmp64.p, c->b_misc.p, c->b_misc.cap, list, &c->pair_cnt[k],
                      s);
        const int64_t n = c->pair_cnt[k];
        if (e == hipSuccess) e = ensure(c->b_pair_desc[k], (size_t)(n > 0 ? n : 1) * sizeof(VoxDev));
        if (e == hipSuccess && n > 0)
            hipLaunchKernelGGL(pair_desc_k, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, (const uint32_t*)list.p, n,
                               (const uint32_t*)pstart, (VoxDev*)c->b_pair_desc[k].p);
        if (e == hipSuccess) e = hipStreamSynchronize(s);   // list is rewritten by the next class
        if (e != hipSuccess) {
            hipFree(list.p);
            return e;
        }
    }
    hipFree(list.p);

    // touched voxels with their pair ranges, class by class
    int64_t nv = 0;
    for (int k = 0; k < kVoxClasses; ++k) nv += c->vox_cnt[k];
    c->n_kf_vox = nv;
    if ((e = ensure(c->b_kf_vox, (size_t)(nv > 0 ? nv : 1) * sizeof(VoxDev))) != hipSuccess) return e;
    int64_t off = 0;
    for (int k = 0; k < kVoxClasses; ++k) {
        const int64_t n = c->vox_cnt[k];
        if (n > 0)
            hipLaunchKernelGGL(kf_vox_k, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, (const SceneDev*)c->b_scenes.p,
                               c->n_scenes, (const uint32_t*)c->b_vox_list[k].p, n, (const int64_t*)c->b_vptr.p,
                               (const uint32_t*)pos, (VoxDev*)c->b_kf_vox.p + off);
        off += n;
    }

    // weights: chord length over the pair's summed chord length, in list order;
    // the chord lengths (slot order, b_kflen) are summed per pair by the pair phase
    double* wsum = (double*)c->b_pair_m.p;
    if ((e = ensure(c->b_kfw, sizeof(float) * (size_t)(E > 0 ? E : 1))) != hipSuccess) return e;
    float* w = (float*)c->b_kfw.p;
    if ((e = launch_pair_phase(c, (const float*)c->b_kflen.p, nullptr, wsum, s)) != hipSuccess) return e;
    if (E > 0) {
        int64_t b = cdiv(E, 256);
        if (b > 65536) b = 65536;
        hipLaunchKernelGGL(pair_weight_k, dim3((unsigned)b), dim3(256), 0, s, vedge, (const uint32_t*)pos, E,
                           (const uint32_t*)pstart, (const float*)c->b_kflen.p, (const double*)wsum, w);
    }
    return hipGetLastError();
}

}  // namespace mrf

namespace mrf {

hipError_t export_canonical_incidence(const mrf_ctx* c, int64_t* vptr, uint32_t* vedge, hipStream_t s)
{
    hipError_t e;
    mrf_ctx* m = const_cast<mrf_ctx*>(c);
    const SceneDev* sc = (const SceneDev*)c->b_scenes.p;
    if (vptr) {
        // canonical vptr: exclusive scan of the degree of every linear voxel id
        if ((e = ensure(m->b_tmp64, sizeof(int32_t) * (size_t)(c->V + 1))) != hipSuccess) return e;
        const size_t sb = scan_tmp_bytes(c->V + 1);
        if ((e = ensure(m->b_misc, sb)) != hipSuccess) return e;
        int32_t* deg = (int32_t*)c->b_tmp64.p;
        if (c->V > 0)
            hipLaunchKernelGGL(canon_degree_k, dim3((unsigned)cdiv(c->V, 256)), dim3(256), 0, s, sc, c->n_scenes,
                               (const int64_t*)c->b_vptr.p, c->V, deg);
        if ((e = scan_rec(LoadI32{deg}, c->V, vptr, (int64_t*)m->b_misc.p, s)) != hipSuccess) return e;
    }
    if (vedge && c->E > 0) {
        // canonical vedge: stable radix sort of canonical edge ids by linear voxel id
        // (O(E) temporaries: this export is a checking facility)
        const size_t E = (size_t)c->E;
        const size_t Ep = (E + 63) & ~(size_t)63;   // 256-byte aligned sub-arrays (vector loads)
        if ((e = ensure(m->b_export, 5 * Ep * sizeof(uint32_t))) != hipSuccess) return e;
        uint32_t* keys = (uint32_t*)c->b_export.p;
        uint32_t *ka = keys + Ep, *va = keys + 2 * Ep, *kb = keys + 3 * Ep, *vb = keys + 4 * Ep;
        if ((e = export_canonical_edges(c, c->b_col.p, keys, 4, s)) != hipSuccess) return e;
        const int64_t nh = (int64_t)radix_hist_entries(c->E);
        if ((e = ensure(m->b_tmp64, sizeof(int64_t) * (size_t)(nh + 1) + sizeof(int32_t) * (size_t)nh)) != hipSuccess)
            return e;
        int64_t* offs = (int64_t*)c->b_tmp64.p;
        int32_t* hist = (int32_t*)(offs + nh + 1);
        const size_t sb2 = radix_tmp_bytes(c->E);
        if ((e = ensure(m->b_misc, sb2 > m->b_misc.cap ? sb2 : m->b_misc.cap)) != hipSuccess) return e;
        int bits = 1;
        while (bits < 31 && (int64_t(1) << bits) <= c->V - 1) ++bits;
        const int passes = bits <= 8 ? 1 : (bits + 7) / 8;
        uint32_t* kout = passes == 1 ? kb : keys;   // the first pass is the only reader of `keys`
        if ((e = radix_sort_pairs(keys, ka, va, kb, vb, kout, vedge, c->E, bits, hist, offs, m->b_misc.p,
                                  m->b_misc.cap, s)) != hipSuccess)
            return e;
    }
    return hipGetLastError();
}

hipError_t export_canonical_edges(const mrf_ctx* c, const void* in_slots, void* out, int elem_bytes, hipStream_t s)
{
    if (c->R <= 0 || c->E <= 0) return hipSuccess;
    const dim3 g((unsigned)cdiv(c->R, 256)), b(256);
    const FrameDev* fr = (const FrameDev*)c->b_frames.p;
    const SceneDev* sc = (const SceneDev*)c->b_scenes.p;
    const int64_t* tb = (const int64_t*)c->b_tbase.p;
    const int64_t* rp = (const int64_t*)c->b_rowptr.p;
    switch (elem_bytes) {
        case 1:
            hipLaunchKernelGGL(canon_edges_k<uint8_t>, g, b, 0, s, fr, c->n_frames, sc, tb, rp, c->R,
                               (const uint8_t*)in_slots, (uint8_t*)out);
            break;
        case 4:
            hipLaunchKernelGGL(canon_edges_k<uint32_t>, g, b, 0, s, fr, c->n_frames, sc, tb, rp, c->R,
                               (const uint32_t*)in_slots, (uint32_t*)out);
            break;
        case 8:
            hipLaunchKernelGGL(canon_edges_k<uint64_t>, g, b, 0, s, fr, c->n_frames, sc, tb, rp, c->R,
                               (const uint64_t*)in_slots, (uint64_t*)out);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


// ============================================================== per-frame counts

__global__ void frame_counts_k(const FrameDev* __restrict__ frames, const SceneDev* __restrict__ scenes, int nf,
                               const int64_t* __restrict__ tbase, const int64_t* __restrict__ rowptr,
                               int64_t* __restrict__ out)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const FrameDev fr = frames[f];
    const SceneDev& sd = scenes[fr.scene];
    const int64_t nt = (int64_t)fr.ntx * ((sd.H + kTileW - 1) / kTileW);
    const int64_t hw = (int64_t)sd.W * sd.H;
    out[2 * f] = tbase[fr.tile_base + nt] - tbase[fr.tile_base];
    out[2 * f + 1] = rowptr[fr.ray_base + hw] - rowptr[fr.ray_base];
}

hipError_t launch_frame_counts(const mrf_ctx* c, int64_t* out, hipStream_t s)
{
    if (c->n_frames <= 0) return hipSuccess;
    hipLaunchKernelGGL(frame_counts_k, dim3((unsigned)cdiv(c->n_frames, 256)), dim3(256), 0, s,
                       (const FrameDev*)c->b_frames.p, (const SceneDev*)c->b_scenes.p, c->n_frames,
                       (const int64_t*)c->b_tbase.p, (const int64_t*)c->b_rowptr.p, out);
    return hipGetLastError();
}

// ============================================================== accuracy metric

// Sec. III-D: a voxel is a region of constant occlusion density alpha, chosen
// so that crossing one voxel side h blocks a ray with the voxel's occupancy
// probability: alpha = -ln(1 - p) / h = softplus(L) / h for log-odds L.  Per
// voxel of one scene, FP64: alpha and log alpha.
__global__ void metric_alpha_k(const float* __restrict__ logit, int64_t n, double inv_h,
                               double* __restrict__ alpha, double* __restrict__ lalpha)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = (double)logit[i];
        const double sp = (x > 0.0 ? x : 0.0) + log1p(exp(-fabs(x)));
        const double a = sp * inv_h;
        alpha[i] = a;
        lalpha[i] = log(a);
    }
}

// Along a ray (Euclidean length s) vis(s) = exp(-integral of alpha) and the
// density of the generating surface omega(s) = alpha(s) vis(s) decays inside
// a voxel, so its maximum is at the entry of the voxel maximising
// log alpha_n - sum_{i<n} alpha_i l_i (the first on ties).
struct MetricEmit {
    const double* alpha;
    const double* lalpha;
    int64_t vb;              // the scene's first global voxel id
    int32_t nx, ny;
    double wn;               // |w|: Euclidean length per unit of z-depth
    double acc = 0.0;        // sum of alpha_i l_i so far
    double best = -__builtin_huge_val();
    double btin = 0.0, btout = 0.0;

    __device__ void operator()(int, int i, int j, int kz, double tin, double tout)
    {
        const int64_t v = vb + (int64_t)(i + nx * (j + ny * kz));
        const double a = alpha[v];
        const double lw = lalpha[v] - acc;
        if (lw > best) {
            best = lw;
            btin = tin;
            btout = tout;
        }
        acc += a * ((tout - tin) * wn);
    }
};

// One thread per pixel of one frame (blockIdx.y): the ray clipped to the grid
// box and walked to the grid exit.  Exit visibility of at least vis_min (log:
// lvmin) means the map leaves the ray visible, and the ray is accurate iff its
// measurement lies beyond the exit; otherwise iff the measurement lies inside
// the chord [t_in, t_out) of the voxel of the most likely surface, or, with
// tol > 0 (the paper's evaluation rule), iff that surface (the voxel's entry)
// lies within tol sigma(Z) of Z, sigma(Z) = max(c0 + c2 Z^2, smin).  The
// measurement is the built frame's, or ref[global ray] when ref is given
// (e.g. noise-free depth from the same poses).  code: 1
// accurate, 0 not, -1 not evaluated; surf: z-depth of the chosen voxel's
// entry, +inf when the surface is taken to lie beyond the map, NaN when not
// evaluated.  Per-scene counts (evaluated, accurate) by block counts and one
// atomic per block.
__global__ __launch_bounds__(256) void accuracy_k(const SceneDev* __restrict__ scenes,
                                                  const FrameDev* __restrict__ frames, BuildDev bp,
                                                  const double* __restrict__ alpha,
                                                  const double* __restrict__ lalpha, double lvmin,
                                                  const float* __restrict__ ref, double tol,
                                                  int8_t* __restrict__ code, double* __restrict__ surf,
                                                  unsigned long long* __restrict__ counts)
{
    const FrameDev fr = frames[blockIdx.y];
    const SceneDev& sd = scenes[fr.scene];
    const int pix = blockIdx.x * 256 + threadIdx.x;
    int ev = 0, ok = 0;
    if (pix < sd.W * sd.H) {
        const int v = pix / sd.W, u = pix - v * sd.W;
        Ray r;
        double ts, texit;
        int8_t cd = -1;
        double sf = __builtin_nan("");
        const float zm = ref ? ref[fr.ray_base + pix] : fr.depth[pix];
        if (clip_ray(sd, bp, fr.T, zm, v, u, r, ts, texit) && ts < texit) {
            r.ts = ts;
            r.te = texit;
            MetricEmit m;
            m.alpha = alpha;
            m.lalpha = lalpha;
            m.vb = sd.voxel_base;
            m.nx = sd.n[0];
            m.ny = sd.n[1];
            m.wn = sqrt(r.w[0] * r.w[0] + r.w[1] * r.w[1] + r.w[2] * r.w[2]);
            walk(sd, r, nullptr, m);   // the metric walks the whole grid
            if (-m.acc >= lvmin) {
                cd = r.Z > texit ? 1 : 0;
                sf = __builtin_huge_val();
            } else if (tol > 0.0) {
                double sig = bp.c2 * r.Z;
                sig = sig * r.Z;
                sig = bp.c0 + sig;
                if (sig < bp.smin) sig = bp.smin;
                cd = fabs(m.btin - r.Z) <= tol * sig ? 1 : 0;
                sf = m.btin;
            } else {
                cd = (m.btin <= r.Z && r.Z < m.btout) ? 1 : 0;
                sf = m.btin;
            }
            ev = 1;
            ok = cd;
        }
        const int64_t gr = fr.ray_base + pix;
        if (code) code[gr] = cd;
        if (surf) surf[gr] = sf;
    }
    const int nev = __syncthreads_count(ev);
    const int nok = __syncthreads_count(ok);
    if (counts && threadIdx.x == 0 && nev > 0) {
        atomicAdd(&counts[2 * fr.scene], (unsigned long long)nev);
        atomicAdd(&counts[2 * fr.scene + 1], (unsigned long long)nok);
    }
}

hipError_t launch_accuracy(mrf_ctx* c, const float* logit, double vis_min, const float* ref, double tol,
                           int8_t* code, double* surf, int64_t* counts, double* work, hipStream_t s)
{
    double* alpha = work;
    double* lalpha = alpha + c->V;
    for (const SceneDev& sd : c->scenes_h) {
        const int64_t n = (int64_t)sd.n[0] * sd.n[1] * sd.n[2];
        int64_t b = (n + 255) / 256;
        if (b > 65536) b = 65536;
        hipLaunchKernelGGL(metric_alpha_k, dim3((unsigned)b), dim3(256), 0, s, logit + sd.voxel_base, n, 1.0 / sd.h,
                           alpha + sd.voxel_base, lalpha + sd.voxel_base);
    }
    if (counts) {
        hipError_t e = launch_fill_u32((uint32_t*)counts, 0u, 4 * (int64_t)c->n_scenes, s);
        if (e != hipSuccess) return e;
    }
    dim3 grid((c->max_hw + 255) / 256, c->n_frames);
    hipLaunchKernelGGL(accuracy_k, grid, dim3(256), 0, s, (const SceneDev*)c->b_scenes.p,
                       (const FrameDev*)c->b_frames.p, c->bp, (const double*)alpha, (const double*)lalpha,
                       std::log(vis_min), ref, tol, code, surf, (unsigned long long*)counts);
    return hipGetLastError();
}

// ------------------------------------------------------------ static scratch
//
// The accuracy metric's per-voxel alpha and log alpha for callers that cannot
// allocate device memory (mrf_accuracy_static): a file-scope device array of
// kStaticMetricVoxels voxels (two doubles each, 32 MiB), one copy per GPU,
// held until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is a stand-in, not a device address): its device
// address is looked up once per device, with that device current, and kept.
static __device__ __align__(256) double scratch[2 * kStaticMetricVoxels];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {nullptr};
hipError_t g_scratch_err[kMaxDevices] = {hipSuccess};
bool g_scratch_done[kMaxDevices] = {false};
}  // namespace

hipError_t static_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));   // the current device's copy
        g_scratch_ptr[device] = e == hipSuccess ? (double*)ptr : nullptr;
        g_scratch_err[device] = e;
        g_scratch_done[device] = true;
        if (e != hipSuccess) hipGetLastError();
    }
    return g_scratch_err[device];
}

hipError_t static_scratch(int device, double** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[device]) return hipErrorNotInitialized;
    *out = g_scratch_ptr[device];
    return g_scratch_err[device];
}

}  // namespace mrf
