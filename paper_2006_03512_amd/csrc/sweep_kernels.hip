// Forward message passing on gfx950 (Sec. III-B/C, IV-A of MRFMap).
//
// Messages to binary occupancy variables are log-odds, so every message is
// normalised by construction (supplement, Sec. II-A).  Per edge e (one ray
// crossing one voxel):
//   lam_e  voxel -> ray factor  (Eq. node_to_factor: prior plus every other
//          ray's message into the voxel)
//   ell_e  ray factor -> voxel  (Eqs. pos and neg)
//   g_e    log nu(d_e) = log N(Z; d_e, sigma(d_e))   (Eq. noise)
//
// Voxel phase: per touched voxel the total tot_v = theta_v + sum of every
// incoming ray message, a fixed-order FP64 reduction over its edge list kept
// as the FP32 pair (hi, lo).  Eq. node_to_factor (every incoming message but
// the receiving ray's own) is then lam_e = (hi_v(e) - ell_e) + lo_v(e), which
// the ray kernels form as they stage their tiles: no per-edge scatter.  When
// the edge's own message is most of the total (a message of 1e9 against
// others summing to a few units), hi - ell_e is exact and lam_e keeps the
// accuracy of the FP64 sum.
// Ray phase: one group of lanes per ray.  With P_i = sum_{k<i} log mu_k(0),
//   S_i = LSE_{j<i} (log mu_j(1) + g_j + P_j)
//   Q_i = LSE(log mu_{i+1}(1) + g_{i+1}, log mu_{i+1}(0) + Q_{i+1})
//   ell_i = LSE(S_i, g_i + P_i) - LSE(S_i, P_i + Q_i)
// is Eq. pos over Eq. neg with the second sum of Eq. neg in its division-free
// form (sum over j > i of the product over k < j, k != i).  The kernels carry
// R_i = S_i - P_i instead of S and P (see ray_body).
#include <hip/hip_runtime.h>

#include <array>
#include <utility>

#include "dev_common.hpp"
#include "mrf_internal.hpp"
#include "tile_lds.hpp"

namespace mrf {

static inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// ------------------------------------------------------------ elementwise

__global__ void fill_k(float* __restrict__ p, float v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void copy_k(float* __restrict__ d, const float* __restrict__ s, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}

__global__ void pair_k(const float* __restrict__ in, float2* __restrict__ out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = make_float2(in[i], 0.0f);
}

__global__ void excl_k(const int32_t* __restrict__ col, ExclDev x, float* __restrict__ out, int64_t E)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x)
    {
        const int32_t v = col[i];
        out[i] = excl_value(v, x.tot[v < 0 ? 0 : v], x.own[i], x.has_own);
    }
}

__global__ void sigmoid_k(const float* __restrict__ L, float* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 1.0f / (1.0f + __expf(-L[i]));
}

// g_e = log N(Z; d_e + mu_b, sigma_b) = -((delta_e - mu_b) / sigma_b)^2 / 2 -
// log sigma_b - log(2 pi) / 2, delta_e = Z - d_e, mu_b the learnt depth bias
// (the predicted mean measurement at depth d is d + mu(d)).  A lane takes 4
// consecutive slots and consecutive lanes consecutive groups, so every load
// (4 bins, 4 deltas) and store (4 g) instruction of a wave covers one
// contiguous run; S is a multiple of 16, so a group lies wholly inside or
// outside [0, S).  Grid-stride, so each block builds its tables once.
// Padding slots (bin 255) are left as they are.
constexpr int kPotGroups = 4;   // potentials: groups of 4 slots in flight per lane

__global__ __launch_bounds__(256) void potentials_k(const float* __restrict__ delta, const uint8_t* __restrict__ bin,
                                                    int64_t S, const float* __restrict__ sigma,
                                                    const float* __restrict__ bias, float* __restrict__ g)
{
    __shared__ float inv[kBins], cst[kBins], mu[kBins];
    if (threadIdx.x < kBins) {
        const float s = sigma[threadIdx.x];
        inv[threadIdx.x] = 1.0f / s;
        cst[threadIdx.x] = logf(s) + 0.91893853320467274f;
        mu[threadIdx.x] = bias[threadIdx.x];
    }
    __syncthreads();
    const int64_t ng = S / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x * kPotGroups + threadIdx.x; g0 < ng;
         g0 += stride * kPotGroups) {
        uint32_t bw[kPotGroups];
        float4 dv[kPotGroups];
#pragma unroll
        for (int u = 0; u < kPotGroups; ++u) {
            const int64_t gi = g0 + (int64_t)u * blockDim.x;
            const int64_t at = gi < ng ? gi : ng - 1;
            bw[u] = ((const uint32_t*)bin)[at];
            dv[u] = ((const float4*)delta)[at];
        }
#pragma unroll
        for (int u = 0; u < kPotGroups; ++u) {
            const int64_t gi = g0 + (int64_t)u * blockDim.x;
            if (gi >= ng) break;
            float out[4];
            bool all = true;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int b = (int)((bw[u] >> (8 * j)) & 255u);
                const float dj = j == 0 ? dv[u].x : j == 1 ? dv[u].y : j == 2 ? dv[u].z : dv[u].w;
                const int bb = b < kBins ? b : 0;
                const float x = (dj - mu[bb]) * inv[bb];   // residual about the predicted mean d + mu
                out[j] = -0.5f * x * x - cst[bb];
                all = all && b < kBins;
            }
            if (all) {
                ((float4*)g)[gi] = make_float4(out[0], out[1], out[2], out[3]);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (((bw[u] >> (8 * j)) & 255u) < kBins) g[4 * gi + j] = out[j];
            }
        }
    }
}

// potentials_k with per-region tables: one block per tile (grid-stride), the
// region's row staged in LDS, the tile's 16 len slots in groups of 4 with the
// same arithmetic as potentials_k.
__global__ __launch_bounds__(256) void potentials_cells_k(const TileDev* __restrict__ tiles, int64_t T,
                                                          const FrameDev* __restrict__ frames, int cp,
                                                          const float* __restrict__ delta,
                                                          const uint8_t* __restrict__ bin,
                                                          const float* __restrict__ sigma,
                                                          const float* __restrict__ bias, float* __restrict__ g)
{
    __shared__ float inv[kBins], cst[kBins], mu[kBins];
    for (int64_t ti = blockIdx.x; ti < T; ti += gridDim.x) {
        const TileDev t = tiles[ti];
        const int64_t row = tile_cell(t, frames, cp) * kBins;
        __syncthreads();   // the previous tile's readers are done
        if (threadIdx.x < kBins) {
            const float s = sigma[row + threadIdx.x];
            inv[threadIdx.x] = 1.0f / s;
            cst[threadIdx.x] = logf(s) + 0.91893853320467274f;
            mu[threadIdx.x] = bias[row + threadIdx.x];
        }
        __syncthreads();
        const int64_t g0 = t.base / 4, ng = 4 * (int64_t)t.len;
        for (int64_t k = threadIdx.x; k < ng; k += blockDim.x) {
            const int64_t gi = g0 + k;
            const uint32_t bw = ((const uint32_t*)bin)[gi];
            const float4 dv = ((const float4*)delta)[gi];
            float out[4];
            bool all = true;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int b = (int)((bw >> (8 * j)) & 255u);
                const float dj = j == 0 ? dv.x : j == 1 ? dv.y : j == 2 ? dv.z : dv.w;
                const int bb = b < kBins ? b : 0;
                const float x = (dj - mu[bb]) * inv[bb];
                out[j] = -0.5f * x * x - cst[bb];
                all = all && b < kBins;
            }
            if (all) {
                ((float4*)g)[gi] = make_float4(out[0], out[1], out[2], out[3]);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (((bw >> (8 * j)) & 255u) < kBins) g[4 * gi + j] = out[j];
            }
        }
    }
}

static unsigned grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return (unsigned)(b > 0 ? b : 1);
}

hipError_t launch_fill(float* p, float v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_k, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_copy(float* d, const float* src, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_k, dim3(grid_for(n)), dim3(256), 0, s, d, src, n);
    return hipGetLastError();
}

hipError_t launch_pair(const float* in, float2* out, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(pair_k, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_excl(const mrf_ctx* c, ExclSrc x, float* out, hipStream_t s)
{
    if (c->S <= 0) return hipSuccess;
    hipLaunchKernelGGL(excl_k, dim3(grid_for(c->S)), dim3(256), 0, s, (const int32_t*)c->b_col.p, excl_dev(c, x),
                       out, c->S);
    return hipGetLastError();
}

hipError_t launch_sigmoid(const float* L, float* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(sigmoid_k, dim3(grid_for(n)), dim3(256), 0, s, L, p, n);
    return hipGetLastError();
}

hipError_t launch_potentials(mrf_ctx* c, hipStream_t s)
{
    if (c->S <= 0) return hipSuccess;
    ProfScope ps(c, KID_POT, s);
    if (c->cell_px > 0) {
        const int64_t blocks = c->T < 65536 ? c->T : 65536;
        hipLaunchKernelGGL(potentials_cells_k, dim3((unsigned)blocks), dim3(256), 0, s, (const TileDev*)c->b_tiles.p,
                           c->T, (const FrameDev*)c->b_frames.p, c->cell_px, (const float*)c->b_delta.p,
                           (const uint8_t*)c->b_bin.p, (const float*)c->b_sigma.p, (const float*)c->b_bias.p,
                           (float*)c->b_g.p);
        return hipGetLastError();
    }
    int64_t blocks = nblk(c->S / 4, 256 * kPotGroups);
    if (blocks > 4096) blocks = 4096;   // grid-stride over at most 16 blocks per CU
    hipLaunchKernelGGL(potentials_k, dim3((unsigned)blocks), dim3(256), 0, s, (const float*)c->b_delta.p,
                       (const uint8_t*)c->b_bin.p, c->S, (const float*)c->b_sigma.p,
                       (const float*)c->b_bias.p, (float*)c->b_g.p);
    return hipGetLastError();
}

// ------------------------------------------------------------ voxel phase
//
// The voxel phase reduces: for every touched voxel v, sum_v = the sum of its
// incoming per-edge values (ray messages forward, d/d lambda in reverse), in a
// fixed order and in FP64 (every FP32 term is exact there), written as VoxOut
// describes.  The voxel -> ray message of edge e is then formed from the total
// pair and the edge's own term by the ray kernels as they stage their tiles
// (no per-edge scatter here).

// FP64 sum over items base + 64 k + l (k < N, l the lane) of the edge list
// [s, s+m) of one voxel (0 past m).  Branchless, with item indices clamped to
// m - 1 (m >= 1), so that every load is issued before the first wait.
// An item's term: in[vedge[j]], times the list-order weight w[j] when the
// sum is weighted (per-keyframe averages); the product of two FP32 values is
// exact in FP64.
template <bool WT>
__device__ __forceinline__ double vox_term(float x, const float* __restrict__ w, int64_t j)
{
    if constexpr (WT)
        return (double)x * (double)w[j];
    else
        return (double)x;
}

template <int N, bool WT = false>
__device__ __forceinline__ double vox_lane_sum(int64_t s, int m, int base, const uint32_t* __restrict__ vedge,
                                               const float* __restrict__ in, const float* __restrict__ w = nullptr)
{
    const int l = threadIdx.x & 63;
    uint32_t e[N];
    float x[N], wt[N];
#pragma unroll
    for (int k = 0; k < N; ++k) e[k] = vedge[s + min(base + k * 64 + l, m - 1)];
    if constexpr (WT) {
#pragma unroll
        for (int k = 0; k < N; ++k) wt[k] = w[s + min(base + k * 64 + l, m - 1)];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] = in[e[k]];
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double t = WT ? (double)x[k] * (double)wt[k] : (double)x[k];
        a += base + k * 64 + l < m ? t : 0.0;
    }
    return a;
}

__device__ __forceinline__ void vox_store(uint32_t v, double sum, const VoxOut& o)
{
    const double t = (o.base ? (double)o.base[v] : 0.0) + sum;
    if (o.tot2) o.tot2[v] = split_pair(t);
    if (o.totf) o.totf[v] = (float)t;
    if (o.acc) o.acc[v] += (float)sum;
    if (o.dsum) o.dsum[v] = sum;
}

// One voxel's edge list [s, s+m) summed by NW waves, each owning 64*IPL
// consecutive edges (striped over its lanes); the wave sums meet in LDS and
// are added in wave order.  NW == 1: four waves per 256-thread block, each
// summing VPW consecutive voxels of the list with all their loads issued
// before the first wait (more bytes in flight per wave for low degrees).
// Voxels arrive in brick-major order and blocks are remapped so each XCD
// takes a contiguous range of them.
template <int NW, int IPL, int VPW, bool WT = false, bool MG = false>
__global__ __launch_bounds__(NW == 1 ? 256 : 64 * NW) void voxel_k(const VoxDev* __restrict__ vd, int64_t n,
                                                                   const uint32_t* __restrict__ vedge,
                                                                   const float* __restrict__ in, VoxOut out,
                                                                   const float* __restrict__ w,
                                                                   const SlotGroups sg)
{
    static_assert(NW == 1 || VPW == 1, "several voxels per wave only with one wave per voxel");
    // the wave index is uniform across the wave: said so, the voxel descriptors
    // below become scalar loads and their address and group arithmetic scalar
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    if constexpr (NW == 1) {
        const int64_t v0 = (lb * 4 + wv) * VPW;
        if (v0 >= n) return;   // whole wave
        VoxDev d[VPW];
#pragma unroll
        for (int u = 0; u < VPW; ++u) d[u] = vd[min(v0 + u, n - 1)];   // past the list: a repeat, not stored
        uint32_t e[VPW][IPL];
        float x[VPW][IPL], wt[VPW][IPL];
#pragma unroll
        for (int u = 0; u < VPW; ++u)
#pragma unroll
            for (int k = 0; k < IPL; ++k) e[u][k] = vedge[d[u].start + min(k * 64 + l, d[u].m - 1)];
        if constexpr (WT) {
#pragma unroll
            for (int u = 0; u < VPW; ++u)
#pragma unroll
                for (int k = 0; k < IPL; ++k) wt[u][k] = w[d[u].start + min(k * 64 + l, d[u].m - 1)];
        }
#pragma unroll
        for (int u = 0; u < VPW; ++u) {
            const float* ing = in + (MG ? group_slot_base(sg, d[u].start) : 0);
#pragma unroll
            for (int k = 0; k < IPL; ++k) x[u][k] = ing[e[u][k]];
        }
        double a[VPW];
#pragma unroll
        for (int u = 0; u < VPW; ++u) {
            a[u] = 0.0;
#pragma unroll
            for (int k = 0; k < IPL; ++k) {
                const double t = WT ? (double)x[u][k] * (double)wt[u][k] : (double)x[u][k];
                a[u] += k * 64 + l < d[u].m ? t : 0.0;
            }
        }
        if constexpr (VPW == 1) {
            const double t = dgroup_sum_d<64>(a[0]);
            if (l == 0) vox_store(d[0].v, t, out);
        } else {
            // the wave's VPW x 64 lane sums transposed through LDS: voxel u
            // goes to the LG = 64 / VPW lanes [u LG, (u + 1) LG), lane p of
            // them adding the sums of lanes [p VPW, (p + 1) VPW) in order, then
            // a group sum over the LG lanes (one reduction for all voxels)
            constexpr int LG = 64 / VPW;
            static_assert(LG == 8 || LG == 16, "four or eight voxels per wave");
            __shared__ double red[4][VPW][64];
#pragma unroll
            for (int u = 0; u < VPW; ++u) red[wv][u][l] = a[u];
            // LDS accesses of one wave complete in order: the fences only keep
            // the compiler from moving the reads above the writes
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int u = l / LG, p = l % LG;
            double t = 0.0;
#pragma unroll
            for (int j = 0; j < VPW; ++j) t += red[wv][u][p * VPW + j];
            t = dgroup_sum_d<LG>(t);   // at the group's first lane
            if (p == 0 && v0 + u < n) vox_store(vd[v0 + u].v, t, out);
        }
    } else {
        const int64_t vi = lb;
        if (vi >= n) return;   // whole block
        const VoxDev d = vd[vi];
        const double a = dgroup_sum_d<64>(
            vox_lane_sum<IPL, WT>(d.start, d.m, wv * 64 * IPL, vedge, in + (MG ? group_slot_base(sg, d.start) : 0), w));
        __shared__ double wsum[NW];
        if (l == 0) wsum[wv] = a;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot = 0.0;
            for (int q = 0; q < NW; ++q) tot += wsum[q];
            vox_store(d.v, tot, out);
        }
    }
}

// Voxels of at most G edges (G = 16 or 32): 64 / G lane groups per wave, 256
// / G per block, each group summing VPG consecutive voxels of the list (lane
// l holds edge l of each; group reductions), every load issued first.
template <int G, int VPG, bool WT = false, bool MG = false>
__global__ __launch_bounds__(256) void voxel_small_k(const VoxDev* __restrict__ vd, int64_t n,
                                                     const uint32_t* __restrict__ vedge, const float* __restrict__ in,
                                                     VoxOut out, const float* __restrict__ w, const SlotGroups sg)
{
    constexpr int GPB = 256 / G;   // groups per block
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    if (lb * GPB * VPG >= n) return;   // whole block
    const int64_t v0 = (lb * GPB + (int)threadIdx.x / G) * VPG;
    const int l = (int)threadIdx.x % G;
    VoxDev d[VPG];
#pragma unroll
    for (int u = 0; u < VPG; ++u) d[u] = vd[min(v0 + u, n - 1)];   // past the list: a repeat, not stored
    uint32_t e[VPG];
    float x[VPG], wt[VPG];
#pragma unroll
    for (int u = 0; u < VPG; ++u) e[u] = vedge[d[u].start + min(l, d[u].m - 1)];
    if constexpr (WT) {
#pragma unroll
        for (int u = 0; u < VPG; ++u) wt[u] = w[d[u].start + min(l, d[u].m - 1)];
    }
#pragma unroll
    for (int u = 0; u < VPG; ++u) x[u] = in[(MG ? group_slot_base(sg, d[u].start) : 0) + e[u]];
#pragma unroll
    for (int u = 0; u < VPG; ++u) {
        const double t = WT ? (double)x[u] * (double)wt[u] : (double)x[u];
        const double sum = dgroup_sum_d<G>(l < d[u].m ? t : 0.0);   // at group lane 0
        if (l == 0 && v0 + u < n) vox_store(d[u].v, sum, out);
    }
}

// One 1024-thread block per voxel of degree above the largest single-pass
// class: wave w sums pieces w, w + 16, ... of 1024 edges in order, and the 16
// wave sums are added in wave order.
template <bool WT = false, bool MG = false>
__global__ __launch_bounds__(1024) void voxel_chunked_k(const VoxDev* __restrict__ vd, int64_t n,
                                                        const uint32_t* __restrict__ vedge,
                                                        const float* __restrict__ in, VoxOut out,
                                                        const float* __restrict__ w, const SlotGroups sg)
{
    __shared__ double wsum[16];
    const int64_t b = xcd_block(blockIdx.x, gridDim.x);
    if (b >= n) return;
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    const VoxDev d = vd[b];
    const int nch = (d.m + kVoxChunk - 1) / kVoxChunk;
    const float* ing = in + (MG ? group_slot_base(sg, d.start) : 0);
    double a = 0.0;
    for (int c = wv; c < nch; c += 16)
        a += vox_lane_sum<kVoxChunk / 64, WT>(d.start, d.m, c * kVoxChunk, vedge, ing, w);
    a = dgroup_sum_d<64>(a);
    if (l == 0) wsum[wv] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int q = 0; q < 16; ++q) tot += wsum[q];
        vox_store(d.v, tot, out);
    }
}

// Class K of a segment list (voxels, or keyframe pairs with weights w) with n
// work items described by desc.  MG: several slot groups (each voxel's list
// entries are relative to its group's first slot); a single group, the common
// case, skips the group lookup.
template <int K, bool WT, bool MG>
static void launch_seg_class_t(const VoxDev* desc, int64_t n, const uint32_t* vedge, const SlotGroups& sg,
                               const float* in, VoxOut out, const float* w, hipStream_t s)
{
    constexpr int NW = kVoxNW[K];
    if constexpr (NW == 0) {
        constexpr int G = kVoxCap[K];
        constexpr int VPG = kVoxVPW[K];
        hipLaunchKernelGGL((voxel_small_k<G, VPG, WT, MG>), dim3(nblk(n, 256 / G * VPG)), dim3(256), 0, s, desc, n,
                           vedge, in, out, w, sg);
    } else {
        constexpr int IPL = kVoxCap[K] / (64 * NW);
        constexpr int VPW = kVoxVPW[K];
        const unsigned blocks = NW == 1 ? nblk(n, 4 * VPW) : (unsigned)n;
        hipLaunchKernelGGL((voxel_k<NW, IPL, VPW, WT, MG>), dim3(blocks), dim3(NW == 1 ? 256 : 64 * NW), 0, s, desc,
                           n, vedge, in, out, w, sg);
    }
}

template <int K, bool WT>
static void launch_seg_class(const VoxDev* desc, int64_t n, const uint32_t* vedge, const SlotGroups& sg,
                             const float* in, VoxOut out, const float* w, hipStream_t s)
{
    if (n <= 0) return;
    if (sg.n > 1)
        launch_seg_class_t<K, WT, true>(desc, n, vedge, sg, in, out, w, s);
    else
        launch_seg_class_t<K, WT, false>(desc, n, vedge, sg, in, out, w, s);
}

template <bool WT>
static void launch_seg_chunked(const VoxDev* desc, int64_t n, const uint32_t* vedge, const SlotGroups& sg,
                               const float* in, VoxOut out, const float* w, hipStream_t s)
{
    if (n <= 0) return;
    if (sg.n > 1)
        hipLaunchKernelGGL((voxel_chunked_k<WT, true>), dim3((unsigned)n), dim3(1024), 0, s, desc, n, vedge, in, out,
                           w, sg);
    else
        hipLaunchKernelGGL((voxel_chunked_k<WT, false>), dim3((unsigned)n), dim3(1024), 0, s, desc, n, vedge, in,
                           out, w, sg);
}

template <int K>
static void launch_voxel_class(mrf_ctx* c, const float* in, VoxOut out, hipStream_t s)
{
    if (c->vox_cnt[K] <= 0) return;
    ProfScope ps(c, KID_VOX0 + K, s);
    launch_seg_class<K, false>((const VoxDev*)c->b_vox_desc[K].p, c->vox_cnt[K], (const uint32_t*)c->b_vedge.p,
                               c->sg, in, out, nullptr, s);
}

template <int... K>
static void voxel_classes(std::integer_sequence<int, K...>, mrf_ctx* c, const float* in, VoxOut out, hipStream_t s)
{
    (launch_voxel_class<K>(c, in, out, s), ...);
}

hipError_t launch_voxel_phase(mrf_ctx* c, const float* in, VoxOut out, hipStream_t s)
{
    voxel_classes(std::make_integer_sequence<int, kVoxClasses - 1>{}, c, in, out, s);
    const int kc = kVoxClasses - 1;
    if (c->vox_cnt[kc] > 0) {
        ProfScope ps(c, KID_VOX0 + kc, s);
        launch_seg_chunked<false>((const VoxDev*)c->b_vox_desc[kc].p, c->vox_cnt[kc], (const uint32_t*)c->b_vedge.p,
                                  c->sg, in, out, nullptr, s);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ keyframe pairs
//
// Per-keyframe averaged messages (Sec. IV-A): keyframe f sends voxel v the
// average M_fv = sum_j w_j ell_j of its rays' messages, w_j the edge's chord
// length over the pair's summed chord length, and a ray of keyframe f
// receives theta_v plus the other keyframes' averages.  The pair phase forms
// every M (FP64, fixed order); the voxel step sums them per voxel and writes,
// per pair, x = fl(T - M_fv) into keyframe f's message buffer.

template <int... K>
static void pair_classes(std::integer_sequence<int, K...>, mrf_ctx* c, const float* in, VoxOut out,
                         const float* w, hipStream_t s)
{
    ((w ? launch_seg_class<K, true>((const VoxDev*)c->b_pair_desc[K].p, c->pair_cnt[K],
                                    (const uint32_t*)c->b_vedge.p, c->sg, in, out, w, s)
        : launch_seg_class<K, false>((const VoxDev*)c->b_pair_desc[K].p, c->pair_cnt[K],
                                     (const uint32_t*)c->b_vedge.p, c->sg, in, out, nullptr, s)),
     ...);
}

hipError_t launch_pair_phase(mrf_ctx* c, const float* in, const float* w, double* M, hipStream_t s)
{
    VoxOut out{nullptr, nullptr, nullptr, nullptr, M};
    ProfScope ps(c, KID_PAIR, s);
    pair_classes(std::make_integer_sequence<int, kVoxClasses - 1>{}, c, in, out, w, s);
    const int kc = kVoxClasses - 1;
    const VoxDev* d = (const VoxDev*)c->b_pair_desc[kc].p;
    if (w)
        launch_seg_chunked<true>(d, c->pair_cnt[kc], (const uint32_t*)c->b_vedge.p, c->sg, in, out, w, s);
    else
        launch_seg_chunked<false>(d, c->pair_cnt[kc], (const uint32_t*)c->b_vedge.p, c->sg, in, out, nullptr, s);
    return hipGetLastError();
}

// One 16-lane group per touched voxel: T = theta_v + the sum of the voxel's
// pair averages (FP64; lane-strided partial sums added in a fixed order), then
// every pair's message x = fl(T - M) into its keyframe's buffer, and L_v = fl(T).
// M null: every average is 0 (x = theta).
__global__ __launch_bounds__(256) void kf_voxel_k(const VoxDev* __restrict__ vd, int64_t n,
                                                  const double* __restrict__ M, const uint32_t* __restrict__ px,
                                                  const float* __restrict__ theta, float* __restrict__ x,
                                                  float* __restrict__ L)
{
    const int64_t vi = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 16 + (int)(threadIdx.x >> 4);
    if (vi >= n) return;   // whole group
    const int l = (int)(threadIdx.x & 15);
    const VoxDev d = vd[vi];
    double a = 0.0;
    if (M)
        for (int q = l; q < d.m; q += 16) a += M[d.start + q];
    a = dgroup_sum_d<16>(a);
    const double T = (double)theta[d.v] + __shfl(a, (int)(threadIdx.x & 48), 64);
    if (x)
        for (int q = l; q < d.m; q += 16) x[px[d.start + q]] = (float)(T - (M ? M[d.start + q] : 0.0));
    if (L && l == 0) L[d.v] = (float)T;
}

hipError_t launch_kf_voxel(mrf_ctx* c, const double* M, const float* theta, float* x, float* L, hipStream_t s)
{
    if (c->n_kf_vox <= 0) return hipSuccess;
    ProfScope ps(c, KID_KFVOX, s);
    hipLaunchKernelGGL(kf_voxel_k, dim3(nblk(c->n_kf_vox, 16)), dim3(256), 0, s, (const VoxDev*)c->b_kf_vox.p,
                       c->n_kf_vox, M, (const uint32_t*)c->b_pair_x.p, theta, x, L);
    return hipGetLastError();
}

// Reverse of kf_voxel_k: with s_p the pair sums of d/d lambda (FP64), S_v =
// their sum over the voxel's pairs (the same fixed order); acc_v += fl(S_v)
// (d/d theta) and, when y is given, y = fl(S_v - s_p) into the pair's keyframe
// buffer: the derivative reaching the pair's average through every other
// keyframe's incoming message.
__global__ __launch_bounds__(256) void kf_voxel_rev_k(const VoxDev* __restrict__ vd, int64_t n,
                                                      const double* __restrict__ sp, const uint32_t* __restrict__ px,
                                                      float* __restrict__ acc, float* __restrict__ y)
{
    const int64_t vi = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 16 + (int)(threadIdx.x >> 4);
    if (vi >= n) return;   // whole group
    const int l = (int)(threadIdx.x & 15);
    const VoxDev d = vd[vi];
    double a = 0.0;
    for (int q = l; q < d.m; q += 16) a += sp[d.start + q];
    a = dgroup_sum_d<16>(a);
    const double S = __shfl(a, (int)(threadIdx.x & 48), 64);
    if (y)
        for (int q = l; q < d.m; q += 16) y[px[d.start + q]] = (float)(S - sp[d.start + q]);
    if (l == 0) acc[d.v] += (float)S;
}

hipError_t launch_kf_voxel_rev(mrf_ctx* c, const double* sp, float* acc, float* y, hipStream_t s)
{
    if (c->n_kf_vox <= 0) return hipSuccess;
    ProfScope ps(c, KID_KFVOX, s);
    hipLaunchKernelGGL(kf_voxel_rev_k, dim3(nblk(c->n_kf_vox, 16)), dim3(256), 0, s, (const VoxDev*)c->b_kf_vox.p,
                       c->n_kf_vox, sp, (const uint32_t*)c->b_pair_x.p, acc, y);
    return hipGetLastError();
}

// ------------------------------------------------------------ ray phase

// Messages of one ray held by a group of G lanes, blocked: lane l holds steps
// [i0, i0 + IPL), i0 = l IPL, as base-2 log mu(0) (al), log mu(1) (be) and g,
// with neutral padding past the ray's m steps.  With c_i = log mu_i(1) + g_i
// the kernel carries P-free quantities (P_i, the log visibility up to voxel i,
// can reach 1e6 and would leak its rounding into every message):
//   R_i = S_i - P_i:  R_0 = log 0,  R_{i+1} = LSE(R_i, c_i) - log mu_i(0)
//   Q_i:              Q_{m-1} = log 0,  Q_{i-1} = LSE(c_i, log mu_i(0) + Q_i)
//   ell_i = LSE(R_i, g_i) - LSE(R_i, Q_i)
// Both recurrences are maps x -> LSE(c, a + x), scanned once across the group
// on the lane aggregates and walked sequentially inside the lane.
// put(j, ok, ell) receives the natural-log message of step i0 + j (meaningful
// when ok, i.e. i0 + j < m).
template <int G, int IPL, class Put>
__device__ __forceinline__ void ray_body(const float (&al)[IPL], const float (&be)[IPL], const float (&gg)[IPL],
                                         int m, int i0, Put&& put)
{
    // lane aggregate Cl = LSE_j (c_j + lp_j), lp_j the lane-local prefix of
    // log mu(0), a the lane sum: the lane's R map is (-a, Cl - a) and its Q
    // map (a, Cl)
    float c[IPL], cw[IPL];
    float a = 0.0f;
#pragma unroll
    for (int j = 0; j < IPL; ++j) {
        c[j] = be[j] + gg[j];
        cw[j] = c[j] + a;
        a += al[j];
    }
    const float Cl = lse_items<IPL>(cw);
    float R[IPL];
    {
        const LMap left = dscan_lmap<G>(LMap{-a, Cl - a});
        float r = dexcl<G>(left.c, MRF_NINF);
#pragma unroll
        for (int j = 0; j < IPL; ++j) {
            R[j] = r;
            r = lse(r, c[j]) - al[j];
        }
    }
    const LMap right = drscan_lmap<G>(LMap{a, Cl});
    float Q = drexcl<G>(right.c, MRF_NINF);
#pragma unroll
    for (int j = IPL - 1; j >= 0; --j) {
        put(j, i0 + j < m, lse_diff(R[j], gg[j], Q) * kLn2);
        Q = lse(c[j], al[j] + Q);
    }
}

// Direct variant: each group reads its ray's steps from global memory (one
// 64-byte row per step holds the 16 rays of the tile); lambda_e = tot[col_e] -
// own_e.  Step indices are clamped to the ray (m >= 1) so that every load is
// issued before the first wait.
// With KF (per-keyframe averaged messages, Sec. IV-A) lambda_e is the message
// of the ray's keyframe, kf.x[kf.xb[frame] + col_e], instead.
template <int G, int IPL, bool KF>
__global__ __launch_bounds__(256) void ray_k(const uint32_t* __restrict__ list, int64_t ntiles,
                                             const TileDev* __restrict__ tiles, const int32_t* __restrict__ counts,
                                             const int32_t* __restrict__ col, ExclDev lam, KfSrc kf,
                                             const float* __restrict__ g, float* __restrict__ ell)
{
    static_assert(G == 64 || IPL == 1, "16-lane groups hold a whole ray");
    int64_t s;
    int m, frame = 0;
    if (!tile_ray<G>(list, ntiles, tiles, counts, s, m, &frame)) return;
    const int i0 = (int)(threadIdx.x & (G - 1)) * IPL;
    int32_t cv[IPL];
    float ov[IPL], gv[IPL], lv[IPL];
    float2 tv[IPL];
#pragma unroll
    for (int j = 0; j < IPL; ++j) {
        const int64_t at = s + kTile * (int64_t)min(i0 + j, m - 1);
        cv[j] = col[at];
        if constexpr (!KF) ov[j] = lam.own[at];
        gv[j] = g[at];
    }
    if constexpr (KF) {
        const float* xf = kf.x + kf.xb[frame];
#pragma unroll
        for (int j = 0; j < IPL; ++j) lv[j] = cv[j] >= 0 ? xf[cv[j]] : 0.0f;
    } else {
#pragma unroll
        for (int j = 0; j < IPL; ++j) tv[j] = lam.tot[max(cv[j], 0)];
#pragma unroll
        for (int j = 0; j < IPL; ++j) lv[j] = excl_value(cv[j], tv[j], ov[j], lam.has_own);
    }
    float al[IPL], be[IPL], gg[IPL];
#pragma unroll
    for (int j = 0; j < IPL; ++j) load_step(lv[j], gv[j], i0 + j < m, al[j], be[j], gg[j]);
    ray_body<G, IPL>(al, be, gg, m, i0, [&](int j, bool ok, float v) {
        if (ok) ell[s + kTile * (i0 + j)] = v;
    });
}

// Tile-staged variant for tiles of at most G*IPL steps: one block of 16 groups
// per tile.  The block reads the tile's col, own and g (16 rays x len steps,
// contiguous) with coalesced loads, gathers the voxel totals, and puts lambda
// = tot[col] - own and g into LDS; every group runs the scans of its own ray
// on its LDS column and writes ell back into that column (0 past the ray),
// and the block stores the tile coalesced.
template <int G, int IPL, bool KF>
__global__ __launch_bounds__(kTile * G) void ray_lds_k(const uint32_t* __restrict__ list, int64_t ntiles,
                                                       const TileDev* __restrict__ tiles,
                                                       const int32_t* __restrict__ counts,
                                                       const int32_t* __restrict__ col, ExclDev lam, KfSrc kf,
                                                       const float* __restrict__ g, float* __restrict__ ell)
{
    constexpr int NT = kTile * G;
    __shared__ float sl[kTile * G * IPL];
    __shared__ float sg[kTile * G * IPL];
    const int64_t ti = xcd_block(blockIdx.x, gridDim.x);
    if (ti >= ntiles) return;   // whole block
    const TileDev td = tiles[list[ti]];
    const int nf = kTile * td.len;   // 1 <= td.len <= G * IPL by class
    const int i = (int)threadIdx.x / G;   // this group's ray: lane i of the tile
    const int gl = (int)threadIdx.x % G;
    const int i0 = gl * IPL;
    const int cb = lds_col(i0, gl, i);
    const int m = tile_ray_len(td, counts, i);
    {
        int32_t vc[IPL];
        float vo[IPL], vg[IPL], vt[IPL];
        float2 vp[IPL];
        tile_fetch_i<NT, IPL>(col, td.base, nf, vc);
        if constexpr (!KF) tile_fetch<NT, IPL>(lam.own, td.base, nf, vo);
        tile_fetch<NT, IPL>(g, td.base, nf, vg);
        if constexpr (KF) {
            const float* xf = kf.x + kf.xb[td.frame];
#pragma unroll
            for (int r = 0; r < IPL; ++r) vt[r] = vc[r] >= 0 ? xf[vc[r]] : 0.0f;
        } else {
#pragma unroll
            for (int r = 0; r < IPL; ++r) vp[r] = lam.tot[max(vc[r], 0)];
#pragma unroll
            for (int r = 0; r < IPL; ++r) vt[r] = excl_value(vc[r], vp[r], vo[r], lam.has_own);
        }
        tile_to_lds<NT, IPL, IPL>(sl, vt);
        tile_to_lds<NT, IPL, IPL>(sg, vg);
    }
    __syncthreads();
    if (__ballot(m > 0)) {   // skip waves whose rays are all empty
        float al[IPL], be[IPL], gg[IPL];
#pragma unroll
        for (int j = 0; j < IPL; ++j)   // column rows are inside the LDS tile even past the ray
            load_step(sl[cb + kTile * j], sg[cb + kTile * j], i0 + j < m, al[j], be[j], gg[j]);
        ray_body<G, IPL>(al, be, gg, m, i0, [&](int j, bool ok, float v) { sl[cb + kTile * j] = ok ? v : 0.0f; });
    }
    __syncthreads();
    tile_store<NT, IPL, IPL>(ell, td.base, nf, [&](int, int at) { return sl[at]; });
}

// The voxel -> ray messages one ray-phase launch reads: per-edge exclusion
// from the voxel totals, or (kf) the per-keyframe message buffers.
struct RaySrc {
    ExclDev lam;
    KfSrc kf;
    bool is_kf;
};

template <int Q, int I, bool KF>
static void launch_ray_shape_t(const mrf_ctx* c, int64_t off, int64_t n, const RaySrc& src, float* ell, hipStream_t s)
{
    constexpr int G = kFwdShapes[Q][I].g;
    if constexpr (G != 0) {
        constexpr int CAP = kRayCap[Q];
        const uint32_t* list = (const uint32_t*)c->b_ray_list[Q].p + off;
        if constexpr (ray_class_lds(Q)) {
            hipLaunchKernelGGL((ray_lds_k<G, CAP / G, KF>), dim3((unsigned)n), dim3(kTile * G), 0, s, list, n,
                               (const TileDev*)c->b_tiles.p, (const int32_t*)c->b_counts.p,
                               (const int32_t*)c->b_col.p, src.lam, src.kf, (const float*)c->b_g.p, ell);
        } else {
            hipLaunchKernelGGL((ray_k<G, CAP / G, KF>), dim3((unsigned)(n * tile_blocks<G>())), dim3(256), 0, s,
                               list, n, (const TileDev*)c->b_tiles.p, (const int32_t*)c->b_counts.p,
                               (const int32_t*)c->b_col.p, src.lam, src.kf, (const float*)c->b_g.p, ell);
        }
    }
}

template <int Q, int I>
static void launch_ray_shape(const mrf_ctx* c, int64_t off, int64_t n, const RaySrc& src, float* ell, hipStream_t s)
{
    if (src.is_kf)
        launch_ray_shape_t<Q, I, true>(c, off, n, src, ell, s);
    else
        launch_ray_shape_t<Q, I, false>(c, off, n, src, ell, s);
}

template <int Q, int... I>
static void launch_ray_sel(int sel, const mrf_ctx* c, int64_t off, int64_t n, const RaySrc& src, float* ell,
                           hipStream_t s, std::integer_sequence<int, I...>)
{
    ((sel == I ? launch_ray_shape<Q, I>(c, off, n, src, ell, s) : void()), ...);
}

// class Q of the ray phase with launch shape sel, over n tiles of its list from off
template <int Q>
static void launch_ray_class(const mrf_ctx* c, int sel, int64_t off, int64_t n, const RaySrc& src, float* ell,
                             hipStream_t s)
{
    if (n <= 0) return;
    ProfScope ps(c, KID_RAY0 + Q, s);
    launch_ray_sel<Q>(sel, c, off, n, src, ell, s, std::make_integer_sequence<int, kNShapes>{});
}

// The untuned shape of the plain schedule: one 64-lane wave per ray where the
// class has such a shape (the 16-step class holds a ray in 16 lanes).
constexpr int plain_shape(int q)
{
    for (int i = 0; i < ray_shape_count(q, false); ++i)
        if (kFwdShapes[q][i].g == 64) return i;
    return 0;
}

template <int... Q>
static void ray_classes(std::integer_sequence<int, Q...>, const mrf_ctx* c, const int64_t* off, const int64_t* cnt,
                        const RaySrc& src, float* ell, bool plain, hipStream_t s)
{
    (launch_ray_class<Q>(c, plain ? plain_shape(Q) : c->fwd_sel[Q], off[Q], cnt[Q], src, ell, s), ...);
}

static void ray_classes(const mrf_ctx* c, const int64_t* off, const int64_t* cnt, const RaySrc& src, float* ell,
                        bool plain, hipStream_t s)
{
    ray_classes(std::make_integer_sequence<int, kRayClasses>{}, c, off, cnt, src, ell, plain, s);
}

using RayClassFn = void (*)(const mrf_ctx*, int, int64_t, int64_t, const RaySrc&, float*, hipStream_t);
template <int... Q>
static constexpr std::array<RayClassFn, kRayClasses> ray_class_fns(std::integer_sequence<int, Q...>)
{
    return {&launch_ray_class<Q>...};
}

static hipError_t ray_class_shape(const mrf_ctx* c, int q, int sel, const RaySrc& src, float* ell, hipStream_t s)
{
    static constexpr std::array<RayClassFn, kRayClasses> fns =
        ray_class_fns(std::make_integer_sequence<int, kRayClasses>{});
    if (q < 0 || q >= kRayClasses || sel < 0 || sel >= ray_shape_count(q, false)) return hipErrorInvalidValue;
    fns[q](c, sel, 0, c->ray_cnt[q], src, ell, s);
    return hipGetLastError();
}

hipError_t launch_ray_class_shape(const mrf_ctx* c, int q, int sel, ExclSrc lam, float* ell, hipStream_t s)
{
    return ray_class_shape(c, q, sel, RaySrc{excl_dev(c, lam), KfSrc{nullptr, nullptr}, false}, ell, s);
}

hipError_t launch_ray_class_shape_kf(const mrf_ctx* c, int q, int sel, KfSrc lam, float* ell, hipStream_t s)
{
    return ray_class_shape(c, q, sel, RaySrc{excl_dev(c, ExclSrc{nullptr, nullptr}), lam, true}, ell, s);
}

static hipError_t ray_phase(mrf_ctx* c, const RaySrc& src, float* ell, bool plain, hipStream_t s)
{
    int64_t off[kRayClasses] = {0}, cnt[kRayClasses];
    if (!plain) {
        for (int k = 0; k < kRayClasses; ++k) cnt[k] = c->ray_cnt[k];
        ray_classes(c, off, cnt, src, ell, false, s);
    } else {
        // the plain per-frame schedule: one launch per frame (per class), untuned shapes
        const int nf = c->n_frames;
        for (int f = 0; f < nf; ++f) {
            for (int k = 0; k < kRayClasses; ++k) {
                const int64_t* fo = c->frame_ray_off.data() + (size_t)k * (nf + 1);
                off[k] = fo[f];
                cnt[k] = fo[f + 1] - fo[f];
            }
            ray_classes(c, off, cnt, src, ell, true, s);
        }
    }
    return hipGetLastError();
}

hipError_t launch_ray_phase(mrf_ctx* c, ExclSrc lam_src, float* ell, bool plain, hipStream_t s)
{
    return ray_phase(c, RaySrc{excl_dev(c, lam_src), KfSrc{nullptr, nullptr}, false}, ell, plain, s);
}

hipError_t launch_ray_phase_kf(mrf_ctx* c, KfSrc lam, float* ell, bool plain, hipStream_t s)
{
    return ray_phase(c, RaySrc{excl_dev(c, ExclSrc{nullptr, nullptr}), lam, true}, ell, plain, s);
}

// lambda_e of the per-keyframe messages on every slot (exports)
__global__ void excl_kf_k(const int32_t* __restrict__ col, const int64_t* __restrict__ fs, int nf, KfSrc x,
                          float* __restrict__ out, int64_t S)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = col[i];
        int lo = 0, hi = nf;   // frame of slot i: the last f with fs[f] <= i
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (fs[mid] <= i)
                lo = mid;
            else
                hi = mid;
        }
        out[i] = v >= 0 ? x.x[x.xb[lo] + v] : 0.0f;
    }
}

hipError_t launch_excl_kf(const mrf_ctx* c, KfSrc x, float* out, hipStream_t s)
{
    if (c->S <= 0) return hipSuccess;
    const int64_t* fs = (const int64_t*)c->b_kfxb.p + c->n_frames + 1;
    hipLaunchKernelGGL(excl_kf_k, dim3(grid_for(c->S)), dim3(256), 0, s, (const int32_t*)c->b_col.p, fs, c->n_frames,
                       x, out, c->S);
    return hipGetLastError();
}

}  // namespace mrf

namespace mrf {

// ------------------------------------------------------------ depth messages
//
// The ray factor's message to its depth variable (Eq. depth_message, Sec.
// III-C): the measurement came from voxel i's depth with weight
// nu(d_i) mu_i(1) prod_{k<i} mu_k(0), mu the voxel -> ray messages of the last
// sweep, normalised over the ray (the all-empty configuration has potential
// zero).  One thread per ray walks its steps twice: the log2 weights W_i =
// log2 mu_i(1) + log2 nu_i + P_i, with the visibility P_i summed in FP64, give
// the running maximum (the mode, first on ties) and the normaliser; then
// q_i = 2^(W_i - max) / sum and the mean depth sum_i q_i d_i, d_i = Z - delta_i.
__global__ __launch_bounds__(256) void depth_dist_k(const TileDev* __restrict__ tiles, int64_t T,
                                                    const FrameDev* __restrict__ frames,
                                                    const int32_t* __restrict__ counts,
                                                    const int32_t* __restrict__ col, ExclDev lam, KfSrc kf,
                                                    int is_kf, const float* __restrict__ g,
                                                    const float* __restrict__ delta, float* __restrict__ q,
                                                    int32_t* __restrict__ mode, float* __restrict__ mean)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ti = t / kTile;
    if (ti >= T) return;
    const int i = (int)(t % kTile);
    const TileDev td = tiles[ti];
    const int ux = i & (kTileW - 1), vy = i / kTileW;
    if (ux >= td.nu || vy >= td.nv) return;
    const int64_t r = td.ray0 + (int64_t)vy * td.W + ux;
    const int m = counts[r];
    if (m == 0) {
        if (mode) mode[r] = -1;
        if (mean) mean[r] = __builtin_nanf("");
        return;
    }
    const int64_t s0 = td.base + i;
    const float* xf = is_kf ? kf.x + kf.xb[td.frame] : nullptr;
    auto weight = [&](int k, double& P) {   // W_k (log2), then P += log2 mu_k(0)
        const int64_t at = s0 + (int64_t)kTile * k;
        const int32_t v = col[at];
        const float lm = is_kf ? xf[v] : excl_value(v, lam.tot[v], lam.own[at], lam.has_own);
        float al, be, gg;
        load_step(lm, g[at], true, al, be, gg);
        const double W = ((double)be + (double)gg) + P;
        P += (double)al;
        return W;
    };
    double P = 0.0, M = -__builtin_huge_val(), S = 0.0;
    int best = 0;
    for (int k = 0; k < m; ++k) {
        const double W = weight(k, P);
        if (W > M) {
            S = S * (double)ex2((float)(M - W)) + 1.0;
            M = W;
            best = k;
        } else {
            S += (double)ex2((float)(W - M));
        }
    }
    if (mode) mode[r] = best;
    const FrameDev fr = frames[td.frame];
    const double Z = (double)fr.depth[r - fr.ray_base];
    double mq = 0.0;
    P = 0.0;
    for (int k = 0; k < m; ++k) {
        const double W = weight(k, P);
        const double qk = (double)ex2((float)(W - M)) / S;
        if (q) q[s0 + (int64_t)kTile * k] = (float)qk;
        mq += qk * (Z - (double)delta[s0 + (int64_t)kTile * k]);
    }
    if (mean) mean[r] = (float)mq;
}

hipError_t launch_depth_distribution(const mrf_ctx* c, ExclSrc lam, const KfSrc* kf, float* q, int32_t* mode,
                                     float* mean, hipStream_t s)
{
    if (c->T <= 0) return hipSuccess;
    const int64_t n = c->T * kTile;
    hipLaunchKernelGGL(depth_dist_k, dim3(nblk(n, 256)), dim3(256), 0, s, (const TileDev*)c->b_tiles.p, c->T,
                       (const FrameDev*)c->b_frames.p, (const int32_t*)c->b_counts.p, (const int32_t*)c->b_col.p,
                       excl_dev(c, lam), kf ? *kf : KfSrc{nullptr, nullptr}, kf ? 1 : 0, (const float*)c->b_g.p,
                       (const float*)c->b_delta.p, q, mode, mean);
    return hipGetLastError();
}

}  // namespace mrf
