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
// Voxel phase: one group of lanes per voxel's edge list (or per 1024-edge
// piece of a hub voxel), exclusive prefix and suffix sums, never a
// difference, so large log-odds never cancel.
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

__global__ void gather_voxel_k(const int32_t* __restrict__ col, const float* __restrict__ vox,
                               float* __restrict__ edge, int64_t E)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x)
    {
        const int32_t v = col[i];
        if (v >= 0) edge[i] = vox[v];   // padding slots carry col = -1
    }
}

__global__ void sigmoid_k(const float* __restrict__ L, float* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 1.0f / (1.0f + __expf(-L[i]));
}

// g_e = -(delta_e / sigma_b)^2 / 2 - log sigma_b - log(2 pi) / 2
__global__ __launch_bounds__(256) void potentials_k(const float* __restrict__ delta, const uint8_t* __restrict__ bin,
                                                    int64_t E, const float* __restrict__ sigma, float* __restrict__ g)
{
    __shared__ float inv[kBins], cst[kBins];
    if (threadIdx.x < kBins) {
        const float s = sigma[threadIdx.x];
        inv[threadIdx.x] = 1.0f / s;
        cst[threadIdx.x] = logf(s) + 0.91893853320467274f;
    }
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        const int b = bin[e];
        if (b >= kBins) continue;   // padding slot
        const float x = delta[e] * inv[b];
        g[e] = -0.5f * x * x - cst[b];
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

hipError_t launch_gather_voxel(const int32_t* col, const float* vox, float* edge, int64_t E, hipStream_t s)
{
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_voxel_k, dim3(grid_for(E)), dim3(256), 0, s, col, vox, edge, E);
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
    hipLaunchKernelGGL(potentials_k, dim3(grid_for(c->S)), dim3(256), 0, s, (const float*)c->b_delta.p,
                       (const uint8_t*)c->b_bin.p, c->S, (const float*)c->b_sigma.p, (float*)c->b_g.p);
    return hipGetLastError();
}

// ------------------------------------------------------------ voxel phase

constexpr int VIPL = kVoxChunk / 64;   // items per lane in a 256-edge chunk

// Items base + 64 k + l (k < N, l the lane) of the edge list [s, s+m) of one
// voxel: their slots into e and incoming messages into x (0 past m, or
// everywhere when in is null).  Branchless, with item indices clamped to
// m - 1 (m >= 1), so that every load is issued before the first wait.
template <int N>
__device__ __forceinline__ void vox_gather(int64_t s, int m, int base, const uint32_t* __restrict__ vedge,
                                           const float* __restrict__ in, uint32_t (&e)[N], float (&x)[N])
{
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < N; ++k) e[k] = vedge[s + min(base + k * 64 + l, m - 1)];
    if (in) {
#pragma unroll
        for (int k = 0; k < N; ++k) x[k] = in[e[k]];
#pragma unroll
        for (int k = 0; k < N; ++k) x[k] = base + k * 64 + l < m ? x[k] : 0.0f;
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) x[k] = 0.0f;
    }
}

// Sum of chunk c of the segment [s, s+m) (every lane gets it).
__device__ __forceinline__ float vox_chunk_sum(int64_t s, int m, int c, const uint32_t* __restrict__ vedge,
                                               const float* __restrict__ in)
{
    if (!in) return 0.0f;
    float x[VIPL];
    uint32_t e[VIPL];
    vox_gather<VIPL>(s, m, c * kVoxChunk, vedge, in, e, x);
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < VIPL; ++k) acc += x[k];
    return wave_sum(acc);
}

// Chunk c of the segment: out_e = (b0 + sum of earlier edges) + sum of later
// edges, with pre0 / suf0 the sums of the chunks before / after this one.
// Returns pre0 + the chunk's sum.
__device__ __forceinline__ float vox_chunk(int64_t s, int m, int c, const uint32_t* __restrict__ vedge,
                                           const float* __restrict__ in, float* __restrict__ out, float b0,
                                           float pre0, float suf0)
{
    const int l = threadIdx.x & 63;
    float x[VIPL];
    uint32_t e[VIPL];
    vox_gather<VIPL>(s, m, c * kVoxChunk, vedge, in, e, x);
    float pre[VIPL];
    float carry = pre0;
#pragma unroll
    for (int k = 0; k < VIPL; ++k) {
        const float incl = dscan<64, OpAdd>(x[k]) + carry;
        pre[k] = dexcl<64>(incl, carry);
        carry = readlane(incl, 63);
    }
    if (out) {
        float sc = suf0;
#pragma unroll
        for (int k = VIPL - 1; k >= 0; --k) {
            const float incl = drscan<64, OpAdd>(x[k]) + sc;
            const float suf = drexcl<64>(incl, sc);
            sc = readlane(incl, 0);
            if (c * kVoxChunk + k * 64 + l < m) out[e[k]] = (b0 + pre[k]) + suf;
        }
    }
    return carry;
}

// One voxel's edge list [s, s+m) held by NW waves, each owning 64*IPL
// consecutive edges (striped over its lanes) gathered once into registers.
// Waves exchange their sums through LDS for the carries.  NW == 1 packs four
// voxels per 256-thread block.  Voxels arrive in brick-major order and blocks
// are remapped so each XCD takes a contiguous range of them.
template <int NW, int IPL>
__global__ __launch_bounds__(NW == 1 ? 256 : 64 * NW) void voxel_k(
    const VoxDev* __restrict__ vd, int64_t n, const uint32_t* __restrict__ vedge, const float* __restrict__ base,
    const float* __restrict__ in, float* __restrict__ out, float* __restrict__ total, int total_mode)
{
    constexpr int SPAN = 64 * IPL;
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t vi = NW == 1 ? lb * 4 + wv : lb;
    const int part = NW == 1 ? 0 : wv;
    if (vi >= n) return;   // whole waves (NW == 1) or whole blocks (NW > 1)
    const VoxDev d = vd[vi];
    const uint32_t v = d.v;
    const int64_t s = d.start;
    const int m = d.m;
    const float b0 = base ? base[v] : 0.0f;

    float x[IPL];
    uint32_t e[IPL];
    vox_gather<IPL>(s, m, part * SPAN, vedge, in, e, x);
    float pre0 = 0.0f, suf0 = 0.0f, tot = 0.0f;
    if (NW > 1) {
        __shared__ float wsum[NW > 1 ? NW : 1];
        float a = 0.0f;
#pragma unroll
        for (int k = 0; k < IPL; ++k) a += x[k];
        a = wave_sum(a);
        if (l == 0) wsum[wv] = a;
        __syncthreads();
        for (int q = 0; q < NW; ++q) {
            if (q < wv) pre0 += wsum[q];
            tot += wsum[q];
        }
        for (int q = NW - 1; q > wv; --q) suf0 += wsum[q];
    }
    float pre[IPL];
    float carry = pre0;
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const float incl = dscan<64, OpAdd>(x[k]) + carry;
        pre[k] = dexcl<64>(incl, carry);
        carry = readlane(incl, 63);
    }
    if (NW == 1) tot = carry;
    if (out) {
        float sc = suf0;
#pragma unroll
        for (int k = IPL - 1; k >= 0; --k) {
            const float incl = drscan<64, OpAdd>(x[k]) + sc;
            const float suf = drexcl<64>(incl, sc);
            sc = readlane(incl, 0);
            if (part * SPAN + k * 64 + l < m) out[e[k]] = (b0 + pre[k]) + suf;
        }
    }
    if (total_mode && l == 0 && part == 0) {
        if (total_mode == 1)
            total[v] = b0 + tot;
        else
            total[v] += tot;
    }
}

// Voxels of at most G edges (G = 16 or 32), 64 / G per wave and 256 / G per
// block: lane l of a group holds edge l of its voxel, and the exclusive prefix
// and suffix come from group scans.  Groups past the list take no edges.
template <int G>
__global__ __launch_bounds__(256) void voxel_small_k(const VoxDev* __restrict__ vd, int64_t n,
                                                     const uint32_t* __restrict__ vedge,
                                                     const float* __restrict__ base, const float* __restrict__ in,
                                                     float* __restrict__ out, float* __restrict__ total,
                                                     int total_mode)
{
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    if (lb * (256 / G) >= n) return;   // whole block
    const int64_t vi = lb * (256 / G) + (int)threadIdx.x / G;
    const int l = (int)threadIdx.x % G;
    VoxDev d{0, 0, 0};
    if (vi < n) d = vd[vi];
    const int m = d.m;
    uint32_t e = 0;
    float x = 0.0f;
    if (m > 0) {
        e = vedge[d.start + min(l, m - 1)];
        if (in) {
            const float y = in[e];
            x = l < m ? y : 0.0f;
        }
    }
    const float b0 = (m > 0 && base) ? base[d.v] : 0.0f;
    const float pre = dexcl<G>(dscan<G, OpAdd>(x), 0.0f);
    const float sinc = drscan<G, OpAdd>(x);   // at group lane 0: the voxel's sum
    const float suf = drexcl<G>(sinc, 0.0f);
    if (out && l < m) out[e] = (b0 + pre) + suf;
    if (total_mode && l == 0 && m > 0) {
        if (total_mode == 1)
            total[d.v] = b0 + sinc;
        else
            total[d.v] += sinc;
    }
}

// One 1024-thread block per voxel of degree above the largest single-pass
// class: chunk sums into LDS, exclusive prefix / suffix of the chunk sums by
// wave 0 in fixed order, then every wave revisits its chunks with both carries.
__global__ __launch_bounds__(1024) void voxel_chunked_k(const VoxDev* __restrict__ vd, int64_t n,
                                                        const uint32_t* __restrict__ vedge,
                                                        const float* __restrict__ base, const float* __restrict__ in,
                                                        float* __restrict__ out, float* __restrict__ total,
                                                        int total_mode)
{
    __shared__ float csum[kVoxMaxChunks];
    __shared__ float cpre[kVoxMaxChunks];
    __shared__ float csuf[kVoxMaxChunks];
    __shared__ float stot;
    const int64_t b = xcd_block(blockIdx.x, gridDim.x);
    if (b >= n) return;
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    const VoxDev d = vd[b];
    const uint32_t v = d.v;
    const int64_t s = d.start;
    const int m = d.m;
    const float b0 = base ? base[v] : 0.0f;
    const int nch = (m + kVoxChunk - 1) / kVoxChunk;   // <= kVoxMaxChunks (checked at build)
    for (int c = wv; c < nch; c += 16) {
        const float cs = vox_chunk_sum(s, m, c, vedge, in);
        if (l == 0) csum[c] = cs;
    }
    __syncthreads();
    if (wv == 0) {
        float carry = 0.0f;
        for (int c0 = 0; c0 < nch; c0 += 64) {
            const float x = c0 + l < nch ? csum[c0 + l] : 0.0f;
            const float incl = dscan<64, OpAdd>(x) + carry;
            if (c0 + l < nch) cpre[c0 + l] = dexcl<64>(incl, carry);
            carry = readlane(incl, 63);
        }
        if (l == 0) stot = carry;
        float sc = 0.0f;
        for (int c0 = ((nch - 1) / 64) * 64; c0 >= 0; c0 -= 64) {
            const float x = c0 + l < nch ? csum[c0 + l] : 0.0f;
            const float incl = drscan<64, OpAdd>(x) + sc;
            if (c0 + l < nch) csuf[c0 + l] = drexcl<64>(incl, sc);
            sc = readlane(incl, 0);
        }
    }
    __syncthreads();
    if (out)
        for (int c = wv; c < nch; c += 16) vox_chunk(s, m, c, vedge, in, out, b0, cpre[c], csuf[c]);
    if (total_mode && threadIdx.x == 0) {
        if (total_mode == 1)
            total[v] = b0 + stot;
        else
            total[v] += stot;
    }
}

template <int K>
static void launch_voxel_class(mrf_ctx* c, const float* base, const float* in, float* out, float* total, int mode,
                               hipStream_t s)
{
    const int64_t n = c->vox_cnt[K];
    if (n <= 0) return;
    ProfScope ps(c, KID_VOX0 + K, s);
    constexpr int NW = kVoxNW[K];
    if constexpr (NW == 0) {
        constexpr int G = kVoxCap[K];
        hipLaunchKernelGGL((voxel_small_k<G>), dim3(nblk(n, 256 / G)), dim3(256), 0, s,
                           (const VoxDev*)c->b_vox_desc[K].p, n, (const uint32_t*)c->b_vedge.p, base, in, out,
                           total, mode);
    } else {
        constexpr int IPL = kVoxCap[K] / (64 * NW);
        const unsigned blocks = NW == 1 ? nblk(n, 4) : (unsigned)n;
        hipLaunchKernelGGL((voxel_k<NW, IPL>), dim3(blocks), dim3(NW == 1 ? 256 : 64 * NW), 0, s,
                           (const VoxDev*)c->b_vox_desc[K].p, n, (const uint32_t*)c->b_vedge.p, base, in, out,
                           total, mode);
    }
}

template <int... K>
static void voxel_classes(std::integer_sequence<int, K...>, mrf_ctx* c, const float* base, const float* in,
                          float* out, float* total, int mode, hipStream_t s)
{
    (launch_voxel_class<K>(c, base, in, out, total, mode, s), ...);
}

hipError_t launch_voxel_phase(mrf_ctx* c, const float* base, const float* in, float* out, float* total,
                              int total_mode, bool /*plain*/, hipStream_t s)
{
    voxel_classes(std::make_integer_sequence<int, kVoxClasses - 1>{}, c, base, in, out, total, total_mode, s);
    const int kc = kVoxClasses - 1;
    if (c->vox_cnt[kc] > 0) {
        ProfScope ps(c, KID_VOX0 + kc, s);
        hipLaunchKernelGGL(voxel_chunked_k, dim3((unsigned)c->vox_cnt[kc]), dim3(1024), 0, s,
                           (const VoxDev*)c->b_vox_desc[kc].p, c->vox_cnt[kc], (const uint32_t*)c->b_vedge.p, base,
                           in, out, total, total_mode);
    }
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
// 64-byte row per step holds the 16 rays of the tile).
template <int G, int IPL>
__global__ __launch_bounds__(256) void ray_k(const uint32_t* __restrict__ list, int64_t ntiles,
                                             const TileDev* __restrict__ tiles, const int32_t* __restrict__ counts,
                                             const float* __restrict__ lam, const float* __restrict__ g,
                                             float* __restrict__ ell)
{
    static_assert(G == 64 || IPL == 1, "16-lane groups hold a whole ray");
    int64_t s;
    int m;
    if (!tile_ray<G>(list, ntiles, tiles, counts, s, m)) return;
    const int i0 = (int)(threadIdx.x & (G - 1)) * IPL;
    float al[IPL], be[IPL], gg[IPL];
#pragma unroll
    for (int j = 0; j < IPL; ++j) {
        const int i = i0 + j;
        const bool ok = i < m;
        load_step(ok ? lam[s + kTile * i] : 0.0f, ok ? g[s + kTile * i] : 0.0f, ok, al[j], be[j], gg[j]);
    }
    ray_body<G, IPL>(al, be, gg, m, i0, [&](int j, bool ok, float v) {
        if (ok) ell[s + kTile * (i0 + j)] = v;
    });
}

// Tile-staged variant for tiles of at most G*IPL steps: one block of 16 groups
// per tile.  The block copies the tile's lambda and g (16 rays x len steps,
// contiguous) into LDS with coalesced loads, every group runs the scans of its
// own ray on its LDS column and writes ell back into that column (0 past the
// ray), and the block stores the tile coalesced.
template <int G, int IPL>
__global__ __launch_bounds__(kTile * G) void ray_lds_k(const uint32_t* __restrict__ list, int64_t ntiles,
                                                       const TileDev* __restrict__ tiles,
                                                       const int32_t* __restrict__ counts,
                                                       const float* __restrict__ lam, const float* __restrict__ g,
                                                       float* __restrict__ ell)
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
        float vl[IPL], vg[IPL];
        tile_fetch<NT, IPL>(lam, td.base, nf, vl);
        tile_fetch<NT, IPL>(g, td.base, nf, vg);
        tile_to_lds<NT, IPL, IPL>(sl, nf, vl);
        tile_to_lds<NT, IPL, IPL>(sg, nf, vg);
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
#pragma unroll
    for (int r = 0; r < IPL; ++r) {
        const int idx = (int)threadIdx.x + r * NT;
        if (idx < nf) ell[td.base + idx] = sl[lds_at<IPL>(idx >> 4, idx & (kTile - 1))];
    }
}

template <int Q, int I>
static void launch_ray_shape(const mrf_ctx* c, int64_t off, int64_t n, const float* lam, float* ell, hipStream_t s)
{
    constexpr int G = kFwdShapes[Q][I].g;
    if constexpr (G != 0) {
        constexpr int CAP = kRayCap[Q];
        const uint32_t* list = (const uint32_t*)c->b_ray_list[Q].p + off;
        if constexpr (ray_class_lds(Q)) {
            hipLaunchKernelGGL((ray_lds_k<G, CAP / G>), dim3((unsigned)n), dim3(kTile * G), 0, s, list, n,
                               (const TileDev*)c->b_tiles.p, (const int32_t*)c->b_counts.p, lam,
                               (const float*)c->b_g.p, ell);
        } else {
            hipLaunchKernelGGL((ray_k<G, CAP / G>), dim3((unsigned)(n * tile_blocks<G>())), dim3(256), 0, s, list,
                               n, (const TileDev*)c->b_tiles.p, (const int32_t*)c->b_counts.p, lam,
                               (const float*)c->b_g.p, ell);
        }
    }
}

template <int Q, int... I>
static void launch_ray_sel(int sel, const mrf_ctx* c, int64_t off, int64_t n, const float* lam, float* ell,
                           hipStream_t s, std::integer_sequence<int, I...>)
{
    ((sel == I ? launch_ray_shape<Q, I>(c, off, n, lam, ell, s) : void()), ...);
}

// class Q of the ray phase with launch shape sel, over n tiles of its list from off
template <int Q>
static void launch_ray_class(const mrf_ctx* c, int sel, int64_t off, int64_t n, const float* lam, float* ell,
                             hipStream_t s)
{
    if (n <= 0) return;
    ProfScope ps(c, KID_RAY0 + Q, s);
    launch_ray_sel<Q>(sel, c, off, n, lam, ell, s, std::make_integer_sequence<int, kNShapes>{});
}

template <int... Q>
static void ray_classes(std::integer_sequence<int, Q...>, const mrf_ctx* c, const int64_t* off, const int64_t* cnt,
                        const float* lam, float* ell, hipStream_t s)
{
    (launch_ray_class<Q>(c, c->fwd_sel[Q], off[Q], cnt[Q], lam, ell, s), ...);
}

static void ray_classes(const mrf_ctx* c, const int64_t* off, const int64_t* cnt, const float* lam, float* ell,
                        hipStream_t s)
{
    ray_classes(std::make_integer_sequence<int, kRayClasses>{}, c, off, cnt, lam, ell, s);
}

using RayClassFn = void (*)(const mrf_ctx*, int, int64_t, int64_t, const float*, float*, hipStream_t);
template <int... Q>
static constexpr std::array<RayClassFn, kRayClasses> ray_class_fns(std::integer_sequence<int, Q...>)
{
    return {&launch_ray_class<Q>...};
}

hipError_t launch_ray_class_shape(const mrf_ctx* c, int q, int sel, const float* lam, float* ell, hipStream_t s)
{
    static constexpr std::array<RayClassFn, kRayClasses> fns =
        ray_class_fns(std::make_integer_sequence<int, kRayClasses>{});
    if (q < 0 || q >= kRayClasses || sel < 0 || sel >= ray_shape_count(q, false)) return hipErrorInvalidValue;
    fns[q](c, sel, 0, c->ray_cnt[q], lam, ell, s);
    return hipGetLastError();
}

hipError_t launch_ray_phase(mrf_ctx* c, const float* lam, float* ell, bool plain, hipStream_t s)
{
    int64_t off[kRayClasses] = {0}, cnt[kRayClasses];
    if (!plain) {
        for (int k = 0; k < kRayClasses; ++k) cnt[k] = c->ray_cnt[k];
        ray_classes(c, off, cnt, lam, ell, s);
    } else {
        // one launch per frame (per class): the plain per-frame schedule
        const int nf = c->n_frames;
        for (int f = 0; f < nf; ++f) {
            for (int k = 0; k < kRayClasses; ++k) {
                const int64_t* fo = c->frame_ray_off.data() + (size_t)k * (nf + 1);
                off[k] = fo[f];
                cnt[k] = fo[f + 1] - fo[f];
            }
            ray_classes(c, off, cnt, lam, ell, s);
        }
    }
    return hipGetLastError();
}

}  // namespace mrf
