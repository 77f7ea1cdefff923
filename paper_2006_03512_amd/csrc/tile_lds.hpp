// Helpers shared by the ray-phase and reverse-pass kernels that stage a tile
// of 16 rays (step-major, 16 floats per step) through LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "dev_common.hpp"
#include "mrf_internal.hpp"

namespace mrf {

// Per-region sensor tables (Sec. IV-C): the row of a tile's rays is that of
// their pixel region.  Region sides are multiples of 4 pixels, so a 4x4 tile
// lies in one region, found from the tile's top-left pixel.
__device__ __forceinline__ int64_t tile_cell(const TileDev& t, const FrameDev* __restrict__ frames, int cp)
{
    const int64_t pix = (int64_t)t.ray0 - frames[t.frame].ray_base;
    const int v0 = (int)(pix / t.W), u0 = (int)(pix - (int64_t)v0 * t.W);
    return (int64_t)(v0 / cp) * ((t.W + cp - 1) / cp) + u0 / cp;
}

// LDS word of (step k, tile lane i) for rays held IPL steps per lane: row k
// of 16 words, the lane index XOR-ed with (k / IPL) mod 16.  Coalesced
// staging (16 consecutive threads per step) still fills whole rows, and the
// column reads of a group (lane l at steps l IPL + j) see a different XOR in
// every lane, which spreads them over the banks.
template <int IPL>
__device__ __forceinline__ int lds_at(int k, int i)
{
    return k * kTile + (i ^ ((k / IPL) & (kTile - 1)));
}

// lds_at<IPL>(i0 + j, i) for the steps [i0, i0 + IPL) of group lane gl
// (i0 = gl IPL, so (i0 + j) / IPL = gl): the column base; step i0 + j is at
// base + 16 j, an immediate offset.
__device__ __forceinline__ int lds_col(int i0, int gl, int i)
{
    return i0 * kTile + (i ^ (gl & (kTile - 1)));
}

// A block of NT threads moves a tile's nf = 16 len floats (nf <= NT NR) in NR
// rounds.  With NR a multiple of 4, thread t handles four consecutive floats per
// group of rounds, idx = 4 (t + q NT) + b for round r = 4 q + b (16-byte loads
// and stores); otherwise idx = t + r NT.  Loads go through registers so that
// every round's load is issued before the first wait; indices past nf are
// clamped to the tile's last floats and their values dropped.  The tile starts
// 64-byte aligned (tile bases are multiples of 16 slots).
template <int NT, int NR>
__device__ __forceinline__ int tile_idx(int r)
{
    if constexpr (NR % 4 == 0)
        return 4 * ((int)threadIdx.x + (r >> 2) * NT) + (r & 3);
    else
        return (int)threadIdx.x + r * NT;
}

template <int NT, int NR, class T>
__device__ __forceinline__ void tile_fetch_t(const T* __restrict__ src, int64_t base, int nf, T (&v)[NR])
{
    static_assert(sizeof(T) == 4, "32-bit items");
    if constexpr (NR % 4 == 0) {
        using V4 = typename std::conditional<std::is_same<T, float>::value, float4, int4>::type;
        const V4* p = (const V4*)(src + base);
        const int n4 = nf >> 2;
#pragma unroll
        for (int q = 0; q < NR / 4; ++q) {
            const V4 w = p[min((int)threadIdx.x + q * NT, n4 - 1)];
            v[4 * q] = w.x;
            v[4 * q + 1] = w.y;
            v[4 * q + 2] = w.z;
            v[4 * q + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = src[base + min((int)threadIdx.x + r * NT, nf - 1)];
    }
}

template <int NT, int NR>
__device__ __forceinline__ void tile_fetch(const float* __restrict__ src, int64_t base, int nf, float (&v)[NR])
{
    tile_fetch_t<NT, NR, float>(src, base, nf, v);
}

template <int NT, int NR>
__device__ __forceinline__ void tile_fetch_i(const int32_t* __restrict__ src, int64_t base, int nf, int32_t (&v)[NR])
{
    tile_fetch_t<NT, NR, int32_t>(src, base, nf, v);
}

// Values of the LDS image (layout lds_at<IPL>) to global memory, in the
// mapping of tile_idx: 16-byte stores when NR is a multiple of 4.
template <int NT, int NR, int IPL, class F>
__device__ __forceinline__ void tile_store(float* __restrict__ dst, int64_t base, int nf, F val)
{
    if constexpr (NR % 4 == 0) {
        float4* p = (float4*)(dst + base);
#pragma unroll
        for (int q = 0; q < NR / 4; ++q) {
            const int i4 = (int)threadIdx.x + q * NT;
            if (4 * i4 < nf) {
                const int k = i4 >> 2, l0 = (i4 & 3) << 2;
                p[i4] = make_float4(val(4 * q, lds_at<IPL>(k, l0)), val(4 * q + 1, lds_at<IPL>(k, l0 + 1)),
                                    val(4 * q + 2, lds_at<IPL>(k, l0 + 2)), val(4 * q + 3, lds_at<IPL>(k, l0 + 3)));
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int idx = (int)threadIdx.x + r * NT;
            if (idx < nf) dst[base + idx] = val(r, lds_at<IPL>(idx >> 4, idx & (kTile - 1)));
        }
    }
}

// Per-edge value tot[col] - own (the voxel's total less the edge's own term;
// own absent when has_own is 0), 0 on padding slots (col < 0).  t is the
// gathered total pair (hi, lo) of tot[max(col, 0)]: (hi - own) + lo, where
// hi - own is exact whenever own is within a factor two of hi (Sterbenz), so
// a near-total cancellation leaves lo and the FP64 sum's accuracy.  Selects,
// so stale bits on padding never propagate.
__device__ __forceinline__ float excl_value(int32_t col, float2 t, float own, int has_own)
{
    return col >= 0 ? (t.x - (has_own ? own : 0.0f)) + t.y : 0.0f;
}

// The fetched values into the LDS image of the tile (layout lds_at<IPL>).
template <int NT, int NR, int IPL>
__device__ __forceinline__ void tile_to_lds(float* __restrict__ lds, int nf, const float (&v)[NR])
{
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int idx = tile_idx<NT, NR>(r);
        if (idx < nf) lds[lds_at<IPL>(idx >> 4, idx & (kTile - 1))] = v[r];
    }
}

// steps of tile lane i (0 for pixels outside the image)
__device__ __forceinline__ int tile_ray_len(const TileDev& td, const int32_t* __restrict__ counts, int i)
{
    const int ux = i & (kTileW - 1), vy = i / kTileW;
    return (ux < td.nu && vy < td.nv) ? counts[td.ray0 + (int64_t)vy * td.W + ux] : 0;
}

// base-2 log mu(0), log mu(1) and g of one step from lambda and g (natural
// log); neutral padding (0, log 0, 0) when the step is past the ray.  With
// x = lambda log2(e) and t = log2(1 + 2^-|x|): log mu(0) = -(max(x, 0) + t),
// log mu(1) = -(max(-x, 0) + t), both free of cancellation (x - softplus(x)
// would lose the small one to the rounding of x once |lambda| is large).  No
// branch: past the ray the inputs may be any bits and are discarded by the
// selects.
__device__ __forceinline__ void load_step(float lam, float g, bool ok, float& al, float& be, float& gg)
{
    const float x = lam * kLog2e;
    const float t = lg2(1.0f + ex2(-fabsf(x)));
    al = ok ? -(fmaxf(x, 0.0f) + t) : 0.0f;
    be = ok ? -(fmaxf(-x, 0.0f) + t) : MRF_NINF;
    gg = ok ? g * kLog2e : 0.0f;
}

}  // namespace mrf
