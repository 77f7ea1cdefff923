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
// rounds, W = 4, 2 or 1 consecutive floats per access (the widest that
// divides NR): thread t handles idx = W (t + q NT) + b for round r = W q + b
// (16- or 8-byte loads and stores).  Loads go through registers so that every
// round's load is issued before the first wait; indices past nf are clamped to
// the tile's last floats and their values dropped.  The tile starts 64-byte
// aligned (tile bases are multiples of 16 slots), and nf is a multiple of 16.
template <int NR>
constexpr int tile_vec()
{
    return NR % 4 == 0 ? 4 : NR % 2 == 0 ? 2 : 1;
}

template <int NT, int NR>
__device__ __forceinline__ int tile_idx(int r)
{
    constexpr int W = tile_vec<NR>();
    return W * ((int)threadIdx.x + (r / W) * NT) + (r % W);
}

// LDS word (layout lds_at<IPL>) of the first item of this thread's access
// group q (rounds W q .. W q + W - 1).  The W items of a group share their row
// k and start at a lane l0 that is a multiple of W, so item b lies at
// k 16 + ((l0 + b) ^ x) = (k 16 + (l0 ^ x)) ^ b: one XOR per item instead of
// the row's division by IPL per item.
template <int NT, int NR, int IPL>
__device__ __forceinline__ int tile_lds_group(int q)
{
    constexpr int W = tile_vec<NR>();
    const int idx = W * ((int)threadIdx.x + q * NT);
    return lds_at<IPL>(idx >> 4, idx & (kTile - 1));
}

// LDS word of this thread's item of round r
template <int NT, int NR, int IPL>
__device__ __forceinline__ int tile_lds_word(int r)
{
    constexpr int W = tile_vec<NR>();
    return tile_lds_group<NT, NR, IPL>(r / W) ^ (r % W);
}

template <int W, class T>
struct VecT;
template <class T>
struct VecT<1, T> {
    T v[1];
};
template <class T>
struct alignas(8) VecT<2, T> {
    T v[2];
};
template <class T>
struct alignas(16) VecT<4, T> {
    T v[4];
};

// Element iw (of W items) after the uniform base p, addressed by a 32-bit
// lane offset (tiles hold at most 2^15 items), so that the uniform base stays
// in scalar registers and every array of a round shares one offset.
template <int W, class T>
__device__ __forceinline__ const VecT<W, T>& vec_at(const T* p, int iw)
{
    return *(const VecT<W, T>*)((const char*)p + (uint32_t)iw * (uint32_t)(W * sizeof(T)));
}
template <int W, class T>
__device__ __forceinline__ VecT<W, T>& vec_at(T* p, int iw)
{
    return *(VecT<W, T>*)((char*)p + (uint32_t)iw * (uint32_t)(W * sizeof(T)));
}

template <int NT, int NR, class T>
__device__ __forceinline__ void tile_fetch_t(const T* __restrict__ src, int64_t base, int nf, T (&v)[NR])
{
    static_assert(sizeof(T) == 4, "32-bit items");
    constexpr int W = tile_vec<NR>();
    const T* p = src + base;
    const int nw = nf / W;
#pragma unroll
    for (int q = 0; q < NR / W; ++q) {
        const VecT<W, T> w = vec_at<W>(p, min((int)threadIdx.x + q * NT, nw - 1));
#pragma unroll
        for (int b = 0; b < W; ++b) v[W * q + b] = w.v[b];
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
// mapping of tile_idx, for one destination or (TWO) two sharing each access
// group's branch and LDS words: val(r, word) is round r's value from LDS word
// `word`.
template <int NT, int NR, int IPL, bool TWO, class F1, class F2>
__device__ __forceinline__ void tile_store_t(float* __restrict__ d1, F1 v1, float* __restrict__ d2, F2 v2,
                                             int64_t base, int nf)
{
    constexpr int W = tile_vec<NR>();
    float* p1 = d1 + base;
    float* p2 = d2 + (TWO ? base : 0);
#pragma unroll
    for (int q = 0; q < NR / W; ++q) {
        const int iw = (int)threadIdx.x + q * NT;
        if (W * iw < nf) {
            VecT<W, float> a, b;
            const int g0 = tile_lds_group<NT, NR, IPL>(q);
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const int at = g0 ^ e;
                a.v[e] = v1(W * q + e, at);
                if constexpr (TWO) b.v[e] = v2(W * q + e, at);
            }
            vec_at<W>(p1, iw) = a;
            if constexpr (TWO) vec_at<W>(p2, iw) = b;
        }
    }
}

template <int NT, int NR, int IPL, class F>
__device__ __forceinline__ void tile_store(float* __restrict__ dst, int64_t base, int nf, F val)
{
    tile_store_t<NT, NR, IPL, false>(dst, val, dst, val, base, nf);
}

template <int NT, int NR, int IPL, class F1, class F2>
__device__ __forceinline__ void tile_store2(float* __restrict__ d1, F1 v1, float* __restrict__ d2, F2 v2,
                                            int64_t base, int nf)
{
    tile_store_t<NT, NR, IPL, true>(d1, v1, d2, v2, base, nf);
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
// Every round is written, also past nf: the image holds NT NR words, and its
// words past the tile are never read as data (the rays' steps end inside it).
// No branch, so the rounds' LDS words are computed once for all arrays.
template <int NT, int NR, int IPL, int N>
__device__ __forceinline__ void tile_to_lds(float (&lds)[N], const float (&v)[NR])
{
    static_assert(N >= NT * NR, "the LDS image holds every round");
    constexpr int W = tile_vec<NR>();
#pragma unroll
    for (int q = 0; q < NR / W; ++q) {
        const int g0 = tile_lds_group<NT, NR, IPL>(q);
#pragma unroll
        for (int b = 0; b < W; ++b) lds[g0 ^ b] = v[W * q + b];
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
