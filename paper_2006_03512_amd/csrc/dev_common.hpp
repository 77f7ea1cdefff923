// Device helpers shared by the gfx950 kernels of libmrf: log-domain
// arithmetic and group-level (16- or 64-lane) scans built on wave shuffles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// log 0 inside the message kernels: a finite -2^100 instead of -inf.  For every
// genuine log-domain value x (|x| far below 2^76; log-odds of 1e9 are already
// extreme) x + MRF_NINF rounds to MRF_NINF and 2^(MRF_NINF - x) is 0, so LSE
// needs no special case for log 0 and every message equals its -inf form (rays
// have at least two voxels; a one-voxel ray would send 2^100 ln 2, not +inf).
#define MRF_NINF (-0x1p100f)

namespace mrf {

// The message kernels work with base-2 logarithms: the hardware's v_exp_f32
// and v_log_f32 compute 2^x and log2 x directly.  Every softmax weight
// exp(x - y) equals 2^(x2 - y2) for the base-2 versions x2 = x log2(e), so only
// inputs and outputs change scale.
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float lg2(float x) { return __builtin_amdgcn_logf(x); }

// log2(2^a + 2^b) for finite a, b (log 0 is MRF_NINF)
__device__ __forceinline__ float lse(float a, float b)
{
    return fmaxf(a, b) + lg2(1.0f + ex2(-fabsf(a - b)));
}

// Softmax weights (2^(a - L), 2^(b - L)) of L = LSE(a, b): with t = 2^-|a-b|
// the larger is 1 / (1 + t) and the smaller t / (1 + t) (no subtraction; two
// transcendental operations where L and two exponentials take four).
__device__ __forceinline__ void lse_weights(float a, float b, float& wa, float& wb)
{
    const float t = ex2(-fabsf(a - b));
    const float big = __builtin_amdgcn_rcpf(1.0f + t);
    const float small = t * big;
    const bool ge = a >= b;
    wa = ge ? big : small;
    wb = ge ? small : big;
}

// LSE(r, x) - LSE(r, y) as (max(r, x) - max(r, y)) + (softplus differences): a
// common dominant r cancels exactly instead of through rounded sums
__device__ __forceinline__ float lse_diff(float r, float x, float y)
{
    const float hx = fmaxf(r, x), hy = fmaxf(r, y);
    return (hx - hy) + (lg2(1.0f + ex2(-fabsf(r - x))) - lg2(1.0f + ex2(-fabsf(r - y))));
}

// log2 sum_j 2^x_j of a lane's items: maximum first, then one exp2 per item
template <int N>
__device__ __forceinline__ float lse_items(const float (&x)[N])
{
    float mx = MRF_NINF;
#pragma unroll
    for (int j = 0; j < N; ++j) mx = fmaxf(mx, x[j]);
    float sm = 0.0f;
#pragma unroll
    for (int j = 0; j < N; ++j) sm += ex2(x[j] - mx);
    return mx + lg2(sm);
}

// x -> LSE(c, a + x): one voxel's step of the suffix recurrence of the second
// sum of Eq. neg.  Identity is (0, log 0).
struct LMap {
    float a, c;
};

// (first o second)(x) = first(second(x))
__device__ __forceinline__ LMap lmap_compose(LMap f, LMap s)
{
    LMap r;
    r.a = f.a + s.a;
    r.c = lse(f.c, f.a + s.c);
    return r;
}

// x -> m x + b in linear arithmetic (adjoint recurrences).  Identity (1, 0).
struct AMap {
    float m, b;
};

// apply `first` then `second`
__device__ __forceinline__ AMap amap_then(AMap first, AMap second)
{
    AMap r;
    r.m = first.m * second.m;
    r.b = second.m * first.b + second.b;
    return r;
}

template <int G>
__device__ __forceinline__ int glane()
{
    return threadIdx.x & (G - 1);
}

template <int G>
__device__ __forceinline__ float gshfl_up(float x, int d)
{
    return __shfl_up(x, d, G);
}

template <int G>
__device__ __forceinline__ float gshfl_down(float x, int d)
{
    return __shfl_down(x, d, G);
}

template <int G>
__device__ __forceinline__ float gbcast(float x, int src)
{
    return __shfl(x, src, G);
}

// ---------------------------------------------------------------- sums
template <int G>
__device__ __forceinline__ float gscan_add(float x)
{
    const int l = glane<G>();
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        float y = gshfl_up<G>(x, d);
        if (l >= d) x = y + x;
    }
    return x;
}

template <int G>
__device__ __forceinline__ float grscan_add(float x)
{
    const int l = glane<G>();
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        float y = gshfl_down<G>(x, d);
        if (l + d < G) x = x + y;
    }
    return x;
}

template <int G>
__device__ __forceinline__ float greduce_add(float x)
{
#pragma unroll
    for (int d = G / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, G);
    return x;
}

// ---------------------------------------------------------------- LSE
template <int G>
__device__ __forceinline__ float gscan_lse(float x)
{
    const int l = glane<G>();
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        float y = gshfl_up<G>(x, d);
        if (l >= d) x = lse(y, x);
    }
    return x;
}

// ---------------------------------------------------------------- maps
template <int G>
__device__ __forceinline__ LMap grscan_lmap(LMap x)
{
    const int l = glane<G>();
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        LMap y;
        y.a = gshfl_down<G>(x.a, d);
        y.c = gshfl_down<G>(x.c, d);
        if (l + d < G) x = lmap_compose(x, y);
    }
    return x;
}

// prefix: element i gets first_0 then ... then first_i
template <int G>
__device__ __forceinline__ AMap gscan_amap(AMap x)
{
    const int l = glane<G>();
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        AMap y;
        y.m = gshfl_up<G>(x.m, d);
        y.b = gshfl_up<G>(x.b, d);
        if (l >= d) x = amap_then(y, x);
    }
    return x;
}

// suffix: element i gets map_{N-1} then ... then map_i
template <int G>
__device__ __forceinline__ AMap grscan_amap(AMap x)
{
    const int l = glane<G>();
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        AMap y;
        y.m = gshfl_down<G>(x.m, d);
        y.b = gshfl_down<G>(x.b, d);
        if (l + d < G) x = amap_then(y, x);
    }
    return x;
}

}  // namespace mrf

// ---------------------------------------------------------------------------
// DPP-based scans over groups of G = 16, 32 or 64 consecutive lanes.  A wave64
// is four rows of 16 lanes; row_shr:n moves data to lane + n inside a row,
// row_shl:n to lane - n, wave_shr:1 / wave_shl:1 move it by one lane across the
// whole wave.  Lanes without a source keep `old`.  Row results are combined
// across the rows of a group through readlane.
// ---------------------------------------------------------------------------
namespace mrf {

enum : int {
    DPP_ROW_SHL1 = 0x101, DPP_ROW_SHL2 = 0x102, DPP_ROW_SHL4 = 0x104, DPP_ROW_SHL8 = 0x108,
    DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118,
    DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138
};

template <int CTRL>
__device__ __forceinline__ float dpp(float old, float src)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                 __builtin_bit_cast(int, src), CTRL, 0xF, 0xF,
                                                                 false));
}

__device__ __forceinline__ float readlane(float x, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}

struct OpAdd {
    __device__ static float id() { return 0.0f; }
    __device__ static float op(float a, float b) { return a + b; }
};
struct OpLse {
    __device__ static float id() { return MRF_NINF; }
    __device__ static float op(float a, float b) { return lse(a, b); }
};

// inclusive prefix: element i gets x_0 op ... op x_i over the group
template <int G, class O>
__device__ __forceinline__ float dscan(float x)
{
    static_assert(G == 16 || G == 32 || G == 64, "groups are rows, half-waves or waves");
    const float I = O::id();
    x = O::op(dpp<DPP_ROW_SHR1>(I, x), x);
    x = O::op(dpp<DPP_ROW_SHR2>(I, x), x);
    x = O::op(dpp<DPP_ROW_SHR4>(I, x), x);
    x = O::op(dpp<DPP_ROW_SHR8>(I, x), x);
    if (G == 32) {
        const float r0 = readlane(x, 15), r2 = readlane(x, 47);
        const int row = (threadIdx.x & 63) >> 4;
        if (row & 1) x = O::op(row == 1 ? r0 : r2, x);
    }
    if (G == 64) {
        const float r0 = readlane(x, 15), r1 = readlane(x, 31), r2 = readlane(x, 47);
        const float c2 = O::op(r0, r1);
        const float c3 = O::op(c2, r2);
        const int row = (threadIdx.x & 63) >> 4;
        const float c = row == 1 ? r0 : (row == 2 ? c2 : c3);
        if (row) x = O::op(c, x);
    }
    return x;
}

// inclusive suffix: element i gets x_i op ... op x_{G-1}
template <int G, class O>
__device__ __forceinline__ float drscan(float x)
{
    static_assert(G == 16 || G == 32 || G == 64, "groups are rows, half-waves or waves");
    const float I = O::id();
    x = O::op(x, dpp<DPP_ROW_SHL1>(I, x));
    x = O::op(x, dpp<DPP_ROW_SHL2>(I, x));
    x = O::op(x, dpp<DPP_ROW_SHL4>(I, x));
    x = O::op(x, dpp<DPP_ROW_SHL8>(I, x));
    if (G == 32) {
        const float t1 = readlane(x, 16), t3 = readlane(x, 48);
        const int row = (threadIdx.x & 63) >> 4;
        if (!(row & 1)) x = O::op(x, row == 0 ? t1 : t3);
    }
    if (G == 64) {
        const float t1 = readlane(x, 16), t2 = readlane(x, 32), t3 = readlane(x, 48);
        const float c1 = O::op(t2, t3);
        const float c0 = O::op(t1, c1);
        const int row = (threadIdx.x & 63) >> 4;
        const float c = row == 2 ? t3 : (row == 1 ? c1 : c0);
        if (row != 3) x = O::op(x, c);
    }
    return x;
}

// exclusive from inclusive: element i gets incl_{i-1}; the first gets `first`
template <int G>
__device__ __forceinline__ float dexcl(float incl, float first)
{
    if (G == 32) {
        const float y = dpp<DPP_WAVE_SHR1>(first, incl);
        return (threadIdx.x & 31) == 0 ? first : y;
    }
    return G == 64 ? dpp<DPP_WAVE_SHR1>(first, incl) : dpp<DPP_ROW_SHR1>(first, incl);
}

// exclusive suffix from inclusive: element i gets incl_{i+1}; the last gets `last`
template <int G>
__device__ __forceinline__ float drexcl(float incl, float last)
{
    if (G == 32) {
        const float y = dpp<DPP_WAVE_SHL1>(last, incl);
        return (threadIdx.x & 31) == 31 ? last : y;
    }
    return G == 64 ? dpp<DPP_WAVE_SHL1>(last, incl) : dpp<DPP_ROW_SHL1>(last, incl);
}

// log-semiring maps x -> LSE(c, a + x): suffix composition (first o second)
__device__ __forceinline__ LMap lmap_id() { return LMap{0.0f, MRF_NINF}; }

template <int CTRL>
__device__ __forceinline__ LMap dpp_lmap(LMap old, LMap src)
{
    return LMap{dpp<CTRL>(old.a, src.a), dpp<CTRL>(old.c, src.c)};
}

__device__ __forceinline__ LMap readlane_lmap(LMap x, int l) { return LMap{readlane(x.a, l), readlane(x.c, l)}; }

// prefix: element i gets map_i o ... o map_0 (maps applied left to right)
template <int G>
__device__ __forceinline__ LMap dscan_lmap(LMap x)
{
    const LMap I = lmap_id();
    x = lmap_compose(x, dpp_lmap<DPP_ROW_SHR1>(I, x));
    x = lmap_compose(x, dpp_lmap<DPP_ROW_SHR2>(I, x));
    x = lmap_compose(x, dpp_lmap<DPP_ROW_SHR4>(I, x));
    x = lmap_compose(x, dpp_lmap<DPP_ROW_SHR8>(I, x));
    if (G == 32) {
        const LMap r0 = readlane_lmap(x, 15), r2 = readlane_lmap(x, 47);
        const int row = (threadIdx.x & 63) >> 4;
        if (row & 1) x = lmap_compose(x, row == 1 ? r0 : r2);
    }
    if (G == 64) {
        const LMap r0 = readlane_lmap(x, 15), r1 = readlane_lmap(x, 31), r2 = readlane_lmap(x, 47);
        const LMap c2 = lmap_compose(r1, r0);
        const LMap c3 = lmap_compose(r2, c2);
        const int row = (threadIdx.x & 63) >> 4;
        const LMap c = row == 1 ? r0 : (row == 2 ? c2 : c3);
        if (row) x = lmap_compose(x, c);
    }
    return x;
}

template <int G>
__device__ __forceinline__ LMap drscan_lmap(LMap x)
{
    const LMap I = lmap_id();
    x = lmap_compose(x, dpp_lmap<DPP_ROW_SHL1>(I, x));
    x = lmap_compose(x, dpp_lmap<DPP_ROW_SHL2>(I, x));
    x = lmap_compose(x, dpp_lmap<DPP_ROW_SHL4>(I, x));
    x = lmap_compose(x, dpp_lmap<DPP_ROW_SHL8>(I, x));
    if (G == 32) {
        const LMap t1 = readlane_lmap(x, 16), t3 = readlane_lmap(x, 48);
        const int row = (threadIdx.x & 63) >> 4;
        if (!(row & 1)) x = lmap_compose(x, row == 0 ? t1 : t3);
    }
    if (G == 64) {
        const LMap t1 = readlane_lmap(x, 16), t2 = readlane_lmap(x, 32), t3 = readlane_lmap(x, 48);
        const LMap c1 = lmap_compose(t2, t3);
        const LMap c0 = lmap_compose(t1, c1);
        const int row = (threadIdx.x & 63) >> 4;
        const LMap c = row == 2 ? t3 : (row == 1 ? c1 : c0);
        if (row != 3) x = lmap_compose(x, c);
    }
    return x;
}

// linear affine maps x -> m x + b
__device__ __forceinline__ AMap amap_id() { return AMap{1.0f, 0.0f}; }

template <int CTRL>
__device__ __forceinline__ AMap dpp_amap(AMap old, AMap src)
{
    return AMap{dpp<CTRL>(old.m, src.m), dpp<CTRL>(old.b, src.b)};
}

__device__ __forceinline__ AMap readlane_amap(AMap x, int l) { return AMap{readlane(x.m, l), readlane(x.b, l)}; }

// prefix: element i gets map_0 then ... then map_i
template <int G>
__device__ __forceinline__ AMap dscan_amap(AMap x)
{
    const AMap I = amap_id();
    x = amap_then(dpp_amap<DPP_ROW_SHR1>(I, x), x);
    x = amap_then(dpp_amap<DPP_ROW_SHR2>(I, x), x);
    x = amap_then(dpp_amap<DPP_ROW_SHR4>(I, x), x);
    x = amap_then(dpp_amap<DPP_ROW_SHR8>(I, x), x);
    if (G == 32) {
        const AMap r0 = readlane_amap(x, 15), r2 = readlane_amap(x, 47);
        const int row = (threadIdx.x & 63) >> 4;
        if (row & 1) x = amap_then(row == 1 ? r0 : r2, x);
    }
    if (G == 64) {
        const AMap r0 = readlane_amap(x, 15), r1 = readlane_amap(x, 31), r2 = readlane_amap(x, 47);
        const AMap c2 = amap_then(r0, r1);
        const AMap c3 = amap_then(c2, r2);
        const int row = (threadIdx.x & 63) >> 4;
        const AMap c = row == 1 ? r0 : (row == 2 ? c2 : c3);
        if (row) x = amap_then(c, x);
    }
    return x;
}

// suffix: element i gets map_{G-1} then ... then map_i
template <int G>
__device__ __forceinline__ AMap drscan_amap(AMap x)
{
    const AMap I = amap_id();
    x = amap_then(dpp_amap<DPP_ROW_SHL1>(I, x), x);
    x = amap_then(dpp_amap<DPP_ROW_SHL2>(I, x), x);
    x = amap_then(dpp_amap<DPP_ROW_SHL4>(I, x), x);
    x = amap_then(dpp_amap<DPP_ROW_SHL8>(I, x), x);
    if (G == 32) {
        const AMap t1 = readlane_amap(x, 16), t3 = readlane_amap(x, 48);
        const int row = (threadIdx.x & 63) >> 4;
        if (!(row & 1)) x = amap_then(row == 0 ? t1 : t3, x);
    }
    if (G == 64) {
        const AMap t1 = readlane_amap(x, 16), t2 = readlane_amap(x, 32), t3 = readlane_amap(x, 48);
        const AMap c1 = amap_then(t3, t2);
        const AMap c0 = amap_then(c1, t1);
        const int row = (threadIdx.x & 63) >> 4;
        const AMap c = row == 2 ? t3 : (row == 1 ? c1 : c0);
        if (row != 3) x = amap_then(c, x);
    }
    return x;
}

// sum over a wave, result in every lane
__device__ __forceinline__ float wave_sum(float x)
{
    x = dscan<64, OpAdd>(x);
    return readlane(x, 63);
}

// ---------------------------------------------------------------- FP64 sums
// The voxel totals are accumulated in FP64: every FP32 term is exact in FP64,
// so a total that nearly cancels against one of its own terms (a voxel whose
// receiving ray sent a message of 1e9 while the others sum to a few units)
// keeps the small remainder.  DPP moves a double as its two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double old, double src)
{
    const uint64_t o = __builtin_bit_cast(uint64_t, old), s = __builtin_bit_cast(uint64_t, src);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)s, CTRL, 0xF, 0xF,
                                                              false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(s >> 32),
                                                              CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double readlane_d(double x, int l)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over each group of G = 8, 16, 32 or 64 consecutive lanes in a fixed
// order (a suffix scan inside each 8- or 16-lane piece of a row, then the rows
// of the group in order), valid at the group's first lane.
template <int G>
__device__ __forceinline__ double dgroup_sum_d(double x)
{
    static_assert(G == 8 || G == 16 || G == 32 || G == 64, "groups are half-rows, rows, half-waves or waves");
    x = x + dpp_d<DPP_ROW_SHL1>(0.0, x);
    x = x + dpp_d<DPP_ROW_SHL2>(0.0, x);
    x = x + dpp_d<DPP_ROW_SHL4>(0.0, x);
    if (G >= 16) x = x + dpp_d<DPP_ROW_SHL8>(0.0, x);
    if (G == 32) {
        const double t1 = readlane_d(x, 16), t3 = readlane_d(x, 48);
        x = x + ((threadIdx.x & 32) ? t3 : t1);   // meaningful at lanes 0 and 32
    }
    if (G == 64) {
        const double t1 = readlane_d(x, 16), t2 = readlane_d(x, 32), t3 = readlane_d(x, 48);
        x = x + (t1 + (t2 + t3));   // meaningful at lane 0
    }
    return x;
}

// sum over a wave in FP64, the same value in every lane
__device__ __forceinline__ double wave_sum_d(double x) { return readlane_d(dgroup_sum_d<64>(x), 0); }

// A double as the unevaluated FP32 pair (hi, lo), hi = fl(x), lo = fl(x - hi):
// x to about 2^-48 of its magnitude.
__device__ __forceinline__ float2 split_pair(double x)
{
    const float hi = (float)x;
    return make_float2(hi, (float)(x - (double)hi));
}

// Block index remapped so that each XCD (blocks are dealt to the 8 XCDs
// round-robin) works on one contiguous range of logical blocks, keeping
// neighbouring work items in the same L2.
__device__ __forceinline__ unsigned xcd_block(unsigned bid, unsigned nb)
{
    const unsigned q = nb >> 3, r = nb & 7, x = bid & 7, i = bid >> 3;
    return x * q + (x < r ? x : r) + i;
}

}  // namespace mrf

// Work item of the ray kernels: a 4x4-pixel tile of rays.  A 256-thread block
// holds 16 rays of 16 lanes (G == 16) or 4 rays of one wave (G == 64, four
// consecutive blocks per tile, kept on one XCD by the block remap).
namespace mrf {

template <int G>
constexpr int tile_blocks()
{
    return 16 * G / 256;
}

// Slot of step 0 and length of this group's ray (and, when frame is not
// null, the tile's frame); false if the group has none.
template <int G, class Tile>
__device__ __forceinline__ bool tile_ray(const uint32_t* __restrict__ list, int64_t ntiles,
                                         const Tile* __restrict__ tiles, const int32_t* __restrict__ counts,
                                         int64_t& s0, int& m, int* frame = nullptr)
{
    constexpr int BPT = tile_blocks<G>();
    constexpr int GPB = 256 / G;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t ti = lb / BPT;
    if (ti >= ntiles) return false;
    const int i = (int)(lb % BPT) * GPB + (int)(threadIdx.x / G);
    const Tile td = tiles[list[ti]];
    const int ux = i & 3, vy = i >> 2;
    if (ux >= td.nu || vy >= td.nv) return false;
    m = counts[td.ray0 + (int64_t)vy * td.W + ux];
    s0 = td.base + i;
    if (frame) *frame = td.frame;
    return m > 0;
}

}  // namespace mrf
