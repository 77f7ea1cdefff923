// Device helpers shared by the gfx950 kernels of libmrf: log-domain
// arithmetic and group-level (16- or 64-lane) scans built on wave shuffles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MRF_NINF (-__builtin_huge_valf())

namespace mrf {

// log(exp(a) + exp(b)); log(0 + 0) = -inf.  Never forms inf - inf.
__device__ __forceinline__ float lse(float a, float b)
{
    const float hi = fmaxf(a, b);
    const float lo = fminf(a, b);
    if (hi == MRF_NINF) return MRF_NINF;
    return hi + __logf(1.0f + __expf(lo - hi));
}

// log(1 + exp(x))
__device__ __forceinline__ float softplus(float x)
{
    return fmaxf(x, 0.0f) + __logf(1.0f + __expf(-fabsf(x)));
}

// x -> LSE(c, a + x): one voxel's step of the suffix recurrence of the second
// sum of Eq. neg.  Identity is (0, -inf).
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
