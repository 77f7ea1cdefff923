// Helpers shared by the ray-phase and reverse-pass kernels that stage a tile
// of 16 rays (step-major, 16 floats per step) through LDS.
#pragma once

#include <hip/hip_runtime.h>

#include "dev_common.hpp"
#include "mrf_internal.hpp"

namespace mrf {

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

// steps of tile lane i (0 for pixels outside the image)
__device__ __forceinline__ int tile_ray_len(const TileDev& td, const int32_t* __restrict__ counts, int i)
{
    const int ux = i & (kTileW - 1), vy = i / kTileW;
    return (ux < td.nu && vy < td.nv) ? counts[td.ray0 + (int64_t)vy * td.W + ux] : 0;
}

// base-2 log mu(0), log mu(1) and g of one step from lambda and g (natural
// log); neutral padding (0, -inf, 0) when the step is past the ray
__device__ __forceinline__ void load_step(float lam, float g, bool ok, float& al, float& be, float& gg)
{
    if (ok) {
        const float x = lam * kLog2e;
        const float sp = softplus(x);
        al = -sp;
        be = x - sp;
        gg = g * kLog2e;
    } else {
        al = 0.0f;
        be = MRF_NINF;
        gg = 0.0f;
    }
}

}  // namespace mrf
