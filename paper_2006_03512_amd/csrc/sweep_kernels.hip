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
// difference, so +-inf and large log-odds stay exact.
// Ray phase: one group of lanes per ray, three group scans over the ray:
//   P_i = sum_{k<i} log mu_k(0)                    prefix sum
//   S_i = LSE_{j<i} (log mu_j(1) + g_j + P_j)      prefix log-sum-exp
//   Q_i = LSE(log mu_{i+1}(1) + g_{i+1}, log mu_{i+1}(0) + Q_{i+1})
//                                                  suffix scan of maps
//   ell_i = LSE(S_i, g_i + P_i) - LSE(S_i, P_i + Q_i)
// which is Eq. pos over Eq. neg with the second sum of Eq. neg in its
// division-free form (sum over j > i of the product over k < j, k != i).
#include <hip/hip_runtime.h>

#include "dev_common.hpp"
#include "mrf_internal.hpp"

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
        edge[i] = vox[col[i]];
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
    if (c->E <= 0) return hipSuccess;
    ProfScope ps(c, KID_POT, s);
    hipLaunchKernelGGL(potentials_k, dim3(grid_for(c->E)), dim3(256), 0, s, (const float*)c->b_delta.p,
                       (const uint8_t*)c->b_bin.p, c->E, (const float*)c->b_sigma.p, (float*)c->b_g.p);
    return hipGetLastError();
}

// ------------------------------------------------------------ voxel phase

// One voxel segment [s, s+m) of the voxel->ray CSR held by a group of G lanes,
// IPL striped items per lane.  pre0 / suf0 are the sums of the segment's
// edges before / after this piece (0 unless a hub is split).
template <int G, int IPL>
__device__ __forceinline__ float voxel_segment(int64_t s, int m, const uint32_t* __restrict__ vedge,
                                               const float* __restrict__ in, float* __restrict__ out, float b0,
                                               float pre0, float suf0)
{
    const int l = glane<G>();
    float x[IPL];
    uint32_t e[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = k * G + l;
        e[k] = 0;
        x[k] = 0.0f;
        if (i < m) {
            e[k] = vedge[s + i];
            if (in) x[k] = in[e[k]];
        }
    }
    float pre[IPL];
    float carry = pre0;
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const float incl = gscan_add<G>(x[k]) + carry;
        const float up = gshfl_up<G>(incl, 1);
        pre[k] = l == 0 ? carry : up;
        carry = gbcast<G>(incl, G - 1);
    }
    if (out) {
        float sc = suf0;
#pragma unroll
        for (int k = IPL - 1; k >= 0; --k) {
            const float incl = grscan_add<G>(x[k]) + sc;
            const float dn = gshfl_down<G>(incl, 1);
            const float suf = l == G - 1 ? sc : dn;
            sc = gbcast<G>(incl, 0);
            if (k * G + l < m) out[e[k]] = (b0 + pre[k]) + suf;
        }
    }
    return carry;   // pre0 + sum of this piece
}

template <int G, int IPL>
__global__ __launch_bounds__(256) void voxel_k(const uint32_t* __restrict__ vox, int64_t n,
                                               const int64_t* __restrict__ vptr, const uint32_t* __restrict__ vedge,
                                               const float* __restrict__ base, const float* __restrict__ in,
                                               float* __restrict__ out, float* __restrict__ total, int total_mode)
{
    const int64_t gid = ((int64_t)blockIdx.x * 256 + threadIdx.x) / G;
    if (gid >= n) return;
    const uint32_t v = vox[gid];
    const int64_t s = vptr[v];
    const int m = (int)(vptr[v + 1] - s);
    const float b0 = base ? base[v] : 0.0f;
    const float tot = voxel_segment<G, IPL>(s, m, vedge, in, out, b0, 0.0f, 0.0f);
    if (total_mode && glane<G>() == 0) {
        if (total_mode == 1)
            total[v] = b0 + tot;
        else
            total[v] += tot;
    }
}

// hub pieces: sums, per-hub carries (sequential, fixed order), final pass
__global__ __launch_bounds__(256) void hub_sum_k(HubTables H, const uint32_t* __restrict__ vedge,
                                                 const float* __restrict__ in)
{
    const int64_t p = ((int64_t)blockIdx.x * 256 + threadIdx.x) / 64;
    if (p >= H.n_pieces) return;
    const int l = threadIdx.x & 63;
    const int64_t s = H.piece_start[p];
    const int m = (int)H.piece_len[p];
    float acc = 0.0f;
    for (int i = l; i < m; i += 64) acc += in ? in[vedge[s + i]] : 0.0f;
    acc = greduce_add<64>(acc);
    if (l == 0) H.piece_sum[p] = acc;
}

__global__ void hub_carry_k(HubTables H, const float* __restrict__ base, float* __restrict__ total, int total_mode)
{
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= H.n_hubs) return;
    const uint32_t p0 = H.hub_piece0[h], p1 = H.hub_piece0[h + 1];
    float run = 0.0f;
    for (uint32_t p = p0; p < p1; ++p) {
        H.piece_pre[p] = run;
        run += H.piece_sum[p];
    }
    float suf = 0.0f;
    for (uint32_t p = p1; p-- > p0;) {
        H.piece_suf[p] = suf;
        suf += H.piece_sum[p];
    }
    const uint32_t v = H.hub_voxel[h];
    if (total_mode == 1)
        total[v] = (base ? base[v] : 0.0f) + run;
    else if (total_mode == 2)
        total[v] += run;
}

__global__ __launch_bounds__(256) void hub_piece_k(HubTables H, const uint32_t* __restrict__ vedge,
                                                   const float* __restrict__ base, const float* __restrict__ in,
                                                   float* __restrict__ out)
{
    const int64_t p = ((int64_t)blockIdx.x * 256 + threadIdx.x) / 64;
    if (p >= H.n_pieces) return;
    const uint32_t v = H.piece_voxel[p];
    const float b0 = base ? base[v] : 0.0f;
    voxel_segment<64, kPiece / 64>(H.piece_start[p], (int)H.piece_len[p], vedge, in, out, b0, H.piece_pre[p],
                                   H.piece_suf[p]);
}

template <int G, int IPL>
static void launch_voxel_class(const mrf_ctx* c, int k, const float* base, const float* in, float* out,
                               float* total, int mode, hipStream_t s)
{
    const int64_t n = c->vox_cnt[k];
    if (n <= 0) return;
    ProfScope ps(c, KID_VOX0 + k, s);
    hipLaunchKernelGGL((voxel_k<G, IPL>), dim3(nblk(n, 256 / G)), dim3(256), 0, s,
                       (const uint32_t*)c->b_vox_list[k].p, n, (const int64_t*)c->b_vptr.p,
                       (const uint32_t*)c->b_vedge.p, base, in, out, total, mode);
}

hipError_t launch_voxel_phase(mrf_ctx* c, const float* base, const float* in, float* out, float* total,
                              int total_mode, bool /*plain*/, hipStream_t s)
{
    launch_voxel_class<16, 1>(c, 0, base, in, out, total, total_mode, s);
    launch_voxel_class<64, 1>(c, 1, base, in, out, total, total_mode, s);
    launch_voxel_class<64, 4>(c, 2, base, in, out, total, total_mode, s);
    launch_voxel_class<64, 16>(c, 3, base, in, out, total, total_mode, s);
    const HubTables& H = c->hub;
    if (H.n_pieces > 0) {
        const uint32_t* ve = (const uint32_t*)c->b_vedge.p;
        {
            ProfScope ps(c, KID_HUB_SUM, s);
            hipLaunchKernelGGL(hub_sum_k, dim3(nblk(H.n_pieces, 4)), dim3(256), 0, s, H, ve, in);
        }
        {
            ProfScope ps(c, KID_HUB_CARRY, s);
            hipLaunchKernelGGL(hub_carry_k, dim3(nblk(H.n_hubs, 64)), dim3(64), 0, s, H, base, total, total_mode);
        }
        if (out) {
            ProfScope ps(c, KID_HUB_PIECE, s);
            hipLaunchKernelGGL(hub_piece_k, dim3(nblk(H.n_pieces, 4)), dim3(256), 0, s, H, ve, base, in, out);
        }
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ ray phase

template <int G, int IPL>
__global__ __launch_bounds__(256) void ray_k(const uint32_t* __restrict__ rays, int64_t n,
                                             const int64_t* __restrict__ row_ptr, const float* __restrict__ lam,
                                             const float* __restrict__ g, float* __restrict__ ell)
{
    const int64_t gid = ((int64_t)blockIdx.x * 256 + threadIdx.x) / G;
    if (gid >= n) return;
    const int l = glane<G>();
    const uint32_t r = rays[gid];
    const int64_t s = row_ptr[r];
    const int m = (int)(row_ptr[r + 1] - s);

    float al[IPL], be[IPL], gg[IPL], P[IPL], S[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = k * G + l;
        if (i < m) {
            const float x = lam[s + i];
            const float sp = softplus(x);
            al[k] = -sp;          // log mu(o=0)
            be[k] = x - sp;       // log mu(o=1)
            gg[k] = g[s + i];
        } else {                  // neutral padding
            al[k] = 0.0f;
            be[k] = MRF_NINF;
            gg[k] = 0.0f;
        }
    }
    // P: exclusive prefix sum of log mu(0)
    float cp = 0.0f;
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const float incl = gscan_add<G>(al[k]) + cp;
        const float up = gshfl_up<G>(incl, 1);
        P[k] = l == 0 ? cp : up;
        cp = gbcast<G>(incl, G - 1);
    }
    // S: exclusive prefix LSE of W_j = log mu_j(1) + g_j + P_j
    float cs = MRF_NINF;
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const float incl = lse(cs, gscan_lse<G>(be[k] + gg[k] + P[k]));
        const float up = gshfl_up<G>(incl, 1);
        S[k] = l == 0 ? cs : up;
        cs = gbcast<G>(incl, G - 1);
    }
    // Q: exclusive suffix composition of x -> LSE(c_j, a_j + x), then ell
    LMap cq{0.0f, MRF_NINF};
#pragma unroll
    for (int k = IPL - 1; k >= 0; --k) {
        LMap mp{al[k], be[k] + gg[k]};
        LMap incl = lmap_compose(grscan_lmap<G>(mp), cq);
        const float dn = gshfl_down<G>(incl.c, 1);
        const float Q = l == G - 1 ? cq.c : dn;
        cq.a = gbcast<G>(incl.a, 0);
        cq.c = gbcast<G>(incl.c, 0);
        const int i = k * G + l;
        if (i < m) {
            const float m1 = lse(S[k], gg[k] + P[k]);
            const float m0 = lse(S[k], P[k] + Q);
            ell[s + i] = m1 - m0;
        }
    }
}

template <int G, int IPL>
static void launch_ray_class(const mrf_ctx* c, int k, int64_t off, int64_t n, const float* lam, float* ell,
                             hipStream_t s)
{
    if (n <= 0) return;
    ProfScope ps(c, KID_RAY0 + k, s);
    hipLaunchKernelGGL((ray_k<G, IPL>), dim3(nblk(n, 256 / G)), dim3(256), 0, s,
                       (const uint32_t*)c->b_ray_list[k].p + off, n, (const int64_t*)c->b_rowptr.p, lam,
                       (const float*)c->b_g.p, ell);
}

static void ray_classes(const mrf_ctx* c, const int64_t* off, const int64_t* cnt, const float* lam, float* ell,
                        hipStream_t s)
{
    launch_ray_class<16, 1>(c, 0, off[0], cnt[0], lam, ell, s);
    launch_ray_class<64, 1>(c, 1, off[1], cnt[1], lam, ell, s);
    launch_ray_class<64, 4>(c, 2, off[2], cnt[2], lam, ell, s);
    launch_ray_class<64, 16>(c, 3, off[3], cnt[3], lam, ell, s);
    launch_ray_class<64, 32>(c, 4, off[4], cnt[4], lam, ell, s);
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
