// Reverse-mode derivative of the unrolled sweeps on gfx950 (a project
// extension; the paper's BP has no gradients).
//
// Ray adjoint: for one ray, given d/d ell_i, the chain rule through the
// P-free form of the ray phase (c_i = log mu_i(1) + g_i)
//   ell_i = M1_i - M0_i,  M1_i = LSE(R_i, g_i),  M0_i = LSE(R_i, Q_i),
//   R_{i+1} = U_i - log mu_i(0),  U_i = LSE(R_i, c_i),
//   Q_{i-1} = LSE(c_i, log mu_i(0) + Q_i)
// gives two linear recurrences with weights in [0, 1] (softmax weights of
// the LSEs), run as affine group scans:
//   Tb_i = Qbar_i + rho_i Tb_{i-1}      left to right,  rho_i = 2^(log mu_i(0) + Q_i - Q_{i-1})
//   Rb_i = Rbar_i + r_i Rb_{i+1}        right to left,  r_i = 2^(R_i - U_i)
// where Tb and Rb are the total derivatives with respect to Q_i and R_i.
// d log mu(0)/d lam = -mu(1), d log mu(1)/d lam = mu(0).
//
// Sigma-table gradient: d g_e / d sigma_b = delta_e^2 / sigma_b^3 - 1 / sigma_b,
// reduced per bin deterministically: fixed-order double sums over runs of
// equal bins within each lane's 16 consecutive slots, then 128-bit fixed-point
// integer accumulation (order-independent, hence bit-reproducible).
#include <hip/hip_runtime.h>

#include <array>
#include <utility>

#include "dev_common.hpp"
#include "mrf_internal.hpp"
#include "tile_lds.hpp"

namespace mrf {

static inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Reverse pass of one ray, blocked like the forward ray kernel: lane l holds
// steps [i0, i0 + IPL) with i0 = l IPL; al / be / gg are base-2 log mu(0),
// log mu(1) and g of those steps (neutral padding beyond m), eb the incoming
// d/d ell.  Outputs d/d lambda and d/d g per step.  Every recurrence runs
// sequentially inside the lane after one group scan of the lane aggregates.
template <int G, int IPL>
__device__ __forceinline__ void ray_adj_body(const float (&al)[IPL], const float (&be)[IPL], const float (&gg)[IPL],
                                             const float (&eb)[IPL], int m, int i0, float (&lamb)[IPL],
                                             float (&gb)[IPL])
{
    float c[IPL], R[IPL], U[IPL], Q[IPL];
    // ---- forward recomputation (as in the ray phase)
    {
        float cw[IPL];
        float a = 0.0f;
#pragma unroll
        for (int j = 0; j < IPL; ++j) {
            c[j] = be[j] + gg[j];
            cw[j] = c[j] + a;
            a += al[j];
        }
        const float Cl = lse_items<IPL>(cw);
        const LMap left = dscan_lmap<G>(LMap{-a, Cl - a});
        float r = dexcl<G>(left.c, MRF_NINF);
#pragma unroll
        for (int j = 0; j < IPL; ++j) {
            R[j] = r;
            U[j] = lse(r, c[j]);
            r = U[j] - al[j];
        }
        const LMap right = drscan_lmap<G>(LMap{a, Cl});
        float q = drexcl<G>(right.c, MRF_NINF);
#pragma unroll
        for (int j = IPL - 1; j >= 0; --j) {
            Q[j] = q;
            q = lse(c[j], al[j] + q);
        }
    }
    // ---- direct partials of ell_i = M1_i - M0_i: the softmax weights of the
    // two LSEs (M1 and M0 themselves are not needed)
    float Fd[IPL], Bb[IPL], lab[IPL], lbb[IPL];
#pragma unroll
    for (int j = 0; j < IPL; ++j) {   // weights are finite, so e = 0 past the ray zeroes all three
        const float e = i0 + j < m ? eb[j] : 0.0f;
        float wr1, wg1, wr0, wq0;
        lse_weights(R[j], gg[j], wr1, wg1);
        lse_weights(R[j], Q[j], wr0, wq0);
        Fd[j] = e * (wr1 - wr0);
        gb[j] = e * wg1;
        Bb[j] = -e * wq0;
        lab[j] = 0.0f;
        lbb[j] = 0.0f;
    }
    // ---- Q adjoint: Tb_i = Bb_i + rho_i Tb_{i-1} (left to right)
    {
        const float qlast_prev_lane = dexcl<G>(Q[IPL - 1], MRF_NINF);
        float rho[IPL], kap[IPL];
        AMap lm = amap_id();
#pragma unroll
        for (int j = 0; j < IPL; ++j) {
            const int i = i0 + j;
            const float qprev = j == 0 ? qlast_prev_lane : Q[j - 1];   // Q_{i-1}
            const bool v = i >= 1 && i < m;
            rho[j] = v ? ex2(al[j] + Q[j] - qprev) : 0.0f;
            kap[j] = v ? ex2(c[j] - qprev) : 0.0f;
            lm = amap_then(lm, AMap{rho[j], Bb[j]});
        }
        const AMap incl = dscan_amap<G>(lm);
        float tb = dexcl<G>(incl.b, 0.0f);   // Tb_{i0-1}: every earlier lane's maps applied to 0
#pragma unroll
        for (int j = 0; j < IPL; ++j) {   // rho = kap = 0 outside [1, m): no branch needed
            const float tk = tb * kap[j];
            lbb[j] += tk;
            gb[j] += tk;
            lab[j] += tb * rho[j];
            tb = rho[j] * tb + Bb[j];
        }
    }
    // ---- R adjoint: Rb_i = Fd_i + r_i Rb_{i+1} (right to left); R_{i+1}
    // depends on c_i with weight w_i = 2^(c_i - U_i) and on log mu_i(0) with -1
    {
        float rr[IPL], ww[IPL];
        AMap lm = amap_id();
#pragma unroll
        for (int j = IPL - 1; j >= 0; --j) {
            rr[j] = ex2(R[j] - U[j]);
            ww[j] = ex2(c[j] - U[j]);
            lm = amap_then(lm, AMap{rr[j], Fd[j]});
        }
        const AMap incl = drscan_amap<G>(lm);
        float fb = drexcl<G>(incl.b, 0.0f);   // Rb_{i0+IPL}; 0 past the ray (R_m feeds nothing)
#pragma unroll
        for (int j = IPL - 1; j >= 0; --j) {
            const float wb = fb * ww[j];
            lbb[j] += wb;
            gb[j] += wb;
            lab[j] -= fb;
            fb = rr[j] * fb + Fd[j];
        }
    }
#pragma unroll
    for (int j = 0; j < IPL; ++j)   // d log mu(0)/d lam = -mu(1), d log mu(1)/d lam = mu(0)
        lamb[j] = -ex2(be[j]) * lab[j] + ex2(al[j]) * lbb[j];
}

// Inputs of both reverse-pass kernels per edge: lambda_e = lam.tot[col_e] -
// lam.own_e (the forward messages of the sweep) and d/d ell_e = eb.tot[col_e] -
// eb.own_e (the later sweep's d/d lambda summed over the voxel, less the
// edge's own: the adjoint of the forward's total-minus-own).
// With KF (per-keyframe averaged messages) lambda_e and d/d ell_e come from
// the keyframe buffers of kfa instead (AdjKf).
template <int G, int IPL, bool KF>
__global__ __launch_bounds__(256) void ray_adj_k(const uint32_t* __restrict__ list, int64_t ntiles,
                                                 const TileDev* __restrict__ tiles, const int32_t* __restrict__ counts,
                                                 const int32_t* __restrict__ col, ExclDev lam,
                                                 const float* __restrict__ g, ExclDev eb, AdjKf kfa,
                                                 float* __restrict__ lambar, float* __restrict__ gsum, int first)
{
    static_assert(G == 64 || IPL == 1, "16-lane groups hold a whole ray");
    int64_t s;
    int m, frame = 0;
    if (!tile_ray<G>(list, ntiles, tiles, counts, s, m, &frame)) return;
    const int i0 = (int)(threadIdx.x & (G - 1)) * IPL;
    int32_t cv[IPL];
    float lo[IPL], eo[IPL], gv[IPL], lv[IPL], ev[IPL];
    float2 lt[IPL], et[IPL];
#pragma unroll
    for (int j = 0; j < IPL; ++j) {   // indices clamped to the ray (m >= 1): loads issued before any wait
        const int64_t at = s + kTile * (int64_t)min(i0 + j, m - 1);
        cv[j] = col[at];
        if constexpr (KF) {
            eo[j] = kfa.w[at];
        } else {
            lo[j] = lam.own[at];
            eo[j] = eb.own[at];
        }
        gv[j] = g[at];
    }
    if constexpr (KF) {
        const int64_t xb = kfa.x.xb[frame];
#pragma unroll
        for (int j = 0; j < IPL; ++j) {
            lv[j] = cv[j] >= 0 ? kfa.x.x[xb + cv[j]] : 0.0f;
            ev[j] = cv[j] >= 0 ? eo[j] * kfa.y[xb + cv[j]] : 0.0f;
        }
    } else {
#pragma unroll
        for (int j = 0; j < IPL; ++j) {
            const int cc = max(cv[j], 0);
            lt[j] = lam.tot[cc];
            et[j] = eb.tot[cc];
        }
#pragma unroll
        for (int j = 0; j < IPL; ++j) {
            lv[j] = excl_value(cv[j], lt[j], lo[j], lam.has_own);
            ev[j] = excl_value(cv[j], et[j], eo[j], eb.has_own);
        }
    }
    float al[IPL], be[IPL], gg[IPL], ebar[IPL], lamb[IPL], gb[IPL];
#pragma unroll
    for (int j = 0; j < IPL; ++j) {
        const bool ok = i0 + j < m;
        load_step(lv[j], gv[j], ok, al[j], be[j], gg[j]);
        ebar[j] = ok ? ev[j] : 0.0f;
    }
    ray_adj_body<G, IPL>(al, be, gg, ebar, m, i0, lamb, gb);
#pragma unroll
    for (int j = 0; j < IPL; ++j) {
        const int i = i0 + j;
        if (i < m) {
            const int64_t at = s + kTile * i;
            lambar[at] = lamb[j];
            gsum[at] = first ? gb[j] : gsum[at] + gb[j];
        }
    }
}

// Tile-staged reverse pass for tiles of at most G*IPL steps: one block of
// 16 / RPW groups per tile, each group walking RPW rays in turn.  The block
// reads col, the two own terms and g with coalesced loads, gathers both voxel
// totals, and stages lambda, g and ell-bar through LDS (RPW == 1 stages
// ell-bar after the groups have read their lambda, which saves a third LDS
// array); each group writes lambda-bar and g-bar into its rays' columns (zeros
// past the ray), and the block stores lambda-bar and accumulates the g-bar sum
// coalesced.
template <int G, int IPL, int RPW, bool KF>
__global__ __launch_bounds__(kTile * G / RPW) void ray_adj_lds_k(const uint32_t* __restrict__ list, int64_t ntiles,
                                                                 const TileDev* __restrict__ tiles,
                                                                 const int32_t* __restrict__ counts,
                                                                 const int32_t* __restrict__ col, ExclDev lam,
                                                                 const float* __restrict__ g, ExclDev eb, AdjKf kfa,
                                                                 float* __restrict__ lambar, float* __restrict__ gsum,
                                                                 int first)
{
    constexpr int NT = kTile * G / RPW;   // threads
    constexpr int NG = kTile / RPW;       // groups
    constexpr int NR = IPL * RPW;         // staging rounds per thread
    constexpr int CAP = G * IPL;
    __shared__ float sa[kTile * CAP];
    __shared__ float sb[kTile * CAP];
    __shared__ float se[RPW > 1 ? kTile * CAP : 1];
    const int64_t ti = xcd_block(blockIdx.x, gridDim.x);
    if (ti >= ntiles) return;   // whole block
    const TileDev td = tiles[list[ti]];
    const int nf = kTile * td.len;   // 1 <= td.len <= G * IPL by class
    const int grp = (int)threadIdx.x / G;
    const int gl = (int)threadIdx.x % G;
    const int i0 = gl * IPL;
    int mr[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) mr[r] = tile_ray_len(td, counts, grp + r * NG);
    float ve[NR];   // ell-bar
    {
        int32_t vc[NR];
        float vo[NR], vb[NR], vg[NR], vt[NR];
        float2 pt[NR], pe[NR];
        tile_fetch_i<NT, NR>(col, td.base, nf, vc);
        if constexpr (KF) {
            tile_fetch<NT, NR>(kfa.w, td.base, nf, vb);
        } else {
            tile_fetch<NT, NR>(lam.own, td.base, nf, vo);
            tile_fetch<NT, NR>(eb.own, td.base, nf, vb);
        }
        tile_fetch<NT, NR>(g, td.base, nf, vg);
        if constexpr (KF) {
            const int64_t xb = kfa.x.xb[td.frame];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                vt[r] = vc[r] >= 0 ? kfa.x.x[xb + vc[r]] : 0.0f;
                ve[r] = vc[r] >= 0 ? vb[r] * kfa.y[xb + vc[r]] : 0.0f;
            }
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int cc = max(vc[r], 0);
                pt[r] = lam.tot[cc];
                pe[r] = eb.tot[cc];
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                vt[r] = excl_value(vc[r], pt[r], vo[r], lam.has_own);
                ve[r] = excl_value(vc[r], pe[r], vb[r], eb.has_own);
            }
        }
        tile_to_lds<NT, NR, IPL>(sa, vt);
        tile_to_lds<NT, NR, IPL>(sb, vg);
        if constexpr (RPW > 1) tile_to_lds<NT, NR, IPL>(se, ve);
    }
    __syncthreads();
    // g-bar sums of earlier sweeps, fetched before the scans so that their
    // latency hides behind them (unconditionally: a branch here would make
    // the compiler wait for the loads at its end; unused on the first sweep)
    float vs[NR];
    tile_fetch<NT, NR>(gsum, td.base, nf, vs);
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int i = grp + r * NG;   // this group's ray: lane i of the tile
        const int m = mr[r];
        const int cb = lds_col(i0, gl, i);
        float al[IPL], be[IPL], gg[IPL], ebar[IPL], lamb[IPL], gb[IPL];
#pragma unroll
        for (int j = 0; j < IPL; ++j)   // column rows are inside the LDS tile even past the ray
            load_step(sa[cb + kTile * j], sb[cb + kTile * j], i0 + j < m, al[j], be[j], gg[j]);
        if constexpr (RPW == 1) {
            __syncthreads();   // every group has its lambda: reuse sa for ell-bar
            tile_to_lds<NT, NR, IPL>(sa, ve);
            __syncthreads();
        }
        const float* sev = RPW > 1 ? se : sa;
#pragma unroll
        for (int j = 0; j < IPL; ++j) {
            const float v = sev[cb + kTile * j];
            ebar[j] = i0 + j < m ? v : 0.0f;
        }
        if (__ballot(m > 0)) {   // skip waves whose rays are all empty; empty rays give zeros
            ray_adj_body<G, IPL>(al, be, gg, ebar, m, i0, lamb, gb);
        } else {
#pragma unroll
            for (int j = 0; j < IPL; ++j) lamb[j] = gb[j] = 0.0f;
        }
#pragma unroll
        for (int j = 0; j < IPL; ++j) {   // own column only; zeros past the ray
            const bool ok = i0 + j < m;
            sa[cb + kTile * j] = ok ? lamb[j] : 0.0f;
            sb[cb + kTile * j] = ok ? gb[j] : 0.0f;
        }
    }
    __syncthreads();
    tile_store2<NT, NR, IPL>(
        lambar, [&](int, int at) { return sa[at]; }, gsum,
        [&](int r, int at) { return first ? sb[at] : vs[r] + sb[at]; }, td.base, nf);
}

// The reverse pass's per-edge inputs: the voxel totals less the own terms, or
// (is_kf) the keyframe buffers.
struct AdjSrc {
    ExclDev lam, eb;
    AdjKf kf;
    bool is_kf;
};

template <int Q, int I, bool KF>
static void launch_adj_shape_t(const mrf_ctx* c, const AdjSrc& a, float* lambar, float* gsum, int first,
                               hipStream_t s)
{
    constexpr int G = kAdjShapes[Q][I].g;
    if constexpr (G != 0) {
        constexpr int CAP = kRayCap[Q];
        const int64_t n = c->ray_cnt[Q];
        const uint32_t* list = (const uint32_t*)c->b_ray_list[Q].p;
        if constexpr (ray_class_lds(Q)) {
            constexpr int RPW = kAdjShapes[Q][I].rpw;
            hipLaunchKernelGGL((ray_adj_lds_k<G, CAP / G, RPW, KF>), dim3((unsigned)n), dim3(kTile * G / RPW), 0, s,
                               list, n, (const TileDev*)c->b_tiles.p, (const int32_t*)c->b_counts.p,
                               (const int32_t*)c->b_col.p, a.lam, (const float*)c->b_g.p, a.eb, a.kf, lambar, gsum,
                               first);
        } else {
            hipLaunchKernelGGL((ray_adj_k<G, CAP / G, KF>), dim3((unsigned)(n * tile_blocks<G>())), dim3(256), 0, s,
                               list, n, (const TileDev*)c->b_tiles.p, (const int32_t*)c->b_counts.p,
                               (const int32_t*)c->b_col.p, a.lam, (const float*)c->b_g.p, a.eb, a.kf, lambar, gsum,
                               first);
        }
    }
}

template <int Q, int I>
static void launch_adj_shape(const mrf_ctx* c, const AdjSrc& a, float* lambar, float* gsum, int first, hipStream_t s)
{
    if (a.is_kf)
        launch_adj_shape_t<Q, I, true>(c, a, lambar, gsum, first, s);
    else
        launch_adj_shape_t<Q, I, false>(c, a, lambar, gsum, first, s);
}

template <int Q, int... I>
static void launch_adj_sel(int sel, const mrf_ctx* c, const AdjSrc& a, float* lambar, float* gsum, int first,
                           hipStream_t s, std::integer_sequence<int, I...>)
{
    ((sel == I ? launch_adj_shape<Q, I>(c, a, lambar, gsum, first, s) : void()), ...);
}

template <int Q>
static void launch_adj_class(const mrf_ctx* c, int sel, const AdjSrc& a, float* lambar, float* gsum, int first,
                             hipStream_t s)
{
    if (c->ray_cnt[Q] <= 0) return;
    ProfScope ps(c, KID_ADJ0 + Q, s);
    launch_adj_sel<Q>(sel, c, a, lambar, gsum, first, s, std::make_integer_sequence<int, kNShapes>{});
}

template <int... Q>
static void adj_classes(std::integer_sequence<int, Q...>, const mrf_ctx* c, const AdjSrc& a, float* lambar,
                        float* gsum, int first, hipStream_t s)
{
    (launch_adj_class<Q>(c, c->adj_sel[Q], a, lambar, gsum, first, s), ...);
}

hipError_t launch_ray_adjoint(mrf_ctx* c, ExclSrc lam, ExclSrc ellbar, float* lambar, float* gsum, bool first,
                              hipStream_t s)
{
    const AdjSrc a{excl_dev(c, lam), excl_dev(c, ellbar), AdjKf{KfSrc{nullptr, nullptr}, nullptr, nullptr}, false};
    adj_classes(std::make_integer_sequence<int, kRayClasses>{}, c, a, lambar, gsum, first ? 1 : 0, s);
    return hipGetLastError();
}

hipError_t launch_ray_adjoint_kf(mrf_ctx* c, AdjKf kf, float* lambar, float* gsum, bool first, hipStream_t s)
{
    // the exact-scheme sources are unused; any readable arrays stand in
    const ExclDev none{(const float2*)c->b_theta2.p, (const float*)c->b_g.p, 0};
    const AdjSrc a{none, none, kf, true};
    adj_classes(std::make_integer_sequence<int, kRayClasses>{}, c, a, lambar, gsum, first ? 1 : 0, s);
    return hipGetLastError();
}

using AdjClassFn = void (*)(const mrf_ctx*, int, const AdjSrc&, float*, float*, int, hipStream_t);
template <int... Q>
static constexpr std::array<AdjClassFn, kRayClasses> adj_class_fns(std::integer_sequence<int, Q...>)
{
    return {&launch_adj_class<Q>...};
}

hipError_t launch_adj_class_shape(const mrf_ctx* c, int q, int sel, ExclSrc lam, ExclSrc ellbar, float* lambar,
                                  float* gsum, int first, hipStream_t s)
{
    static constexpr std::array<AdjClassFn, kRayClasses> fns =
        adj_class_fns(std::make_integer_sequence<int, kRayClasses>{});
    if (q < 0 || q >= kRayClasses || sel < 0 || sel >= ray_shape_count(q, true)) return hipErrorInvalidValue;
    const AdjSrc a{excl_dev(c, lam), excl_dev(c, ellbar), AdjKf{KfSrc{nullptr, nullptr}, nullptr, nullptr}, false};
    fns[q](c, sel, a, lambar, gsum, first, s);
    return hipGetLastError();
}

// ------------------------------------------------------------ sigma table

constexpr int SG_BLOCKS = 4096;   // blocks of the sigma-table reduction (at most)

__device__ __forceinline__ void fx_add(unsigned long long* lo, long long* hi, double v)
{
    // v as a signed 128-bit fixed-point number with 64 fractional bits
    double fl = floor(v);
    double fr = v - fl;   // in [0, 1] and exact, but it rounds to 1 for -2^-53 < v < 0
    if (fr >= 1.0) {      // such a v is -0 in 64 fractional bits as well
        fr = 0.0;
        fl += 1.0;
    }
    const unsigned long long l = (unsigned long long)(fr * 18446744073709551616.0);
    const long long h = (long long)fl;
    const unsigned long long old = atomicAdd(lo, l);
    const long long carry = (old + l < old) ? 1 : 0;
    atomicAdd((unsigned long long*)hi, (unsigned long long)(h + carry));
}

// d loss / d sigma_b and, with BIAS, d loss / d mu_b: sums over the slots of
// bin b of gbar_e times d g / d sigma = r^2 / sigma^3 - 1 / sigma and
// d g / d mu = r / sigma^2, r = delta_e - mu_b the residual about the
// predicted mean.  Every lane sums runs of equal bins over 16 consecutive slots
// in slot order (double), and adds each run's sum to its bin in LDS as a
// 128-bit fixed-point integer; each block then adds its 64 bins to the global
// accumulators.  The partition of slots into lanes is fixed and integer sums
// do not depend on order, so the result is bit-reproducible.  S is a multiple
// of 16 (16 slots per tile step), so a lane's 16 slots are three 16-byte
// vector loads.
template <bool BIAS>
__global__ __launch_bounds__(256) void sigma_grad_k(const float* __restrict__ gsum, const float* __restrict__ delta,
                                                    const uint8_t* __restrict__ bin, int64_t S,
                                                    const float* __restrict__ sigma, const float* __restrict__ bias,
                                                    unsigned long long* __restrict__ glo, long long* __restrict__ ghi)
{
    constexpr int NT = BIAS ? 2 : 1;   // accumulated tables: sigma, then bias
    __shared__ unsigned long long slo[NT * kBins];
    __shared__ long long shi[NT * kBins];
    __shared__ double inv[kBins], inv2[kBins], inv3[kBins], mu[kBins];
    if (threadIdx.x < kBins) {
        for (int t = 0; t < NT; ++t) {
            slo[t * kBins + threadIdx.x] = 0;
            shi[t * kBins + threadIdx.x] = 0;
        }
        const double sg = (double)sigma[threadIdx.x];
        inv[threadIdx.x] = 1.0 / sg;
        inv2[threadIdx.x] = 1.0 / (sg * sg);
        inv3[threadIdx.x] = 1.0 / (sg * sg * sg);
        mu[threadIdx.x] = (double)bias[threadIdx.x];
    }
    __syncthreads();
    const int64_t nch = S / 16;
    for (int64_t ch = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ch < nch;
         ch += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e0 = ch * 16;
        float4 gv[4], dv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            gv[q] = *(const float4*)(gsum + e0 + 4 * q);
            dv[q] = *(const float4*)(delta + e0 + 4 * q);
        }
        const uint4 bw = *(const uint4*)(bin + e0);
        const uint32_t bwords[4] = {bw.x, bw.y, bw.z, bw.w};
        int cur = -1;
        double acc = 0.0, accb = 0.0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int b = (int)((bwords[j >> 2] >> (8 * (j & 3))) & 255u);
            const float4 g4 = gv[j >> 2], d4 = dv[j >> 2];
            const float gj = (j & 3) == 0 ? g4.x : (j & 3) == 1 ? g4.y : (j & 3) == 2 ? g4.z : g4.w;
            const float dj = (j & 3) == 0 ? d4.x : (j & 3) == 1 ? d4.y : (j & 3) == 2 ? d4.z : d4.w;
            if (b >= kBins) continue;   // padding slots carry bin 255
            if (b != cur) {
                if (cur >= 0) {
                    fx_add(&slo[cur], &shi[cur], acc);
                    if (BIAS) fx_add(&slo[kBins + cur], &shi[kBins + cur], accb);
                }
                cur = b;
                acc = 0.0;
                accb = 0.0;
            }
            const double r = (double)dj - mu[b];
            acc += (double)gj * (r * r * inv3[b] - inv[b]);
            if (BIAS) accb += (double)gj * (r * inv2[b]);
        }
        if (cur >= 0) {
            fx_add(&slo[cur], &shi[cur], acc);
            if (BIAS) fx_add(&slo[kBins + cur], &shi[kBins + cur], accb);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NT * kBins; i += blockDim.x) {
        const unsigned long long l = slo[i];
        const long long h = shi[i];
        const unsigned long long old = atomicAdd(&glo[i], l);
        const long long carry = (old + l < old) ? 1 : 0;
        atomicAdd((unsigned long long*)&ghi[i], (unsigned long long)(h + carry));
    }
}

// sigma_grad_k with per-region tables: one block per tile (grid-stride).  The
// tile's 16-slot steps are the same lane partition as sigma_grad_k's, summed
// the same way into LDS accumulators of the tile's region row, which the block
// then adds (entries it touched) to the row's global accumulators; integer
// sums, so the result is bit-reproducible and, when every region holds the
// same table, the regions' accumulators add up exactly to sigma_grad_k's.
template <bool BIAS>
__global__ __launch_bounds__(256) void sigma_grad_cells_k(const TileDev* __restrict__ tiles, int64_t T,
                                                          const FrameDev* __restrict__ frames, int cp,
                                                          int64_t n_ent, const float* __restrict__ gsum,
                                                          const float* __restrict__ delta,
                                                          const uint8_t* __restrict__ bin,
                                                          const float* __restrict__ sigma,
                                                          const float* __restrict__ bias,
                                                          unsigned long long* __restrict__ glo,
                                                          long long* __restrict__ ghi)
{
    constexpr int NT = BIAS ? 2 : 1;
    __shared__ unsigned long long slo[NT * kBins];
    __shared__ long long shi[NT * kBins];
    __shared__ double inv[kBins], inv2[kBins], inv3[kBins], mu[kBins];
    for (int64_t ti = blockIdx.x; ti < T; ti += gridDim.x) {
        const TileDev t = tiles[ti];
        const int64_t row = tile_cell(t, frames, cp) * kBins;
        __syncthreads();   // the previous tile's flush is done
        if (threadIdx.x < kBins) {
            for (int q = 0; q < NT; ++q) {
                slo[q * kBins + threadIdx.x] = 0;
                shi[q * kBins + threadIdx.x] = 0;
            }
            const double sg = (double)sigma[row + threadIdx.x];
            inv[threadIdx.x] = 1.0 / sg;
            inv2[threadIdx.x] = 1.0 / (sg * sg);
            inv3[threadIdx.x] = 1.0 / (sg * sg * sg);
            mu[threadIdx.x] = (double)bias[row + threadIdx.x];
        }
        __syncthreads();
        for (int ch = threadIdx.x; ch < t.len; ch += blockDim.x) {
            const int64_t e0 = t.base + 16 * (int64_t)ch;
            float4 gv[4], dv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                gv[q] = *(const float4*)(gsum + e0 + 4 * q);
                dv[q] = *(const float4*)(delta + e0 + 4 * q);
            }
            const uint4 bw = *(const uint4*)(bin + e0);
            const uint32_t bwords[4] = {bw.x, bw.y, bw.z, bw.w};
            int cur = -1;
            double acc = 0.0, accb = 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int b = (int)((bwords[j >> 2] >> (8 * (j & 3))) & 255u);
                const float4 g4 = gv[j >> 2], d4 = dv[j >> 2];
                const float gj = (j & 3) == 0 ? g4.x : (j & 3) == 1 ? g4.y : (j & 3) == 2 ? g4.z : g4.w;
                const float dj = (j & 3) == 0 ? d4.x : (j & 3) == 1 ? d4.y : (j & 3) == 2 ? d4.z : d4.w;
                if (b >= kBins) continue;
                if (b != cur) {
                    if (cur >= 0) {
                        fx_add(&slo[cur], &shi[cur], acc);
                        if (BIAS) fx_add(&slo[kBins + cur], &shi[kBins + cur], accb);
                    }
                    cur = b;
                    acc = 0.0;
                    accb = 0.0;
                }
                const double r = (double)dj - mu[b];
                acc += (double)gj * (r * r * inv3[b] - inv[b]);
                if (BIAS) accb += (double)gj * (r * inv2[b]);
            }
            if (cur >= 0) {
                fx_add(&slo[cur], &shi[cur], acc);
                if (BIAS) fx_add(&slo[kBins + cur], &shi[kBins + cur], accb);
            }
        }
        __syncthreads();
        if (threadIdx.x < NT * kBins) {
            const unsigned long long l = slo[threadIdx.x];
            const long long h = shi[threadIdx.x];
            if (l != 0 || h != 0) {
                const int64_t at = (threadIdx.x / kBins) * n_ent + row + (threadIdx.x % kBins);
                const unsigned long long old = atomicAdd(&glo[at], l);
                const long long carry = (old + l < old) ? 1 : 0;
                atomicAdd((unsigned long long*)&ghi[at], (unsigned long long)(h + carry));
            }
        }
    }
}

// accumulators of the sigma and bias tables (n entries each): glo[2 n] then ghi[2 n]
__global__ void sigma_zero_k(unsigned long long* glo, long long* ghi, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * n; i += (int64_t)gridDim.x * blockDim.x) {
        glo[i] = 0;
        ghi[i] = 0;
    }
}

__global__ void sigma_final_k(const unsigned long long* glo, const long long* ghi, int64_t n, float* out,
                              float* out_bias)
{
    const auto fx = [&](int64_t k) { return (float)((double)ghi[k] + (double)glo[k] * 5.421010862427522e-20); };
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (out) out[i] = fx(i);
        if (out_bias) out_bias[i] = fx(n + i);
    }
}

hipError_t launch_sigma_grad(mrf_ctx* c, float* dsigma, float* dbias, hipStream_t s)
{
    const int64_t n = table_entries(c);
    unsigned long long* glo = (unsigned long long*)c->b_sigpart.p;
    long long* ghi = (long long*)(glo + 2 * n);
    const unsigned nb = (unsigned)((2 * n + 255) / 256 < 1024 ? (2 * n + 255) / 256 : 1024);
    hipLaunchKernelGGL(sigma_zero_k, dim3(nb), dim3(256), 0, s, glo, ghi, n);
    if (c->S > 0 && c->cell_px > 0) {
        ProfScope ps(c, KID_SIGMA, s);
        const int64_t blocks = c->T < 65536 ? c->T : 65536;
        if (dbias)
            hipLaunchKernelGGL(sigma_grad_cells_k<true>, dim3((unsigned)blocks), dim3(256), 0, s,
                               (const TileDev*)c->b_tiles.p, c->T, (const FrameDev*)c->b_frames.p, c->cell_px, n,
                               (const float*)c->b_gsum.p, (const float*)c->b_delta.p, (const uint8_t*)c->b_bin.p,
                               (const float*)c->b_sigma.p, (const float*)c->b_bias.p, glo, ghi);
        else
            hipLaunchKernelGGL(sigma_grad_cells_k<false>, dim3((unsigned)blocks), dim3(256), 0, s,
                               (const TileDev*)c->b_tiles.p, c->T, (const FrameDev*)c->b_frames.p, c->cell_px, n,
                               (const float*)c->b_gsum.p, (const float*)c->b_delta.p, (const uint8_t*)c->b_bin.p,
                               (const float*)c->b_sigma.p, (const float*)c->b_bias.p, glo, ghi);
    } else if (c->S > 0) {
        ProfScope ps(c, KID_SIGMA, s);
        int64_t blocks = (c->S / 16 + 255) / 256;
        if (blocks > SG_BLOCKS) blocks = SG_BLOCKS;
        if (dbias)
            hipLaunchKernelGGL(sigma_grad_k<true>, dim3((unsigned)blocks), dim3(256), 0, s,
                               (const float*)c->b_gsum.p, (const float*)c->b_delta.p, (const uint8_t*)c->b_bin.p,
                               c->S, (const float*)c->b_sigma.p, (const float*)c->b_bias.p, glo, ghi);
        else
            hipLaunchKernelGGL(sigma_grad_k<false>, dim3((unsigned)blocks), dim3(256), 0, s,
                               (const float*)c->b_gsum.p, (const float*)c->b_delta.p, (const uint8_t*)c->b_bin.p,
                               c->S, (const float*)c->b_sigma.p, (const float*)c->b_bias.p, glo, ghi);
    }
    hipLaunchKernelGGL(sigma_final_k, dim3(nb), dim3(256), 0, s, (const unsigned long long*)glo,
                       (const long long*)ghi, n, dsigma, dbias);
    return hipGetLastError();
}

}  // namespace mrf
