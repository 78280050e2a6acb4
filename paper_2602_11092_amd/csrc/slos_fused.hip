// Fused, LDS-resident kernels of the photon-by-photon recursion
// (arXiv 2602.11092, Sec. II-A-2 and II-A-3).
//
// One workgroup owns one sample at a time (persistent loop over a
// largest-first work order, so batches with mixed photon numbers share one
// launch).  With i_1 <= ... <= i_n the sample's input photon modes, layer k
// holds every k-photon state t and
//
//     d_k[t] = sum_{j : t_j >= 1} U[j][i_k] * d_{k-1}[t - e_j],   d_0 = 1,
//
// so that a_t = d_n[t] * sqrt(prod t! / prod s!).  Layers 1..n-1 live in LDS;
// the last layer is streamed straight to HBM (forward) or consumed in
// LDS-sized chunks (backward).  Each state pulls its predecessors through
// the precomputed transition tables (four entries per 16-byte load, several
// states per thread so that many table loads are in flight).  No atomics:
// results are bitwise reproducible.
//
// Backward (adjoint of the recursion): with G the gradient convention
// dL/dRe + i dL/dIm,
//   g_n[t]      = 2 dL/dp_t c_t^2 d_n[t]    (probabilities, c_t = sqrt(prod t!/prod s!))
//               = c_t G_a[t]                (amplitudes)
//   g_{k-1}[t'] = sum_j conj(U[j][i_k]) g_k[t' + e_j]
//   G_U[j][i_k] += sum_t' conj(d_{k-1}[t']) g_k[t' + e_j]
// Layers are recomputed rather than stored.  Every thread owns fixed states
// t' of layer k-1 (register accumulators for g_{k-1}); for each output mode j
// it gathers g_k[t' + e_j] from LDS.  The top layer is consumed in chunks of
// consecutive "smallest occupied mode" blocks: for a chunk of smallest modes
// [a, b) the pairs (t', j) whose successor falls in it are exactly
// {min(t') in [a,b), j >= a} (whole groups of four modes per owned state)
// and {min(t') >= b, a <= j < b} (a few modes, one at a time; there the
// successor's rank is t' plus a per-mode constant, so no table is read),
// two contiguous ranges of t', so the pull stays a plain gather from LDS.
// Both keep the G_U partials per lane in registers, reduced in a fixed order
// once per layer, and a wave skips the owned slots where none of its lanes is
// in range.  The smaller lower layers take g_{k-1} from the same pull and
// G_U from mode-per-wave dot products.
#include <type_traits>

#include "slos_internal.h"

namespace slos {
namespace {

// LDS map, byte addresses (the kernels declare no static LDS, so dynamic LDS
// starts at address 0): the coefficient column, then the state buffers.
constexpr uint32_t kUcolAddr = 0;                    // [33] column i_k of U; slot 32 stays zero
constexpr uint32_t kXAddr = kUcolSlots * 8;          // state buffers
static_assert(kUcolAddr == 0, "compact entries address the coefficient column directly");

constexpr int kLU = 4;  // states per thread per iteration in the forward gathers
constexpr int kLP = 2;  // states whose gathers are issued together

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

// Sum over the 64 lanes of a wave in a fixed order; lane 63 ends up holding it.
__device__ __forceinline__ float wave_sum63(float v) {
    v += dpp<0xB1>(v);        // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);        // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);       // row_half_mirror
    v += dpp<0x140>(v);       // row_mirror: every lane holds its row's sum
    v += dpp<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3: lane 63 holds the total
    return v;
}

// A wave-uniform value re-materialised at its point of use: tests on it
// become a scalar compare right before the branch instead of lane masks
// hoisted to the kernel entry (which exhaust the scalar registers).
__device__ __forceinline__ int fresh(int x) {
    x = __builtin_amdgcn_readfirstlane(x);
    asm volatile("" : "+s"(x));
    return x;
}
// A fresh copy of a per-lane value (no reuse of values derived from it
// across unrolled blocks, which would keep them live throughout).
__device__ __forceinline__ int fresh_v(int x) {
    asm volatile("" : "+v"(x));
    return x;
}
// bit i of x, tested on a fresh copy
__device__ __forceinline__ bool has(int x, int i) { return (fresh(x) >> i) & 1; }
// does [s*BLOCK, (s+1)*BLOCK) meet [lo, hi)?
template <int BLOCK>
__device__ __forceinline__ bool slot_meets(int s, int lo, int hi) {
    return (s + 1) * BLOCK > fresh(lo) && s * BLOCK < fresh(hi);
}
// does this wave's piece of slot s, [s*BLOCK + 64*wave, +64), meet [lo, hi)?
// (a wave whose lanes all fall outside the range skips the slot)
template <int BLOCK>
__device__ __forceinline__ bool piece_meets(int s, int lo, int hi) {
    const int p = s * BLOCK + 64 * fresh((int)threadIdx.x >> 6);
    return p + 64 > fresh(lo) && p < fresh(hi);
}
// f(std::integral_constant<int, i>) for the one i in [LO, HI) equal to the
// wave-uniform s, through a binary tree of scalar branches: element s of a
// register array without a copy through memory.  The branch bodies pin the
// element they touch so that no level turns into selects over every element.
template <int LO, int HI, typename F>
__device__ __forceinline__ void on_index(int s, F&& f) {
    if constexpr (HI - LO == 1) {
        f(std::integral_constant<int, LO>{});
    } else {
        constexpr int MID = (LO + HI) / 2;
        if (fresh(s) < MID) on_index<LO, MID>(s, f);
        else on_index<MID, HI>(s, f);
    }
}
__device__ __forceinline__ void pin(float2& v) { asm volatile("" : "+v"(v.x), "+v"(v.y)); }
template <int N>
__device__ __forceinline__ float2 elem_get(const float2 (&a)[N], int s) {
    float2 v;
    on_index<0, N>(s, [&](auto I) { v = a[decltype(I)::value]; pin(v); });
    return v;
}
template <int N>
__device__ __forceinline__ void elem_set(float2 (&a)[N], int s, float2 v) {
    on_index<0, N>(s, [&](auto I) { a[decltype(I)::value] = v; pin(a[decltype(I)::value]); });
}

__host__ __device__ constexpr uint32_t range_bits(int lo, int hi) {
    return (hi >= 32 ? 0xFFFFFFFFu : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
}

__device__ __forceinline__ uint32_t comp(const uint4& e, int q) { return q == 0 ? e.x : q == 1 ? e.y : q == 2 ? e.z : e.w; }

// The first NQ entries of predecessor group h for states u0..u0+SP-1,
// branch-free so that all their LDS reads issue before one wait.  A compact
// entry holds two byte offsets: e >> 22 into the coefficient column (an
// empty entry names its zero slot) and e & 0x3FFFF8 into layer k-1 at pb.
template <int SU, int NG, int SP, int NQ>
__device__ __forceinline__ void gather_group(const uint4 (&e)[SU][NG], int h, int u0, uint32_t pb,
                                             float2 (&acc)[SU]) {
    float2 uv[NQ][SP], dv[NQ][SP];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int v = 0; v < SP; ++v) {
            const uint32_t x = comp(e[u0 + v][h], q);
            uv[q][v] = lds_ld(kUcolAddr + (x >> kPredCompactModeShift));
            dv[q][v] = lds_ld(pb + (x & kPredCompactRankMask));
        }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int v = 0; v < SP; ++v) c_fma(acc[u0 + v], uv[q][v], dv[q][v]);
}

// Gathers for SU states whose table entries (groups g0 .. g0+NGX-1) are loaded.
template <int SU, int SP, int NGX>
__device__ __forceinline__ void gather_loaded(const uint4 (&e)[SU][NGX], int g0, int k, uint32_t pb,
                                              float2 (&acc)[SU]) {
#pragma unroll
    for (int h = 0; h < NGX; ++h) {
        const int valid = k - 4 * (g0 + h);  // entries of this group that exist (uniform)
#pragma unroll
        for (int u0 = 0; u0 < SU; u0 += SP) {
            if (valid >= 4) gather_group<SU, NGX, SP, 4>(e, h, u0, pb, acc);
            else if (valid == 3) gather_group<SU, NGX, SP, 3>(e, h, u0, pb, acc);
            else if (valid == 2) gather_group<SU, NGX, SP, 2>(e, h, u0, pb, acc);
            else gather_group<SU, NGX, SP, 1>(e, h, u0, pb, acc);
        }
    }
}

template <int SU, int NGX>
__device__ __forceinline__ void load_entries(__amdgpu_buffer_rsrc_t r, const uint32_t (&vo)[SU], uint32_t gstride,
                                             int g0, uint4 (&e)[SU][NGX]) {
#pragma unroll
    for (int u = 0; u < SU; ++u)
#pragma unroll
        for (int h = 0; h < NGX; ++h) e[u][h] = buf_ld4(r, vo[u], (uint32_t)(g0 + h) * gstride);
}

// NGX consecutive groups from g0 for SU states: table loads first, then the gathers.
template <int SU, int SP, int NGX>
__device__ __forceinline__ void gather_groups(__amdgpu_buffer_rsrc_t r, const uint32_t (&vo)[SU], uint32_t gstride,
                                              int g0, int k, uint32_t pb, float2 (&acc)[SU]) {
    uint4 e[SU][NGX];
    load_entries<SU, NGX>(r, vo, gstride, g0, e);
    gather_loaded<SU, SP, NGX>(e, g0, k, pb, acc);
}

// acc[u] = d_k of the state whose table row starts at byte vo[u] (row * 16),
// pulled from layer k-1 at LDS address pb with coefficients U[j][i_k] from
// the coefficient column.  With k = 1 the row is the state itself.
// KC > 0: k is KC, known when compiling, so every predecessor group's entry
// count is a constant and no branch on it remains.
template <int SU, int SPR, int NG, int KC = 0>
__device__ __forceinline__ void gather_rows(const LayerDev& L, int k, const uint32_t (&vo)[SU], uint32_t pb,
                                            float2 (&acc)[SU]) {
    constexpr int SP = SPR < SU ? SPR : SU;
    static_assert(SU % SP == 0, "states must split evenly into gather sets");
#pragma unroll
    for (int u = 0; u < SU; ++u) acc[u] = c_zero();
    if ((KC > 0 ? KC : k) == 1) {  // d_1[t] = U[t][i_1]
#pragma unroll
        for (int u = 0; u < SU; ++u) acc[u] = lds_ld(kUcolAddr + (vo[u] >> 1));
        return;
    }
    const uint32_t gstride = (uint32_t)L.N * 16u;
    const __amdgpu_buffer_rsrc_t r = buf_rsrc(L.predv, (uint32_t)L.ngrp * gstride);
    if constexpr (KC > 0) {
        constexpr int NGRP = (KC + 3) / 4;  // the table's predecessor groups for layer KC
        constexpr int NPAIR = NG >= 2 ? NGRP / 2 : 0;
#pragma unroll
        for (int p = 0; p < NPAIR; ++p) gather_groups<SU, SP, 2>(r, vo, gstride, 2 * p, KC, pb, acc);
#pragma unroll
        for (int g = 2 * NPAIR; g < NGRP; ++g) gather_groups<SU, SP, 1>(r, vo, gstride, g, KC, pb, acc);
    } else {
        int g0 = 0;
        if (NG >= 2)
            for (; g0 + 2 <= L.ngrp; g0 += 2) gather_groups<SU, SP, 2>(r, vo, gstride, g0, k, pb, acc);
        for (; g0 < L.ngrp; ++g0) gather_groups<SU, SP, 1>(r, vo, gstride, g0, k, pb, acc);
    }
}

// acc[u] = d_k of table row t0 + u*BLOCK for u < SU.  Lanes past tlim
// compute the value of row tlim-1 (callers do not store it).
template <int BLOCK, int SU, int SPR, int NG, int KC = 0>
__device__ __forceinline__ void gather_states(const LayerDev& L, int k, int t0, int tlim, uint32_t pb,
                                              float2 (&acc)[SU]) {
    uint32_t vo[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) vo[u] = (uint32_t)min(t0 + u * BLOCK, tlim - 1) * 16u;
    gather_rows<SU, SPR, NG, KC>(L, k, vo, pb, acc);
}

// One layer of the recursion, LDS to LDS, SU states per thread per iteration.
template <int BLOCK, int SU>
__device__ __forceinline__ void layer_into_lds(const LayerDev& L, int k, uint32_t prev, uint32_t cur) {
    const int N = (int)L.N;
    for (int t0 = threadIdx.x; t0 < N; t0 += BLOCK * SU) {
        float2 acc[SU];
        gather_states<BLOCK, SU, kLP, SU >= 4 ? 2 : 1>(L, k, t0, N, prev, acc);
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int t = t0 + u * BLOCK;
            if (t < N) lds_st(cur + 8u * (uint32_t)t, acc[u]);
        }
    }
}

// Layer record k, read with scalar loads.
__device__ __forceinline__ LayerDev layer(const LayerDev* Ls, int k) {
    const LayerDev* p = Ls + k;
    LayerDev L;
    L.predv = ldc(&p->predv);
    L.succ = ldc(&p->succ);
    L.nrm = ldc(&p->nrm);
    L.minoff = ldc(&p->minoff);
    L.N = ldc(&p->N);
    L.cum = ldc(&p->cum);
    L.ngrp = ldc(&p->ngrp);
    L.pred_shift = ldc(&p->pred_shift);
    return L;
}

// ------------------------------------------------------------------ forward

// Adds pv[u] to the accumulator of each photon's mode of state t0 + u*BLOCK
// (lane tid's column of the [m][BLOCK] float array at accb).  The state's
// photons come from its predecessor entries: an empty entry repeats the
// previous slot's mode.  The group loads of all SU states are issued
// together.  The lane's own column needs no atomics (LDS float atomics are
// several times slower here than a read and a write).
template <int BLOCK, int SU, bool DISTINCT>
__device__ __forceinline__ void photons_into_lds(const LayerDev& L, int k, int t0, int N, const float (&pv)[SU],
                                                 uint32_t accb) {
    const uint32_t gstride = (uint32_t)N * 16u;
    const __amdgpu_buffer_rsrc_t r = buf_rsrc(L.predv, (uint32_t)L.ngrp * gstride);
    const uint32_t col = accb + 4u * threadIdx.x;
    int cur[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) cur[u] = 0;
    for (int g = 0; g < L.ngrp; ++g) {
        uint4 e[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) e[u] = buf_ld4(r, (uint32_t)min(t0 + u * BLOCK, N - 1) * 16u, (uint32_t)g * gstride);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (4 * g + q >= k) break;
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int md = (int)(comp(e[u], q) >> L.pred_shift);
                cur[u] = md == 32 ? cur[u] : md;
                const uint32_t a = col + 4u * (uint32_t)(cur[u] * BLOCK);
                if (!DISTINCT || md != 32) lds_stf(a, lds_ldf(a) + pv[u]);
            }
        }
    }
}

// EPI 0: amplitudes, 1: probabilities (both [out_len]); 2: per-mode photon
// expectations, out[b][j] = sum_t t_j p_t ([B][m]): p_t is added to a
// per-lane LDS accumulator for each photon's mode (lane tid owns column tid
// of the [m][BLOCK] array after the state buffers, so no atomics), and the
// columns are summed once per sample; p is never written.  3: the same with
// one count per occupied mode, sum_t [t_j > 0] p_t (threshold detectors).
// 4: threshold-detector click probabilities, out[thr_off_b + q] = sum of p
// over click pattern q's states: the last layer is taken in runs of whole
// patterns, state by state in pattern order (the plan keeps its predecessor
// rows and norms in that order as well), p into an LDS float array, then one
// thread per pattern adds its states' p in ascending state order; p is never
// written.
template <int BLOCK, int EPI>
__global__ __launch_bounds__(BLOCK) void fused_fwd_kernel(int m, const LayerDev* __restrict__ Ls, BatchDev Bt,
                                                          const float2* __restrict__ U, void* __restrict__ out,
                                                          int S) {
    constexpr bool PROBS = EPI >= 1;
    constexpr bool EXPECT = EPI == 2 || EPI == 3;  // 2: per photon (<n_j>), 3: per occupied mode (clicks)
    constexpr bool THR = EPI == 4;
    extern __shared__ float2 lds[];  // ucol at kUcolAddr, photon layers from kXAddr, accumulators after them
    const int tid = threadIdx.x;
    const uint32_t accb = kXAddr + 8u * (uint32_t)S;
    if (tid < kUcolSlots) lds_st(kUcolAddr + 8 * tid, c_zero());  // slots m..32 stay zero
    for (int item = blockIdx.x; item < Bt.B; item += gridDim.x) {
        const int b = ldc(Bt.order + item);
        const int n = ldc(Bt.n + b);
        const int64_t off = ldc(Bt.off + b);
        const float innorm = ldc(Bt.innorm + b);
        const float2* Ub = U + (size_t)b * m * m;
        const int32_t* modes = Bt.modes + (size_t)b * kMaxPhotons;  // read through ldg
        if (n == 0) {
            if (EXPECT) {
                if (tid < m) ((float*)out)[(size_t)b * m + tid] = 0.f;  // the vacuum has no photons
            } else if (THR) {
                if (tid == 0) ((float*)out)[ldc(Bt.thr_off + b)] = 1.f;  // the empty pattern
            } else if (tid == 0) {
                if (PROBS) ((float*)out)[off] = 1.f;
                else ((float2*)out)[off] = make_float2(1.f, 0.f);
            }
            continue;
        }
        if (EXPECT)
            for (int j = 0; j < m; ++j) lds_stf(accb + 4u * (uint32_t)(j * BLOCK + tid), 0.f);
        for (int k = 1; k <= n; ++k) {
            if (tid < m) lds_st(kUcolAddr + 8 * tid, Ub[tid * m + ldc(modes + (k - 1))]);
            __syncthreads();
            const LayerDev L = layer(Ls, k);
            const int N = (int)L.N;
            // layers alternate between the two ends of the buffer; layer n-1 sits at its start
            if (k < n) {
                const int Np = (int)ldc(&Ls[k - 1].N);
                const uint32_t prev = kXAddr + 8u * (uint32_t)((((n - k) & 1) == 0) ? 0 : S - Np);
                const uint32_t cur = kXAddr + 8u * (uint32_t)((((n - 1 - k) & 1) == 0) ? 0 : S - N);
                layer_into_lds<BLOCK, kLU>(L, k, prev, cur);
            } else if (THR) {
                const int32_t* tptr = ldc(&Ls[k].thr_ptr);
                const int32_t* tch = ldc(&Ls[k].thr_chunk);
                const int nch = ldc(&Ls[k].thr_nchunk);
                float* ob = (float*)out + ldc(Bt.thr_off + b);
                // the tables in pattern order (with one photon that is the state order
                // itself, which the k = 1 gather assumes)
                LayerDev Lp = L;
                Lp.predv = ldc(&Ls[k].thr_predv);
                const __amdgpu_buffer_rsrc_t rn = buf_rsrc(ldc(&Ls[k].thr_nrm), (uint32_t)N * 4u);
                for (int r = 0; r < nch; ++r) {
                    const int q0 = ldc(tch + r), q1 = ldc(tch + r + 1);
                    const int P0 = ldc(tptr + q0), P1 = ldc(tptr + q1);
                    for (int s0 = P0 + tid; s0 < P1; s0 += BLOCK * kLU) {
                        float c[kLU];
#pragma unroll
                        for (int u = 0; u < kLU; ++u)
                            c[u] = buf_ldf(rn, (uint32_t)min(s0 + u * BLOCK, P1 - 1) * 4u, 0) * innorm;
                        float2 acc[kLU];
                        gather_states<BLOCK, kLU, kLP, 2>(Lp, k, s0, P1, kXAddr, acc);
#pragma unroll
                        for (int u = 0; u < kLU; ++u) {
                            const int sp = s0 + u * BLOCK;
                            if (sp < P1)
                                lds_stf(accb + 4u * (uint32_t)(sp - P0),
                                        c[u] * c[u] * (acc[u].x * acc[u].x + acc[u].y * acc[u].y));
                        }
                    }
                    __syncthreads();
                    for (int q = q0 + tid; q < q1; q += BLOCK) {
                        const int lo = ldg(tptr + q) - P0, hi = ldg(tptr + q + 1) - P0;
                        float v = 0.f;
                        for (int i = lo; i < hi; ++i) v += lds_ldf(accb + 4u * (uint32_t)i);
                        ob[q] = v;
                    }
                    __syncthreads();  // before the next run overwrites the array
                }
            } else {
                const __amdgpu_buffer_rsrc_t rn = buf_rsrc(L.nrm, (uint32_t)N * 4u);
                const __amdgpu_buffer_rsrc_t ro =
                    buf_rsrc(PROBS ? (const void*)((float*)out + off) : (const void*)((float2*)out + off),
                             EXPECT ? 0u : (uint32_t)N * (PROBS ? 4u : 8u));
                // the last layer with the photon count as a compile-time constant
                // where it is small (no branch on a group's entry count)
                auto last_layer = [&](auto KCc) {
                    constexpr int KC = decltype(KCc)::value;
                    for (int t0 = tid; t0 < N; t0 += BLOCK * kLU) {
                        float c[kLU];
#pragma unroll
                        for (int u = 0; u < kLU; ++u)
                            c[u] = buf_ldf(rn, (uint32_t)min(t0 + u * BLOCK, N - 1) * 4u, 0) * innorm;
                        float2 acc[kLU];
                        gather_states<BLOCK, kLU, kLP, 2, KC>(L, k, t0, N, kXAddr, acc);
#pragma unroll
                        for (int u = 0; u < kLU; ++u) {
                            const int t = t0 + u * BLOCK;
                            if (!EXPECT && t < N) {
                                if (PROBS) {
                                    const float p = c[u] * c[u] * (acc[u].x * acc[u].x + acc[u].y * acc[u].y);
                                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(p), ro, t * 4, 0, kCpolStream);
                                } else {
                                    const float2 a = c_scale(acc[u], c[u]);
                                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(
                                        __attribute__((ext_vector_type(2))) unsigned int, a), ro, t * 8, 0, kCpolStream);
                                }
                            }
                        }
                        if (EXPECT) {
                            float pv[kLU];
#pragma unroll
                            for (int u = 0; u < kLU; ++u)  // lanes past N add zero
                                pv[u] = t0 + u * BLOCK < N ? c[u] * c[u] * (acc[u].x * acc[u].x + acc[u].y * acc[u].y) : 0.f;
                            photons_into_lds<BLOCK, kLU, EPI == 3>(L, k, t0, N, pv, accb);
                        }
                    }
                };
                switch (k) {
                    case 2: last_layer(std::integral_constant<int, 2>{}); break;
                    case 3: last_layer(std::integral_constant<int, 3>{}); break;
                    case 4: last_layer(std::integral_constant<int, 4>{}); break;
                    case 5: last_layer(std::integral_constant<int, 5>{}); break;
                    case 6: last_layer(std::integral_constant<int, 6>{}); break;
                    case 7: last_layer(std::integral_constant<int, 7>{}); break;
                    case 8: last_layer(std::integral_constant<int, 8>{}); break;
                    default: last_layer(std::integral_constant<int, 0>{}); break;
                }
            }
            __syncthreads();
        }
        if (EXPECT) {
            // column sums: wave w takes modes w, w + BLOCK/64, ...; fixed order
            const int w = tid >> 6, lane = tid & 63;
            for (int j = w; j < m; j += BLOCK / 64) {
                float v = 0.f;
                for (int i = lane; i < BLOCK; i += 64) v += lds_ldf(accb + 4u * (uint32_t)(j * BLOCK + i));
                v = wave_sum63(v);
                if (lane == 63) ((float*)out)[(size_t)b * m + j] = v;
            }
            __syncthreads();  // before the next sample clears the accumulators
        }
    }
}

// ------------------------------------------------------------------ backward

// Every thread owns states t' = tid + s*BLOCK (s < OWN) of layer k-1: acc[s]
// accumulates g_{k-1}[t'] and h[j] this lane's share of
// G_U[j][i_k] = sum_t' conj(d_{k-1}[t']) g_k[t' + e_j].  For owned t' in
// [lo, hi) and output modes j in [jlo, jhi):
//   g = g_k[t' + e_j] (LDS, srcb + successor byte offset),
//   acc[s] += conj(u_j) g,  h[j] += conj(d_{k-1}[t']) g  (d_{k-1} at Db).
// Successor offsets come in groups of four modes, [j/4][t'][4]: one
// coalesced 16-byte load serves four pairs.

// u_j read at its point of use (a broadcast LDS read; volatile so that it is
// not kept in registers where registers are short).
__device__ __forceinline__ float2 coeff(uint32_t j) {
    typedef __attribute__((address_space(3))) const volatile unsigned long long lds_vu64;
    return __builtin_bit_cast(float2, *(lds_vu64*)(size_t)(kUcolAddr + 8 * j));
}

// Owned t' in [lo, hi), modes j in [jlo, jhi), by groups of four modes, one
// owned slot (t' = tid + s*BLOCK) per iteration of a loop over the slots that
// meet the range: the slot's successor loads (one 16-byte load per group)
// issue together, then per group its four LDS gathers, then their products;
// g_{k-1} of the slot is taken out of and put back into acc[s] by a scalar
// branch tree, so the code holds one slot's pairs, not OWN of them (the
// kernel's instruction footprint is what this keeps small).  Branch-free per
// pair: a lane whose t' lies outside the range gathers the zero slot (one
// select on the slot's lane mask), and so do the modes outside [jlo, jhi) of
// the (at most two) groups that straddle its ends, whose successor offsets
// are replaced by the zero slot's once per group.  The coefficient column
// conj(u_j) sits in registers for the whole call where the workgroup shape
// leaves room (below 1024 threads).
template <int BLOCK, int OWN, int MMAX, bool WITH_H = true, bool RS = false>
__device__ __forceinline__ void pull(int lo, int hi, int jlo, int jhi, __amdgpu_buffer_rsrc_t rs, uint32_t gstride,
                                     uint32_t srcb, uint32_t Db, float2 (&acc)[OWN], float2 (&h)[MMAX]) {
    constexpr int NG = MMAX / 4;
    constexpr bool kCoefRegs = BLOCK < 1024;
    if (lo >= hi || jlo >= jhi) return;
    const int tid = threadIdx.x;
    const int gbits = (int)range_bits(jlo >> 2, (jhi + 3) >> 2);  // the groups that meet [jlo, jhi)
    const int fbits = (int)range_bits((jlo + 3) >> 2, jhi >> 2);  // the groups inside it
    const uint32_t zoff = kUcolAddr + 32 * 8 - srcb;  // srcb + zoff: the zero slot
    float2 cu[kCoefRegs ? MMAX : 1];
    if (kCoefRegs) {
#pragma unroll
        for (int j = 0; j < (kCoefRegs ? MMAX : 1); ++j) cu[j] = lds_ld(kUcolAddr + 8u * (uint32_t)j);
    }
    const int s_end = min(OWN, (hi + BLOCK - 1) / BLOCK);
    for (int s = lo / BLOCK; s < s_end; ++s) {  // the owned slots that meet [lo, hi) (uniform)
        if (!piece_meets<BLOCK>(s, lo, hi)) continue;  // none of this wave's lanes in range
        const int tp = tid + s * BLOCK;
        const bool act = tp >= lo && tp < hi;
        const int tc = min(max(tp, lo), hi - 1);
        const uint32_t vo = (uint32_t)tc * 16u;
        uint4 sv[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) sv[g] = buf_ld4(rs, vo, (uint32_t)g * gstride);
        float2 dv = lds_ld(Db + 8u * (uint32_t)tc);
        float2 a = elem_get<OWN>(acc, s);
        // Standard spaces: a lane out of range works on state tc instead, which
        // is in range, so its successors in [jlo, jhi) lie in the source range
        // too (finite values); its products are dropped once per slot (d set to
        // zero for the G_U shares, its accumulator kept) rather than by a select
        // per gather.  Restricted spaces select per gather, as their tables
        // mark successors outside the space.
        const float2 a0 = a;
        if constexpr (!RS) dv = act ? dv : c_zero();
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if (!has(gbits, g)) continue;  // no mode of this group in range (uniform)
            uint32_t c[4] = {sv[g].x, sv[g].y, sv[g].z, sv[g].w};
            if (!has(fbits, g)) {  // a group straddling an end of the range (uniform)
                const int jl = fresh(jlo), jh = fresh(jhi);  // tests formed here, not hoisted
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (4 * g + q < jl || 4 * g + q >= jh) c[q] = zoff;
            }
            // the group's four gathers, then its products
            float2 gv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if constexpr (RS) {
                    // a successor outside the space was never formed
                    const bool ok = act && c[q] != kNoSuccessor;
                    gv[q] = lds_ld(srcb + (ok ? c[q] : zoff));
                } else {
                    gv[q] = lds_ld(srcb + c[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = 4 * g + q;
                c_fma_conj(a, kCoefRegs ? cu[kCoefRegs ? j : 0] : coeff(j), gv[q]);
                if (WITH_H) c_fma_conj(h[j], dv, gv[q]);
            }
        }
        if constexpr (!RS) a = act ? a : a0;
        elem_set<OWN>(acc, s, a);
    }
}

// A few modes j in [jlo, jhi) below the smallest occupied mode of every
// owned t' in [lo, hi) (t' from the end of layer k-1: its smallest mode is at
// least jhi).  Such a successor needs no table: in the basis order the
// states of layer k whose smallest mode is j and holds one photon are e_j + t'
// for the t' whose smallest mode exceeds j, in the order of t', and they end
// the block of smallest mode j, so rank(t' + e_j) = t' + minoff_k(j+1) - N_{k-1}
// (a per-mode constant).  conj(d_{k-1}) of the owned states is read once;
// then mode by mode (a uniform test per mode): the mode's coefficient and
// offset, the gathers of every owned slot from the first that meets the
// range, issued together (lanes out of range gather the zero slot), then
// their products.  G_U shares go to the same per-lane h[j] as
// the wide pull.  Restricted spaces (where such a successor may leave the
// space) read their successor tables instead, slot by slot.
template <int BLOCK, int OWN, int MMAX, bool RS = false>
__device__ __forceinline__ void pull_narrow(int lo, int hi, int jlo, int jhi, __amdgpu_buffer_rsrc_t rs,
                                            uint32_t gstride, uint32_t srcb, uint32_t Db, float2 (&acc)[OWN],
                                            float2 (&h)[MMAX], uint32_t MOk, int Nkm1) {
    if (lo >= hi || jlo >= jhi) return;
    const int tid = threadIdx.x;
    const int jbits = (int)range_bits(jlo, jhi);
    const uint32_t zaddr = kUcolAddr + 32 * 8;  // the zero slot
    const uint32_t zoff = zaddr - srcb;         // srcb + zoff: the zero slot
    // slots below s_first hold no owned state in range (uniform)
    const int s_first = fresh(lo) / BLOCK;
    float2 dv[OWN];  // conj(d_{k-1}) of the owned states, read once
#pragma unroll
    for (int s = 0; s < OWN; ++s) {
        if (s < fresh(s_first)) continue;
        const int tp = fresh_v(tid) + s * BLOCK;
        dv[s] = lds_ld(Db + 8u * (uint32_t)min(max(tp, lo), hi - 1));
    }
#pragma unroll
    for (int j = 0; j < MMAX; ++j) {
        if (!has(jbits, j)) continue;  // uniform, once per mode
        const float2 uj = coeff(j);
        float2 g[OWN];
        if constexpr (RS) {
            const uint32_t soff = (uint32_t)(j >> 2) * gstride + 4u * (uint32_t)(j & 3);
#pragma unroll
            for (int s = 0; s < OWN; ++s) {
                if (s < fresh(s_first)) continue;
                const int tp = fresh_v(tid) + s * BLOCK;
                const bool act = tp >= lo && tp < hi;
                const uint32_t sv = buf_ld1(rs, (uint32_t)min(max(tp, lo), hi - 1) * 16u, soff);
                g[s] = lds_ld(srcb + ((act && sv != kNoSuccessor) ? sv : zoff));
            }
        } else {
            // successor t' + minoff_k(j+1) - N_{k-1}: a uniform byte offset from the state's own
            const uint32_t dj = srcb + 8u * (uint32_t)(__builtin_amdgcn_readfirstlane(lds_ldi(MOk + 4u * (uint32_t)(j + 1))) - Nkm1);
#pragma unroll
            for (int s = 0; s < OWN; ++s) {
                if (s < fresh(s_first)) continue;
                const int tp = fresh_v(tid) + s * BLOCK;
                const bool act = tp >= lo && tp < hi;
                g[s] = lds_ld(act ? dj + 8u * (uint32_t)tp : zaddr);
            }
        }
#pragma unroll
        for (int s = 0; s < OWN; ++s) {
            if (s < fresh(s_first)) continue;
            c_fma_conj(acc[s], uj, g[s]);
            c_fma_conj(h[j], dv[s], g[s]);
        }
    }
}

// G_U[j][i_k] = sum_t' conj(d_{k-1}[t']) g_k[t' + e_j] for a small layer:
// wave w takes the modes j = w + NW r (r < R, all in one loop so that their
// loads overlap), its lanes stride over t', and lane 63 writes each mode's
// fixed-order wave sum straight to GUcol[j] (one wave per mode, so no
// cross-wave step).  Modes past m read the zero slot and are not written.
template <int BLOCK, int MMAX, bool RS = false>
__device__ __forceinline__ void lower_h(int m, int Nkm1, __amdgpu_buffer_rsrc_t rs, uint32_t gstride, uint32_t gk,
                                        uint32_t Dk, uint32_t GUcol) {
    constexpr int NW = BLOCK / 64;
    constexpr int R = (MMAX + NW - 1) / NW;
    constexpr int U = 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t zero = kUcolAddr + 32 * 8;
    float2 hj[R];
#pragma unroll
    for (int r = 0; r < R; ++r) hj[r] = c_zero();
    for (int t0 = lane; t0 < Nkm1; t0 += 64 * U) {
        uint32_t sv[R][U];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = min(wave + NW * r, m - 1);
            const uint32_t col = 4u * (uint32_t)(j & 3), goff = (uint32_t)(j >> 2) * gstride;
#pragma unroll
            for (int u = 0; u < U; ++u) sv[r][u] = buf_ld1(rs, (uint32_t)min(t0 + 64 * u, Nkm1 - 1) * 16u + col, goff);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int tp = t0 + 64 * u;
            const float2 dv = lds_ld(Dk + 8u * (uint32_t)min(tp, Nkm1 - 1));
#pragma unroll
            for (int r = 0; r < R; ++r) {
                // past the layer or past m: the zero slot
                bool ok = tp < Nkm1 && wave + NW * r < m;
                if constexpr (RS) ok = ok && sv[r][u] != kNoSuccessor;
                const float2 g = lds_ld(ok ? gk + sv[r][u] : zero);
                c_fma_conj(hj[r], dv, g);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float re = wave_sum63(hj[r].x);
        const float im = wave_sum63(hj[r].y);
        const int j = wave + NW * r;
        if (lane == 63 && j < m) lds_st(GUcol + 8u * (uint32_t)j, make_float2(re, im));
    }
}

// One halving exchange of a wave-wide sum of C values per lane: lanes with
// bit D of the lane index set keep the upper C/2 values, the others the lower
// C/2, and each adds its partner's (lane ^ D) copy of the half it keeps.
template <int C, int D, int T>
__device__ __forceinline__ void halve_across(float (&v)[T], int lane) {
    const bool up = (lane & D) != 0;
    const int from = (lane ^ D) << 2;
#pragma unroll
    for (int i = 0; i < C / 2; ++i) {
        const float send = up ? v[i] : v[i + C / 2];
        const float keep = up ? v[i + C / 2] : v[i];
        float recv;
        if constexpr (D >= 16) recv = __int_as_float(__builtin_amdgcn_ds_bpermute(from, __float_as_int(send)));
        else recv = dpp<0x128>(send);  // row_ror:8: lane ^ 8 within the 16-lane row
        v[i] = keep + recv;
    }
}

// The sums over a wave's 64 lanes of the 2*MMAX floats of h (value 2j is
// Re h[j], 2j+1 is Im h[j]), written to the wave's row of Hw (float2 per j).
// Three halving exchanges, with the lanes 32, 16 and 8 away, leave each group
// of eight lanes (g = lane / 8) with partial sums of the values
// [g*T/8, (g+1)*T/8); three DPP steps finish them inside the group, and lane
// 8g writes them.  A fixed order, in about a third of the VALU instructions of
// one six-step DPP reduction per value.
template <int MMAX>
__device__ __forceinline__ void wave_sum_columns(const float2 (&h)[MMAX], uint32_t row) {
    constexpr int T = 2 * MMAX;
    static_assert(T % 8 == 0, "three halvings of the values");
    const int lane = threadIdx.x & 63;
    float v[T];
#pragma unroll
    for (int j = 0; j < MMAX; ++j) {
        v[2 * j] = h[j].x;
        v[2 * j + 1] = h[j].y;
    }
    halve_across<T, 32>(v, lane);
    halve_across<T / 2, 16>(v, lane);
    halve_across<T / 4, 8>(v, lane);
#pragma unroll
    for (int i = 0; i < T / 8; ++i) {
        float x = v[i];
        x += dpp<0xB1>(x);   // quad_perm [1,0,3,2]
        x += dpp<0x4E>(x);   // quad_perm [2,3,0,1]
        x += dpp<0x141>(x);  // row_half_mirror: every lane holds its group's sum
        v[i] = x;
    }
    if ((lane & 7) == 0) {
        const int g = lane >> 3;
#pragma unroll
        for (int i = 0; i < T / 8; ++i) lds_stf(row + 4u * (uint32_t)(g * (T / 8) + i), v[i]);
    }
}

// Sums h[j] over the workgroup (per wave, then over the waves in a fixed
// order) into the LDS column at GUcol, j < MMAX (h[j] = 0 for j >= m).
// Hw: [NW][32] LDS scratch.
template <int BLOCK, int MMAX>
__device__ __forceinline__ void reduce_columns(const float2 (&h)[MMAX], int m, uint32_t Hw, uint32_t GUcol) {
    constexpr int NW = BLOCK / 64;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    wave_sum_columns<MMAX>(h, Hw + 8u * (uint32_t)(wave * 32));
    __syncthreads();
    if (tid < m) {
        float2 sum = c_zero();
        for (int w = 0; w < NW; ++w) sum = c_add(sum, lds_ld(Hw + 8u * (uint32_t)(w * 32 + tid)));
        lds_st(GUcol + 8u * (uint32_t)tid, sum);
    }
}

// RS: plans of a restricted space (unbunched, dual-rail), whose successor
// tables mark successors outside the space; those pairs read the zero slot.
template <int BLOCK, int OWN, int MMAX, bool RS>
__global__ __launch_bounds__(BLOCK) void fused_bwd_kernel(int m, const LayerDev* __restrict__ Ls, BatchDev Bt,
                                                          const float2* __restrict__ U,
                                                          const void* __restrict__ gin,
                                                          float2* __restrict__ gU, int S, int PROBS, int KR) {
    constexpr int NW = BLOCK / 64;
    // states per thread in the gathers (register budget: acc and h stay live)
    // (the layer recomputes run while acc and h are dead: the forward's width)
    constexpr int GU = kLU;
    constexpr int GM = BLOCK <= 512 ? 4 : BLOCK <= 768 ? 2 : 1;  // wider gathers where registers allow
    // KR: layers d_0..d_KR stay in LDS from the first recompute to the lower
    // layers' pulls, in the last slots of X (KR = -1: none)
    // LDS: ucol | X[S] layers and chunks | Hw[NW][32] | GUacc[16][32] | the
    // sample's U [m][m] | minoff of layers n and n-1 [2][m+1] | photon modes
    extern __shared__ float2 lds[];
    const uint32_t Hw = kXAddr + 8u * (uint32_t)S;
    const uint32_t GUacc = Hw + 8u * NW * 32;
    const uint32_t Ust = GUacc + 8u * kMaxPhotons * 32;
    const uint32_t MOn = Ust + 8u * (uint32_t)(m * m);
    const uint32_t MOp = MOn + 4u * (uint32_t)(m + 1);
    const uint32_t MDs = MOp + 4u * (uint32_t)(m + 1);
    // wave-uniform reads of the staged index rows
    auto mode_of = [&](int i) { return __builtin_amdgcn_readfirstlane(lds_ldi(MDs + 4u * (uint32_t)i)); };
    auto minoff_n = [&](int c) { return __builtin_amdgcn_readfirstlane(lds_ldi(MOn + 4u * (uint32_t)c)); };
    auto minoff_p = [&](int c) { return __builtin_amdgcn_readfirstlane(lds_ldi(MOp + 4u * (uint32_t)c)); };
    // column i_k of U into the coefficient column (slots m..32 stay zero)
    auto load_ucol = [&](int k) {
        const int tid = threadIdx.x;
        if (tid < m) lds_st(kUcolAddr + 8 * tid, lds_ld(Ust + 8u * (uint32_t)(tid * m + mode_of(k - 1))));
    };
    const int tid = threadIdx.x;
    if (tid < kUcolSlots) lds_st(kUcolAddr + 8 * tid, c_zero());  // slots m..32 stay zero

    for (int item = blockIdx.x; item < Bt.B; item += gridDim.x) {
        const int b = ldc(Bt.order + item);
        const int n = ldc(Bt.n + b);
        const int64_t off = ldc(Bt.off + b);
        const float innorm = ldc(Bt.innorm + b);
        const float2* Ub = U + (size_t)b * m * m;
        const int32_t* modes = Bt.modes + (size_t)b * kMaxPhotons;
        float2* gUb = gU + (size_t)b * m * m;

        for (int q = tid; q < kMaxPhotons * 32; q += BLOCK) lds_st(GUacc + 8u * q, c_zero());
        // the sample's U, the index rows its layers consult, and its photon
        // modes, staged once (one round of loads instead of one per layer)
        for (int q = tid; q < m * m; q += BLOCK) lds_st(Ust + 8u * q, Ub[q]);
        if (n >= 2) {
            const int32_t* mon = ldc(&Ls[n].minoff);
            const int32_t* mop = ldc(&Ls[n - 1].minoff);
            for (int q = tid; q <= m; q += BLOCK) {
                lds_sti(MOn + 4u * q, ldg(mon + q));
                lds_sti(MOp + 4u * q, ldg(mop + q));
            }
        }
        if (tid < kMaxPhotons) lds_sti(MDs + 4u * tid, tid < n ? ldg(modes + tid) : -1);
        __syncthreads();

        if (n == 1) {
            // g_1[j] is G_U[j][i_1] itself (d_0 = 1)
            if (tid < m) {
                // (addresses formed here: hoisted out of the sample loop they would
                // hold registers through the whole kernel)
                const int j = fresh_v(tid);
                const float c = ldg(layer(Ls, 1).nrm + j) * innorm;
                const float2 v = PROBS ? c_scale(lds_ld(Ust + 8u * (uint32_t)(j * m + mode_of(0))), 2.f * ((const float*)gin)[off + j] * c * c)
                                       : c_scale(((const float2*)gin)[off + j], c);
                lds_st(GUacc + 8u * j, v);
            }
            __syncthreads();
        } else if (n >= 2) {
            const LayerDev Ln = layer(Ls, n);
            const LayerDev Lp = layer(Ls, n - 1);
            const int Np = (int)Lp.N;
            // the kept layers d_0..d_KRs sit at E + (states with fewer photons)
            const int KRs = min(KR, n - 2);
            const int E = S - (KR >= 0 ? (int)ldc(&Ls[KR + 1].cum) : 0);
            if (KRs >= 0 && tid == 0)
                lds_st(kXAddr + 8u * (uint32_t)E, make_float2(__int_as_float(fresh_v(0x3f800000)), 0.f));
            // ---- recompute layers 1..n-1; layer n-1 ends at the start of X,
            // the others alternate ends of X[0, E) unless kept
            for (int k = 1; k <= n - 1; ++k) {
                load_ucol(k);
                __syncthreads();
                const LayerDev Lk = layer(Ls, k);
                const int Nk = (int)Lk.N;
                const int Nkm1 = (int)ldc(&Ls[k - 1].N);
                const int ps =
                    (k - 1 <= KRs) ? E + (int)ldc(&Ls[k - 1].cum) : ((((n - k) & 1) == 0) ? 0 : E - Nkm1);
                const int cs = (k <= KRs) ? E + (int)Lk.cum : ((((n - 1 - k) & 1) == 0) ? 0 : E - Nk);
                layer_into_lds<BLOCK, GU>(Lk, k, kXAddr + 8u * (uint32_t)ps, kXAddr + 8u * (uint32_t)cs);
                __syncthreads();
            }
            // ---- top layer, in chunks of smallest-mode blocks
            load_ucol(n);
            const uint32_t D = kXAddr;                     // d_{n-1}
            const uint32_t C = kXAddr + 8u * (uint32_t)Np;  // the chunk of g_n
            const int cap = E - Np;
            const uint32_t gstride = (uint32_t)Np * 16u;  // one group of four successor columns
            const __amdgpu_buffer_rsrc_t rs = buf_rsrc(Ln.succ, (uint32_t)((m + 3) / 4) * gstride);
            const __amdgpu_buffer_rsrc_t rn = buf_rsrc(Ln.nrm, (uint32_t)Ln.N * 4u);
            const __amdgpu_buffer_rsrc_t rg =
                buf_rsrc(PROBS ? (const void*)((const float*)gin + off) : (const void*)((const float2*)gin + off),
                         (uint32_t)Ln.N * (PROBS ? 4u : 8u));
            float2 acc[OWN];
            float2 h[MMAX];
#pragma unroll
            for (int s = 0; s < OWN; ++s) acc[s] = c_zero();
#pragma unroll
            for (int j = 0; j < MMAX; ++j) h[j] = c_zero();
            __syncthreads();
            int a = 0;
            while (a < m) {
                int bb = a + 1;
                const int base = minoff_n(a);
                while (bb < m && minoff_n(bb + 1) - base <= cap) ++bb;
                const int end = minoff_n(bb);
                // g_n on the chunk: 2 dL/dp_t c_t^2 d_n[t] (probabilities; the
                // factor loads issue together with the gather's table loads) or
                // c_t G_a[t] (amplitudes, a streaming pass).
                if (PROBS) {
                    for (int t0 = base + tid; t0 < end; t0 += BLOCK * GM) {
                        float cv[GM], gv[GM];
#pragma unroll
                        for (int q = 0; q < GM; ++q) {
                            const uint32_t tc = (uint32_t)min(t0 + q * BLOCK, end - 1);
                            cv[q] = buf_ldf(rn, tc * 4u, 0) * innorm;
                            gv[q] = buf_ldf_stream(rg, tc * 4u);
                        }
                        float2 d[GM];
                        gather_states<BLOCK, GM, kLP, 2>(Ln, n, t0, end, D, d);
#pragma unroll
                        for (int q = 0; q < GM; ++q) {
                            const int t = t0 + q * BLOCK;
                            if (t < end) lds_st(C + 8u * (uint32_t)(t - base), c_scale(d[q], 2.f * gv[q] * cv[q] * cv[q]));
                        }
                    }
                } else {
                    for (int t0 = base + tid; t0 < end; t0 += BLOCK * 4) {
                        float cv[4];
                        float2 gv[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const uint32_t tc = (uint32_t)min(t0 + q * BLOCK, end - 1);
                            cv[q] = buf_ldf(rn, tc * 4u, 0) * innorm;
                            gv[q] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rg, (int)(tc * 8u), 0, kCpolStream));
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int t = t0 + q * BLOCK;
                            if (t < end) lds_st(C + 8u * (uint32_t)(t - base), c_scale(gv[q], cv[q]));
                        }
                    }
                }
                __syncthreads();
                // {min(t') in [a, bb), j >= a} and {min(t') >= bb, a <= j < bb}
                const uint32_t srcb = C - 8u * (uint32_t)base;
                const int wlo = minoff_p(a), whi = minoff_p(bb);
                pull<BLOCK, OWN, MMAX, true, RS>(wlo, whi, a, m, rs, gstride, srcb, D, acc, h);
                pull_narrow<BLOCK, OWN, MMAX, RS>(whi, Np, a, bb, rs, gstride, srcb, D, acc, h, MOn, Np);
                __syncthreads();
                a = bb;
            }
            // g_{n-1} replaces d_{n-1}; the top layer's column of G_U
#pragma unroll
            for (int s = 0; s < OWN; ++s) {
                const int tp = fresh_v(tid) + s * BLOCK;
                if (tp < Np) lds_st(kXAddr + 8u * (uint32_t)tp, acc[s]);
            }
            reduce_columns<BLOCK, MMAX>(h, m, Hw, GUacc + 8u * (uint32_t)((n - 1) * 32));
            // ---- lower layers.  d_0..d_{n-2} not kept are recomputed after
            // g_{n-1} (layer k at Np + number of states with < k photons); g
            // ping-pongs between 0 and R.
            const int R = Np + (int)Lp.cum;
            auto dslot = [&](int k) { return (k <= KRs ? E : Np) + (int)ldc(&Ls[k].cum); };
            // d_0 = 1 (the constant formed here, not kept in registers from the kernel entry)
            if (KRs < 0 && tid == 0)
                lds_st(kXAddr + 8u * (uint32_t)Np, make_float2(__int_as_float(fresh_v(0x3f800000)), 0.f));
            __syncthreads();
            for (int k = max(1, KRs + 1); k <= n - 2; ++k) {
                load_ucol(k);
                __syncthreads();
                const LayerDev Lk = layer(Ls, k);
                layer_into_lds<BLOCK, GU>(Lk, k, kXAddr + 8u * (uint32_t)dslot(k - 1),
                                          kXAddr + 8u * (uint32_t)dslot(k));
                __syncthreads();
            }
            for (int k = n - 1; k >= 1; --k) {
                load_ucol(k);
                const uint32_t gk = kXAddr + 8u * (uint32_t)((((n - 1 - k) & 1) == 0) ? 0 : R);
                const uint32_t gkm1 = kXAddr + 8u * (uint32_t)((((n - k) & 1) == 0) ? 0 : R);
                const LayerDev Lkm1 = layer(Ls, k - 1);
                const uint32_t dkm1 = kXAddr + 8u * (uint32_t)dslot(k - 1);
                const int Nkm1 = (int)Lkm1.N;
                const uint32_t gsk = (uint32_t)Nkm1 * 16u;
                const __amdgpu_buffer_rsrc_t rsk = buf_rsrc(ldc(&Ls[k].succ), (uint32_t)((m + 3) / 4) * gsk);
                __syncthreads();
                if (Nkm1 > BLOCK / 2) {
                    // a layer that fills the lanes: g_{k-1} and G_U from one pull, then a column reduction
#pragma unroll
                    for (int s = 0; s < OWN; ++s) acc[s] = c_zero();
#pragma unroll
                    for (int j = 0; j < MMAX; ++j) h[j] = c_zero();
                    pull<BLOCK, OWN, MMAX, true, RS>(0, Nkm1, 0, m, rsk, gsk, gk, dkm1, acc, h);
                    if (k >= 2) {
#pragma unroll
                        for (int s = 0; s < OWN; ++s) {
                            const int tp = fresh_v(tid) + s * BLOCK;
                            if (tp < Nkm1) lds_st(gkm1 + 8u * (uint32_t)tp, acc[s]);
                        }
                    }
                    reduce_columns<BLOCK, MMAX>(h, m, Hw, GUacc + 8u * (uint32_t)((k - 1) * 32));
                } else {
                    if (k >= 2) {
#pragma unroll
                        for (int s = 0; s < OWN; ++s) acc[s] = c_zero();
                        pull<BLOCK, OWN, MMAX, false, RS>(0, Nkm1, 0, m, rsk, gsk, gk, dkm1, acc, h);
#pragma unroll
                        for (int s = 0; s < OWN; ++s) {
                            const int tp = fresh_v(tid) + s * BLOCK;
                            if (tp < Nkm1) lds_st(gkm1 + 8u * (uint32_t)tp, acc[s]);
                        }
                    }
                    if (!RS && k == 1) {
                        // layer 1 is e_0 .. e_{m-1} in rank order and d_0 = 1:
                        // G_U[j][i_1] = g_1[j]
                        if (tid < m) lds_st(GUacc + 8u * (uint32_t)tid, lds_ld(gk + 8u * (uint32_t)tid));
                    } else {
                        lower_h<BLOCK, MMAX, RS>(m, Nkm1, rsk, gsk, gk, dkm1, GUacc + 8u * (uint32_t)((k - 1) * 32));
                    }
                }
                __syncthreads();
            }
        }
        // assemble G_U[b]: column i collects the layers whose photon sits in mode i
        __syncthreads();
        for (int q = tid; q < m * m; q += BLOCK) {
            const int j = q / m, i = q % m;
            float2 v = c_zero();
            for (int k = 1; k <= n; ++k)
                if (mode_of(k - 1) == i) v = c_add(v, lds_ld(GUacc + 8u * (uint32_t)((k - 1) * 32 + j)));
            gUb[q] = v;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host side

// photon-layer-(n-1) states per thread in the register-resident pulls
int own_for(int block, int64_t Np) {
    const int64_t need = (Np + block - 1) / block;
    if (block == 256) return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : -1;
    if (block == 512) return need <= 4 ? 4 : need <= 10 ? 10 : need <= 18 ? 18 : -1;
    if (block == 768) return need <= 12 ? 12 : -1;
    if (block == 1024) return need <= 10 ? 10 : -1;
    return -1;
}

int mmax_for(int m) { return m <= 8 ? 8 : m <= 12 ? 12 : m <= 16 ? 16 : m <= 20 ? 20 : m <= 24 ? 24 : 32; }

template <int BLOCK, int OWN, bool R>
void* bwd_by_m(int mm) {
    if constexpr (BLOCK >= 768) {
        if (mm > 20) return nullptr;  // h and acc do not fit the registers of 12 or 16 waves
    }
    switch (mm) {
        case 8: return (void*)&fused_bwd_kernel<BLOCK, OWN, 8, R>;
        case 12: return (void*)&fused_bwd_kernel<BLOCK, OWN, 12, R>;
        case 16: return (void*)&fused_bwd_kernel<BLOCK, OWN, 16, R>;
        case 20: return (void*)&fused_bwd_kernel<BLOCK, OWN, 20, R>;
        case 24:
            if constexpr (BLOCK < 768) return (void*)&fused_bwd_kernel<BLOCK, OWN, 24, R>;
            return nullptr;
        case 32:
            // h and acc do not fit the registers; no restricted instances at 32 modes
            if constexpr (OWN <= 10 && BLOCK < 768 && !R) return (void*)&fused_bwd_kernel<BLOCK, OWN, 32, R>;
            return nullptr;
    }
    return nullptr;
}

#ifdef SLOS_FUSED_RESTRICTED_INSTANCES
}  // namespace

// The adjoint instances for restricted spaces (workgroups of 256 and 512,
// at most 24 modes); this translation unit holds only them.
void* pick_bwd_restricted(int block, int m, int64_t Np) {
    const int own = own_for(block, Np);
    const int mm = mmax_for(m);
    if (mm > 24) return nullptr;
    if (block == 256) {
        switch (own) {
            case 1: return bwd_by_m<256, 1, true>(mm);
            case 2: return bwd_by_m<256, 2, true>(mm);
            case 4: return bwd_by_m<256, 4, true>(mm);
        }
    } else if (block == 512) {
        switch (own) {
            case 4: return bwd_by_m<512, 4, true>(mm);
            case 10: return bwd_by_m<512, 10, true>(mm);
            case 18: return bwd_by_m<512, 18, true>(mm);
        }
    }
    return nullptr;
}

}  // namespace slos
#else

int64_t lds_fwd_states(const slos_plan_s& P, int n_max) {
    int64_t S = 0;
    for (int k = 1; k <= n_max - 1; ++k) S = std::max<int64_t>(S, (k >= 2 ? P.N[k - 1] : 0) + P.N[k]);
    return S;
}

int64_t lds_bwd_states(const slos_plan_s& P, int n_max) {
    if (n_max < 2) return 0;
    int64_t S = lds_fwd_states(P, n_max);
    const int64_t Np = P.N[n_max - 1];
    S = std::max<int64_t>(S, 2 * Np);
    int64_t R = Np;
    for (int k = 0; k <= n_max - 2; ++k) R += P.N[k];
    S = std::max<int64_t>(S, R + P.N[n_max - 2]);
    return S;
}

// every layer's predecessor entries must be compact (LDS byte offsets)
bool compact_tables(const slos_plan_s& P, int n_max) {
    for (int k = 1; k <= n_max && k < (int)P.layers.size(); ++k)
        if (P.layers[k].pred_shift != kPredShiftCompact) return false;
    return true;
}

template <int BLOCK>
void* fwd_fn(int epi) {
    return epi == 0   ? (void*)&fused_fwd_kernel<BLOCK, 0>
           : epi == 1 ? (void*)&fused_fwd_kernel<BLOCK, 1>
           : epi == 2 ? (void*)&fused_fwd_kernel<BLOCK, 2>
           : epi == 3 ? (void*)&fused_fwd_kernel<BLOCK, 3>
                      : (void*)&fused_fwd_kernel<BLOCK, 4>;
}

void* pick_fwd(int block, int epi) {
    switch (block) {
        case 256: return fwd_fn<256>(epi);
        case 512: return fwd_fn<512>(epi);
        case 1024: return fwd_fn<1024>(epi);
        default: return nullptr;
    }
}

// LDS bytes of the fused forward: the coefficient column, the state
// buffers and, for the expectation epilogues, [m][block] float
// accumulators; for the click-pattern epilogue, a run's probabilities
size_t fwd_lds_for(const slos_plan_s& P, int n_max, int block, bool expect, bool thr = false) {
    return (size_t)(lds_fwd_states(P, n_max) + kUcolSlots) * sizeof(float2) +
           (expect ? (size_t)P.m * block * sizeof(float) : 0) + (thr ? (size_t)kThrChunkStates * sizeof(float) : 0);
}

void* pick_bwd(int block, int m, int64_t Np, bool restricted) {
    if (restricted) return pick_bwd_restricted(block, m, Np);
    const int own = own_for(block, Np);
    const int mm = mmax_for(m);
    if (block == 256) {
        switch (own) {
            case 1: return bwd_by_m<256, 1, false>(mm);
            case 2: return bwd_by_m<256, 2, false>(mm);
            case 4: return bwd_by_m<256, 4, false>(mm);
        }
    } else if (block == 512) {
        switch (own) {
            case 4: return bwd_by_m<512, 4, false>(mm);
            case 10: return bwd_by_m<512, 10, false>(mm);
            case 18: return bwd_by_m<512, 18, false>(mm);
        }
    } else if (block == 768) {
        if (own == 12) return bwd_by_m<768, 12, false>(mm);
    } else if (block == 1024) {
        if (own == 10) return bwd_by_m<1024, 10, false>(mm);
    }
    return nullptr;
}

size_t bwd_lds_for_block(const slos_plan_s& P, int n_max, int block) {
    // + the staged U [m][m] and the int rows (two minoff rows, the photon modes)
    const size_t rows = (size_t)(2 * (P.m + 1) + kMaxPhotons) * 4;
    return (size_t)(lds_bwd_states(P, n_max) + kUcolSlots + (block / 64) * 32 + kMaxPhotons * 32 + P.m * P.m) *
               sizeof(float2) + rows;
}

int grid_for(const slos_plan_s& P, const void* fn, int block, size_t lds, int B) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int g = per_cu * std::max(1, P.num_cu);
    return std::max(1, std::min(B, g));
}

}  // namespace

size_t fused_fwd_lds_bytes(const slos_plan_s& P, int n_max) {
    return (size_t)(lds_fwd_states(P, n_max) + kUcolSlots) * sizeof(float2);
}

size_t fused_bwd_lds_bytes(const slos_plan_s& P, int n_max) { return bwd_lds_for_block(P, n_max, 512); }

bool fused_fwd_supported(const slos_plan_s& P, int n_max, int block, std::string* why, bool expect) {
    if (block != 256 && block != 512 && block != 1024) {
        if (why) *why = "block must be 256, 512 or 1024";
        return false;
    }
    if (fwd_lds_for(P, n_max, block, expect) > P.max_lds) {
        if (why) *why = "photon layers do not fit in LDS";
        return false;
    }
    if (!compact_tables(P, n_max)) {
        if (why) *why = "photon layers too large for compact tables";
        return false;
    }
    return true;
}

bool fused_bwd_supported(const slos_plan_s& P, int n_max, int block, std::string* why) {
    if (block != 256 && block != 512 && block != 768 && block != 1024) {
        if (why) *why = "block must be 256, 512, 768 or 1024";
        return false;
    }
    if (!compact_tables(P, n_max)) {
        if (why) *why = "photon layers too large for compact tables";
        return false;
    }
    if (P.n_max >= 1 && P.layers.size() > 1 && P.layers[1].succ == nullptr) {
        if (why) *why = "plan has no successor tables";
        return false;
    }
    if (bwd_lds_for_block(P, n_max, block) > P.max_lds) {
        if (why) *why = "photon layers do not fit in LDS";
        return false;
    }
    if (n_max >= 2 && own_for(block, P.N[n_max - 1]) < 0) {
        if (why) *why = "layer n-1 too large for the register-resident adjoint at this block size";
        return false;
    }
    if (n_max >= 2 && pick_bwd(block, P.m, P.N[n_max - 1], restricted_plan(P)) == nullptr) {
        if (why) *why = "no register-resident adjoint for this block size and mode count";
        return false;
    }
    return true;
}

int fused_default_block(const slos_plan_s& P, int n_max, bool backward) {
    if (backward) {
        const int64_t Np = n_max >= 2 ? P.N[n_max - 1] : 1;
        // restricted spaces have adjoint instances at 256 and 512 threads only
        return Np <= 1024 ? 256 : (Np <= 5120 || P.m > 20 || restricted_plan(P)) ? 512 : 768;
    }
    const int64_t Nbig = n_max >= 1 ? P.N[n_max] : 1;
    return Nbig >= 8192 ? 1024 : 256;
}

bool fused_threshold_supported(const slos_plan_s& P, int n_max, int block) {
    return fused_fwd_supported(P, n_max, block, nullptr) && P.layers.size() > (size_t)n_max &&
           (n_max == 0 || P.layers[n_max].thr_chunk != nullptr) &&
           fwd_lds_for(P, n_max, block, false, true) <= P.max_lds;
}

int launch_fused_fwd(const slos_batch_s& Bt, int block, const float2* U, void* out, int epi,
                     hipStream_t stream) {
    const slos_plan_s& P = *Bt.plan;
    std::string why;
    const bool expect = epi == 2 || epi == 3, thr = epi == 4;
    if (!fused_fwd_supported(P, Bt.n_max, block, &why, expect))
        return fail(SLOS_EUNSUPPORTED, "fused forward: " + why);
    if (thr && !fused_threshold_supported(P, Bt.n_max, block))
        return fail(SLOS_EUNSUPPORTED, "fused forward: click-pattern runs do not fit in LDS");
    void* fn = pick_fwd(block, epi);
    const size_t lds = fwd_lds_for(P, Bt.n_max, block, expect, thr);
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int grid = grid_for(P, fn, block, lds, Bt.B);
    const int S = (int)lds_fwd_states(P, Bt.n_max);
    void* args[] = {(void*)&P.m, (void*)&P.d_layers, (void*)&Bt.dev, (void*)&U, (void*)&out, (void*)&S};
    hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("fused forward launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

int launch_fused_bwd(const slos_batch_s& Bt, int block, const float2* U, const void* gin, bool probs,
                     float2* gU, hipStream_t stream) {
    const slos_plan_s& P = *Bt.plan;
    std::string why;
    if (!fused_bwd_supported(P, Bt.n_max, block, &why)) return fail(SLOS_EUNSUPPORTED, "fused backward: " + why);
    const int64_t Np = Bt.n_max >= 2 ? P.N[Bt.n_max - 1] : 1;
    void* fn = pick_bwd(block, P.m, Np, restricted_plan(P));
    if (!fn) return fail(SLOS_EUNSUPPORTED, "fused backward: no kernel instance for this shape");
    const size_t base = bwd_lds_for_block(P, Bt.n_max, block);
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.max_lds);
    // keep the smallest layers d_0..d_KR in LDS between the first recompute and
    // the lower layers' pulls, as far as the spare LDS allows without fewer
    // workgroups per CU
    int KR = -1;
    int64_t kept = 0;
    size_t lds = base;
    if (Bt.n_max >= 2) {
        int per_base = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_base, fn, block, base) != hipSuccess)
            per_base = 1 << 30;  // unknown: keep no layers
        int64_t r = 0;
        for (int K = 0; K <= Bt.n_max - 2; ++K) {
            r += P.N[K];
            const size_t l = base + (size_t)r * sizeof(float2);
            int pc = 0;
            if (l > P.max_lds || hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, fn, block, l) != hipSuccess ||
                pc < per_base)
                break;
            KR = K;
            kept = r;
            lds = l;
        }
    }
    const int grid = grid_for(P, fn, block, lds, Bt.B);
    const int S = (int)(lds_bwd_states(P, Bt.n_max) + kept);
    int pr = probs ? 1 : 0;
    void* args[] = {(void*)&P.m, (void*)&P.d_layers, (void*)&Bt.dev, (void*)&U, (void*)&gin, (void*)&gU,
                    (void*)&S, (void*)&pr, (void*)&KR};
    hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("fused backward launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

}  // namespace slos
#endif  // SLOS_FUSED_RESTRICTED_INSTANCES
