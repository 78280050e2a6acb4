// Forward recursion for two samples per workgroup (arXiv 2602.11092,
// Sec. II-A-2 and II-A-3; amplitudes and probabilities as normalised
// permanents, Sec. II-A-1).
//
// A work item is a pair of samples with the same photon number (consecutive
// in the largest-first work order; a sample without a partner is processed
// alone).  The pair shares the transition graph of every photon layer, so
// each table entry is loaded and decoded once for both samples.  Their
// layers sit interleaved in LDS, 16 bytes per state (A.re, A.im, B.re, B.im),
// and so does the coefficient column (U_A[j][i_k^A], U_B[j][i_k^B]): one
// 128-bit LDS read returns both samples' predecessor amplitudes, another both
// coefficients.  On gfx950 a 128-bit LDS read issues at the rate of a 64-bit
// one, so the pair needs half the LDS reads of two single-sample passes.
//
// Layers 1..n-1 alternate between the two ends of the state buffer (layer
// n-1 at its start); the last layer streams to HBM.  When the two largest
// layers do not both fit, the few states of layer k whose slots meet layer
// k-1's are computed first, held in registers (one per thread), and written
// once the workgroup has finished reading layer k-1.  No atomics: results are
// bitwise reproducible, and equal to the single-sample kernel's (the same
// operations in the same order).
#include <type_traits>

#include "slos_internal.h"

namespace slos {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) f4v lds_f4v;
__device__ __forceinline__ f4v lds_ld4(uint32_t a) { return *(const lds_f4v*)(size_t)a; }
__device__ __forceinline__ void lds_st4(uint32_t a, f4v v) { *(lds_f4v*)(size_t)a = v; }

constexpr uint32_t kCol2Addr = 0;                         // [33] coefficient pairs; slot 32 stays zero
constexpr uint32_t kX2Addr = (uint32_t)kUcolSlots * 16u;  // state pairs
constexpr int kSU2 = 4;                                    // lower layers: states per thread per iteration
constexpr int kLP2 = 2;                                    // states whose gathers issue together
// A compact entry (mode << 25) | (rank << 3) gives the 16-byte coefficient
// slot as e >> 21 when the rank is below 2^18, and the 16-byte state slot
// as (e & 0x3FFFF8) << 1.
constexpr int64_t kPairRanks = (int64_t)1 << 18;

__device__ __forceinline__ uint32_t comp4(const uint4& e, int q) { return q == 0 ? e.x : q == 1 ? e.y : q == 2 ? e.z : e.w; }

// acc += c d for both samples of the pair
__device__ __forceinline__ void c2_fma(f4v& acc, f4v c, f4v d) {
    acc.x = fmaf(c.x, d.x, acc.x);
    acc.x = fmaf(-c.y, d.y, acc.x);
    acc.y = fmaf(c.x, d.y, acc.y);
    acc.y = fmaf(c.y, d.x, acc.y);
    acc.z = fmaf(c.z, d.z, acc.z);
    acc.z = fmaf(-c.w, d.w, acc.z);
    acc.w = fmaf(c.z, d.w, acc.w);
    acc.w = fmaf(c.w, d.z, acc.w);
}

// Entries q < NQ of predecessor group h for states u0 .. u0+SP-1, all LDS
// reads issued before the multiply-adds.
template <int SU, int NG, int SP, int NQ>
__device__ __forceinline__ void gather2_group(const uint4 (&e)[SU][NG], int h, int u0, uint32_t pb,
                                              f4v (&acc)[SU]) {
    f4v cv[NQ][SP], dv[NQ][SP];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int v = 0; v < SP; ++v) {
            const uint32_t x = comp4(e[u0 + v][h], q);
            cv[q][v] = lds_ld4(kCol2Addr + (x >> 21));
            dv[q][v] = lds_ld4(pb + ((x & kPredCompactRankMask) << 1));
        }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int v = 0; v < SP; ++v) c2_fma(acc[u0 + v], cv[q][v], dv[q][v]);
}

template <int SU, int SP, int NGX>
__device__ __forceinline__ void gather2_loaded(const uint4 (&e)[SU][NGX], int g0, int k, uint32_t pb,
                                               f4v (&acc)[SU]) {
#pragma unroll
    for (int h = 0; h < NGX; ++h) {
        const int valid = k - 4 * (g0 + h);  // entries of this group that exist (uniform)
#pragma unroll
        for (int u0 = 0; u0 < SU; u0 += SP) {
            if (valid >= 4) gather2_group<SU, NGX, SP, 4>(e, h, u0, pb, acc);
            else if (valid == 3) gather2_group<SU, NGX, SP, 3>(e, h, u0, pb, acc);
            else if (valid == 2) gather2_group<SU, NGX, SP, 2>(e, h, u0, pb, acc);
            else gather2_group<SU, NGX, SP, 1>(e, h, u0, pb, acc);
        }
    }
}

// acc[u] = the pair's d_k[t0 + u*BLOCK] (u < SU), pulled from layer k-1 at
// LDS address pb.  Lanes past tlim compute state tlim-1 (callers do not store it).
// KC > 0: k is KC, known when compiling, so every predecessor group's entry
// count is a constant and no branch on it remains.
template <int BLOCK, int SU, int SPR, int KC = 0>
__device__ __forceinline__ void gather2_states(const LayerDev& L, int k, int t0, int tlim, uint32_t pb,
                                               f4v (&acc)[SU]) {
    constexpr int SP = SPR < SU ? SPR : SU;
    static_assert(SU % SP == 0, "states must split evenly into gather sets");
#pragma unroll
    for (int u = 0; u < SU; ++u) acc[u] = f4v{0.f, 0.f, 0.f, 0.f};
    if ((KC > 0 ? KC : k) == 1) {  // d_1[t] = U[t][i_1]
#pragma unroll
        for (int u = 0; u < SU; ++u) acc[u] = lds_ld4(kCol2Addr + 16u * (uint32_t)min(t0 + u * BLOCK, tlim - 1));
        return;
    }
    const uint32_t gstride = (uint32_t)L.N * 16u;
    const __amdgpu_buffer_rsrc_t r = buf_rsrc(L.predv, (uint32_t)L.ngrp * gstride);
    uint32_t vo[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) vo[u] = (uint32_t)min(t0 + u * BLOCK, tlim - 1) * 16u;
    if constexpr (KC > 0) {
        constexpr int NGRP = (KC + 3) / 4;  // the table's predecessor groups for layer KC
#pragma unroll
        for (int g0 = 0; g0 + 2 <= NGRP; g0 += 2) {
            uint4 e[SU][2];
#pragma unroll
            for (int u = 0; u < SU; ++u)
#pragma unroll
                for (int h = 0; h < 2; ++h) e[u][h] = buf_ld4(r, vo[u], (uint32_t)(g0 + h) * gstride);
            gather2_loaded<SU, SP, 2>(e, g0, KC, pb, acc);
        }
        if constexpr (NGRP % 2 == 1) {
            uint4 e[SU][1];
#pragma unroll
            for (int u = 0; u < SU; ++u) e[u][0] = buf_ld4(r, vo[u], (uint32_t)(NGRP - 1) * gstride);
            gather2_loaded<SU, SP, 1>(e, NGRP - 1, KC, pb, acc);
        }
    } else {
        int g0 = 0;
        for (; g0 + 2 <= L.ngrp; g0 += 2) {
            uint4 e[SU][2];
#pragma unroll
            for (int u = 0; u < SU; ++u)
#pragma unroll
                for (int h = 0; h < 2; ++h) e[u][h] = buf_ld4(r, vo[u], (uint32_t)(g0 + h) * gstride);
            gather2_loaded<SU, SP, 2>(e, g0, k, pb, acc);
        }
        for (; g0 < L.ngrp; ++g0) {
            uint4 e[SU][1];
#pragma unroll
            for (int u = 0; u < SU; ++u) e[u][0] = buf_ld4(r, vo[u], (uint32_t)g0 * gstride);
            gather2_loaded<SU, SP, 1>(e, g0, k, pb, acc);
        }
    }
}

// One lower layer for the pair, LDS to LDS.  States [hlo, hhi) of layer k
// (at most BLOCK of them) land on slots of layer k-1: they are computed
// first, held in registers, and stored after the workgroup has finished
// reading layer k-1.
template <int BLOCK>
__device__ __forceinline__ void layer2_into_lds(const LayerDev& L, int k, uint32_t prev, uint32_t cur, int hlo,
                                                int hhi) {
    const int N = (int)L.N;
    const int tid = threadIdx.x;
    const int th = hlo + tid;
    f4v held = f4v{0.f, 0.f, 0.f, 0.f};
    if (hhi > hlo) {  // uniform
        f4v a[1];
        gather2_states<BLOCK, 1, 1>(L, k, th, hhi, prev, a);
        held = a[0];
    }
    for (int t0 = tid; t0 < N; t0 += BLOCK * kSU2) {
        f4v acc[kSU2];
        gather2_states<BLOCK, kSU2, kLP2>(L, k, t0, N, prev, acc);
#pragma unroll
        for (int u = 0; u < kSU2; ++u) {
            const int t = t0 + u * BLOCK;
            if (t < N && (t < hlo || t >= hhi)) lds_st4(cur + 16u * (uint32_t)t, acc[u]);
        }
    }
    if (hhi > hlo) {  // uniform
        __syncthreads();
        if (th < hhi) lds_st4(cur + 16u * (uint32_t)th, held);
    }
}

__device__ __forceinline__ LayerDev layer2(const LayerDev* Ls, int k) {
    const LayerDev* p = Ls + k;
    LayerDev L;
    L.predv = ldc(&p->predv);
    L.nrm = ldc(&p->nrm);
    L.N = ldc(&p->N);
    L.ngrp = ldc(&p->ngrp);
    return L;
}

// State slots [start, start + size) of photon layer k of an n-photon sample
// in a buffer of C slots: layers alternate ends, layer n-1 at the start.
__host__ __device__ __forceinline__ int64_t layer_start(int n, int k, int64_t N_k, int64_t C) {
    return (((n - 1 - k) & 1) == 0) ? 0 : C - N_k;
}

// EPI 0: amplitudes, 1: probabilities ([out_len], each sample at its offset).
// TU: last-layer states per thread per iteration (the tile the autotuner picks).
template <int BLOCK, int EPI, int TU>
__global__ __launch_bounds__(BLOCK) void fused_pairs_fwd_kernel(int m, const LayerDev* __restrict__ Ls, BatchDev Bt,
                                                                const float2* __restrict__ U, void* __restrict__ out,
                                                                int C) {
    constexpr bool PROBS = EPI == 1;
    extern __shared__ f4v lds2[];
    const int tid = threadIdx.x;
    if (tid < kUcolSlots) lds_st4(kCol2Addr + 16u * tid, f4v{0.f, 0.f, 0.f, 0.f});  // slots m..32 stay zero
    for (int item = blockIdx.x; item < Bt.npairs; item += gridDim.x) {
        const int* pr = (const int*)(Bt.pairs + item);
        const int ba = ldc(pr), pb1 = ldc(pr + 1);
        const bool two = pb1 >= 0;
        const int bb = two ? pb1 : ba;
        const int n = ldc(Bt.n + ba);
        const int64_t offa = ldc(Bt.off + ba), offb = ldc(Bt.off + bb);
        const float ina = ldc(Bt.innorm + ba), inb = ldc(Bt.innorm + bb);
        const float2* Ua = U + (size_t)ba * m * m;
        const float2* Ub = U + (size_t)bb * m * m;
        const int32_t* ma = Bt.modes + (size_t)ba * kMaxPhotons;
        const int32_t* mb = Bt.modes + (size_t)bb * kMaxPhotons;
        if (n == 0) {
            if (tid == 0) {
                if (PROBS) {
                    ((float*)out)[offa] = 1.f;
                    if (two) ((float*)out)[offb] = 1.f;
                } else {
                    ((float2*)out)[offa] = make_float2(1.f, 0.f);
                    if (two) ((float2*)out)[offb] = make_float2(1.f, 0.f);
                }
            }
            continue;
        }
        for (int k = 1; k <= n; ++k) {
            if (tid < m) {
                const float2 ca = Ua[tid * m + ldc(ma + (k - 1))];
                const float2 cb = Ub[tid * m + ldc(mb + (k - 1))];
                lds_st4(kCol2Addr + 16u * tid, f4v{ca.x, ca.y, cb.x, cb.y});
            }
            __syncthreads();
            const LayerDev L = layer2(Ls, k);
            const int N = (int)L.N;
            if (k < n) {
                const int Np = (int)ldc(&Ls[k - 1].N);
                const int cs = (int)layer_start(n, k, N, C);
                const int ps = (int)layer_start(n, k - 1, Np, C);
                // states of layer k whose slots meet layer k-1's (layer 0 is not in LDS)
                int hlo = 0, hhi = 0;
                if (k >= 2) {
                    hlo = max(cs, ps) - cs;
                    hhi = max(min(cs + N, ps + Np) - cs, hlo);
                }
                layer2_into_lds<BLOCK>(L, k, kX2Addr + 16u * (uint32_t)ps, kX2Addr + 16u * (uint32_t)cs, hlo, hhi);
            } else {
                const __amdgpu_buffer_rsrc_t rn = buf_rsrc(L.nrm, (uint32_t)N * 4u);
                const __amdgpu_buffer_rsrc_t ra =
                    buf_rsrc(PROBS ? (const void*)((float*)out + offa) : (const void*)((float2*)out + offa),
                             (uint32_t)N * (PROBS ? 4u : 8u));
                const __amdgpu_buffer_rsrc_t rb =
                    buf_rsrc(PROBS ? (const void*)((float*)out + offb) : (const void*)((float2*)out + offb),
                             two ? (uint32_t)N * (PROBS ? 4u : 8u) : 0u);
                // the last layer, with the photon count as a compile-time constant
                // where it is small (no branch on a group's entry count)
                auto last_layer = [&](auto KCc) {
                    constexpr int KC = decltype(KCc)::value;
                    for (int t0 = tid; t0 < N; t0 += BLOCK * TU) {
                        float c[TU];
#pragma unroll
                        for (int u = 0; u < TU; ++u)
                            c[u] = buf_ldf(rn, (uint32_t)min(t0 + u * BLOCK, N - 1) * 4u, 0);
                        f4v acc[TU];
                        gather2_states<BLOCK, TU, kLP2, KC>(L, k, t0, N, kX2Addr, acc);
#pragma unroll
                        for (int u = 0; u < TU; ++u) {
                            const int t = t0 + u * BLOCK;
                            if (t >= N) continue;
                            const float cA = c[u] * ina, cB = c[u] * inb;
                            if (PROBS) {
                                const float pA = cA * cA * (acc[u].x * acc[u].x + acc[u].y * acc[u].y);
                                const float pB = cB * cB * (acc[u].z * acc[u].z + acc[u].w * acc[u].w);
                                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(pA), ra, t * 4, 0,
                                                                      kCpolStream);
                                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(pB), rb, t * 4, 0,
                                                                      kCpolStream);
                            } else {
                                typedef __attribute__((ext_vector_type(2))) unsigned int u2;
                                const float2 aA = make_float2(acc[u].x * cA, acc[u].y * cA);
                                const float2 aB = make_float2(acc[u].z * cB, acc[u].w * cB);
                                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, aA), ra, t * 8, 0,
                                                                      kCpolStream);
                                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, aB), rb, t * 8, 0,
                                                                      kCpolStream);
                            }
                        }
                    }
                };
                // (two states per thread only: with more, the unrolled gathers
                // of all their groups exceed the register budget)
                switch (TU == 2 ? k : 0) {
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
    }
}

// State slots the pair kernel needs for samples of up to n_max photons, and
// whether they fit `lds` bytes; *C receives the buffer size in slots.
bool pair_layout(const slos_plan_s& P, int n_max, int block, size_t lds, int64_t* C, std::string* why) {
    if (n_max < 1) {
        *C = 1;
        return true;
    }
    int64_t need = P.N[n_max - 1];
    for (int k = 2; k <= n_max - 1; ++k) need = std::max<int64_t>(need, P.N[k] + P.N[k - 1]);
    const int64_t room = (int64_t)(lds / 16) - kUcolSlots;
    if (need <= room) {
        *C = std::max<int64_t>(need, 1);
        return true;
    }
    if (P.N[n_max - 1] > room) {
        if (why) *why = "photon layer n-1 of two samples does not fit in LDS";
        return false;
    }
    // the buffer is full: states whose slots overlap the previous layer are held in registers
    for (int n = 2; n <= n_max; ++n)
        for (int k = 2; k <= n - 1; ++k) {
            const int64_t cs = layer_start(n, k, P.N[k], room), ps = layer_start(n, k - 1, P.N[k - 1], room);
            if (P.N[k] > room || P.N[k - 1] > room) {
                if (why) *why = "a photon layer of two samples does not fit in LDS";
                return false;
            }
            const int64_t ov = std::min(cs + P.N[k], ps + P.N[k - 1]) - std::max(cs, ps);
            if (ov > block) {
                if (why) *why = "two photon layers of two samples overlap by more states than threads";
                return false;
            }
        }
    *C = room;
    return true;
}

template <int BLOCK, int TU>
void* pairs_fn(bool probs) {
    return probs ? (void*)&fused_pairs_fwd_kernel<BLOCK, 1, TU> : (void*)&fused_pairs_fwd_kernel<BLOCK, 0, TU>;
}

template <int BLOCK>
void* pairs_fn_tile(bool probs, int tile) {
    return tile == 2 ? pairs_fn<BLOCK, 2>(probs) : tile == 8 ? pairs_fn<BLOCK, 8>(probs) : pairs_fn<BLOCK, 4>(probs);
}

}  // namespace

bool fused_pairs_supported(const slos_plan_s& P, int n_max, int block, std::string* why) {
    if (block != 512 && block != 1024) {
        if (why) *why = "block must be 512 or 1024";
        return false;
    }
    for (int k = 1; k <= n_max && k < (int)P.layers.size(); ++k)
        if (P.layers[k].pred_shift != kPredShiftCompact || P.N[k - 1] >= kPairRanks) {
            if (why) *why = "photon layers too large for the two-sample tables";
            return false;
        }
    int64_t C = 0;
    return pair_layout(P, n_max, block, P.max_lds, &C, why);
}

int launch_fused_pairs_fwd(const slos_batch_s& Bt, int block, int tile, const float2* U, void* out, bool probs,
                           hipStream_t stream) {
    const slos_plan_s& P = *Bt.plan;
    std::string why;
    if (!fused_pairs_supported(P, Bt.n_max, block, &why)) return fail(SLOS_EUNSUPPORTED, "fused pairs forward: " + why);
    int64_t C = 0;
    pair_layout(P, Bt.n_max, block, P.max_lds, &C, nullptr);
    const size_t lds = (size_t)(kUcolSlots + C) * 16;
    void* fn = block == 512 ? pairs_fn_tile<512>(probs, tile) : pairs_fn_tile<1024>(probs, tile);
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    const int grid = std::max(1, std::min(Bt.npairs, per_cu * std::max(1, P.num_cu)));
    int Ci = (int)C;
    void* args[] = {(void*)&P.m, (void*)&P.d_layers, (void*)&Bt.dev, (void*)&U, (void*)&out, (void*)&Ci};
    hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("fused pairs forward launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

}  // namespace slos
