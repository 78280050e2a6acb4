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
// it gathers g_k[t' + e_j] and the workgroup sums the G_U contributions per
// wave (DPP) into LDS.  The top layer is consumed in chunks of consecutive
// "smallest occupied mode" blocks: for a chunk of smallest modes [a, b) the
// pairs (t', j) whose successor falls in it are exactly
// {min(t') in [a,b), j >= a} and {min(t') >= b, a <= j < b}, two contiguous
// ranges of t', so the pull stays a plain gather from LDS.
#include "slos_internal.h"

namespace slos {
namespace {

constexpr int kSU = 2;     // states per thread per iteration in the gathers

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

// Sum over the 64 lanes of a wave in a fixed order; the result is uniform.
__device__ __forceinline__ float wave_total(float v) {
    v += dpp<0xB1>(v);        // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);        // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);       // row_half_mirror
    v += dpp<0x140>(v);       // row_mirror: every lane holds its row's sum
    v += dpp<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3: lane 63 holds the total
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ int comp(const int4& e, int q) { return q == 0 ? e.x : q == 1 ? e.y : q == 2 ? e.z : e.w; }

// The first NQ entries of predecessor group h for states u0..u0+SP-1,
// branch-free, so all their LDS reads issue before one wait.  Entries are byte
// offsets, (rank << 11) | (mode << 3); an empty entry names the zero slot of
// the coefficient column, so it needs no test.
template <int SU, int NG, int SP, int NQ>
__device__ __forceinline__ void gather_group(const int4 (&e)[SU][NG], int h, int u0, const float2* __restrict__ prev,
                                             const float2* __restrict__ ucol, float2 (&acc)[SU]) {
    const char* pb = (const char*)prev;
    const char* ub = (const char*)ucol;
    float2 uv[NQ][SP], dv[NQ][SP];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int v = 0; v < SP; ++v) {
            const unsigned x = (unsigned)comp(e[u0 + v][h], q);
            uv[q][v] = *(const float2*)(ub + (x & kPredModeMask));
            dv[q][v] = *(const float2*)(pb + ((x >> kPredRankShift) << 3));
        }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int v = 0; v < SP; ++v) c_fma(acc[u0 + v], uv[q][v], dv[q][v]);
}

// acc[u] = d_k[t0 + u*BLOCK] for u < SU (0 where t >= tlim), pulled from
// layer k-1 in LDS (prev) with coefficients ucol[j] = U[j][i_k].  The table
// entries of all SU states and NG groups are loaded first (many loads in
// flight), then the gathers run SP states at a time.
template <int BLOCK, int SU, int SPR, int NG>
__device__ __forceinline__ void gather_states(const LayerDev& L, int k, int t0, int tlim,
                                              const float2* __restrict__ prev, const float2* __restrict__ ucol,
                                              float2 (&acc)[SU]) {
    constexpr int SP = SPR < SU ? SPR : SU;
    static_assert(SU % SP == 0, "states must split evenly into gather sets");
#pragma unroll
    for (int u = 0; u < SU; ++u) acc[u] = c_zero();
    if (k == 1) {
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int t = t0 + u * BLOCK;
            if (t < tlim) acc[u] = ucol[t];
        }
        return;
    }
    const size_t N = (size_t)L.N;
    g_int4* pv = (g_int4*)L.predv;
    for (int g0 = 0; g0 < L.ngrp; g0 += NG) {
        int4 e[SU][NG];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int t = t0 + u * BLOCK;
#pragma unroll
            for (int h = 0; h < NG; ++h) {
                const int g = g0 + h;
                e[u][h] = make_int4(kPredEmpty, kPredEmpty, kPredEmpty, kPredEmpty);
                if (t < tlim && g < L.ngrp) {
                    g_int* q4 = (g_int*)(pv + (size_t)g * N + t);
                    e[u][h] = make_int4(q4[0], q4[1], q4[2], q4[3]);
                }
            }
        }
#pragma unroll
        for (int h = 0; h < NG; ++h) {
            const int valid = k - 4 * (g0 + h);  // entries of this group that exist (uniform)
#pragma unroll
            for (int u0 = 0; u0 < SU; u0 += SP) {
                if (valid >= 4) gather_group<SU, NG, SP, 4>(e, h, u0, prev, ucol, acc);
                else if (valid == 3) gather_group<SU, NG, SP, 3>(e, h, u0, prev, ucol, acc);
                else if (valid == 2) gather_group<SU, NG, SP, 2>(e, h, u0, prev, ucol, acc);
                else if (valid == 1) gather_group<SU, NG, SP, 1>(e, h, u0, prev, ucol, acc);
            }
        }
    }
}

constexpr int kLU = 4;  // states whose table entries are in flight per thread
constexpr int kLP = 2;  // states gathered together

// One layer of the recursion into LDS, SU states per thread per iteration.
template <int BLOCK, int SU = kLU>
__device__ __forceinline__ void layer_into_lds(const LayerDev& L, int k, const float2* __restrict__ prev,
                                               float2* __restrict__ cur, const float2* __restrict__ ucol) {
    const int N = (int)L.N;
    for (int t0 = threadIdx.x; t0 < N; t0 += BLOCK * SU) {
        float2 acc[SU];
        gather_states<BLOCK, SU, kLP, SU >= 4 ? 2 : 1>(L, k, t0, N, prev, ucol, acc);
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int t = t0 + u * BLOCK;
            if (t < N) cur[t] = acc[u];
        }
    }
}

// ------------------------------------------------------------------ forward

template <int BLOCK, bool PROBS>
__global__ __launch_bounds__(BLOCK) void fused_fwd_kernel(int m, const LayerDev* __restrict__ Ls, BatchDev Bt,
                                                          const float2* __restrict__ U, void* __restrict__ out,
                                                          int S) {
    extern __shared__ float2 lds[];
    float2* ucol = lds;               // [33] column i_k of U; slot 32 stays zero
    float2* X = lds + kUcolSlots;     // [S] photon layers
    const int tid = threadIdx.x;
    if (tid == 32) ucol[32] = c_zero();
    for (int item = blockIdx.x; item < Bt.B; item += gridDim.x) {
        const int b = ldg(Bt.order + (item));
        const int n = ldg(Bt.n + (b));
        const int64_t off = ldg(Bt.off + (b));
        const float innorm = ldg(Bt.innorm + (b));
        const float2* Ub = U + (size_t)b * m * m;
        const int32_t* modes = Bt.modes + (size_t)b * kMaxPhotons;  // read through ldg
        if (n == 0) {
            if (tid == 0) {
                if (PROBS) ((float*)out)[off] = 1.f;
                else ((float2*)out)[off] = make_float2(1.f, 0.f);
            }
            continue;
        }
        for (int k = 1; k <= n; ++k) {
            if (tid < m) ucol[tid] = Ub[tid * m + ldg(modes + (k - 1))];
            __syncthreads();
            const LayerDev L = Ls[k];
            const int N = (int)L.N;
            // layers alternate between the two ends of X; layer n-1 sits at offset 0
            if (k < n) {
                const float2* prev = X + ((((n - k) & 1) == 0) ? 0 : S - (int)Ls[k - 1].N);
                layer_into_lds<BLOCK>(L, k, prev, X + ((((n - 1 - k) & 1) == 0) ? 0 : S - N), ucol);
            } else {
                const float2* prev = X;
                for (int t0 = tid; t0 < N; t0 += BLOCK * kLU) {
                    float c[kLU];
#pragma unroll
                    for (int u = 0; u < kLU; ++u) {
                        const int t = t0 + u * BLOCK;
                        c[u] = (t < N) ? ldg(L.nrm + t) * innorm : 0.f;
                    }
                    float2 acc[kLU];
                    gather_states<BLOCK, kLU, kLP, 2>(L, k, t0, N, prev, ucol, acc);
#pragma unroll
                    for (int u = 0; u < kLU; ++u) {
                        const int t = t0 + u * BLOCK;
                        if (t < N) {
                            if (PROBS) ((float*)out)[off + t] = c[u] * c[u] * (acc[u].x * acc[u].x + acc[u].y * acc[u].y);
                            else ((float2*)out)[off + t] = c_scale(acc[u], c[u]);
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ backward

// Every thread owns states t' = tid + s*BLOCK (s < OWN) of layer k-1:
// acc[s] accumulates g_{k-1}[t'], and h[j] this lane's share of
// G_U[j][i_k] = sum_t' conj(d_{k-1}[t']) g_k[t' + e_j].  Lanes without work
// read the zero slot of the coefficient column instead of branching.

// t' in [lo, hi), every output mode j in [jlo, m): each owned state loads
// its successor row (16-byte loads) and issues all its gathers together.
template <int BLOCK, int OWN, int MMAX, int JC>
__device__ __forceinline__ void pull_wide(int lo, int hi, int jlo, int m, int MP, const int32_t* __restrict__ succ,
                                          const float2* __restrict__ src, int base, const float2* __restrict__ D,
                                          const float2* __restrict__ ucol, float2 (&acc)[OWN], float2 (&h)[MMAX]) {
    if (lo >= hi) return;
    const int tid = threadIdx.x;
    const int zidx = (int)(ucol + 32 - src);
    g_int* sg = (g_int*)succ;
#pragma unroll
    for (int s = 0; s < OWN; ++s) {
        if ((s + 1) * BLOCK <= lo || s * BLOCK >= hi) continue;  // no owned state in range (uniform)
        const int tp = tid + s * BLOCK;
        const bool act = tp >= lo && tp < hi;
        const int tr = act ? tp : lo;
        const float2 dv = D[tr];
#pragma unroll
        for (int j0 = 0; j0 < MMAX; j0 += JC) {
            if (j0 >= MP) continue;  // past the row (uniform; no break, so j0 stays a constant)
            int sv[JC];
#pragma unroll
            for (int q = 0; q < JC; q += 4) {
                if (j0 + q < MP) {
                    g_int* r = sg + (size_t)tr * MP + j0 + q;
                    sv[q] = r[0];
                    sv[q + 1] = r[1];
                    sv[q + 2] = r[2];
                    sv[q + 3] = r[3];
                } else {
                    sv[q] = sv[q + 1] = sv[q + 2] = sv[q + 3] = 0;
                }
            }
            float2 gv[JC];
#pragma unroll
            for (int q = 0; q < JC; ++q) {
                const int j = j0 + q;
                const bool ok = act && j >= jlo && j < m;
                gv[q] = src[ok ? sv[q] - base : zidx];
            }
#pragma unroll
            for (int q = 0; q < JC; ++q) {
                const float2 u = ucol[j0 + q];
                c_fma_conj(acc[s], u, gv[q]);
                c_fma_conj(h[j0 + q], dv, gv[q]);
            }
        }
    }
}

// t' in [lo, hi) (a long range) and output modes j in [jlo, jhi) (a few):
// per mode, all owned states gather together.
template <int BLOCK, int OWN, int MMAX>
__device__ __forceinline__ void pull_narrow(int lo, int hi, int jlo, int jhi, int MP,
                                            const int32_t* __restrict__ succ, const float2* __restrict__ src,
                                            int base, const float2* __restrict__ D, const float2* __restrict__ ucol,
                                            float2 (&acc)[OWN], float2 (&h)[MMAX]) {
    if (lo >= hi) return;
    const int tid = threadIdx.x;
    const int zidx = (int)(ucol + 32 - src);
    g_int* sg = (g_int*)succ;
#pragma unroll
    for (int j = 0; j < MMAX; ++j) {
        if (j < jlo || j >= jhi) continue;  // uniform
        const float2 u = ucol[j];
        int sidx[OWN];
#pragma unroll
        for (int s = 0; s < OWN; ++s) {
            const int tp = tid + s * BLOCK;
            sidx[s] = zidx;
            if ((s + 1) * BLOCK > lo && s * BLOCK < hi && tp >= lo && tp < hi)
                sidx[s] = sg[(size_t)tp * MP + j] - base;
        }
#pragma unroll
        for (int s = 0; s < OWN; ++s) {
            if ((s + 1) * BLOCK <= lo || s * BLOCK >= hi) continue;  // uniform
            const int tp = tid + s * BLOCK;
            const bool act = tp >= lo && tp < hi;
            const float2 gv = src[sidx[s]];
            const float2 dv = D[act ? tp : lo];
            c_fma_conj(acc[s], u, gv);
            c_fma_conj(h[j], dv, gv);
        }
    }
}

// Sums h[j] over the workgroup (per wave with DPP, then over waves in a fixed
// order) into GUcol[j] for j < m.  Hw: [NW][32] LDS scratch.
template <int BLOCK, int MMAX>
__device__ __forceinline__ void reduce_columns(const float2 (&h)[MMAX], int m, float2* __restrict__ Hw,
                                               float2* __restrict__ GUcol) {
    constexpr int NW = BLOCK / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int j = 0; j < MMAX; ++j) {
        if (j >= m) continue;
        const float re = wave_total(h[j].x);
        const float im = wave_total(h[j].y);
        if (lane == 0) Hw[wave * 32 + j] = make_float2(re, im);
    }
    __syncthreads();
    if (tid < m) {
        float2 sum = c_zero();
        for (int w = 0; w < NW; ++w) sum = c_add(sum, Hw[w * 32 + tid]);
        GUcol[tid] = sum;
    }
}

template <int BLOCK, int OWN, int MMAX>
__global__ __launch_bounds__(BLOCK) void fused_bwd_kernel(int m, const LayerDev* __restrict__ Ls, BatchDev Bt,
                                                          const float2* __restrict__ U,
                                                          const void* __restrict__ gin,
                                                          float2* __restrict__ gU, int S, int PROBS) {
    constexpr int NW = BLOCK / 64;
    constexpr int JC = 4;
    // states per thread in the gathers (register budget: acc and h stay live)
    constexpr int GU = OWN >= 10 ? 2 : kLU;
    constexpr int GM = OWN >= 10 ? 1 : kLU;
    extern __shared__ float2 lds[];
    float2* ucol = lds;                // [33] column i_k of U; slot 32 stays zero
    float2* X = lds + kUcolSlots;      // [S] layers / chunks
    float2* Hw = X + S;                // [NW][32] per-wave column sums
    float2* GUacc = Hw + NW * 32;      // [kMaxPhotons][32] gradient column per photon layer
    const int tid = threadIdx.x;
    if (tid == 32) ucol[32] = c_zero();
    const float* gp = (const float*)gin;
    const float2* ga = (const float2*)gin;
    const int MP = succ_row_len(m);

    for (int item = blockIdx.x; item < Bt.B; item += gridDim.x) {
        const int b = ldg(Bt.order + item);
        const int n = ldg(Bt.n + b);
        const int64_t off = ldg(Bt.off + b);
        const float innorm = ldg(Bt.innorm + b);
        const float2* Ub = U + (size_t)b * m * m;
        const int32_t* modes = Bt.modes + (size_t)b * kMaxPhotons;
        float2* gUb = gU + (size_t)b * m * m;

        for (int q = tid; q < kMaxPhotons * 32; q += BLOCK) GUacc[q] = c_zero();
        __syncthreads();

        if (n == 1) {
            // g_1[j] is G_U[j][i_1] itself (d_0 = 1)
            if (tid < m) {
                const float c = ldg(Ls[1].nrm + tid) * innorm;
                GUacc[tid] = PROBS ? c_scale(Ub[tid * m + ldg(modes)], 2.f * gp[off + tid] * c * c)
                                   : c_scale(ga[off + tid], c);
            }
            __syncthreads();
        } else if (n >= 2) {
            const LayerDev Ln = Ls[n];
            const LayerDev Lp = Ls[n - 1];
            const int Np = (int)Lp.N;
            // ---- recompute layers 1..n-1; layer n-1 ends at offset 0
            for (int k = 1; k <= n - 1; ++k) {
                if (tid < m) ucol[tid] = Ub[tid * m + ldg(modes + k - 1)];
                __syncthreads();
                const int Nk = (int)Ls[k].N;
                const int Nkm1 = (int)Ls[k - 1].N;
                layer_into_lds<BLOCK, GU>(Ls[k], k, X + ((((n - k) & 1) == 0) ? 0 : S - Nkm1),
                                      X + ((((n - 1 - k) & 1) == 0) ? 0 : S - Nk), ucol);
                __syncthreads();
            }
            // ---- top layer, in chunks of smallest-mode blocks
            if (tid < m) ucol[tid] = Ub[tid * m + ldg(modes + n - 1)];
            const float2* D = X;
            float2* C = X + Np;
            const int cap = S - Np;
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
                while (bb < m && ldg(Ln.minoff + bb + 1) - ldg(Ln.minoff + a) <= cap) ++bb;
                const int base = ldg(Ln.minoff + a);
                const int end = ldg(Ln.minoff + bb);
                // g_n on the chunk.  First the per-state factors (a streaming
                // pass with independent loads): 2 dL/dp_t c_t^2 (probabilities,
                // kept in .x) or c_t G_a[t] (amplitudes, final).  Then, for
                // probabilities, d_n[t] from layer n-1; each thread revisits
                // exactly the states it wrote, so no barrier is needed between.
                for (int t0 = base + tid; t0 < end; t0 += BLOCK * 4) {
                    float cv[4];
                    float2 gv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int t = t0 + u * BLOCK;
                        cv[u] = (t < end) ? ldg(Ln.nrm + t) * innorm : 0.f;
                        gv[u] = c_zero();
                        if (t < end) gv[u] = PROBS ? make_float2(gp[off + t], 0.f) : ga[off + t];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int t = t0 + u * BLOCK;
                        if (t < end)
                            C[t - base] = PROBS ? make_float2(2.f * gv[u].x * cv[u] * cv[u], 0.f) : c_scale(gv[u], cv[u]);
                    }
                }
                if (PROBS) {
                    for (int t0 = base + tid; t0 < end; t0 += BLOCK * GM) {
                        float2 d[GM];
                        gather_states<BLOCK, GM, kLP, GM >= 4 ? 2 : 1>(Ln, n, t0, end, D, ucol, d);
#pragma unroll
                        for (int u = 0; u < GM; ++u) {
                            const int t = t0 + u * BLOCK;
                            if (t < end) C[t - base] = c_scale(d[u], C[t - base].x);
                        }
                    }
                }
                __syncthreads();
                // {min(t') in [a, bb), j >= a} and {min(t') >= bb, a <= j < bb}
                pull_wide<BLOCK, OWN, MMAX, JC>(ldg(Lp.minoff + a), ldg(Lp.minoff + bb), a, m, MP, Ln.succ, C,
                                                base, D, ucol, acc, h);
                pull_narrow<BLOCK, OWN, MMAX>(ldg(Lp.minoff + bb), Np, a, bb, MP, Ln.succ, C, base, D, ucol, acc,
                                              h);
                __syncthreads();
                a = bb;
            }
            // g_{n-1} replaces d_{n-1}; the top layer's column of G_U
#pragma unroll
            for (int s = 0; s < OWN; ++s) {
                const int tp = tid + s * BLOCK;
                if (tp < Np) X[tp] = acc[s];
            }
            reduce_columns<BLOCK, MMAX>(h, m, Hw, GUacc + (n - 1) * 32);
            // ---- lower layers.  d_0..d_{n-2} stored after g_{n-1} (layer k at
            // Np + number of states with < k photons); g ping-pongs between 0 and R.
            const int R = Np + (int)Ls[n - 1].cum;
            if (tid == 0) X[Np] = make_float2(1.f, 0.f);
            __syncthreads();
            for (int k = 1; k <= n - 2; ++k) {
                if (tid < m) ucol[tid] = Ub[tid * m + ldg(modes + k - 1)];
                __syncthreads();
                layer_into_lds<BLOCK, GU>(Ls[k], k, X + Np + (int)Ls[k - 1].cum, X + Np + (int)Ls[k].cum, ucol);
                __syncthreads();
            }
            for (int k = n - 1; k >= 1; --k) {
                if (tid < m) ucol[tid] = Ub[tid * m + ldg(modes + k - 1)];
                const float2* gk = X + ((((n - 1 - k) & 1) == 0) ? 0 : R);
                float2* gkm1 = X + ((((n - k) & 1) == 0) ? 0 : R);
                const float2* dkm1 = X + Np + (int)Ls[k - 1].cum;
                const int Nkm1 = (int)Ls[k - 1].N;
#pragma unroll
                for (int s = 0; s < OWN; ++s) acc[s] = c_zero();
#pragma unroll
                for (int j = 0; j < MMAX; ++j) h[j] = c_zero();
                __syncthreads();
                pull_wide<BLOCK, OWN, MMAX, JC>(0, Nkm1, 0, m, MP, Ls[k].succ, gk, 0, dkm1, ucol, acc, h);
                if (k >= 2) {
#pragma unroll
                    for (int s = 0; s < OWN; ++s) {
                        const int tp = tid + s * BLOCK;
                        if (tp < Nkm1) gkm1[tp] = acc[s];
                    }
                }
                reduce_columns<BLOCK, MMAX>(h, m, Hw, GUacc + (k - 1) * 32);
                __syncthreads();
            }
        }
        // assemble G_U[b]: column i collects the layers whose photon sits in mode i
        __syncthreads();
        for (int q = tid; q < m * m; q += BLOCK) {
            const int j = q / m, i = q % m;
            float2 v = c_zero();
            for (int k = 1; k <= n; ++k)
                if (ldg(modes + k - 1) == i) v = c_add(v, GUacc[(k - 1) * 32 + j]);
            gUb[q] = v;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host side

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

// photon-layer-(n-1) states per thread in the register-resident pulls
int own_for(int block, int64_t Np) {
    const int64_t need = (Np + block - 1) / block;
    if (block == 256) return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : -1;
    if (block == 512) return need <= 4 ? 4 : need <= 10 ? 10 : need <= 18 ? 18 : -1;
    return -1;
}

template <int BLOCK, bool PROBS>
void* fwd_fn() { return (void*)&fused_fwd_kernel<BLOCK, PROBS>; }

void* pick_fwd(int block, bool probs) {
    switch (block) {
        case 256: return probs ? fwd_fn<256, true>() : fwd_fn<256, false>();
        case 512: return probs ? fwd_fn<512, true>() : fwd_fn<512, false>();
        case 1024: return probs ? fwd_fn<1024, true>() : fwd_fn<1024, false>();
        default: return nullptr;
    }
}

int mmax_for(int m) { const int r = succ_row_len(m); return r <= 8 ? 8 : r <= 12 ? 12 : r <= 16 ? 16 : r <= 20 ? 20 : r <= 24 ? 24 : 32; }

template <int BLOCK, int OWN>
void* bwd_by_m(int mm) {
    switch (mm) {
        case 8: return (void*)&fused_bwd_kernel<BLOCK, OWN, 8>;
        case 12: return (void*)&fused_bwd_kernel<BLOCK, OWN, 12>;
        case 16: return (void*)&fused_bwd_kernel<BLOCK, OWN, 16>;
        case 20: return (void*)&fused_bwd_kernel<BLOCK, OWN, 20>;
        case 24: return (void*)&fused_bwd_kernel<BLOCK, OWN, 24>;
        case 32: return (void*)&fused_bwd_kernel<BLOCK, OWN, 32>;
    }
    return nullptr;
}

void* pick_bwd(int block, int m, int64_t Np) {
    const int own = own_for(block, Np);
    const int mm = mmax_for(m);
    if (block == 256) {
        switch (own) {
            case 1: return bwd_by_m<256, 1>(mm);
            case 2: return bwd_by_m<256, 2>(mm);
            case 4: return bwd_by_m<256, 4>(mm);
        }
    } else if (block == 512) {
        switch (own) {
            case 4: return bwd_by_m<512, 4>(mm);
            case 10: return bwd_by_m<512, 10>(mm);
            case 18: return bwd_by_m<512, 18>(mm);
        }
    }
    return nullptr;
}

size_t bwd_lds_for_block(const slos_plan_s& P, int n_max, int block) {
    return (size_t)(lds_bwd_states(P, n_max) + kUcolSlots + (block / 64) * 32 + kMaxPhotons * 32) * sizeof(float2);
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

bool fused_fwd_supported(const slos_plan_s& P, int n_max, int block, std::string* why) {
    if (block != 256 && block != 512 && block != 1024) {
        if (why) *why = "block must be 256, 512 or 1024";
        return false;
    }
    if (fused_fwd_lds_bytes(P, n_max) > P.max_lds) {
        if (why) *why = "photon layers do not fit in LDS";
        return false;
    }
    return true;
}

bool fused_bwd_supported(const slos_plan_s& P, int n_max, int block, std::string* why) {
    if (block != 256 && block != 512) {
        if (why) *why = "block must be 256 or 512";
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
    return true;
}

int fused_default_block(const slos_plan_s& P, int n_max, bool backward) {
    if (backward) return (n_max >= 2 && P.N[n_max - 1] > 1024) ? 512 : 256;
    const int64_t Nbig = n_max >= 1 ? P.N[n_max] : 1;
    return Nbig >= 8192 ? 1024 : 256;
}

int launch_fused_fwd(const slos_batch_s& Bt, int block, const float2* U, void* out, bool probs,
                     hipStream_t stream) {
    const slos_plan_s& P = *Bt.plan;
    std::string why;
    if (!fused_fwd_supported(P, Bt.n_max, block, &why)) return fail(SLOS_EUNSUPPORTED, "fused forward: " + why);
    void* fn = pick_fwd(block, probs);
    const size_t lds = fused_fwd_lds_bytes(P, Bt.n_max);
    hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
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
    void* fn = pick_bwd(block, P.m, Np);
    if (!fn) return fail(SLOS_EUNSUPPORTED, "fused backward: no kernel instance for this shape");
    const size_t lds = bwd_lds_for_block(P, Bt.n_max, block);
    hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int grid = grid_for(P, fn, block, lds, Bt.B);
    const int S = (int)lds_bwd_states(P, Bt.n_max);
    int pr = probs ? 1 : 0;
    void* args[] = {(void*)&P.m, (void*)&P.d_layers, (void*)&Bt.dev, (void*)&U, (void*)&gin, (void*)&gU,
                    (void*)&S, (void*)&pr};
    hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("fused backward launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

}  // namespace slos
