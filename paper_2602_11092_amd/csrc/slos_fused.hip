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
// the precomputed transition tables; no atomics, so results are bitwise
// reproducible.
//
// Backward (adjoint of the recursion): with G the gradient convention
// dL/dRe + i dL/dIm,
//   g_n[t]      = 2 dL/dp_t c_t^2 d_n[t]    (probabilities, c_t = sqrt(prod t!/prod s!))
//               = c_t G_a[t]                (amplitudes)
//   g_{k-1}[t'] = sum_j conj(U[j][i_k]) g_k[t' + e_j]
//   G_U[j][i_k] += sum_t' conj(d_{k-1}[t']) g_k[t' + e_j]
// Layers are recomputed rather than stored.  The top layer is processed in
// chunks of consecutive "smallest occupied mode" blocks; for a chunk of
// smallest modes [a, b) the (t', j) pairs whose successor falls in it are
// exactly {min(t') in [a,b), j >= a} and {min(t') >= b, a <= j < b}, both
// contiguous ranges of t', so the pull over t' stays a plain gather.
#include "slos_internal.h"

namespace slos {
namespace {

constexpr int kUcol = 32;  // LDS slots for one column of U

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float half_wave_sum(float v) {
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 32);
    return v;
}
__device__ __forceinline__ float uniform_f(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// One pass of the recursion into LDS: cur[t] = sum_p ucol[j_p] prev[pred_p].
template <int BLOCK>
__device__ __forceinline__ void layer_pull(const LayerDev& L, int k, const float2* __restrict__ prev,
                                           float2* __restrict__ cur, const float2* __restrict__ ucol) {
    const int N = (int)L.N;
    if (k == 1) {
        for (int t = threadIdx.x; t < N; t += BLOCK) cur[t] = ucol[t];
        return;
    }
    for (int t = threadIdx.x; t < N; t += BLOCK) {
        float2 acc = c_zero();
        for (int p = 0; p < k; ++p) {
            const int e = L.pred[(size_t)p * N + t];
            if (e >= 0) c_fma(acc, ucol[e & 31], prev[e >> kModeBits]);
        }
        cur[t] = acc;
    }
}

// ------------------------------------------------------------------ forward

template <int BLOCK, bool PROBS>
__global__ __launch_bounds__(BLOCK) void fused_fwd_kernel(int m, const LayerDev* __restrict__ Ls, BatchDev Bt,
                                                          const float2* __restrict__ U, void* __restrict__ out,
                                                          int S) {
    extern __shared__ float2 lds[];
    float2* ucol = lds + S;
    const int tid = threadIdx.x;
    for (int item = blockIdx.x; item < Bt.B; item += gridDim.x) {
        const int b = Bt.order[item];
        const int n = Bt.n[b];
        const int64_t off = Bt.off[b];
        const float innorm = Bt.innorm[b];
        const float2* Ub = U + (size_t)b * m * m;
        const int32_t* modes = Bt.modes + (size_t)b * kMaxPhotons;
        if (n == 0) {
            if (tid == 0) {
                if (PROBS) ((float*)out)[off] = 1.f;
                else ((float2*)out)[off] = make_float2(1.f, 0.f);
            }
            continue;
        }
        for (int k = 1; k <= n; ++k) {
            const int ik = modes[k - 1];
            if (tid < m) ucol[tid] = Ub[tid * m + ik];
            __syncthreads();
            const LayerDev L = Ls[k];
            const int N = (int)L.N;
            const float2* prev = lds + ((((n - 1 - (k - 1)) & 1) == 0) ? 0 : S - (int)Ls[k - 1].N);
            if (k < n) {
                float2* cur = lds + ((((n - 1 - k) & 1) == 0) ? 0 : S - N);
                layer_pull<BLOCK>(L, k, prev, cur, ucol);
            } else {
                for (int t = tid; t < N; t += BLOCK) {
                    float2 acc = c_zero();
                    if (k == 1) {
                        acc = ucol[t];
                    } else {
                        for (int p = 0; p < k; ++p) {
                            const int e = L.pred[(size_t)p * N + t];
                            if (e >= 0) c_fma(acc, ucol[e & 31], prev[e >> kModeBits]);
                        }
                    }
                    const float c = L.nrm[t] * innorm;
                    if (PROBS) {
                        ((float*)out)[off + t] = c * c * (acc.x * acc.x + acc.y * acc.y);
                    } else {
                        ((float2*)out)[off + t] = c_scale(acc, c);
                    }
                }
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ backward

template <int BLOCK, int MMAX, int OWN>
__global__ __launch_bounds__(BLOCK) void fused_bwd_kernel(int m, const LayerDev* __restrict__ Ls, BatchDev Bt,
                                                          const float2* __restrict__ U,
                                                          const void* __restrict__ gin,
                                                          float2* __restrict__ gU, int S, int PROBS) {
    constexpr int NW = BLOCK / 64;
    constexpr int NG = BLOCK / 32;
    extern __shared__ float2 lds[];
    float2* X = lds;                 // [S] layers / chunks
    float2* ucol = X + S;            // [32]
    float2* scratch = ucol + kUcol;  // [BLOCK] reduction scratch
    float2* GUacc = scratch + BLOCK; // [kMaxPhotons][32] gradient column per photon layer
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    for (int item = blockIdx.x; item < Bt.B; item += gridDim.x) {
        const int b = Bt.order[item];
        const int n = Bt.n[b];
        const int64_t off = Bt.off[b];
        const float innorm = Bt.innorm[b];
        const float2* Ub = U + (size_t)b * m * m;
        const int32_t* modes = Bt.modes + (size_t)b * kMaxPhotons;
        float2* gUb = gU + (size_t)b * m * m;

        for (int q = tid; q < kMaxPhotons * 32; q += BLOCK) GUacc[q] = c_zero();
        __syncthreads();

        if (n == 1) {
            // g_1[j] seeds G_U[j][i_1] directly (d_0 = 1)
            const int i1 = modes[0];
            if (tid < m) {
                const float2 u = Ub[tid * m + i1];
                const float c = Ls[1].nrm[tid] * innorm;
                float2 g;
                if (PROBS) {
                    const float w = 2.f * ((const float*)gin)[off + tid] * c * c;
                    g = c_scale(u, w);
                } else {
                    g = c_scale(((const float2*)gin)[off + tid], c);
                }
                GUacc[tid] = g;
            }
            __syncthreads();
        } else if (n >= 2) {
            const LayerDev Ln = Ls[n];
            const LayerDev Lp = Ls[n - 1];
            const int Np = (int)Lp.N;
            // ---- recompute layers 1..n-1; layer n-1 ends at offset 0
            for (int k = 1; k <= n - 1; ++k) {
                if (tid < m) ucol[tid] = Ub[tid * m + modes[k - 1]];
                __syncthreads();
                const int Nk = (int)Ls[k].N;
                const int Nkm1 = (int)Ls[k - 1].N;
                float2* cur = X + ((((n - 1 - k) & 1) == 0) ? 0 : S - Nk);
                const float2* prev = X + ((((n - 1 - (k - 1)) & 1) == 0) ? 0 : S - Nkm1);
                layer_pull<BLOCK>(Ls[k], k, prev, cur, ucol);
                __syncthreads();
            }
            // ---- top layer
            const int in_ = modes[n - 1];
            if (tid < m) ucol[tid] = Ub[tid * m + in_];
            const float2* D = X;
            float2* C = X + Np;
            const int cap = S - Np;
            float2 acc[OWN];
            float2 dreg[OWN];
#pragma unroll
            for (int s = 0; s < OWN; ++s) {
                const int tp = tid + s * BLOCK;
                acc[s] = c_zero();
                dreg[s] = (tp < Np) ? D[tp] : c_zero();
            }
            float2 h[MMAX];
#pragma unroll
            for (int j = 0; j < MMAX; ++j) h[j] = c_zero();
            __syncthreads();

            const float* gp = (const float*)gin;
            const float2* ga = (const float2*)gin;
            int a = 0;
            while (a < m) {
                int bb = a + 1;
                while (bb < m && Ln.minoff[bb + 1] - Ln.minoff[a] <= cap) ++bb;
                const int base = Ln.minoff[a];
                const int end = Ln.minoff[bb];
                // materialise g_n on the chunk
                for (int t = base + tid; t < end; t += BLOCK) {
                    const float c = Ln.nrm[t] * innorm;
                    float2 g;
                    if (PROBS) {
                        float2 d = c_zero();
                        for (int p = 0; p < n; ++p) {
                            const int e = Ln.pred[(size_t)p * Ln.N + t];
                            if (e >= 0) c_fma(d, ucol[e & 31], D[e >> kModeBits]);
                        }
                        g = c_scale(d, 2.f * gp[off + t] * c * c);
                    } else {
                        g = c_scale(ga[off + t], c);
                    }
                    C[t - base] = g;
                }
                __syncthreads();
                // pull: sub-pass 0 = {min(t') in [a,bb), j >= a}, sub-pass 1 = {min(t') >= bb, a <= j < bb}
#pragma unroll 1
                for (int sp = 0; sp < 2; ++sp) {
                    const int lo = sp == 0 ? Lp.minoff[a] : Lp.minoff[bb];
                    const int hi = sp == 0 ? Lp.minoff[bb] : Np;
                    const int jlo = a;
                    const int jhi = sp == 0 ? m : bb;
                    if (lo >= hi) continue;
#pragma unroll
                    for (int j = 0; j < MMAX; ++j) {
                        if (j < jlo || j >= jhi) continue;
                        // Rematerialise the row offset and reload u_j here: left to the
                        // compiler, all MMAX of them would be hoisted and kept live.
                        asm volatile("" ::: "memory");
                        int joff = j * Np;
                        asm volatile("" : "+s"(joff));
                        const int32_t* sj = Ln.succ + joff;
                        const float2 uj = ucol[j];  // same address on every lane
                        float2 hj = c_zero();
#pragma unroll
                        for (int s = 0; s < OWN; ++s) {
                            if ((s + 1) * BLOCK <= lo || s * BLOCK >= hi) continue;
                            const int tp = tid + s * BLOCK;
                            if (tp >= lo && tp < hi) {
                                const int cidx = sj[tp] - base;
                                if ((unsigned)cidx < (unsigned)(end - base)) {
                                    const float2 g = C[cidx];
                                    c_fma_conj(acc[s], uj, g);
                                    c_fma_conj(hj, dreg[s], g);
                                }
                            }
                        }
                        h[j] = c_add(h[j], hj);
                        // keep the scheduler from hoisting later j's table loads (register pressure)
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                __syncthreads();
                a = bb;
            }
            // G_U[:, i_n] from the top layer: wave sums, then a fixed-order sum over waves
#pragma unroll
            for (int j = 0; j < MMAX; ++j) {
                if (j < m) {
                    const float re = wave_sum(h[j].x);
                    const float im = wave_sum(h[j].y);
                    if (lane == 0) scratch[wave * 32 + j] = make_float2(re, im);
                }
            }
            // g_{n-1} replaces d_{n-1} (no longer read)
#pragma unroll
            for (int s = 0; s < OWN; ++s) {
                const int tp = tid + s * BLOCK;
                if (tp < Np) X[tp] = acc[s];
            }
            __syncthreads();
            if (tid < m) {
                float2 sum = c_zero();
                for (int w = 0; w < NW; ++w) sum = c_add(sum, scratch[w * 32 + tid]);
                GUacc[(n - 1) * 32 + tid] = sum;
            }
            // ---- lower layers.  d_0..d_{n-2} stored after g_{n-1}; g ping-pongs
            // between offset 0 and R.
            // layer k of the store starts at Np + (number of states with < k photons)
            const int R = Np + (int)Ls[n - 1].cum;
            if (tid == 0) X[Np] = make_float2(1.f, 0.f);
            __syncthreads();
            for (int k = 1; k <= n - 2; ++k) {
                if (tid < m) ucol[tid] = Ub[tid * m + modes[k - 1]];
                __syncthreads();
                layer_pull<BLOCK>(Ls[k], k, X + Np + (int)Ls[k - 1].cum, X + Np + (int)Ls[k].cum, ucol);
                __syncthreads();
            }
            const int grp = tid >> 5;
            const int jj = tid & 31;
            for (int k = n - 1; k >= 1; --k) {
                if (tid < m) ucol[tid] = Ub[tid * m + modes[k - 1]];
                __syncthreads();
                const float2* gk = X + ((((n - 1 - k) & 1) == 0) ? 0 : R);
                float2* gkm1 = X + ((((n - 1 - (k - 1)) & 1) == 0) ? 0 : R);
                const float2* dkm1 = X + Np + (int)Ls[k - 1].cum;
                const int Nkm1 = (int)Ls[k - 1].N;
                const int32_t* succ = Ls[k].succ;
                const float2 uj = (jj < m) ? ucol[jj] : c_zero();
                float2 hj = c_zero();
                for (int tp = grp; tp < Nkm1; tp += NG) {
                    float2 contrib = c_zero();
                    if (jj < m) {
                        const float2 g = gk[succ[(size_t)jj * Nkm1 + tp]];
                        c_fma_conj(contrib, uj, g);
                        c_fma_conj(hj, dkm1[tp], g);
                    }
                    const float re = half_wave_sum(contrib.x);
                    const float im = half_wave_sum(contrib.y);
                    if (jj == 0 && k >= 2) gkm1[tp] = make_float2(re, im);
                }
                scratch[grp * 32 + jj] = hj;
                __syncthreads();
                if (tid < m) {
                    float2 sum = c_zero();
                    for (int g2 = 0; g2 < NG; ++g2) sum = c_add(sum, scratch[g2 * 32 + tid]);
                    GUacc[(k - 1) * 32 + tid] = sum;
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
                if (modes[k - 1] == i) v = c_add(v, GUacc[(k - 1) * 32 + j]);
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

int mmax_for(int m) { return m <= 8 ? 8 : m <= 12 ? 12 : m <= 16 ? 16 : m <= 20 ? 20 : m <= 24 ? 24 : 32; }

// photon-layer-(n-1) states per thread in the register-resident top-layer pull
int own_for(int block, int64_t Np) {
    const int64_t need = (Np + block - 1) / block;
    if (block == 256) return need <= 1 ? 1 : need <= 4 ? 4 : need <= 8 ? 8 : -1;
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

template <int BLOCK, int MMAX>
void* bwd_fn2(int own) {
    if constexpr (BLOCK == 256) {
        switch (own) {
            case 1: return (void*)&fused_bwd_kernel<BLOCK, MMAX, 1>;
            case 4: return (void*)&fused_bwd_kernel<BLOCK, MMAX, 4>;
            case 8: return (void*)&fused_bwd_kernel<BLOCK, MMAX, 8>;
        }
    } else {
        switch (own) {
            case 4: return (void*)&fused_bwd_kernel<BLOCK, MMAX, 4>;
            case 10: return (void*)&fused_bwd_kernel<BLOCK, MMAX, 10>;
            case 18: return (void*)&fused_bwd_kernel<BLOCK, MMAX, 18>;
        }
    }
    return nullptr;
}
template <int BLOCK>
void* bwd_fn1(int mmax, int own) {
    switch (mmax) {
        case 8: return bwd_fn2<BLOCK, 8>(own);
        case 12: return bwd_fn2<BLOCK, 12>(own);
        case 16: return bwd_fn2<BLOCK, 16>(own);
        case 20: return bwd_fn2<BLOCK, 20>(own);
        case 24: return bwd_fn2<BLOCK, 24>(own);
        case 32: return bwd_fn2<BLOCK, 32>(own);
    }
    return nullptr;
}
void* pick_bwd(int block, int m, int64_t Np) {
    const int own = own_for(block, Np);
    if (own < 0) return nullptr;
    if (block == 256) return bwd_fn1<256>(mmax_for(m), own);
    if (block == 512) return bwd_fn1<512>(mmax_for(m), own);
    return nullptr;
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
    return (size_t)(lds_fwd_states(P, n_max) + kUcol) * sizeof(float2);
}

size_t fused_bwd_lds_bytes(const slos_plan_s& P, int n_max) {
    // block-dependent scratch is added at launch; report the 512-thread figure
    return (size_t)(lds_bwd_states(P, n_max) + kUcol + 512 + kMaxPhotons * 32) * sizeof(float2);
}

static size_t bwd_lds_for_block(const slos_plan_s& P, int n_max, int block) {
    return (size_t)(lds_bwd_states(P, n_max) + kUcol + block + kMaxPhotons * 32) * sizeof(float2);
}

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
    if (!P.layers.empty() && P.n_max >= 1 && P.layers[1].succ == nullptr) {
        if (why) *why = "plan has no successor tables";
        return false;
    }
    if (bwd_lds_for_block(P, n_max, block) > P.max_lds) {
        if (why) *why = "photon layers do not fit in LDS";
        return false;
    }
    if (n_max >= 2 && own_for(block, P.N[n_max - 1]) < 0) {
        if (why) *why = "layer n-1 too large for the register-resident adjoint";
        return false;
    }
    return true;
}

int fused_default_block(const slos_plan_s& P, int n_max, bool backward) {
    const int64_t Nbig = n_max >= 1 ? P.N[n_max] : 1;
    if (backward) return (n_max >= 2 && P.N[n_max - 1] > 1024) ? 512 : 256;
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
    void* args[] = {(void*)&P.m, (void*)&P.d_layers, (void*)&Bt.dev, (void*)&U, (void*)&gin, (void*)&gU, (void*)&S, (void*)&pr};
    hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("fused backward launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

}  // namespace slos
