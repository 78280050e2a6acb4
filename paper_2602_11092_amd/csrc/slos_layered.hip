// Layered kernels: one launch per photon layer, with the layers kept in the
// caller's workspace instead of LDS.  They handle Fock spaces of any size
// (a photon layer may be far larger than a workgroup's LDS) and, with
// B = 1, serve as the unbatched per-sample path.
//
// Same recursion as the fused kernels (arXiv 2602.11092, Sec. II-A-3):
// layer k is pulled from layer k-1 through the transition tables.  The
// batch is split into groups of SG samples (SG a power of two <= 64) and
// each layer is stored [group][state][SG], so the SG lanes that share a
// state read one contiguous SG*8-byte segment per gather.  The backward
// recomputes layers 1..n-1 into the workspace, then walks k = n..1 with a
// seed launch (top-layer gradient of the samples whose top is layer k), a
// pull launch (g_{k-1} and the partial sums of G_U[:, i_k]) and, at the
// end, one launch that adds the partial sums in a fixed order.
#include "slos_internal.h"

namespace slos {
namespace {

struct Shape {
    int SG;    // samples per group (lanes sharing a state)
    int NGRP;  // number of groups
    int GX;    // blocks along the state axis in the pull launches
};

Shape shape_of(const slos_batch_s& Bt) {
    int sg = 1;
    while (sg < Bt.B && sg < 64) sg <<= 1;
    const int ngrp = (Bt.B + sg - 1) / sg;
    // no more blocks than the largest pull range needs (256 threads each); with
    // one group, 1024 blocks (four per CU, what the pull's LDS allows) keep 4
    // waves per SIMD waiting on the gathers
    const int64_t Nmax = Bt.n_max >= 1 ? Bt.plan->N[Bt.n_max - 1] : 1;
    const int64_t need = (Nmax * sg + 255) / 256;
    const int cap = std::max(8, std::min(1024, 2048 / ngrp));
    return Shape{sg, ngrp, (int)std::max<int64_t>(1, std::min<int64_t>(need, cap))};
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace layout.
struct Layout {
    size_t store_off[kMaxPhotons + 1];  // bwd: layer k at store_off[k] (k = 1..n_max-1)
    size_t buf0, buf1;                  // fwd: ping-pong layers; bwd: g ping-pong
    size_t partial;                     // bwd: [n_max][NGRP][GX][SG][32] float2
    size_t col;                         // bwd: [B][kMaxPhotons][32] float2, G_U[:, i_k] per layer
    size_t total;
};

Layout layout_of(const slos_batch_s& Bt, bool backward) {
    const slos_plan_s& P = *Bt.plan;
    const Shape sh = shape_of(Bt);
    const size_t per_state = (size_t)sh.NGRP * sh.SG * sizeof(float2);
    Layout L{};
    size_t off = 0;
    int64_t maxN = 1;
    if (backward) {
        for (int k = 1; k <= Bt.n_max - 1; ++k) {
            L.store_off[k] = off;
            off += align256((size_t)P.N[k] * per_state);
        }
        for (int k = 1; k <= Bt.n_max; ++k) maxN = std::max(maxN, P.N[k]);
    } else {
        for (int k = 1; k <= Bt.n_max - 1; ++k) maxN = std::max(maxN, P.N[k]);
    }
    L.buf0 = off;
    off += align256((size_t)maxN * per_state);
    L.buf1 = off;
    off += align256((size_t)maxN * per_state);
    L.partial = off;
    if (backward) off += align256((size_t)std::max(Bt.n_max, 1) * sh.NGRP * sh.GX * sh.SG * 32 * sizeof(float2));
    L.col = off;
    if (backward) off += align256((size_t)Bt.B * kMaxPhotons * 32 * sizeof(float2));
    L.total = off;
    return L;
}

enum Mode { kForward = 0, kRecompute = 1, kSeed = 2 };

// One layer for every active sample of a group.  kForward: samples whose top
// layer is k write their outputs, the others write layer k.  kRecompute:
// only samples with more than k photons, writing layer k.  kSeed: only
// samples whose top layer is k, writing g_k.
template <int BLOCK, bool PROBS>
__global__ __launch_bounds__(BLOCK) void layered_layer_kernel(int m, const LayerDev* __restrict__ Ls, BatchDev Bt,
                                                              const float2* __restrict__ U, int k, int mode,
                                                              const float2* __restrict__ prev, float2* __restrict__ cur,
                                                              void* __restrict__ out, const void* __restrict__ gin,
                                                              int SG) {
    __shared__ float2 us[64 * kUcolSlots];
    const int tid = threadIdx.x;
    const int bl = tid % SG;
    const int tl = tid / SG;
    const int TPB = BLOCK / SG;
    const int g = blockIdx.y;
    const int b = g * SG + bl;
    const int n_b = (b < Bt.B) ? Bt.n[b] : -1;
    const bool active = (mode == kForward) ? n_b >= k : (mode == kRecompute) ? n_b > k : n_b == k;
    // stage column i_k of U for every sample of the group (slot 32 = 0)
    for (int q = tid; q < SG; q += BLOCK) us[q * kUcolSlots + 32] = c_zero();
    for (int q = tid; q < SG * m; q += BLOCK) {
        const int bq = q % SG, j = q / SG;
        const int bb = g * SG + bq;
        if (bb < Bt.B && Bt.n[bb] >= k) {
            const int ik = Bt.modes[(size_t)bb * kMaxPhotons + k - 1];
            us[bq * kUcolSlots + j] = U[((size_t)bb * m + j) * m + ik];
        }
    }
    __syncthreads();
    if (!active) return;
    const LayerDev L = Ls[k];
    const int N = (int)L.N;
    const int Nprev = (int)Ls[k - 1].N;
    const bool top = (n_b == k);
    const float innorm = Bt.innorm[b];
    const int64_t off = Bt.off[b];
    for (int t = blockIdx.x * TPB + tl; t < N; t += gridDim.x * TPB) {
        float2 acc = c_zero();
        const bool need_d = !(mode == kSeed && !PROBS);
        if (need_d) {
            if (k == 1) {
                acc = us[bl * kUcolSlots + t];
            } else {
                const int sh = L.pred_shift;
                const uint32_t rmask = pred_rank_mask(sh);
                for (int gq = 0; gq < L.ngrp; ++gq) {
                    const uint4 e4 = L.predv[(size_t)gq * N + t];
                    const uint32_t es[4] = {e4.x, e4.y, e4.z, e4.w};
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        // empty entries name the zero slot 32 of the coefficient column
                        const uint32_t e = es[q];
                        c_fma(acc, us[bl * kUcolSlots + (e >> sh)],
                              prev[((size_t)g * Nprev + ((e & rmask) >> 3)) * SG + bl]);
                    }
                }
            }
        }
        if (mode == kForward && top) {
            const float c = L.nrm[t] * innorm;
            if (PROBS) ((float*)out)[off + t] = c * c * (acc.x * acc.x + acc.y * acc.y);
            else ((float2*)out)[off + t] = c_scale(acc, c);
        } else if (mode == kSeed) {
            const float c = L.nrm[t] * innorm;
            float2 gv;
            if (PROBS) gv = c_scale(acc, 2.f * ((const float*)gin)[off + t] * c * c);
            else gv = c_scale(((const float2*)gin)[off + t], c);
            cur[((size_t)g * N + t) * SG + bl] = gv;
        } else {
            cur[((size_t)g * N + t) * SG + bl] = acc;
        }
    }
}

// g_{k-1}[t'] = sum_j conj(u_j) g_k[t'+e_j]; partial sums of
// G_U[j][i_k] = sum_t' conj(d_{k-1}[t']) g_k[t'+e_j] per block.  Each lane
// keeps its G_U partials for MMAX modes in registers (modes past m read
// padding successors and zero coefficients and are never written out),
// loads the successors of four modes at once, and the block adds the lanes
// of each sample in a fixed order through an LDS window of 8 modes.
// RESTRICTED: plans of a restricted space, whose successor tables mark
// successors outside the space with kNoSuccessor; those pairs contribute
// nothing (the forward never formed such states).

template <int BLOCK, int MMAX, bool RESTRICTED>
__global__ __launch_bounds__(BLOCK) void layered_pull_kernel(int m, const LayerDev* __restrict__ Ls, BatchDev Bt,
                                                             const float2* __restrict__ U, int k,
                                                             const float2* __restrict__ gk, float2* __restrict__ gkm1,
                                                             const float2* __restrict__ dkm1,
                                                             float2* __restrict__ partial, int SG, int NGRP) {
    constexpr int WIN = 8;
    __shared__ float2 us[64 * kUcolSlots];
    __shared__ float2 Hs[WIN * BLOCK];
    const int tid = threadIdx.x;
    const int bl = tid % SG;
    const int tl = tid / SG;
    const int TPB = BLOCK / SG;
    const int g = blockIdx.y;
    const int b = g * SG + bl;
    const int n_b = (b < Bt.B) ? Bt.n[b] : -1;
    const bool active = n_b >= k;
    for (int q = tid; q < SG * kUcolSlots; q += BLOCK) us[q] = c_zero();
    __syncthreads();
    for (int q = tid; q < SG * m; q += BLOCK) {
        const int bq = q % SG, j = q / SG;
        const int bb = g * SG + bq;
        if (bb < Bt.B && Bt.n[bb] >= k) {
            const int ik = Bt.modes[(size_t)bb * kMaxPhotons + k - 1];
            us[bq * kUcolSlots + j] = U[((size_t)bb * m + j) * m + ik];
        }
    }
    __syncthreads();
    float2 h[MMAX];
#pragma unroll
    for (int j = 0; j < MMAX; ++j) h[j] = c_zero();
    if (active) {
        const int Nk = (int)Ls[k].N;
        const int Nkm1 = (int)Ls[k - 1].N;
        const uint4* succ4 = (const uint4*)Ls[k].succ;
        const int ngs = (m + 3) >> 2;  // successor groups in the table
        const float2* gkg = gk + (size_t)g * Nk * SG + bl;
        for (int tp = blockIdx.x * TPB + tl; tp < Nkm1; tp += gridDim.x * TPB) {
            const float2 dv = (k >= 2) ? dkm1[((size_t)g * Nkm1 + tp) * SG + bl] : make_float2(1.f, 0.f);
            float2 acc = c_zero();
#pragma unroll
            for (int q4 = 0; q4 < MMAX / 4; ++q4) {
                if (q4 >= ngs) continue;  // uniform
                const uint4 s4 = succ4[(size_t)q4 * Nkm1 + tp];
                const uint32_t sv[4] = {s4.x, s4.y, s4.z, s4.w};
                float2 gv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (RESTRICTED) {
                        const bool none = sv[q] == kNoSuccessor;
                        const float2 v = gkg[(size_t)((none ? 0u : sv[q]) >> 3) * SG];
                        gv[q] = none ? c_zero() : v;
                    } else {
                        gv[q] = gkg[(size_t)(sv[q] >> 3) * SG];
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    c_fma_conj(acc, us[bl * kUcolSlots + 4 * q4 + q], gv[q]);
                    c_fma_conj(h[4 * q4 + q], dv, gv[q]);
                }
            }
            if (k >= 2) gkm1[((size_t)g * Nkm1 + tp) * SG + bl] = acc;
        }
    }
    // fixed-order sum over the lanes that share a sample, WIN modes at a time
#pragma unroll
    for (int j0 = 0; j0 < MMAX; j0 += WIN) {
        __syncthreads();
#pragma unroll
        for (int w = 0; w < WIN; ++w)
            if (j0 + w < MMAX) Hs[w * BLOCK + tid] = h[j0 + w];
        __syncthreads();
        for (int q = tid; q < SG * WIN; q += BLOCK) {
            const int bq = q % SG, w = q / SG;
            const int j = j0 + w;
            if (j >= 32) continue;
            float2 sum = c_zero();
            for (int tq = 0; tq < TPB; ++tq) sum = c_add(sum, Hs[w * BLOCK + tq * SG + bq]);
            partial[((((size_t)(k - 1) * NGRP + g) * gridDim.x + blockIdx.x) * SG + bq) * 32 + j] = sum;
        }
    }
}

// Column i_k of G_U for sample b from layer k's block partials.  One block
// per (sample, layer): 32 slices of 32 lanes (one lane per mode) each add
// every 32nd block partial with eight independent accumulators, then the
// slices are added in order.  The order is fixed, so results are
// reproducible; the loads of a slice are all independent.
__global__ __launch_bounds__(1024) void layered_reduce_kernel(BatchDev Bt, const float2* __restrict__ partial,
                                                              float2* __restrict__ col, int SG, int NGRP, int GX) {
    __shared__ float2 part[32][33];
    const int b = blockIdx.x;
    const int k = blockIdx.y + 1;
    if (k > Bt.n[b]) return;  // uniform over the block
    const int g = b / SG, bl = b % SG;
    const int tid = threadIdx.x, j = tid & 31, sl = tid >> 5;
    const float2* src = partial + (((size_t)(k - 1) * NGRP + g) * GX * SG + bl) * 32 + j;
    const size_t xs = (size_t)SG * 32;  // stride between consecutive block partials
    float2 a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = c_zero();
    int x = sl;
    for (; x + 7 * 32 < GX; x += 8 * 32) {
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] = c_add(a[q], src[(size_t)(x + q * 32) * xs]);
    }
    for (; x < GX; x += 32) a[0] = c_add(a[0], src[(size_t)x * xs]);
    float2 v = c_zero();
#pragma unroll
    for (int q = 0; q < 8; ++q) v = c_add(v, a[q]);
    part[sl][j] = v;
    __syncthreads();
    if (tid < 32) {
        float2 sum = c_zero();
        for (int q = 0; q < 32; ++q) sum = c_add(sum, part[q][tid]);
        col[((size_t)b * kMaxPhotons + k - 1) * 32 + tid] = sum;
    }
}

// G_U[b][j][i] = sum over photon layers k with i_k = i of column k, in k order.
__global__ __launch_bounds__(256) void layered_final_kernel(int m, BatchDev Bt, const float2* __restrict__ col,
                                                            float2* __restrict__ gU) {
    const int b = blockIdx.x;
    const int n_b = Bt.n[b];
    const int32_t* modes = Bt.modes + (size_t)b * kMaxPhotons;
    const float2* cb = col + (size_t)b * kMaxPhotons * 32;
    for (int q = threadIdx.x; q < m * m; q += blockDim.x) {
        const int jj = q / m, i = q % m;
        float2 v = c_zero();
        for (int k = 1; k <= n_b; ++k)
            if (modes[k - 1] == i) v = c_add(v, cb[(k - 1) * 32 + jj]);
        gU[(size_t)b * m * m + q] = v;
    }
}

// Samples without photons: the only output is the vacuum, amplitude 1.
__global__ void vacuum_kernel(BatchDev Bt, void* out, int probs) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= Bt.B || Bt.n[b] != 0) return;
    if (probs) ((float*)out)[Bt.off[b]] = 1.f;
    else ((float2*)out)[Bt.off[b]] = make_float2(1.f, 0.f);
}

template <bool PROBS>
void* layer_fn(int block) {
    switch (block) {
        case 64: return (void*)&layered_layer_kernel<64, PROBS>;
        case 128: return (void*)&layered_layer_kernel<128, PROBS>;
        case 256: return (void*)&layered_layer_kernel<256, PROBS>;
        case 512: return (void*)&layered_layer_kernel<512, PROBS>;
        case 1024: return (void*)&layered_layer_kernel<1024, PROBS>;
    }
    return nullptr;
}

int launch_layer(const slos_batch_s& Bt, int block, const float2* U, int k, int mode, const float2* prev,
                 float2* cur, void* out, const void* gin, bool probs, hipStream_t stream) {
    const slos_plan_s& P = *Bt.plan;
    const Shape sh = shape_of(Bt);
    if (block < sh.SG) block = sh.SG;
    void* fn = probs ? layer_fn<true>(block) : layer_fn<false>(block);
    if (!fn) return fail(SLOS_EUNSUPPORTED, "layered: bad block size");
    const int TPB = block / sh.SG;
    const int64_t N = P.N[k];
    const int gx = (int)std::max<int64_t>(1, std::min<int64_t>((N + TPB - 1) / TPB, 8192));
    int m = P.m;
    const LayerDev* Ls = P.d_layers;
    int SG = sh.SG;
    void* args[] = {(void*)&m, (void*)&Ls, (void*)&Bt.dev, (void*)&U, (void*)&k, (void*)&mode,
                    (void*)&prev, (void*)&cur, (void*)&out, (void*)&gin, (void*)&SG};
    hipError_t e = hipLaunchKernel(fn, dim3(gx, sh.NGRP), dim3(block), args, 0, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("layered layer launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

}  // namespace

size_t layered_ws_bytes(const slos_batch_s& Bt, bool backward) {
    if (Bt.B == 0 || Bt.n_max == 0) return 0;
    return layout_of(Bt, backward).total;
}

int layered_default_block(const slos_batch_s& Bt) {
    (void)Bt;
    return 256;
}

int launch_layered_fwd(const slos_batch_s& Bt, int block, const float2* U, void* out, bool probs, void* ws,
                       hipStream_t stream) {
    const Layout L = layout_of(Bt, false);
    char* base = (char*)ws;
    float2* bufs[2] = {(float2*)(base + L.buf0), (float2*)(base + L.buf1)};
    for (int k = 1; k <= Bt.n_max; ++k) {
        const float2* prev = bufs[(k - 1) & 1];
        float2* cur = bufs[k & 1];
        int rc = launch_layer(Bt, block, U, k, kForward, prev, cur, out, nullptr, probs, stream);
        if (rc != SLOS_OK) return rc;
    }
    bool any_vacuum = false;
    for (int b = 0; b < Bt.B; ++b) any_vacuum |= (Bt.n_host[b] == 0);
    if (any_vacuum) {
        int pr = probs ? 1 : 0;
        void* args[] = {(void*)&Bt.dev, (void*)&out, (void*)&pr};
        hipError_t e = hipLaunchKernel((void*)&vacuum_kernel, dim3((Bt.B + 255) / 256), dim3(256), args, 0, stream);
        if (e != hipSuccess) return fail(SLOS_EHIP, std::string("vacuum launch: ") + hipGetErrorString(e));
    }
    return SLOS_OK;
}

template <bool R>
static void* pull_fn_r(int m) {
    if (m <= 8) return (void*)&layered_pull_kernel<256, 8, R>;
    if (m <= 12) return (void*)&layered_pull_kernel<256, 12, R>;
    if (m <= 16) return (void*)&layered_pull_kernel<256, 16, R>;
    if (m <= 20) return (void*)&layered_pull_kernel<256, 20, R>;
    if (m <= 24) return (void*)&layered_pull_kernel<256, 24, R>;
    return (void*)&layered_pull_kernel<256, 32, R>;
}

static void* pull_fn(int m, bool restricted) { return restricted ? pull_fn_r<true>(m) : pull_fn_r<false>(m); }

int launch_layered_bwd(const slos_batch_s& Bt, int block, const float2* U, const void* gin, bool probs, float2* gU,
                       void* ws, hipStream_t stream) {
    const slos_plan_s& P = *Bt.plan;
    const Shape sh = shape_of(Bt);
    const Layout L = layout_of(Bt, true);
    char* base = (char*)ws;
    auto store = [&](int k) -> float2* { return (k >= 1) ? (float2*)(base + L.store_off[k]) : nullptr; };
    float2* gbuf[2] = {(float2*)(base + L.buf0), (float2*)(base + L.buf1)};
    float2* partial = (float2*)(base + L.partial);
    int rc;
    for (int k = 1; k <= Bt.n_max - 1; ++k) {
        rc = launch_layer(Bt, block, U, k, kRecompute, store(k - 1), store(k), nullptr, nullptr, probs, stream);
        if (rc != SLOS_OK) return rc;
    }
    int m = P.m;
    const LayerDev* Ls = P.d_layers;
    int SG = sh.SG, NGRP = sh.NGRP;
    for (int k = Bt.n_max; k >= 1; --k) {
        float2* gk = gbuf[(Bt.n_max - k) & 1];
        float2* gkm1 = gbuf[(Bt.n_max - k + 1) & 1];
        // the seed writes g_k of the samples whose top layer is k; with none, g_k
        // is the previous pull's output as it stands
        bool any_top = false;
        for (int b = 0; b < Bt.B && !any_top; ++b) any_top = (Bt.n_host[b] == k);
        if (any_top) {
            rc = launch_layer(Bt, block, U, k, kSeed, store(k - 1), gk, nullptr, gin, probs, stream);
            if (rc != SLOS_OK) return rc;
        }
        const float2* dkm1 = store(k - 1);
        void* args[] = {(void*)&m, (void*)&Ls, (void*)&Bt.dev, (void*)&U, (void*)&k, (void*)&gk,
                        (void*)&gkm1, (void*)&dkm1, (void*)&partial, (void*)&SG, (void*)&NGRP};
        const bool restricted = (P.flags & (SLOS_PLAN_UNBUNCHED | SLOS_PLAN_DUAL_RAIL)) != 0;
        hipError_t e = hipLaunchKernel(pull_fn(m, restricted), dim3(sh.GX, NGRP), dim3(256), args, 0, stream);
        if (e != hipSuccess) return fail(SLOS_EHIP, std::string("layered pull launch: ") + hipGetErrorString(e));
    }
    int GX = sh.GX;
    float2* col = (float2*)(base + L.col);
    {
        void* args[] = {(void*)&Bt.dev, (void*)&partial, (void*)&col, (void*)&SG, (void*)&NGRP, (void*)&GX};
        hipError_t e = hipLaunchKernel((void*)&layered_reduce_kernel, dim3(Bt.B, std::max(Bt.n_max, 1)), dim3(1024), args, 0, stream);
        if (e != hipSuccess) return fail(SLOS_EHIP, std::string("layered reduce launch: ") + hipGetErrorString(e));
    }
    void* args[] = {(void*)&m, (void*)&Bt.dev, (void*)&col, (void*)&gU};
    hipError_t e = hipLaunchKernel((void*)&layered_final_kernel, dim3(Bt.B), dim3(256), args, 0, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("layered final launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

}  // namespace slos
