// Measurement kernels over a batch's output states (Sec. II-B, measurement
// strategies): per-mode photon-number expectations from probabilities, and
// the weight expansion of their adjoint.
//
//   <n_j>_b      = sum_t t_j p_b[t]     (mode_expect_partial_kernel, then
//                                         mode_expect_final_kernel)
//   dL/dp_b[t]   = sum_j t_j dL/d<n_j>_b  (expand_kernel)
//   (DISTINCT instances: t_j replaced by [t_j > 0], the per-mode click
//    probabilities of threshold detectors and their adjoint)
//   P_b(c)       = sum of p_b over the states of click pattern c
//                                         (threshold_gather_kernel)
//   dL/dp_b[t]   = dL/dP_b(pattern of t)  (threshold_scatter_kernel)
//   cdf_b[t]     = sum_{t' <= t} p_b[t'], FP64 (cdf_partial_kernel, cdf_scan_kernel)
//   shot         = first t with cdf_b[t] > u cdf_b[N-1]  (sample_kernel)
//
// A state's photons are read from its predecessor entries in the transition
// table of its photon layer (for_each_photon).  Workgroup b * C + c takes
// chunk c (kChunkStates states) of sample b, so large samples spread over
// many workgroups; partial sums are combined in chunk order, so results are
// deterministic.
#include "slos_internal.h"

namespace slos {
namespace {

constexpr int kMeasureBlock = 256;
constexpr int kParts = kMeasureBlock / kMaxModes;  // partial sums per mode in the final reduction
constexpr int64_t kChunkStates = kMeasureChunkStates;  // states per workgroup in the (sample, chunk) grids
static_assert(kParts * kMaxModes == kMeasureBlock, "one thread per (mode, part)");

// Stage 1: workgroup (b, c) sums states [c*kChunkStates, (c+1)*kChunkStates)
// of sample b into part[b][c][j] (zero where the chunk holds no state).
template <bool DISTINCT>
__global__ __launch_bounds__(kMeasureBlock) void mode_expect_partial_kernel(int m, const LayerDev* __restrict__ Ls,
                                                                            BatchDev Bt, const float* __restrict__ p,
                                                                            float* __restrict__ part, int C) {
    // lane tid owns column tid: acc[j][tid] = sum of p over its states, per photon in mode j
    __shared__ float acc[kMaxModes][kMeasureBlock];
    const int tid = threadIdx.x;
    const int b = blockIdx.x / C, c = blockIdx.x % C;
    for (int j = 0; j < kMaxModes; ++j) acc[j][tid] = 0.f;
    const int n = ldg(Bt.n + b);
    if (n > 0) {
        const int64_t off = ldg(Bt.off + b);
        const LayerDev L = Ls[n];
        const int64_t lo = (int64_t)c * kChunkStates, hi = lo + kChunkStates < L.N ? lo + kChunkStates : L.N;
        for (int64_t t = lo + tid; t < hi; t += kMeasureBlock) {
            const float v = p[off + t];
            for_each_photon<DISTINCT>(L, n, t, [&](int j) { acc[j][tid] += v; });
        }
    }
    __syncthreads();
    // thread (j, part) sums a strip of kMeasureBlock / kParts columns, then the parts combine
    const int j = tid / kParts, q = tid % kParts;
    constexpr int strip = kMeasureBlock / kParts;
    float v = 0.f;
    for (int i = 0; i < strip; ++i) v += acc[j][q * strip + i];
    for (int s = kParts / 2; s >= 1; s >>= 1) v += __shfl_xor(v, s, kParts);
    if (q == 0 && j < m) part[((size_t)b * C + c) * m + j] = v;
}

// Stage 2: out[b][j] = sum_c part[b][c][j], in chunk order.
__global__ __launch_bounds__(kMeasureBlock) void mode_expect_final_kernel(int m, int B, int C,
                                                                          const float* __restrict__ part,
                                                                          float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kMeasureBlock + threadIdx.x;
    if (i >= (int64_t)B * m) return;
    const int64_t b = i / m, j = i % m;
    float v = 0.f;
    for (int c = 0; c < C; ++c) v += part[(b * C + c) * m + j];
    out[i] = v;
}

// gp[off_b + t] = sum_j t_j w[b][j] for the states of chunk c of sample b
// (workgroup b * C + c).
template <bool DISTINCT>
__global__ __launch_bounds__(kMeasureBlock) void expand_kernel(int m, const LayerDev* __restrict__ Ls, BatchDev Bt,
                                                               const float* __restrict__ w,
                                                               float* __restrict__ gp, int C) {
    __shared__ float wb[kMaxModes];
    const int tid = threadIdx.x;
    const int b = blockIdx.x / C, c = blockIdx.x % C;
    if (tid < m) wb[tid] = w[(size_t)b * m + tid];
    __syncthreads();
    const int n = ldg(Bt.n + b);
    const int64_t off = ldg(Bt.off + b);
    if (n == 0) {
        if (c == 0 && tid == 0) gp[off] = 0.f;  // <n_j> does not depend on the vacuum's probability
        return;
    }
    const LayerDev L = Ls[n];
    const int64_t lo = (int64_t)c * kChunkStates, hi = lo + kChunkStates < L.N ? lo + kChunkStates : L.N;
    for (int64_t t = lo + tid; t < hi; t += kMeasureBlock) {
        float g = 0.f;
        for_each_photon<DISTINCT>(L, n, t, [&](int j) { g += wb[j]; });
        gp[off + t] = g;
    }
}

// Click patterns per workgroup in the threshold kernels.
constexpr int64_t kChunkPatterns = (int64_t)kMeasureBlock * 16;

// Workgroup b * C + c: patterns [c * kChunkPatterns, ...) of sample b, one
// thread per pattern, its states summed in ascending order.
__global__ __launch_bounds__(kMeasureBlock) void threshold_gather_kernel(const LayerDev* __restrict__ Ls, BatchDev Bt,
                                                                         const float* __restrict__ p,
                                                                         float* __restrict__ out, int C) {
    const int b = blockIdx.x / C, c = blockIdx.x % C;
    const int n = ldg(Bt.n + b);
    const int64_t off = ldg(Bt.off + b), toff = ldg(Bt.thr_off + b);
    if (n == 0) {  // the empty pattern: the vacuum itself
        if (c == 0 && threadIdx.x == 0) out[toff] = p[off];
        return;
    }
    const LayerDev L = Ls[n];
    const int64_t q = (int64_t)c * kChunkPatterns + threadIdx.x;
    for (int64_t r = q; r < L.Q && r < (int64_t)(c + 1) * kChunkPatterns; r += kMeasureBlock) {
        const int32_t lo = ldg(L.thr_ptr + r), hi = ldg(L.thr_ptr + r + 1);
        float v = 0.f;
        for (int32_t i = lo; i < hi; ++i) v += p[off + ldg(L.thr_idx + i)];
        out[toff + r] = v;
    }
}

// The adjoint: every state of pattern r receives dL/dP(r) (each state is in
// exactly one pattern, so the writes do not overlap).
__global__ __launch_bounds__(kMeasureBlock) void threshold_scatter_kernel(const LayerDev* __restrict__ Ls, BatchDev Bt,
                                                                          const float* __restrict__ gP,
                                                                          float* __restrict__ gp, int C) {
    const int b = blockIdx.x / C, c = blockIdx.x % C;
    const int n = ldg(Bt.n + b);
    const int64_t off = ldg(Bt.off + b), toff = ldg(Bt.thr_off + b);
    if (n == 0) {
        if (c == 0 && threadIdx.x == 0) gp[off] = gP[toff];
        return;
    }
    const LayerDev L = Ls[n];
    const int64_t q = (int64_t)c * kChunkPatterns + threadIdx.x;
    for (int64_t r = q; r < L.Q && r < (int64_t)(c + 1) * kChunkPatterns; r += kMeasureBlock) {
        const int32_t lo = ldg(L.thr_ptr + r), hi = ldg(L.thr_ptr + r + 1);
        const float g = gP[toff + r];
        for (int32_t i = lo; i < hi; ++i) gp[off + ldg(L.thr_idx + i)] = g;
    }
}

// Cumulative sums for sampling, in two passes over (sample, chunk) pairs of
// kChunkStates states: chunk totals, then each chunk scans its states from
// the sum of the chunks before it.  FP64 sums, fixed order.
__global__ __launch_bounds__(kMeasureBlock) void cdf_partial_kernel(BatchDev Bt, const float* __restrict__ p,
                                                                    double* __restrict__ part, int C) {
    __shared__ double red[kMeasureBlock / 64];
    const int b = blockIdx.x / C, c = blockIdx.x % C;
    const int64_t off = ldg(Bt.off + b), N = ldg(Bt.off + b + 1) - off;
    const int64_t lo = (int64_t)c * kChunkStates, hi = lo + kChunkStates < N ? lo + kChunkStates : N;
    double v = 0.0;
    for (int64_t t = lo + threadIdx.x; t < hi; t += kMeasureBlock) v += p[off + t];
    for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kMeasureBlock / 64; ++w) t += red[w];
        part[(size_t)b * C + c] = t;
    }
}

__global__ __launch_bounds__(kMeasureBlock) void cdf_scan_kernel(BatchDev Bt, const float* __restrict__ p,
                                                                 const double* __restrict__ part, int C,
                                                                 double* __restrict__ cdf) {
    constexpr int V = 4;  // consecutive states per thread per tile
    constexpr int kWaves = kMeasureBlock / 64;
    __shared__ double wtot[kWaves];
    __shared__ double carry_s;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int b = blockIdx.x / C, c = blockIdx.x % C;
    const int64_t off = ldg(Bt.off + b), N = ldg(Bt.off + b + 1) - off;
    const int64_t lo = (int64_t)c * kChunkStates, hi = lo + kChunkStates < N ? lo + kChunkStates : N;
    if (tid == 0) {
        double s0 = 0.0;
        for (int q = 0; q < c; ++q) s0 += part[(size_t)b * C + q];
        carry_s = s0;
    }
    __syncthreads();
    for (int64_t t0 = lo; t0 < hi; t0 += (int64_t)kMeasureBlock * V) {
        double v[V];
        const int64_t tb = t0 + (int64_t)tid * V;
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = (tb + i < hi) ? (double)p[off + tb + i] : 0.0;
#pragma unroll
        for (int i = 1; i < V; ++i) v[i] += v[i - 1];
        // inclusive scan of the thread totals within the wave
        double x = v[V - 1];
        for (int s = 1; s < 64; s <<= 1) {
            const double y = __shfl_up(x, s, 64);
            if (lane >= s) x += y;
        }
        if (lane == 63) wtot[w] = x;
        __syncthreads();
        double before = carry_s;
        for (int q = 0; q < w; ++q) before += wtot[q];
        before += x - v[V - 1];  // exclusive within the wave
#pragma unroll
        for (int i = 0; i < V; ++i)
            if (tb + i < hi) cdf[off + tb + i] = before + v[i];
        __syncthreads();  // every thread has read carry_s and wtot
        if (tid == 0) {
            double t = carry_s;
            for (int q = 0; q < kWaves; ++q) t += wtot[q];
            carry_s = t;
        }
        __syncthreads();
    }
}

// Thread per shot: the first state whose cumulative probability exceeds
// u * (the sample's total), clamped to the last state.
__global__ __launch_bounds__(kMeasureBlock) void sample_kernel(BatchDev Bt, const double* __restrict__ cdf,
                                                               const float* __restrict__ u, int S,
                                                               int32_t* __restrict__ shots) {
    const int64_t i = (int64_t)blockIdx.x * kMeasureBlock + threadIdx.x;
    if (i >= (int64_t)Bt.B * S) return;
    const int64_t b = i / S;
    const int64_t off = ldg(Bt.off + b), N = ldg(Bt.off + b + 1) - off;
    const double* cb = cdf + off;
    const double target = (double)u[i] * cb[N - 1];
    int64_t lo = 0, hi = N - 1;  // answer in [lo, hi]
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (cb[mid] > target) hi = mid;
        else lo = mid + 1;
    }
    shots[i] = (int32_t)lo;
}

// ---- amplitude-encoded inputs: components c in [goff[g], goff[g+1]) of group g

// Uc[c] = U[group[c]]
__global__ __launch_bounds__(kMeasureBlock) void replicate_u_kernel(int mm, int C, const int32_t* __restrict__ group,
                                                                    const float2* __restrict__ U,
                                                                    float2* __restrict__ Uc) {
    const int64_t i = (int64_t)blockIdx.x * kMeasureBlock + threadIdx.x;
    if (i >= (int64_t)C * mm) return;
    const int64_t c = i / mm, e = i % mm;
    Uc[i] = U[(int64_t)ldg(group + c) * mm + e];
}

// out[ooff[g] + t] = sum_c x_c A[off_c + t], components in order; workgroup
// g * T + chunk covers kChunkStates output states of group g
__global__ __launch_bounds__(kMeasureBlock) void combine_kernel(BatchDev Bt, const int64_t* __restrict__ goff,
                                                                const int64_t* __restrict__ ooff, int T,
                                                                const float2* __restrict__ x,
                                                                const float2* __restrict__ A,
                                                                float2* __restrict__ out) {
    const int g = blockIdx.x / T, ch = blockIdx.x % T;
    const int64_t c0 = ldg(goff + g), c1 = ldg(goff + g + 1);
    const int64_t o = ldg(ooff + g), N = ldg(ooff + g + 1) - o;
    const int64_t lo = (int64_t)ch * kChunkStates, hi = lo + kChunkStates < N ? lo + kChunkStates : N;
    for (int64_t t = lo + threadIdx.x; t < hi; t += kMeasureBlock) {
        float2 acc = make_float2(0.f, 0.f);
        for (int64_t c = c0; c < c1; ++c) {
            const float2 w = x[c], a = A[ldg(Bt.off + c) + t];
            acc.x += w.x * a.x - w.y * a.y;
            acc.y += w.x * a.y + w.y * a.x;
        }
        out[o + t] = acc;
    }
}

// gA[off_c + t] = conj(x_c) G[ooff[group c] + t]; workgroup c * T + chunk
__global__ __launch_bounds__(kMeasureBlock) void expand_sup_kernel(BatchDev Bt, const int32_t* __restrict__ group,
                                                                   const int64_t* __restrict__ ooff, int T,
                                                                   const float2* __restrict__ x,
                                                                   const float2* __restrict__ G,
                                                                   float2* __restrict__ gA) {
    const int64_t c = blockIdx.x / T;
    const int ch = blockIdx.x % T;
    const int64_t off = ldg(Bt.off + c), N = ldg(Bt.off + c + 1) - off;
    const int64_t o = ldg(ooff + ldg(group + c));
    const float2 w = x[c];
    const int64_t lo = (int64_t)ch * kChunkStates, hi = lo + kChunkStates < N ? lo + kChunkStates : N;
    for (int64_t t = lo + threadIdx.x; t < hi; t += kMeasureBlock) {
        const float2 gv = G[o + t];
        gA[off + t] = make_float2(w.x * gv.x + w.y * gv.y, w.x * gv.y - w.y * gv.x);
    }
}

// grad_x[c] = sum_t conj(A[off_c + t]) G[ooff[group c] + t], one workgroup per component
__global__ __launch_bounds__(kMeasureBlock) void grad_x_kernel(BatchDev Bt, const int32_t* __restrict__ group,
                                                               const int64_t* __restrict__ ooff,
                                                               const float2* __restrict__ A,
                                                               const float2* __restrict__ G,
                                                               float2* __restrict__ gx) {
    __shared__ double red[2][kMeasureBlock / 64];
    const int64_t c = blockIdx.x;
    const int64_t off = ldg(Bt.off + c), N = ldg(Bt.off + c + 1) - off;
    const int64_t o = ldg(ooff + ldg(group + c));
    double re = 0.0, im = 0.0;
    for (int64_t t = threadIdx.x; t < N; t += kMeasureBlock) {
        const float2 a = A[off + t], gv = G[o + t];
        re += (double)a.x * gv.x + (double)a.y * gv.y;
        im += (double)a.x * gv.y - (double)a.y * gv.x;
    }
    for (int s = 32; s >= 1; s >>= 1) {
        re += __shfl_xor(re, s, 64);
        im += __shfl_xor(im, s, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = re;
        red[1][threadIdx.x >> 6] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0, i = 0.0;
        for (int w = 0; w < kMeasureBlock / 64; ++w) {
            r += red[0][w];
            i += red[1][w];
        }
        gx[c] = make_float2((float)r, (float)i);
    }
}

// gU[g] = sum of gUc[c] over the group's components, in order
__global__ __launch_bounds__(kMeasureBlock) void group_sum_kernel(int mm, int G, const int64_t* __restrict__ goff,
                                                                  const float2* __restrict__ gUc,
                                                                  float2* __restrict__ gU) {
    const int64_t i = (int64_t)blockIdx.x * kMeasureBlock + threadIdx.x;
    if (i >= (int64_t)G * mm) return;
    const int64_t g = i / mm, e = i % mm;
    float2 acc = make_float2(0.f, 0.f);
    for (int64_t c = ldg(goff + g); c < ldg(goff + g + 1); ++c) {
        const float2 v = gUc[c * mm + e];
        acc.x += v.x;
        acc.y += v.y;
    }
    gU[i] = acc;
}

// p[i] = |a[i]|^2, the probability epilogue on amplitudes formed elsewhere
__global__ __launch_bounds__(kMeasureBlock) void abs2_kernel(int64_t n, const float2* __restrict__ a,
                                                             float* __restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * kMeasureBlock + threadIdx.x;
    if (i >= n) return;
    const float2 v = a[i];
    p[i] = v.x * v.x + v.y * v.y;
}

// ga[i] = 2 gp[i] a[i], the adjoint of p = |a|^2 (gradient dL/dRe + i dL/dIm)
__global__ __launch_bounds__(kMeasureBlock) void abs2_backward_kernel(int64_t n, const float2* __restrict__ a,
                                                                      const float* __restrict__ gp,
                                                                      float2* __restrict__ ga) {
    const int64_t i = (int64_t)blockIdx.x * kMeasureBlock + threadIdx.x;
    if (i >= n) return;
    const float2 v = a[i];
    const float w = 2.f * gp[i];
    ga[i] = make_float2(w * v.x, w * v.y);
}

// z[i] = 0 (a kernel, not a memset, so that captured graphs replay it as written)
__global__ __launch_bounds__(kMeasureBlock) void zero_c64_kernel(int64_t n, float2* __restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * kMeasureBlock + threadIdx.x;
    if (i < n) z[i] = make_float2(0.f, 0.f);
}

int threshold_chunks(const slos_batch_s& Bt) {
    const int64_t Q = threshold_dim(Bt.plan->m, Bt.n_max);
    return (int)std::max<int64_t>(1, (Q + kChunkPatterns - 1) / kChunkPatterns);
}

int launch_threshold(const void* fn, const slos_batch_s& Bt, const float* in, float* out, hipStream_t stream,
                     const char* what) {
    int C = threshold_chunks(Bt);
    if ((int64_t)Bt.B * C >= ((int64_t)1 << 31)) return fail(SLOS_EUNSUPPORTED, std::string(what) + ": batch too large");
    void* args[] = {(void*)&Bt.plan->d_layers, (void*)&Bt.dev, (void*)&in, (void*)&out, (void*)&C};
    hipError_t e = hipLaunchKernel(fn, dim3((unsigned)(Bt.B * C)), dim3(kMeasureBlock), args, 0, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string(what) + " launch: " + hipGetErrorString(e));
    return SLOS_OK;
}

}  // namespace

int launch_threshold_gather(const slos_batch_s& Bt, const float* p, float* out, hipStream_t stream) {
    return launch_threshold((const void*)&threshold_gather_kernel, Bt, p, out, stream, "threshold gather");
}

int launch_threshold_scatter(const slos_batch_s& Bt, const float* gP, float* gp, hipStream_t stream) {
    return launch_threshold((const void*)&threshold_scatter_kernel, Bt, gP, gp, stream, "threshold scatter");
}

int launch_sample(const slos_batch_s& Bt, const float* p, double* part, double* cdf, const float* u, int S,
                  int32_t* shots, hipStream_t stream) {
    int C = (int)mode_expect_chunks(Bt);
    if ((int64_t)Bt.B * C >= ((int64_t)1 << 31)) return fail(SLOS_EUNSUPPORTED, "fock_sample: batch too large");
    if (((int64_t)Bt.B * S + kMeasureBlock - 1) / kMeasureBlock >= ((int64_t)1 << 31))
        return fail(SLOS_EUNSUPPORTED, "fock_sample: too many shots for one launch");
    void* a1[] = {(void*)&Bt.dev, (void*)&p, (void*)&part, (void*)&C};
    hipError_t e = hipLaunchKernel((void*)&cdf_partial_kernel, dim3((unsigned)(Bt.B * C)), dim3(kMeasureBlock), a1, 0,
                                   stream);
    void* a2[] = {(void*)&Bt.dev, (void*)&p, (void*)&part, (void*)&C, (void*)&cdf};
    if (e == hipSuccess)
        e = hipLaunchKernel((void*)&cdf_scan_kernel, dim3((unsigned)(Bt.B * C)), dim3(kMeasureBlock), a2, 0, stream);
    const int64_t shots_n = (int64_t)Bt.B * S;
    if (e == hipSuccess && shots_n > 0) {
        void* a3[] = {(void*)&Bt.dev, (void*)&cdf, (void*)&u, (void*)&S, (void*)&shots};
        e = hipLaunchKernel((void*)&sample_kernel, dim3((unsigned)((shots_n + kMeasureBlock - 1) / kMeasureBlock)),
                            dim3(kMeasureBlock), a3, 0, stream);
    }
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("fock_sample launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + kMeasureBlock - 1) / kMeasureBlock); }

int launch_superposition(int kind, const SupDev& S, const slos_batch_s& Bt, const void* a0, const void* a1,
                         const void* a2, void* outp, hipStream_t stream) {
    const int m = Bt.plan->m, mm = m * m, C = Bt.B, G = S.G;
    const int T = (int)std::max<int64_t>(1, (S.max_n_states + kChunkStates - 1) / kChunkStates);
    hipError_t e = hipSuccess;
    if (kind == kSupReplicateU) {
        void* args[] = {(void*)&mm, (void*)&C, (void*)&S.group, (void*)&a0, (void*)&outp};
        e = hipLaunchKernel((void*)&replicate_u_kernel, dim3(blocks_for((int64_t)C * mm)), dim3(kMeasureBlock), args, 0,
                            stream);
    } else if (kind == kSupCombine) {  // a0 = x, a1 = A
        void* args[] = {(void*)&Bt.dev, (void*)&S.goff, (void*)&S.ooff, (void*)&T, (void*)&a0, (void*)&a1, (void*)&outp};
        e = hipLaunchKernel((void*)&combine_kernel, dim3((unsigned)((int64_t)G * T)), dim3(kMeasureBlock), args, 0,
                            stream);
    } else if (kind == kSupExpand) {  // a0 = x, a1 = G
        void* args[] = {(void*)&Bt.dev, (void*)&S.group, (void*)&S.ooff, (void*)&T, (void*)&a0, (void*)&a1, (void*)&outp};
        e = hipLaunchKernel((void*)&expand_sup_kernel, dim3((unsigned)((int64_t)C * T)), dim3(kMeasureBlock), args, 0,
                            stream);
    } else if (kind == kSupGradX) {  // a0 = A, a1 = G
        void* args[] = {(void*)&Bt.dev, (void*)&S.group, (void*)&S.ooff, (void*)&a0, (void*)&a1, (void*)&outp};
        e = hipLaunchKernel((void*)&grad_x_kernel, dim3((unsigned)C), dim3(kMeasureBlock), args, 0, stream);
    } else {  // kSupGroupSum, a0 = per-component gradients
        void* args[] = {(void*)&mm, (void*)&G, (void*)&S.goff, (void*)&a0, (void*)&outp};
        e = hipLaunchKernel((void*)&group_sum_kernel, dim3(blocks_for((int64_t)G * mm)), dim3(kMeasureBlock), args, 0,
                            stream);
    }
    (void)a2;
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("superposition kernel launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

int launch_abs2(int64_t n, const float2* a, float* p, hipStream_t stream) {
    if (n <= 0) return SLOS_OK;
    if ((n + kMeasureBlock - 1) / kMeasureBlock >= ((int64_t)1 << 31))
        return fail(SLOS_EUNSUPPORTED, "probabilities from amplitudes: too many values for one launch");
    void* args[] = {(void*)&n, (void*)&a, (void*)&p};
    hipError_t e = hipLaunchKernel((void*)&abs2_kernel, dim3(blocks_for(n)), dim3(kMeasureBlock), args, 0, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("abs2 launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

int launch_abs2_backward(int64_t n, const float2* a, const float* gp, float2* ga, hipStream_t stream) {
    if (n <= 0) return SLOS_OK;
    if ((n + kMeasureBlock - 1) / kMeasureBlock >= ((int64_t)1 << 31))
        return fail(SLOS_EUNSUPPORTED, "probabilities from amplitudes: too many values for one launch");
    void* args[] = {(void*)&n, (void*)&a, (void*)&gp, (void*)&ga};
    hipError_t e =
        hipLaunchKernel((void*)&abs2_backward_kernel, dim3(blocks_for(n)), dim3(kMeasureBlock), args, 0, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("abs2 adjoint launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

int launch_zero_c64(int64_t n, float2* z, hipStream_t stream) {
    if (n <= 0) return SLOS_OK;
    if ((n + kMeasureBlock - 1) / kMeasureBlock >= ((int64_t)1 << 31))
        return fail(SLOS_EUNSUPPORTED, "zero fill: too many values for one launch");
    void* args[] = {(void*)&n, (void*)&z};
    hipError_t e = hipLaunchKernel((void*)&zero_c64_kernel, dim3(blocks_for(n)), dim3(kMeasureBlock), args, 0, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("zero fill launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

int64_t mode_expect_chunks(const slos_batch_s& Bt) {
    const int64_t N = Bt.n_max >= 0 ? Bt.plan->N[Bt.n_max] : 1;
    return std::max<int64_t>(1, (N + kChunkStates - 1) / kChunkStates);
}

size_t mode_expect_part_bytes(const slos_batch_s& Bt) {
    return (size_t)Bt.B * mode_expect_chunks(Bt) * Bt.plan->m * sizeof(float);
}

int launch_mode_expect(const slos_batch_s& Bt, const float* p, float* part, float* out, bool distinct,
                       hipStream_t stream) {
    const slos_plan_s& P = *Bt.plan;
    int m = P.m, B = Bt.B;
    int C = (int)mode_expect_chunks(Bt);
    if ((int64_t)B * C >= ((int64_t)1 << 31)) return fail(SLOS_EUNSUPPORTED, "mode expectations: batch too large");
    void* a1[] = {(void*)&m, (void*)&P.d_layers, (void*)&Bt.dev, (void*)&p, (void*)&part, (void*)&C};
    void* fn = distinct ? (void*)&mode_expect_partial_kernel<true> : (void*)&mode_expect_partial_kernel<false>;
    hipError_t e = hipLaunchKernel(fn, dim3((unsigned)(B * C)), dim3(kMeasureBlock), a1, 0, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("mode expectation launch: ") + hipGetErrorString(e));
    void* a2[] = {(void*)&m, (void*)&B, (void*)&C, (void*)&part, (void*)&out};
    const unsigned g2 = (unsigned)(((int64_t)B * m + kMeasureBlock - 1) / kMeasureBlock);
    e = hipLaunchKernel((void*)&mode_expect_final_kernel, dim3(g2), dim3(kMeasureBlock), a2, 0, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("mode expectation launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

int launch_expand_mode_weights(const slos_batch_s& Bt, const float* w, float* gp, bool distinct, hipStream_t stream) {
    const slos_plan_s& P = *Bt.plan;
    int m = P.m;
    int C = (int)mode_expect_chunks(Bt);
    if ((int64_t)Bt.B * C >= ((int64_t)1 << 31)) return fail(SLOS_EUNSUPPORTED, "mode weight expansion: batch too large");
    void* args[] = {(void*)&m, (void*)&P.d_layers, (void*)&Bt.dev, (void*)&w, (void*)&gp, (void*)&C};
    void* fn = distinct ? (void*)&expand_kernel<true> : (void*)&expand_kernel<false>;
    hipError_t e = hipLaunchKernel(fn, dim3((unsigned)(Bt.B * C)), dim3(kMeasureBlock), args, 0, stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("mode weight expansion launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

}  // namespace slos
