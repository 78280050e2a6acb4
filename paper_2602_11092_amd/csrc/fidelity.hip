// Fidelity kernel between output states of one input Fock state under two
// interferometers (the kernel-methods reproduction of Sec. III-A):
//
//   K[a][b] = |<phi(U1_a)|phi(U2_b)>|^2,   |phi(U)> = U|s>,
//   <phi(U1)|phi(U2)> = Perm(M) / prod_i s_i!,   M = U1[:, C]^H U2[:, C],
//
// where C lists the input modes with multiplicity (n x n; Cauchy-Binet over
// the output basis turns the inner product of two C(m+n-1, n)-dimensional
// vectors into one n x n permanent).  Perm(M) by Ryser's formula,
//   Perm(M) = (-1)^n sum_{S subset of [n]} (-1)^|S| prod_i sum_{j in S} M[i][j],
// with the subsets walked in Gray-code order so that each step changes one
// column of the row sums.  FP64 arithmetic on the complex64 inputs (the
// chip's FP64 vector rate equals its unpacked FP32 rate, and Ryser's sum
// cancels strongly).
//
// Two kernels:
//  * n <= 7: one thread per (a, b) pair.  M lives in registers and the
//    2^n - 1 Gray-code steps are unrolled for the compile-time n, so every
//    index into M is static.  Lanes of a wave share a (U1 loads broadcast).
//    n = 7 takes all 256 VGPRs (one wave per SIMD) and still runs several
//    times faster than a wave per pair; n = 8 would spill.
//  * n >= 8 (and n = 0): one wave per pair.  Its lanes build M in LDS, then
//    lane l walks the Gray-code positions [l K, (l+1) K), K = ceil(2^n / 64),
//    from row sums formed directly; a fixed-order shuffle reduction combines
//    the lanes.
#include "slos_internal.h"

namespace slos {
namespace {

constexpr int kFidBlock = 256;
constexpr int kFidWaves = kFidBlock / 64;
constexpr int kFidMaxN = kMaxPhotons;

struct FidModes {
    int32_t c[kFidMaxN];  // input modes with multiplicity, ascending
};

__device__ __forceinline__ double2 z_mul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int N>
__global__ __launch_bounds__(kFidBlock) void fidelity_thread_kernel(int m, FidModes C, double scale,
                                                                    const float2* __restrict__ U1, int B1,
                                                                    const float2* __restrict__ U2, int B2,
                                                                    float* __restrict__ K) {
    const int64_t pair = (int64_t)blockIdx.x * kFidBlock + threadIdx.x;
    if (pair >= (int64_t)B1 * B2) return;
    const int64_t a = pair / B2, b = pair % B2;
    const float2* u1 = U1 + a * m * m;
    const float2* u2 = U2 + b * m * m;
    // M[r][c] = sum_k conj(U1[a][k][C_r]) U2[b][k][C_c]
    double2 M[N][N];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) M[r][c] = make_double2(0.0, 0.0);
    for (int k = 0; k < m; ++k) {
        double2 x[N], y[N];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const float2 v = u1[k * m + C.c[r]], w = u2[k * m + C.c[r]];
            x[r] = make_double2(v.x, v.y);
            y[r] = make_double2(w.x, w.y);
        }
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
            for (int c = 0; c < N; ++c) {
                M[r][c].x += x[r].x * y[c].x + x[r].y * y[c].y;
                M[r][c].y += x[r].x * y[c].y - x[r].y * y[c].x;
            }
    }
    // Ryser over the subsets in Gray-code order, starting from the empty set
    double2 rs[N];
#pragma unroll
    for (int i = 0; i < N; ++i) rs[i] = make_double2(0.0, 0.0);
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 1; q < (1 << N); ++q) {
        const int j = __builtin_ctz(q);
        const int g = q ^ (q >> 1);
        const double sgn = ((g >> j) & 1) ? 1.0 : -1.0;  // column j enters or leaves
#pragma unroll
        for (int i = 0; i < N; ++i) {
            rs[i].x += sgn * M[i][j].x;
            rs[i].y += sgn * M[i][j].y;
        }
        double2 prod = rs[0];
#pragma unroll
        for (int i = 1; i < N; ++i) prod = z_mul(prod, rs[i]);
        const double sg = (__builtin_popcount(g) & 1) ? -1.0 : 1.0;
        acc.x += sg * prod.x;
        acc.y += sg * prod.y;
    }
    const double sn = (N & 1) ? -1.0 : 1.0;
    const double re = sn * acc.x * scale, im = sn * acc.y * scale;
    K[pair] = (float)(re * re + im * im);
}

__global__ __launch_bounds__(kFidBlock) void fidelity_kernel(int m, int n, FidModes C, double scale,
                                                             const float2* __restrict__ U1, int B1,
                                                             const float2* __restrict__ U2, int B2,
                                                             float* __restrict__ K) {
    __shared__ double2 Ms[kFidWaves][kFidMaxN * kFidMaxN];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t npairs = (int64_t)B1 * B2;
    const int T = 1 << n;                       // subsets
    const int chunk = (T + 63) / 64;            // Gray-code positions per lane
    // uniform trip count over the workgroup (the barriers below need it)
    for (int64_t base = (int64_t)blockIdx.x * kFidWaves; base < npairs; base += (int64_t)gridDim.x * kFidWaves) {
        const int64_t pair = base + w;
        const bool active = pair < npairs;
        const int64_t a = active ? pair / B2 : 0, b = active ? pair % B2 : 0;
        // M[r][c] = sum_k conj(U1[a][k][C_r]) U2[b][k][C_c]
        if (active) {
            const float2* u1 = U1 + a * m * m;
            const float2* u2 = U2 + b * m * m;
            for (int e = lane; e < n * n; e += 64) {
                const int r = e / n, c = e % n;
                const int cr = C.c[r], cc = C.c[c];
                double re = 0.0, im = 0.0;
                for (int k = 0; k < m; ++k) {
                    const float2 x = u1[k * m + cr], y = u2[k * m + cc];
                    re += (double)x.x * y.x + (double)x.y * y.y;
                    im += (double)x.x * y.y - (double)x.y * y.x;
                }
                Ms[w][e] = make_double2(re, im);
            }
        }
        __syncthreads();
        double2 acc = make_double2(0.0, 0.0);
        if (active) {
            const double2* M = Ms[w];
            const int q0 = lane * chunk, q1 = min(q0 + chunk, T);
            if (q0 < q1) {
                // row sums of the subset at Gray position q0
                const int g0 = q0 ^ (q0 >> 1);
                double2 rs[kFidMaxN];
#pragma unroll
                for (int i = 0; i < kFidMaxN; ++i) {
                    rs[i] = make_double2(0.0, 0.0);
                    if (i < n)
                        for (int j = 0; j < n; ++j)
                            if ((g0 >> j) & 1) {
                                rs[i].x += M[i * n + j].x;
                                rs[i].y += M[i * n + j].y;
                            }
                }
                int g = g0;
                for (int q = q0; q < q1; ++q) {
                    if (q > q0) {  // step to position q: one column enters or leaves
                        const int j = __builtin_ctz(q);
                        const double sgn = ((g >> j) & 1) ? -1.0 : 1.0;
                        g ^= 1 << j;
#pragma unroll
                        for (int i = 0; i < kFidMaxN; ++i)
                            if (i < n) {
                                rs[i].x += sgn * M[i * n + j].x;
                                rs[i].y += sgn * M[i * n + j].y;
                            }
                    }
                    double2 prod = make_double2(1.0, 0.0);
#pragma unroll
                    for (int i = 0; i < kFidMaxN; ++i)
                        if (i < n) prod = z_mul(prod, rs[i]);
                    const double sg = (__builtin_popcount(g) & 1) ? -1.0 : 1.0;
                    acc.x += sg * prod.x;
                    acc.y += sg * prod.y;
                }
            }
        }
        // fixed-order butterfly over the wave
        for (int s = 32; s >= 1; s >>= 1) {
            acc.x += __shfl_xor(acc.x, s, 64);
            acc.y += __shfl_xor(acc.y, s, 64);
        }
        if (active && lane == 0) {
            const double sn = (n & 1) ? -1.0 : 1.0;
            const double re = sn * acc.x * scale, im = sn * acc.y * scale;
            K[pair] = (float)(re * re + im * im);
        }
        __syncthreads();  // before the next pair overwrites Ms
    }
}

}  // namespace
}  // namespace slos

using namespace slos;

extern "C" int fock_fidelity_kernel(int m, const int32_t* occ, const float* U1, int B1, const float* U2, int B2,
                                    float* K, void* stream) {
    if (m < 1 || m > kMaxModes) return fail(SLOS_EINVAL, "fock_fidelity_kernel: m must be in [1, 32]");
    if (!occ) return fail(SLOS_EINVAL, "fock_fidelity_kernel: occ is NULL");
    if (B1 < 0 || B2 < 0) return fail(SLOS_EINVAL, "fock_fidelity_kernel: negative batch size");
    FidModes C{};
    int n = 0;
    double fact = 1.0;
    for (int i = 0; i < m; ++i) {
        if (occ[i] < 0) return fail(SLOS_EINVAL, "fock_fidelity_kernel: negative occupation");
        for (int q = 0; q < occ[i]; ++q) {
            if (n == kFidMaxN) return fail(SLOS_EUNSUPPORTED, "fock_fidelity_kernel: more than 16 photons");
            C.c[n++] = i;
            fact *= (q + 1);
        }
    }
    if ((int64_t)B1 * B2 == 0) return SLOS_OK;
    if (!U1 || !U2 || !K) return fail(SLOS_EINVAL, "fock_fidelity_kernel: NULL device pointer");
    const double scale = 1.0 / fact;
    if (n >= 1 && n <= 7) {
        static void* const thread_fns[7] = {(void*)&fidelity_thread_kernel<1>, (void*)&fidelity_thread_kernel<2>,
                                            (void*)&fidelity_thread_kernel<3>, (void*)&fidelity_thread_kernel<4>,
                                            (void*)&fidelity_thread_kernel<5>, (void*)&fidelity_thread_kernel<6>,
                                            (void*)&fidelity_thread_kernel<7>};
        const int64_t blocks = ((int64_t)B1 * B2 + kFidBlock - 1) / kFidBlock;
        if (blocks >= ((int64_t)1 << 31)) return fail(SLOS_EUNSUPPORTED, "fock_fidelity_kernel: too many pairs");
        void* args[] = {(void*)&m, (void*)&C, (void*)&scale, (void*)&U1, (void*)&B1, (void*)&U2, (void*)&B2, (void*)&K};
        hipError_t e = hipLaunchKernel(thread_fns[n - 1], dim3((unsigned)blocks), dim3(kFidBlock), args, 0,
                                       (hipStream_t)stream);
        if (e != hipSuccess)
            return fail(SLOS_EHIP, std::string("fock_fidelity_kernel launch: ") + hipGetErrorString(e));
        return SLOS_OK;
    }
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SLOS_EHIP, "fock_fidelity_kernel: no HIP device");
    hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t blocks = ((int64_t)B1 * B2 + kFidWaves - 1) / kFidWaves;
    const int grid = (int)std::min<int64_t>(blocks, (int64_t)std::max(cu, 1) * 8);
    void* args[] = {(void*)&m, (void*)&n, (void*)&C, (void*)&scale, (void*)&U1, (void*)&B1,
                    (void*)&U2, (void*)&B2, (void*)&K};
    hipError_t e = hipLaunchKernel((void*)&fidelity_kernel, dim3(grid), dim3(kFidBlock), args, 0,
                                   (hipStream_t)stream);
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("fock_fidelity_kernel launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}
