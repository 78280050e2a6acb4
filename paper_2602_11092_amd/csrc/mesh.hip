// Interferometer mesh U(x, theta) of phase shifters and beam splitters
// (arXiv 2602.11092, Sec. II-A-3: trainable phases define U(theta);
// Sec. II-C-1: angle encoding U(x, theta) = W2 S(x) W1) and its adjoint.
//
// Rectangular mesh: column c holds MZIs on pairs (k, k+1), k = c mod 2 + 2p.
// MZIs of one column touch disjoint pairs, so a column is applied to all
// rows at once.  W1 = columns [0, m/2), W2 = the rest.  For batches that fit
// one resident round of workgroups, every workgroup of the forward (one per
// sample) forms all 2x2 MZI matrices and sweeps the columns of both factors
// in its own LDS, which keeps a separate single-workgroup launch off the
// serial chain; larger batches form the factors once, in one workgroup, as
// the adjoint does.  The forward then forms U_b = W2 diag(e^{i enc x_b}) W1.
// The adjoint computes each sample's contribution to dL/dW1 and dL/dW2 (and
// dL/dx_b) in its own workgroup, sums them over the batch in a fixed order,
// then sweeps the columns backwards, recovering each column's input as
// T^H times its output (T unitary).
#include <mutex>

#include "slos_internal.h"

namespace slos {
namespace {

struct Mzi {
    float2 t00, t01, t10, t11;
    float2 eth, etp;  // e^{i theta}, e^{i (theta + phi)} (for dT/dtheta)
};

// MZI(theta, phi) = BS PS(theta) BS PS(phi), BS = (1/sqrt2)[[1,i],[i,1]],
// PS(a) = diag(e^{ia}, 1):
//   T = 1/2 [[ (e^{i th} - 1) e^{i ph},  i (e^{i th} + 1) ],
//            [ i (e^{i th} + 1) e^{i ph}, 1 - e^{i th}     ]]
__device__ __forceinline__ Mzi mzi(float th, float ph) {
    float st, ct, sp, cp;
    sincosf(th, &st, &ct);
    sincosf(ph, &sp, &cp);
    const float2 em1 = make_float2(0.5f * (ct - 1.f), 0.5f * st);  // (e^{i th} - 1)/2
    const float2 ep1 = make_float2(0.5f * (ct + 1.f), 0.5f * st);  // (e^{i th} + 1)/2
    const float2 iep1 = make_float2(-ep1.y, ep1.x);                // i (e^{i th} + 1)/2
    const float2 eph = make_float2(cp, sp);
    Mzi T;
    T.t00 = make_float2(em1.x * eph.x - em1.y * eph.y, em1.x * eph.y + em1.y * eph.x);
    T.t01 = iep1;
    T.t10 = make_float2(iep1.x * eph.x - iep1.y * eph.y, iep1.x * eph.y + iep1.y * eph.x);
    T.t11 = make_float2(-em1.x, -em1.y);
    T.eth = make_float2(ct, st);
    T.etp = make_float2(ct * cp - st * sp, ct * sp + st * cp);
    return T;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}
// Sum over each half-wave (lanes 0..31, 32..63) in a fixed order; lanes 31
// and 63 end up holding the two sums.
__device__ __forceinline__ float sum32(float v) {
    v += dpp<0xB1>(v);        // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);        // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);       // row_half_mirror
    v += dpp<0x140>(v);       // row_mirror: every lane holds its row's sum
    v += dpp<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    return v;
}

__host__ __device__ __forceinline__ int col_start(int c, int m) {
    return ((c + 1) / 2) * (m / 2) + (c / 2) * ((m - 1) / 2);
}
__host__ __device__ __forceinline__ int num_mzi(int m) { return m * (m - 1) / 2; }

// Workspace layout (float2 units): W[2][m][m] | T[nmzi][6] | G[2][m][m] | partial[B][2][m][m]
struct MeshWs {
    float2* W;
    Mzi* T;
    float2* G;
    float2* partial;
};
__host__ __device__ inline size_t mesh_ws_floats2(int m, int B) {
    return (size_t)2 * m * m + (size_t)num_mzi(m) * 6 + (size_t)2 * m * m + (size_t)B * 2 * m * m;
}
__host__ __device__ inline MeshWs mesh_ws_split(void* ws, int m) {
    MeshWs w;
    w.W = (float2*)ws;
    w.T = (Mzi*)(w.W + 2 * m * m);
    w.G = (float2*)(w.T + num_mzi(m));
    w.partial = w.G + 2 * m * m;
    return w;
}

// Builds W1 (W[0]) and W2 (W[1]) in LDS and every MZI matrix in Ts.  Needs
// a workgroup of 1024 threads: half = tid / 512, pair slot = (tid % 512) / 32,
// column of W = tid % 32.  With Wout and Tout non-NULL, workgroup 0 also
// stores the factors in Wout[2][m][m] and the MZI records in Tout (the
// adjoint's per-sample kernel and sweep read them).
__device__ __forceinline__ void factors_into_lds(int m, const float* __restrict__ theta, float2 (&W)[2][32][33],
                                                 Mzi (&Ts)[496], float2* __restrict__ Wout,
                                                 Mzi* __restrict__ Tout) {
    const int tid = threadIdx.x;
    const bool store = Wout != nullptr && blockIdx.x == 0;
    const int nm = num_mzi(m);
    for (int q = tid; q < nm; q += 1024) {
        const Mzi T = mzi(theta[2 * q], theta[2 * q + 1]);
        Ts[q] = T;
        if (store) Tout[q] = T;
    }
    const int half = tid >> 9, pr = (tid >> 5) & 15, col = tid & 31;
    for (int r = pr; r < 32; r += 16) W[half][r][col] = make_float2((r == col) ? 1.f : 0.f, 0.f);
    __syncthreads();
    const int split = m / 2;
    const int nsteps = max(split, m - split);
    for (int s = 0; s < nsteps; ++s) {
        const int c = half == 0 ? s : split + s;
        const int cend = half == 0 ? split : m;
        const int k = (c & 1) + 2 * pr;
        if (c < cend && k <= m - 2 && col < m) {
            const Mzi T = Ts[col_start(c, m) + pr];
            const float2 x0 = W[half][k][col], x1 = W[half][k + 1][col];
            float2 y0 = cmul(T.t00, x0), y1 = cmul(T.t10, x0);
            c_fma(y0, T.t01, x1);
            c_fma(y1, T.t11, x1);
            W[half][k][col] = y0;
            W[half][k + 1][col] = y1;
        }
        __syncthreads();
    }
    if (store)
        for (int r = pr; r < m; r += 16)
            if (col < m) Wout[((size_t)half * m + r) * m + col] = W[half][r][col];
}

// The factors alone (the adjoint's per-sample kernel reads them from the
// workspace): one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void mesh_factors_kernel(int m, const float* __restrict__ theta,
                                                            float2* __restrict__ Wout, Mzi* __restrict__ Tout) {
    __shared__ float2 W[2][32][33];
    __shared__ Mzi Ts[496];
    factors_into_lds(m, theta, W, Ts, Wout, Tout);
}

// U_b = W2 diag(S_b) W1, one sample per block (the factors formed in LDS).
constexpr int kMeshNT = 1024;  // threads of mesh_apply_kernel: the layout factors_into_lds needs

__global__ __launch_bounds__(kMeshNT) void mesh_apply_kernel(int m, const float* __restrict__ theta,
                                                         const float* __restrict__ x, float enc,
                                                         float2* __restrict__ U) {
    __shared__ float2 W[2][32][33];
    __shared__ Mzi Ts[496];
    __shared__ float2 A[32][33];  // diag(S) W1
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    factors_into_lds(m, theta, W, Ts, nullptr, nullptr);
    for (int q = tid; q < m * m; q += kMeshNT) {
        const int r = q / m, c = q % m;
        float2 s = make_float2(1.f, 0.f);
        if (x) {
            float sn, cs;
            sincosf(enc * x[(size_t)b * m + r], &sn, &cs);
            s = make_float2(cs, sn);
        }
        A[r][c] = cmul(s, W[0][r][c]);
    }
    __syncthreads();
    for (int q = tid; q < m * m; q += kMeshNT) {
        const int j = q / m, i = q % m;
        float2 acc = c_zero();
        for (int k = 0; k < m; ++k) c_fma(acc, W[1][j][k], A[k][i]);
        U[(size_t)b * m * m + q] = acc;
    }
}

// U_b = W2 diag(S_b) W1, one sample per block, from factors formed once by
// mesh_factors_kernel (the forward's path for batches beyond one resident
// round of mesh_apply_kernel workgroups, where sweeping the factors in every
// workgroup would cost more than the shared launch).
__global__ __launch_bounds__(256) void mesh_apply_shared_kernel(int m, const float2* __restrict__ Wf,
                                                                const float* __restrict__ x, float enc,
                                                                float2* __restrict__ U) {
    __shared__ float2 W2[32][33];
    __shared__ float2 A[32][33];  // diag(S) W1
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    for (int q = tid; q < m * m; q += 256) {
        const int r = q / m, c = q % m;
        float2 s = make_float2(1.f, 0.f);
        if (x) {
            float sn, cs;
            sincosf(enc * x[(size_t)b * m + r], &sn, &cs);
            s = make_float2(cs, sn);
        }
        A[r][c] = cmul(s, Wf[(size_t)r * m + c]);
        W2[r][c] = Wf[(size_t)m * m + q];
    }
    __syncthreads();
    for (int q = tid; q < m * m; q += 256) {
        const int j = q / m, i = q % m;
        float2 acc = c_zero();
        for (int k = 0; k < m; ++k) c_fma(acc, W2[j][k], A[k][i]);
        U[(size_t)b * m * m + q] = acc;
    }
}

// One sample per block: Y = W2^H G_b, V = G_b W1^H; contributions
// conj(S_b[r]) Y[r][c] to dL/dW1 and V[r][c] conj(S_b[c]) to dL/dW2, and
// dL/dx_b[k] = -enc Im(conj((W2^H G_b W1^H)[k][k]) S_b[k]).
__global__ __launch_bounds__(256) void mesh_bwd_samples_kernel(int m, const float2* __restrict__ Wf,
                                                               const float* __restrict__ x, float enc,
                                                               const float2* __restrict__ gU,
                                                               float* __restrict__ gx,
                                                               float2* __restrict__ partial) {
    __shared__ float2 W1[32][33], W2[32][33], G[32][33], Y[32][33];
    __shared__ float2 S[32];
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    for (int q = tid; q < m * m; q += 256) {
        const int r = q / m, c = q % m;
        W1[r][c] = Wf[q];
        W2[r][c] = Wf[(size_t)m * m + q];
        G[r][c] = gU[(size_t)b * m * m + q];
    }
    if (tid < m) {
        float2 s = make_float2(1.f, 0.f);
        if (x) {
            float sn, cs;
            sincosf(enc * x[(size_t)b * m + tid], &sn, &cs);
            s = make_float2(cs, sn);
        }
        S[tid] = s;
    }
    __syncthreads();
    float2* pa = partial + (size_t)b * 2 * m * m;
    float2* pb = pa + m * m;
    for (int q = tid; q < m * m; q += 256) {
        const int r = q / m, c = q % m;
        float2 y = c_zero(), v = c_zero();
        for (int k = 0; k < m; ++k) {
            c_fma_conj(y, W2[k][r], G[k][c]);    // (W2^H G)[r][c]
            c_fma(v, G[r][k], cconj(W1[c][k]));  // (G W1^H)[r][c]
        }
        Y[r][c] = y;
        pa[q] = cmul(cconj(S[r]), y);
        pb[q] = cmul(v, cconj(S[c]));
    }
    if (gx) {
        __syncthreads();
        if (tid < m) {
            float2 gs = c_zero();  // (W2^H G W1^H)[k][k]
            for (int i = 0; i < m; ++i) c_fma(gs, Y[tid][i], cconj(W1[tid][i]));
            const float2 z = cmul(cconj(gs), S[tid]);
            gx[(size_t)b * m + tid] = -enc * z.y;
        }
    }
}

// G[e] = sum_b partial[b][e] for e < 2 m^2, in a fixed order: 64 lanes per
// entry take the samples in a strided order, then a fixed tree.
__global__ __launch_bounds__(256) void mesh_bwd_reduce_kernel(int m, int B, const float2* __restrict__ partial,
                                                              float2* __restrict__ G) {
    __shared__ float2 red[256];
    const int E = 2 * m * m;
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int r = threadIdx.x & 63;
    float2 s = c_zero();
    if (e < E) {
#pragma unroll 8
        for (int b = r; b < B; b += 64) s = c_add(s, partial[(size_t)b * E + e]);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (r < w) red[threadIdx.x] = c_add(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (r == 0 && e < E) G[e] = red[threadIdx.x];
}

// Reverse column sweeps of both factors.  1024 threads: half = tid / 512,
// pair slot = (tid % 512) / 32, column of W = tid % 32.
// Each step keeps its MZIs' reduced products G_T (four complex numbers per
// MZI) in LDS; the gradients are formed from them after the sweep, one
// thread per MZI, off the sequential path.
__global__ __launch_bounds__(1024) void mesh_bwd_sweep_kernel(int m, const float* __restrict__ theta,
                                                              const float2* __restrict__ Wf,
                                                              const Mzi* __restrict__ Tm,
                                                              const float2* __restrict__ Gf,
                                                              float* __restrict__ gtheta) {
    __shared__ float2 X[2][32][33], G[2][32][33];
    __shared__ Mzi Ts[496];    // every MZI record, staged once (the sweep's steps read them in order)
    __shared__ float2 GT[496][4];  // each MZI's G_T
    const int tid = threadIdx.x;
    const int half = tid >> 9, pr = (tid >> 5) & 15, col = tid & 31;
    for (int q = tid; q < num_mzi(m); q += 1024) Ts[q] = Tm[q];
    for (int r = pr; r < m; r += 16) {
        if (col < m) {
            const int q = r * m + col;
            G[half][r][col] = Gf[(size_t)half * m * m + q];
            X[half][r][col] = Wf[(size_t)half * m * m + q];
        }
    }
    __syncthreads();
    const int split = m / 2;
    const int nsteps = max(split, m - split);
    for (int s = nsteps - 1; s >= 0; --s) {
        const int c = half == 0 ? s : split + s;
        const int cend = half == 0 ? split : m;
        const int k = (c & 1) + 2 * pr;
        if (c < cend && k <= m - 2) {  // uniform over the 32 lanes of this pair slot
            const int q = col_start(c, m) + pr;
            const Mzi T = Ts[q];
            float2 r0 = c_zero(), r1 = c_zero(), g0 = c_zero(), g1 = c_zero();
            if (col < m) {
                const float2 x0 = X[half][k][col], x1 = X[half][k + 1][col];
                c_fma_conj(r0, T.t00, x0);  // (T^H X) row 0
                c_fma_conj(r0, T.t10, x1);
                c_fma_conj(r1, T.t01, x0);  // row 1
                c_fma_conj(r1, T.t11, x1);
                g0 = G[half][k][col];
                g1 = G[half][k + 1][col];
            }
            // G_T[a][b] = sum_col g_a conj(r_b)  (half-wave sums: lane col 31 holds them)
            float2 p[4] = {cmul(g0, cconj(r0)), cmul(g0, cconj(r1)), cmul(g1, cconj(r0)), cmul(g1, cconj(r1))};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                p[e].x = sum32(p[e].x);
                p[e].y = sum32(p[e].y);
            }
            if (col == 31) {
#pragma unroll
                for (int e = 0; e < 4; ++e) GT[q][e] = p[e];
            }
            if (col < m) {
                X[half][k][col] = r0;
                X[half][k + 1][col] = r1;
                float2 h0 = c_zero(), h1 = c_zero();
                c_fma_conj(h0, T.t00, g0);
                c_fma_conj(h0, T.t10, g1);
                c_fma_conj(h1, T.t01, g0);
                c_fma_conj(h1, T.t11, g1);
                G[half][k][col] = h0;
                G[half][k + 1][col] = h1;
            }
        }
        __syncthreads();
    }
    for (int q = tid; q < num_mzi(m); q += 1024) {
        const Mzi T = Ts[q];
        const float2 p0 = GT[q][0], p1 = GT[q][1], p2 = GT[q][2], p3 = GT[q][3];
        const float2 eth = T.eth;
        const float2 etp = T.etp;
        // dT/dtheta = 1/2 [[ i e^{i(th+ph)}, -e^{i th} ], [ -e^{i(th+ph)}, -i e^{i th} ]]
        const float2 d00 = make_float2(-0.5f * etp.y, 0.5f * etp.x);
        const float2 d01 = make_float2(-0.5f * eth.x, -0.5f * eth.y);
        const float2 d10 = make_float2(-0.5f * etp.x, -0.5f * etp.y);
        const float2 d11 = make_float2(0.5f * eth.y, -0.5f * eth.x);
        float gth = 0.f;
        gth += p0.x * d00.x + p0.y * d00.y;
        gth += p1.x * d01.x + p1.y * d01.y;
        gth += p2.x * d10.x + p2.y * d10.y;
        gth += p3.x * d11.x + p3.y * d11.y;
        // dT/dphi = [[ i t00, 0 ], [ i t10, 0 ]]
        const float2 e00 = make_float2(-T.t00.y, T.t00.x);
        const float2 e10 = make_float2(-T.t10.y, T.t10.x);
        const float gph = p0.x * e00.x + p0.y * e00.y + p2.x * e10.x + p2.y * e10.y;
        gtheta[2 * q] = gth;
        gtheta[2 * q + 1] = gph;
    }
}

size_t mesh_ws(int m, int B) { return mesh_ws_floats2(m, B) * sizeof(float2); }

}  // namespace

// ---- scratch of the allocation-free adjoint (mesh_to_unitary_backward_noalloc)
// One copy per device, held until the process ends.  In host code `scratch`
// names a host-side stand-in, never the device memory: kernels and copies
// take the address hipGetSymbolAddress returns for the current device.
constexpr size_t kMeshScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kMeshScratchBytes];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0)
        return fail(SLOS_EHIP, "mesh_to_unitary_backward_noalloc: no current HIP device");
    if (dev >= kScratchDevices)
        return fail(SLOS_EUNSUPPORTED, "mesh_to_unitary_backward_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SLOS_EHIP, std::string("mesh_to_unitary_backward_noalloc: scratch lookup failed: ") +
                                       hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SLOS_OK;
}

}  // namespace
}  // namespace slos

using namespace slos;

extern "C" int mesh_workspace_bytes(int m, int B, size_t* bytes) {
    if (!bytes) return fail(SLOS_EINVAL, "mesh_workspace_bytes: bytes is NULL");
    if (m < 2 || m > kMaxModes || B < 0) return fail(SLOS_EINVAL, "mesh_workspace_bytes: bad m or B");
    *bytes = mesh_ws(m, std::max(B, 1));
    return SLOS_OK;
}

extern "C" int mesh_to_unitary(int m, int B, const float* theta, const float* x, float enc_scale, float* U,
                               void* ws, size_t ws_bytes, void* stream) {
    if (m < 2 || m > kMaxModes) return fail(SLOS_EINVAL, "mesh_to_unitary: m must be in [2, 32]");
    if (B < 0) return fail(SLOS_EINVAL, "mesh_to_unitary: B < 0");
    if (!x && B != 1) return fail(SLOS_EINVAL, "mesh_to_unitary: B must be 1 when x is NULL");
    if (B == 0) return SLOS_OK;
    if (!theta || !U) return fail(SLOS_EINVAL, "mesh_to_unitary: NULL pointer");
    if (!ws || ws_bytes < mesh_ws(m, B)) return fail(SLOS_EWORKSPACE, "mesh_to_unitary: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    // up to one resident round of workgroups (two of 1024 threads per CU),
    // every workgroup forms the factors itself; beyond that, once, shared
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SLOS_EHIP, "mesh_to_unitary: no HIP device");
    (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (B <= 2 * std::max(cu, 1)) {
        hipLaunchKernelGGL(mesh_apply_kernel, dim3(B), dim3(kMeshNT), 0, s, m, theta, x, enc_scale, (float2*)U);
    } else {
        MeshWs w = mesh_ws_split(ws, m);
        hipLaunchKernelGGL(mesh_factors_kernel, dim3(1), dim3(1024), 0, s, m, theta, w.W, w.T);
        hipLaunchKernelGGL(mesh_apply_shared_kernel, dim3(B), dim3(256), 0, s, m, (const float2*)w.W, x, enc_scale,
                           (float2*)U);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("mesh_to_unitary launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

extern "C" int mesh_to_unitary_backward(int m, int B, const float* theta, const float* x, float enc_scale,
                                        const float* grad_U, float* grad_theta, float* grad_x, void* ws,
                                        size_t ws_bytes, void* stream) {
    if (m < 2 || m > kMaxModes) return fail(SLOS_EINVAL, "mesh_to_unitary_backward: m must be in [2, 32]");
    if (B < 1) return fail(SLOS_EINVAL, "mesh_to_unitary_backward: B < 1");
    if (!x && B != 1) return fail(SLOS_EINVAL, "mesh_to_unitary_backward: B must be 1 when x is NULL");
    if (!x && grad_x) return fail(SLOS_EINVAL, "mesh_to_unitary_backward: grad_x must be NULL when x is NULL");
    if (!theta || !grad_U || !grad_theta) return fail(SLOS_EINVAL, "mesh_to_unitary_backward: NULL pointer");
    if (!ws || ws_bytes < mesh_ws(m, B)) return fail(SLOS_EWORKSPACE, "mesh_to_unitary_backward: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    MeshWs w = mesh_ws_split(ws, m);
    float* gx = (x && grad_x) ? grad_x : nullptr;
    hipLaunchKernelGGL(mesh_factors_kernel, dim3(1), dim3(1024), 0, s, m, theta, w.W, w.T);
    hipLaunchKernelGGL(mesh_bwd_samples_kernel, dim3(B), dim3(256), 0, s, m, (const float2*)w.W, x, enc_scale,
                       (const float2*)grad_U, gx, w.partial);
    hipLaunchKernelGGL(mesh_bwd_reduce_kernel, dim3((2 * m * m + 3) / 4), dim3(256), 0, s, m, B,
                       (const float2*)w.partial, w.G);
    hipLaunchKernelGGL(mesh_bwd_sweep_kernel, dim3(1), dim3(1024), 0, s, m, theta, (const float2*)w.W,
                       (const Mzi*)w.T, (const float2*)w.G, grad_theta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SLOS_EHIP, std::string("mesh_to_unitary_backward launch: ") + hipGetErrorString(e));
    return SLOS_OK;
}

extern "C" int mesh_to_unitary_backward_noalloc(int m, int B, const float* theta, const float* x, float enc_scale,
                                                const float* grad_U, float* grad_theta, float* grad_x,
                                                void* stream) {
    if (m < 2 || m > kMaxModes) return fail(SLOS_EINVAL, "mesh_to_unitary_backward_noalloc: m must be in [2, 32]");
    if (B < 1) return fail(SLOS_EINVAL, "mesh_to_unitary_backward_noalloc: B < 1");
    if (mesh_ws(m, B) > kMeshScratchBytes)
        return fail(SLOS_EUNSUPPORTED, "mesh_to_unitary_backward_noalloc: needs " + std::to_string(mesh_ws(m, B)) +
                                           " bytes of scratch, more than the " + std::to_string(kMeshScratchBytes) +
                                           " the library holds");
    void* ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != SLOS_OK) return rc;
    // the same kernels as the workspace call; every scratch word they read is
    // written earlier in the same call, so nothing needs clearing
    return mesh_to_unitary_backward(m, B, theta, x, enc_scale, grad_U, grad_theta, grad_x, ws, kMeshScratchBytes,
                                    stream);
}
