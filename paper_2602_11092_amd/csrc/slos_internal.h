// Internal declarations shared by the host code and the HIP kernels of the
// strong-simulation library.  Not part of the public ABI (include/slos.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/slos.h"

namespace slos {

constexpr int kMaxModes = SLOS_MAX_MODES;
constexpr int kMaxPhotons = SLOS_MAX_PHOTONS;
constexpr int kModeBits = 5;  // predecessor entries pack (rank << 5) | mode
static_assert((1 << kModeBits) >= kMaxModes, "mode field too narrow");

// One photon layer k of the transition graph (all k-photon states over m
// modes, in basis order).  Device pointers.
struct LayerDev {
    const int32_t* pred;    // [k][N]: (rank of t - e_j in layer k-1) << 5 | j for the p-th
                            // entry of t's sorted mode list, -1 when that entry repeats
                            // the previous one (the same predecessor)
    const int32_t* succ;    // [m][N_{k-1}]: rank of t' + e_j in layer k (nullptr if forward-only)
    const float* nrm;       // [N]: sqrt(prod_j t_j!)
    const int32_t* minoff;  // [m+1]: first rank whose smallest occupied mode is >= c
    int64_t N;              // number of states C(m+k-1, k)
    int64_t cum;            // number of states with fewer than k photons (sum of N_0..N_{k-1})
};

// Per-sample description of a batch (device pointers).
struct BatchDev {
    int B;
    int n_max;               // largest photon number in the batch
    const int32_t* n;        // [B] photon number
    const int32_t* modes;    // [B][kMaxPhotons] input photon modes, ascending
    const int64_t* off;      // [B+1] output offsets
    const float* innorm;     // [B] 1/sqrt(prod_i s_i!)
    const int32_t* order;    // [B] work order (largest photon number first)
};

struct Config {
    int variant = SLOS_VARIANT_AUTO;
    int block = 0;
};

}  // namespace slos

struct slos_plan_s {
    int m = 0, n_max = 0, flags = 0;
    int device = 0;
    int num_cu = 0;
    size_t max_lds = 0;
    std::vector<int64_t> N;           // N[k], k = 0..n_max
    void* dmem = nullptr;             // all tables, one allocation
    slos::LayerDev* d_layers = nullptr;  // device copy of layers[0..n_max]
    std::vector<slos::LayerDev> layers;  // host copy (device pointers)
};

struct slos_batch_s {
    slos_plan_s* plan = nullptr;
    int B = 0;
    int n_max = 0;
    std::vector<int32_t> n_host;
    std::vector<int64_t> off_host;
    void* dmem = nullptr;
    slos::BatchDev dev{};
    slos::Config cfg[4];
};

namespace slos {

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

// ---- fused (LDS-resident) kernels: slos_fused.hip ----
size_t fused_fwd_lds_bytes(const slos_plan_s& P, int n_max);
size_t fused_bwd_lds_bytes(const slos_plan_s& P, int n_max);
bool fused_fwd_supported(const slos_plan_s& P, int n_max, int block, std::string* why);
bool fused_bwd_supported(const slos_plan_s& P, int n_max, int block, std::string* why);
int fused_default_block(const slos_plan_s& P, int n_max, bool backward);
int launch_fused_fwd(const slos_batch_s& Bt, int block, const float2* U, void* out, bool probs,
                     hipStream_t stream);
int launch_fused_bwd(const slos_batch_s& Bt, int block, const float2* U, const void* gin, bool probs,
                     float2* gU, hipStream_t stream);

// ---- layered (workspace-resident) kernels: slos_layered.hip ----
size_t layered_ws_bytes(const slos_batch_s& Bt, bool backward);
int layered_default_block(const slos_batch_s& Bt);
int launch_layered_fwd(const slos_batch_s& Bt, int block, const float2* U, void* out, bool probs,
                       void* ws, hipStream_t stream);
int launch_layered_bwd(const slos_batch_s& Bt, int block, const float2* U, const void* gin, bool probs,
                       float2* gU, void* ws, hipStream_t stream);

}  // namespace slos

// complex helpers (device)
__device__ __forceinline__ float2 c_zero() { return make_float2(0.f, 0.f); }
// acc += a * b
__device__ __forceinline__ void c_fma(float2& acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
}
// acc += conj(a) * b
__device__ __forceinline__ void c_fma_conj(float2& acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(-a.y, b.x, acc.y);
}
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
