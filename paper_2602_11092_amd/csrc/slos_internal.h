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
constexpr int kModeBits = 5;  // host tables pack (rank << 5) | mode
static_assert((1 << kModeBits) >= kMaxModes, "mode field too narrow");
// Device predecessor entries hold two byte offsets: (rank << 11) | (mode << 3),
// the LDS offset of the predecessor's amplitude (rank * 8 = (e >> 11) << 3)
// and of the coefficient U[mode][i_k] in a 33-slot column whose slot 32 is
// zero.  An empty entry points at that zero slot (and at predecessor 0).
// successor rows are padded to a multiple of four entries (16-byte loads)
__host__ __device__ constexpr int succ_row_len(int m) { return (m + 3) & ~3; }
constexpr int kPredRankShift = 11;
constexpr int kPredModeMask = 0x7FF;
constexpr int kPredEmpty = 32 << 3;
constexpr int kUcolSlots = 33;

// One photon layer k of the transition graph (all k-photon states over m
// modes, in basis order).  Device pointers.
struct LayerDev {
    const int4* predv;      // [ngrp][N] int4: entries 4g..4g+3 of t's predecessor list, each
                            // (rank of t - e_j in layer k-1) << 5 | j for that entry of t's
                            // sorted mode list, -1 when it repeats the previous entry (same
                            // predecessor) or lies past k
    const int32_t* succ;    // [N_{k-1}][MP]: rank in layer k of t' + e_j, one row per t'
                            // (MP = succ_row_len(m); nullptr if forward-only)
    const float* nrm;       // [N]: sqrt(prod_j t_j!)
    const int32_t* minoff;  // [m+1]: first rank whose smallest occupied mode is >= c
    int64_t N;              // number of states C(m+k-1, k)
    int64_t cum;            // number of states with fewer than k photons (sum of N_0..N_{k-1})
    int32_t ngrp;           // ceil(k / 4)
    int32_t pad;
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

// Global-address-space views of table pointers that kernels read out of
// descriptor structs (such loads would otherwise be emitted as flat loads).
typedef __attribute__((address_space(1))) const int4 g_int4;
typedef __attribute__((address_space(1))) const int32_t g_int;
typedef __attribute__((address_space(1))) const float g_float;
typedef __attribute__((address_space(1))) const float2 g_float2;

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

// Load through a global-address-space view of p.
template <class T>
__device__ __forceinline__ T ldg(const T* p) {
    return *(__attribute__((address_space(1))) const T*)p;
}
