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
// Device predecessor entries (uint32): (mode << shift) | (rank << 3), the
// rank of t - e_mode in layer k-1 and the output mode.  With shift 25
// ("compact", layer k-1 below 2^19 states) e >> 22 is the byte offset of the
// coefficient U[mode][i_k] in a 33-slot column and e & 0x3FFFF8 the byte
// offset of the predecessor's amplitude, one instruction each; larger layers
// use shift 26 (ranks below 2^23).  An empty entry (a repeated predecessor,
// or past the photon number) names mode 32, the column's zero slot, and
// rank 0.  Successor entries (uint32) are byte offsets, rank * 8.
constexpr int kPredShiftCompact = 25;
constexpr int kPredShiftWide = 26;
constexpr int64_t kPredCompactStates = (int64_t)1 << 19;
constexpr int64_t kPredWideStates = (int64_t)1 << 23;
constexpr uint32_t kPredCompactRankMask = 0x3FFFF8u;  // rank * 8 in a compact entry
constexpr int kPredCompactModeShift = 22;             // e >> 22 = mode * 8 in a compact entry
__host__ __device__ constexpr uint32_t pred_empty(int shift) { return 32u << shift; }
__host__ __device__ constexpr uint32_t pred_rank_mask(int shift) { return ((1u << shift) - 1u) & ~7u; }
constexpr int kUcolSlots = 33;

// One photon layer k of the transition graph (all k-photon states over m
// modes, in basis order).  Device pointers.
struct LayerDev {
    const uint4* predv;     // [ngrp][N] groups of four predecessor entries: entries 4g..4g+3
                            // of t's sorted mode list (empty past k or where a mode repeats)
    const uint32_t* succ;   // [ceil(m/4)][N_{k-1}][4]: entry j & 3 of group j / 4 is the byte
                            // offset (rank * 8) in layer k of t' + e_j; padding entries are 0
                            // (nullptr if forward-only)
    const float* nrm;       // [N]: sqrt(prod_j t_j!)
    const int32_t* minoff;  // [m+1]: first rank whose smallest occupied mode is >= c
    int64_t N;              // number of states C(m+k-1, k)
    int64_t cum;            // number of states with fewer than k photons (sum of N_0..N_{k-1})
    int32_t ngrp;           // ceil(k / 4)
    int32_t pred_shift;     // kPredShiftCompact or kPredShiftWide
    // threshold-detector tables (plans created with SLOS_PLAN_THRESHOLD, else nullptr):
    // click pattern q (by click count, then lexicographic) holds the states
    // thr_idx[thr_ptr[q] .. thr_ptr[q+1]), ascending
    const int32_t* thr_ptr; // [Q + 1]
    const int32_t* thr_idx; // [N]
    int64_t Q;              // number of click patterns of k photons
    // the patterns cut into runs of whole patterns holding at most
    // kThrChunkStates states: run r is patterns [thr_chunk[r], thr_chunk[r+1])
    const int32_t* thr_chunk; // [thr_nchunk + 1]
    int32_t thr_nchunk;
    // predv and nrm with the states in click-pattern order (row s is state
    // thr_idx[s]), so that a pass in that order loads them coalesced
    const uint4* thr_predv;   // [ngrp][N]
    const float* thr_nrm;     // [N]
};

// States per run of whole click patterns in the fused threshold epilogue
// (their probabilities are staged in LDS as floats).
constexpr int kThrChunkStates = 16384;

// Per-sample description of a batch (device pointers).
struct BatchDev {
    int B;
    int n_max;               // largest photon number in the batch
    const int32_t* n;        // [B] photon number
    const int32_t* modes;    // [B][kMaxPhotons] input photon modes, ascending
    const int64_t* off;      // [B+1] output offsets
    const float* innorm;     // [B] 1/sqrt(prod_i s_i!)
    const int32_t* order;    // [B] work order (largest photon number first)
    const int64_t* thr_off;  // [B+1] offsets of the click-pattern outputs
    // work items of the two-sample kernels: consecutive samples of the work
    // order with equal photon numbers, (a, b); b = -1 for a sample alone
    const int2* pairs;       // [npairs]
    int npairs;
};

struct Config {
    int variant = SLOS_VARIANT_AUTO;
    int block = 0;
    int tile = 0;  // states per thread of the variant's main loop (0: its default)
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
    std::vector<int64_t> thr_off_host;  // click-pattern output offsets
    void* dmem = nullptr;
    slos::BatchDev dev{};
    slos::Config cfg[9];
    int npairs = 0;
};

namespace slos {

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

// ---- fused (LDS-resident) kernels: slos_fused.hip ----
size_t fused_fwd_lds_bytes(const slos_plan_s& P, int n_max);
size_t fused_bwd_lds_bytes(const slos_plan_s& P, int n_max);
// expect: the per-mode expectation epilogue (per-lane LDS accumulators)
bool fused_fwd_supported(const slos_plan_s& P, int n_max, int block, std::string* why, bool expect = false);
// the fused adjoint's instances for restricted-space plans (slos_fused_r.hip)
void* pick_bwd_restricted(int block, int m, int64_t Np);
// successors that leave a restricted space are marked so in the successor tables
constexpr uint32_t kNoSuccessor = 0xFFFFFFF8u;  // (uint32)(-1) << 3
inline bool restricted_plan(const slos_plan_s& P) { return (P.flags & (SLOS_PLAN_UNBUNCHED | SLOS_PLAN_DUAL_RAIL)) != 0; }
// whether the fused forward's click-pattern epilogue (epi 4) serves this plan and block
bool fused_threshold_supported(const slos_plan_s& P, int n_max, int block);
bool fused_bwd_supported(const slos_plan_s& P, int n_max, int block, std::string* why);
int fused_default_block(const slos_plan_s& P, int n_max, bool backward);
// epi: 0 amplitudes, 1 probabilities, 2 per-mode expectations, 3 per-mode
// click probabilities (both [B][m] floats)
int launch_fused_fwd(const slos_batch_s& Bt, int block, const float2* U, void* out, int epi,
                     hipStream_t stream);
int launch_fused_bwd(const slos_batch_s& Bt, int block, const float2* U, const void* gin, bool probs,
                     float2* gU, hipStream_t stream);

// ---- two samples per workgroup (forward amplitudes and probabilities): slos_fused2.hip ----
bool fused_pairs_supported(const slos_plan_s& P, int n_max, int block, std::string* why);
// tile: last-layer states per thread per iteration, 2, 4 or 8 (0: 4)
int launch_fused_pairs_fwd(const slos_batch_s& Bt, int block, int tile, const float2* U, void* out, bool probs,
                           hipStream_t stream);

// ---- layered (workspace-resident) kernels: slos_layered.hip ----
size_t layered_ws_bytes(const slos_batch_s& Bt, bool backward);
int layered_default_block(const slos_batch_s& Bt);
int launch_layered_fwd(const slos_batch_s& Bt, int block, const float2* U, void* out, bool probs,
                       void* ws, hipStream_t stream);
int launch_layered_bwd(const slos_batch_s& Bt, int block, const float2* U, const void* gin, bool probs,
                       float2* gU, void* ws, hipStream_t stream);

// ---- measurement kernels: slos_measure.hip ----
// States per workgroup in the measurement kernels' (sample, chunk) grids.
constexpr int64_t kMeasureChunkStates = 16384;
// out[b][j] = sum_t t_j p[off_b + t] (p: the batch's probabilities), via
// per-chunk partial sums in `part` (mode_expect_part_bytes bytes)
// (distinct: per-mode click probabilities, sum_t [t_j > 0] p[off_b + t])
size_t mode_expect_part_bytes(const slos_batch_s& Bt);
int launch_mode_expect(const slos_batch_s& Bt, const float* p, float* part, float* out, bool distinct,
                       hipStream_t stream);
// gp[off_b + t] = sum_j t_j w[b][j]  (distinct: sum_j [t_j > 0] w[b][j])
int launch_expand_mode_weights(const slos_batch_s& Bt, const float* w, float* gp, bool distinct, hipStream_t stream);
// out[thr_off_b + q] = sum of p over click pattern q's states
int launch_threshold_gather(const slos_batch_s& Bt, const float* p, float* out, hipStream_t stream);
// gp[off_b + t] = gP[thr_off_b + pattern(t)]
int launch_threshold_scatter(const slos_batch_s& Bt, const float* gP, float* gp, hipStream_t stream);
int64_t threshold_dim(int m, int n);
// shots[b][s] <- first t with cdf_b[t] > u[b][s] cdf_b[N_b - 1]; part: B * chunks doubles
// (chunks = mode_expect_chunks), cdf: out_len doubles
int64_t mode_expect_chunks(const slos_batch_s& Bt);

// Amplitude-encoded inputs: the batch's samples are components; group g
// holds components [goff[g], goff[g+1]) and owns outputs [ooff[g], ooff[g+1]).
struct SupDev {
    int G = 0;
    const int32_t* group = nullptr;  // [C] group of each component
    const int64_t* goff = nullptr;   // [G+1]
    const int64_t* ooff = nullptr;   // [G+1]
    int64_t max_n_states = 1;        // largest output block of a group
};
enum { kSupReplicateU, kSupCombine, kSupExpand, kSupGradX, kSupGroupSum };
int launch_superposition(int kind, const SupDev& S, const slos_batch_s& Bt, const void* a0, const void* a1,
                         const void* a2, void* out, hipStream_t stream);
// p[i] = |a[i]|^2 and its adjoint ga[i] = 2 gp[i] a[i], over n values
int launch_abs2(int64_t n, const float2* a, float* p, hipStream_t stream);
int launch_abs2_backward(int64_t n, const float2* a, const float* gp, float2* ga, hipStream_t stream);
// z[0..n) = 0 by a fill kernel (capture-safe, unlike a memset node)
int launch_zero_c64(int64_t n, float2* z, hipStream_t stream);
int launch_sample(const slos_batch_s& Bt, const float* p, double* part, double* cdf, const float* u, int S,
                  int32_t* shots, hipStream_t stream);

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

// Wave-uniform read of read-only data (batch descriptors, layer records,
// offsets) through the constant address space: a scalar load, the value in
// scalar registers.
template <class T>
__device__ __forceinline__ T ldc(const T* p) {
    return *(__attribute__((address_space(4))) const T*)p;
}

// Load through a global-address-space view of p.
template <class T>
__device__ __forceinline__ T ldg(const T* p) {
    return *(__attribute__((address_space(1))) const T*)p;
}

// LDS accessed through byte addresses.  The fused kernels declare no static
// LDS, so their dynamic LDS starts at address 0 and a region's address is a
// plain integer (which folds into the instruction's offset field).
typedef __attribute__((address_space(3))) unsigned long long lds_u64;
__device__ __forceinline__ float2 lds_ld(uint32_t a) { return __builtin_bit_cast(float2, *(const lds_u64*)(size_t)a); }
__device__ __forceinline__ void lds_st(uint32_t a, float2 v) { *(lds_u64*)(size_t)a = __builtin_bit_cast(unsigned long long, v); }

// Raw buffer access: 32-bit per-lane byte offset plus a wave-uniform offset,
// no 64-bit address arithmetic.  Every offset used stays inside the buffer.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ uint4 buf_ld4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ uint32_t buf_ld1(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ float buf_ldf(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
// Streaming (non-temporal) access for data touched once per call (per-sample
// inputs and outputs), so that it does not push the transition tables out of
// the L2 cache.  Cache-policy bits: 2 = non-temporal.
constexpr int kCpolStream = 2;
__device__ __forceinline__ float buf_ldf_stream(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, 0, kCpolStream));
}

typedef __attribute__((address_space(3))) float lds_f32;
__device__ __forceinline__ float lds_ldf(uint32_t a) { return *(const lds_f32*)(size_t)a; }
__device__ __forceinline__ void lds_stf(uint32_t a, float v) { *(lds_f32*)(size_t)a = v; }
typedef __attribute__((address_space(3))) int lds_i32;
__device__ __forceinline__ int lds_ldi(uint32_t a) { return *(const lds_i32*)(size_t)a; }
__device__ __forceinline__ void lds_sti(uint32_t a, int v) { *(lds_i32*)(size_t)a = v; }


// Calls f(mode) once per photon of state t of photon layer L (k photons),
// or, with DISTINCT, once per occupied mode.  The state's predecessor
// entries list its sorted modes, one slot per photon; an empty entry (mode
// field 32) repeats the previous slot's mode, and slots past k are padding.
// 64-bit indexing: any layer size.
template <bool DISTINCT = false, class F>
__device__ __forceinline__ void for_each_photon(const slos::LayerDev& L, int k, int64_t t, F&& f) {
    int cur = 0;
    for (int g = 0; g < L.ngrp; ++g) {
        typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
        const u32x4 e = *(__attribute__((address_space(1))) const u32x4*)(L.predv + (int64_t)g * L.N + t);
        const uint32_t ev[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (4 * g + q >= k) break;
            const int md = (int)(ev[q] >> L.pred_shift);
            if (md != 32) cur = md;
            if (!DISTINCT || md != 32) f(cur);
        }
    }
}
