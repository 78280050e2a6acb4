/*
 * slos.h -- C ABI of the MI355X (gfx950) strong-simulation library.
 *
 * The library computes, for n photons in m modes of a linear-optical
 * interferometer with unitary U, every output Fock amplitude
 *
 *     a_t = Perm(U[R(t), C(s)]) / sqrt(prod_i s_i! prod_j t_j!)
 *
 * (arXiv 2602.11092, Sec. II-A-1: output probabilities are permanents of
 * sub-matrices of U up to normalisation; the Fock space has C(m+n-1, n)
 * states), by the photon-by-photon recursion of Sec. II-A-2/II-A-3: starting
 * from one photon, the k-photon state is built from the (k-1)-photon state
 * through a transition graph that depends only on (m, k), while only the
 * coefficients taken from U change between calls.  The graph is built once
 * per plan (Sec. II-A-3, "prebuilding the sparse transition graph once").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Complex numbers are interleaved float pairs (re, im), i.e. the memory
 *   layout of complex64 / float2.  Pointers typed `float*` that hold complex
 *   data say so in their comment.
 * - U is row-major [B][m][m] with U[b][j][i] = amplitude for a photon entering
 *   mode i to leave in mode j (a single photon in mode i gives p_j = |U[j][i]|^2).
 * - Fock basis order: lexicographic order of the sorted list of occupied
 *   modes; |n,0,...,0> has rank 0, |0,...,0,n> rank C(m+n-1,n)-1.
 *   slos_fock_unrank / slos_fock_rank are the reference for this order.
 * - Batches may mix photon numbers.  Sample b's outputs occupy
 *   out[off_b .. off_b + C(m+n_b-1, n_b)) with off_b the exclusive prefix sum
 *   of the per-sample Fock dimensions (slos_batch_out_offsets).
 * - Gradients follow the convention G = dL/dRe + i dL/dIm of a real loss L
 *   (the one PyTorch uses).  Backward calls OVERWRITE their gradient outputs.
 * - Ownership: the caller allocates every device buffer passed to a compute
 *   call (inputs, outputs, workspace).  The library allocates device memory
 *   only in slos_plan_create and slos_batch_create, and frees it in the
 *   matching destroy call.
 * - Compute calls are asynchronous and ordered on `stream` (a hipStream_t
 *   passed as void*; NULL = the default stream).  They neither synchronise
 *   nor allocate, so they may be captured into a HIP graph.  The caller keeps
 *   inputs alive and does not read outputs until the stream has reached them.
 * - Errors: every call returns SLOS_OK (0) or a negative status.  Argument
 *   errors are detected on the host before anything is enqueued, so a failed
 *   call leaves all buffers untouched.  slos_last_error() gives a message for
 *   the calling thread's most recent failure.
 * - Thread safety: plans and batches are read-only after creation and may be
 *   used from several host threads and streams at once, provided each
 *   concurrent call has its own workspace.
 */
#ifndef SLOS_H
#define SLOS_H

#include <stddef.h>
#include <stdint.h>

#ifndef SLOS_API
#define SLOS_API __attribute__((visibility("default")))
#endif

#ifdef __cplusplus
extern "C" {
#endif

#define SLOS_OK 0
#define SLOS_EINVAL (-1)        /* bad argument (null pointer, bad size, bad occupation) */
#define SLOS_ENOMEM (-2)        /* device or host allocation failed (create calls only) */
#define SLOS_EHIP (-3)          /* a HIP runtime call or kernel launch failed */
#define SLOS_EWORKSPACE (-4)    /* workspace pointer null or smaller than required */
#define SLOS_EUNSUPPORTED (-5)  /* valid request outside what this plan/build supports */

/* Library limits. */
#define SLOS_MAX_MODES 32
#define SLOS_MAX_PHOTONS 16

/* Operation codes for slos_workspace_bytes / slos_batch_set_config.  The
 * measurement ops (4, 6, 8) configure the forward pass behind their entry
 * point (fock_mode_expectations, fock_threshold_probs, fock_sample), and
 * their backward ops (5, 7) the probability adjoint behind theirs. */
#define SLOS_OP_AMPLITUDES 0
#define SLOS_OP_PROBS 1
#define SLOS_OP_AMPLITUDES_BACKWARD 2
#define SLOS_OP_PROBS_BACKWARD 3
#define SLOS_OP_MODE_EXPECTATIONS 4
#define SLOS_OP_MODE_EXPECTATIONS_BACKWARD 5
#define SLOS_OP_THRESHOLD_PROBS 6
#define SLOS_OP_THRESHOLD_PROBS_BACKWARD 7
#define SLOS_OP_SAMPLE 8

/* Plan flags. */
#define SLOS_PLAN_DEFAULT 0
#define SLOS_PLAN_FORWARD_ONLY 1  /* skip the successor tables; backward calls return SLOS_EUNSUPPORTED */
/* Restricted computation space (Sec. II-B: computation spaces; the
 * QuantumBridge example of Sec. II-D uses it): only unbunched outputs,
 * t_j <= 1, C(m, n) of them, in the basis order above restricted to them.
 * The recursion stays exact (removing a photon keeps a state unbunched).
 * Input states may be bunched.  In the adjoint, successors outside the
 * space contribute nothing; the fused adjoint serves these plans with
 * workgroups of 256 or 512 threads and at most 24 modes (other sizes report
 * SLOS_EUNSUPPORTED for the fused variant and run layered by default).
 * Requires n_max <= m. */
#define SLOS_PLAN_UNBUNCHED 2
/* Dual-rail computation space (Sec. II-B: computation spaces; Sec. II-D:
 * the qubit-photon bridge): qubit g is the mode pair (2g, 2g+1) and every
 * state holds at most one photon per pair, C(m/2, n) 2^n states.  With
 * n = m/2 photons these are the 2^n logical states |q_0 ... q_{n-1}> (the
 * photon of qubit g in mode 2g + q_g), in big-endian binary order.  The
 * recursion stays exact (removing a photon keeps the constraint).  Inputs
 * may be any Fock state.  Adjoint as for SLOS_PLAN_UNBUNCHED; requires an
 * even m and n_max <= m/2; excludes SLOS_PLAN_UNBUNCHED. */
#define SLOS_PLAN_DUAL_RAIL 4
/* Also build the threshold-detector tables (Sec. II-B: detector models)
 * used by fock_threshold_probs: per photon layer, the states of each click
 * pattern (about 4 bytes per state), runs of whole patterns of at most 16384
 * states, and the predecessor rows and norms in pattern order
 * (16 ceil(k/4) + 4 bytes per state), which the fused forward reads when it
 * sums the patterns itself. */
#define SLOS_PLAN_THRESHOLD 8

/* Kernel variants for slos_batch_set_config. */
#define SLOS_VARIANT_AUTO 0    /* library heuristic (or the last value set) */
#define SLOS_VARIANT_FUSED 1   /* one persistent launch; each workgroup keeps a sample's photon layers in LDS */
#define SLOS_VARIANT_LAYERED 2 /* one launch per photon layer; layers kept in the workspace (any size) */
/* Two samples with equal photon numbers per workgroup, their layers
 * interleaved in LDS so that one 128-bit read serves both: the forward of
 * the amplitude and probability ops (also behind fock_threshold_probs and
 * fock_sample); workgroup size 512 or 1024 (default 1024). */
#define SLOS_VARIANT_FUSED_PAIRS 3

typedef struct slos_plan_s* slos_plan_t;
typedef struct slos_batch_s* slos_batch_t;

/* ---- Fock-space combinatorics (host only, no device work) ---------------- */

/* C(m+n-1, n), the dimension of the n-photon Fock space over m modes
 * (Sec. II-A-1).  Returns -1 if m < 1, n < 0 or the value overflows int64. */
SLOS_API int64_t slos_fock_dim(int m, int n);

/* C(m, n), the number of unbunched n-photon states (t_j <= 1) over m modes;
 * -1 if m < 1 or n < 0. */
SLOS_API int64_t slos_unbunched_dim(int m, int n);

/* Number of n-photon states of the space a plan with these flags uses:
 * slos_fock_dim, slos_unbunched_dim or C(m/2, n) 2^n for dual-rail.  -1 for
 * bad flags, m or n (dual-rail with an odd m included); 0 when no state fits. */
SLOS_API int64_t slos_space_dim(int m, int n, int flags);

/* Occupation vector (occ[0..m-1], host) of the state of the given rank in
 * the space of plans with these flags (the basis order restricted to the
 * space).  SLOS_EINVAL for bad flags, m, n, rank or NULL. */
SLOS_API int slos_space_unrank(int m, int n, int flags, int64_t rank, int32_t* occ);

/* Rank of occ (host, m entries summing to n) in that space; -1 if invalid
 * or outside the space. */
SLOS_API int64_t slos_space_rank(int m, int n, int flags, const int32_t* occ);

/* clicks[0..m-1] (host) <- 1 for the modes of click pattern q of n photons
 * (the order of slos_threshold_dim), else 0.  SLOS_EINVAL for a bad q. */
SLOS_API int slos_threshold_pattern(int m, int n, int64_t q, int32_t* clicks);

/* Occupation vector (occ[0..m-1], host) of the state of the given rank in
 * the basis order above.  Returns SLOS_EINVAL for a bad m, n, rank or NULL. */
SLOS_API int slos_fock_unrank(int m, int n, int64_t rank, int32_t* occ);

/* Rank of an occupation vector (host, m entries summing to n); -1 if invalid. */
SLOS_API int64_t slos_fock_rank(int m, int n, const int32_t* occ);

/* Host copy of the transition graph of photon layer k (1 <= k <= 16) over m
 * modes, the tables a plan uploads (host only, no device work; for
 * inspection and tests).  Each output may be NULL.  Sizes, N_k = C(m+k-1,k):
 *   pred   [k][N_k]      (rank of t - e_j in layer k-1) << 5 | j for the p-th
 *                        entry of t's sorted mode list; -1 where that entry
 *                        repeats the previous one;
 *   succ   [m][N_{k-1}]  rank in layer k of t' + e_j;
 *   nrm    [N_k]         sqrt(prod_j t_j!);
 *   minoff [m+1]         first rank of layer k whose smallest occupied mode is >= c.
 * Returns SLOS_EINVAL for bad m or k, SLOS_EUNSUPPORTED if N_k >= 2^26. */
SLOS_API int slos_transition_tables(int m, int k, int32_t* pred, int32_t* succ, float* nrm, int32_t* minoff);

/* The same with plan flags: SLOS_PLAN_UNBUNCHED or SLOS_PLAN_DUAL_RAIL give
 * the tables of that space (N_k = slos_space_dim(m, k, flags); succ is -1
 * where t' + e_j leaves the space).  SLOS_EINVAL for unknown or conflicting
 * flags, or k beyond what the space holds. */
SLOS_API int slos_transition_tables_ex(int m, int k, int flags, int32_t* pred, int32_t* succ, float* nrm,
                                       int32_t* minoff);

/* Message for the calling thread's most recent failed call ("" if none). */
SLOS_API const char* slos_last_error(void);

/* ---- Plans: transition graph for (m, n <= n_max) ------------------------- */

/* Builds, once, the transition graph of Sec. II-A-3 for every photon layer
 * k = 1..n_max over m modes and uploads it to the current HIP device:
 * predecessor lists (which (k-1)-photon states feed each k-photon state, and
 * through which output mode), successor tables (the reverse map, for the
 * backward pass), and sqrt(prod_j t_j!) per state.  Synchronous; allocates.
 * m in [1, SLOS_MAX_MODES], n_max in [1, SLOS_MAX_PHOTONS].
 * Returns SLOS_EINVAL, SLOS_ENOMEM, SLOS_EHIP or SLOS_OK (*out set). */
SLOS_API int slos_plan_create(int m, int n_max, int flags, slos_plan_t* out);
SLOS_API int slos_plan_destroy(slos_plan_t plan);  /* NULL is accepted; waits for the device */

/* ---- Batches: the input states of one call's samples --------------------- */

/* Describes B samples with input occupation vectors occ_host[b*m .. b*m+m-1]
 * (host memory, each entry >= 0, sum n_b in [0, n_max]).  Validates them,
 * derives per-sample photon lists, normalisation 1/sqrt(prod s!), output
 * offsets and a longest-first work order, and uploads them (synchronous,
 * allocates).  The batch keeps a reference to `plan`; destroy the batch first. */
SLOS_API int slos_batch_create(slos_plan_t plan, int B, const int32_t* occ_host, slos_batch_t* out);
SLOS_API int slos_batch_destroy(slos_batch_t batch);

/* Total number of outputs (sum of the per-sample Fock dimensions), or -1. */
SLOS_API int64_t slos_batch_out_len(slos_batch_t batch);

/* Writes the B+1 output offsets into off_host (host memory). */
SLOS_API int slos_batch_out_offsets(slos_batch_t batch, int64_t* off_host);

/* Device workspace needed by `op` on this batch with its current
 * configuration (0 is possible).  *bytes receives the size. */
SLOS_API int slos_workspace_bytes(slos_batch_t batch, int op, size_t* bytes);

/* Chooses the kernel variant and workgroup size used for `op` on this batch
 * (the autotuner's hook).  block = 0 keeps the library's choice; otherwise
 * one of 64, 128, 256, 512, 1024 (layered; fused forward: 256, 512, 1024) or
 * 256, 512, 768, 1024 (fused adjoint).  Returns SLOS_EINVAL for other sizes and
 * SLOS_EUNSUPPORTED if the variant cannot run this batch at that size (the
 * fused variant needs a sample's photon layers to fit in LDS and, in the
 * adjoint, layer n-1 to fit the per-thread registers). */
SLOS_API int slos_batch_set_config(slos_batch_t batch, int op, int variant, int block);

/* Reads back the configuration in use for `op` (variant, block). */
SLOS_API int slos_batch_get_config(slos_batch_t batch, int op, int* variant, int* block);

/* slos_batch_set_config with a tile size: the last-layer states each thread
 * takes per iteration in the two-sample forward (2, 4 or 8; 0 = default 4).
 * Other variants take tile = 0 only (SLOS_EINVAL otherwise). */
SLOS_API int slos_batch_set_config_ex(slos_batch_t batch, int op, int variant, int block, int tile);
/* Reads back (variant, block, tile); tile is 0 for variants without one. */
SLOS_API int slos_batch_get_config_ex(slos_batch_t batch, int op, int* variant, int* block, int* tile);

/* ---- Forward: amplitudes and probabilities (Sec. II-A-1/2/3, Sec. II-B) --- */

/* amps (device, complex, [out_len]) <- a_t for every sample and output state.
 * U (device, complex, [B][m][m]).  ws: device workspace of at least
 * slos_workspace_bytes(batch, SLOS_OP_AMPLITUDES) bytes (may be NULL if 0). */
SLOS_API int fock_amplitudes(slos_batch_t batch, const float* U, float* amps,
                    void* ws, size_t ws_bytes, void* stream);

/* probs (device, float, [out_len]) <- |a_t|^2 (no renormalisation). */
SLOS_API int fock_probs(slos_batch_t batch, const float* U, float* probs,
               void* ws, size_t ws_bytes, void* stream);

/* ---- Backward (Sec. II-A-3: the trainable phases of U are optimised by
 *      gradient descent through the simulation, so the recursion needs an
 *      adjoint).  With G = dL/dRe + i dL/dIm and the layers d_k of the
 *      recursion, g_n = c G_a (amplitudes) or 2 (dL/dp) c^2 d_n
 *      (probabilities), g_{k-1}[t'] = sum_j conj(U[j][i_k]) g_k[t' + e_j] and
 *      G_U[j][i_k] += sum_t' conj(d_{k-1}[t']) g_k[t' + e_j].  Intermediate
 *      photon layers are recomputed, not stored, so calls are stateless. -- */

/* grad_U (device, complex, [B][m][m]) <- dL/dU given grad_amps = dL/da
 * (device, complex, [out_len]).  Columns of U that carry no input photon get
 * zero gradient. */
SLOS_API int fock_amplitudes_backward(slos_batch_t batch, const float* U, const float* grad_amps,
                             float* grad_U, void* ws, size_t ws_bytes, void* stream);

/* grad_U (device, complex, [B][m][m]) <- dL/dU given grad_probs = dL/dp
 * (device, float, [out_len]). */
SLOS_API int fock_probs_backward(slos_batch_t batch, const float* U, const float* grad_probs,
                        float* grad_U, void* ws, size_t ws_bytes, void* stream);

/* ---- Measurement: per-mode photon-number expectations (Sec. II-B) ------- */

/* out (device, float, [B][m], sample order) <- <n_j> = sum_t t_j p_t over the
 * plan's output states (no renormalisation; for the full Fock space this
 * equals sum_i s_i |U[j][i]|^2).  The fused variant accumulates inside the
 * last photon layer and never writes p; the layered one writes p into the
 * workspace first.  ws: slos_workspace_bytes(batch, SLOS_OP_MODE_EXPECTATIONS)
 * bytes (the layered variant needs out_len * 4 bytes more than fock_probs).
 * Works on restricted plans (SLOS_PLAN_UNBUNCHED, SLOS_PLAN_DUAL_RAIL). */
SLOS_API int fock_mode_expectations(slos_batch_t batch, const float* U, float* out,
                                    void* ws, size_t ws_bytes, void* stream);

/* grad_U (device, complex, [B][m][m]) <- dL/dU given grad_out = dL/d<n_j>
 * (device, float, [B][m]).  Forms dL/dp_t = sum_j t_j grad_out[b][j] in the
 * workspace (out_len floats) and runs the probability adjoint with the
 * configuration set for SLOS_OP_MODE_EXPECTATIONS_BACKWARD.  Plans with
 * successor tables only (SLOS_EUNSUPPORTED otherwise). */
SLOS_API int fock_mode_expectations_backward(slos_batch_t batch, const float* U, const float* grad_out,
                                             float* grad_U, void* ws, size_t ws_bytes, void* stream);

/* Detector models for the per-mode expectations (Sec. II-B; Fig. 3). */
#define SLOS_DETECTOR_PNR 0        /* photon-number resolving: <n_j> = sum_t t_j p_t */
#define SLOS_DETECTOR_THRESHOLD 1  /* click or no click: P(t_j > 0) = sum_t [t_j > 0] p_t */

/* fock_mode_expectations / fock_mode_expectations_backward with a detector
 * model (the plain calls are SLOS_DETECTOR_PNR); same buffers, workspace
 * and configuration.  SLOS_EINVAL for an unknown model. */
SLOS_API int fock_mode_expectations_ex(slos_batch_t batch, const float* U, float* out, int detector,
                                       void* ws, size_t ws_bytes, void* stream);
SLOS_API int fock_mode_expectations_backward_ex(slos_batch_t batch, const float* U, const float* grad_out,
                                                float* grad_U, int detector, void* ws, size_t ws_bytes,
                                                void* stream);

/* ---- Amplitude-encoded inputs (Sec. II-C-2) -------------------------------- */
/*
 * An amplitude-encoded input is a superposition sum_c x_c |s_c> of Fock
 * states of one photon number; U maps it to sum_c x_c U|s_c> (linearity).
 * The batch's samples are the components s_c; a superposition groups them:
 * input g holds components [group_off[g], group_off[g+1]) (all with one
 * photon number n_g) and owns the output block [out_off[g], out_off[g+1])
 * of length C(m+n_g-1, n_g), basis order.  The components' amplitudes use
 * the batch's configuration for SLOS_OP_AMPLITUDES (forward) and
 * SLOS_OP_AMPLITUDES_BACKWARD (adjoint).  Cost: one SLOS per component.
 */
typedef struct slos_superposition_s* slos_superposition_t;

/* group_off: host, G+1 non-decreasing offsets from 0 to the batch size.
 * SLOS_EINVAL if a group mixes photon numbers or the offsets are bad.  The
 * batch must outlive the superposition. */
SLOS_API int slos_superposition_create(slos_batch_t components, int G, const int64_t* group_off,
                                       slos_superposition_t* out);
SLOS_API int slos_superposition_destroy(slos_superposition_t sup);
SLOS_API int64_t slos_superposition_out_len(slos_superposition_t sup);
SLOS_API int slos_superposition_out_offsets(slos_superposition_t sup, int64_t* off_host);
/* Device workspace of the forward (backward = 0) or the adjoint (1). */
SLOS_API int slos_superposition_workspace_bytes(slos_superposition_t sup, int backward, size_t* bytes);

/* out (device, complex, [out_len]) <- sum_c x_c a(U_g, s_c) for every group g.
 * U: device, complex, [G][m][m] (one interferometer per group); x: device,
 * complex, [C] weights.  Sums run over components in order (deterministic). */
SLOS_API int fock_superposition_amplitudes(slos_superposition_t sup, const float* U, const float* x, float* out,
                                           void* ws, size_t ws_bytes, void* stream);

/* Given grad_out = dL/dout (device, complex, [out_len]):
 * grad_U (device, complex, [G][m][m]) <- dL/dU_g = sum over g's components of
 * the amplitude adjoint at dL/da_c = conj(x_c) grad_out_g;
 * grad_x (device, complex, [C], may be NULL) <- dL/dx_c = sum_t conj(a_c[t]) grad_out_g[t].
 * Gradients use the dL/dRe + i dL/dIm convention. */
SLOS_API int fock_superposition_amplitudes_backward(slos_superposition_t sup, const float* U, const float* x,
                                                    const float* grad_out, float* grad_U, float* grad_x,
                                                    void* ws, size_t ws_bytes, void* stream);

/* Inputs that all go through one interferometer, each a dense vector over
 * the n-photon basis (basis order): Uhat, U's n-photon representation, is
 * built once per call (one SLOS per basis state, A[c][t] = a_t(U, basis_c))
 * and the G inputs go through a complex GEMM, out = X A (rocBLAS cgemm on
 * the caller's stream).  The object owns its buffers (about 2 N^2 complex
 * plus the basis batch); calls that share it on one device race.  At most
 * 16384 basis states (SLOS_EUNSUPPORTED beyond). */
typedef struct slos_shared_superposition_s* slos_shared_superposition_t;
SLOS_API int slos_shared_superposition_create(slos_plan_t plan, int n, slos_shared_superposition_t* out);
SLOS_API int slos_shared_superposition_destroy(slos_shared_superposition_t s);
SLOS_API int64_t slos_shared_superposition_dim(slos_shared_superposition_t s);
/* out, X: device, complex, [G][N] row-major; U: device, complex, [m][m]. */
SLOS_API int fock_shared_superposition_amplitudes(slos_shared_superposition_t s, const float* U, const float* X,
                                                  int G, float* out, void* stream);
/* grad_U [m][m] <- dL/dU; grad_X [G][N] (may be NULL) <- dL/dX, from
 * grad_out = dL/dout [G][N] (dL/dRe + i dL/dIm convention). */
SLOS_API int fock_shared_superposition_amplitudes_backward(slos_shared_superposition_t s, const float* U,
                                                           const float* X, int G, const float* grad_out,
                                                           float* grad_U, float* grad_X, void* stream);

/* Probabilities of amplitudes formed by another call (Sec. II-A-1: an output
 * probability is the squared modulus of its amplitude), e.g. the outputs of
 * fock_shared_superposition_amplitudes: probs[i] (device, float) <- |amps[i]|^2
 * for i < n, amps device complex.  Asynchronous; n = 0 does nothing;
 * SLOS_EINVAL for n < 0 or a NULL pointer when n > 0. */
SLOS_API int fock_probs_from_amplitudes(const float* amps, int64_t n, float* probs, void* stream);
/* Its adjoint: grad_amps[i] (device, complex) <- 2 grad_probs[i] amps[i], the
 * gradient dL/dRe + i dL/dIm of a real loss through p = |a|^2. */
SLOS_API int fock_probs_from_amplitudes_backward(const float* amps, const float* grad_probs, int64_t n,
                                                 float* grad_amps, void* stream);

/* ---- Measurement: threshold detectors (Sec. II-B: detector models) ------- */

/* Number of click patterns of n photons over m modes: the non-empty sets of
 * at most n modes, sum_{k=1}^{min(n,m)} C(m, k); 1 (the empty pattern) for
 * n = 0; -1 for a bad m or n.  Patterns are ordered by click count, then by
 * the lexicographic order of the clicked modes. */
SLOS_API int64_t slos_threshold_dim(int m, int n);

/* Total length of the batch's click-pattern outputs, and their B+1 offsets
 * (host memory): sample b owns [off[b], off[b+1]). */
SLOS_API int64_t slos_batch_threshold_len(slos_batch_t batch);
SLOS_API int slos_batch_threshold_offsets(slos_batch_t batch, int64_t* off_host);

/* out (device, float, [threshold_len]) <- P(c) = sum of p_t over the states
 * t whose occupied modes are exactly c (threshold detectors register
 * presence, not number).  Needs a plan created with SLOS_PLAN_THRESHOLD
 * (else SLOS_EUNSUPPORTED).  Each pattern's states are summed in ascending
 * order (deterministic): with the fused variant inside the forward, in runs
 * of whole patterns held in LDS (p is never written), where they fit; else p
 * is formed in the workspace with the configuration set for
 * SLOS_OP_THRESHOLD_PROBS and a second kernel sums it.  ws:
 * slos_workspace_bytes(batch, SLOS_OP_THRESHOLD_PROBS) bytes either way. */
SLOS_API int fock_threshold_probs(slos_batch_t batch, const float* U, float* out,
                                  void* ws, size_t ws_bytes, void* stream);

/* grad_U <- dL/dU given grad_out = dL/dP (device, float, [threshold_len]):
 * dL/dp_t = dL/dP(pattern of t) in the workspace, then the probability
 * adjoint.  Plans with successor tables only. */
SLOS_API int fock_threshold_probs_backward(slos_batch_t batch, const float* U, const float* grad_out,
                                           float* grad_U, void* ws, size_t ws_bytes, void* stream);

/* ---- Measurement: shot sampling (Sec. II-D: hardware returns shot-based samples) */

/* shots (device, int32, [B][S]) <- output-state indices (within each
 * sample's output block, basis order) drawn from p / sum(p) by inverse
 * transform of the caller's uniforms u (device, float, [B][S], in [0, 1)):
 * the first state whose cumulative probability exceeds u * sum(p), the last
 * state if none does.  p comes from the configuration set for
 * SLOS_OP_SAMPLE; its cumulative sums are formed in FP64 in the workspace
 * (slos_workspace_bytes(batch, SLOS_OP_SAMPLE) bytes) in a fixed order, so
 * equal uniforms give equal shots.  S >= 0. */
SLOS_API int fock_sample(slos_batch_t batch, const float* U, const float* u, int S, int32_t* shots,
                         void* ws, size_t ws_bytes, void* stream);

/* ---- Fidelity kernel (Sec. III-A: kernel methods) ------------------------ */

/* K (device, float, [B1][B2], row-major) <- |<phi(U1_a)|phi(U2_b)>|^2 with
 * |phi(U)> = U|s>, s = occ (host, m non-negative ints, n = sum <= 16):
 * |Perm(U1_a[:, C]^H U2_b[:, C])|^2 / (prod s!)^2, C the input modes with
 * multiplicity (one n x n permanent per pair instead of two Fock vectors).
 * U1 (device, complex, [B1][m][m]) and U2 ([B2][m][m]) may be the same
 * buffer (a Gram matrix).  FP64 arithmetic on the complex64 inputs; the
 * vacuum (n = 0) gives 1.  Asynchronous on `stream`; no plan needed.
 * SLOS_EINVAL for bad sizes or NULL pointers, SLOS_EUNSUPPORTED for n > 16. */
SLOS_API int fock_fidelity_kernel(int m, const int32_t* occ, const float* U1, int B1, const float* U2, int B2,
                                  float* K, void* stream);

/* ---- Interferometer mesh U(x, theta) (Sec. II-A-3, Sec. II-C-1) ---------- */
/*
 * Rectangular mesh of m(m-1)/2 Mach-Zehnder interferometers.  Column
 * c = 0..m-1 holds MZIs on mode pairs (k, k+1), k = c mod 2, c mod 2 + 2, ...,
 * k <= m-2.  MZI(theta, phi) = BS . PS(theta) . BS . PS(phi) with
 * BS = (1/sqrt2)[[1, i], [i, 1]] and PS(a) = diag(exp(i a), 1) on the upper
 * mode.  theta (device, float, [m(m-1)]) holds (theta_q, phi_q) per MZI,
 * MZIs ordered column-major, top-down.  The mesh is split after column
 * m/2 - 1 into W1 (columns < m/2) and W2, and the angle-encoding layer sits
 * between them (Sec. II-C-1, U(x, theta) = W2 S(x) W1):
 *
 *     U_b = W2 diag(exp(i * enc_scale * x[b][:])) W1,
 *
 * or U = W2 W1 (B must be 1) when x is NULL.
 */

/* Workspace for the mesh calls (both directions). */
SLOS_API int mesh_workspace_bytes(int m, int B, size_t* bytes);

/* U (device, complex, [B][m][m]) <- U(x_b, theta).  x: device [B][m] or NULL.
 * ws: at least mesh_workspace_bytes(m, B) bytes (checked).  Batches of up to
 * two samples per compute unit form the mesh factors on chip and leave the
 * workspace untouched; larger ones form them once into the workspace. */
SLOS_API int mesh_to_unitary(int m, int B, const float* theta, const float* x, float enc_scale,
                    float* U, void* ws, size_t ws_bytes, void* stream);

/* grad_theta (device, float, [m(m-1)]) and grad_x (device, float, [B][m],
 * may be NULL; must be NULL when x is NULL) <- gradients of a real loss given
 * grad_U (device, complex, [B][m][m]).  The reduction over the batch is done
 * in a fixed order (bitwise reproducible). */
SLOS_API int mesh_to_unitary_backward(int m, int B, const float* theta, const float* x, float enc_scale,
                             const float* grad_U, float* grad_theta, float* grad_x,
                             void* ws, size_t ws_bytes, void* stream);

/* mesh_to_unitary_backward for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same computation and results, with no workspace argument.  Its scratch is a
 * static device array of SLOS_MESH_NOALLOC_SCRATCH_BYTES (16 MiB) per device,
 * held until the process ends; the call allocates nothing and issues no
 * memset.  Sizes with mesh_workspace_bytes(m, B) above that are rejected
 * with SLOS_EUNSUPPORTED before anything is enqueued (B up to 2618 at
 * m = 20, 1020 at m = 32).  The first call on a device looks up the array's
 * address (hipGetSymbolAddress with that device current); make it outside a
 * graph capture.  Every call on a device shares that device's array, so calls
 * that overlap on one device (other streams, other threads) race; calls
 * ordered on one stream do not. */
#define SLOS_MESH_NOALLOC_SCRATCH_BYTES (16u << 20)
SLOS_API int mesh_to_unitary_backward_noalloc(int m, int B, const float* theta, const float* x, float enc_scale,
                                              const float* grad_U, float* grad_theta, float* grad_x, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SLOS_H */
