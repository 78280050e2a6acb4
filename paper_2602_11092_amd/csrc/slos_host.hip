// Host side of the strong-simulation library: Fock-basis combinatorics, the
// transition graph of every photon layer (built once per plan, Sec. II-A-3
// of arXiv 2602.11092), batch descriptors, and the C ABI entry points that
// validate arguments and dispatch to the fused or layered kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include <rocblas/rocblas.h>

#include "slos_internal.h"

namespace slos {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

namespace {

// C(a, b) in int64, -1 on overflow or invalid input.
int64_t binom(int64_t a, int64_t b) {
    if (b < 0 || a < 0 || b > a) return 0;
    if (b > a - b) b = a - b;
    __int128 r = 1;
    for (int64_t i = 1; i <= b; ++i) {
        r = r * (a - b + i) / i;
        if (r > (__int128)INT64_MAX) return -1;
    }
    return (int64_t)r;
}

// Counting helper for the basis order: sorted mode lists in lexicographic
// order.  group = 0: non-decreasing lists (every Fock state).  group = G >= 1:
// at most one photon in each block of G consecutive modes, so the list is
// strictly increasing in mode / G (G = 1: the unbunched states, t_j <= 1;
// G = 2: dual-rail, at most one photon per qubit's pair of modes).  The
// restricted orders are the full order restricted to those states.
// below[r][c] = number of lists of length r + 1 whose first entry is < c: the
// rank offset contributed by a position holding c when r more entries follow.
struct Counter {
    int m = 0;
    int K = 0;
    int group = 0;
    std::vector<std::vector<int64_t>> below;  // [r][c], r = 0..K, c = 0..m

    Counter(int m_, int K_, int group_ = 0)
        : m(m_), K(K_), group(group_), below(K_ + 1, std::vector<int64_t>(m_ + 1, 0)) {
        for (int r = 0; r <= K; ++r) {
            int64_t acc = 0;
            for (int c = 0; c <= m; ++c) {
                below[r][c] = acc;
                if (c < m) acc += count_after(c, r);
            }
        }
    }
    // number of lists of length r with entries in [c, m)
    int64_t count_from(int c, int r) const {
        if (r == 0) return 1;
        if (c >= m) return 0;
        if (group == 0) return binom((int64_t)(m - c) + r - 1, r);
        // the first entry either sits in c's own block (from c on) or in one
        // of the F whole blocks after it; each later entry picks a later block
        const int G = group, g0 = c / G, F = m / G - g0 - 1;
        const int64_t head = (int64_t)(g0 + 1) * G - c;
        auto pw = [&](int e) { int64_t v = 1; for (int i = 0; i < e; ++i) v *= G; return v; };
        return head * pw(r - 1) * binom(F, r - 1) + pw(r) * binom(F, r);
    }
    // smallest entry allowed after an entry c
    int next_lo(int c) const { return group == 0 ? c : (c / group + 1) * group; }
    // completions of length r after an entry c
    int64_t count_after(int c, int r) const { return count_from(next_lo(c), r); }
    // rank of sorted list L[0..len) skipping index `skip` (-1: none)
    int64_t rank(const int* L, int len, int skip = -1) const {
        const int K2 = (skip >= 0) ? len - 1 : len;
        int64_t r = 0;
        int lo = 0;
        int pos = 0;
        for (int q = 0; q < len; ++q) {
            if (q == skip) continue;
            const int rem = K2 - pos - 1;
            r += below[rem][L[q]] - below[rem][lo];
            lo = next_lo(L[q]);
            ++pos;
        }
        return r;
    }
    void unrank(int64_t r, int len, int* L) const {
        int lo = 0;
        for (int pos = 0; pos < len; ++pos) {
            const int rem = len - pos - 1;
            int j = lo;
            while (true) {
                const int64_t blk = count_after(j, rem);
                if (r < blk) break;
                r -= blk;
                ++j;
            }
            L[pos] = j;
            lo = next_lo(j);
        }
    }
    // next list in the order; false after the last one
    bool next(int* L, int len) const {
        for (int q = len - 1; q >= 0; --q) {
            const int v = L[q] + 1;
            if (v >= m) continue;
            if (group > 0 && m / group - v / group - 1 < len - q - 1) continue;  // no room for the rest
            L[q] = v;
            for (int r = q + 1; r < len; ++r) L[r] = next_lo(L[r - 1]);
            return true;
        }
        return false;
    }
    // whether inserting mode j into L keeps the list in the space
    bool admits(const int* L, int len, int j) const {
        if (group == 0) return true;
        for (int p = 0; p < len; ++p)
            if (L[p] / group == j / group) return false;
        return true;
    }
};

// Size of layer n of a space (group as in Counter); -1 if invalid.
int64_t space_dim(int m, int n, int group) {
    if (m < 1 || n < 0) return -1;
    if (group == 0) return binom((int64_t)m + n - 1, n);
    if (m % group) return -1;
    const int64_t c = binom((int64_t)(m / group), n);
    if (c <= 0) return c;
    __int128 v = c;
    for (int i = 0; i < n; ++i) v *= group;
    return v > (__int128)INT64_MAX ? -1 : (int64_t)v;
}

constexpr int kPlanFlags = SLOS_PLAN_FORWARD_ONLY | SLOS_PLAN_UNBUNCHED | SLOS_PLAN_DUAL_RAIL | SLOS_PLAN_THRESHOLD;

// group size of a plan's flags
int flags_group(int flags) {
    return (flags & SLOS_PLAN_DUAL_RAIL) ? 2 : (flags & SLOS_PLAN_UNBUNCHED) ? 1 : 0;
}

// flags known and consistent with m modes and n photons
bool space_flags_ok(int m, int n, int flags, std::string* why) {
    if (flags & ~kPlanFlags) return *why = "unknown flags", false;
    if ((flags & SLOS_PLAN_UNBUNCHED) && (flags & SLOS_PLAN_DUAL_RAIL))
        return *why = "SLOS_PLAN_UNBUNCHED and SLOS_PLAN_DUAL_RAIL exclude each other", false;
    const int G = flags_group(flags);
    if (G > 1 && m % G) return *why = "dual-rail needs an even number of modes", false;
    if (G > 0 && n > m / G)
        return *why = G == 1 ? "unbunched spaces need at most m photons" : "dual-rail needs at most m/2 photons", false;
    return true;
}

template <class F>
void parallel_ranges(int64_t total, F&& body) {
    unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (total < 20000) hw = 1;
    std::vector<std::thread> th;
    const int64_t step = (total + hw - 1) / hw;
    for (unsigned w = 0; w < hw; ++w) {
        const int64_t lo = (int64_t)w * step, hi = std::min(total, lo + step);
        if (lo >= hi) break;
        th.emplace_back([=, &body] { body(lo, hi); });
    }
    for (auto& t : th) t.join();
}

struct HostLayer {
    std::vector<int32_t> pred, succ, minoff;
    std::vector<float> nrm;
    std::vector<int32_t> thr_ptr, thr_idx;  // click-pattern tables (SLOS_PLAN_THRESHOLD)
    std::vector<int32_t> thr_chunk;         // runs of whole patterns of at most kThrChunkStates states
    std::vector<int32_t> thr_pred;          // packed pred rows in click-pattern order
    std::vector<float> thr_nrm;             // nrm in click-pattern order
};

// Transition graph of layer k (k >= 1): predecessor entries for every
// k-photon state, successor ranks for every (k-1)-photon state and output
// mode, sqrt(prod t!) and the smallest-mode block offsets.
void build_layer(int m, int k, const Counter& Ck, const Counter& Ckm1, int64_t Nk, int64_t Nkm1,
                 bool want_succ, HostLayer& H) {
    H.pred.assign((size_t)k * Nk, -1);
    H.nrm.assign(Nk, 1.f);
    parallel_ranges(Nk, [&](int64_t lo, int64_t hi) {
        int L[kMaxPhotons];
        Ck.unrank(lo, k, L);
        for (int64_t t = lo; t < hi; ++t) {
            double f = 1.0;
            int run = 1;
            for (int p = 0; p < k; ++p) {
                if (p > 0 && L[p] == L[p - 1]) {
                    ++run;
                    f *= run;
                } else {
                    run = 1;
                    const int64_t r = Ckm1.rank(L, k, p);
                    H.pred[(size_t)p * Nk + t] = (int32_t)((r << kModeBits) | L[p]);
                }
            }
            H.nrm[t] = (float)std::sqrt(f);
            Ck.next(L, k);
        }
    });
    if (want_succ) {
        H.succ.assign((size_t)m * Nkm1, 0);
        parallel_ranges(Nkm1, [&](int64_t lo, int64_t hi) {
            int L[kMaxPhotons + 1], T[kMaxPhotons + 1];
            if (k - 1 > 0) Ckm1.unrank(lo, k - 1, L);
            for (int64_t t = lo; t < hi; ++t) {
                for (int j = 0; j < m; ++j) {
                    // insert j into the sorted list (-1 when the result leaves a restricted space)
                    if (!Ck.admits(L, k - 1, j)) {
                        H.succ[(size_t)j * Nkm1 + t] = -1;
                        continue;
                    }
                    int o = 0;
                    bool done = false;
                    for (int p = 0; p < k - 1; ++p) {
                        if (!done && j < L[p]) { T[o++] = j; done = true; }
                        T[o++] = L[p];
                    }
                    if (!done) T[o++] = j;
                    H.succ[(size_t)j * Nkm1 + t] = (int32_t)Ck.rank(T, k);
                }
                if (k - 1 > 0) Ckm1.next(L, k - 1);
            }
        });
    }
    H.minoff.assign(m + 1, 0);
    for (int c = 0; c <= m; ++c) H.minoff[c] = (int32_t)Ck.below[k - 1][c];
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Click-pattern tables of layer k (Counter Ck of the plan's space): pattern
// q's states, ascending, in idx[ptr[q] .. ptr[q+1]).  Pattern index of a
// state: offset of its click count j plus the rank of its occupied modes
// among the j-sets (unbunched order).
void build_threshold(int m, int k, const Counter& Ck, int64_t Nk, std::vector<int32_t>& ptr,
                     std::vector<int32_t>& idx) {
    const int jmax = std::min(k, m);
    std::vector<int64_t> off(jmax + 2, 0);
    std::vector<Counter> sets;
    sets.reserve(jmax + 1);
    for (int j = 0; j <= jmax; ++j) sets.emplace_back(m, j, 1);
    for (int j = 1; j <= jmax; ++j) off[j + 1] = off[j] + binom(m, j);
    const int64_t Q = off[jmax + 1];
    std::vector<int32_t> pat(Nk);
    parallel_ranges(Nk, [&](int64_t lo, int64_t hi) {
        int L[kMaxPhotons], D[kMaxPhotons];
        Ck.unrank(lo, k, L);
        for (int64_t t = lo; t < hi; ++t) {
            int j = 0;
            for (int p = 0; p < k; ++p)
                if (p == 0 || L[p] != L[p - 1]) D[j++] = L[p];
            pat[t] = (int32_t)(off[j] + sets[j].rank(D, j));
            Ck.next(L, k);
        }
    });
    ptr.assign(Q + 1, 0);
    for (int64_t t = 0; t < Nk; ++t) ++ptr[pat[t] + 1];
    for (int64_t q = 0; q < Q; ++q) ptr[q + 1] += ptr[q];
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    idx.assign(Nk, 0);
    for (int64_t t = 0; t < Nk; ++t) idx[fill[pat[t]]++] = (int32_t)t;
}

}  // namespace

int64_t threshold_dim(int m, int n) {
    if (m < 1 || n < 0) return -1;
    if (n == 0) return 1;
    int64_t q = 0;
    for (int j = 1; j <= std::min(n, m); ++j) q += binom(m, j);
    return q;
}

}  // namespace slos

using namespace slos;

// ===================================================================== ABI

extern "C" const char* slos_last_error(void) { return g_last_error.c_str(); }

extern "C" int64_t slos_fock_dim(int m, int n) {
    if (m < 1 || n < 0) return -1;
    return binom((int64_t)m + n - 1, n);
}

extern "C" int slos_fock_unrank(int m, int n, int64_t rank, int32_t* occ) {
    if (!occ) return fail(SLOS_EINVAL, "slos_fock_unrank: occ is NULL");
    if (m < 1 || m > kMaxModes || n < 0 || n > 64) return fail(SLOS_EINVAL, "slos_fock_unrank: bad m or n");
    const int64_t N = slos_fock_dim(m, n);
    if (N < 0 || rank < 0 || rank >= N) return fail(SLOS_EINVAL, "slos_fock_unrank: rank out of range");
    Counter C(m, n);
    std::vector<int> L(n > 0 ? n : 1);
    C.unrank(rank, n, L.data());
    for (int j = 0; j < m; ++j) occ[j] = 0;
    for (int p = 0; p < n; ++p) occ[L[p]] += 1;
    return SLOS_OK;
}

extern "C" int64_t slos_fock_rank(int m, int n, const int32_t* occ) {
    if (!occ || m < 1 || m > kMaxModes || n < 0 || n > 64) return -1;
    std::vector<int> L;
    for (int j = 0; j < m; ++j) {
        if (occ[j] < 0) return -1;
        for (int q = 0; q < occ[j]; ++q) L.push_back(j);
    }
    if ((int)L.size() != n) return -1;
    Counter C(m, n);
    return C.rank(L.data(), n);
}

extern "C" int64_t slos_unbunched_dim(int m, int n) { return space_dim(m, n, 1); }

extern "C" int slos_space_unrank(int m, int n, int flags, int64_t rank, int32_t* occ) {
    if (!occ) return fail(SLOS_EINVAL, "slos_space_unrank: occ is NULL");
    if (m < 1 || m > kMaxModes || n < 0 || n > 64) return fail(SLOS_EINVAL, "slos_space_unrank: bad m or n");
    const int64_t N = slos_space_dim(m, n, flags);
    if (N < 0 || rank < 0 || rank >= N) return fail(SLOS_EINVAL, "slos_space_unrank: bad flags or rank out of range");
    Counter C(m, n, flags_group(flags));
    std::vector<int> L(n > 0 ? n : 1);
    C.unrank(rank, n, L.data());
    for (int j = 0; j < m; ++j) occ[j] = 0;
    for (int p = 0; p < n; ++p) occ[L[p]] += 1;
    return SLOS_OK;
}

extern "C" int64_t slos_space_rank(int m, int n, int flags, const int32_t* occ) {
    if (!occ || m < 1 || m > kMaxModes || n < 0 || n > 64 || slos_space_dim(m, n, flags) < 0) return -1;
    std::vector<int> L;
    for (int j = 0; j < m; ++j) {
        if (occ[j] < 0) return -1;
        for (int q = 0; q < occ[j]; ++q) L.push_back(j);
    }
    if ((int)L.size() != n) return -1;
    Counter C(m, n, flags_group(flags));
    for (int p = 0; p < n; ++p)  // the state must lie in the space
        if (p > 0 && L[p] < C.next_lo(L[p - 1])) return -1;
    return C.rank(L.data(), n);
}

extern "C" int slos_threshold_pattern(int m, int n, int64_t q, int32_t* clicks) {
    if (!clicks) return fail(SLOS_EINVAL, "slos_threshold_pattern: clicks is NULL");
    const int64_t Q = threshold_dim(m, n);
    if (m > kMaxModes || Q < 0 || q < 0 || q >= Q) return fail(SLOS_EINVAL, "slos_threshold_pattern: bad m, n or q");
    for (int j = 0; j < m; ++j) clicks[j] = 0;
    if (n == 0) return SLOS_OK;  // the empty pattern
    int k = 1;
    while (q >= binom(m, k)) q -= binom(m, k++);
    Counter C(m, k, 1);
    int L[kMaxModes];
    C.unrank(q, k, L);
    for (int p = 0; p < k; ++p) clicks[L[p]] = 1;
    return SLOS_OK;
}

extern "C" int64_t slos_space_dim(int m, int n, int flags) {
    if (flags & ~kPlanFlags || (flags & SLOS_PLAN_UNBUNCHED && flags & SLOS_PLAN_DUAL_RAIL)) return -1;
    return space_dim(m, n, flags_group(flags));
}

extern "C" int slos_transition_tables(int m, int k, int32_t* pred, int32_t* succ, float* nrm, int32_t* minoff) {
    return slos_transition_tables_ex(m, k, SLOS_PLAN_DEFAULT, pred, succ, nrm, minoff);
}

extern "C" int slos_transition_tables_ex(int m, int k, int flags, int32_t* pred, int32_t* succ, float* nrm,
                                         int32_t* minoff) {
    if (m < 1 || m > kMaxModes) return fail(SLOS_EINVAL, "slos_transition_tables: m must be in [1, 32]");
    if (k < 1 || k > kMaxPhotons) return fail(SLOS_EINVAL, "slos_transition_tables: k must be in [1, 16]");
    std::string why;
    if (!space_flags_ok(m, k, flags, &why)) return fail(SLOS_EINVAL, "slos_transition_tables: " + why);
    const int group = flags_group(flags);
    const int64_t Nk = space_dim(m, k, group);
    const int64_t Nkm1 = space_dim(m, k - 1, group);
    if (Nk < 0 || Nk >= ((int64_t)1 << (31 - kModeBits)))
        return fail(SLOS_EUNSUPPORTED, "slos_transition_tables: layer too large for 32-bit tables");
    Counter Ck(m, k, group), Ckm1(m, k - 1, group);
    HostLayer H;
    build_layer(m, k, Ck, Ckm1, Nk, Nkm1, succ != nullptr, H);
    if (pred) std::memcpy(pred, H.pred.data(), H.pred.size() * 4);
    if (succ) std::memcpy(succ, H.succ.data(), H.succ.size() * 4);
    if (nrm) std::memcpy(nrm, H.nrm.data(), H.nrm.size() * 4);
    if (minoff) std::memcpy(minoff, H.minoff.data(), H.minoff.size() * 4);
    return SLOS_OK;
}

extern "C" int slos_plan_create(int m, int n_max, int flags, slos_plan_t* out) {
    if (!out) return fail(SLOS_EINVAL, "slos_plan_create: out is NULL");
    *out = nullptr;
    if (m < 1 || m > kMaxModes) return fail(SLOS_EINVAL, "slos_plan_create: m must be in [1, 32]");
    if (n_max < 1 || n_max > kMaxPhotons) return fail(SLOS_EINVAL, "slos_plan_create: n_max must be in [1, 16]");
    std::string why;
    if (!space_flags_ok(m, n_max, flags, &why)) return fail(SLOS_EINVAL, "slos_plan_create: " + why);
    const int group = flags_group(flags);
    const int64_t Ntop = space_dim(m, n_max, group);
    // successor byte offsets (rank * 8) must fit 32 bits, predecessor ranks the wide entry
    if (Ntop < 0 || Ntop >= ((int64_t)1 << 29) || space_dim(m, n_max - 1, group) >= kPredWideStates)
        return fail(SLOS_EUNSUPPORTED, "slos_plan_create: Fock space too large for 32-bit tables");

    auto* P = new slos_plan_s();
    P->m = m;
    P->n_max = n_max;
    P->flags = flags;
    P->N.resize(n_max + 1);
    for (int k = 0; k <= n_max; ++k) P->N[k] = space_dim(m, k, group);

    if (hipGetDevice(&P->device) != hipSuccess) {
        delete P;
        return fail(SLOS_EHIP, "slos_plan_create: no HIP device");
    }
    int cu = 0, lds = 0;
    hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, P->device);
    hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device);
    P->num_cu = cu;
    P->max_lds = (size_t)lds;

    // successors that leave a restricted space are marked (-1 << 3) for the layered adjoint
    const bool want_succ = !(flags & SLOS_PLAN_FORWARD_ONLY);
    std::vector<HostLayer> H(n_max + 1);
    std::vector<int> shifts(n_max + 1, kPredShiftCompact);
    std::vector<Counter> C;
    C.reserve(n_max + 1);
    for (int k = 0; k <= n_max; ++k) C.emplace_back(m, k, group);
    for (int k = 1; k <= n_max; ++k) {
        build_layer(m, k, C[k], C[k - 1], P->N[k], P->N[k - 1], want_succ, H[k]);
        // device layout: groups of four predecessor entries per state, [group][state][4],
        // each (mode << shift) | (rank << 3), an empty one pred_empty(shift)
        const int ngrp = (k + 3) / 4;
        const int64_t Nk = P->N[k];
        const int shift = P->N[k - 1] <= kPredCompactStates ? kPredShiftCompact : kPredShiftWide;
        std::vector<int32_t> packed((size_t)ngrp * Nk * 4, (int32_t)pred_empty(shift));
        for (int p = 0; p < k; ++p)
            for (int64_t t = 0; t < Nk; ++t) {
                const int32_t e = H[k].pred[(size_t)p * Nk + t];
                if (e >= 0)
                    packed[((size_t)(p / 4) * Nk + t) * 4 + (p % 4)] =
                        (int32_t)(((uint32_t)(e & 31) << shift) | ((uint32_t)(e >> kModeBits) << 3));
            }
        H[k].pred.swap(packed);
        shifts[k] = shift;
        if (flags & SLOS_PLAN_THRESHOLD) {
            build_threshold(m, k, C[k], Nk, H[k].thr_ptr, H[k].thr_idx);
            // greedy runs of whole patterns (a pattern holds at most C(15, 7) states, fewer than a run)
            const int32_t Qk = (int32_t)H[k].thr_ptr.size() - 1;
            for (int32_t q0 = 0; q0 < Qk;) {
                H[k].thr_chunk.push_back(q0);
                int32_t q1 = q0 + 1;
                while (q1 < Qk && H[k].thr_ptr[q1 + 1] - H[k].thr_ptr[q0] <= kThrChunkStates) ++q1;
                q0 = q1;
            }
            H[k].thr_chunk.push_back(Qk);
            // the predecessor rows and norms in pattern order
            H[k].thr_pred.resize(H[k].pred.size());
            H[k].thr_nrm.resize((size_t)Nk);
            for (int64_t sp = 0; sp < Nk; ++sp) {
                const int64_t t = H[k].thr_idx[(size_t)sp];
                H[k].thr_nrm[(size_t)sp] = H[k].nrm[(size_t)t];
                for (int g = 0; g < ngrp; ++g)
                    for (int q = 0; q < 4; ++q)
                        H[k].thr_pred[((size_t)g * Nk + sp) * 4 + q] = H[k].pred[((size_t)g * Nk + t) * 4 + q];
            }
        }
        // device successors: groups of four modes, [j/4][t'][4], byte offsets rank * 8
        if (want_succ) {
            const int64_t Nkm1 = P->N[k - 1];
            const int sg = (m + 3) / 4;
            std::vector<int32_t> grouped((size_t)sg * Nkm1 * 4, 0);
            for (int j = 0; j < m; ++j)
                for (int64_t t = 0; t < Nkm1; ++t)
                    grouped[((size_t)(j / 4) * Nkm1 + t) * 4 + (j % 4)] =
                        (int32_t)((uint32_t)H[k].succ[(size_t)j * Nkm1 + t] << 3);
            H[k].succ.swap(grouped);
        }
    }

    // one device allocation for every table
    size_t total = align256(sizeof(LayerDev) * (n_max + 1));
    std::vector<size_t> o_pred(n_max + 1), o_succ(n_max + 1), o_nrm(n_max + 1), o_min(n_max + 1);
    std::vector<size_t> o_tp(n_max + 1), o_ti(n_max + 1), o_tc(n_max + 1), o_tpr(n_max + 1), o_tnr(n_max + 1);
    for (int k = 1; k <= n_max; ++k) {
        o_pred[k] = total; total += align256(H[k].pred.size() * 4);
        o_succ[k] = total; total += align256(H[k].succ.size() * 4);
        o_nrm[k] = total;  total += align256(H[k].nrm.size() * 4);
        o_min[k] = total;  total += align256(H[k].minoff.size() * 4);
        o_tp[k] = total;   total += align256(H[k].thr_ptr.size() * 4);
        o_ti[k] = total;   total += align256(H[k].thr_idx.size() * 4);
        o_tc[k] = total;   total += align256(H[k].thr_chunk.size() * 4);
        o_tpr[k] = total;  total += align256(H[k].thr_pred.size() * 4);
        o_tnr[k] = total;  total += align256(H[k].thr_nrm.size() * 4);
    }
    if (hipMalloc(&P->dmem, total) != hipSuccess) {
        delete P;
        return fail(SLOS_ENOMEM, "slos_plan_create: hipMalloc of the transition tables failed");
    }
    char* base = (char*)P->dmem;
    P->layers.assign(n_max + 1, LayerDev{});
    P->layers[0].N = 1;
    P->layers[0].cum = 0;
    hipError_t e = hipSuccess;
    for (int k = 1; k <= n_max && e == hipSuccess; ++k) {
        LayerDev& L = P->layers[k];
        L.N = P->N[k];
        L.cum = P->layers[k - 1].cum + P->N[k - 1];
        L.predv = (const uint4*)(base + o_pred[k]);
        L.ngrp = (k + 3) / 4;
        L.pred_shift = shifts[k];
        L.succ = want_succ ? (const uint32_t*)(base + o_succ[k]) : nullptr;
        L.nrm = (const float*)(base + o_nrm[k]);
        L.minoff = (const int32_t*)(base + o_min[k]);
        const bool thr = !H[k].thr_ptr.empty();
        L.thr_ptr = thr ? (const int32_t*)(base + o_tp[k]) : nullptr;
        L.thr_idx = thr ? (const int32_t*)(base + o_ti[k]) : nullptr;
        L.Q = thr ? (int64_t)H[k].thr_ptr.size() - 1 : 0;
        L.thr_chunk = thr ? (const int32_t*)(base + o_tc[k]) : nullptr;
        L.thr_nchunk = thr ? (int32_t)H[k].thr_chunk.size() - 1 : 0;
        L.thr_predv = thr ? (const uint4*)(base + o_tpr[k]) : nullptr;
        L.thr_nrm = thr ? (const float*)(base + o_tnr[k]) : nullptr;
        e = hipMemcpy(base + o_pred[k], H[k].pred.data(), H[k].pred.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess && thr)
            e = hipMemcpy(base + o_tp[k], H[k].thr_ptr.data(), H[k].thr_ptr.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess && thr)
            e = hipMemcpy(base + o_ti[k], H[k].thr_idx.data(), H[k].thr_idx.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess && thr)
            e = hipMemcpy(base + o_tc[k], H[k].thr_chunk.data(), H[k].thr_chunk.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess && thr)
            e = hipMemcpy(base + o_tpr[k], H[k].thr_pred.data(), H[k].thr_pred.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess && thr)
            e = hipMemcpy(base + o_tnr[k], H[k].thr_nrm.data(), H[k].thr_nrm.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess && want_succ)
            e = hipMemcpy(base + o_succ[k], H[k].succ.data(), H[k].succ.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(base + o_nrm[k], H[k].nrm.data(), H[k].nrm.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(base + o_min[k], H[k].minoff.data(), H[k].minoff.size() * 4, hipMemcpyHostToDevice);
    }
    P->d_layers = (LayerDev*)base;
    if (e == hipSuccess)
        e = hipMemcpy(P->d_layers, P->layers.data(), sizeof(LayerDev) * (n_max + 1), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(P->dmem);
        delete P;
        return fail(SLOS_EHIP, std::string("slos_plan_create: upload failed: ") + hipGetErrorString(e));
    }
    *out = P;
    return SLOS_OK;
}

extern "C" int slos_plan_destroy(slos_plan_t plan) {
    if (!plan) return SLOS_OK;
    hipDeviceSynchronize();
    if (plan->dmem) hipFree(plan->dmem);
    delete plan;
    return SLOS_OK;
}

extern "C" int slos_batch_create(slos_plan_t plan, int B, const int32_t* occ_host, slos_batch_t* out) {
    if (!out) return fail(SLOS_EINVAL, "slos_batch_create: out is NULL");
    *out = nullptr;
    if (!plan) return fail(SLOS_EINVAL, "slos_batch_create: plan is NULL");
    if (B < 0) return fail(SLOS_EINVAL, "slos_batch_create: B < 0");
    if (B > 0 && !occ_host) return fail(SLOS_EINVAL, "slos_batch_create: occ_host is NULL");
    const int m = plan->m;
    auto* Bt = new slos_batch_s();
    Bt->plan = plan;
    Bt->B = B;
    Bt->n_host.resize(B);
    Bt->off_host.assign(B + 1, 0);
    Bt->thr_off_host.assign(B + 1, 0);
    std::vector<int32_t> modes((size_t)std::max(B, 1) * kMaxPhotons, 0);
    std::vector<float> innorm(std::max(B, 1), 1.f);
    for (int b = 0; b < B; ++b) {
        int n = 0;
        double f = 1.0;
        for (int i = 0; i < m; ++i) {
            const int32_t s = occ_host[(size_t)b * m + i];
            if (s < 0) { delete Bt; return fail(SLOS_EINVAL, "slos_batch_create: negative occupation"); }
            if (n + s > plan->n_max) {
                delete Bt;
                return fail(SLOS_EUNSUPPORTED, "slos_batch_create: a sample has more photons than the plan's n_max");
            }
            for (int q = 0; q < s; ++q) {
                modes[(size_t)b * kMaxPhotons + n + q] = i;
                f *= (q + 1);
            }
            n += s;
        }
        Bt->n_host[b] = n;
        innorm[b] = (float)(1.0 / std::sqrt(f));
        Bt->off_host[b + 1] = Bt->off_host[b] + plan->N[n];
        Bt->thr_off_host[b + 1] = Bt->thr_off_host[b] + threshold_dim(m, n);
        Bt->n_max = std::max(Bt->n_max, n);
    }
    std::vector<int32_t> order(B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return Bt->n_host[a] > Bt->n_host[b]; });
    // two-sample work items: consecutive samples of the work order with equal photon numbers
    std::vector<int2> pairs;
    pairs.reserve((B + 1) / 2);
    for (int i = 0; i < B;) {
        if (i + 1 < B && Bt->n_host[order[i]] == Bt->n_host[order[i + 1]]) {
            pairs.push_back(make_int2(order[i], order[i + 1]));
            i += 2;
        } else {
            pairs.push_back(make_int2(order[i], -1));
            i += 1;
        }
    }
    Bt->npairs = (int)pairs.size();

    const size_t Bs = std::max(B, 1);
    size_t o_n = 0, o_modes = align256(Bs * 4), o_off = o_modes + align256(Bs * kMaxPhotons * 4);
    size_t o_in = o_off + align256((Bs + 1) * 8), o_ord = o_in + align256(Bs * 4);
    size_t o_thr = o_ord + align256(Bs * 4);
    size_t o_pair = o_thr + align256((Bs + 1) * 8);
    size_t total = o_pair + align256(Bs * sizeof(int2));
    if (hipMalloc(&Bt->dmem, total) != hipSuccess) {
        delete Bt;
        return fail(SLOS_ENOMEM, "slos_batch_create: hipMalloc failed");
    }
    char* base = (char*)Bt->dmem;
    hipError_t e = hipSuccess;
    if (B > 0) {
        e = hipMemcpy(base + o_n, Bt->n_host.data(), B * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(base + o_modes, modes.data(), (size_t)B * kMaxPhotons * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(base + o_in, innorm.data(), B * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(base + o_ord, order.data(), B * 4, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemcpy(base + o_off, Bt->off_host.data(), (B + 1) * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + o_thr, Bt->thr_off_host.data(), (B + 1) * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess && !pairs.empty())
        e = hipMemcpy(base + o_pair, pairs.data(), pairs.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(Bt->dmem);
        delete Bt;
        return fail(SLOS_EHIP, "slos_batch_create: upload failed");
    }
    Bt->dev.B = B;
    Bt->dev.n_max = Bt->n_max;
    Bt->dev.n = (const int32_t*)(base + o_n);
    Bt->dev.modes = (const int32_t*)(base + o_modes);
    Bt->dev.off = (const int64_t*)(base + o_off);
    Bt->dev.innorm = (const float*)(base + o_in);
    Bt->dev.order = (const int32_t*)(base + o_ord);
    Bt->dev.thr_off = (const int64_t*)(base + o_thr);
    Bt->dev.pairs = (const int2*)(base + o_pair);
    Bt->dev.npairs = Bt->npairs;
    *out = Bt;
    return SLOS_OK;
}

extern "C" int slos_batch_destroy(slos_batch_t batch) {
    if (!batch) return SLOS_OK;
    hipDeviceSynchronize();
    if (batch->dmem) hipFree(batch->dmem);
    delete batch;
    return SLOS_OK;
}

extern "C" int64_t slos_batch_out_len(slos_batch_t batch) {
    if (!batch) return -1;
    return batch->off_host[batch->B];
}

extern "C" int slos_batch_out_offsets(slos_batch_t batch, int64_t* off_host) {
    if (!batch || !off_host) return fail(SLOS_EINVAL, "slos_batch_out_offsets: NULL argument");
    std::memcpy(off_host, batch->off_host.data(), (batch->B + 1) * sizeof(int64_t));
    return SLOS_OK;
}

namespace {

bool op_valid(int op) { return op >= SLOS_OP_AMPLITUDES && op <= SLOS_OP_SAMPLE; }
bool op_backward(int op) {
    return op == SLOS_OP_AMPLITUDES_BACKWARD || op == SLOS_OP_PROBS_BACKWARD ||
           op == SLOS_OP_MODE_EXPECTATIONS_BACKWARD || op == SLOS_OP_THRESHOLD_PROBS_BACKWARD;
}
bool op_threshold(int op) { return op == SLOS_OP_THRESHOLD_PROBS || op == SLOS_OP_THRESHOLD_PROBS_BACKWARD; }
bool op_expect(int op) { return op == SLOS_OP_MODE_EXPECTATIONS || op == SLOS_OP_MODE_EXPECTATIONS_BACKWARD; }
// ops whose forward forms amplitudes or probabilities (the two-sample kernel's outputs)
bool op_pairs_ok(int op) {
    return op == SLOS_OP_AMPLITUDES || op == SLOS_OP_PROBS || op == SLOS_OP_THRESHOLD_PROBS || op == SLOS_OP_SAMPLE;
}
bool variant_fused(int v) { return v == SLOS_VARIANT_FUSED || v == SLOS_VARIANT_FUSED_PAIRS; }

// the expectation ops keep dL/dp or p (out_len floats) at the start of their workspace
size_t expect_head_bytes(const slos_batch_s& Bt) { return align256((size_t)Bt.off_host[Bt.B] * sizeof(float)); }
// sampling keeps p, the FP64 cumulative sums and the chunk totals
size_t sample_head_bytes(const slos_batch_s& Bt) {
    return expect_head_bytes(Bt) + align256((size_t)Bt.off_host[Bt.B] * sizeof(double)) +
           align256((size_t)Bt.B * mode_expect_chunks(Bt) * sizeof(double));
}

// Default fused block size of an op: the expectation epilogue's [m][block]
// accumulators share LDS with the photon layers, so it steps down to the
// largest size that fits.
int fused_block_for(const slos_batch_s& Bt, int op) {
    const bool bwd = op_backward(op);
    int blk = fused_default_block(*Bt.plan, Bt.n_max, bwd);
    if (op == SLOS_OP_MODE_EXPECTATIONS)
        while (blk > 256 && !fused_fwd_supported(*Bt.plan, Bt.n_max, blk, nullptr, true)) blk /= 2;
    return blk;
}

// Resolves AUTO and the default block size for one op.
int resolve(const slos_batch_s& Bt, int op, int* variant, int* block) {
    const slos_plan_s& P = *Bt.plan;
    const bool bwd = op_backward(op);
    Config c = Bt.cfg[op];
    int v = c.variant;
    if (v == SLOS_VARIANT_AUTO) {
        const int blk = fused_block_for(Bt, op);
        const bool ok = bwd ? fused_bwd_supported(P, Bt.n_max, blk, nullptr)
                            : fused_fwd_supported(P, Bt.n_max, blk, nullptr, op_expect(op));
        v = ok ? SLOS_VARIANT_FUSED : SLOS_VARIANT_LAYERED;
    }
    int blk = c.block;
    if (blk == 0)
        blk = (v == SLOS_VARIANT_FUSED_PAIRS) ? 1024
              : (v == SLOS_VARIANT_FUSED)     ? fused_block_for(Bt, op)
                                              : layered_default_block(Bt);
    *variant = v;
    *block = blk;
    return SLOS_OK;
}

}  // namespace

extern "C" int slos_workspace_bytes(slos_batch_t batch, int op, size_t* bytes) {
    if (!batch || !bytes) return fail(SLOS_EINVAL, "slos_workspace_bytes: NULL argument");
    if (!op_valid(op)) return fail(SLOS_EINVAL, "slos_workspace_bytes: bad op");
    int v, blk;
    resolve(*batch, op, &v, &blk);
    *bytes = variant_fused(v) ? 0 : layered_ws_bytes(*batch, op_backward(op));
    // the expectation forward keeps p and partial sums in the workspace only
    // when layered; the backward always keeps dL/dp
    if (op == SLOS_OP_MODE_EXPECTATIONS_BACKWARD) *bytes += expect_head_bytes(*batch);
    if (op == SLOS_OP_MODE_EXPECTATIONS && v != SLOS_VARIANT_FUSED)
        *bytes += expect_head_bytes(*batch) + align256(mode_expect_part_bytes(*batch));
    // the threshold ops keep p or dL/dp in the workspace
    if (op_threshold(op)) *bytes += expect_head_bytes(*batch);
    if (op == SLOS_OP_SAMPLE) *bytes += sample_head_bytes(*batch);
    return SLOS_OK;
}

extern "C" int slos_batch_set_config(slos_batch_t batch, int op, int variant, int block) {
    return slos_batch_set_config_ex(batch, op, variant, block, 0);
}

extern "C" int slos_batch_set_config_ex(slos_batch_t batch, int op, int variant, int block, int tile) {
    if (!batch) return fail(SLOS_EINVAL, "slos_batch_set_config: batch is NULL");
    if (!op_valid(op)) return fail(SLOS_EINVAL, "slos_batch_set_config: bad op");
    if (variant < SLOS_VARIANT_AUTO || variant > SLOS_VARIANT_FUSED_PAIRS)
        return fail(SLOS_EINVAL, "slos_batch_set_config: bad variant");
    if (block != 0 && block != 64 && block != 128 && block != 256 && block != 512 && block != 768 && block != 1024)
        return fail(SLOS_EINVAL, "slos_batch_set_config: block must be 0, 64, 128, 256, 512, 768 or 1024");
    const bool bwd = op_backward(op);
    if (block == 768 && variant != SLOS_VARIANT_FUSED)
        return fail(SLOS_EUNSUPPORTED, "slos_batch_set_config: 768 is a fused-adjoint workgroup size only");
    if (variant == SLOS_VARIANT_FUSED_PAIRS) {
        if (!op_pairs_ok(op))
            return fail(SLOS_EUNSUPPORTED, "slos_batch_set_config: the two-sample variant serves the amplitude and "
                                           "probability forwards only");
        std::string why;
        if (!fused_pairs_supported(*batch->plan, batch->n_max, block ? block : 1024, &why))
            return fail(SLOS_EUNSUPPORTED, "slos_batch_set_config: two-sample variant unavailable: " + why);
    }
    if (variant == SLOS_VARIANT_FUSED) {
        std::string why;
        const int blk = block ? block : fused_block_for(*batch, op);
        const bool ok = bwd ? fused_bwd_supported(*batch->plan, batch->n_max, blk, &why)
                            : fused_fwd_supported(*batch->plan, batch->n_max, blk, &why, op_expect(op));
        if (!ok) return fail(SLOS_EUNSUPPORTED, "slos_batch_set_config: fused variant unavailable: " + why);
    }
    if (tile != 0 && !(variant == SLOS_VARIANT_FUSED_PAIRS && (tile == 2 || tile == 4 || tile == 8)))
        return fail(SLOS_EINVAL, "slos_batch_set_config_ex: tile must be 0, or 2, 4 or 8 with the two-sample variant");
    batch->cfg[op].variant = variant;
    batch->cfg[op].block = block;
    batch->cfg[op].tile = tile;
    return SLOS_OK;
}

extern "C" int slos_batch_get_config(slos_batch_t batch, int op, int* variant, int* block) {
    if (!batch || !variant || !block) return fail(SLOS_EINVAL, "slos_batch_get_config: NULL argument");
    if (!op_valid(op)) return fail(SLOS_EINVAL, "slos_batch_get_config: bad op");
    return resolve(*batch, op, variant, block);
}

extern "C" int slos_batch_get_config_ex(slos_batch_t batch, int op, int* variant, int* block, int* tile) {
    if (!tile) return fail(SLOS_EINVAL, "slos_batch_get_config_ex: NULL argument");
    const int rc = slos_batch_get_config(batch, op, variant, block);
    if (rc != SLOS_OK) return rc;
    *tile = batch->cfg[op].tile != 0 ? batch->cfg[op].tile : (*variant == SLOS_VARIANT_FUSED_PAIRS ? 4 : 0);
    return SLOS_OK;
}

namespace {

// Per-mode expectations and their adjoint: the fused forward accumulates in
// its last-layer epilogue; the layered forward writes p into the workspace
// and reduces it; the adjoint expands dL/d<n_j> into dL/dp in the workspace
// and runs the probability adjoint on it.
int run_expect(const slos_batch_s& Bt, int op, int v, int blk, const float* U, const void* gin, void* out,
               void* ws, size_t ws_bytes, hipStream_t s, const std::string& nm, bool clicks) {
    const bool bwd = op == SLOS_OP_MODE_EXPECTATIONS_BACKWARD;
    const bool fused = v == SLOS_VARIANT_FUSED;
    if (!bwd && fused) return launch_fused_fwd(Bt, blk, (const float2*)U, out, clicks ? 3 : 2, s);
    // workspace: [p or dL/dp][partial sums (forward)][layered workspace]
    const size_t head = expect_head_bytes(Bt);
    const size_t parts = bwd ? 0 : align256(mode_expect_part_bytes(Bt));
    const size_t need = head + parts + (fused ? 0 : layered_ws_bytes(Bt, bwd));
    if (!ws || ws_bytes < need)
        return fail(SLOS_EWORKSPACE, nm + ": workspace missing or too small (need " + std::to_string(need) + " bytes)");
    float* pv = (float*)ws;
    void* rest = (char*)ws + head + parts;
    int rc;
    if (!bwd) {
        rc = launch_layered_fwd(Bt, blk, (const float2*)U, pv, true, rest, s);
        if (rc == SLOS_OK) rc = launch_mode_expect(Bt, pv, (float*)((char*)ws + head), (float*)out, clicks, s);
        return rc;
    }
    rc = launch_expand_mode_weights(Bt, (const float*)gin, pv, clicks, s);
    if (rc != SLOS_OK) return rc;
    return fused ? launch_fused_bwd(Bt, blk, (const float2*)U, pv, true, (float2*)out, s)
                 : launch_layered_bwd(Bt, blk, (const float2*)U, pv, true, (float2*)out, rest, s);
}

// Threshold-detector click probabilities and their adjoint: p (or dL/dp)
// lives at the start of the workspace; the forward gathers each pattern's
// states (inside the fused forward where its LDS holds a run of patterns),
// the adjoint scatters dL/dP back onto them.
int run_threshold(const slos_batch_s& Bt, int op, int v, int blk, const float* U, const void* gin, void* out,
                  void* ws, size_t ws_bytes, hipStream_t s, const std::string& nm) {
    if (!(Bt.plan->flags & SLOS_PLAN_THRESHOLD))
        return fail(SLOS_EUNSUPPORTED, nm + ": plan was created without SLOS_PLAN_THRESHOLD");
    const bool bwd = op == SLOS_OP_THRESHOLD_PROBS_BACKWARD;
    const bool fused = variant_fused(v);
    const size_t head = expect_head_bytes(Bt);
    const size_t need = head + (fused ? 0 : layered_ws_bytes(Bt, bwd));
    if (!ws || ws_bytes < need)
        return fail(SLOS_EWORKSPACE, nm + ": workspace missing or too small (need " + std::to_string(need) + " bytes)");
    float* pv = (float*)ws;
    void* rest = (char*)ws + head;
    int rc;
    if (!bwd) {
        // the fused variant sums the patterns inside the forward (p never leaves LDS)
        if (v == SLOS_VARIANT_FUSED && fused_threshold_supported(*Bt.plan, Bt.n_max, blk))
            return launch_fused_fwd(Bt, blk, (const float2*)U, out, 4, s);
        rc = v == SLOS_VARIANT_FUSED_PAIRS ? launch_fused_pairs_fwd(Bt, blk, Bt.cfg[op].tile, (const float2*)U, pv, true, s)
             : fused                        ? launch_fused_fwd(Bt, blk, (const float2*)U, pv, 1, s)
                                            : launch_layered_fwd(Bt, blk, (const float2*)U, pv, true, rest, s);
        if (rc == SLOS_OK) rc = launch_threshold_gather(Bt, pv, (float*)out, s);
        return rc;
    }
    rc = launch_threshold_scatter(Bt, (const float*)gin, pv, s);
    if (rc != SLOS_OK) return rc;
    return fused ? launch_fused_bwd(Bt, blk, (const float2*)U, pv, true, (float2*)out, s)
                 : launch_layered_bwd(Bt, blk, (const float2*)U, pv, true, (float2*)out, rest, s);
}

int run(slos_batch_t batch, int op, const float* U, const void* gin, void* out, void* ws, size_t ws_bytes,
        void* stream, int detector = SLOS_DETECTOR_PNR) {
    static const char* names[8] = {"fock_amplitudes", "fock_probs", "fock_amplitudes_backward",
                                   "fock_probs_backward", "fock_mode_expectations",
                                   "fock_mode_expectations_backward", "fock_threshold_probs",
                                   "fock_threshold_probs_backward"};
    const std::string nm = names[op];
    if (!batch) return fail(SLOS_EINVAL, nm + ": batch is NULL");
    if (batch->B == 0) return SLOS_OK;
    if (!U) return fail(SLOS_EINVAL, nm + ": U is NULL");
    if (!out) return fail(SLOS_EINVAL, nm + ": output pointer is NULL");
    const bool bwd = op_backward(op);
    if (bwd && !gin) return fail(SLOS_EINVAL, nm + ": gradient input is NULL");
    if (bwd && (batch->plan->flags & SLOS_PLAN_FORWARD_ONLY))
        return fail(SLOS_EUNSUPPORTED, nm + ": plan was created forward-only");
    int v, blk;
    resolve(*batch, op, &v, &blk);
    const bool probs = (op == SLOS_OP_PROBS || op == SLOS_OP_PROBS_BACKWARD);
    hipStream_t s = (hipStream_t)stream;
    if (op_expect(op))
        return run_expect(*batch, op, v, blk, U, gin, out, ws, ws_bytes, s, nm, detector == SLOS_DETECTOR_THRESHOLD);
    if (op_threshold(op)) return run_threshold(*batch, op, v, blk, U, gin, out, ws, ws_bytes, s, nm);
    int rc;
    if (v == SLOS_VARIANT_FUSED_PAIRS && !bwd) {
        rc = launch_fused_pairs_fwd(*batch, blk, batch->cfg[op].tile, (const float2*)U, out, probs, s);
    } else if (v == SLOS_VARIANT_FUSED) {
        rc = bwd ? launch_fused_bwd(*batch, blk, (const float2*)U, gin, probs, (float2*)out, s)
                 : launch_fused_fwd(*batch, blk, (const float2*)U, out, probs ? 1 : 0, s);
    } else {
        const size_t need = layered_ws_bytes(*batch, bwd);
        if (need > 0 && (!ws || ws_bytes < need))
            return fail(SLOS_EWORKSPACE, nm + ": workspace missing or too small (need " + std::to_string(need) +
                                             " bytes)");
        rc = bwd ? launch_layered_bwd(*batch, blk, (const float2*)U, gin, probs, (float2*)out, ws, s)
                 : launch_layered_fwd(*batch, blk, (const float2*)U, out, probs, ws, s);
    }
    return rc;
}

}  // namespace

extern "C" int fock_amplitudes(slos_batch_t batch, const float* U, float* amps, void* ws, size_t ws_bytes,
                               void* stream) {
    return run(batch, SLOS_OP_AMPLITUDES, U, nullptr, amps, ws, ws_bytes, stream);
}

extern "C" int fock_probs(slos_batch_t batch, const float* U, float* probs, void* ws, size_t ws_bytes,
                          void* stream) {
    return run(batch, SLOS_OP_PROBS, U, nullptr, probs, ws, ws_bytes, stream);
}

extern "C" int fock_amplitudes_backward(slos_batch_t batch, const float* U, const float* grad_amps,
                                        float* grad_U, void* ws, size_t ws_bytes, void* stream) {
    return run(batch, SLOS_OP_AMPLITUDES_BACKWARD, U, grad_amps, grad_U, ws, ws_bytes, stream);
}

extern "C" int fock_probs_backward(slos_batch_t batch, const float* U, const float* grad_probs, float* grad_U,
                                   void* ws, size_t ws_bytes, void* stream) {
    return run(batch, SLOS_OP_PROBS_BACKWARD, U, grad_probs, grad_U, ws, ws_bytes, stream);
}

// ------------------------------------------------------------ superpositions

struct slos_superposition_s {
    slos_batch_s* batch = nullptr;
    std::vector<int64_t> goff, ooff;
    void* dmem = nullptr;
    SupDev dev;
};

namespace {

size_t sup_ws_parts(const slos_superposition_s& S, bool bwd, size_t* uc, size_t* a, size_t* ga, size_t* guc,
                    size_t* amp) {
    const slos_batch_s& Bt = *S.batch;
    const size_t mm = (size_t)Bt.plan->m * Bt.plan->m;
    *uc = align256((size_t)Bt.B * mm * 8);
    *a = align256((size_t)Bt.off_host[Bt.B] * 8);
    *ga = bwd ? *a : 0;
    *guc = bwd ? *uc : 0;
    size_t w = 0;
    slos_workspace_bytes(S.batch, SLOS_OP_AMPLITUDES, &w);
    *amp = w;
    if (bwd) {
        slos_workspace_bytes(S.batch, SLOS_OP_AMPLITUDES_BACKWARD, &w);
        *amp = std::max(*amp, w);
    }
    return *uc + *a + *ga + *guc + align256(*amp);
}

}  // namespace

extern "C" int slos_superposition_create(slos_batch_t components, int G, const int64_t* group_off,
                                         slos_superposition_t* out) {
    if (!out) return fail(SLOS_EINVAL, "slos_superposition_create: out is NULL");
    *out = nullptr;
    if (!components || !group_off || G < 0) return fail(SLOS_EINVAL, "slos_superposition_create: bad argument");
    const slos_batch_s& Bt = *components;
    if (group_off[0] != 0 || group_off[G] != Bt.B)
        return fail(SLOS_EINVAL, "slos_superposition_create: offsets must run from 0 to the batch size");
    for (int g = 0; g < G; ++g)  // every offset is checked before any is used
        if (group_off[g + 1] <= group_off[g] || group_off[g + 1] > Bt.B)
            return fail(SLOS_EINVAL, "slos_superposition_create: offsets must increase (one component or more per group)");
    auto* S = new slos_superposition_s();
    S->batch = components;
    S->goff.assign(group_off, group_off + G + 1);
    S->ooff.assign(G + 1, 0);
    std::vector<int32_t> group(std::max(Bt.B, 1), 0);
    int64_t maxN = 1;
    for (int g = 0; g < G; ++g) {
        const int64_t c0 = group_off[g], c1 = group_off[g + 1];
        if (c1 < c0 || c1 - c0 < 1) {
            delete S;
            return fail(SLOS_EINVAL, "slos_superposition_create: every group needs at least one component");
        }
        const int n = Bt.n_host[c0];
        for (int64_t c = c0; c < c1; ++c) {
            if (Bt.n_host[c] != n) {
                delete S;
                return fail(SLOS_EINVAL, "slos_superposition_create: a group mixes photon numbers");
            }
            group[c] = g;
        }
        const int64_t N = Bt.plan->N[n];
        S->ooff[g + 1] = S->ooff[g] + N;
        maxN = std::max(maxN, N);
    }
    // the combine and expand grids are (group or component) x (state chunk)
    const int64_t chunks = (maxN + kMeasureChunkStates - 1) / kMeasureChunkStates;
    if ((int64_t)std::max(G, Bt.B) * chunks >= ((int64_t)1 << 31)) {
        delete S;
        return fail(SLOS_EUNSUPPORTED, "slos_superposition_create: too many components for one launch");
    }
    const size_t o_grp = 0, o_goff = align256((size_t)std::max(Bt.B, 1) * 4), o_ooff = o_goff + align256((G + 1) * 8);
    const size_t total = o_ooff + align256((G + 1) * 8);
    if (hipMalloc(&S->dmem, total) != hipSuccess) {
        delete S;
        return fail(SLOS_ENOMEM, "slos_superposition_create: hipMalloc failed");
    }
    char* base = (char*)S->dmem;
    hipError_t e = hipMemcpy(base + o_grp, group.data(), group.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + o_goff, S->goff.data(), (G + 1) * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + o_ooff, S->ooff.data(), (G + 1) * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(S->dmem);
        delete S;
        return fail(SLOS_EHIP, "slos_superposition_create: upload failed");
    }
    S->dev.G = G;
    S->dev.group = (const int32_t*)(base + o_grp);
    S->dev.goff = (const int64_t*)(base + o_goff);
    S->dev.ooff = (const int64_t*)(base + o_ooff);
    S->dev.max_n_states = maxN;
    *out = S;
    return SLOS_OK;
}

extern "C" int slos_superposition_destroy(slos_superposition_t sup) {
    if (!sup) return SLOS_OK;
    hipDeviceSynchronize();
    if (sup->dmem) hipFree(sup->dmem);
    delete sup;
    return SLOS_OK;
}

extern "C" int64_t slos_superposition_out_len(slos_superposition_t sup) { return sup ? sup->ooff.back() : -1; }

extern "C" int slos_superposition_out_offsets(slos_superposition_t sup, int64_t* off_host) {
    if (!sup || !off_host) return fail(SLOS_EINVAL, "slos_superposition_out_offsets: NULL argument");
    std::memcpy(off_host, sup->ooff.data(), sup->ooff.size() * 8);
    return SLOS_OK;
}

extern "C" int slos_superposition_workspace_bytes(slos_superposition_t sup, int backward, size_t* bytes) {
    if (!sup || !bytes) return fail(SLOS_EINVAL, "slos_superposition_workspace_bytes: NULL argument");
    size_t uc, a, ga, guc, amp;
    *bytes = sup_ws_parts(*sup, backward != 0, &uc, &a, &ga, &guc, &amp);
    return SLOS_OK;
}

extern "C" int fock_superposition_amplitudes(slos_superposition_t sup, const float* U, const float* x, float* out,
                                             void* ws, size_t ws_bytes, void* stream) {
    const std::string nm = "fock_superposition_amplitudes";
    if (!sup) return fail(SLOS_EINVAL, nm + ": sup is NULL");
    if (sup->dev.G == 0) return SLOS_OK;
    if (!U || !x || !out) return fail(SLOS_EINVAL, nm + ": NULL device pointer");
    size_t uc, a, ga, guc, amp;
    const size_t need = sup_ws_parts(*sup, false, &uc, &a, &ga, &guc, &amp);
    if (!ws || ws_bytes < need)
        return fail(SLOS_EWORKSPACE, nm + ": workspace missing or too small (need " + std::to_string(need) + " bytes)");
    char* base = (char*)ws;
    float2* Uc = (float2*)base;
    float2* A = (float2*)(base + uc);
    void* rest = base + uc + a;
    hipStream_t s = (hipStream_t)stream;
    const slos_batch_s& Bt = *sup->batch;
    int rc = launch_superposition(kSupReplicateU, sup->dev, Bt, U, nullptr, nullptr, Uc, s);
    if (rc == SLOS_OK) rc = run(sup->batch, SLOS_OP_AMPLITUDES, (const float*)Uc, nullptr, A, rest, amp, stream);
    if (rc == SLOS_OK) rc = launch_superposition(kSupCombine, sup->dev, Bt, x, A, nullptr, out, s);
    return rc;
}

extern "C" int fock_superposition_amplitudes_backward(slos_superposition_t sup, const float* U, const float* x,
                                                      const float* grad_out, float* grad_U, float* grad_x, void* ws,
                                                      size_t ws_bytes, void* stream) {
    const std::string nm = "fock_superposition_amplitudes_backward";
    if (!sup) return fail(SLOS_EINVAL, nm + ": sup is NULL");
    if (sup->dev.G == 0) return SLOS_OK;
    if (!U || !x || !grad_out || !grad_U) return fail(SLOS_EINVAL, nm + ": NULL device pointer");
    size_t uc, a, ga, guc, amp;
    const size_t need = sup_ws_parts(*sup, true, &uc, &a, &ga, &guc, &amp);
    if (!ws || ws_bytes < need)
        return fail(SLOS_EWORKSPACE, nm + ": workspace missing or too small (need " + std::to_string(need) + " bytes)");
    char* base = (char*)ws;
    float2* Uc = (float2*)base;
    float2* A = (float2*)(base + uc);
    float2* gA = (float2*)(base + uc + a);
    float2* gUc = (float2*)(base + uc + a + ga);
    void* rest = base + uc + a + ga + guc;
    hipStream_t s = (hipStream_t)stream;
    const slos_batch_s& Bt = *sup->batch;
    int rc = launch_superposition(kSupReplicateU, sup->dev, Bt, U, nullptr, nullptr, Uc, s);
    if (rc == SLOS_OK && grad_x) {
        rc = run(sup->batch, SLOS_OP_AMPLITUDES, (const float*)Uc, nullptr, A, rest, amp, stream);
        if (rc == SLOS_OK) rc = launch_superposition(kSupGradX, sup->dev, Bt, A, grad_out, nullptr, grad_x, s);
    }
    if (rc == SLOS_OK) rc = launch_superposition(kSupExpand, sup->dev, Bt, x, grad_out, nullptr, gA, s);
    if (rc == SLOS_OK)
        rc = run(sup->batch, SLOS_OP_AMPLITUDES_BACKWARD, (const float*)Uc, gA, (float*)gUc, rest, amp, stream);
    if (rc == SLOS_OK) rc = launch_superposition(kSupGroupSum, sup->dev, Bt, gUc, nullptr, nullptr, grad_U, s);
    return rc;
}

// ------------------------------------------- superpositions through one U

// Every input is a dense vector over the n-photon basis and all inputs share
// one interferometer, so U's n-photon representation Uhat is built once per
// call (one SLOS per basis state: row c of A holds a(U, basis_c)) and the
// inputs go through one complex GEMM: out[g][t] = sum_c X[g][c] A[c][t].
struct slos_shared_superposition_s {
    slos_batch_t basis = nullptr;  // the N basis states of n photons, one per sample
    int N = 0;
    int m = 0;
    void* dmem = nullptr;
    float2 *Urep = nullptr, *A = nullptr, *gA = nullptr, *gUc = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    SupDev dev;  // one group holding every basis state
    rocblas_handle blas = nullptr;
};

extern "C" int slos_shared_superposition_create(slos_plan_t plan, int n, slos_shared_superposition_t* out) {
    if (!out) return fail(SLOS_EINVAL, "slos_shared_superposition_create: out is NULL");
    *out = nullptr;
    if (!plan || n < 0 || n > plan->n_max) return fail(SLOS_EINVAL, "slos_shared_superposition_create: bad plan or n");
    const int64_t N = plan->N[n];
    if (N > 16384) return fail(SLOS_EUNSUPPORTED, "slos_shared_superposition_create: more than 16384 basis states");
    const int m = plan->m;
    std::vector<int32_t> occ((size_t)N * m, 0);
    const int group = flags_group(plan->flags);
    Counter C(m, n, group);
    std::vector<int> L(std::max(n, 1));
    for (int64_t c = 0; c < N; ++c) {
        C.unrank(c, n, L.data());
        for (int p = 0; p < n; ++p) occ[(size_t)c * m + L[p]] += 1;
    }
    auto* S = new slos_shared_superposition_s();
    S->N = (int)N;
    S->m = m;
    int rc = slos_batch_create(plan, (int)N, occ.data(), &S->basis);
    if (rc != SLOS_OK) {
        delete S;
        return rc;
    }
    size_t wf = 0, wb = 0;
    slos_workspace_bytes(S->basis, SLOS_OP_AMPLITUDES, &wf);
    slos_workspace_bytes(S->basis, SLOS_OP_AMPLITUDES_BACKWARD, &wb);
    S->ws_bytes = std::max(wf, wb);
    const size_t mm = (size_t)m * m, NN = (size_t)N * N;
    const size_t o_u = 0, o_a = o_u + align256(N * mm * 8), o_ga = o_a + align256(NN * 8);
    const size_t o_guc = o_ga + align256(NN * 8), o_ws = o_guc + align256(N * mm * 8);
    const size_t o_grp = o_ws + align256(S->ws_bytes), o_goff = o_grp + align256(N * 4);
    const size_t total = o_goff + 256;
    if (hipMalloc(&S->dmem, total) != hipSuccess) {
        slos_batch_destroy(S->basis);
        delete S;
        return fail(SLOS_ENOMEM, "slos_shared_superposition_create: hipMalloc failed");
    }
    char* base = (char*)S->dmem;
    S->Urep = (float2*)(base + o_u);
    S->A = (float2*)(base + o_a);
    S->gA = (float2*)(base + o_ga);
    S->gUc = (float2*)(base + o_guc);
    S->ws = base + o_ws;
    std::vector<int32_t> zeros(N, 0);
    const int64_t goff[2] = {0, N};
    hipError_t e = hipMemcpy(base + o_grp, zeros.data(), N * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + o_goff, goff, sizeof(goff), hipMemcpyHostToDevice);
    if (e != hipSuccess || rocblas_create_handle(&S->blas) != rocblas_status_success) {
        hipFree(S->dmem);
        slos_batch_destroy(S->basis);
        delete S;
        return fail(SLOS_EHIP, "slos_shared_superposition_create: setup failed");
    }
    S->dev.G = 1;
    S->dev.group = (const int32_t*)(base + o_grp);
    S->dev.goff = (const int64_t*)(base + o_goff);
    S->dev.ooff = (const int64_t*)(base + o_goff);
    S->dev.max_n_states = N;
    *out = S;
    return SLOS_OK;
}

extern "C" int slos_shared_superposition_destroy(slos_shared_superposition_t s) {
    if (!s) return SLOS_OK;
    hipDeviceSynchronize();
    if (s->blas) rocblas_destroy_handle(s->blas);
    if (s->dmem) hipFree(s->dmem);
    slos_batch_destroy(s->basis);
    delete s;
    return SLOS_OK;
}

extern "C" int64_t slos_shared_superposition_dim(slos_shared_superposition_t s) { return s ? s->N : -1; }

namespace {

// Uhat's rows into s->A on `stream`
int shared_rows(slos_shared_superposition_s& S, const float* U, hipStream_t stream) {
    const slos_batch_s& Bt = *S.basis;
    int rc = launch_superposition(kSupReplicateU, S.dev, Bt, U, nullptr, nullptr, S.Urep, stream);
    if (rc == SLOS_OK) rc = run(S.basis, SLOS_OP_AMPLITUDES, (const float*)S.Urep, nullptr, S.A, S.ws, S.ws_bytes, stream);
    return rc;
}

// C (column-major, ldc) = op(A) op(B), complex FP32 on `stream`
int cgemm(rocblas_handle h, hipStream_t stream, rocblas_operation ta, rocblas_operation tb, int M, int Nc, int K,
          const float2* A, int lda, const float2* B, int ldb, float2* C, int ldc) {
    const rocblas_float_complex one(1.f, 0.f), zero(0.f, 0.f);
    if (rocblas_set_stream(h, stream) != rocblas_status_success) return fail(SLOS_EHIP, "rocblas_set_stream failed");
    const rocblas_status st = rocblas_cgemm(h, ta, tb, M, Nc, K, &one, (const rocblas_float_complex*)A, lda,
                                            (const rocblas_float_complex*)B, ldb, &zero, (rocblas_float_complex*)C, ldc);
    if (st != rocblas_status_success) return fail(SLOS_EHIP, "rocblas_cgemm failed (" + std::to_string((int)st) + ")");
    return SLOS_OK;
}

}  // namespace

extern "C" int fock_shared_superposition_amplitudes(slos_shared_superposition_t s, const float* U, const float* X,
                                                    int G, float* out, void* stream) {
    const std::string nm = "fock_shared_superposition_amplitudes";
    if (!s || G < 0) return fail(SLOS_EINVAL, nm + ": bad argument");
    if (G == 0) return SLOS_OK;
    if (!U || !X || !out) return fail(SLOS_EINVAL, nm + ": NULL device pointer");
    hipStream_t st = (hipStream_t)stream;
    int rc = shared_rows(*s, U, st);
    // out_cm (N x G) = A_cm (N x N) X_cm (N x G), A_cm = A's rows read column-major
    if (rc == SLOS_OK)
        rc = cgemm(s->blas, st, rocblas_operation_none, rocblas_operation_none, s->N, G, s->N, s->A, s->N,
                   (const float2*)X, s->N, (float2*)out, s->N);
    return rc;
}

extern "C" int fock_shared_superposition_amplitudes_backward(slos_shared_superposition_t s, const float* U,
                                                             const float* X, int G, const float* grad_out,
                                                             float* grad_U, float* grad_X, void* stream) {
    const std::string nm = "fock_shared_superposition_amplitudes_backward";
    if (!s || G < 0) return fail(SLOS_EINVAL, nm + ": bad argument");
    if (!U || !grad_U) return fail(SLOS_EINVAL, nm + ": NULL device pointer");
    if (G > 0 && (!X || !grad_out)) return fail(SLOS_EINVAL, nm + ": NULL device pointer");
    hipStream_t st = (hipStream_t)stream;
    const int N = s->N;
    int rc = shared_rows(*s, U, st);
    // dL/dX[g][c] = sum_t conj(A[c][t]) G[g][t]:  gX_cm (N x G) = A_cm^H G_cm
    if (rc == SLOS_OK && grad_X && G > 0)
        rc = cgemm(s->blas, st, rocblas_operation_conjugate_transpose, rocblas_operation_none, N, G, N, s->A, N,
                   (const float2*)grad_out, N, (float2*)grad_X, N);
    // dL/dA[c][t] = sum_g conj(X[g][c]) G[g][t]:  gA_cm (N x N) = G_cm X_cm^H
    if (rc == SLOS_OK) {
        if (G > 0)
            rc = cgemm(s->blas, st, rocblas_operation_none, rocblas_operation_conjugate_transpose, N, N, G,
                       (const float2*)grad_out, N, (const float2*)X, N, s->gA, N);
        else
            rc = launch_zero_c64((int64_t)N * N, s->gA, st);  // no inputs: dL/dA = 0
    }
    if (rc == SLOS_OK)
        rc = run(s->basis, SLOS_OP_AMPLITUDES_BACKWARD, (const float*)s->Urep, s->gA, (float*)s->gUc, s->ws,
                 s->ws_bytes, stream);
    if (rc == SLOS_OK)
        rc = launch_superposition(kSupGroupSum, s->dev, *s->basis, s->gUc, nullptr, nullptr, grad_U, st);
    return rc;
}

extern "C" int fock_probs_from_amplitudes(const float* amps, int64_t n, float* probs, void* stream) {
    if (n < 0) return fail(SLOS_EINVAL, "fock_probs_from_amplitudes: n < 0");
    if (n == 0) return SLOS_OK;
    if (!amps || !probs) return fail(SLOS_EINVAL, "fock_probs_from_amplitudes: NULL device pointer");
    return launch_abs2(n, (const float2*)amps, probs, (hipStream_t)stream);
}

extern "C" int fock_probs_from_amplitudes_backward(const float* amps, const float* grad_probs, int64_t n,
                                                   float* grad_amps, void* stream) {
    if (n < 0) return fail(SLOS_EINVAL, "fock_probs_from_amplitudes_backward: n < 0");
    if (n == 0) return SLOS_OK;
    if (!amps || !grad_probs || !grad_amps)
        return fail(SLOS_EINVAL, "fock_probs_from_amplitudes_backward: NULL device pointer");
    return launch_abs2_backward(n, (const float2*)amps, grad_probs, (float2*)grad_amps, (hipStream_t)stream);
}

extern "C" int fock_sample(slos_batch_t batch, const float* U, const float* u, int S, int32_t* shots, void* ws,
                           size_t ws_bytes, void* stream) {
    const std::string nm = "fock_sample";
    if (!batch) return fail(SLOS_EINVAL, nm + ": batch is NULL");
    if (S < 0) return fail(SLOS_EINVAL, nm + ": S must be >= 0");
    if (batch->B == 0) return SLOS_OK;
    if (!U) return fail(SLOS_EINVAL, nm + ": U is NULL");
    if (S > 0 && (!u || !shots)) return fail(SLOS_EINVAL, nm + ": uniforms or shots pointer is NULL");
    if (((int64_t)batch->B * S + 255) / 256 >= ((int64_t)1 << 31) ||
        (int64_t)batch->B * mode_expect_chunks(*batch) >= ((int64_t)1 << 31))
        return fail(SLOS_EUNSUPPORTED, nm + ": too many samples or shots for one launch");
    int v, blk;
    resolve(*batch, SLOS_OP_SAMPLE, &v, &blk);
    const bool fused = variant_fused(v);
    const size_t head = sample_head_bytes(*batch);
    const size_t need = head + (fused ? 0 : layered_ws_bytes(*batch, false));
    if (!ws || ws_bytes < need)
        return fail(SLOS_EWORKSPACE, nm + ": workspace missing or too small (need " + std::to_string(need) + " bytes)");
    char* base = (char*)ws;
    float* pv = (float*)base;
    double* cdf = (double*)(base + expect_head_bytes(*batch));
    double* part = (double*)(base + expect_head_bytes(*batch) + align256((size_t)batch->off_host[batch->B] * 8));
    hipStream_t s = (hipStream_t)stream;
    int rc = v == SLOS_VARIANT_FUSED_PAIRS ? launch_fused_pairs_fwd(*batch, blk, batch->cfg[SLOS_OP_SAMPLE].tile, (const float2*)U, pv, true, s)
             : fused                        ? launch_fused_fwd(*batch, blk, (const float2*)U, pv, 1, s)
                                            : launch_layered_fwd(*batch, blk, (const float2*)U, pv, true, base + head, s);
    if (rc != SLOS_OK) return rc;
    return launch_sample(*batch, pv, part, cdf, u, S, shots, s);
}

extern "C" int64_t slos_threshold_dim(int m, int n) { return threshold_dim(m, n); }

extern "C" int64_t slos_batch_threshold_len(slos_batch_t batch) {
    if (!batch) return -1;
    return batch->thr_off_host[batch->B];
}

extern "C" int slos_batch_threshold_offsets(slos_batch_t batch, int64_t* off_host) {
    if (!batch || !off_host) return fail(SLOS_EINVAL, "slos_batch_threshold_offsets: NULL argument");
    std::memcpy(off_host, batch->thr_off_host.data(), (batch->B + 1) * sizeof(int64_t));
    return SLOS_OK;
}

extern "C" int fock_threshold_probs(slos_batch_t batch, const float* U, float* out, void* ws, size_t ws_bytes,
                                    void* stream) {
    return run(batch, SLOS_OP_THRESHOLD_PROBS, U, nullptr, out, ws, ws_bytes, stream);
}

extern "C" int fock_threshold_probs_backward(slos_batch_t batch, const float* U, const float* grad_out,
                                             float* grad_U, void* ws, size_t ws_bytes, void* stream) {
    return run(batch, SLOS_OP_THRESHOLD_PROBS_BACKWARD, U, grad_out, grad_U, ws, ws_bytes, stream);
}

extern "C" int fock_mode_expectations(slos_batch_t batch, const float* U, float* out, void* ws, size_t ws_bytes,
                                      void* stream) {
    return run(batch, SLOS_OP_MODE_EXPECTATIONS, U, nullptr, out, ws, ws_bytes, stream);
}

extern "C" int fock_mode_expectations_backward(slos_batch_t batch, const float* U, const float* grad_out,
                                               float* grad_U, void* ws, size_t ws_bytes, void* stream) {
    return run(batch, SLOS_OP_MODE_EXPECTATIONS_BACKWARD, U, grad_out, grad_U, ws, ws_bytes, stream);
}

extern "C" int fock_mode_expectations_ex(slos_batch_t batch, const float* U, float* out, int detector, void* ws,
                                         size_t ws_bytes, void* stream) {
    if (detector != SLOS_DETECTOR_PNR && detector != SLOS_DETECTOR_THRESHOLD)
        return fail(SLOS_EINVAL, "fock_mode_expectations_ex: unknown detector model");
    return run(batch, SLOS_OP_MODE_EXPECTATIONS, U, nullptr, out, ws, ws_bytes, stream, detector);
}

extern "C" int fock_mode_expectations_backward_ex(slos_batch_t batch, const float* U, const float* grad_out,
                                                  float* grad_U, int detector, void* ws, size_t ws_bytes,
                                                  void* stream) {
    if (detector != SLOS_DETECTOR_PNR && detector != SLOS_DETECTOR_THRESHOLD)
        return fail(SLOS_EINVAL, "fock_mode_expectations_backward_ex: unknown detector model");
    return run(batch, SLOS_OP_MODE_EXPECTATIONS_BACKWARD, U, grad_out, grad_U, ws, ws_bytes, stream, detector);
}
