/*
 * FP64 reference ("oracle") for strong simulation of a linear-optical
 * interferometer.  TEST INFRASTRUCTURE ONLY: it exists to check the GPU
 * library, and only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code, header or table with the
 * GPU library.
 *
 * What it computes (paper, Sec. II-A-1 "Essentials of linear optics"): for an
 * n-photon input Fock state s over m modes and an m x m unitary U, the output
 * state t is reached with an amplitude given by the permanent of a
 * sub-matrix of U, up to normalisation factors.  Written out:
 *
 *   a_t = Perm(A) / sqrt(prod_i s_i! * prod_j t_j!),
 *   A[r][c] = U[R_r][C_c],
 *
 * with R = output modes j repeated t_j times (ascending) and C = input modes
 * i repeated s_i times (ascending).  U[j][i] is the single-photon amplitude
 * from input mode i to output mode j (row-major, U[j*m + i]).
 *
 * The permanent is taken by Ryser's inclusion-exclusion formula
 *
 *   Perm(A) = (-1)^n sum_{S subset of columns} (-1)^{|S|} prod_r sum_{c in S} A[r][c]
 *
 * visiting the subsets S in reflected-Gray-code order, so that one column
 * enters or leaves S per step and the row sums are updated by one add.
 * Everything is complex128; no blocking, fusion or reuse of intermediates
 * across outputs (that reuse is what the method under test does).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_NMAX 24

/* Ryser's formula, Gray-code order.  A is n x n row-major.  Perm of the
 * empty matrix (n == 0) is 1. */
double complex oracle_permanent(int n, const double complex* A)
{
    if (n == 0) return 1.0;
    if (n > ORACLE_NMAX) return NAN;
    double complex rowsum[ORACLE_NMAX];
    for (int r = 0; r < n; ++r) rowsum[r] = 0.0;
    double complex total = 0.0;
    uint64_t gray_prev = 0;
    const uint64_t nsub = (uint64_t)1 << n;
    for (uint64_t k = 1; k < nsub; ++k) {
        uint64_t gray = k ^ (k >> 1);
        uint64_t diff = gray ^ gray_prev; /* exactly one bit */
        int c = __builtin_ctzll(diff);
        double sign_in = (gray & diff) ? 1.0 : -1.0; /* column entered or left */
        for (int r = 0; r < n; ++r) rowsum[r] += sign_in * A[r * n + c];
        gray_prev = gray;
        double complex prod = 1.0;
        for (int r = 0; r < n; ++r) prod *= rowsum[r];
        int size = __builtin_popcountll(gray);
        total += (size & 1) ? -prod : prod;
    }
    return (n & 1) ? -total : total;
}

static double factorial(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= (double)i;
    return f;
}

/* Expand an occupation vector into the ascending list of its modes. */
static int expand_modes(int m, const int32_t* occ, int* modes)
{
    int n = 0;
    for (int j = 0; j < m; ++j)
        for (int q = 0; q < occ[j]; ++q) modes[n++] = j;
    return n;
}

static double occ_factorial_product(int m, const int32_t* occ)
{
    double f = 1.0;
    for (int j = 0; j < m; ++j) f *= factorial(occ[j]);
    return f;
}

/* Amplitudes a_t for n_out output states t_occ[k*m .. k*m+m-1] (all with the
 * same photon number as s).  out[k] receives a_t.  Returns 0, or -1 if an
 * output state has a different photon number than the input. */
int oracle_amplitudes(int m, const int32_t* s_occ, const double complex* U,
                      int64_t n_out, const int32_t* t_occ, double complex* out)
{
    int cols[ORACLE_NMAX];
    const int n = expand_modes(m, s_occ, cols);
    if (n > ORACLE_NMAX) return -1;
    const double s_fact = occ_factorial_product(m, s_occ);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (int64_t k = 0; k < n_out; ++k) {
        const int32_t* t = t_occ + k * m;
        int rows[ORACLE_NMAX];
        int nt = 0;
        for (int j = 0; j < m; ++j) nt += t[j];
        if (nt != n) { bad = 1; continue; }
        expand_modes(m, t, rows);
        double complex A[ORACLE_NMAX * ORACLE_NMAX];
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) A[r * n + c] = U[rows[r] * m + cols[c]];
        const double norm = sqrt(s_fact * occ_factorial_product(m, t));
        out[k] = oracle_permanent(n, A) / norm;
    }
    return bad ? -1 : 0;
}

/* Gradient of a real loss with respect to U, given the loss gradient G_a with
 * respect to each listed output amplitude, both in the convention
 * G = dL/dRe + i dL/dIm.  Since a_t is holomorphic in U,
 *
 *   G_U[j][i] = sum_t G_a[t] * conj(d a_t / d U[j][i]),
 *
 * and the derivative of a permanent with respect to one entry is the
 * permanent of the minor without that entry's row and column.  Every copy of
 * output mode j among the rows (t_j of them) and of input mode i among the
 * columns (s_i of them) gives the same minor A(t - e_j, s - e_i), so
 *
 *   d a_t / d U[j][i] = t_j * s_i * Perm(U[R(t-e_j), C(s-e_i)]) / sqrt(prod s! prod t!).
 *
 * GU (m*m, row-major) is overwritten.  Returns 0 or -1 on bad input. */
int oracle_amplitude_grad(int m, const int32_t* s_occ, const double complex* U,
                          int64_t n_out, const int32_t* t_occ,
                          const double complex* Ga, double complex* GU)
{
    int cols_all[ORACLE_NMAX];
    const int n = expand_modes(m, s_occ, cols_all);
    if (n > ORACLE_NMAX || n < 1) return -1;
    const double s_fact = occ_factorial_product(m, s_occ);
    for (int q = 0; q < m * m; ++q) GU[q] = 0.0;
    int bad = 0;
#pragma omp parallel reduction(| : bad)
    {
        double complex* acc = (double complex*)calloc((size_t)m * m, sizeof(double complex));
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < n_out; ++k) {
            const int32_t* t = t_occ + k * m;
            int nt = 0;
            for (int j = 0; j < m; ++j) nt += t[j];
            if (nt != n) { bad = 1; continue; }
            const double norm = sqrt(s_fact * occ_factorial_product(m, t));
            int32_t tm[64], sm[64];
            for (int j = 0; j < m; ++j) { tm[j] = t[j]; sm[j] = s_occ[j]; }
            for (int j = 0; j < m; ++j) {
                if (t[j] == 0) continue;
                for (int i = 0; i < m; ++i) {
                    if (s_occ[i] == 0) continue;
                    tm[j] -= 1; sm[i] -= 1;
                    int rows[ORACLE_NMAX], cols[ORACLE_NMAX];
                    expand_modes(m, tm, rows);
                    expand_modes(m, sm, cols);
                    double complex A[ORACLE_NMAX * ORACLE_NMAX];
                    for (int r = 0; r < n - 1; ++r)
                        for (int c = 0; c < n - 1; ++c)
                            A[r * (n - 1) + c] = U[rows[r] * m + cols[c]];
                    double complex dperm = (double)t[j] * (double)s_occ[i] * oracle_permanent(n - 1, A);
                    tm[j] += 1; sm[i] += 1;
                    acc[j * m + i] += Ga[k] * conj(dperm / norm);
                }
            }
        }
#pragma omp critical
        for (int q = 0; q < m * m; ++q) GU[q] += acc[q];
        free(acc);
    }
    return bad ? -1 : 0;
}
