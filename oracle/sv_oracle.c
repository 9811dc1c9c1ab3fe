/*
 * FP64 CPU oracle for Schroedinger-style state-vector simulation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call
 * this file; it exists so tests and benchmarks can check the GPU library
 * against a plain, slow, obviously correct implementation.
 *
 * Everything here follows the "fast Schroedinger simulation" definition of
 * Sec. 3 (Baseline Simulation Algorithms): a q-qubit gate with matrix U on
 * qubits i_0..i_{q-1} updates, in place, each of the 2^{n-q} disjoint sets of
 * 2^q amplitudes whose indices share the other n-q bits (the "set id").  The
 * oracle uses this one generic path for every gate; it has no special cases
 * for diagonal or permutation gates.
 *
 * Layout: psi is 2^n complex doubles, interleaved (re, im).  Qubit q is bit q
 * of the amplitude index.  A gate's local index is l = sum_t bit(j, q[t]) 2^t
 * and its matrix is row-major 2^k x 2^k complex, interleaved.
 *
 * Norms and expectations use the compensated summation the paper recommends
 * for the norm check (Sec. 4.1): the Sum2 algorithm of Ogita, Rump and Oishi
 * (cascaded TwoSum with the rounding errors summed separately).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* Set id s (n-k bits) -> base index with zeros at the gate's qubits
 * (positions given in ascending order in qs). */
static inline uint64_t insert_zero_bits(uint64_t s, const int *qs_sorted, int k)
{
    for (int t = 0; t < k; ++t) {
        uint64_t low = s & ((1ull << qs_sorted[t]) - 1ull);
        s = ((s >> qs_sorted[t]) << (qs_sorted[t] + 1)) | low;
    }
    return s;
}

/* Apply a k-qubit gate (k <= 10) to psi in place. Returns 0 on success. */
int or_apply(int n, double *psi, int k, const int *q, const double *u, int nthreads)
{
    if (k < 1 || k > 10 || k > n) return 1;
    int qs[10];
    for (int t = 0; t < k; ++t) {
        if (q[t] < 0 || q[t] >= n) return 2;
        qs[t] = q[t];
    }
    /* sort positions ascending for the zero-insertion */
    for (int a = 0; a < k; ++a)
        for (int b = a + 1; b < k; ++b)
            if (qs[b] < qs[a]) { int tmp = qs[a]; qs[a] = qs[b]; qs[b] = tmp; }
    for (int a = 1; a < k; ++a)
        if (qs[a] == qs[a - 1]) return 3;

    const uint64_t dim = 1ull << k;
    /* offset of local index l: sum_t bit(l, t) << q[t] (gate's own order) */
    uint64_t *off = (uint64_t *)malloc(sizeof(uint64_t) * dim);
    for (uint64_t l = 0; l < dim; ++l) {
        uint64_t o = 0;
        for (int t = 0; t < k; ++t)
            if ((l >> t) & 1ull) o |= 1ull << q[t];
        off[l] = o;
    }
    const int64_t nsets = (int64_t)(1ull << (n - k));
    if (nthreads <= 0) nthreads = omp_get_max_threads();

#pragma omp parallel num_threads(nthreads)
    {
        double *a = (double *)malloc(sizeof(double) * 2 * dim);
#pragma omp for schedule(static)
        for (int64_t s = 0; s < nsets; ++s) {
            uint64_t base = insert_zero_bits((uint64_t)s, qs, k);
            for (uint64_t l = 0; l < dim; ++l) {
                a[2 * l] = psi[2 * (base | off[l])];
                a[2 * l + 1] = psi[2 * (base | off[l]) + 1];
            }
            for (uint64_t r = 0; r < dim; ++r) {
                double re = 0.0, im = 0.0;
                const double *row = u + 2 * r * dim;
                for (uint64_t c = 0; c < dim; ++c) {
                    double ur = row[2 * c], ui = row[2 * c + 1];
                    double ar = a[2 * c], ai = a[2 * c + 1];
                    re += ur * ar - ui * ai;
                    im += ur * ai + ui * ar;
                }
                psi[2 * (base | off[r])] = re;
                psi[2 * (base | off[r]) + 1] = im;
            }
        }
        free(a);
    }
    free(off);
    return 0;
}

/* ---- compensated summation (Sum2 of Ogita, Rump and Oishi) ---- */
typedef struct { double s, e; } sum2_t;

static inline void two_sum_acc(sum2_t *acc, double x)
{
    double s = acc->s + x;
    double bp = s - acc->s;
    double err = (acc->s - (s - bp)) + (x - bp);
    acc->s = s;
    acc->e += err;
}

static double sum2_combine(sum2_t *parts, int m)
{
    sum2_t tot = {0.0, 0.0};
    for (int i = 0; i < m; ++i) {
        two_sum_acc(&tot, parts[i].s);
        tot.e += parts[i].e;
    }
    return tot.s + tot.e;
}

/* sum_j |psi_j|^2 */
double or_norm2(int n, const double *psi, int nthreads)
{
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    sum2_t *parts = (sum2_t *)calloc((size_t)nthreads, sizeof(sum2_t));
    const int64_t N = (int64_t)(1ull << n);
#pragma omp parallel num_threads(nthreads)
    {
        sum2_t acc = {0.0, 0.0};
        int tid = omp_get_thread_num();
#pragma omp for schedule(static)
        for (int64_t j = 0; j < N; ++j) {
            double r = psi[2 * j], i = psi[2 * j + 1];
            two_sum_acc(&acc, r * r);
            two_sum_acc(&acc, i * i);
        }
        parts[tid] = acc;
    }
    double v = sum2_combine(parts, nthreads);
    free(parts);
    return v;
}

/* <psi| X^x Z^z |psi> where (X^x Z^z psi)[j] = (-1)^{|(j^x)&z|} psi[j^x].
 * Returns real and imaginary parts (the i^{|x&z|} factor that turns XZ into
 * Y is applied by the caller). */
void or_pauli_expect(int n, const double *psi, uint64_t x, uint64_t z,
                     double *out_re, double *out_im, int nthreads)
{
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    sum2_t *pr = (sum2_t *)calloc((size_t)nthreads, sizeof(sum2_t));
    sum2_t *pi = (sum2_t *)calloc((size_t)nthreads, sizeof(sum2_t));
    const int64_t N = (int64_t)(1ull << n);
#pragma omp parallel num_threads(nthreads)
    {
        sum2_t ar = {0.0, 0.0}, ai = {0.0, 0.0};
        int tid = omp_get_thread_num();
#pragma omp for schedule(static)
        for (int64_t j = 0; j < N; ++j) {
            uint64_t jj = (uint64_t)j ^ x;
            double sgn = (__builtin_popcountll(jj & z) & 1) ? -1.0 : 1.0;
            /* conj(psi[j]) * sgn * psi[jj] */
            double a = psi[2 * j], b = psi[2 * j + 1];
            double c = psi[2 * jj], d = psi[2 * jj + 1];
            two_sum_acc(&ar, sgn * (a * c + b * d));
            two_sum_acc(&ai, sgn * (a * d - b * c));
        }
        pr[tid] = ar;
        pi[tid] = ai;
    }
    *out_re = sum2_combine(pr, nthreads);
    *out_im = sum2_combine(pi, nthreads);
    free(pr);
    free(pi);
}

/* <a|b> (conjugate-linear in a), compensated. */
void or_inner(int n, const double *a, const double *b, double *out_re, double *out_im, int nthreads)
{
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    sum2_t *pr = (sum2_t *)calloc((size_t)nthreads, sizeof(sum2_t));
    sum2_t *pi = (sum2_t *)calloc((size_t)nthreads, sizeof(sum2_t));
    const int64_t N = (int64_t)(1ull << n);
#pragma omp parallel num_threads(nthreads)
    {
        sum2_t ar = {0.0, 0.0}, ai = {0.0, 0.0};
        int tid = omp_get_thread_num();
#pragma omp for schedule(static)
        for (int64_t j = 0; j < N; ++j) {
            double p = a[2 * j], q = a[2 * j + 1];
            double r = b[2 * j], s = b[2 * j + 1];
            two_sum_acc(&ar, p * r + q * s);
            two_sum_acc(&ai, p * s - q * r);
        }
        pr[tid] = ar;
        pi[tid] = ai;
    }
    *out_re = sum2_combine(pr, nthreads);
    *out_im = sum2_combine(pi, nthreads);
    free(pr);
    free(pi);
}

int or_max_threads(void) { return omp_get_max_threads(); }
