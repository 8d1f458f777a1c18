/* Plain C state-vector simulator (oracle, complex128).
 *
 * Schroedinger method: the 2^n amplitudes are stored and every gate is
 * applied in place, in circuit order.  Qubit q is bit (n-1-q) of the basis
 * index.  Gate matrices are row-major, (re, im) interleaved, row = output,
 * column = input, two-qubit basis |q0 q1> with q0 the more significant bit.
 *
 * Test infrastructure only; never linked into the GPU library.
 */
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cplx;

static inline cplx cmul(cplx a, cplx b) {
    cplx r = { a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re };
    return r;
}
static inline cplx cadd(cplx a, cplx b) { cplx r = { a.re + b.re, a.im + b.im }; return r; }

static void apply1(cplx* psi, int n, int q, const double* m) {
    long long stride = 1LL << (n - 1 - q);
    long long total = 1LL << n;
    cplx u[4];
    for (int i = 0; i < 4; ++i) { u[i].re = m[2 * i]; u[i].im = m[2 * i + 1]; }
    #pragma omp parallel for schedule(static)
    for (long long base = 0; base < total / 2; ++base) {
        /* insert a zero bit at position log2(stride) */
        long long lo = base & (stride - 1);
        long long i0 = ((base - lo) << 1) | lo;
        long long i1 = i0 | stride;
        cplx a = psi[i0], b = psi[i1];
        psi[i0] = cadd(cmul(u[0], a), cmul(u[1], b));
        psi[i1] = cadd(cmul(u[2], a), cmul(u[3], b));
    }
}

static void apply2(cplx* psi, int n, int q0, int q1, const double* m) {
    long long s0 = 1LL << (n - 1 - q0);
    long long s1 = 1LL << (n - 1 - q1);
    long long slo = s0 < s1 ? s0 : s1, shi = s0 < s1 ? s1 : s0;
    long long total = 1LL << n;
    cplx u[16];
    for (int i = 0; i < 16; ++i) { u[i].re = m[2 * i]; u[i].im = m[2 * i + 1]; }
    #pragma omp parallel for schedule(static)
    for (long long base = 0; base < total / 4; ++base) {
        long long x = base;
        long long lo = x & (slo - 1);
        x = ((x - lo) << 1) | lo;             /* zero bit at slo */
        long long lo2 = x & (shi - 1);
        x = ((x - lo2) << 1) | lo2;           /* zero bit at shi */
        long long idx[4] = { x, x | s1, x | s0, x | s0 | s1 };  /* |q0 q1> = 00,01,10,11 */
        cplx v[4];
        for (int k = 0; k < 4; ++k) v[k] = psi[idx[k]];
        for (int r = 0; r < 4; ++r) {
            cplx acc = { 0.0, 0.0 };
            for (int c = 0; c < 4; ++c) acc = cadd(acc, cmul(u[4 * r + c], v[c]));
            psi[idx[r]] = acc;
        }
    }
}

int oracle_sv_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* qubits: n_gates x 2 (second = -1 for a single-qubit gate);
 * mats: n_gates x 32 doubles (2x2 uses the first 8);
 * psi: 2 * 2^n doubles, overwritten with the final state. */
int oracle_sv_run(int n, int n_gates, const int* qubits, const double* mats, double* psi_out) {
    if (n < 1 || n > 34) return -1;
    cplx* psi = (cplx*)psi_out;
    long long total = 1LL << n;
    memset(psi, 0, sizeof(cplx) * (size_t)total);
    psi[0].re = 1.0;
    for (int g = 0; g < n_gates; ++g) {
        int q0 = qubits[2 * g], q1 = qubits[2 * g + 1];
        if (q0 < 0 || q0 >= n || q1 >= n || q1 == q0) return -2;
        if (q1 < 0) apply1(psi, n, q0, mats + 32 * g);
        else apply2(psi, n, q0, q1, mats + 32 * g);
    }
    return 0;
}
