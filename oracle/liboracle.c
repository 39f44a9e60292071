/*
 * CPU FP64 oracle for state-vector gate application — TEST INFRASTRUCTURE ONLY.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load this
 * library. It shares no code with the GPU path.
 *
 * What it computes is the plain definition of full-state simulation (paper
 * Sec. II-A, the equations U = I^(k-1) (x) G (x) I^(n-k) and U|phi>): every gate
 * is applied as a dense 2x2, 4x4 or 8x8 complex matrix on the amplitudes it couples,
 * in double precision, with no use of sparsity, diagonality or Hadamard
 * structure. The one n-qubit gate, MARK(m) (sign flip of basis state |m>, the
 * Grover phase oracle of Sec. IV-D), is applied by its definition.
 *
 * Conventions: amplitude index i = sum_q b_q 2^q (qubit q is bit q). A 2-qubit
 * gate matrix is indexed by the local index (b_q0 << 1) | b_q1, so the first
 * operand q0 is the high local bit; a 3-qubit gate's local index is
 * (b_q0 << 2) | (b_q1 << 1) | b_q2. Complex numbers are C99 double complex,
 * interleaved (re, im) in memory.
 */
#include <complex.h>
#include <stdint.h>
#include <stddef.h>
#include <math.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Below this many amplitudes the loops stay single-threaded. */
#define OR_PAR_MIN (1LL << 14)

int or_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int k) {
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/* Insert a zero bit at position q into x. */
static inline int64_t ins0(int64_t x, int q) {
    int64_t lo = x & ((1LL << q) - 1);
    return ((x >> q) << (q + 1)) | lo;
}

/* psi <- (I (x) .. (x) G (x) .. (x) I) psi for a 2x2 matrix G on qubit q. */
void or_apply_1q(cplx *psi, int n, int q, const cplx *m) {
    const int64_t half = 1LL << (n - 1);
    const cplx g00 = m[0], g01 = m[1], g10 = m[2], g11 = m[3];
    const int64_t step = 1LL << q;
#pragma omp parallel for schedule(static) if (half >= OR_PAR_MIN)
    for (int64_t p = 0; p < half; ++p) {
        int64_t i0 = ins0(p, q);
        int64_t i1 = i0 | step;
        cplx a0 = psi[i0], a1 = psi[i1];
        psi[i0] = g00 * a0 + g01 * a1;
        psi[i1] = g10 * a0 + g11 * a1;
    }
}

/* 4x4 matrix on qubits (q0, q1); row/column index (b_q0 << 1) | b_q1. */
void or_apply_2q(cplx *psi, int n, int q0, int q1, const cplx *m) {
    const int64_t quarter = 1LL << (n - 2);
    const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
    const int64_t s0 = 1LL << q0, s1 = 1LL << q1;
#pragma omp parallel for schedule(static) if (quarter >= OR_PAR_MIN)
    for (int64_t p = 0; p < quarter; ++p) {
        int64_t base = ins0(ins0(p, lo), hi);
        int64_t idx[4];
        cplx a[4];
        for (int l = 0; l < 4; ++l) {
            idx[l] = base | ((l >> 1) ? s0 : 0) | ((l & 1) ? s1 : 0);
            a[l] = psi[idx[l]];
        }
        for (int r = 0; r < 4; ++r) {
            cplx acc = 0.0;
            for (int c = 0; c < 4; ++c) acc += m[4 * r + c] * a[c];
            psi[idx[r]] = acc;
        }
    }
}

/* 8x8 matrix on qubits (q0, q1, q2); row/column index (b_q0 << 2) | (b_q1 << 1) | b_q2. */
void or_apply_3q(cplx *psi, int n, int q0, int q1, int q2, const cplx *m) {
    const int64_t eighth = 1LL << (n - 3);
    int srt[3] = {q0, q1, q2};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (srt[j] < srt[i]) { int t = srt[i]; srt[i] = srt[j]; srt[j] = t; }
    const int64_t s0 = 1LL << q0, s1 = 1LL << q1, s2 = 1LL << q2;
#pragma omp parallel for schedule(static) if (eighth >= OR_PAR_MIN)
    for (int64_t p = 0; p < eighth; ++p) {
        int64_t base = ins0(ins0(ins0(p, srt[0]), srt[1]), srt[2]);
        int64_t idx[8];
        cplx a[8];
        for (int l = 0; l < 8; ++l) {
            idx[l] = base | ((l >> 2) & 1 ? s0 : 0) | ((l >> 1) & 1 ? s1 : 0) | ((l & 1) ? s2 : 0);
            a[l] = psi[idx[l]];
        }
        for (int r = 0; r < 8; ++r) {
            cplx acc = 0.0;
            for (int c = 0; c < 8; ++c) acc += m[8 * r + c] * a[c];
            psi[idx[r]] = acc;
        }
    }
}

/* MARK(m): the diagonal operator I - 2|m><m|. */
void or_apply_mark(cplx *psi, int n, uint64_t mk) {
    (void)n;
    psi[mk] = -psi[mk];
}

/*
 * Apply a whole gate list. kind[g] = 1 (1-qubit, matrix mats[64g .. 64g+3]),
 * 2 (2-qubit, mats[64g .. 64g+15]), 3 (MARK, basis index idx[g]) or
 * 4 (3-qubit on q0, q1, q2, mats[64g .. 64g+63]).
 * Returns the number of gates applied, or -(g+1) for a bad record g.
 */
int64_t or_run(cplx *psi, int n, int64_t ng, const int32_t *kind,
               const int32_t *q0, const int32_t *q1, const int32_t *q2, const cplx *mats,
               const uint64_t *idx) {
    for (int64_t g = 0; g < ng; ++g) {
        switch (kind[g]) {
        case 1:
            if (q0[g] < 0 || q0[g] >= n) return -(g + 1);
            or_apply_1q(psi, n, q0[g], mats + 64 * g);
            break;
        case 2:
            if (q0[g] < 0 || q0[g] >= n || q1[g] < 0 || q1[g] >= n || q0[g] == q1[g])
                return -(g + 1);
            or_apply_2q(psi, n, q0[g], q1[g], mats + 64 * g);
            break;
        case 3:
            if (idx[g] >= (1ULL << n)) return -(g + 1);
            or_apply_mark(psi, n, idx[g]);
            break;
        case 4:
            if (n < 3 || q0[g] < 0 || q0[g] >= n || q1[g] < 0 || q1[g] >= n || q2[g] < 0 || q2[g] >= n ||
                q0[g] == q1[g] || q0[g] == q2[g] || q1[g] == q2[g])
                return -(g + 1);
            or_apply_3q(psi, n, q0[g], q1[g], q2[g], mats + 64 * g);
            break;
        default:
            return -(g + 1);
        }
    }
    return ng;
}

/*
 * Sums of |a_i|^2 * w_i by pairwise summation over fixed blocks: the result
 * does not depend on the thread count. w_i = 1 (norm) or 1 - 2 b_q(i) (<Z_q>).
 */
#define OR_BLOCK 4096

static double pairwise(const double *v, int64_t len) {
    if (len <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < len; ++i) s += v[i];
        return s;
    }
    int64_t h = len / 2;
    return pairwise(v, h) + pairwise(v + h, len - h);
}

static double block_sum(const cplx *psi, int64_t start, int64_t len, int q) {
    double buf[OR_BLOCK];
    for (int64_t i = 0; i < len; ++i) {
        int64_t j = start + i;
        double re = creal(psi[j]), im = cimag(psi[j]);
        double p = re * re + im * im;
        if (q >= 0 && ((j >> q) & 1)) p = -p;
        buf[i] = p;
    }
    return pairwise(buf, len);
}

static double weighted_sum(const cplx *psi, int n, int q) {
    const int64_t N = 1LL << n;
    const int64_t nb = (N + OR_BLOCK - 1) / OR_BLOCK;
    double *parts = (double *)malloc((size_t)nb * sizeof(double));
    double result;
    if (!parts) return NAN;
#pragma omp parallel for schedule(static) if (nb >= 8)
    for (int64_t b = 0; b < nb; ++b) {
        int64_t st = b * OR_BLOCK;
        int64_t len = (N - st) < OR_BLOCK ? (N - st) : OR_BLOCK;
        parts[b] = block_sum(psi, st, len, q);
    }
    result = pairwise(parts, nb);
    free(parts);
    return result;
}

double or_norm2(const cplx *psi, int n) { return weighted_sum(psi, n, -1); }

double or_expect_z(const cplx *psi, int n, int q) { return weighted_sum(psi, n, q); }

/* <a|b> = sum conj(a_i) b_i, pairwise over fixed blocks (real and imag parts). */
void or_inner(const cplx *a, const cplx *b, int n, double *out_re, double *out_im) {
    const int64_t N = 1LL << n;
    const int64_t nb = (N + OR_BLOCK - 1) / OR_BLOCK;
    double *pr = (double *)malloc((size_t)nb * sizeof(double));
    double *pi = (double *)malloc((size_t)nb * sizeof(double));
    if (!pr || !pi) { free(pr); free(pi); *out_re = NAN; *out_im = NAN; return; }
#pragma omp parallel for schedule(static) if (nb >= 8)
    for (int64_t blk = 0; blk < nb; ++blk) {
        double br[OR_BLOCK], bi[OR_BLOCK];
        int64_t st = blk * OR_BLOCK;
        int64_t len = (N - st) < OR_BLOCK ? (N - st) : OR_BLOCK;
        for (int64_t i = 0; i < len; ++i) {
            cplx z = conj(a[st + i]) * b[st + i];
            br[i] = creal(z);
            bi[i] = cimag(z);
        }
        pr[blk] = pairwise(br, len);
        pi[blk] = pairwise(bi, len);
    }
    *out_re = pairwise(pr, nb);
    *out_im = pairwise(pi, nb);
    free(pr);
    free(pi);
}
