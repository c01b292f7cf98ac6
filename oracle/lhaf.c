/*
 * Brute-force loop hafnian (oracle; test infrastructure only).
 *
 * Computes lhaf(filldiag(A_m, g_m)) (Eq. gen_loop_haf_def / Eq. lhaf_def):
 * the sum over all single-pair matchings (every vertex either carries a loop,
 * weight g, or is paired with exactly one other vertex, weight A) of the
 * product of weights, for the graph in which vertex type t appears mult[t]
 * times.  Two distinct copies of type t are joined by A[t][t]; the diagonal
 * of the repeated matrix is overwritten by g (filldiag), so a loop on a copy of
 * t weighs g[t].
 *
 * Recursion on the set of unmatched vertices: take one copy of the first type
 * t that still has copies left; it is either a loop, or paired with one of the
 * (mult_t - 1) other copies of t, or with one of the mult_s copies of a later
 * type s.  Copies are indistinguishable in weight, so the state is the vector
 * of remaining multiplicities; it is tabulated over all such vectors in
 * increasing mixed-radix order (every transition goes to a smaller index).
 *
 * Cost: prod_t (mult_t + 1) states times nt transitions.
 */
#include <stdlib.h>

typedef struct { double re, im; } cplx;

static inline cplx cmul(cplx a, cplx b) { cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static inline cplx cscale(cplx a, double s) { cplx r = {a.re * s, a.im * s}; return r; }
static inline cplx cadd(cplx a, cplx b) { cplx r = {a.re + b.re, a.im + b.im}; return r; }

/* A: nt*nt complex (interleaved re,im; row-major), g: nt complex, mult: nt >= 0.
 * out: 2 doubles.  Returns 0 on success, -1 on allocation failure or bad size. */
int oracle_lhaf_multiset(int nt, const double *A, const double *g, const int *mult, double *out)
{
    long stride[64];
    long total = 1;
    if (nt <= 0 || nt > 64) return -1;
    for (int t = 0; t < nt; ++t) {
        if (mult[t] < 0) return -1;
        stride[t] = total;
        total *= (long)(mult[t] + 1);
        if (total > (1L << 31)) return -1;
    }
    cplx *f = (cplx *)malloc(sizeof(cplx) * (size_t)total);
    if (!f) return -1;
    int r[64];
    for (long idx = 0; idx < total; ++idx) {
        long rem = idx;
        int t0 = -1;
        for (int t = 0; t < nt; ++t) {
            r[t] = (int)(rem % (mult[t] + 1));
            rem /= (mult[t] + 1);
            if (t0 < 0 && r[t] > 0) t0 = t;
        }
        if (t0 < 0) { f[idx].re = 1.0; f[idx].im = 0.0; continue; }
        cplx gt = {g[2 * t0], g[2 * t0 + 1]};
        cplx acc = cmul(gt, f[idx - stride[t0]]);
        if (r[t0] >= 2) {
            cplx att = {A[2 * (t0 * nt + t0)], A[2 * (t0 * nt + t0) + 1]};
            acc = cadd(acc, cscale(cmul(att, f[idx - 2 * stride[t0]]), (double)(r[t0] - 1)));
        }
        for (int s = t0 + 1; s < nt; ++s) {
            if (r[s] == 0) continue;
            cplx ats = {A[2 * (t0 * nt + s)], A[2 * (t0 * nt + s) + 1]};
            acc = cadd(acc, cscale(cmul(ats, f[idx - stride[t0] - stride[s]]), (double)r[s]));
        }
        f[idx] = acc;
    }
    out[0] = f[total - 1].re;
    out[1] = f[total - 1].im;
    free(f);
    return 0;
}
