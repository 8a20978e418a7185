/*
 * Plain C numerics for the CPU oracle (test infrastructure only).
 *
 * Built with gcc -O2 -ffp-contract=off (no fast-math), so every operation
 * below is one IEEE-754 double operation rounded to nearest-even, exactly
 * as written.  Nothing here is blocked, reordered or vectorised by hand.
 *
 *  - or_log / or_exp / or_erf / or_pow: call the host C library element by
 *    element (the elementwise transcendental tasks of the paper's stream
 *    model, section 2 and section 7's Black-Scholes benchmark).
 *  - or_spmv: CSR sparse matrix-vector product y = A x with each row summed
 *    sequentially in CSR (column-sorted) order, the product of the sparse
 *    Krylov solvers of section 7.  s = a0*x0; s = s + ak*xk for k = 1..
 *  - or_fsum / or_fsum_prod: the exactly rounded sum of doubles (resp. of
 *    the rounded products x_i*y_i), computed with Shewchuk's
 *    non-overlapping-partials method ("Adaptive Precision Floating-Point
 *    Arithmetic and Fast Robust Geometric Predicates", 1997) with a final
 *    round-half-even correction.  The partials loop and the half-even
 *    correction follow the way CPython's math.fsum applies the method
 *    (Raymond Hettinger's msum recipe, with its final correction across the
 *    remaining partials); the tests check this sum against math.fsum.
 *    This is the reduction privilege's sum (section 3.2) with no
 *    rounding-order choice left.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

void or_log(const double* x, double* y, int64_t n) {
    for (int64_t i = 0; i < n; ++i) y[i] = log(x[i]);
}

void or_exp(const double* x, double* y, int64_t n) {
    for (int64_t i = 0; i < n; ++i) y[i] = exp(x[i]);
}

void or_erf(const double* x, double* y, int64_t n) {
    for (int64_t i = 0; i < n; ++i) y[i] = erf(x[i]);
}

void or_pow(const double* x, const double* e, double* y, int64_t n) {
    for (int64_t i = 0; i < n; ++i) y[i] = pow(x[i], e[i]);
}

void or_spmv(int64_t nrows, const int32_t* rowptr, const int32_t* col,
             const double* val, const double* x, double* y) {
    for (int64_t i = 0; i < nrows; ++i) {
        int32_t b = rowptr[i], e = rowptr[i + 1];
        double s = 0.0;
        if (b < e) {
            s = val[b] * x[col[b]];
            for (int32_t k = b + 1; k < e; ++k) {
                double t = val[k] * x[col[k]];
                s = s + t;
            }
        }
        y[i] = s;
    }
}

/* Partials state for the exactly rounded sum. */
typedef struct {
    double* p;
    int64_t n, cap;
} partials;

static void partials_add(partials* ps, double x) {
    int64_t i = 0;
    for (int64_t j = 0; j < ps->n; ++j) {
        double y = ps->p[j];
        if (fabs(x) < fabs(y)) { double t = x; x = y; y = t; }
        double hi = x + y;
        double lo = y - (hi - x);
        if (lo != 0.0) ps->p[i++] = lo;
        x = hi;
    }
    ps->n = i;
    if (ps->n == ps->cap) {
        ps->cap *= 2;
        ps->p = (double*)realloc(ps->p, (size_t)ps->cap * sizeof(double));
    }
    ps->p[ps->n++] = x;
}

static double partials_round(partials* ps) {
    int64_t n = ps->n;
    double hi = 0.0, lo = 0.0;
    if (n > 0) {
        hi = ps->p[--n];
        while (n > 0) {
            double x = hi;
            double y = ps->p[--n];
            hi = x + y;
            double yr = hi - x;
            lo = y - yr;
            if (lo != 0.0) break;
        }
        /* Round half to even across the remaining partials. */
        if (n > 0 && ((lo < 0.0 && ps->p[n - 1] < 0.0) ||
                      (lo > 0.0 && ps->p[n - 1] > 0.0))) {
            double y = lo * 2.0;
            double x = hi + y;
            double yr = x - hi;
            if (y == yr) hi = x;
        }
    }
    return hi;
}

double or_fsum(const double* x, int64_t n) {
    partials ps;
    ps.cap = 64; ps.n = 0;
    ps.p = (double*)malloc((size_t)ps.cap * sizeof(double));
    for (int64_t i = 0; i < n; ++i) partials_add(&ps, x[i]);
    double r = partials_round(&ps);
    free(ps.p);
    return r;
}

double or_fsum_prod(const double* x, const double* y, int64_t n) {
    partials ps;
    ps.cap = 64; ps.n = 0;
    ps.p = (double*)malloc((size_t)ps.cap * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        double t = x[i] * y[i];
        partials_add(&ps, t);
    }
    double r = partials_round(&ps);
    free(ps.p);
    return r;
}
