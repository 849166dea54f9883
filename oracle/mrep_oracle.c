/*
 * mrep_oracle.c -- slow, plain FP64 CPU oracle for B-spline point projection
 * and inversion (Wu & Zou, "Matrix representation and GPU-optimized parallel
 * B-spline computing").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the GPU path.
 *
 * What it computes, each function citing the passage it follows:
 *   - Cox-de Boor basis values                      (Sec. 4, eq. bsplinebasis)
 *   - curve evaluation by de Boor's algorithm      (Sec. 4, curve definition)
 *   - Bezier pieces by Boehm knot insertion         (Sec. 5.2.1; the textbook
 *     route the paper replaces by its matrix form, used here as the check)
 *   - degree elevation for p <= 2                   (Sec. 5.2.2, special case)
 *   - G1, L2-optimal reduction to cubic              (Sec. 5.2.2, eqs.
 *     G1-condition and epsl; normal equations solved with Gauss-Legendre
 *     quadrature instead of the closed-form Gram matrices)
 *   - error-controlled splitting                    (Sec. 5.2.2, "Error-
 *     controlled approximation"; split by de Casteljau)
 *   - projection: the global minimiser of eq. projection over the whole
 *     parameter domain, on the ORIGINAL B-spline, by dense sampling, Newton on
 *     the orthogonality condition (C-q).C' = 0 (eqs. Et and E't) and a
 *     Lipschitz branch-and-bound that re-examines every sample interval whose
 *     lower bound beats the best distance found.
 *
 * Readings of points the paper leaves open:
 *   - the domain is [t_p, t_{n}] of a clamped knot vector; at the right end the
 *     last non-degenerate span is used;
 *   - "L1-error" of a cubic piece is the same-parameter deviation
 *     max_u |Q(u) - R(u)|, accepted when its value on 129 uniform samples plus
 *     a Lipschitz allowance (h/2 * max|Q'-R'|) is <= tol;
 *   - a piece that fails is split at the sample of largest deviation (clamped
 *     to [1/8, 7/8]; samples within 1e-6 relative of the largest count as
 *     tied maxima and the smallest of them is taken) on the ORIGINAL degree-p
 *     piece, and both halves are
 *     reduced again (this makes the split point lie on the original curve,
 *     the effect of the paper's control-polygon modification);
 *   - a zero end tangent leaves its delta at 1 and the other delta is solved
 *     alone.
 *
 * Parity of every function here is pinned by tests that do not reuse this
 * file's formulas (scipy's B-spline and Bernstein evaluators, closed-form
 * projections, polynomial root finding on tiny inputs, printed matrices).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXP 32

/* ------------------------------------------------------------------------ */
/* Knot spans and basis (Sec. 4, eq. bsplinebasis)                          */
/* ------------------------------------------------------------------------ */

/* Index k with U[k] <= t < U[k+1], p <= k <= n-1; the right end of the domain
 * maps to the last non-degenerate span. */
static int or_find_span(int p, int n, const double *U, double t)
{
    if (t >= U[n]) {
        int k = n - 1;
        while (k > p && !(U[k] < U[k + 1])) k--;
        return k;
    }
    if (t <= U[p]) {
        int k = p;
        while (k < n - 1 && !(U[k] < U[k + 1])) k++;
        return k;
    }
    int lo = p, hi = n; /* U[lo] <= t < U[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (t < U[mid]) hi = mid; else lo = mid;
    }
    return lo;
}

/* All basis values N_{i,p}(t), i = 0..n-1, straight from the recursion with
 * half-open support and 0/0 := 0. */
int orc_basis(int p, int n, const double *U, double t, double *N)
{
    int m = n + p + 1; /* number of knots */
    double *w = (double *)calloc((size_t)m, sizeof(double));
    if (!w) return -1;
    int k = or_find_span(p, n, U, t);
    for (int i = 0; i < m - 1; ++i) w[i] = (i == k) ? 1.0 : 0.0;
    for (int d = 1; d <= p; ++d) {
        for (int i = 0; i < m - 1 - d; ++i) {
            double a = 0.0, b = 0.0;
            double den1 = U[i + d] - U[i];
            double den2 = U[i + d + 1] - U[i + 1];
            if (den1 != 0.0) a = (t - U[i]) / den1 * w[i];
            if (den2 != 0.0) b = (U[i + d + 1] - t) / den2 * w[i + 1];
            w[i] = a + b;
        }
    }
    for (int i = 0; i < n; ++i) N[i] = w[i];
    free(w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* de Boor evaluation of C(t) and of the derivative curves                  */
/* ------------------------------------------------------------------------ */

static void or_deboor(int p, int n, const double *P, const double *U, double t, double *out)
{
    if (p == 0) {
        int k = or_find_span(0, n, U, t);
        out[0] = P[3 * k]; out[1] = P[3 * k + 1]; out[2] = P[3 * k + 2];
        return;
    }
    int k = or_find_span(p, n, U, t);
    double d[OR_MAXP + 1][3];
    for (int j = 0; j <= p; ++j)
        for (int c = 0; c < 3; ++c) d[j][c] = P[3 * (j + k - p) + c];
    for (int r = 1; r <= p; ++r) {
        for (int j = p; j >= r; --j) {
            double den = U[j + 1 + k - r] - U[j + k - p];
            double a = den != 0.0 ? (t - U[j + k - p]) / den : 0.0;
            for (int c = 0; c < 3; ++c) d[j][c] = (1.0 - a) * d[j - 1][c] + a * d[j][c];
        }
    }
    out[0] = d[p][0]; out[1] = d[p][1]; out[2] = d[p][2];
}

/* Control net of the derivative curve: degree p-1, n-1 points, knots U[1..]. */
static void or_deriv_net(int p, int n, const double *P, const double *U, double *P1)
{
    for (int i = 0; i < n - 1; ++i) {
        double den = U[i + p + 1] - U[i + 1];
        double s = den != 0.0 ? (double)p / den : 0.0;
        for (int c = 0; c < 3; ++c) P1[3 * i + c] = s * (P[3 * (i + 1) + c] - P[3 * i + c]);
    }
}

typedef struct {
    int p, n;
    const double *P, *U;
    double *P1, *P2; /* derivative nets; knots are U+1 and U+2 */
    int nspan;
    int *span_k;     /* knot index k of each non-degenerate span */
    double *lip;     /* max |C'| bound on each span (derivative control points) */
    double *lip2;    /* max |C''| bound on each span */
    double diag;     /* control-point box diagonal */
} or_curve;

static void or_curve_init(or_curve *c, int p, int n, const double *P, const double *U)
{
    c->p = p; c->n = n; c->P = P; c->U = U;
    c->P1 = (double *)calloc((size_t)3 * (n > 1 ? n : 1), sizeof(double));
    c->P2 = (double *)calloc((size_t)3 * (n > 2 ? n : 1), sizeof(double));
    if (p >= 1) or_deriv_net(p, n, P, U, c->P1);
    if (p >= 2) or_deriv_net(p - 1, n - 1, c->P1, U + 1, c->P2);
    c->span_k = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    c->lip = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    c->lip2 = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    c->nspan = 0;
    for (int k = p; k <= n - 1; ++k) {
        if (!(U[k] < U[k + 1])) continue;
        double L = 0.0;
        /* on span k the derivative is a convex combination of P1[k-p .. k-1] */
        for (int i = k - p; i <= k - 1; ++i) {
            double x = c->P1[3 * i], y = c->P1[3 * i + 1], z = c->P1[3 * i + 2];
            double v = sqrt(x * x + y * y + z * z);
            if (v > L) L = v;
        }
        double L2 = 0.0;
        /* C'' on span k: convex combination of P2[k-p .. k-2] */
        for (int i = k - p; i <= k - 2; ++i) {
            double x = c->P2[3 * i], y = c->P2[3 * i + 1], z = c->P2[3 * i + 2];
            double v = sqrt(x * x + y * y + z * z);
            if (v > L2) L2 = v;
        }
        c->span_k[c->nspan] = k;
        c->lip[c->nspan] = L;
        c->lip2[c->nspan] = L2;
        c->nspan++;
    }
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            if (P[3 * i + k] < lo[k]) lo[k] = P[3 * i + k];
            if (P[3 * i + k] > hi[k]) hi[k] = P[3 * i + k];
        }
    c->diag = sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                   (hi[2] - lo[2]) * (hi[2] - lo[2]));
}

static void or_curve_free(or_curve *c)
{
    free(c->P1); free(c->P2); free(c->span_k); free(c->lip); free(c->lip2);
}

static void or_curve_eval(const or_curve *c, double t, double *X, double *D1, double *D2)
{
    or_deboor(c->p, c->n, c->P, c->U, t, X);
    if (D1) {
        if (c->p >= 1) or_deboor(c->p - 1, c->n - 1, c->P1, c->U + 1, t, D1);
        else D1[0] = D1[1] = D1[2] = 0.0;
    }
    if (D2) {
        if (c->p >= 2) or_deboor(c->p - 2, c->n - 2, c->P2, c->U + 2, t, D2);
        else D2[0] = D2[1] = D2[2] = 0.0;
    }
}

/* de Boor on the polynomial piece of knot span k (U[k] <= t < U[k+1]), also
 * at the span's right end: the one-sided limit from the left at a knot. */
static void or_deboor_k(int p, const double *P, const double *U, int k, double t, double *out)
{
    double d[OR_MAXP + 1][3];
    for (int j = 0; j <= p; ++j)
        for (int c = 0; c < 3; ++c) d[j][c] = P[3 * (j + k - p) + c];
    for (int r = 1; r <= p; ++r)
        for (int j = p; j >= r; --j) {
            double den = U[j + 1 + k - r] - U[j + k - p];
            double a = den != 0.0 ? (t - U[j + k - p]) / den : 0.0;
            for (int c = 0; c < 3; ++c) d[j][c] = (1.0 - a) * d[j - 1][c] + a * d[j][c];
        }
    out[0] = d[p][0]; out[1] = d[p][1]; out[2] = d[p][2];
}

/* C and C' from the piece of span k (the derivative curve's span is k - 1). */
static void or_curve_eval_k(const or_curve *c, int k, double t, double *X, double *D1)
{
    or_deboor_k(c->p, c->P, c->U, k, t, X);
    if (c->p >= 1) or_deboor_k(c->p - 1, c->P1, c->U + 1, k - 1, t, D1);
    else D1[0] = D1[1] = D1[2] = 0.0;
}

/* ... and C'' (the second derivative curve's span is k - 2). */
static void or_curve_eval_k2(const or_curve *c, int k, double t, double *X, double *D1, double *D2)
{
    or_curve_eval_k(c, k, t, X, D1);
    if (c->p >= 2) or_deboor_k(c->p - 2, c->P2, c->U + 2, k - 2, t, D2);
    else D2[0] = D2[1] = D2[2] = 0.0;
}

int orc_eval(int p, int n, const double *P, const double *U, int64_t m, const double *t,
             double *X, double *D1, double *D2)
{
    if (p < 1 || p > OR_MAXP || n < p + 1) return -1;
    or_curve c;
    or_curve_init(&c, p, n, P, U);
    for (int64_t i = 0; i < m; ++i)
        or_curve_eval(&c, t[i], X + 3 * i, D1 ? D1 + 3 * i : NULL, D2 ? D2 + 3 * i : NULL);
    or_curve_free(&c);
    return 0;
}

/* Batched evaluation over a CSR curve set: X[i] = C_{cid[i]}(t[i]). */
int orc_eval_batch(int ncurves, const int32_t *deg, const int64_t *cp_off, const double *cp,
                   const int64_t *k_off, const double *knots, int64_t m, const int32_t *cid,
                   const double *t, double *X)
{
    for (int64_t i = 0; i < m; ++i) {
        int c = cid[i];
        if (c < 0 || c >= ncurves) return -1;
        int n = (int)(cp_off[c + 1] - cp_off[c]);
        or_deboor(deg[c], n, cp + 3 * cp_off[c], knots + k_off[c], t[i], X + 3 * i);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Boehm knot insertion -> one Bezier piece per non-degenerate span         */
/* ------------------------------------------------------------------------ */

/* Writes the (p+1) control points of each span's Bezier form to bz (span
 * major, xyz interleaved) and [t_q, t_{q+1}] to tab.  Returns the number of
 * spans, or a negative value on bad input / too small buffers. */
int orc_bezier_spans(int p, int n, const double *P, const double *U, int max_spans,
                     double *bz, double *tab)
{
    if (p < 1 || p > OR_MAXP || n < p + 1) return -1;
    int m = n + p + 1;
    int cap_pts = n + p * m + 8;
    double *Q = (double *)malloc(sizeof(double) * 3 * (size_t)cap_pts);
    double *Qn = (double *)malloc(sizeof(double) * 3 * (size_t)cap_pts);
    double *K = (double *)malloc(sizeof(double) * (size_t)(cap_pts + p + 2));
    double *Kn = (double *)malloc(sizeof(double) * (size_t)(cap_pts + p + 2));
    memcpy(Q, P, sizeof(double) * 3 * (size_t)n);
    memcpy(K, U, sizeof(double) * (size_t)m);
    int np = n, nk = m;
    /* walk distinct interior knot values */
    int i = p + 1;
    while (i < nk - p - 1) {
        double v = K[i];
        int s = 0;
        while (i + s < nk && K[i + s] == v) s++;
        for (int ins = s; ins < p; ++ins) {
            /* single insertion of v: k = last index with K[k] <= v */
            int k = i;
            while (k + 1 < nk && K[k + 1] <= v) k++;
            for (int j = 0; j <= k - p; ++j)
                for (int c = 0; c < 3; ++c) Qn[3 * j + c] = Q[3 * j + c];
            for (int j = k - p + 1; j <= k; ++j) {
                double den = K[j + p] - K[j];
                double a = den != 0.0 ? (v - K[j]) / den : 0.0;
                for (int c = 0; c < 3; ++c) Qn[3 * j + c] = a * Q[3 * j + c] + (1.0 - a) * Q[3 * (j - 1) + c];
            }
            for (int j = k + 1; j <= np; ++j)
                for (int c = 0; c < 3; ++c) Qn[3 * j + c] = Q[3 * (j - 1) + c];
            for (int j = 0; j <= k; ++j) Kn[j] = K[j];
            Kn[k + 1] = v;
            for (int j = k + 1; j < nk; ++j) Kn[j + 1] = K[j];
            np++; nk++;
            double *tq = Q; Q = Qn; Qn = tq;
            double *tk = K; K = Kn; Kn = tk;
        }
        /* advance past this value (now multiplicity >= p) */
        while (i < nk && K[i] == v) i++;
    }
    int ns = 0;
    for (int k = p; k <= np - 1; ++k) {
        if (!(K[k] < K[k + 1])) continue;
        if (ns >= max_spans) { ns = -2; break; }
        for (int j = 0; j <= p; ++j)
            for (int c = 0; c < 3; ++c) bz[3 * ((size_t)ns * (p + 1) + j) + c] = Q[3 * (k - p + j) + c];
        tab[2 * ns] = K[k];
        tab[2 * ns + 1] = K[k + 1];
        ns++;
    }
    free(Q); free(Qn); free(K); free(Kn);
    return ns;
}

/* ------------------------------------------------------------------------ */
/* Bezier utilities: de Casteljau, elevation                                */
/* ------------------------------------------------------------------------ */

void orc_bez_eval(int p, const double *Q, double u, double *out);
static void or_bez_eval(int p, const double *Q, double u, double *out) { orc_bez_eval(p, Q, u, out); }

/* de Casteljau evaluation of a Bezier piece. */
void orc_bez_eval(int p, const double *Q, double u, double *out)
{
    double w[OR_MAXP + 1][3];
    for (int j = 0; j <= p; ++j)
        for (int c = 0; c < 3; ++c) w[j][c] = Q[3 * j + c];
    for (int r = 1; r <= p; ++r)
        for (int j = 0; j <= p - r; ++j)
            for (int c = 0; c < 3; ++c) w[j][c] = (1.0 - u) * w[j][c] + u * w[j + 1][c];
    out[0] = w[0][0]; out[1] = w[0][1]; out[2] = w[0][2];
}

/* de Casteljau split at z into left and right pieces of the same degree. */
void orc_bez_split(int p, const double *Q, double z, double *L, double *R)
{
    double w[OR_MAXP + 1][3];
    for (int j = 0; j <= p; ++j)
        for (int c = 0; c < 3; ++c) w[j][c] = Q[3 * j + c];
    for (int c = 0; c < 3; ++c) { L[c] = w[0][c]; R[3 * p + c] = w[p][c]; }
    for (int r = 1; r <= p; ++r) {
        for (int j = 0; j <= p - r; ++j)
            for (int c = 0; c < 3; ++c) w[j][c] = (1.0 - z) * w[j][c] + z * w[j + 1][c];
        for (int c = 0; c < 3; ++c) { L[3 * r + c] = w[0][c]; R[3 * (p - r) + c] = w[p - r][c]; }
    }
}

/* Degree elevation by one: Qe_i = i/(p+1) Q_{i-1} + (1 - i/(p+1)) Q_i. */
static void or_bez_elevate(int p, const double *Q, double *Qe)
{
    for (int i = 0; i <= p + 1; ++i) {
        double a = (double)i / (double)(p + 1);
        for (int c = 0; c < 3; ++c) {
            double lo = i > 0 ? Q[3 * (i - 1) + c] : 0.0;
            double hi = i <= p ? Q[3 * i + c] : 0.0;
            Qe[3 * i + c] = a * lo + (1.0 - a) * hi;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* G1-continuous, L2-optimal reduction to cubic (Sec. 5.2.2)                */
/* ------------------------------------------------------------------------ */

/* OR_GL-point Gauss-Legendre nodes on [0,1], computed once by Newton on
 * P_OR_GL: exact for the Gram integrands B_i,3 B_k,p of degree p + 3 <= 2 OR_GL - 1
 * (eq. gram) at every degree up to OR_MAXP. */
#define OR_GL 24
static double or_gl_x[OR_GL], or_gl_w[OR_GL];
static int or_gl_ready = 0;

static void or_gl_init(void)
{
    if (or_gl_ready) return;
    const int N = OR_GL;
    for (int i = 0; i < N; ++i) {
        double x = cos(M_PI * (i + 0.75) / (N + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= N; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            double dp = N * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= N; ++k) {
            double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1; p1 = p2;
        }
        double dp = N * (x * p1 - p0) / (x * x - 1.0);
        or_gl_x[i] = 0.5 * (1.0 - x);
        or_gl_w[i] = 1.0 / ((1.0 - x * x) * dp * dp); /* 0.5 * 2/((1-x^2) P'^2) */
    }
    or_gl_ready = 1;
}

static double or_bern3(int i, double u)
{
    double v = 1.0 - u;
    switch (i) {
    case 0: return v * v * v;
    case 1: return 3.0 * u * v * v;
    case 2: return 3.0 * u * u * v;
    default: return u * u * u;
    }
}

/* R (4 points) from the degree-p piece Q by the G1 conditions
 *   R0 = Q0, R1 = Q0 + (p/3) dQ0 d0, R2 = Qp - (p/3) dQ_{p-1} d1, R3 = Qp,
 * with (d0, d1) minimising the L2 deviation: the 2x2 normal equations are
 * assembled by quadrature (exact for these polynomial degrees). */
int orc_g1_reduce(int p, const double *Q, double *R, double *delta)
{
    if (p < 1 || p > OR_MAXP) return -1;
    if (p <= 3) {
        double A[OR_MAXP + 2][3], B[OR_MAXP + 2][3];
        memcpy(A, Q, sizeof(double) * 3 * (size_t)(p + 1));
        for (int d = p; d < 3; ++d) { or_bez_elevate(d, &A[0][0], &B[0][0]); memcpy(A, B, sizeof(double) * 3 * (size_t)(d + 2)); }
        memcpy(R, A, sizeof(double) * 12);
        if (delta) { delta[0] = 1.0; delta[1] = 1.0; }
        return 0;
    }
    or_gl_init();
    double a[3], b[3];
    for (int c = 0; c < 3; ++c) {
        a[c] = (double)p / 3.0 * (Q[3 * 1 + c] - Q[c]);
        b[c] = (double)p / 3.0 * (Q[3 * p + c] - Q[3 * (p - 1) + c]);
    }
    /* residual with d0 = d1 = 0:  r0(u) = Q(u) - [B0 Q0 + B1 Q0 + B2 Qp + B3 Qp]
     * full residual: r = r0 - d0 B1 a + d1 B2 b. */
    double m11 = 0, m12 = 0, m22 = 0, r1 = 0, r2 = 0;
    for (int g = 0; g < OR_GL; ++g) {
        double u = or_gl_x[g], w = or_gl_w[g];
        double q[3];
        or_bez_eval(p, Q, u, q);
        double b0 = or_bern3(0, u), b1 = or_bern3(1, u), b2 = or_bern3(2, u), b3 = or_bern3(3, u);
        double r0[3];
        for (int c = 0; c < 3; ++c) r0[c] = q[c] - ((b0 + b1) * Q[c] + (b2 + b3) * Q[3 * p + c]);
        double ra = r0[0] * a[0] + r0[1] * a[1] + r0[2] * a[2];
        double rb = r0[0] * b[0] + r0[1] * b[1] + r0[2] * b[2];
        /* d/dd0: -B1 a . r = 0 ; d/dd1: B2 b . r = 0 */
        m11 += w * b1 * b1;
        m12 += w * b1 * b2;
        m22 += w * b2 * b2;
        r1 += w * b1 * ra;
        r2 += w * b2 * rb;
    }
    double aa = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    double bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    /* equations:  m11 aa d0 - m12 ab d1 = r1
     *            -m12 ab d0 + m22 bb d1 = -r2 */
    double d0 = 1.0, d1 = 1.0;
    if (aa > 0.0 && bb > 0.0) {
        double A11 = m11 * aa, A12 = -m12 * ab, A22 = m22 * bb;
        double det = A11 * A22 - A12 * A12;
        d0 = (r1 * A22 - A12 * (-r2)) / det;
        d1 = (A11 * (-r2) - A12 * r1) / det;
    } else if (aa > 0.0) {
        /* d1 irrelevant (b = 0): fixed at 1 */
        d0 = (r1 + m12 * ab * 1.0) / (m11 * aa);
    } else if (bb > 0.0) {
        d1 = (-r2 + m12 * ab * 1.0) / (m22 * bb);
    }
    for (int c = 0; c < 3; ++c) {
        R[c] = Q[c];
        R[3 + c] = Q[c] + a[c] * d0;
        R[6 + c] = Q[3 * p + c] - b[c] * d1;
        R[9 + c] = Q[3 * p + c];
    }
    if (delta) { delta[0] = d0; delta[1] = d1; }
    return 0;
}

/* Acceptance value and split sample of a cubic R against the degree-p piece Q:
 * max over u_i = i/128 of |Q(u_i) - R(u_i)|, plus (1/256) * a bound on
 * max |Q' - R'| from the hodograph of Q - R written at degree p. */
static double or_piece_error(int p, const double *Q, const double *R, int *imax)
{
    double best = -1.0, ev[129];
    int bi = 64;
    for (int i = 0; i <= 128; ++i) {
        double u = (double)i / 128.0, x[3], y[3];
        or_bez_eval(p, Q, u, x);
        or_bez_eval(3, R, u, y);
        ev[i] = sqrt((x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]) + (x[2] - y[2]) * (x[2] - y[2]));
        if (ev[i] > best) best = ev[i];
    }
    /* tied maxima (within 1e-6 relative): the smallest parameter is split */
    for (int i = 0; i <= 128; ++i)
        if (ev[i] >= best * (1.0 - 1e-6)) { bi = i; break; }
    /* elevate R to degree p */
    double A[OR_MAXP + 2][3], B[OR_MAXP + 2][3];
    memcpy(A, R, sizeof(double) * 12);
    for (int d = 3; d < p; ++d) { or_bez_elevate(d, &A[0][0], &B[0][0]); memcpy(A, B, sizeof(double) * 3 * (size_t)(d + 2)); }
    double L = 0.0;
    for (int i = 0; i < p; ++i) {
        double v2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            double dq = (Q[3 * (i + 1) + c] - A[i + 1][c]) - (Q[3 * i + c] - A[i][c]);
            v2 += dq * dq;
        }
        double v = (double)p * sqrt(v2);
        if (v > L) L = v;
    }
    if (imax) *imax = bi;
    return best + L / 256.0;
}

/* Dense check used by the tests: max same-parameter deviation on `ns`
 * uniform samples. */
double orc_piece_deviation(int p, const double *Q, const double *R, int ns)
{
    double best = 0.0;
    for (int i = 0; i < ns; ++i) {
        double u = (double)i / (double)(ns - 1), x[3], y[3];
        or_bez_eval(p, Q, u, x);
        or_bez_eval(3, R, u, y);
        double e = sqrt((x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]) + (x[2] - y[2]) * (x[2] - y[2]));
        if (e > best) best = e;
    }
    return best;
}

typedef struct {
    double *R;   /* 12 per piece */
    double *tab; /* ta, tb */
    int *span;
    int n, cap;
} or_pieces;

static int or_push(or_pieces *o, const double *R, double ta, double tb, int span)
{
    if (o->n == o->cap) {
        int nc = o->cap ? 2 * o->cap : 64;
        o->R = (double *)realloc(o->R, sizeof(double) * 12 * (size_t)nc);
        o->tab = (double *)realloc(o->tab, sizeof(double) * 2 * (size_t)nc);
        o->span = (int *)realloc(o->span, sizeof(int) * (size_t)nc);
        o->cap = nc;
    }
    memcpy(o->R + 12 * (size_t)o->n, R, sizeof(double) * 12);
    o->tab[2 * o->n] = ta;
    o->tab[2 * o->n + 1] = tb;
    o->span[o->n] = span;
    o->n++;
    return 0;
}

#define OR_PIECE_CAP 4096

static int or_reduce_rec(int p, const double *Q, double ta, double tb, double tol, int span,
                         or_pieces *o, int *budget)
{
    double R[12];
    orc_g1_reduce(p, Q, R, NULL);
    if (p <= 3) { or_push(o, R, ta, tb, span); return 0; }
    int imax = 64;
    double e = or_piece_error(p, Q, R, &imax);
    if (e <= tol) { or_push(o, R, ta, tb, span); return 0; }
    if (--(*budget) <= 0) return -3;
    int iz = imax < 16 ? 16 : (imax > 112 ? 112 : imax);
    double z = (double)iz / 128.0;
    double L[3 * (OR_MAXP + 1)], Rr[3 * (OR_MAXP + 1)];
    orc_bez_split(p, Q, z, L, Rr);
    double tm = ta + z * (tb - ta);
    int rc = or_reduce_rec(p, L, ta, tm, tol, span, o, budget);
    if (rc) return rc;
    return or_reduce_rec(p, Rr, tm, tb, tol, span, o, budget);
}

static int or_decompose_one(int p, int n, const double *P, const double *U, double tol, or_pieces *o)
{
    int maxs = n;
    double *bz = (double *)malloc(sizeof(double) * 3 * (size_t)(p + 1) * (size_t)maxs);
    double *tab = (double *)malloc(sizeof(double) * 2 * (size_t)maxs);
    int ns = orc_bezier_spans(p, n, P, U, maxs, bz, tab);
    int rc = 0;
    if (ns < 0) rc = -1;
    for (int s = 0; s < ns && rc == 0; ++s) {
        int budget = OR_PIECE_CAP;
        rc = or_reduce_rec(p, bz + 3 * (size_t)s * (p + 1), tab[2 * s], tab[2 * s + 1], tol, s, o, &budget);
    }
    free(bz); free(tab);
    return rc;
}

/* Batched decomposition.  tol_abs[c] is the absolute tolerance of curve c.
 * Returns an opaque handle (NULL on failure); counts via orc_dec_counts. */
typedef struct { int ncurves; or_pieces *pc; int rc; } or_dec;

void *orc_decompose_batch(int ncurves, const int32_t *deg, const int64_t *cp_off, const double *cp,
                          const int64_t *k_off, const double *knots, const double *tol_abs, int nthreads)
{
    or_dec *h = (or_dec *)calloc(1, sizeof(or_dec));
    h->ncurves = ncurves;
    h->pc = (or_pieces *)calloc((size_t)(ncurves > 0 ? ncurves : 1), sizeof(or_pieces));
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
#endif
    for (int c = 0; c < ncurves; ++c) {
        int n = (int)(cp_off[c + 1] - cp_off[c]);
        int rc = or_decompose_one(deg[c], n, cp + 3 * cp_off[c], knots + k_off[c], tol_abs[c], &h->pc[c]);
        if (rc) bad |= 1;
    }
    h->rc = bad ? -1 : 0;
    return h;
}

int orc_dec_status(void *hv) { return ((or_dec *)hv)->rc; }

int64_t orc_dec_counts(void *hv, int64_t *counts)
{
    or_dec *h = (or_dec *)hv;
    int64_t tot = 0;
    for (int c = 0; c < h->ncurves; ++c) { if (counts) counts[c] = h->pc[c].n; tot += h->pc[c].n; }
    return tot;
}

void orc_dec_fetch(void *hv, double *R, double *tab, int32_t *span)
{
    or_dec *h = (or_dec *)hv;
    size_t off = 0;
    for (int c = 0; c < h->ncurves; ++c) {
        or_pieces *o = &h->pc[c];
        memcpy(R + 12 * off, o->R, sizeof(double) * 12 * (size_t)o->n);
        memcpy(tab + 2 * off, o->tab, sizeof(double) * 2 * (size_t)o->n);
        for (int i = 0; i < o->n; ++i) span[off + i] = o->span[i];
        off += (size_t)o->n;
    }
}

void orc_dec_free(void *hv)
{
    or_dec *h = (or_dec *)hv;
    for (int c = 0; c < h->ncurves; ++c) { free(h->pc[c].R); free(h->pc[c].tab); free(h->pc[c].span); }
    free(h->pc);
    free(h);
}

/* ------------------------------------------------------------------------ */
/* Projection on the original B-spline (Sec. 4, eq. projection)             */
/* ------------------------------------------------------------------------ */

#define OR_NS 64      /* samples per span, ends included */
/* Local minima within this distance of the best one (relative to the box
 * diagonal) are searched for with the same certified branch and bound, so that
 * the runner-up is exact whenever it matters to the uniqueness test (2e-6). */
#define OR_RUNNER_MARGIN 4e-6
#define OR_MAXMIN 256 /* recorded local minima per query */

typedef struct {
    double t, d;
    int interior; /* converged to a stationary point inside the bracket */
} or_min;

typedef struct {
    const or_curve *c;
    const double *q;
    double best_d, best_t;
    int best_span;
    double margin; /* intervals whose bound is within this of the best are searched too (runner-up) */
    or_min mins[OR_MAXMIN];
    int nmin;
} or_query;

static double or_dist(const or_curve *c, const double *q, double t)
{
    double x[3];
    or_deboor(c->p, c->n, c->P, c->U, t, x);
    double dx = x[0] - q[0], dy = x[1] - q[1], dz = x[2] - q[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* f(t) = (C - q).C' and f'(t) = |C'|^2 + (C - q).C''  (eqs. Et and E't, halved)
 * on the polynomial piece of span s (index into span_k), ends included: at a
 * knot where the curve is only C0 (or C1), f jumps, and each span's search
 * needs its own one-sided values there (Sec. 5.3, Properties 1-2). */
static void or_orth(const or_curve *c, int s, const double *q, double t, double *f, double *fp, double *dist)
{
    double X[3], D1[3], D2[3];
    or_curve_eval_k2(c, c->span_k[s], t, X, D1, D2);
    double r[3] = {X[0] - q[0], X[1] - q[1], X[2] - q[2]};
    *f = r[0] * D1[0] + r[1] * D1[1] + r[2] * D1[2];
    *fp = D1[0] * D1[0] + D1[1] * D1[1] + D1[2] * D1[2] + r[0] * D2[0] + r[1] * D2[1] + r[2] * D2[2];
    *dist = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
}

static void or_record(or_query *Q, double t, double d, int interior, int span)
{
    if (Q->nmin < OR_MAXMIN) {
        Q->mins[Q->nmin].t = t;
        Q->mins[Q->nmin].d = d;
        Q->mins[Q->nmin].interior = interior;
        Q->nmin++;
    }
    if (d < Q->best_d || (d == Q->best_d && t < Q->best_t)) {
        Q->best_d = d; Q->best_t = t; Q->best_span = span;
    }
}

/* Minimum of |C - q| on [a, b] started from t0: Newton on f with bisection
 * safeguard when f changes sign on the bracket; else damped Newton clamped to
 * the bracket.  The bracket ends are always candidates. */
static void or_local_min(or_query *Q, int span, double a, double b, double t0)
{
    const or_curve *c = Q->c;
    const double *q = Q->q;
    double fa, fpa, da, fb, fpb, db;
    or_orth(c, span, q, a, &fa, &fpa, &da);
    or_orth(c, span, q, b, &fb, &fpb, &db);
    or_record(Q, a, da, 0, span);
    or_record(Q, b, db, 0, span);
    if (fa < 0.0 && fb > 0.0) {
        double lo = a, hi = b, t = t0;
        if (!(t > lo && t < hi)) t = 0.5 * (lo + hi);
        double f, fp, d;
        for (int it = 0; it < 100; ++it) {
            or_orth(c, span, q, t, &f, &fp, &d);
            if (f < 0.0) lo = t; else if (f > 0.0) hi = t; else break;
            double tn = (fp > 0.0) ? t - f / fp : 0.5 * (lo + hi);
            if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
            if (fabs(tn - t) <= 1e-15 * (fabs(t) + 1e-300) || hi - lo <= 4e-16 * (fabs(t) + 1e-300)) { t = tn; break; }
            t = tn;
        }
        or_orth(c, span, q, t, &f, &fp, &d);
        or_record(Q, t, d, 1, span);
        return;
    }
    /* no sign change: try a clamped Newton from t0 */
    double t = t0 < a ? a : (t0 > b ? b : t0);
    for (int it = 0; it < 60; ++it) {
        double f, fp, d;
        or_orth(c, span, q, t, &f, &fp, &d);
        if (!(fp > 0.0)) break;
        double tn = t - f / fp;
        if (tn < a) tn = a;
        if (tn > b) tn = b;
        if (fabs(tn - t) <= 1e-15 * (fabs(t) + 1e-300)) { t = tn; break; }
        t = tn;
    }
    double f, fp, d;
    or_orth(c, span, q, t, &f, &fp, &d);
    /* interior only when the end point is a stationary minimum within rounding */
    double X[3], D1[3];
    or_curve_eval_k(c, c->span_k[span], t, X, D1);
    double sp = sqrt(D1[0] * D1[0] + D1[1] * D1[1] + D1[2] * D1[2]);
    int stat = fabs(f) <= 1e-9 * sp * (d + c->diag) && fp > 0.0;
    or_record(Q, t, d, (t > a && t < b) && stat, span);
}

static int or_contains_min(const or_query *Q, double a, double b)
{
    for (int i = 0; i < Q->nmin; ++i)
        if (Q->mins[i].interior && Q->mins[i].t >= a && Q->mins[i].t <= b) return 1;
    return 0;
}

/* Re-examine [a,b] while it could hide a distance below the best one.  It is
 * dropped when (i) its Lipschitz lower bound 0.5(da+db) - 0.5 L1 (b-a) is not
 * below the best distance, (ii) it holds a refined stationary minimum, or
 * (iii) f = (C-q).C' provably keeps one sign on it (|f'| <= F), so that the
 * distance is monotone there and its minimum is an end, i.e. a sample already
 * seen.  Otherwise it is cut in four and Newton runs from every new local
 * minimum of the distance and every sign change of f. */
static void or_bb(or_query *Q, int span, double L1, double L2, double a, double da, double b, double db,
                  int depth)
{
    double w = b - a;
    double lb = 0.5 * (da + db) - 0.5 * L1 * w;
    if (lb >= Q->best_d + Q->margin) return;
    if (or_contains_min(Q, a, b)) return;
    double fa, fpa, fb, fpb, dd;
    or_orth(Q->c, span, Q->q, a, &fa, &fpa, &dd);
    or_orth(Q->c, span, Q->q, b, &fb, &fpb, &dd);
    double F = L1 * L1 + ((da > db ? da : db) + L1 * w) * L2;
    if (fa > F * w || fb < -F * w) return;
    if (depth >= 14) { or_local_min(Q, span, a, b, 0.5 * (a + b)); return; }
    double t[5], d[5], f[5];
    t[0] = a; d[0] = da; f[0] = fa; t[4] = b; d[4] = db; f[4] = fb;
    for (int i = 1; i < 4; ++i) {
        double fp;
        t[i] = a + w * (double)i / 4.0;
        or_orth(Q->c, span, Q->q, t[i], &f[i], &fp, &d[i]);
    }
    for (int i = 1; i < 4; ++i)
        if (d[i] <= d[i - 1] && d[i] <= d[i + 1]) or_local_min(Q, span, t[i - 1], t[i + 1], t[i]);
    for (int i = 0; i < 4; ++i)
        if (f[i] < 0.0 && f[i + 1] > 0.0) or_local_min(Q, span, t[i], t[i + 1], 0.5 * (t[i] + t[i + 1]));
    for (int i = 0; i < 4; ++i) or_bb(Q, span, L1, L2, t[i], d[i], t[i + 1], d[i + 1], depth + 1);
}

static void or_project_one(const or_curve *c, const double *q, double *t_out, double *d_out, int *span_out,
                           double *kappa_out, double *runner_out)
{
    or_query Q;
    Q.c = c; Q.q = q; Q.best_d = INFINITY; Q.best_t = 0.0; Q.best_span = 0; Q.nmin = 0;
    Q.margin = OR_RUNNER_MARGIN * c->diag;
    double ts[OR_NS], ds[OR_NS];
    double *allt = (double *)malloc(sizeof(double) * (size_t)c->nspan * OR_NS);
    double *alld = (double *)malloc(sizeof(double) * (size_t)c->nspan * OR_NS);
    for (int s = 0; s < c->nspan; ++s) {
        int k = c->span_k[s];
        double a = c->U[k], b = c->U[k + 1];
        for (int i = 0; i < OR_NS; ++i) {
            ts[i] = (i == OR_NS - 1) ? b : a + (b - a) * (double)i / (double)(OR_NS - 1);
            ds[i] = or_dist(c, q, ts[i]);
        }
        for (int i = 0; i < OR_NS; ++i) {
            int lm = (i == 0 || ds[i] <= ds[i - 1]) && (i == OR_NS - 1 || ds[i] <= ds[i + 1]);
            if (!lm) continue;
            double lo = ts[i > 0 ? i - 1 : 0], hi = ts[i < OR_NS - 1 ? i + 1 : OR_NS - 1];
            or_local_min(&Q, s, lo, hi, ts[i]);
        }
        memcpy(allt + (size_t)s * OR_NS, ts, sizeof(ts));
        memcpy(alld + (size_t)s * OR_NS, ds, sizeof(ds));
    }
    /* certification pass over every sample interval */
    for (int s = 0; s < c->nspan; ++s) {
        const double *ts2 = allt + (size_t)s * OR_NS, *ds2 = alld + (size_t)s * OR_NS;
        for (int i = 0; i < OR_NS - 1; ++i)
            or_bb(&Q, s, c->lip[s], c->lip2[s], ts2[i], ds2[i], ts2[i + 1], ds2[i + 1], 0);
    }
    free(allt); free(alld);
    /* conditioning at the minimiser and the best distinct local minimum */
    double f, fp, d, X[3], D1[3], D2[3];
    or_orth(c, Q.best_span, q, Q.best_t, &f, &fp, &d);
    or_curve_eval_k2(c, c->span_k[Q.best_span], Q.best_t, X, D1, D2);
    double sp2 = D1[0] * D1[0] + D1[1] * D1[1] + D1[2] * D1[2];
    double kappa = 1.0;
    double tol_f = 1e-9 * (sqrt(sp2) * (d + c->diag) + 1e-300);
    if (fabs(f) <= tol_f && sp2 > 0.0) kappa = fp / sp2; /* stationary point */
    double runner = INFINITY;
    for (int i = 0; i < Q.nmin; ++i) {
        if (fabs(Q.mins[i].t - Q.best_t) <= 1e-6) continue;
        /* distinct local minima: interior stationary points */
        if (Q.mins[i].d < runner && Q.mins[i].interior) runner = Q.mins[i].d;
    }
    /* ... the interior knots where the curve is only C0 and the distance falls
     * on the left of the joint and rises on its right (a corner minimum, with
     * no stationary point: both one-sided derivatives of |C - q|^2 are used) */
    for (int s = 1; s < c->nspan; ++s) {
        const int kl = c->span_k[s - 1], kr = c->span_k[s];
        const double tj = c->U[kr];
        double XL[3], DL[3], XR[3], DR[3];
        or_curve_eval_k(c, kl, tj, XL, DL);
        or_curve_eval_k(c, kr, tj, XR, DR);
        const double fl = (XL[0] - q[0]) * DL[0] + (XL[1] - q[1]) * DL[1] + (XL[2] - q[2]) * DL[2];
        const double fr = (XR[0] - q[0]) * DR[0] + (XR[1] - q[1]) * DR[1] + (XR[2] - q[2]) * DR[2];
        if (fl < 0.0 && fr > 0.0 && fabs(tj - Q.best_t) > 1e-6) {
            const double dj = sqrt((XR[0] - q[0]) * (XR[0] - q[0]) + (XR[1] - q[1]) * (XR[1] - q[1]) +
                                   (XR[2] - q[2]) * (XR[2] - q[2]));
            if (dj < runner) runner = dj;
        }
    }
    /* ... and the domain ends when the distance grows into the domain there */
    {
        double t0 = c->U[c->p], t1 = c->U[c->n];
        double f0, fp0, d0, f1, fp1, d1;
        or_orth(c, 0, q, t0, &f0, &fp0, &d0);
        or_orth(c, c->nspan - 1, q, t1, &f1, &fp1, &d1);
        if (f0 >= 0.0 && fabs(t0 - Q.best_t) > 1e-6 && d0 < runner) runner = d0;
        if (f1 <= 0.0 && fabs(t1 - Q.best_t) > 1e-6 && d1 < runner) runner = d1;
    }
    *t_out = Q.best_t;
    *d_out = Q.best_d;
    *span_out = Q.best_span;
    *kappa_out = kappa;
    *runner_out = runner;
}

/* Batched projection: each query onto its own curve.  Returns 0 or -1. */
int orc_project_batch(int ncurves, const int32_t *deg, const int64_t *cp_off, const double *cp,
                      const int64_t *k_off, const double *knots, int64_t nq, const int32_t *cid,
                      const double *q, double *t_out, double *d_out, int32_t *span_out, double *kappa_out,
                      double *runner_out, int nthreads)
{
    or_curve *cs = (or_curve *)calloc((size_t)(ncurves > 0 ? ncurves : 1), sizeof(or_curve));
    for (int c = 0; c < ncurves; ++c) {
        int n = (int)(cp_off[c + 1] - cp_off[c]);
        if (deg[c] < 1 || deg[c] > OR_MAXP || n < deg[c] + 1) { free(cs); return -1; }
        or_curve_init(&cs[c], deg[c], n, cp + 3 * cp_off[c], knots + k_off[c]);
    }
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
#endif
    for (int64_t i = 0; i < nq; ++i) {
        int c = cid[i];
        if (c < 0 || c >= ncurves) { bad |= 1; continue; }
        int sp;
        or_project_one(&cs[c], q + 3 * i, &t_out[i], &d_out[i], &sp, &kappa_out[i], &runner_out[i]);
        span_out[i] = sp;
    }
    for (int c = 0; c < ncurves; ++c) or_curve_free(&cs[c]);
    free(cs);
    return bad ? -1 : 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
