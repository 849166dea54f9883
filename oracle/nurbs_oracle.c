/*
 * nurbs_oracle.c -- slow, plain FP64 CPU oracle for point projection onto
 * RATIONAL B-spline (NURBS) curves.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite uses it.  It shares no code, header,
 * table or constant with the library.
 *
 * The paper's method is stated for non-rational B-splines (Sec. 6, discussion
 * and limitations; Sec. 7: NURBS are named as future work).  A rational curve
 * is C(t) = sum_i N_i,p(t) w_i P_i / sum_i N_i,p(t) w_i with weights w_i > 0
 * (the Cox-de Boor basis of Sec. 4, eq. bsplinebasis); this file computes the
 * plain definition of the projection (Sec. 4, eq. projections: the global
 * minimiser over the whole parameter domain) on that curve:
 *   - evaluation: de Boor's algorithm on the homogeneous points (w_i P_i, w_i)
 *     and on their derivative nets, then the quotient rule
 *       C = X / W,  C' = (X' - C W') / W,  C'' = (X'' - 2 C' W' - C W'') / W;
 *   - projection: 64 samples per span, safeguarded Newton on the orthogonality
 *     condition f = (C - q).C' = 0 (f' = |C'|^2 + (C - q).C'') from every sampled
 *     local minimum, and a branch and bound over every sample interval, as for
 *     polynomial curves, with bounds valid for positive weights on a span
 *     (D the diameter of its p + 1 control points, C inside their hull, H1 and
 *     H2 the derivative nets of the homogeneous points with scalings s1, s2):
 *       C'  = sum N_{i,p-1} (H1_i,xyz - C H1_i,w) / W,
 *             |C'|  <= L1 = 2 s1 w_max D / w_min;
 *       C'' = (sum N_{i,p-2} (H2_i,xyz - C H2_i,w) - 2 C' W') / W,
 *             |C''| <= L2 = (4 s1 s2 w_max D + 2 L1 max|H1_i,w|) / w_min;
 *   - the runner-up local minimum and kappa = f'/|C'|^2 at a stationary
 *     minimiser, with the same meaning as for polynomial curves.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ON_MAXP 32
#define ON_NS 64           /* samples per span, ends included */
#define ON_RUNNER_MARGIN 4e-6
#define ON_MAXMIN 256

/* k with U[k] <= t < U[k+1], p <= k <= n-1; the right end uses the last non-degenerate span */
static int on_find_span(int p, int n, const double *U, double t)
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
    int lo = p, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (t < U[mid]) hi = mid; else lo = mid;
    }
    return lo;
}

/* de Boor on span k of a degree-p net of 4D points (also at the span's right end) */
static void on_deboor4(int p, const double *H, const double *U, int k, double t, double *out)
{
    double d[ON_MAXP + 1][4];
    for (int j = 0; j <= p; ++j)
        for (int c = 0; c < 4; ++c) d[j][c] = H[4 * (j + k - p) + c];
    for (int r = 1; r <= p; ++r)
        for (int j = p; j >= r; --j) {
            double den = U[j + 1 + k - r] - U[j + k - p];
            double a = den != 0.0 ? (t - U[j + k - p]) / den : 0.0;
            for (int c = 0; c < 4; ++c) d[j][c] = (1.0 - a) * d[j - 1][c] + a * d[j][c];
        }
    for (int c = 0; c < 4; ++c) out[c] = d[p][c];
}

/* derivative net of a degree-p net of n 4D points: degree p-1, n-1 points, knots U+1 */
static void on_deriv_net(int p, int n, const double *H, const double *U, double *H1)
{
    for (int i = 0; i < n - 1; ++i) {
        double den = U[i + p + 1] - U[i + 1];
        double s = den != 0.0 ? (double)p / den : 0.0;
        for (int c = 0; c < 4; ++c) H1[4 * i + c] = s * (H[4 * (i + 1) + c] - H[4 * i + c]);
    }
}

typedef struct {
    int p, n;
    const double *P, *w, *U;
    double *H, *H1, *H2; /* homogeneous net and its derivative nets */
    int nspan;
    int *span_k;
    double *lip;  /* |C'| bound on each span */
    double *lip2; /* |C''| bound on each span */
    double diag;
} on_curve;

static void on_curve_init(on_curve *c, int p, int n, const double *P, const double *w, const double *U)
{
    c->p = p; c->n = n; c->P = P; c->w = w; c->U = U;
    c->H = (double *)calloc((size_t)4 * n, sizeof(double));
    c->H1 = (double *)calloc((size_t)4 * (n > 1 ? n : 1), sizeof(double));
    c->H2 = (double *)calloc((size_t)4 * (n > 2 ? n : 1), sizeof(double));
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < 3; ++k) c->H[4 * i + k] = w[i] * P[3 * i + k];
        c->H[4 * i + 3] = w[i];
    }
    if (p >= 1) on_deriv_net(p, n, c->H, U, c->H1);
    if (p >= 2) on_deriv_net(p - 1, n - 1, c->H1, U + 1, c->H2);
    c->span_k = (int *)malloc(sizeof(int) * (size_t)n);
    c->lip = (double *)malloc(sizeof(double) * (size_t)n);
    c->lip2 = (double *)malloc(sizeof(double) * (size_t)n);
    c->nspan = 0;
    for (int k = p; k <= n - 1; ++k) {
        if (!(U[k] < U[k + 1])) continue;
        double wmin = INFINITY, wmax = 0.0, D = 0.0, s1 = 0.0, s2 = 0.0, w1 = 0.0;
        for (int i = k - p; i <= k; ++i) {
            if (w[i] < wmin) wmin = w[i];
            if (w[i] > wmax) wmax = w[i];
            for (int j = k - p; j < i; ++j) {
                double dx = P[3 * i] - P[3 * j], dy = P[3 * i + 1] - P[3 * j + 1], dz = P[3 * i + 2] - P[3 * j + 2];
                double dd = sqrt(dx * dx + dy * dy + dz * dz);
                if (dd > D) D = dd;
            }
        }
        /* first derivative net on span k: H1_i, i = k-p .. k-1, scaling p / (U[i+p+1] - U[i+1]) */
        for (int i = k - p; i <= k - 1; ++i) {
            double den = U[i + p + 1] - U[i + 1];
            if (den > 0.0 && (double)p / den > s1) s1 = (double)p / den;
            if (fabs(c->H1[4 * i + 3]) > w1) w1 = fabs(c->H1[4 * i + 3]);
        }
        /* second derivative net: H2_i, i = k-p .. k-2, scaling (p-1) / (U[i+p+1] - U[i+2]) */
        for (int i = k - p; i <= k - 2; ++i) {
            double den = U[i + p + 1] - U[i + 2];
            if (den > 0.0 && (double)(p - 1) / den > s2) s2 = (double)(p - 1) / den;
        }
        double L1 = 2.0 * s1 * wmax * D / wmin;
        c->span_k[c->nspan] = k;
        c->lip[c->nspan] = L1;
        c->lip2[c->nspan] = (4.0 * s1 * s2 * wmax * D + 2.0 * L1 * w1) / wmin;
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

static void on_curve_free(on_curve *c)
{
    free(c->H); free(c->H1); free(c->H2); free(c->span_k); free(c->lip); free(c->lip2);
}

/* C, C', C'' at t on the piece of span k (the quotient rule on the homogeneous values) */
static void on_eval_k(const on_curve *c, int k, double t, double *X, double *D1, double *D2)
{
    const int p = c->p;
    double A[4], A1[4] = {0, 0, 0, 0}, A2[4] = {0, 0, 0, 0};
    on_deboor4(p, c->H, c->U, k, t, A);
    if (p >= 1) on_deboor4(p - 1, c->H1, c->U + 1, k - 1, t, A1);
    if (p >= 2) on_deboor4(p - 2, c->H2, c->U + 2, k - 2, t, A2);
    const double W = A[3], W1 = A1[3], W2 = A2[3];
    double C[3], C1[3];
    for (int i = 0; i < 3; ++i) C[i] = A[i] / W;
    for (int i = 0; i < 3; ++i) C1[i] = (A1[i] - C[i] * W1) / W;
    for (int i = 0; i < 3; ++i) {
        X[i] = C[i];
        if (D1) D1[i] = C1[i];
        if (D2) D2[i] = (A2[i] - 2.0 * C1[i] * W1 - C[i] * W2) / W;
    }
}

static void on_eval(const on_curve *c, double t, double *X, double *D1, double *D2)
{
    on_eval_k(c, on_find_span(c->p, c->n, c->U, t), t, X, D1, D2);
}

static double on_dist(const on_curve *c, const double *q, int k, double t)
{
    double X[3];
    on_eval_k(c, k, t, X, NULL, NULL);
    double dx = X[0] - q[0], dy = X[1] - q[1], dz = X[2] - q[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* f = (C - q).C', f' = |C'|^2 + (C - q).C'', distance */
static void on_orth(const on_curve *c, const double *q, int k, double t, double *f, double *fp, double *d)
{
    double X[3], D1[3], D2[3];
    on_eval_k(c, k, t, X, D1, D2);
    double r[3] = {X[0] - q[0], X[1] - q[1], X[2] - q[2]};
    *f = r[0] * D1[0] + r[1] * D1[1] + r[2] * D1[2];
    *fp = D1[0] * D1[0] + D1[1] * D1[1] + D1[2] * D1[2] + r[0] * D2[0] + r[1] * D2[1] + r[2] * D2[2];
    *d = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
}

typedef struct {
    double t, d;
    int interior; /* a stationary point strictly inside its bracket */
} on_min;

typedef struct {
    const on_curve *c;
    const double *q;
    double best_d, best_t;
    double margin;
    int nmin;
    on_min mins[ON_MAXMIN];
} on_query;

static void on_record(on_query *Q, double t, double d, int interior)
{
    if (Q->nmin < ON_MAXMIN) {
        Q->mins[Q->nmin].t = t; Q->mins[Q->nmin].d = d; Q->mins[Q->nmin].interior = interior;
        Q->nmin++;
    }
    if (d < Q->best_d || (d == Q->best_d && t < Q->best_t)) { Q->best_d = d; Q->best_t = t; }
}

/* Minimum of the distance on [a, b] (inside span k) from t0: safeguarded Newton on f when f changes sign
 * from - to + on the bracket, else Newton clamped to the bracket; the bracket ends are candidates. */
static void on_local_min(on_query *Q, int k, double a, double b, double t0)
{
    const on_curve *c = Q->c;
    const double *q = Q->q;
    double fa, fpa, da, fb, fpb, db;
    on_orth(c, q, k, a, &fa, &fpa, &da);
    on_orth(c, q, k, b, &fb, &fpb, &db);
    on_record(Q, a, da, 0);
    on_record(Q, b, db, 0);
    if (fa < 0.0 && fb > 0.0) {
        double lo = a, hi = b, t = t0, f, fp, d;
        if (!(t > lo && t < hi)) t = 0.5 * (lo + hi);
        for (int it = 0; it < 100; ++it) {
            on_orth(c, q, k, t, &f, &fp, &d);
            if (f < 0.0) lo = t; else if (f > 0.0) hi = t; else break;
            double tn = (fp > 0.0) ? t - f / fp : 0.5 * (lo + hi);
            if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
            if (fabs(tn - t) <= 1e-15 * (fabs(t) + 1e-300) || hi - lo <= 4e-16 * (fabs(t) + 1e-300)) { t = tn; break; }
            t = tn;
        }
        on_orth(c, q, k, t, &f, &fp, &d);
        on_record(Q, t, d, 1);
        return;
    }
    double t = t0 < a ? a : (t0 > b ? b : t0), f, fp, d;
    for (int it = 0; it < 60; ++it) {
        on_orth(c, q, k, t, &f, &fp, &d);
        if (!(fp > 0.0)) break;
        double tn = t - f / fp;
        if (tn < a) tn = a;
        if (tn > b) tn = b;
        if (fabs(tn - t) <= 1e-15 * (fabs(t) + 1e-300)) { t = tn; break; }
        t = tn;
    }
    on_orth(c, q, k, t, &f, &fp, &d);
    double X[3], D1[3];
    on_eval_k(c, k, t, X, D1, NULL);
    double sp = sqrt(D1[0] * D1[0] + D1[1] * D1[1] + D1[2] * D1[2]);
    int stat = fabs(f) <= 1e-9 * sp * (d + c->diag) && fp > 0.0;
    on_record(Q, t, d, (t > a && t < b) && stat);
}

static int on_contains_min(const on_query *Q, double a, double b)
{
    for (int i = 0; i < Q->nmin; ++i)
        if (Q->mins[i].interior && Q->mins[i].t >= a && Q->mins[i].t <= b) return 1;
    return 0;
}

/* Re-examine [a, b] of span s while it could hide a distance below the best (plus the runner-up margin):
 * dropped when its Lipschitz lower bound is not below it, when it holds a refined stationary minimum, or
 * when f provably keeps one sign on it (|f'| <= L1^2 + d_max L2), so that its minimum is an end;
 * otherwise cut in four with Newton from every new sampled local minimum and sign change of f. */
static void on_bb(on_query *Q, int s, double a, double da, double b, double db, int depth)
{
    const on_curve *c = Q->c;
    const int k = c->span_k[s];
    const double L1 = c->lip[s], L2 = c->lip2[s];
    double w = b - a;
    double lb = 0.5 * (da + db) - 0.5 * L1 * w;
    if (lb >= Q->best_d + Q->margin) return;
    if (on_contains_min(Q, a, b)) return;
    double fa, fpa, fb, fpb, dd;
    on_orth(c, Q->q, k, a, &fa, &fpa, &dd);
    on_orth(c, Q->q, k, b, &fb, &fpb, &dd);
    double F = L1 * L1 + ((da > db ? da : db) + L1 * w) * L2;
    if (fa > F * w || fb < -F * w) return;
    if (depth >= 14) { on_local_min(Q, k, a, b, 0.5 * (a + b)); return; }
    double t[5], d[5], f[5];
    t[0] = a; d[0] = da; f[0] = fa; t[4] = b; d[4] = db; f[4] = fb;
    for (int i = 1; i < 4; ++i) {
        double fp;
        t[i] = a + w * (double)i / 4.0;
        on_orth(c, Q->q, k, t[i], &f[i], &fp, &d[i]);
    }
    for (int i = 1; i < 4; ++i)
        if (d[i] <= d[i - 1] && d[i] <= d[i + 1]) on_local_min(Q, k, t[i - 1], t[i + 1], t[i]);
    for (int i = 0; i < 4; ++i)
        if (f[i] < 0.0 && f[i + 1] > 0.0) on_local_min(Q, k, t[i], t[i + 1], 0.5 * (t[i] + t[i + 1]));
    for (int i = 0; i < 4; ++i) on_bb(Q, s, t[i], d[i], t[i + 1], d[i + 1], depth + 1);
}

static void on_project_one(const on_curve *c, const double *q, double *t_out, double *d_out, double *kappa_out,
                           double *runner_out)
{
    on_query Q;
    Q.c = c; Q.q = q; Q.best_d = INFINITY; Q.best_t = 0.0; Q.nmin = 0;
    Q.margin = ON_RUNNER_MARGIN * c->diag;
    double *ts = (double *)malloc(sizeof(double) * (size_t)c->nspan * ON_NS);
    double *ds = (double *)malloc(sizeof(double) * (size_t)c->nspan * ON_NS);
    for (int s = 0; s < c->nspan; ++s) {
        int k = c->span_k[s];
        double a = c->U[k], b = c->U[k + 1];
        double *T = ts + (size_t)s * ON_NS, *D = ds + (size_t)s * ON_NS;
        for (int i = 0; i < ON_NS; ++i) {
            T[i] = (i == ON_NS - 1) ? b : a + (b - a) * (double)i / (double)(ON_NS - 1);
            D[i] = on_dist(c, q, k, T[i]);
        }
        for (int i = 0; i < ON_NS; ++i) {
            int lm = (i == 0 || D[i] <= D[i - 1]) && (i == ON_NS - 1 || D[i] <= D[i + 1]);
            if (lm) on_local_min(&Q, k, T[i > 0 ? i - 1 : 0], T[i < ON_NS - 1 ? i + 1 : ON_NS - 1], T[i]);
        }
    }
    for (int s = 0; s < c->nspan; ++s) {
        const double *T = ts + (size_t)s * ON_NS, *D = ds + (size_t)s * ON_NS;
        for (int i = 0; i < ON_NS - 1; ++i) on_bb(&Q, s, T[i], D[i], T[i + 1], D[i + 1], 0);
    }
    free(ts); free(ds);
    /* kappa at a stationary minimiser (1 at an end or corner) */
    int kb = on_find_span(c->p, c->n, c->U, Q.best_t);
    double f, fp, d, X[3], D1[3];
    on_orth(c, q, kb, Q.best_t, &f, &fp, &d);
    on_eval_k(c, kb, Q.best_t, X, D1, NULL);
    double sp2 = D1[0] * D1[0] + D1[1] * D1[1] + D1[2] * D1[2];
    double kappa = 1.0;
    if (fabs(f) <= 1e-9 * (sqrt(sp2) * (d + c->diag) + 1e-300) && sp2 > 0.0) kappa = fp / sp2;
    /* runner-up: the best other interior stationary minimum, C0 corner minimum or domain end */
    double runner = INFINITY;
    for (int i = 0; i < Q.nmin; ++i) {
        if (fabs(Q.mins[i].t - Q.best_t) <= 1e-6) continue;
        if (Q.mins[i].interior && Q.mins[i].d < runner) runner = Q.mins[i].d;
    }
    for (int s = 1; s < c->nspan; ++s) {
        int kl = c->span_k[s - 1], kr = c->span_k[s];
        double tj = c->U[kr], fl, fr, fpl, fpr, dl, dr;
        on_orth(c, q, kl, tj, &fl, &fpl, &dl);
        on_orth(c, q, kr, tj, &fr, &fpr, &dr);
        if (fl < 0.0 && fr > 0.0 && fabs(tj - Q.best_t) > 1e-6 && dr < runner) runner = dr;
    }
    {
        int k0 = c->span_k[0], k1 = c->span_k[c->nspan - 1];
        double t0 = c->U[c->p], t1 = c->U[c->n], f0, fp0, d0, f1, fp1, d1;
        on_orth(c, q, k0, t0, &f0, &fp0, &d0);
        on_orth(c, q, k1, t1, &f1, &fp1, &d1);
        if (f0 >= 0.0 && fabs(t0 - Q.best_t) > 1e-6 && d0 < runner) runner = d0;
        if (f1 <= 0.0 && fabs(t1 - Q.best_t) > 1e-6 && d1 < runner) runner = d1;
    }
    *t_out = Q.best_t;
    *d_out = Q.best_d;
    *kappa_out = kappa;
    *runner_out = runner;
}

static int on_check(int p, int n, const double *w)
{
    if (p < 1 || p > ON_MAXP || n < p + 1) return -1;
    for (int i = 0; i < n; ++i)
        if (!(w[i] > 0.0) || !isfinite(w[i])) return -1;
    return 0;
}

/* C, C', C'' of one rational curve at m parameters */
int onc_eval(int p, int n, const double *P, const double *w, const double *U, int64_t m, const double *t,
             double *X, double *D1, double *D2)
{
    if (on_check(p, n, w)) return -1;
    on_curve c;
    on_curve_init(&c, p, n, P, w, U);
    for (int64_t i = 0; i < m; ++i) on_eval(&c, t[i], X + 3 * i, D1 ? D1 + 3 * i : NULL, D2 ? D2 + 3 * i : NULL);
    on_curve_free(&c);
    return 0;
}

/* X[i] = C_{cid[i]}(t[i]) over a CSR set of rational curves (weights per control point) */
int onc_eval_batch(int ncurves, const int32_t *deg, const int64_t *cp_off, const double *cp, const double *w,
                   const int64_t *k_off, const double *knots, int64_t m, const int32_t *cid, const double *t,
                   double *X)
{
    for (int64_t i = 0; i < m; ++i) {
        int c = cid[i];
        if (c < 0 || c >= ncurves) return -1;
        int n = (int)(cp_off[c + 1] - cp_off[c]);
        if (on_check(deg[c], n, w + cp_off[c])) return -1;
        on_curve cv;
        on_curve_init(&cv, deg[c], n, cp + 3 * cp_off[c], w + cp_off[c], knots + k_off[c]);
        on_eval(&cv, t[i], X + 3 * i, NULL, NULL);
        on_curve_free(&cv);
    }
    return 0;
}

/* Projection of m queries, each onto its own rational curve: t*, distance, kappa, runner-up distance. */
int onc_project_batch(int ncurves, const int32_t *deg, const int64_t *cp_off, const double *cp, const double *w,
                      const int64_t *k_off, const double *knots, int64_t m, const int32_t *cid, const double *q,
                      double *t_out, double *d_out, double *kappa_out, double *runner_out, int nthreads)
{
    on_curve *cs = (on_curve *)calloc((size_t)ncurves, sizeof(on_curve));
    for (int c = 0; c < ncurves; ++c) {
        int n = (int)(cp_off[c + 1] - cp_off[c]);
        if (on_check(deg[c], n, w + cp_off[c])) {
            for (int j = 0; j < c; ++j) on_curve_free(&cs[j]);
            free(cs);
            return -1;
        }
        on_curve_init(&cs[c], deg[c], n, cp + 3 * cp_off[c], w + cp_off[c], knots + k_off[c]);
    }
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t i = 0; i < m; ++i) {
        int c = cid[i];
        if (c < 0 || c >= ncurves) { bad = 1; continue; }
        on_project_one(&cs[c], q + 3 * i, &t_out[i], &d_out[i], &kappa_out[i], &runner_out[i]);
    }
    (void)nthreads;
    for (int c = 0; c < ncurves; ++c) on_curve_free(&cs[c]);
    free(cs);
    return bad ? -1 : 0;
}

/* Largest |C(t) - R(u)| over ns uniform u in [0, 1], t = ta + u (tb - ta): the deviation of a cubic
 * Bezier piece R (4 points) from the rational curve on [ta, tb] (sampled). */
double onc_piece_deviation(int p, int n, const double *P, const double *w, const double *U, double ta, double tb,
                           const double *R, int ns)
{
    if (on_check(p, n, w) || ns < 2) return -1.0;
    on_curve c;
    on_curve_init(&c, p, n, P, w, U);
    double worst = 0.0;
    for (int i = 0; i < ns; ++i) {
        double u = (double)i / (double)(ns - 1), v = 1.0 - u;
        double t = (i == ns - 1) ? tb : ta + u * (tb - ta);
        double X[3];
        on_eval(&c, t, X, NULL, NULL);
        double b0 = v * v * v, b1 = 3.0 * u * v * v, b2 = 3.0 * u * u * v, b3 = u * u * u;
        double dd = 0.0;
        for (int k = 0; k < 3; ++k) {
            double r = b0 * R[k] + b1 * R[3 + k] + b2 * R[6 + k] + b3 * R[9 + k];
            dd += (X[k] - r) * (X[k] - r);
        }
        if (sqrt(dd) > worst) worst = sqrt(dd);
    }
    on_curve_free(&c);
    return worst;
}
