/* FP64 CPU oracle of the paper's refinement path for point projection onto a
 * cubic Bezier piece: monotonic decomposition (Sec. 5.2.3), the elimination
 * criterion (Sec. 5.3, Properties 1-2), rebasement of E to Bernstein form
 * (Sec. 5.3, the matrix T) and Bezier clipping (Sec. 5.4.1, eq.
 * subdivisionmatrix).
 *
 * TEST INFRASTRUCTURE ONLY: the test-suite and the benchmark's CPU-baseline leg
 * are its only users; the product library never links it.
 *
 * Notation follows the paper: D(t) = |C(t) - q|^2 (eq. Dt), E(t) = D'(t)
 * (eq. Et, degree 5 for a cubic), E'(t) (eq. E't, degree 4).  Readings taken
 * where the paper is silent:
 *   - every piece end is a candidate point (the paper's Property 2 names only
 *     the curve's first and last points; a C0 joint can hold the minimum with
 *     E jumping sign and no root of E);
 *   - a kept interval is one with E(t_a) < 0 <= E(t_b) on a monotonic piece
 *     (the negation of Property 1);
 *   - the convex hull of the control points (i/5, b_i) meets the t axis in
 *     [z1, z2] = the hull of the crossings of all point pairs;
 *   - after the last clipping the root is the midpoint of the remaining
 *     interval;
 *   - Ferrari's method is applied to E' at the degree its coefficients show: a
 *     leading coefficient below 1e-6 of the largest lower one is dropped (it
 *     only adds roots far outside [0, 1]; normalising by it leaves no
 *     accurate root in [0, 1], as for the E' of a degree-elevated quadratic,
 *     whose cubic and quartic coefficients are rounding noise), and the roots
 *     in [-0.5, 1.5] are polished by three Newton steps on the full E';
 *   - optional safeguard (off for the paper's three clippings): when a clipping
 *     keeps more than half of the interval, the half holding the sign change
 *     of E (E is monotonic there, so exactly one half) replaces it, and the
 *     clipping repeats until the interval is below tol_t or iters is spent.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

static double binom_d(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

/* Power coefficients of E(t) = 2 (C(t) - q) . C'(t) for the cubic Bezier piece
 * with control points Q[4][3] (eq. Et). */
void orc_clip_e_poly(const double* Q, const double* q, double* a)
{
    double c[4][3];
    for (int k = 0; k < 3; ++k) {
        c[0][k] = Q[k] - q[k];
        c[1][k] = 3.0 * (Q[3 + k] - Q[k]);
        c[2][k] = 3.0 * (Q[6 + k] - 2.0 * Q[3 + k] + Q[k]);
        c[3][k] = Q[9 + k] - 3.0 * Q[6 + k] + 3.0 * Q[3 + k] - Q[k];
    }
    for (int m = 0; m < 6; ++m) a[m] = 0.0;
    /* C - q = sum_j c_j t^j, C' = sum_j (j+1) c_{j+1} t^j */
    for (int j = 0; j < 4; ++j)
        for (int i = 0; i < 3; ++i) {
            const double d = (double)(i + 1);
            for (int k = 0; k < 3; ++k) a[j + i] += 2.0 * c[j][k] * d * c[i + 1][k];
        }
}

static double horner(const double* a, int n, double t)
{
    double r = a[n];
    for (int m = n - 1; m >= 0; --m) r = r * t + a[m];
    return r;
}

/* Real roots of the monic cubic x^3 + A x^2 + B x + C (Cardano, or the
 * trigonometric form for three real roots); returns the largest. */
static double cubic_largest_root(double A, double B, double C)
{
    const double P = B - A * A / 3.0;
    const double Qc = 2.0 * A * A * A / 27.0 - A * B / 3.0 + C;
    const double disc = Qc * Qc / 4.0 + P * P * P / 27.0;
    double w;
    if (disc > 0.0) {
        const double sd = sqrt(disc);
        w = cbrt(-Qc / 2.0 + sd) + cbrt(-Qc / 2.0 - sd);
    } else if (P == 0.0) {
        w = 0.0;
    } else {
        const double r = sqrt(-P / 3.0);
        double cphi = (-Qc / 2.0) / (r * r * r);
        if (cphi > 1.0) cphi = 1.0;
        if (cphi < -1.0) cphi = -1.0;
        w = 2.0 * r * cos(acos(cphi) / 3.0);
    }
    return w - A / 3.0;
}

/* Real roots of y^2 + b y + c, appended to r[*n]. */
static void quad_roots(double b, double c, double* r, int* n)
{
    const double disc = b * b - 4.0 * c;
    if (disc < 0.0) return;
    const double s = sqrt(disc);
    /* the larger-magnitude root first, the other from the product */
    const double y1 = (b >= 0.0) ? (-b - s) / 2.0 : (-b + s) / 2.0;
    r[(*n)++] = y1;
    if (disc > 0.0) r[(*n)++] = (y1 != 0.0) ? c / y1 : -b - y1;
}

/* Real roots of c[0] + c[1] x + ... + c[4] x^4 by Ferrari's method (Sec.
 * 5.2.3): depress, solve the resolvent cubic for m, factor into two
 * quadratics.  Lower degrees when the leading coefficients vanish.  Roots are
 * returned sorted; the count is the return value. */
int orc_ferrari(const double* c, double* roots)
{
    double mx = 0.0;
    for (int i = 0; i < 5; ++i) mx = fmax(mx, fabs(c[i]));
    int n = 0;
    if (mx == 0.0) return 0;
    /* the degree: a leading coefficient below 1e-6 of the largest lower one only
     * adds roots far outside [0, 1] and is dropped (the kept roots are then
     * polished on the full polynomial by orc_ferrari_01) */
    double lower[5];
    lower[0] = 0.0;
    for (int k = 1; k < 5; ++k) lower[k] = fmax(lower[k - 1], fabs(c[k - 1]));
    int deg = 4;
    while (deg > 0 && !(fabs(c[deg]) > 1e-6 * lower[deg])) --deg;
    if (deg < 4) {
        /* degree <= 3 */
        if (deg == 3) {
            const double A = c[2] / c[3], B = c[1] / c[3], C = c[0] / c[3];
            const double P = B - A * A / 3.0;
            const double Qc = 2.0 * A * A * A / 27.0 - A * B / 3.0 + C;
            const double disc = Qc * Qc / 4.0 + P * P * P / 27.0;
            if (disc > 0.0) {
                const double sd = sqrt(disc);
                roots[n++] = cbrt(-Qc / 2.0 + sd) + cbrt(-Qc / 2.0 - sd) - A / 3.0;
            } else if (P == 0.0) {
                roots[n++] = -A / 3.0;
            } else {
                const double r = sqrt(-P / 3.0);
                double cphi = (-Qc / 2.0) / (r * r * r);
                if (cphi > 1.0) cphi = 1.0;
                if (cphi < -1.0) cphi = -1.0;
                const double phi = acos(cphi);
                for (int k = 0; k < 3; ++k) roots[n++] = 2.0 * r * cos((phi - 2.0 * M_PI * k) / 3.0) - A / 3.0;
            }
        } else if (deg == 2) {
            quad_roots(c[1] / c[2], c[0] / c[2], roots, &n);
        } else if (deg == 1) {
            roots[n++] = -c[0] / c[1];
        }
    } else {
        const double b = c[3] / c[4], cc = c[2] / c[4], d = c[1] / c[4], e = c[0] / c[4];
        /* x = y - b/4: y^4 + p y^2 + q y + r */
        const double p = cc - 3.0 * b * b / 8.0;
        const double qd = d - b * cc / 2.0 + b * b * b / 8.0;
        const double r = e - b * d / 4.0 + b * b * cc / 16.0 - 3.0 * b * b * b * b / 256.0;
        double y[4];
        int ny = 0;
        const double scale = fmax(fabs(p), fmax(sqrt(fabs(r)), 1e-300));
        if (fabs(qd) <= 1e-14 * scale * sqrt(scale)) {
            /* biquadratic: z = y^2, z^2 + p z + r = 0 */
            double z[2];
            int nz = 0;
            quad_roots(p, r, z, &nz);
            for (int i = 0; i < nz; ++i)
                if (z[i] >= 0.0) {
                    const double s = sqrt(z[i]);
                    y[ny++] = s;
                    if (s > 0.0) y[ny++] = -s;
                }
        } else {
            /* resolvent: m^3 + p m^2 + (p^2/4 - r) m - q^2/8 = 0, largest root m > 0 */
            const double m = cubic_largest_root(p, p * p / 4.0 - r, -qd * qd / 8.0);
            if (m > 0.0) {
                const double s = sqrt(2.0 * m);
                quad_roots(-s, p / 2.0 + m + qd / (2.0 * s), y, &ny);
                quad_roots(s, p / 2.0 + m - qd / (2.0 * s), y, &ny);
            }
        }
        for (int i = 0; i < ny; ++i) roots[n++] = y[i] - b / 4.0;
    }
    /* sort */
    for (int i = 1; i < n; ++i)
        for (int j = i; j > 0 && roots[j] < roots[j - 1]; --j) {
            const double t = roots[j];
            roots[j] = roots[j - 1];
            roots[j - 1] = t;
        }
    return n;
}

/* Roots of E' used as split points: the roots by Ferrari's method within
 * [-0.5, 1.5], each polished by three Newton steps on the full quartic (a
 * dropped leading term shifts them by a little; the polish removes it). */
int orc_ferrari_01(const double* c, double* roots)
{
    double r[4];
    const int nr = orc_ferrari(c, r);
    int n = 0;
    for (int i = 0; i < nr; ++i) {
        double x = r[i];
        if (!(x > -0.5 && x < 1.5)) continue;
        for (int it = 0; it < 3; ++it) {
            const double f = (((c[4] * x + c[3]) * x + c[2]) * x + c[1]) * x + c[0];
            const double fp = ((4.0 * c[4] * x + 3.0 * c[3]) * x + 2.0 * c[2]) * x + c[1];
            if (fp == 0.0) break;
            x -= f / fp;
        }
        roots[n++] = x;
    }
    for (int i = 1; i < n; ++i)
        for (int j = i; j > 0 && roots[j] < roots[j - 1]; --j) {
            const double t = roots[j];
            roots[j] = roots[j - 1];
            roots[j - 1] = t;
        }
    return n;
}

/* Rebasement b = T a of a degree-n polynomial, T_ij = C(i,j) / C(n,j) for
 * j <= i (Sec. 5.3; the printed 6x6 matrix for n = 5). */
void orc_rebase(int n, const double* a, double* b)
{
    for (int i = 0; i <= n; ++i) {
        double s = 0.0;
        for (int j = 0; j <= i; ++j) s += binom_d(i, j) / binom_d(n, j) * a[j];
        b[i] = s;
    }
}

/* Subdivision matrices of a degree-n Bezier (Sec. 5.2.2): the left part [0, z]
 * has control points L = S_L(z) b, the right part [z, 1] R = S_R(z) b. */
void orc_sub_left(int n, double z, double* S)
{
    for (int i = 0; i <= n; ++i)
        for (int j = 0; j <= n; ++j)
            S[i * (n + 1) + j] = (j <= i) ? binom_d(i, j) * pow(z, j) * pow(1.0 - z, i - j) : 0.0;
}
void orc_sub_right(int n, double z, double* S)
{
    for (int i = 0; i <= n; ++i)
        for (int j = 0; j <= n; ++j)
            S[i * (n + 1) + j] = (j >= i) ? binom_d(n - i, j - i) * pow(z, j - i) * pow(1.0 - z, n - j) : 0.0;
}

/* Intersection of the convex hull of (i/n, b_i) with the t axis: [z1, z2].
 * Returns 0 when the hull does not meet the axis. */
int orc_hull_axis(int n, const double* b, double* z1, double* z2)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i <= n; ++i) {
        if (b[i] == 0.0) {
            lo = fmin(lo, (double)i / n);
            hi = fmax(hi, (double)i / n);
        }
        for (int j = i + 1; j <= n; ++j)
            if ((b[i] < 0.0 && b[j] > 0.0) || (b[i] > 0.0 && b[j] < 0.0)) {
                const double xi = (double)i / n, xj = (double)j / n;
                const double x = xi + (xj - xi) * b[i] / (b[i] - b[j]);
                lo = fmin(lo, x);
                hi = fmax(hi, x);
            }
    }
    if (!(lo <= hi)) return 0;
    *z1 = fmax(lo, 0.0);
    *z2 = fmin(hi, 1.0);
    return 1;
}

/* One Bezier clipping step: out = S_[z1,z2] b = S_L(w) S_R(z1) b with
 * w = (z2 - z1) / (1 - z1) (eq. subdivisionmatrix). */
void orc_clip_apply(int n, const double* b, double z1, double z2, double* out)
{
    double SR[36], SL[36], t[6];
    orc_sub_right(n, z1, SR);
    const double w = (z1 < 1.0) ? (z2 - z1) / (1.0 - z1) : 0.0;
    orc_sub_left(n, w, SL);
    for (int i = 0; i <= n; ++i) {
        double s = 0.0;
        for (int j = 0; j <= n; ++j) s += SR[i * (n + 1) + j] * b[j];
        t[i] = s;
    }
    for (int i = 0; i <= n; ++i) {
        double s = 0.0;
        for (int j = 0; j <= n; ++j) s += SL[i * (n + 1) + j] * t[j];
        out[i] = s;
    }
}

static double piece_d2(const double* Q, const double* q, double t)
{
    const double s = 1.0 - t;
    const double w0 = s * s * s, w1 = 3.0 * s * s * t, w2 = 3.0 * s * t * t, w3 = t * t * t;
    double d = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double x = w0 * Q[k] + w1 * Q[3 + k] + w2 * Q[6 + k] + w3 * Q[9 + k] - q[k];
        d += x * x;
    }
    return d;
}

/* The paper's refinement of one (query, piece) pair:
 *   1. E (eq. Et) and E' (eq. E't) in power form;
 *   2. Ferrari roots of E' in (0, 1) split [0, 1] into monotonic intervals;
 *   3. elimination: an interval is kept iff E(t_a) < 0 <= E(t_b);
 *   4. on a kept interval, E(t_a + h s) in power form of s, rebased to
 *      Bernstein form b = T a;
 *   5. `iters` Bezier clippings of (i/5, b_i); the root is the midpoint of the
 *      remaining interval;
 *   6. candidates: the roots and both piece ends; the best is returned.
 * info (nullable, 4 doubles): monotonic intervals, kept intervals, largest
 * remaining clip width (in t), number of roots of E' in (0, 1). */
static double bern_eval(int n, const double* b, double s)
{
    double w[6];
    for (int i = 0; i <= n; ++i) w[i] = b[i];
    for (int r = 1; r <= n; ++r)
        for (int i = 0; i <= n - r; ++i) w[i] = (1.0 - s) * w[i] + s * w[i + 1];
    return w[0];
}

int orc_clip_piece_ex(const double* Q, const double* q, int iters, int safeguard, double tol_t, double* t_best,
                      double* d2_best, double* info)
{
    double a[6], ep[5], r[4];
    orc_clip_e_poly(Q, q, a);
    for (int m = 0; m < 5; ++m) ep[m] = (double)(m + 1) * a[m + 1];
    const int nr = orc_ferrari_01(ep, r);
    double br[6];
    int nb = 0;
    br[nb++] = 0.0;
    for (int i = 0; i < nr; ++i)
        if (r[i] > 0.0 && r[i] < 1.0 && r[i] > br[nb - 1]) br[nb++] = r[i];
    br[nb++] = 1.0;
    double best_t = 0.0, best_d = piece_d2(Q, q, 0.0);
    const double d1 = piece_d2(Q, q, 1.0);
    if (d1 < best_d) { best_d = d1; best_t = 1.0; }
    int kept = 0;
    double width = 0.0;
    for (int k = 0; k + 1 < nb; ++k) {
        const double ta = br[k], tb = br[k + 1];
        const double ea = horner(a, 5, ta), eb = horner(a, 5, tb);
        if (!(ea < 0.0 && eb >= 0.0)) continue;  /* Property 1 */
        ++kept;
        const double h = tb - ta;
        /* E(ta + h s) = sum_k as_k s^k */
        double as[6], b[6];
        for (int i = 0; i <= 5; ++i) {
            double s = 0.0;
            for (int m = i; m <= 5; ++m) s += a[m] * binom_d(m, i) * pow(ta, m - i);
            as[i] = s * pow(h, i);
        }
        orc_rebase(5, as, b);
        double lo = 0.0, hi = 1.0;
        for (int it = 0; it < iters; ++it) {
            double z1, z2;
            if (!orc_hull_axis(5, b, &z1, &z2)) break;
            if (safeguard && z2 - z1 > 0.5) {
                /* keep the half of [z1, z2] where E changes sign */
                const double zm = 0.5 * (z1 + z2);
                if (bern_eval(5, b, zm) >= 0.0) z2 = zm; else z1 = zm;
            }
            double nb6[6];
            orc_clip_apply(5, b, z1, z2, nb6);
            const double nlo = lo + (hi - lo) * z1, nhi = lo + (hi - lo) * z2;
            lo = nlo;
            hi = nhi;
            memcpy(b, nb6, sizeof nb6);
            if (h * (hi - lo) <= tol_t) break;
        }
        const double t = ta + h * 0.5 * (lo + hi);
        width = fmax(width, h * (hi - lo));
        const double d = piece_d2(Q, q, t);
        if (d < best_d) { best_d = d; best_t = t; }
    }
    *t_best = best_t;
    *d2_best = best_d;
    if (info) {
        info[0] = (double)(nb - 1);
        info[1] = (double)kept;
        info[2] = width;
        info[3] = (double)(nb - 2);
    }
    return kept;
}

/* The paper's path with exactly `iters` clippings and no safeguard. */
int orc_clip_piece(const double* Q, const double* q, int iters, double* t_best, double* d2_best, double* info)
{
    return orc_clip_piece_ex(Q, q, iters, 0, 0.0, t_best, d2_best, info);
}

/* Batch over (query, piece) pairs: Q[n][12], q[n][3]. */
void orc_clip_pairs(int64_t n, const double* Q, const double* q, int iters, int safeguard, double tol_t, double* t,
                    double* d2, double* info)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i)
        orc_clip_piece_ex(Q + 12 * i, q + 3 * i, iters, safeguard, tol_t, t + i, d2 + i, info ? info + 4 * i : 0);
}
