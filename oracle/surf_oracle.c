/*
 * surf_oracle.c -- slow, plain FP64 CPU oracle for tensor-product B-spline
 * surfaces: evaluation, Bezier patches, deviation of approximating bicubic
 * patches, and point projection / inversion.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark; nothing in the product library links,
 * loads or calls it.  Shares no code with the GPU path.
 *
 * The paper treats curves; its surface case is the tensor product of the same
 * constructions (Sec. 4 basis functions in u and in v).  Conventions:
 *   - S(u, v) = sum_i sum_j N_{i,p}(u) N_{j,q}(v) P_ij, net stored u-major
 *     (P[i * nv + j]), clamped knot vectors U (nu + p + 1) and V (nv + q + 1);
 *   - Bezier patches by Boehm knot insertion in u for every column of the net,
 *     then in v for every row of each u-span's net;
 *   - projection: the global minimiser of |q - S(u, v)| over the whole domain,
 *     on the ORIGINAL surface: per Bezier patch a 16 x 16 sample grid, Newton
 *     on the stationarity conditions (S - q).S_u = (S - q).S_v = 0 with box
 *     constraints (a clamped coordinate whose gradient points outward is held
 *     on the edge), and a branch-and-bound over grid cells with the
 *     second-order bound min(corner f) - (M_uu h_u^2 + M_vv h_v^2) / 8 of
 *     f = |S - q|^2 (bilinear interpolation error, M from the hodograph
 *     nets), recursing into every cell that could beat the best value.
 *     Patches whose control-net box is farther than the best distance (plus
 *     the uniqueness margin) are skipped (convex-hull property).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_basis(int p, int n, const double *U, double t, double *N);
int orc_bezier_spans(int p, int n, const double *P, const double *U, int max_spans, double *bz, double *tab);

#define OS_MAXP 15
#define OS_MAXN (OS_MAXP + 1)

/* ------------------------------------------------------------------------ */
/* Evaluation (tensor-product Cox-de Boor)                                   */
/* ------------------------------------------------------------------------ */
static void os_eval(int p, int q, int nu, int nv, const double *P, const double *U, const double *V, double u,
                    double v, double *out)
{
    double *Nu = (double *)malloc(sizeof(double) * (size_t)nu);
    double *Nv = (double *)malloc(sizeof(double) * (size_t)nv);
    orc_basis(p, nu, U, u, Nu);
    orc_basis(q, nv, V, v, Nv);
    out[0] = out[1] = out[2] = 0.0;
    for (int i = 0; i < nu; ++i) {
        if (Nu[i] == 0.0) continue;
        for (int j = 0; j < nv; ++j) {
            const double w = Nu[i] * Nv[j];
            if (w == 0.0) continue;
            for (int c = 0; c < 3; ++c) out[c] += w * P[3 * ((size_t)i * nv + j) + c];
        }
    }
    free(Nu);
    free(Nv);
}

int orc_surf_eval_batch(int nsurf, const int32_t *du, const int32_t *dv, const int32_t *nu, const int32_t *nv,
                        const int64_t *cp_off, const double *cp, const int64_t *ku_off, const double *ku,
                        const int64_t *kv_off, const double *kv, int64_t m, const int32_t *sid, const double *uv,
                        double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < m; ++k) {
        const int s = sid[k];
        if (s < 0 || s >= nsurf) {
            out[3 * k] = out[3 * k + 1] = out[3 * k + 2] = NAN;
            continue;
        }
        os_eval(du[s], dv[s], nu[s], nv[s], cp + 3 * cp_off[s], ku + ku_off[s], kv + kv_off[s], uv[2 * k],
                uv[2 * k + 1], out + 3 * k);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Bezier patches (Boehm in u, then in v)                                    */
/* ------------------------------------------------------------------------ */
/* nets: (p+1) x (q+1) points per patch (u-major), rects: [ua, ub, va, vb].
 * Patches ordered u-span major.  Returns the patch count or < 0. */
int orc_surf_patches(int p, int q, int nu, int nv, const double *P, const double *U, const double *V,
                     int max_patches, double *nets, double *rects)
{
    if (p < 1 || q < 1 || p > OS_MAXP || q > OS_MAXP || nu < p + 1 || nv < q + 1) return -1;
    const int msu = nu, msv = nv; /* at most this many spans */
    double *col = (double *)malloc(sizeof(double) * 3 * (size_t)nu);
    double *bzu = (double *)malloc(sizeof(double) * 3 * (size_t)msu * (p + 1));
    double *tabu = (double *)malloc(sizeof(double) * 2 * (size_t)msu);
    /* T[a][r][j]: u-span a, Bezier row r (0..p), original column j */
    double *T = (double *)malloc(sizeof(double) * 3 * (size_t)msu * (p + 1) * nv);
    int su = 0;
    for (int j = 0; j < nv; ++j) {
        for (int i = 0; i < nu; ++i)
            for (int c = 0; c < 3; ++c) col[3 * i + c] = P[3 * ((size_t)i * nv + j) + c];
        su = orc_bezier_spans(p, nu, col, U, msu, bzu, tabu);
        if (su < 0) { free(col); free(bzu); free(tabu); free(T); return -2; }
        for (int a = 0; a < su; ++a)
            for (int r = 0; r <= p; ++r)
                for (int c = 0; c < 3; ++c)
                    T[3 * (((size_t)a * (p + 1) + r) * nv + j) + c] = bzu[3 * ((size_t)a * (p + 1) + r) + c];
    }
    double *row = (double *)malloc(sizeof(double) * 3 * (size_t)nv);
    double *bzv = (double *)malloc(sizeof(double) * 3 * (size_t)msv * (q + 1));
    double *tabv = (double *)malloc(sizeof(double) * 2 * (size_t)msv);
    int np = 0;
    for (int a = 0; a < su; ++a) {
        int sv = 0;
        for (int r = 0; r <= p; ++r) {
            for (int j = 0; j < nv; ++j)
                for (int c = 0; c < 3; ++c) row[3 * j + c] = T[3 * (((size_t)a * (p + 1) + r) * nv + j) + c];
            sv = orc_bezier_spans(q, nv, row, V, msv, bzv, tabv);
            if (sv < 0 || (size_t)su * sv > (size_t)max_patches) { np = -2; goto done; }
            for (int b = 0; b < sv; ++b)
                for (int k = 0; k <= q; ++k)
                    for (int c = 0; c < 3; ++c)
                        nets[3 * ((((size_t)a * sv + b) * (p + 1) + r) * (q + 1) + k) + c] =
                            bzv[3 * ((size_t)b * (q + 1) + k) + c];
        }
        for (int b = 0; b < sv; ++b) {
            double *rc = rects + 4 * ((size_t)a * sv + b);
            rc[0] = tabu[2 * a];
            rc[1] = tabu[2 * a + 1];
            rc[2] = tabv[2 * b];
            rc[3] = tabv[2 * b + 1];
        }
        np = su * sv;
    }
done:
    free(col); free(bzu); free(tabu); free(T); free(row); free(bzv); free(tabv);
    return np;
}

/* ------------------------------------------------------------------------ */
/* Patch evaluation with derivatives                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int p, q;
    const double *net;                 /* (p+1) x (q+1) points, u-major */
    double rect[4];
    double lo[3], hi[3];               /* control-net box */
    double Lu, Lv, Luu, Lvv;           /* bounds of |S_u|, |S_v|, |S_uu|, |S_vv| from the hodograph nets */
    int dom;                           /* sides on the domain boundary: 1 s=0, 2 s=1, 4 t=0, 8 t=1 */
} os_patch;

/* derivative nets of one patch, built when the patch is searched */
typedef struct {
    const os_patch *pt;
    double du[OS_MAXN * OS_MAXN * 3];  /* p x (q+1): p (P_{i+1,j} - P_ij) */
    double dv[OS_MAXN * OS_MAXN * 3];  /* (p+1) x q */
    double duu[OS_MAXN * OS_MAXN * 3]; /* (p-1) x (q+1) */
    double duv[OS_MAXN * OS_MAXN * 3]; /* p x q */
    double dvv[OS_MAXN * OS_MAXN * 3]; /* (p+1) x (q-1) */
} os_pwork;

/* tensor de Casteljau of an (a+1) x (b+1) net at (u, v) */
static void os_tp_eval(const double *net, int a, int b, double u, double v, double *out)
{
    double w[OS_MAXN][3];
    double colv[OS_MAXN][3];
    if (a < 0 || b < 0) { out[0] = out[1] = out[2] = 0.0; return; }
    for (int i = 0; i <= a; ++i) {
        for (int k = 0; k <= b; ++k)
            for (int c = 0; c < 3; ++c) w[k][c] = net[3 * (i * (b + 1) + k) + c];
        for (int r = 1; r <= b; ++r)
            for (int k = 0; k <= b - r; ++k)
                for (int c = 0; c < 3; ++c) w[k][c] = (1.0 - v) * w[k][c] + v * w[k + 1][c];
        for (int c = 0; c < 3; ++c) colv[i][c] = w[0][c];
    }
    for (int r = 1; r <= a; ++r)
        for (int i = 0; i <= a - r; ++i)
            for (int c = 0; c < 3; ++c) colv[i][c] = (1.0 - u) * colv[i][c] + u * colv[i + 1][c];
    for (int c = 0; c < 3; ++c) out[c] = colv[0][c];
}

static double os_netmax(const double *net, int cnt)
{
    double m = 0.0;
    for (int i = 0; i < cnt; ++i) {
        const double n2 = net[3 * i] * net[3 * i] + net[3 * i + 1] * net[3 * i + 1] + net[3 * i + 2] * net[3 * i + 2];
        if (n2 > m) m = n2;
    }
    return sqrt(m);
}

static void os_derivs(const double *net, int p, int q, double *du, double *dv, double *duu, double *duv, double *dvv)
{
#define NET(i, j, c) net[3 * ((i) * (q + 1) + (j)) + (c)]
    for (int i = 0; i < p; ++i)
        for (int j = 0; j <= q; ++j)
            for (int c = 0; c < 3; ++c) du[3 * (i * (q + 1) + j) + c] = p * (NET(i + 1, j, c) - NET(i, j, c));
    for (int i = 0; i <= p; ++i)
        for (int j = 0; j < q; ++j)
            for (int c = 0; c < 3; ++c) dv[3 * (i * q + j) + c] = q * (NET(i, j + 1, c) - NET(i, j, c));
#undef NET
    for (int i = 0; i < p - 1; ++i)
        for (int j = 0; j <= q; ++j)
            for (int c = 0; c < 3; ++c)
                duu[3 * (i * (q + 1) + j) + c] = (p - 1) * (du[3 * ((i + 1) * (q + 1) + j) + c] - du[3 * (i * (q + 1) + j) + c]);
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < q; ++j)
            for (int c = 0; c < 3; ++c)
                duv[3 * (i * q + j) + c] = q * (du[3 * (i * (q + 1) + j + 1) + c] - du[3 * (i * (q + 1) + j) + c]);
    for (int i = 0; i <= p; ++i)
        for (int j = 0; j < q - 1; ++j)
            for (int c = 0; c < 3; ++c)
                dvv[3 * (i * (q - 1) + j) + c] = (q - 1) * (dv[3 * (i * q + j + 1) + c] - dv[3 * (i * q + j) + c]);
}

static void os_patch_init(os_patch *pt, int p, int q, const double *net, const double *rect)
{
    pt->p = p;
    pt->q = q;
    pt->net = net;
    memcpy(pt->rect, rect, sizeof(double) * 4);
    for (int c = 0; c < 3; ++c) { pt->lo[c] = net[c]; pt->hi[c] = net[c]; }
    for (int i = 0; i < (p + 1) * (q + 1); ++i)
        for (int c = 0; c < 3; ++c) {
            if (net[3 * i + c] < pt->lo[c]) pt->lo[c] = net[3 * i + c];
            if (net[3 * i + c] > pt->hi[c]) pt->hi[c] = net[3 * i + c];
        }
    os_pwork w;
    os_derivs(net, p, q, w.du, w.dv, w.duu, w.duv, w.dvv);
    pt->Lu = os_netmax(w.du, p * (q + 1));
    pt->Lv = os_netmax(w.dv, (p + 1) * q);
    pt->Luu = p >= 2 ? os_netmax(w.duu, (p - 1) * (q + 1)) : 0.0;
    pt->Lvv = q >= 2 ? os_netmax(w.dvv, (p + 1) * (q - 1)) : 0.0;
}

static void os_work_init(os_pwork *w, const os_patch *pt)
{
    w->pt = pt;
    os_derivs(pt->net, pt->p, pt->q, w->du, w->dv, w->duu, w->duv, w->dvv);
}

/* S, S_u, S_v, S_uu, S_uv, S_vv at local (s, t) in [0,1]^2 (derivatives in s, t) */
static void os_patch_eval(const os_pwork *w, double s, double t, double *S, double *Su, double *Sv, double *Suu,
                          double *Suv, double *Svv)
{
    const int p = w->pt->p, q = w->pt->q;
    os_tp_eval(w->pt->net, p, q, s, t, S);
    if (!Su) return;
    os_tp_eval(w->du, p - 1, q, s, t, Su);
    os_tp_eval(w->dv, p, q - 1, s, t, Sv);
    os_tp_eval(w->duu, p - 2, q, s, t, Suu);
    os_tp_eval(w->duv, p - 1, q - 1, s, t, Suv);
    os_tp_eval(w->dvv, p, q - 2, s, t, Svv);
}

static double os_f(const os_patch *pt, const double *x, double s, double t)
{
    double S[3];
    os_tp_eval(pt->net, pt->p, pt->q, s, t, S);
    return (S[0] - x[0]) * (S[0] - x[0]) + (S[1] - x[1]) * (S[1] - x[1]) + (S[2] - x[2]) * (S[2] - x[2]);
}

/* ------------------------------------------------------------------------ */
/* Projection                                                                */
/* ------------------------------------------------------------------------ */
#define OS_MAXCAND 256
typedef struct {
    double u, v, f;  /* global parameters, squared distance */
    int out;         /* sides (as os_patch.dom) inside the domain where the point is held with the
                        gradient pointing across: a minimum of the patch, not of the surface */
    const os_patch *pt;
} os_cand;

typedef struct {
    const double *x;
    double best_f, best_u, best_v, best_kappa;
    double thresh_f;   /* cells / patches below this are explored (best + uniqueness margin) */
    double margin;     /* distance margin of the uniqueness test */
    os_cand cand[OS_MAXCAND];
    int ncand;
    int64_t work;      /* branch-and-bound cells visited (capped; reported) */
} os_query;

static void os_update_thresh(os_query *Q)
{
    const double d = sqrt(Q->best_f) + Q->margin;
    Q->thresh_f = d * d;
}

static void os_record(os_query *Q, const os_patch *pt, double s, double t, double f, double kappa, int out)
{
    const double u = pt->rect[0] + s * (pt->rect[1] - pt->rect[0]);
    const double v = pt->rect[2] + t * (pt->rect[3] - pt->rect[2]);
    if (f < Q->best_f || (f == Q->best_f && (u < Q->best_u || (u == Q->best_u && v < Q->best_v)))) {
        Q->best_f = f;
        Q->best_u = u;
        Q->best_v = v;
        Q->best_kappa = kappa;
        os_update_thresh(Q);
    }
    /* the same point of the same patch, reached again from another start,
     * is one candidate: duplicates of the best must not evict the runner-up */
    for (int i = 0; i < Q->ncand; ++i)
        if (Q->cand[i].pt == pt && fabs(Q->cand[i].u - u) <= 1e-9 && fabs(Q->cand[i].v - v) <= 1e-9) {
            if (f < Q->cand[i].f) { Q->cand[i].f = f; Q->cand[i].out = out; }
            return;
        }
    int w = Q->ncand;
    if (Q->ncand < OS_MAXCAND) {
        Q->ncand++;
    } else {
        /* keep the candidates with the smallest f */
        w = 0;
        for (int i = 1; i < OS_MAXCAND; ++i)
            if (Q->cand[i].f > Q->cand[w].f) w = i;
        if (!(f < Q->cand[w].f)) return;
    }
    Q->cand[w].u = u;
    Q->cand[w].v = v;
    Q->cand[w].f = f;
    Q->cand[w].out = out;
    Q->cand[w].pt = pt;
}

/* Conditioning of a minimiser: smallest generalised eigenvalue of
 * (Hessian of f/2, first fundamental form).  1 on the boundary. */
static double os_kappa(const double *S, const double *Su, const double *Sv, const double *Suu, const double *Suv,
                       const double *Svv, const double *x)
{
    double r[3] = {S[0] - x[0], S[1] - x[1], S[2] - x[2]};
    const double g11 = Su[0] * Su[0] + Su[1] * Su[1] + Su[2] * Su[2];
    const double g12 = Su[0] * Sv[0] + Su[1] * Sv[1] + Su[2] * Sv[2];
    const double g22 = Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2];
    const double h11 = g11 + r[0] * Suu[0] + r[1] * Suu[1] + r[2] * Suu[2];
    const double h12 = g12 + r[0] * Suv[0] + r[1] * Suv[1] + r[2] * Suv[2];
    const double h22 = g22 + r[0] * Svv[0] + r[1] * Svv[1] + r[2] * Svv[2];
    const double dg = g11 * g22 - g12 * g12;
    if (!(dg > 0.0)) return 1.0;
    const double tr = (g22 * h11 - 2.0 * g12 * h12 + g11 * h22) / dg;
    const double dt = (h11 * h22 - h12 * h12) / dg;
    const double disc = tr * tr - 4.0 * dt;
    return 0.5 * (tr - sqrt(disc > 0.0 ? disc : 0.0));
}

/* Newton on the stationarity conditions within [0,1]^2 from (s, t); a
 * coordinate clamped to a side whose gradient points outward stays there and
 * the other coordinate continues alone.  Records the end point when it is a
 * Karush-Kuhn-Tucker point of f on the box. */
static void os_newton(os_query *Q, const os_pwork *w, double s, double t)
{
    const os_patch *pt = w->pt;
    const double *x = Q->x;
    int fix_s = 0, fix_t = 0;
    double S[3], Su[3], Sv[3], Suu[3], Suv[3], Svv[3];
    for (int it = 0; it < 60; ++it) {
        os_patch_eval(w, s, t, S, Su, Sv, Suu, Suv, Svv);
        const double r[3] = {S[0] - x[0], S[1] - x[1], S[2] - x[2]};
        const double gs = r[0] * Su[0] + r[1] * Su[1] + r[2] * Su[2];
        const double gt = r[0] * Sv[0] + r[1] * Sv[1] + r[2] * Sv[2];
        const double h11 = Su[0] * Su[0] + Su[1] * Su[1] + Su[2] * Su[2] + r[0] * Suu[0] + r[1] * Suu[1] + r[2] * Suu[2];
        const double h12 = Su[0] * Sv[0] + Su[1] * Sv[1] + Su[2] * Sv[2] + r[0] * Suv[0] + r[1] * Suv[1] + r[2] * Suv[2];
        const double h22 = Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2] + r[0] * Svv[0] + r[1] * Svv[1] + r[2] * Svv[2];
        /* release a held coordinate whose gradient now points inward */
        if (fix_s && ((s == 0.0 && gs < 0.0) || (s == 1.0 && gs > 0.0))) fix_s = 0;
        if (fix_t && ((t == 0.0 && gt < 0.0) || (t == 1.0 && gt > 0.0))) fix_t = 0;
        double ds = 0.0, dt = 0.0;
        if (!fix_s && !fix_t) {
            const double det = h11 * h22 - h12 * h12;
            if (det > 0.0 && h11 > 0.0) {
                ds = -(h22 * gs - h12 * gt) / det;
                dt = -(h11 * gt - h12 * gs) / det;
            } else {  /* not convex here: gradient step scaled by the metric */
                const double g11 = Su[0] * Su[0] + Su[1] * Su[1] + Su[2] * Su[2] + 1e-300;
                const double g22 = Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2] + 1e-300;
                ds = -gs / g11;
                dt = -gt / g22;
            }
        } else if (!fix_s) {
            ds = h11 > 0.0 ? -gs / h11 : -gs / (Su[0] * Su[0] + Su[1] * Su[1] + Su[2] * Su[2] + 1e-300);
        } else if (!fix_t) {
            dt = h22 > 0.0 ? -gt / h22 : -gt / (Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2] + 1e-300);
        }
        /* limit the step to a quarter of the patch and do not go uphill */
        const double lim = 0.25;
        if (fabs(ds) > lim) { dt *= lim / fabs(ds); ds = ds > 0 ? lim : -lim; }
        if (fabs(dt) > lim) { ds *= lim / fabs(dt); dt = dt > 0 ? lim : -lim; }
        const double f0 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        double sn = s + ds, tn = t + dt, fn;
        for (int bt = 0;; ++bt) {
            sn = sn < 0.0 ? 0.0 : (sn > 1.0 ? 1.0 : sn);
            tn = tn < 0.0 ? 0.0 : (tn > 1.0 ? 1.0 : tn);
            fn = os_f(pt, x, sn, tn);
            if (fn <= f0 || bt == 30) break;
            ds *= 0.5;
            dt *= 0.5;
            sn = s + ds;
            tn = t + dt;
        }
        if (fn > f0) break;
        if (sn == 0.0 || sn == 1.0) fix_s = (sn != s) || fix_s;
        if (tn == 0.0 || tn == 1.0) fix_t = (tn != t) || fix_t;
        const double step = fabs(sn - s) + fabs(tn - t);
        s = sn;
        t = tn;
        if (step <= 1e-15) break;
    }
    os_patch_eval(w, s, t, S, Su, Sv, Suu, Suv, Svv);
    const double r[3] = {S[0] - x[0], S[1] - x[1], S[2] - x[2]};
    const double f = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double gs = r[0] * Su[0] + r[1] * Su[1] + r[2] * Su[2];
    const double gt = r[0] * Sv[0] + r[1] * Sv[1] + r[2] * Sv[2];
    const double nr = sqrt(f);
    const double nsu = sqrt(Su[0] * Su[0] + Su[1] * Su[1] + Su[2] * Su[2]);
    const double nsv = sqrt(Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2]);
    /* stationarity (or the outward sign on a clamped side) within rounding */
    /* relative to |S - x|, with a rounding floor for points on the surface */
    const double scale = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]) + sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const double tol_s = nsu * (1e-9 * nr + 1e-14 * scale) + 1e-300, tol_t = nsv * (1e-9 * nr + 1e-14 * scale) + 1e-300;
    const int ok_s = fabs(gs) <= tol_s || (s == 0.0 && gs > 0.0) || (s == 1.0 && gs < 0.0);
    const int ok_t = fabs(gt) <= tol_t || (t == 0.0 && gt > 0.0) || (t == 1.0 && gt < 0.0);
    if (ok_s && ok_t) {
        const int interior = s > 0.0 && s < 1.0 && t > 0.0 && t < 1.0;
        int out = 0;
        if (s == 0.0 && gs > tol_s) out |= 1;
        if (s == 1.0 && gs < -tol_s) out |= 2;
        if (t == 0.0 && gt > tol_t) out |= 4;
        if (t == 1.0 && gt < -tol_t) out |= 8;
        out &= ~pt->dom;
        os_record(Q, pt, s, t, f, interior ? os_kappa(S, Su, Sv, Suu, Suv, Svv, x) : 1.0, out);
    }
}

/* Best value only (a sample point, not a stationary point). */
static void os_best(os_query *Q, const os_patch *pt, double s, double t, double f)
{
    const double u = pt->rect[0] + s * (pt->rect[1] - pt->rect[0]);
    const double v = pt->rect[2] + t * (pt->rect[3] - pt->rect[2]);
    if (f < Q->best_f) {
        Q->best_f = f;
        Q->best_u = u;
        Q->best_v = v;
        Q->best_kappa = 1.0;
        os_update_thresh(Q);
    }
}

/* Branch and bound over the cell [s0,s1] x [t0,t1] (local) with corner values.
 * A cell whose lower bound could beat the best value is split down to 1e-7 in
 * the global parameter (Newton from every centre).  A cell that could only
 * hold another local minimum within the uniqueness margin (the runner-up) is
 * searched coarsely: Newton from its centre, split at most 3 levels below the
 * sample grid, and skipped within 1e-4 of the best point (the best minimum's
 * own basin). */
static void os_bb(os_query *Q, const os_pwork *w, double Muu, double Mvv, double s0, double s1, double t0,
                  double t1, double f00, double f10, double f01, double f11, int depth)
{
    if (++Q->work > 4000000) return;
    const double hs = s1 - s0, ht = t1 - t0;
    double mn = f00;
    if (f10 < mn) mn = f10;
    if (f01 < mn) mn = f01;
    if (f11 < mn) mn = f11;
    const double lb = mn - (Muu * hs * hs + Mvv * ht * ht) / 8.0;
    if (lb > Q->thresh_f) return;
    const os_patch *pt = w->pt;
    if (f00 < Q->best_f) os_best(Q, pt, s0, t0, f00);
    if (f10 < Q->best_f) os_best(Q, pt, s1, t0, f10);
    if (f01 < Q->best_f) os_best(Q, pt, s0, t1, f01);
    if (f11 < Q->best_f) os_best(Q, pt, s1, t1, f11);
    const double wu = pt->rect[1] - pt->rect[0], wv = pt->rect[3] - pt->rect[2];
    if (lb > Q->best_f) {
        const double u0 = pt->rect[0] + s0 * wu, u1 = pt->rect[0] + s1 * wu;
        const double v0 = pt->rect[2] + t0 * wv, v1 = pt->rect[2] + t1 * wv;
        const double eu = Q->best_u < u0 ? u0 - Q->best_u : (Q->best_u > u1 ? Q->best_u - u1 : 0.0);
        const double ev = Q->best_v < v0 ? v0 - Q->best_v : (Q->best_v > v1 ? Q->best_v - v1 : 0.0);
        if (eu * eu + ev * ev < 1e-8) return;
        os_newton(Q, w, 0.5 * (s0 + s1), 0.5 * (t0 + t1));
        if (depth >= 3) return;
    } else {
        if (depth >= 40 || (hs * wu < 1e-7 && ht * wv < 1e-7)) return;
        os_newton(Q, w, 0.5 * (s0 + s1), 0.5 * (t0 + t1));
    }
    if (lb > Q->thresh_f) return;
    const double sm = 0.5 * (s0 + s1), tm = 0.5 * (t0 + t1);
    const double fm = os_f(pt, Q->x, sm, tm);
    const double fs0 = os_f(pt, Q->x, sm, t0), fs1 = os_f(pt, Q->x, sm, t1);
    const double f0t = os_f(pt, Q->x, s0, tm), f1t = os_f(pt, Q->x, s1, tm);
    os_bb(Q, w, Muu, Mvv, s0, sm, t0, tm, f00, fs0, f0t, fm, depth + 1);
    os_bb(Q, w, Muu, Mvv, sm, s1, t0, tm, fs0, f10, fm, f1t, depth + 1);
    os_bb(Q, w, Muu, Mvv, s0, sm, tm, t1, f0t, fm, f01, fs1, depth + 1);
    os_bb(Q, w, Muu, Mvv, sm, s1, tm, t1, fm, f1t, fs1, f11, depth + 1);
}

static double os_box_dist2(const os_patch *pt, const double *x)
{
    double d2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        double e = 0.0;
        if (x[c] < pt->lo[c]) e = pt->lo[c] - x[c];
        else if (x[c] > pt->hi[c]) e = x[c] - pt->hi[c];
        d2 += e * e;
    }
    return d2;
}

#define OS_G 16
static void os_patch_search(os_query *Q, const os_patch *pt)
{
    const double *x = Q->x;
    os_pwork w;
    os_work_init(&w, pt);
    /* bounds of |f_ss|, |f_tt| on the patch: 2 (|S_s|^2 + |S - x| |S_ss|) */
    double far2 = 0.0;
    for (int i = 0; i < (pt->p + 1) * (pt->q + 1); ++i) {
        double d2 = 0.0;
        for (int c = 0; c < 3; ++c) d2 += (pt->net[3 * i + c] - x[c]) * (pt->net[3 * i + c] - x[c]);
        if (d2 > far2) far2 = d2;
    }
    const double far = sqrt(far2);
    const double Muu = 2.0 * (pt->Lu * pt->Lu + far * pt->Luu);
    const double Mvv = 2.0 * (pt->Lv * pt->Lv + far * pt->Lvv);
    double F[OS_G][OS_G];
    for (int i = 0; i < OS_G; ++i)
        for (int j = 0; j < OS_G; ++j) F[i][j] = os_f(pt, x, (double)i / (OS_G - 1), (double)j / (OS_G - 1));
    /* Newton from every local minimum of the samples (8-neighbourhood, sides included) */
    for (int i = 0; i < OS_G; ++i)
        for (int j = 0; j < OS_G; ++j) {
            int is_min = 1;
            for (int a = -1; a <= 1 && is_min; ++a)
                for (int b = -1; b <= 1; ++b) {
                    const int ii = i + a, jj = j + b;
                    if ((a || b) && ii >= 0 && ii < OS_G && jj >= 0 && jj < OS_G && F[ii][jj] < F[i][j]) {
                        is_min = 0;
                        break;
                    }
                }
            if (is_min) os_newton(Q, &w, (double)i / (OS_G - 1), (double)j / (OS_G - 1));
        }
    for (int i = 0; i + 1 < OS_G; ++i)
        for (int j = 0; j + 1 < OS_G; ++j)
            os_bb(Q, &w, Muu, Mvv, (double)i / (OS_G - 1), (double)(i + 1) / (OS_G - 1), (double)j / (OS_G - 1),
                  (double)(j + 1) / (OS_G - 1), F[i][j], F[i + 1][j], F[i][j + 1], F[i + 1][j + 1], 0);
}

typedef struct {
    int np;
    os_patch *pts;
    double *nets;
} os_surf;

static int os_surf_build(os_surf *S, int p, int q, int nu, int nv, const double *P, const double *U,
                         const double *V)
{
    const int maxp = nu * nv;
    double *nets = (double *)malloc(sizeof(double) * 3 * (size_t)maxp * (p + 1) * (q + 1));
    double *rects = (double *)malloc(sizeof(double) * 4 * (size_t)maxp);
    const int np = orc_surf_patches(p, q, nu, nv, P, U, V, maxp, nets, rects);
    if (np < 0) { free(nets); free(rects); return -1; }
    S->np = np;
    S->pts = (os_patch *)malloc(sizeof(os_patch) * (size_t)(np > 0 ? np : 1));
    double dom[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (int k = 0; k < np; ++k) {
        const double *r = rects + 4 * (size_t)k;
        if (r[0] < dom[0]) dom[0] = r[0];
        if (r[1] > dom[1]) dom[1] = r[1];
        if (r[2] < dom[2]) dom[2] = r[2];
        if (r[3] > dom[3]) dom[3] = r[3];
    }
    for (int k = 0; k < np; ++k) {
        const double *r = rects + 4 * (size_t)k;
        os_patch_init(&S->pts[k], p, q, nets + 3 * (size_t)k * (p + 1) * (q + 1), r);
        S->pts[k].dom = (r[0] == dom[0] ? 1 : 0) | (r[1] == dom[1] ? 2 : 0) | (r[2] == dom[2] ? 4 : 0) |
                        (r[3] == dom[3] ? 8 : 0);
    }
    S->nets = nets;
    free(rects);
    return 0;
}

typedef struct { double d2; int k; } os_order;
static int os_cmp(const void *a, const void *b)
{
    const double x = ((const os_order *)a)->d2, y = ((const os_order *)b)->d2;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Projection of x onto surface S: global minimiser (u, v), distance, the
 * runner-up local minimum farther than 1e-6 in parameter (inf if none within
 * the uniqueness margin) and the conditioning kappa. */
static void os_project_one(const os_surf *S, const double *x, double margin, double *uv, double *dist,
                           double *runner, double *kappa)
{
    os_query Q;
    memset(&Q, 0, sizeof(Q));
    Q.x = x;
    Q.best_f = INFINITY;
    Q.best_u = Q.best_v = 0.0;
    Q.best_kappa = 1.0;
    Q.margin = margin;
    Q.thresh_f = INFINITY;
    os_order *ord = (os_order *)malloc(sizeof(os_order) * (size_t)(S->np > 0 ? S->np : 1));
    for (int k = 0; k < S->np; ++k) {
        ord[k].d2 = os_box_dist2(&S->pts[k], x);
        ord[k].k = k;
    }
    qsort(ord, (size_t)S->np, sizeof(os_order), os_cmp);
    for (int m = 0; m < S->np; ++m) {
        if (ord[m].d2 > Q.thresh_f) break;
        os_patch_search(&Q, &S->pts[ord[m].k]);
    }
    free(ord);
    uv[0] = Q.best_u;
    uv[1] = Q.best_v;
    *dist = sqrt(Q.best_f);
    *kappa = Q.work > 4000000 ? NAN : Q.best_kappa;  /* NaN: the search hit its work cap */
    double rn = INFINITY;
    for (int i = 0; i < Q.ncand; ++i) {
        const double du = Q.cand[i].u - Q.best_u, dv = Q.cand[i].v - Q.best_v;
        if (!(sqrt(du * du + dv * dv) > 1e-6)) continue;
        /* a point held on a side inside the domain with the gradient pointing
         * across is the minimum of its patch only: the surface goes on falling
         * in the neighbour, unless the neighbour's search stopped at the same
         * point against the same side (a crease where the surface is only C0) */
        if (Q.cand[i].out) {
            int crease = 0;
            for (int j = 0; j < Q.ncand && !crease; ++j)
                crease = j != i && Q.cand[j].pt != Q.cand[i].pt && Q.cand[j].out &&
                         fabs(Q.cand[j].u - Q.cand[i].u) <= 1e-8 && fabs(Q.cand[j].v - Q.cand[i].v) <= 1e-8;
            if (!crease) continue;
        }
        const double d = sqrt(Q.cand[i].f);
        if (d < rn) rn = d;
    }
    *runner = rn;
}

int orc_surf_project_batch(int nsurf, const int32_t *du, const int32_t *dv, const int32_t *nu, const int32_t *nv,
                           const int64_t *cp_off, const double *cp, const int64_t *ku_off, const double *ku,
                           const int64_t *kv_off, const double *kv, int64_t m, const int32_t *sid, const double *x,
                           double *uv, double *dist, double *runner, double *kappa, int nthreads)
{
    /* surfaces are built once, queries run in parallel */
    os_surf *S = (os_surf *)calloc((size_t)nsurf, sizeof(os_surf));
    char *need = (char *)calloc((size_t)nsurf, 1);
    for (int64_t k = 0; k < m; ++k)
        if (sid[k] >= 0 && sid[k] < nsurf) need[sid[k]] = 1;
    int rc = 0;
    for (int s = 0; s < nsurf; ++s) {
        if (!need[s]) continue;
        if (os_surf_build(&S[s], du[s], dv[s], nu[s], nv[s], cp + 3 * cp_off[s], ku + ku_off[s], kv + kv_off[s]))
            rc = -1;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < m; ++k) {
        const int s = sid[k];
        if (s < 0 || s >= nsurf || !need[s]) {
            uv[2 * k] = uv[2 * k + 1] = dist[k] = runner[k] = kappa[k] = NAN;
            continue;
        }
        /* uniqueness margin: 3e-6 of the control-net box diagonal */
        const double *P = cp + 3 * cp_off[s];
        double lo[3] = {P[0], P[1], P[2]}, hi[3] = {P[0], P[1], P[2]};
        for (int i = 0; i < nu[s] * nv[s]; ++i)
            for (int c = 0; c < 3; ++c) {
                if (P[3 * i + c] < lo[c]) lo[c] = P[3 * i + c];
                if (P[3 * i + c] > hi[c]) hi[c] = P[3 * i + c];
            }
        const double diag = sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                 (hi[2] - lo[2]) * (hi[2] - lo[2]));
        os_project_one(&S[s], x + 3 * k, 3e-6 * diag, uv + 2 * k, dist + k, runner + k, kappa + k);
    }
    for (int s = 0; s < nsurf; ++s)
        if (need[s]) { free(S[s].pts); free(S[s].nets); }
    free(S);
    free(need);
    return rc;
}

/* Largest distance between an approximating bicubic patch R (4 x 4 net on the
 * rectangle rect) and the exact surface, on an (ns x ns) grid of the
 * rectangle. */
double orc_surf_patch_deviation(int p, int q, int nu, int nv, const double *P, const double *U, const double *V,
                                const double *R, const double *rect, int ns)
{
    double worst = 0.0;
    for (int i = 0; i < ns; ++i)
        for (int j = 0; j < ns; ++j) {
            const double s = (double)i / (ns - 1), t = (double)j / (ns - 1);
            double a[3], b[3];
            os_tp_eval(R, 3, 3, s, t, a);
            os_eval(p, q, nu, nv, P, U, V, rect[0] + s * (rect[1] - rect[0]), rect[2] + t * (rect[3] - rect[2]), b);
            const double d = sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) + (a[2] - b[2]) * (a[2] - b[2]));
            if (d > worst) worst = d;
        }
    return worst;
}
