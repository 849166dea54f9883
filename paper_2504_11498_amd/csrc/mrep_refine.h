// Device-side refine helpers shared by the HIP translation units of libmrep:
// cubic pieces in local frames, safeguarded Newton on the orthogonality
// condition (C - q).C' = 0 (eqs. Et and E't), the certified minimum of one
// piece, the FP64 polish on the exact degree-p span, and the per-query finish
// (Sec. 5.4.2 reparameterisation to the curve parameter).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/mrep.h"
#include "mrep_dev.h"

namespace mrep {

template <typename T>
struct V3 {
    T x, y, z;
};
template <typename T>
__device__ __forceinline__ T dot(const V3<T>& a, const V3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Cubic piece in its local frame: C(u) = a0 + a1 u + a2 u^2 + a3 u^3 (relative
// to the query), i.e. r(u) = C(u) - q.
template <typename T>
struct Cubic {
    V3<T> a0, a1, a2, a3;
    __device__ void eval(T u, V3<T>& r, V3<T>& d1, V3<T>& d2) const
    {
        r.x = a0.x + u * (a1.x + u * (a2.x + u * a3.x));
        r.y = a0.y + u * (a1.y + u * (a2.y + u * a3.y));
        r.z = a0.z + u * (a1.z + u * (a2.z + u * a3.z));
        d1.x = a1.x + u * ((T)2 * a2.x + u * (T)3 * a3.x);
        d1.y = a1.y + u * ((T)2 * a2.y + u * (T)3 * a3.y);
        d1.z = a1.z + u * ((T)2 * a2.z + u * (T)3 * a3.z);
        d2.x = (T)2 * a2.x + u * (T)6 * a3.x;
        d2.y = (T)2 * a2.y + u * (T)6 * a3.y;
        d2.z = (T)2 * a2.z + u * (T)6 * a3.z;
    }
    __device__ T dist2(T u) const
    {
        T x = a0.x + u * (a1.x + u * (a2.x + u * a3.x));
        T y = a0.y + u * (a1.y + u * (a2.y + u * a3.y));
        T z = a0.z + u * (a1.z + u * (a2.z + u * a3.z));
        return x * x + y * y + z * z;
    }
};

// Load piece s as a cubic relative to q.  FP32: local control points minus the
// local query (q - c computed in FP64).  FP64: global control points minus q.
__device__ __forceinline__ void load_cubic(const DevGeom& G, const DCurve& cv, int64_t s, const double* q, Cubic<float>& C)
{
    const float* lp = G.lcp + s * 12;
    const float* ax = G.aux + s * 8;
    const double cx = cv.origin[0] + (double)ax[AUX_CX];
    const double cy = cv.origin[1] + (double)ax[AUX_CY];
    const double cz = cv.origin[2] + (double)ax[AUX_CZ];
    const float qx = (float)(q[0] - cx), qy = (float)(q[1] - cy), qz = (float)(q[2] - cz);
    float P[12];
    for (int i = 0; i < 12; ++i) P[i] = lp[i];
    C.a0 = {P[0] - qx, P[1] - qy, P[2] - qz};
    C.a1 = {3.f * (P[3] - P[0]), 3.f * (P[4] - P[1]), 3.f * (P[5] - P[2])};
    C.a2 = {3.f * (P[6] - 2.f * P[3] + P[0]), 3.f * (P[7] - 2.f * P[4] + P[1]), 3.f * (P[8] - 2.f * P[5] + P[2])};
    C.a3 = {P[9] - 3.f * P[6] + 3.f * P[3] - P[0], P[10] - 3.f * P[7] + 3.f * P[4] - P[1],
            P[11] - 3.f * P[8] + 3.f * P[5] - P[2]};
}

__device__ __forceinline__ void load_cubic(const DevGeom& G, const DCurve& cv, int64_t s, const double* q, Cubic<double>& C)
{
    const double* P = G.gcp + s * 12;
    double R[12];
    for (int i = 0; i < 12; ++i) R[i] = P[i];
    C.a0 = {R[0] - q[0], R[1] - q[1], R[2] - q[2]};
    C.a1 = {3.0 * (R[3] - R[0]), 3.0 * (R[4] - R[1]), 3.0 * (R[5] - R[2])};
    C.a2 = {3.0 * (R[6] - 2.0 * R[3] + R[0]), 3.0 * (R[7] - 2.0 * R[4] + R[1]), 3.0 * (R[8] - 2.0 * R[5] + R[2])};
    C.a3 = {R[9] - 3.0 * R[6] + 3.0 * R[3] - R[0], R[10] - 3.0 * R[7] + 3.0 * R[4] - R[1],
            R[11] - 3.0 * R[8] + 3.0 * R[5] - R[2]};
}

template <typename T>
struct Newt {
    static constexpr int iters = 8;
    static constexpr T eps = (T)1e-6;
};
template <>
struct Newt<double> {
    static constexpr int iters = 40;
    static constexpr double eps = 1e-15;
};

// Minimum of |C(u) - q|^2 on [lo, hi] near the sample u0: safeguarded Newton on
// f = r.C' when f changes sign on the bracket; otherwise the better bracket end.
template <typename T>
__device__ __forceinline__ void newton_min(const Cubic<T>& C, T lo, T hi, T u0, T& u_best, T& d_best, T& kappa)
{
    V3<T> r, d1, d2;
    C.eval(lo, r, d1, d2);
    T flo = dot(r, d1), dlo = dot(r, r);
    C.eval(hi, r, d1, d2);
    T fhi = dot(r, d1), dhi = dot(r, r);
    T u = u0;
    kappa = (T)1;
    if (flo < (T)0 && fhi > (T)0) {
        T a = lo, b = hi;
        for (int it = 0; it < Newt<T>::iters; ++it) {
            C.eval(u, r, d1, d2);
            T f = dot(r, d1);
            T fp = dot(d1, d1) + dot(r, d2);
            if (f < (T)0) a = u; else if (f > (T)0) b = u; else break;
            T un = fp > (T)0 ? u - f / fp : (T)0.5 * (a + b);
            // closed bracket: a converged step that rounds onto u (= a or b)
            // must end the iteration, not trigger a bisection
            if (!(un >= a && un <= b)) un = (T)0.5 * (a + b);
            T du = un - u;
            u = un;
            if (fabs(du) <= Newt<T>::eps * ((T)1 + fabs(u))) break;
        }
        C.eval(u, r, d1, d2);
        T sp = dot(d1, d1);
        T fp = sp + dot(r, d2);
        kappa = sp > (T)0 ? fp / sp : (T)1;
        T d = dot(r, r);
        u_best = u;
        d_best = d;
        if (dlo < d_best) { u_best = lo; d_best = dlo; kappa = (T)1; }
        if (dhi < d_best) { u_best = hi; d_best = dhi; kappa = (T)1; }
        return;
    }
    u_best = dlo <= dhi ? lo : hi;
    d_best = dlo <= dhi ? dlo : dhi;
    T d0 = C.dist2(u0);
    if (d0 < d_best) { u_best = u0; d_best = d0; }
}

// Sample k of a piece's local parameter: k / (S-1), the last one exactly 1.
template <typename T>
__device__ __forceinline__ T sample_u(int k)
{
    return k == kSamples - 1 ? (T)1 : (T)k / (T)(kSamples - 1);
}

template <typename T>
__device__ __forceinline__ T norm3(const V3<T>& a) { return sqrt(dot(a, a)); }

// Minimum of one piece.  Rescan S samples; Newton from every local minimum of
// the samples; then every sample interval not covered by those brackets whose
// second-order lower bound  min(D_k, D_k+1) - M h^2 / 8  still reaches below
// the best value gets a Newton solve of its own (M >= |D''| = 2(|C'|^2 +
// r.C'') from the hodograph control polygons), so the minimum over the piece
// is certified, not only the sampled one.  Returns squared distance, u, kappa.
// One unrolled pass produces bit masks; the Newton solves run in compact loops
// over the set bits, which keeps the kernels small.
template <typename T>
__device__ void piece_min(const Cubic<T>& C, T& u_out, T& d_out, T& k_out)
{
    // C' has Bezier control points a1, a1 + a2, a1 + 2 a2 + 3 a3; C'' has 2 a2, 2 a2 + 6 a3
    const V3<T> h1 = {C.a1.x + C.a2.x, C.a1.y + C.a2.y, C.a1.z + C.a2.z};
    const V3<T> h2 = {C.a1.x + (T)2 * C.a2.x + (T)3 * C.a3.x, C.a1.y + (T)2 * C.a2.y + (T)3 * C.a3.y,
                      C.a1.z + (T)2 * C.a2.z + (T)3 * C.a3.z};
    const V3<T> g0 = {(T)2 * C.a2.x, (T)2 * C.a2.y, (T)2 * C.a2.z};
    const V3<T> g1 = {g0.x + (T)6 * C.a3.x, g0.y + (T)6 * C.a3.y, g0.z + (T)6 * C.a3.z};
    const T L1 = fmax(norm3(C.a1), fmax(norm3(h1), norm3(h2)));
    const T L2 = fmax(norm3(g0), norm3(g1));
    const T h = (T)1 / (T)(kSamples - 1);

    T D[kSamples];
    T dmax = (T)0, dmin = (T)INFINITY;
#pragma unroll
    for (int k = 0; k < kSamples; ++k) {
        D[k] = C.dist2(sample_u<T>(k));
        dmax = fmax(dmax, D[k]);
        dmin = fmin(dmin, D[k]);
    }
    const T rmax = sqrt(dmax) + L1 * h;
    const T gap = (T)2 * (L1 * L1 + rmax * L2) * h * h * (T)0.125;
    uint32_t lm = 0, chk = 0;  // local minima of the samples; intervals whose bound reaches the sampled minimum
#pragma unroll
    for (int k = 0; k < kSamples; ++k) {
        const bool m = (k == 0 || D[k] <= D[k - 1]) && (k == kSamples - 1 || D[k] <= D[k + 1]);
        lm |= (uint32_t)m << k;
        if (k < kSamples - 1) chk |= (uint32_t)(fmin(D[k], D[k + 1]) - gap < dmin) << k;
    }
    u_out = (T)0; d_out = (T)INFINITY; k_out = (T)1;
    uint32_t covered = 0;  // bit k: interval (k, k+1) lies inside a refined bracket
    for (uint32_t bits = lm; bits; bits &= bits - 1) {
        const int k = __builtin_ctz(bits);
        const int a = k > 0 ? k - 1 : 0, b = k < kSamples - 1 ? k + 1 : kSamples - 1;
        T ub, db, kb;
        newton_min(C, sample_u<T>(a), sample_u<T>(b), sample_u<T>(k), ub, db, kb);
        if (db < d_out) { d_out = db; u_out = ub; k_out = kb; }
        covered |= ((1u << b) - 1u) & ~((1u << a) - 1u);
    }
    const T best = d_out * ((T)1 - (T)(sizeof(T) == 4 ? 8e-6 : 2e-14));
    for (uint32_t bits = chk & ~covered; bits; bits &= bits - 1) {
        const int k = __builtin_ctz(bits);
        const T ua = sample_u<T>(k), ub_ = sample_u<T>(k + 1);
        if (fmin(C.dist2(ua), C.dist2(ub_)) - gap < best) {
            T ub, db, kb;
            newton_min(C, ua, ub_, (T)0.5 * (ua + ub_), ub, db, kb);
            if (db < d_out) { d_out = db; u_out = ub; k_out = kb; }
        }
    }
}

// Exact degree-p span in local power form: C(v) = sum_j c_j v^j, v in [0,1].
__device__ __forceinline__ void span_eval(const double* cf, int p, double v, const double* q, double* r, double* d1, double* d2)
{
    double x[3], y[3], z[3];
    for (int c = 0; c < 3; ++c) { x[c] = cf[3 * p + c]; y[c] = 0.0; z[c] = 0.0; }
    for (int j = p - 1; j >= 0; --j)
        for (int c = 0; c < 3; ++c) {
            z[c] = z[c] * v + 2.0 * y[c];
            y[c] = y[c] * v + x[c];
            x[c] = x[c] * v + cf[3 * j + c];
        }
    for (int c = 0; c < 3; ++c) { r[c] = x[c] - q[c]; d1[c] = y[c]; d2[c] = z[c]; }
}

// FP64 Newton on the exact span from global parameter t0; returns (t, dist, kappa).
__device__ __forceinline__ void polish(const DevGeom& G, const DCurve& cv, int32_t span, double t0, const double* q, double& t_out,
                       double& d_out, double& k_out)
{
    const int p = cv.degree;
    const double tq = G.spant[2 * span], tq1 = G.spant[2 * span + 1];
    const double h = tq1 - tq;
    const double* cf = G.coef + cv.coef_off + (int64_t)(span - cv.span_off) * 3 * (p + 1);
    double v = (t0 - tq) / h;
    v = fmin(fmax(v, 0.0), 1.0);
    double r[3], d1[3], d2[3];
    span_eval(cf, p, v, q, r, d1, d2);
    double best_v = v, best_d = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    for (int it = 0; it < 12; ++it) {
        double f = r[0] * d1[0] + r[1] * d1[1] + r[2] * d1[2];
        double fp = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2] + r[0] * d2[0] + r[1] * d2[1] + r[2] * d2[2];
        if (!(fp > 0.0)) break;
        double vn = fmin(fmax(v - f / fp, 0.0), 1.0);
        double dv = vn - v;
        v = vn;
        span_eval(cf, p, v, q, r, d1, d2);
        double d = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (d <= best_d) { best_d = d; best_v = v; }
        if (fabs(dv) <= 1e-15) break;
    }
    span_eval(cf, p, best_v, q, r, d1, d2);
    double sp = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
    double fp = sp + r[0] * d2[0] + r[1] * d2[1] + r[2] * d2[2];
    k_out = sp > 0.0 ? fp / sp : 1.0;
    t_out = (best_v == 1.0) ? tq1 : tq + best_v * h;
    d_out = sqrt(best_d);
}

struct Cand {
    double t, d2;   // FP64 global parameter, squared distance (refine precision)
    double kappa;
    double t_err;   // bound on the parameter error left by the refine precision
    int32_t seg;
};

template <typename T>
struct Eps;
template <>
struct Eps<float> {
    static constexpr double v = 5.97e-8;  // 2^-24
};
template <>
struct Eps<double> {
    static constexpr double v = 1.12e-16;  // 2^-53
};

// Bound on the parameter error the refine precision leaves at u: rounding of
// the terms of f = r.C' (magnitude <= scale * |C'|) moves the root by about
// 8 eps scale / (|C'| kappa) in u.
template <typename T>
__device__ double param_error(const Cubic<T>& C, T u, T k, double ta, double tb)
{
    V3<T> r, d1, d2;
    C.eval(u, r, d1, d2);
    const double sp = sqrt((double)dot(d1, d1));
    const double scale = sqrt((double)dot(C.a0, C.a0)) + sqrt((double)dot(C.a1, C.a1)) +
                         sqrt((double)dot(C.a2, C.a2)) + sqrt((double)dot(C.a3, C.a3));
    const double kap = fabs((double)k);
    return (sp > 0.0 && kap > 0.0) ? 8.0 * Eps<T>::v * scale / (sp * kap) * (tb - ta) : 1.0;
}

__device__ __forceinline__ void cand_select(bool c, const Cand& a, Cand& dst)
{
    dst.t = c ? a.t : dst.t;
    dst.d2 = c ? a.d2 : dst.d2;
    dst.kappa = c ? a.kappa : dst.kappa;
    dst.t_err = c ? a.t_err : dst.t_err;
    dst.seg = c ? a.seg : dst.seg;
}

// Keep the two best candidates (squared distance, then parameter); field-wise
// selects keep the candidates in registers.
__device__ __forceinline__ void top2(const Cand& x, Cand& b1, Cand& b2)
{
    const bool first = x.d2 < b1.d2 || (x.d2 == b1.d2 && x.t < b1.t);
    const bool second = !first && x.d2 < b2.d2;
    cand_select(first, b1, b2);
    cand_select(second, x, b2);
    cand_select(first, x, b1);
}

__device__ __forceinline__ Cand make_cand(const DevGeom& G, int64_t s, double u, double d2, double kappa, double t_err)
{
    const double ta = G.segt[2 * s], tb = G.segt[2 * s + 1];
    Cand x;
    x.t = (u == 1.0) ? tb : ta + u * (tb - ta);
    x.d2 = d2;
    x.kappa = kappa;
    x.t_err = t_err;
    x.seg = (int32_t)s;
    return x;
}

template <typename T>
__device__ void consider(const DevGeom& G, const DCurve& cv, int64_t s, const double* q, Cand& b1, Cand& b2)
{
    Cubic<T> C;
    load_cubic(G, cv, s, q, C);
    T u, d, k;
    piece_min(C, u, d, k);
    const double ta = G.segt[2 * s], tb = G.segt[2 * s + 1];
    top2(make_cand(G, s, (double)u, (double)d, (double)k, param_error(C, u, k, ta, tb)), b1, b2);
}

// Minimum sampled squared distance of a piece (the full-scan prune).
template <typename T>
__device__ T piece_sample_min(const DevGeom& G, const DCurve& cv, int64_t s, const double* q)
{
    Cubic<T> C;
    load_cubic(G, cv, s, q, C);
    T m = C.dist2((T)0);
    for (int k = 1; k < kSamples; ++k) m = fmin(m, C.dist2(sample_u<T>(k)));
    return m;
}

// Decide one query from its two best candidates: FP64 polish on the exact span
// where the cubic is an approximation (p >= 4), the minimiser is near-tangent,
// the refine precision cannot certify the parameter to 1e-8, or the runner-up
// is within the tie margin; then write t, distance, piece and flags.
template <typename T>
__device__ __forceinline__ void finish(const DevGeom& G, const DCurve& cv, const double* q, const Cand& b1, const Cand& b2,
                       uint32_t flags, double tie_rel, int invert, int32_t qi, const Outs& o)
{
    const double d1 = sqrt(b1.d2), d2 = sqrt(b2.d2);
    const double margin = 2.0 * cv.tol_eff + (sizeof(T) == 4 ? 2e-6 : 1e-12) * (d1 + cv.diag) + tie_rel * cv.diag;
    const bool tie = b2.d2 < INFINITY && (d2 - d1) <= margin;
    const bool approx = cv.degree >= 4;
    const bool illc = b1.kappa < 1e-2;
    const bool coarse = b1.t_err > 1e-8;
    double t, dist, kap = b1.kappa;
    int32_t seg = b1.seg;
    if (approx || tie || illc || coarse) {
        flags |= MREP_F_POLISHED;
        polish(G, cv, G.segspan[b1.seg], b1.t, q, t, dist, kap);
        if (tie) {
            double tt, dd, kk;
            polish(G, cv, G.segspan[b2.seg], b2.t, q, tt, dd, kk);
            if (dd < dist || (dd == dist && tt < t)) { t = tt; dist = dd; kap = kk; seg = b2.seg; }
            if (fabs(dd - dist) <= tie_rel * cv.diag && fabs(tt - t) > 1e-6) flags |= MREP_F_NEAR_TIE;
        }
    } else {
        // exact cubic (p <= 3): FP64 distance at the refined parameter
        Cubic<double> C;
        load_cubic(G, cv, seg, q, C);
        const double ta = G.segt[2 * seg], tb = G.segt[2 * seg + 1];
        double u = (b1.t - ta) / (tb - ta);
        u = fmin(fmax(u, 0.0), 1.0);
        t = b1.t;
        dist = sqrt(C.dist2(u));
    }
    if (kap < 1e-2) flags |= MREP_F_ILL_COND;
    // piece holding t: [t_a, t_b), the last piece closed
    {
        const int64_t s0 = cv.seg_off, s1 = cv.seg_off + cv.n_seg - 1;
        int64_t s = seg;
        while (s > s0 && t < G.segt[2 * s]) --s;
        while (s < s1 && t >= G.segt[2 * s + 1]) ++s;
        seg = (int32_t)s;
    }
    const double dom0 = G.spant[2 * cv.span_off], dom1 = G.spant[2 * (cv.span_off + cv.n_span - 1) + 1];
    if (t <= dom0 + 1e-12 * (dom1 - dom0) || t >= dom1 - 1e-12 * (dom1 - dom0)) flags |= MREP_F_ENDPOINT;
    if (invert && dist > cv.tol_user) flags |= MREP_F_OFFCURVE;
    o.t[qi] = t;
    o.d[qi] = dist;
    o.s[qi] = (int32_t)(seg - cv.seg_off);
    o.f[qi] = flags;
}

__device__ __forceinline__ Cand empty_cand(const DCurve& cv)
{
    Cand b;
    b.d2 = INFINITY; b.t = 0.0; b.seg = (int32_t)cv.seg_off; b.kappa = 1.0; b.t_err = 0.0;
    return b;
}

}  // namespace mrep
