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
    __device__ T size() const
    {
        return fabs(a0.x) + fabs(a0.y) + fabs(a0.z) + fabs(a1.x) + fabs(a1.y) + fabs(a1.z) + fabs(a2.x) + fabs(a2.y) +
               fabs(a2.z) + fabs(a3.x) + fabs(a3.y) + fabs(a3.z);
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
    static constexpr T stat = (T)1e-5;  // |r.C'| <= stat |r||C'|: stationary to rounding
};
template <>
struct Newt<double> {
    static constexpr int iters = 40;
    static constexpr double eps = 1e-15;
    static constexpr double stat = 1e-12;
};

// Square root for bounds, scales and conditioning: in FP32 the raw hardware
// one (<= 1 ulp; the correctly rounded one costs a dozen instructions with its
// range scaling), in FP64 the library's.
__device__ __forceinline__ float bsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double bsqrt(double x) { return sqrt(x); }
// Quotient for Newton steps and conditioning: in FP32 through the hardware
// reciprocal (<= 1 ulp; the iteration corrects its own step), in FP64 exact.
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double qdiv(double a, double b) { return a / b; }

// unit roundoff of the refine precision
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

template <typename T>
__device__ __forceinline__ T norm3(const V3<T>& a) { return bsqrt(dot(a, a)); }

// kappa = f'/|C'|^2 at a bracket end where f = r.C' vanishes to rounding (a
// stationary minimiser that lies on the end, e.g. on a piece joint); 1 at an
// end the distance leaves with a slope (the end conditions the minimum)
template <typename T>
__device__ __forceinline__ T end_kappa(const V3<T>& r, const V3<T>& d1, const V3<T>& d2)
{
    const T sp = dot(d1, d1), f = dot(r, d1);
    return (sp > (T)0 && fabs(f) <= Newt<T>::stat * bsqrt(dot(r, r) * sp)) ? qdiv(sp + dot(r, d2), sp) : (T)1;
}

// Minimum of |C(u) - q|^2 on [lo, hi] near the sample u0: safeguarded Newton on
// f = r.C' when f changes sign on the bracket; otherwise the better bracket end.
// loc (nullable) tells whether the result stands for a local minimum of the
// piece: a bracket over which f changes sign holds one (the result may be a
// bracket end where rounding made it lower than the stationary point), as does
// a piece end (u = 0 or 1) where the distance grows into the piece; an
// interior bracket end without a sign change of f does not.
template <typename T>
__device__ __forceinline__ void newton_min(const Cubic<T>& C, T lo, T hi, T u0, T& u_best, T& d_best, T& kappa,
                                           bool* loc = nullptr)
{
    V3<T> r, d1, d2;
    C.eval(lo, r, d1, d2);
    T flo = dot(r, d1), dlo = dot(r, r);
    const T klo = end_kappa(r, d1, d2);
    C.eval(hi, r, d1, d2);
    T fhi = dot(r, d1), dhi = dot(r, r);
    const T khi = end_kappa(r, d1, d2);
    T u = u0;
    kappa = (T)1;
    if (flo < (T)0 && fhi > (T)0) {
        T a = lo, b = hi;
        for (int it = 0; it < Newt<T>::iters; ++it) {
            C.eval(u, r, d1, d2);
            T f = dot(r, d1);
            T fp = dot(d1, d1) + dot(r, d2);
            if (f < (T)0) a = u; else if (f > (T)0) b = u; else break;
            T un = fp > (T)0 ? u - qdiv(f, fp) : (T)0.5 * (a + b);
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
        kappa = sp > (T)0 ? qdiv(fp, sp) : (T)1;
        T d = dot(r, r);
        u_best = u;
        d_best = d;
        // a bracket end replaces the stationary point only when it is lower by
        // more than the rounding of the squared distances (about 8 eps S |r|,
        // S the coefficients' size): within that, the end is only rounding
        // lower, and taking it moved an interior minimum a few 1e-5 from a piece
        // end onto the end (a parameter error the FP64 polish never saw).  S, the
        // sum of the coefficients' absolute components, bounds |C - q| and each
        // of its terms on [0, 1].
        // (in FP64 the rounding is far below any parameter tolerance: no margin,
        // which also keeps the FP64 full scan within 256 registers)
        T nz = (T)0;
        if constexpr (sizeof(T) == 4) {
            const T S = C.size();
            nz = (T)(16.0 * Eps<T>::v) * S * (bsqrt(d) + S);
        }
        if (dlo < d_best - nz) { u_best = lo; d_best = dlo; kappa = klo; }
        if (dhi < d_best - nz) { u_best = hi; d_best = dhi; kappa = khi; }
        if (loc) *loc = true;
        return;
    }
    u_best = dlo <= dhi ? lo : hi;
    d_best = dlo <= dhi ? dlo : dhi;
    kappa = dlo <= dhi ? klo : khi;
    T d0 = C.dist2(u0);
    if (d0 < d_best) { u_best = u0; d_best = d0; kappa = (T)1; }
    if (loc) *loc = (u_best == (T)0 && flo >= (T)0) || (u_best == (T)1 && fhi <= (T)0);
}

// Sample k of a piece's local parameter: k / (S-1), the last one exactly 1.
template <typename T>
__device__ __forceinline__ T sample_u(int k)
{
    return k == kSamples - 1 ? (T)1 : (T)k / (T)(kSamples - 1);
}

// parameters of a piece closer than this are one minimum, not two
constexpr float kDistinctU = 1e-4f;

// Keep the best and the second best of the piece's local minima.  Two points
// are two minima only when they are kDistinctU apart with a barrier between
// them (the distance at the midpoint above both, beyond rounding): solves that
// stop at different points of one shallow minimum are one minimum.  Only a
// local minimum of the piece (loc; l1 for the current best) can become the
// second: a bracket end that the certification pass reached is a bound.
template <typename T>
__device__ __forceinline__ void keep2(const Cubic<T>& C, T u, T d, T k, bool loc, T& u1, T& d1, T& k1, bool& l1, T& u2,
                                      T& d2)
{
    bool apart = fabs(u - u1) > (T)kDistinctU;
    if (apart && d1 < (T)INFINITY)
        apart = C.dist2((T)0.5 * (u + u1)) > fmax(d, d1) * ((T)1 + (T)(sizeof(T) == 4 ? 4e-6 : 1e-13));
    if (d < d1) {
        if (l1 && apart) { u2 = u1; d2 = d1; }
        u1 = u; d1 = d; k1 = k; l1 = loc;
    } else if (loc && d < d2 && apart) {
        u2 = u; d2 = d;
    }
}

// Minimum of one piece.  Rescan S samples; Newton from every local minimum of
// the samples; then every sample interval not covered by those brackets whose
// second-order lower bound  min(D_k, D_k+1) - M h^2 / 8  still reaches below
// the best value gets a Newton solve of its own (M >= |D''| = 2(|C'|^2 +
// r.C'') from the hodograph control polygons), so the minimum over the piece
// is certified, not only the sampled one.  Returns squared distance, u, kappa,
// and the second best distinct local minimum found (u2, d2; d2 = inf when
// none), which a tie between two minima of one piece needs.  One unrolled
// pass produces bit masks; the Newton solves run in compact loops over the
// set bits, which keeps the kernels small.
template <typename T>
__device__ void piece_min(const Cubic<T>& C, T& u_out, T& d_out, T& k_out, T& u2_out, T& d2_out,
                          T lim2 = (T)INFINITY)
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
    const T rmax = bsqrt(dmax) + L1 * h;
    const T gap = (T)2 * (L1 * L1 + rmax * L2) * h * h * (T)0.125;
    uint32_t lm = 0, chk = 0;  // local minima of the samples; intervals whose bound reaches the sampled minimum
#pragma unroll
    for (int k = 0; k < kSamples; ++k) {
        const bool m = (k == 0 || D[k] <= D[k - 1]) && (k == kSamples - 1 || D[k] <= D[k + 1]);
        lm |= (uint32_t)m << k;
        if (k < kSamples - 1) chk |= (uint32_t)(fmin(D[k], D[k + 1]) - gap < dmin) << k;
    }
    u_out = (T)0; d_out = (T)INFINITY; k_out = (T)1;
    u2_out = (T)0; d2_out = (T)INFINITY;
    // the piece's squared distance stays above dmin - gap: beyond the caller's
    // limit (lim2), no point of it can be the minimum or a runner-up that
    // counts, so it is not refined (reported as its sampled minimum, interior)
    if ((dmin - gap) * ((T)1 - (T)(sizeof(T) == 4 ? 8e-6 : 2e-14)) > lim2) {
        u_out = (T)0.5;
        d_out = dmin;
        return;
    }
    bool l1 = false;
    uint32_t covered = 0;  // bit k: interval (k, k+1) lies inside a refined bracket
    for (uint32_t bits = lm; bits; bits &= bits - 1) {
        const int k = __builtin_ctz(bits);
        const int a = k > 0 ? k - 1 : 0, b = k < kSamples - 1 ? k + 1 : kSamples - 1;
        T ub, db, kb;
        newton_min(C, sample_u<T>(a), sample_u<T>(b), sample_u<T>(k), ub, db, kb);
        // a local minimum of the samples: the bracket holds a local minimum of the piece
        keep2(C, ub, db, kb, true, u_out, d_out, k_out, l1, u2_out, d2_out);
        covered |= ((1u << b) - 1u) & ~((1u << a) - 1u);
    }
    const T best = d_out * ((T)1 - (T)(sizeof(T) == 4 ? 8e-6 : 2e-14));
    for (uint32_t bits = chk & ~covered; bits; bits &= bits - 1) {
        const int k = __builtin_ctz(bits);
        const T ua = sample_u<T>(k), ub_ = sample_u<T>(k + 1);
        if (fmin(C.dist2(ua), C.dist2(ub_)) - gap < best) {
            T ub, db, kb;
            bool loc;
            newton_min(C, ua, ub_, (T)0.5 * (ua + ub_), ub, db, kb, &loc);
            keep2(C, ub, db, kb, loc, u_out, d_out, k_out, l1, u2_out, d2_out);
        }
    }
}
template <typename T>
__device__ __forceinline__ void piece_min(const Cubic<T>& C, T& u_out, T& d_out, T& k_out)
{
    T u2, d2;
    piece_min(C, u_out, d_out, k_out, u2, d2);
}

// Bernstein sums without a local array: sum_{i=0..m} C(m,i) v^i (1-v)^{m-i} c_i
// with c_i = get(i), by Horner in r = v/(1-v) for v <= 1/2 and in (1-v)/v
// above, scaled by (1-v)^m or v^m.  The ratio stays in [0, 1], and the large
// binomial terms of the intermediate sum are scaled back by that power, so the
// rounding stays of the order of the largest |c_i|.  Binomials are exact
// integers updated in place (m <= 32).
template <typename F>
__device__ __forceinline__ double bern_sum(int m, double v, F get)
{
    if (m == 0) return get(0);
    const double s = 1.0 - v;
    double acc, bin = 1.0, pw = 1.0;
    if (v <= 0.5) {
        const double r = v / s;
        acc = get(m);
        for (int i = m - 1; i >= 0; --i) {
            bin = bin * (double)(i + 1) / (double)(m - i);
            acc = acc * r + bin * get(i);
        }
        for (int i = 0; i < m; ++i) pw *= s;
    } else {
        const double r = s / v;
        acc = get(0);
        for (int i = 1; i <= m; ++i) {
            bin = bin * (double)(m - i + 1) / (double)i;
            acc = acc * r + bin * get(i);
        }
        for (int i = 0; i < m; ++i) pw *= v;
    }
    return acc * pw;
}

// X, X', X'' at v of component c of a degree-p Bezier span stored with `stride`
// doubles per point (3: Bezier points, 4: homogeneous points of a rational span).
__device__ __forceinline__ void bern_eval(const double* cf, int stride, int c, int p, double v, double& x, double& x1,
                                          double& x2)
{
    x = bern_sum(p, v, [&](int i) { return cf[stride * i + c]; });
    x1 = p >= 1 ? (double)p * bern_sum(p - 1, v, [&](int i) { return cf[stride * (i + 1) + c] - cf[stride * i + c]; })
                : 0.0;
    x2 = p >= 2 ? (double)(p * (p - 1)) * bern_sum(p - 2, v, [&](int i) {
             return (cf[stride * (i + 2) + c] - cf[stride * (i + 1) + c]) - (cf[stride * (i + 1) + c] - cf[stride * i + c]);
         })
                : 0.0;
}

// Exact degree-p span as Bezier points (p > MREP_POWER_MAX_DEGREE): C, C', C''.
__device__ __forceinline__ void span_eval_bezier(const double* cf, int p, double v, const double* q, double* r,
                                                 double* d1, double* d2)
{
    for (int c = 0; c < 3; ++c) {
        double x, x1, x2;
        bern_eval(cf, 3, c, p, v, x, x1, x2);
        r[c] = x - q[c];
        d1[c] = x1;
        d2[c] = x2;
    }
}

// Exact rational span as homogeneous Bezier points (w x, w y, w z, w): X, X',
// X'' and W, W', W'' at v, then the quotient rule  C = X/W,  C' = (X' - C W')/W,
// C'' = (X'' - 2 C' W' - C W'')/W.
__device__ __forceinline__ void span_eval_rational(const double* cf, int p, double v, const double* q, double* r,
                                                   double* d1, double* d2)
{
    double W, W1, W2;
    bern_eval(cf, 4, 3, p, v, W, W1, W2);
    for (int c = 0; c < 3; ++c) {
        double x, x1, x2;
        bern_eval(cf, 4, c, p, v, x, x1, x2);
        const double C = x / W;
        const double C1 = (x1 - C * W1) / W;
        r[c] = C - q[c];
        d1[c] = C1;
        d2[c] = (x2 - 2.0 * C1 * W1 - C * W2) / W;
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

// The exact form of one span of curve cv, and its evaluation (power form,
// Bezier points, or homogeneous Bezier points of a rational curve).
__device__ __forceinline__ const double* span_coef(const DevGeom& G, const DCurve& cv, int64_t span)
{
    return G.coef + cv.coef_off + (span - cv.span_off) * (int64_t)(cv.rational ? 4 : 3) * (cv.degree + 1);
}
// kGen: the geometry has spans beyond the power form (degree above
// MREP_POWER_MAX_DEGREE or rational curves); kernels are instantiated both
// ways so that the common geometry does not carry the Bernstein and rational
// evaluations in its registers.
template <bool kGen>
__device__ __forceinline__ void span_eval_cv(const DCurve& cv, const double* cf, double v, const double* q, double* r,
                                             double* d1, double* d2)
{
    if constexpr (kGen) {
        if (cv.rational) {
            span_eval_rational(cf, cv.degree, v, q, r, d1, d2);
            return;
        }
        if (cv.degree > MREP_POWER_MAX_DEGREE) {
            span_eval_bezier(cf, cv.degree, v, q, r, d1, d2);
            return;
        }
    }
    span_eval(cf, cv.degree, v, q, r, d1, d2);
}

// FP64 Newton on the exact span from global parameter t0; returns (t, dist,
// kappa).  Newton on a span keeps its best iterate; when that lies on an end of
// the span that is an interior joint of the curve, the polish continues on the
// neighbouring span from the joint (at most 3 hops) and keeps the result only
// if it goes lower: the result is then a local minimum of the exact curve, not
// of one span.  One loop with one evaluation site keeps the kernels that inline
// this small (the evaluation may be Bernstein or rational).
template <bool kGen>
__device__ __forceinline__ void polish(const DevGeom& G, const DCurve& cv, int32_t span, double t0, const double* q,
                                       double& t_out, double& d_out, double& k_out, double* sp_out = nullptr,
                                       bool* conv_out = nullptr)
{
    const int32_t sp0 = (int32_t)cv.span_off, sp1 = (int32_t)(cv.span_off + cv.n_span - 1);
    double v = (t0 - G.spant[2 * span]) / (G.spant[2 * span + 1] - G.spant[2 * span]);
    v = fmin(fmax(v, 0.0), 1.0);
    // best over all spans visited, and best of the current span
    double best_v = v, best_d = INFINITY, best_k = 1.0, best_sp = 0.0;
    int32_t best_span = span;
    bool best_c = false;
    double cur_v = v, cur_d = INFINITY, cur_k = 1.0, cur_sp = 0.0;
    bool cur_c = false;
    int hop = 0, it = 0;
    bool last = false;  // the step just taken was below 1e-12: this evaluation ends the span
    // the coordinates' scale: the evaluation rounds at about 1e-16 of it, so a
    // step that moves the point by less than 1e-15 of it is rounding noise
    const double scale = fmax(fabs(q[0]), fmax(fabs(q[1]), fabs(q[2]))) + cv.diag;
    for (int guard = 0; guard < 64; ++guard) {
        double r[3], d1[3], d2[3];
        span_eval_cv<kGen>(cv, span_coef(G, cv, span), v, q, r, d1, d2);
        const double d = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const double f = r[0] * d1[0] + r[1] * d1[1] + r[2] * d1[2];
        const double sp = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
        const double fp = sp + r[0] * d2[0] + r[1] * d2[1] + r[2] * d2[2];
        if (d <= cur_d) {
            cur_d = d;
            cur_v = v;
            // conditioning of a stationary minimiser (inside the span, or where f
            // vanishes); a minimum held at an end or a corner without a
            // stationary point is conditioned by the end: 1.  Near a centre of
            // curvature Newton converges only linearly, so an interior iterate
            // counts as stationary without a residual test.
            cur_c = fabs(f) <= 1e-9 * sqrt(sp) * (sqrt(d) + cv.diag);
            const bool stationary = (v > 0.0 && v < 1.0) || cur_c;
            cur_k = (sp > 0.0 && stationary) ? fp / sp : 1.0;
            cur_sp = sp;
        }
        bool done_span = !(fp > 0.0) || it >= 12 || last;
        if (!done_span) {
            const double vn = fmin(fmax(v - f / fp, 0.0), 1.0);
            const double step = fabs(vn - v);
            // Converged: a step that moves the point by less than the rounding
            // noise ends the span at the evaluated point; a step below 1e-12 of
            // the span is taken and evaluated once more (Newton's next error is
            // about its square).  A fixed 1e-15 in v lies below the noise on short
            // spans far from the origin, where Newton then ran to its cap.
            done_span = step * sqrt(sp) <= 1e-15 * scale;
            if (!done_span) {
                last = step <= 1e-12;
                v = vn;
                ++it;
                continue;
            }
        }
        // this span is done: keep it if it went lower (always for the first span)
        if (hop > 0 && !(cur_d < best_d)) break;
        best_v = cur_v; best_d = cur_d; best_k = cur_k; best_span = span; best_sp = cur_sp; best_c = cur_c;
        if (hop >= 3) break;
        if (best_v == 0.0 && span > sp0) { --span; v = 1.0; }
        else if (best_v == 1.0 && span < sp1) { ++span; v = 0.0; }
        else break;
        ++hop;
        it = 0;
        last = false;
        cur_d = INFINITY;
    }
    const double ta = G.spant[2 * best_span], tb = G.spant[2 * best_span + 1];
    k_out = best_k;
    t_out = (best_v == 1.0) ? tb : ta + best_v * (tb - ta);
    d_out = sqrt(best_d);
    if (sp_out) *sp_out = best_sp / ((tb - ta) * (tb - ta));  // |C'|^2 in the curve's parameter
    if (conv_out) *conv_out = best_c;
}

struct Cand {
    double t, d2;   // FP64 global parameter, squared distance (refine precision)
    float kappa;    // conditioning at the candidate (only compared with 1e-2)
    float t_err;    // bound on the parameter error left by the refine precision (compared with 1e-8)
    int32_t seg;
    int32_t across; // a piece end at an interior joint where the distance falls into the neighbour
    int32_t end;    // bits 0-1: 1 at the piece's start (u = 0), 2 at its end (u = 1), else 0;
                    // bit 2 (kSecond): the piece's second local minimum, not its minimum
};
constexpr int32_t kSecond = 4;

// Bound on the parameter error the refine precision leaves at u: rounding of
// the terms of f = r.C' (magnitude <= scale * |C'|) moves the root by about
// 8 eps scale / (|C'| kappa) in u; an unconverged solve adds |f| / f'.
template <typename T>
__device__ double param_error(const Cubic<T>& C, T u, T k, double ta, double tb)
{
    V3<T> r, d1, d2;
    C.eval(u, r, d1, d2);
    const double sp = (double)norm3(d1);
    const double scale = (double)(norm3(C.a0) + norm3(C.a1) + norm3(C.a2) + norm3(C.a3));
    const double kap = fabs((double)k);
    if (!(sp > 0.0 && kap > 0.0)) return 1.0;
    double e = 8.0 * Eps<T>::v * scale / (sp * kap);
    // at an interior point, plus the Newton correction that is left (|f| / f'):
    // a solve that ended on its iteration cap or after bisection steps is
    // farther from the root than the rounding alone (a piece end is exact)
    if (u > (T)0 && u < (T)1) e += fabs((double)dot(r, d1)) / (kap * sp * sp);
    return e * (tb - ta);
}

// x is the joint it shares with candidate y's piece, and y is that piece's
// minimum (false when y is empty or a second minimum)
__device__ __forceinline__ bool on_piece(const Cand& x, const Cand& y)
{
    const int32_t e = x.end & 3;
    return y.d2 < INFINITY && !(y.end & kSecond) && ((e == 1 && x.seg == y.seg + 1) || (e == 2 && x.seg == y.seg - 1));
}

// Keep the two best candidates (squared distance, then parameter); field-wise
// selects keep the candidates in registers.  A candidate at the joint it shares
// with the piece whose minimum is the best is no lower than that minimum and is
// no other local minimum of the curve: it is dropped, and when the best itself
// sits on the piece whose minimum the new candidate is, the new one replaces it
// without becoming the runner-up (a piece's second local minimum has no such
// bound, and takes its place by distance alone).  Without this, the two pieces' copies of one minimum (or a
// joint next to it) would hold both places and push a genuine second minimum
// out of the tie test.  A candidate whose distance falls into the neighbouring
// piece (across) is no local minimum of the curve either: it may hold the first
// place until a lower candidate comes, but it never becomes the runner-up.
__device__ __forceinline__ void top2(const Cand& x, Cand& b1, Cand& b2)
{
    // decisions first, then every field of both places written unconditionally
    // from selects: branches that store into b1 or b2 get merged by the compiler
    // into one store through a pointer chosen at run time, which keeps both
    // candidates in scratch memory
    const bool live = x.d2 < INFINITY && !on_piece(x, b1);
    const bool repl = live && on_piece(b1, x);
    const bool first = live && (repl || x.d2 < b1.d2 || (x.d2 == b1.d2 && x.t < b1.t));
    const bool demote = first && !repl && !b1.across;
    const bool second = live && !first && !x.across && !on_piece(x, b2) &&
                        (x.d2 < b2.d2 || (x.d2 == b2.d2 && x.t < b2.t));
    const bool clear2 = repl && on_piece(b2, x);  // a runner-up on the new best's piece goes too
    Cand n1, n2;
    n2.t = demote ? b1.t : (second ? x.t : b2.t);
    n2.d2 = clear2 ? (double)INFINITY : (demote ? b1.d2 : (second ? x.d2 : b2.d2));
    n2.kappa = demote ? b1.kappa : (second ? x.kappa : b2.kappa);
    n2.t_err = demote ? b1.t_err : (second ? x.t_err : b2.t_err);
    n2.seg = demote ? b1.seg : (second ? x.seg : b2.seg);
    n2.across = demote ? b1.across : (second ? x.across : b2.across);
    n2.end = demote ? b1.end : (second ? x.end : b2.end);
    n1.t = first ? x.t : b1.t;
    n1.d2 = first ? x.d2 : b1.d2;
    n1.kappa = first ? x.kappa : b1.kappa;
    n1.t_err = first ? x.t_err : b1.t_err;
    n1.seg = first ? x.seg : b1.seg;
    n1.across = first ? x.across : b1.across;
    n1.end = first ? x.end : b1.end;
    b1 = n1;
    b2 = n2;
}

// Piece s's candidate at its end u (0 or 1) when that end is an interior joint
// of the curve: true when the squared distance keeps falling into the
// neighbouring piece (its (C - q).C' at the joint, from the FP64 control points,
// points back across), so the end is not a local minimum of the curve.
__device__ __forceinline__ bool end_falls_across(const DevGeom& G, const DCurve& cv, int64_t s, double u, const double* q)
{
    double r[3], d[3];
    bool left;
    if (u == 0.0 && s > cv.seg_off) {
        const double* P = G.gcp + (s - 1) * 12;  // previous piece: joint P3, tangent along P3 - P2
        for (int c = 0; c < 3; ++c) { r[c] = P[9 + c] - q[c]; d[c] = P[9 + c] - P[6 + c]; }
        left = true;
    } else if (u == 1.0 && s < cv.seg_off + cv.n_seg - 1) {
        const double* P = G.gcp + (s + 1) * 12;  // next piece: joint P0, tangent along P1 - P0
        for (int c = 0; c < 3; ++c) { r[c] = P[c] - q[c]; d[c] = P[3 + c] - P[c]; }
        left = false;
    } else {
        return false;
    }
    // f beyond 1e-12 |r| |d| in the falling direction, compared squared (no square root)
    const double f = r[0] * d[0] + r[1] * d[1] + r[2] * d[2];
    const double s2 = 1e-24 * (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    return (left ? f > 0.0 : f < 0.0) && f * f > s2;
}

__device__ __forceinline__ Cand make_cand(const DevGeom& G, int64_t s, double u, double d2, double kappa, double t_err)
{
    const double ta = G.segt[2 * s], tb = G.segt[2 * s + 1];
    Cand x;
    x.t = (u == 1.0) ? tb : ta + u * (tb - ta);
    x.d2 = d2;
    x.kappa = (float)kappa;
    x.t_err = (float)t_err;
    x.seg = (int32_t)s;
    x.across = 0;
    x.end = u == 0.0 ? 1 : (u == 1.0 ? 2 : 0);
    return x;
}

// a piece's second local minimum as a candidate (kappa 1, no parameter error:
// only its distance and t enter the tie test)
__device__ __forceinline__ Cand second_cand(Cand x)
{
    x.end |= kSecond;
    return x;
}

// make_cand, classifying a piece-end candidate at an interior joint
__device__ __forceinline__ Cand make_cand_q(const DevGeom& G, const DCurve& cv, int64_t s, double u, double d2,
                                            double kappa, double t_err, const double* q)
{
    Cand x = make_cand(G, s, u, d2, kappa, t_err);
    x.across = (u == 0.0 || u == 1.0) ? (int32_t)end_falls_across(G, cv, s, u, q) : 0;
    return x;
}

// Result of the refine for one (query, piece) pair, already in the curve's
// parameter and classified (piece end, distance falling across the joint), so
// that the finish reads one contiguous record per pair and no piece table.
struct alignas(16) PairRes {
    double t;       // the piece's minimum (global parameter)
    float dt2;      // its second local minimum t2 - t (when d2b < inf): within the piece, so FP32 keeps it to
                    // 6e-8 of the piece's parameter length (the runner-up's start, polished in FP64 when it counts)
    float d2;       // squared distance at t (refine precision)
    float kappa;
    float t_err;    // bound on the parameter error left by the refine precision
    float d2b;      // squared distance at t2; +inf when the piece has no second minimum
    uint32_t tag;   // bits 0-1: t at the piece's start (1) or end (2); bit 2: across; bits 4-6: the same for t2
};
static_assert(sizeof(PairRes) == 32, "PairRes layout");

__device__ __forceinline__ PairRes pair_result(const DevGeom& G, const DCurve& cv, int64_t s, const double* q,
                                               double u, double d, double k, double err, double u2, double d2)
{
    const Cand c1 = make_cand_q(G, cv, s, u, d, k, err, q);
    PairRes r;
    r.t = c1.t;
    r.d2 = (float)d;
    r.kappa = (float)k;
    r.t_err = (float)err;
    uint32_t tag = (uint32_t)c1.end | ((uint32_t)c1.across << 2);
    if (d2 < INFINITY) {
        const Cand c2 = make_cand_q(G, cv, s, u2, d2, 1.0, 0.0, q);
        r.dt2 = (float)(c2.t - c1.t);
        r.d2b = (float)d2;
        tag |= ((uint32_t)c2.end | ((uint32_t)c2.across << 2)) << 4;
    } else {
        r.dt2 = 0.f;
        r.d2b = INFINITY;
    }
    r.tag = tag;
    return r;
}

// candidate i of a pair record: its minimum (i = 0) or its second minimum (1)
__device__ __forceinline__ Cand pair_cand(const PairRes& r, int32_t seg, bool sec)
{
    Cand x;
    x.t = sec ? r.t + (double)r.dt2 : r.t;
    x.d2 = (double)(sec ? r.d2b : r.d2);
    x.kappa = sec ? 1.f : r.kappa;
    x.t_err = sec ? 0.f : r.t_err;
    x.seg = seg;
    const uint32_t tg = sec ? (r.tag >> 4) : r.tag;
    x.end = (int32_t)(tg & 3u) | (sec ? kSecond : 0);
    x.across = (int32_t)((tg >> 2) & 1u);
    return x;
}

template <typename T>
__device__ void consider(const DevGeom& G, const DCurve& cv, int64_t s, const double* q, Cand& b1, Cand& b2)
{
    Cubic<T> C;
    load_cubic(G, cv, s, q, C);
    T u, d, k, u2, d2;
    piece_min(C, u, d, k, u2, d2);
    const double ta = G.segt[2 * s], tb = G.segt[2 * s + 1];
    top2(make_cand_q(G, cv, s, (double)u, (double)d, (double)k, param_error(C, u, k, ta, tb), q), b1, b2);
    // a second minimum of the same piece: a runner-up candidate (its parameter
    // error does not matter: only its distance and t enter the tie test)
    if (d2 < (T)INFINITY) top2(second_cand(make_cand_q(G, cv, s, (double)u2, (double)d2, 1.0, 0.0, q)), b1, b2);
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
template <typename T, bool kGen>
__device__ __forceinline__ void finish(const DevGeom& G, const DCurve& cv, const double* q, const Cand& b1, const Cand& b2,
                       uint32_t flags, double tie_rel, int invert, int32_t qi, const Outs& o)
{
    const double d1 = sqrt(b1.d2), d2 = sqrt(b2.d2);
    const double margin = 2.0 * cv.tol_eff + (sizeof(T) == 4 ? 2e-6 : 1e-12) * (d1 + cv.diag) + tie_rel * cv.diag;
    const bool tie = b2.d2 < INFINITY && (d2 - d1) <= margin;
    const bool approx = cv.degree >= 4 || cv.rational;
    const bool illc = b1.kappa < 1e-2;
    const bool coarse = b1.t_err > 1e-8;
    double t, dist, kap = b1.kappa;
    int32_t seg = b1.seg;
    if (approx || tie || illc || coarse) {
        flags |= MREP_F_POLISHED;
        // the best, then (near tie) the runner-up, then (an ill-conditioned
        // best) two probes of its valley, through one polish site
        dist = INFINITY;
        t = b1.t;
        int nk = tie ? 2 : 1;
        bool conv = false;
        double h = 0.0;
        // the start points as scalars: selecting fields of b1 / b2 by the loop
        // index would make the compiler keep both candidates in scratch memory
        const double t1s = b1.t, t2s = b2.t;
        const int32_t s1s = b1.seg, s2s = b2.seg;
        for (int k = 0; k < nk; ++k) {
            const bool probe = k >= (tie ? 2 : 1);
            const int32_t ks = probe ? seg : (k ? s2s : s1s);
            int32_t span = G.segspan[ks];
            double t0 = k == 0 ? t1s : t2s;
            if (probe) {
                const double ta = G.spant[2 * span], tb = G.spant[2 * span + 1];
                t0 = fmin(fmax(t + ((k & 1) ? -h : h), ta), tb);
            }
            double tt, dd, kk, sp;
            bool cv_ok;
            polish<kGen>(G, cv, span, t0, q, tt, dd, kk, &sp, &cv_ok);
            if (k == 0) {
                t = tt; dist = dd; kap = kk; conv = cv_ok;
                // An ill-conditioned minimum lies in a flat valley that the refine
                // precision cannot resolve into one or two minima: probe it in FP64
                // from both sides, h = the parameter offset at which the distance
                // rises by the tie margin (f = d^2/2 grows by d m, f'' = kappa |C'|^2).
                if (kk < 1e-2 && kk > 0.0 && sp > 0.0 && conv) {
                    h = sqrt(2.0 * dd * tie_rel * cv.diag / (kk * sp));
                    nk += 2;
                }
                continue;
            }
            // both polished points are local minima of the exact curve (the polish
            // follows the distance across span joints): a second one within the
            // margin and apart in t is a near tie, whichever of the two wins (a
            // probe counts only where its Newton converged)
            if (fabs(dd - dist) <= tie_rel * cv.diag && fabs(tt - t) > 1e-6 && (!probe || cv_ok))
                flags |= MREP_F_NEAR_TIE;
            if (dd < dist || (dd == dist && tt < t)) { t = tt; dist = dd; kap = kk; seg = ks; }
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
    b.d2 = INFINITY; b.t = 0.0; b.seg = (int32_t)cv.seg_off; b.kappa = 1.f; b.t_err = 0.f; b.across = 0; b.end = 0;
    return b;
}

}  // namespace mrep
