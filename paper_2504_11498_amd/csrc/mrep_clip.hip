// The paper's refinement path for candidate (query, piece) pairs, as an
// alternative to the sampled minimum + Newton of k_pairs (FP64, one thread
// per pair):
//   1. E(u) = 2 (C(u) - q).C'(u) (eq. Et, degree 5 for a cubic) and E'(u)
//      (eq. E't, degree 4) in power form;
//   2. the real roots of E' by Ferrari's method split [0, 1] into monotonic
//      intervals of E (Sec. 5.2.3);
//   3. elimination: an interval can hold a local minimum of D only when E goes
//      from negative to non-negative across it (Sec. 5.3, Property 1); both
//      ends of every piece are candidates (Property 2 for the curve's ends,
//      and a C0 joint can hold the minimum without a root of E);
//   4. rebasement of E to Bernstein form, b = T a with T_ij = C(i,j)/C(5,j)
//      (Sec. 5.3); a kept interval [ta, tb] is cut out of it with the
//      subdivision operator S_[ta,tb] used by the clipping;
//   5. Bezier clipping (Sec. 5.4.1): the convex hull of (i/5, b_i) meets the
//      axis in [z1, z2], b <- S_L((z2 - z1)/(1 - z1)) S_R(z1) b, until the
//      interval is below kClipTol.  When a clipping keeps more than half of the
//      interval, the half where E changes sign replaces it (E is monotonic, so
//      exactly one half holds the root; this keeps one task per interval).
// The rebasement is a constant 6x6 lower-triangular product, 21 multiply-adds
// per pair, done in registers: a GEMM formulation would stage every pair's
// coefficients through memory for a contraction of depth 6.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/mrep.h"
#include "mrep_dev.h"
#include "mrep_refine.h"

namespace mrep {

namespace {

constexpr int kClipIters = 24;      // clippings per interval at most
constexpr double kClipTol = 1e-8;   // interval width in the piece parameter that ends the clipping (the
                                    // pair result keeps u in FP32; the finish polishes in FP64)

// real roots of y^2 + b y + c, appended to r
__device__ __forceinline__ void quad_real(double b, double c, double* r, int& n)
{
    const double disc = b * b - 4.0 * c;
    if (disc < 0.0) return;
    const double sq = sqrt(disc);
    const double big = -0.5 * (b + copysign(sq, b));  // no cancellation
    r[n++] = big;
    if (disc > 0.0) r[n++] = big != 0.0 ? c / big : 0.0;
}

// real roots of the monic cubic x^3 + A x^2 + B x + C; returns their count
__device__ __forceinline__ int cubic_real(double A, double B, double C, double* r)
{
    const double a3 = A / 3.0;
    const double P = B - A * a3;                              // depressed: w^3 + P w + Q, x = w - A/3
    const double Q = C - a3 * B + 2.0 * a3 * a3 * a3;
    const double h = 0.25 * Q * Q + P * P * P / 27.0;
    if (h > 0.0) {  // one real root (Cardano)
        const double s = sqrt(h);
        r[0] = cbrt(-0.5 * Q + s) + cbrt(-0.5 * Q - s) - a3;
        return 1;
    }
    if (P == 0.0) {
        r[0] = -a3;
        return 1;
    }
    const double m = sqrt(-P / 3.0);  // three real roots (trigonometric form)
    const double c = fmin(fmax(-0.5 * Q / (m * m * m), -1.0), 1.0);
    const double phi = acos(c) / 3.0;
    r[0] = 2.0 * m * cos(phi) - a3;
    r[1] = 2.0 * m * cos(phi - 2.0943951023931957) - a3;
    r[2] = 2.0 * m * cos(phi + 2.0943951023931957) - a3;
    return 3;
}

// Real roots of e0 + e1 x + ... + e4 x^4 by Ferrari's method, at the degree
// the coefficients show: a leading coefficient below 1e-6 of the largest
// lower one only adds roots far outside [0, 1], and normalising by it would
// leave no accurate root in [0, 1] (the E' of a degree-elevated quadratic
// piece has cubic and quartic coefficients at rounding level), so it is
// dropped; the roots within [-0.5, 1.5] are then polished by three Newton
// steps on the full quartic.  Unsorted, count returned.
__device__ int quartic_real(const double* e, double* r)
{
    int deg = 4;
    {
        const double l4 = fmax(fmax(fabs(e[0]), fabs(e[1])), fmax(fabs(e[2]), fabs(e[3])));
        const double l3 = fmax(fmax(fabs(e[0]), fabs(e[1])), fabs(e[2]));
        const double l2 = fmax(fabs(e[0]), fabs(e[1]));
        if (!(fabs(e[4]) > 1e-6 * l4)) {
            deg = 3;
            if (!(fabs(e[3]) > 1e-6 * l3)) {
                deg = 2;
                if (!(fabs(e[2]) > 1e-6 * l2)) deg = fabs(e[1]) > 1e-6 * fabs(e[0]) ? 1 : 0;
            }
        }
    }
    double x[4];
    int n = 0;
    if (deg == 4) {
        const double b = e[3] / e[4], c = e[2] / e[4], d = e[1] / e[4], f = e[0] / e[4];
        const double b4 = 0.25 * b;
        // x = y - b/4: y^4 + p y^2 + q y + s
        const double p = c - 6.0 * b4 * b4;
        const double q = d - 2.0 * c * b4 + 8.0 * b4 * b4 * b4;
        const double s = f - d * b4 + c * b4 * b4 - 3.0 * b4 * b4 * b4 * b4;
        const double sc = fmax(fabs(p), sqrt(fabs(s)));
        double y[4];
        int ny = 0;
        if (fabs(q) <= 1e-14 * sc * sqrt(sc) || sc == 0.0) {
            // y^4 + p y^2 + s: quadratic in y^2
            double z[2];
            int nz = 0;
            quad_real(p, s, z, nz);
            for (int i = 0; i < nz; ++i)
                if (z[i] >= 0.0) {
                    y[ny++] = sqrt(z[i]);
                    y[ny++] = -sqrt(z[i]);
                }
        } else {
            // resolvent m^3 + p m^2 + (p^2/4 - s) m - q^2/8 = 0: its largest root
            // m > 0 makes y^4 + p y^2 + q y + s = (y^2 + p/2 + m)^2 - 2m (y - q/(4m))^2
            double rc[3];
            const int nc = cubic_real(p, 0.25 * p * p - s, -0.125 * q * q, rc);
            double m = rc[0];
            for (int i = 1; i < nc; ++i) m = fmax(m, rc[i]);
            if (m > 0.0) {
                const double w = sqrt(2.0 * m);
                const double t = 0.5 * p + m, u = 0.5 * q / w;
                quad_real(-w, t + u, y, ny);
                quad_real(w, t - u, y, ny);
            }
        }
        for (int i = 0; i < ny; ++i) x[n++] = y[i] - b4;
    } else if (deg == 3) {
        n = cubic_real(e[2] / e[3], e[1] / e[3], e[0] / e[3], x);
    } else if (deg == 2) {
        quad_real(e[1] / e[2], e[0] / e[2], x, n);
    } else if (deg == 1) {
        x[n++] = -e[0] / e[1];
    }
    int m = 0;
    for (int i = 0; i < n; ++i) {
        double v = x[i];
        if (!(v > -0.5 && v < 1.5)) continue;
        for (int it = 0; it < 3; ++it) {
            const double f = fma(fma(fma(fma(e[4], v, e[3]), v, e[2]), v, e[1]), v, e[0]);
            const double fp = fma(fma(fma(4.0 * e[4], v, 3.0 * e[3]), v, 2.0 * e[2]), v, e[1]);
            if (fp == 0.0) break;
            v -= f / fp;
        }
        r[m++] = v;
    }
    return m;
}

// de Casteljau in place on Bernstein coefficients b[0..5]: the part [z, 1]
__device__ __forceinline__ void right_part(double* b, double z)
{
#pragma unroll
    for (int r = 1; r <= 5; ++r)
#pragma unroll
        for (int i = 0; i <= 5 - r; ++i) b[i] = fma(z, b[i + 1] - b[i], b[i]);
}
// ... and the part [0, z]
__device__ __forceinline__ void left_part(double* b, double z)
{
#pragma unroll
    for (int r = 1; r <= 5; ++r)
#pragma unroll
        for (int i = 5; i >= r; --i) b[i] = fma(z, b[i] - b[i - 1], b[i - 1]);
}
// S_[z1,z2] b = S_L((z2 - z1)/(1 - z1)) S_R(z1) b (eq. subdivisionmatrix)
__device__ __forceinline__ void clip_to(double* b, double z1, double z2)
{
    if (z1 > 0.0) right_part(b, z1);
    if (z2 < 1.0) left_part(b, z1 < 1.0 ? (z2 - z1) / (1.0 - z1) : 0.0);
}
__device__ __forceinline__ double bern_at(const double* b, double z)
{
    double w[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) w[i] = b[i];
    right_part(w, z);
    return w[0];
}

// Convex hull of (i/5, b_i) against the axis: [z1, z2], false when they do not
// meet (only the pairs of opposite signs cross; a few per clipping).
__device__ __forceinline__ bool hull_axis(const double* b, double& z1, double& z2)
{
    double lo = INFINITY, hi = -INFINITY;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        if (b[i] == 0.0) {
            lo = fmin(lo, 0.2 * i);
            hi = fmax(hi, 0.2 * i);
        }
#pragma unroll
        for (int j = i + 1; j < 6; ++j)
            if ((b[i] < 0.0) != (b[j] < 0.0) && b[i] != 0.0 && b[j] != 0.0) {
                const double x = 0.2 * (i + (j - i) * b[i] / (b[i] - b[j]));
                lo = fmin(lo, x);
                hi = fmax(hi, x);
            }
    }
    z1 = fmax(lo, 0.0);
    z2 = fmin(hi, 1.0);
    return lo <= hi;
}

// The refinement of one pair: the best of the piece ends and the roots of E
// found by clipping on the kept monotonic intervals.  u, squared distance,
// kappa = (|C'|^2 + r.C'')/|C'|^2 at u (1 at an end), the width left in u.
__device__ void clip_piece_min(const Cubic<double>& C, double& u_out, double& d_out, double& k_out, double& w_out,
                               double& u2_out, double& d2_out)
{
    // E = 2 r.C' with r = C - q = a0 + a1 u + a2 u^2 + a3 u^3, C' = a1 + 2 a2 u + 3 a3 u^2
    const V3<double> a[4] = {C.a0, C.a1, C.a2, C.a3};
    double E[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 1; i < 4; ++i) E[j + i - 1] += 2.0 * (double)i * dot(a[j], a[i]);
    double Ep[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) Ep[m] = (double)(m + 1) * E[m + 1];
    // monotonic intervals: the roots of E' in (0, 1), sorted
    double br[6];
    int nb = 0;
    {
        double r[4];
        const int nr = quartic_real(Ep, r);
        for (int i = 0; i < nr; ++i)
            if (r[i] > 0.0 && r[i] < 1.0) br[nb++] = r[i];
        for (int i = 1; i < nb; ++i)
            for (int j = i; j > 0 && br[j] < br[j - 1]; --j) {
                const double t = br[j];
                br[j] = br[j - 1];
                br[j - 1] = t;
            }
    }
    // Bernstein coefficients of E on [0, 1]: b = T E, T_ij = C(i,j)/C(5,j)
    const double bf[6] = {E[0],
                          E[0] + 0.2 * E[1],
                          E[0] + 0.4 * E[1] + 0.1 * E[2],
                          E[0] + 0.6 * E[1] + 0.3 * E[2] + 0.1 * E[3],
                          E[0] + 0.8 * E[1] + 0.6 * E[2] + 0.4 * E[3] + 0.2 * E[4],
                          E[0] + E[1] + E[2] + E[3] + E[4] + E[5]};
    V3<double> er, e1, e2;
    C.eval(0.0, er, e1, e2);
    const double k0 = end_kappa(er, e1, e2);
    C.eval(1.0, er, e1, e2);
    const double k1 = end_kappa(er, e1, e2);
    u_out = 0.0;
    d_out = C.dist2(0.0);
    k_out = k0;
    w_out = 0.0;
    u2_out = 0.0;
    d2_out = INFINITY;
    // an end is a local minimum of the piece only where the distance grows into
    // the piece; only local minima become the second minimum
    bool l_out = E[0] >= 0.0;
    {
        const double d1 = C.dist2(1.0);
        const bool l1 = bf[5] <= 0.0;
        if (d1 < d_out) {
            if (l_out) { u2_out = 0.0; d2_out = d_out; }
            d_out = d1; u_out = 1.0; l_out = l1; k_out = k1;
        } else if (l1) {
            u2_out = 1.0; d2_out = d1;
        }
    }
    double ta = 0.0, ea = E[0];
    for (int k = 0; k <= nb; ++k) {
        const double tb = k < nb ? br[k] : 1.0;
        const double eb = E[0] + tb * (E[1] + tb * (E[2] + tb * (E[3] + tb * (E[4] + tb * E[5]))));
        if (ea < 0.0 && eb >= 0.0) {  // Property 1 does not eliminate it
            double b[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) b[i] = bf[i];
            clip_to(b, ta, tb);
            const double h = tb - ta;
            double lo = 0.0, hi = 1.0;
            for (int it = 0; it < kClipIters && h * (hi - lo) > kClipTol; ++it) {
                double z1, z2;
                if (!hull_axis(b, z1, z2)) break;
                if (z2 - z1 > 0.5) {  // slow clipping: keep the half where E changes sign
                    const double zm = 0.5 * (z1 + z2);
                    if (bern_at(b, zm) >= 0.0) z2 = zm; else z1 = zm;
                }
                clip_to(b, z1, z2);
                const double span = hi - lo;
                hi = lo + span * z2;
                lo = lo + span * z1;
            }
            const double u = ta + h * 0.5 * (lo + hi);
            const double d = C.dist2(u);
            w_out = fmax(w_out, h * (hi - lo));
            // two minima only with a barrier between them (as in piece_min)
            const bool apart = fabs(u - u_out) > (double)kDistinctU &&
                               C.dist2(0.5 * (u + u_out)) > fmax(d, d_out) * (1.0 + 1e-13);
            if (d < d_out) {
                if (l_out && apart) { u2_out = u_out; d2_out = d_out; }
                d_out = d;
                u_out = u;
                l_out = true;
                V3<double> r, d1, d2;
                C.eval(u, r, d1, d2);
                const double sp = dot(d1, d1);
                k_out = sp > 0.0 ? (sp + dot(r, d2)) / sp : 1.0;
            } else if (d < d2_out && apart) {
                u2_out = u;
                d2_out = d;
            }
        }
        ta = tb;
        ea = eb;
    }
    // A minimum that the clipping left within its resolution of an end whose
    // distance is no higher (up to rounding) is that end: where the distance
    // keeps falling into the neighbouring piece, E at the end is a rounding
    // level either way.  The candidate selection knows a joint by u = 0 or 1.
    for (int e = 0; e < 2; ++e) {
        const double ue = (double)e;
        if (u_out != ue && fabs(u_out - ue) <= kClipTol) {
            const double de = C.dist2(ue);
            if (de <= d_out * (1.0 + 1e-12)) {
                u_out = ue;
                d_out = de;
            }
        }
    }
}

// 3 waves per SIMD (168 VGPRs, some FP64 temporaries spill): refine 1.03 ms
// on the batched curves against 1.16 ms with 2 waves (211 VGPRs, no spill)
#ifndef MREP_CLIP_MIN_WAVES
#define MREP_CLIP_MIN_WAVES 3
#endif
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MREP_CLIP_MIN_WAVES, 8))) void k_pairs_clip(DevGeom G, const int32_t* __restrict__ cid,
                                                    const double* __restrict__ qxyz, const int32_t* __restrict__ perm,
                                                    const int32_t* __restrict__ pair_seg,
                                                    const int32_t* __restrict__ pair_j,
                                                    const int32_t* __restrict__ pair_count, int64_t pair_cap,
                                                    const uint8_t* __restrict__ done, PairRes* __restrict__ pair_res)
{
    const int64_t total = min((int64_t)*pair_count, pair_cap);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t jj = pair_j[p];
        if (jj < 0) continue;  // reserved by a query that then overflowed the capacity
        if (done && done[jj]) continue;
        const int64_t s = pair_seg[p];
        if (s < 0 || s >= G.n_seg) continue;
        const int32_t qi = perm[jj];
        const DCurve cv = G.curves[cid[qi]];
        const double q[3] = {qxyz[3 * (int64_t)qi], qxyz[3 * (int64_t)qi + 1], qxyz[3 * (int64_t)qi + 2]};
        Cubic<double> C;
        load_cubic(G, cv, s, q, C);
        double u, d, k, w, u2, d2;
        clip_piece_min(C, u, d, k, w, u2, d2);
        // parameter error: the clipping's remaining half-width, plus rounding
        const double err = (0.5 * w + 1e-15) * (G.segt[2 * s + 1] - G.segt[2 * s]);
        pair_res[p] = pair_result(G, cv, s, q, u, d, k, err, u2, d2);
    }
}

// Monotonic split of one (query, piece) pair: the roots of E' in (0, 1),
// ascending.  kNewton: Newton's iteration from 8 uniform starts instead of
// Ferrari's method.
template <bool kNewton>
__global__ __launch_bounds__(256) void k_split(DevGeom G, int64_t n, const int32_t* __restrict__ cid,
                                               const int32_t* __restrict__ piece, const double* __restrict__ qxyz,
                                               double* __restrict__ roots, int32_t* __restrict__ count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = cid[i];
    if (c < 0 || c >= G.n_curves) { count[i] = -1; return; }
    const DCurve cv = G.curves[c];
    const int32_t k = piece[i];
    if (k < 0 || k >= cv.n_seg) { count[i] = -1; return; }
    const double q[3] = {qxyz[3 * i], qxyz[3 * i + 1], qxyz[3 * i + 2]};
    Cubic<double> C;
    load_cubic(G, cv, cv.seg_off + k, q, C);
    const V3<double> a[4] = {C.a0, C.a1, C.a2, C.a3};
    double E[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int m = 1; m < 4; ++m) E[j + m - 1] += 2.0 * (double)m * dot(a[j], a[m]);
    double ep[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) ep[m] = (double)(m + 1) * E[m + 1];
    double r[8];
    int nr = 0;
    if (!kNewton) {
        double x[4];
        const int nx = quartic_real(ep, x);
        for (int j = 0; j < nx; ++j)
            if (x[j] > 0.0 && x[j] < 1.0) r[nr++] = x[j];
    } else {
        const double scale = fabs(ep[0]) + fabs(ep[1]) + fabs(ep[2]) + fabs(ep[3]) + fabs(ep[4]);
        for (int s = 0; s < 8; ++s) {
            double u = (s + 0.5) / 8.0;
            bool conv = false;
            for (int it = 0; it < 20; ++it) {
                const double f = fma(fma(fma(fma(ep[4], u, ep[3]), u, ep[2]), u, ep[1]), u, ep[0]);
                const double fp = fma(fma(fma(4.0 * ep[4], u, 3.0 * ep[3]), u, 2.0 * ep[2]), u, ep[1]);
                if (fp == 0.0) break;
                const double du = f / fp;
                u -= du;
                if (fabs(du) <= 1e-14 * (1.0 + fabs(u))) { conv = fabs(f) <= 1e-10 * scale; break; }
            }
            if (!conv || !(u > 0.0 && u < 1.0)) continue;
            bool dup = false;
            for (int j = 0; j < nr; ++j) dup |= fabs(r[j] - u) <= 1e-9;
            if (!dup && nr < 4) r[nr++] = u;
        }
    }
    for (int j = 1; j < nr; ++j)
        for (int m = j; m > 0 && r[m] < r[m - 1]; --m) {
            const double t = r[m];
            r[m] = r[m - 1];
            r[m - 1] = t;
        }
    for (int j = 0; j < 4; ++j) roots[4 * i + j] = j < nr ? r[j] : 0.0;
    count[i] = nr;
}

}  // namespace

hipError_t launch_pairs_clip(const DevGeom& G, const int32_t* curve_id, const double* q_xyz, const int32_t* perm,
                             const ScreenOut& so, const uint8_t* done, PairRes* pair_res, hipStream_t st)
{
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((so.pair_cap + 255) / 256, 8192));
    hipLaunchKernelGGL(k_pairs_clip, dim3(blocks), dim3(256), 0, st, G, curve_id, q_xyz, perm,
                       (const int32_t*)so.pair_seg, (const int32_t*)so.pair_j, (const int32_t*)so.pair_count,
                       so.pair_cap, done, pair_res);
    return hipGetLastError();
}

}  // namespace mrep

extern "C" int32_t mrep_monotonic_split(const mrep_geom* geom, int64_t n, const int32_t* curve_id,
                                        const int32_t* piece, const double* q_xyz, int32_t method,
                                        double* roots_out, int32_t* count_out, void* stream)
{
    if (!geom || n < 0 || geom->kind != MREP_GEOM_CURVES ||
        (n > 0 && (!curve_id || !piece || !q_xyz || !roots_out || !count_out)) ||
        (method != MREP_ROOTS_FERRARI && method != MREP_ROOTS_NEWTON)) {
        mrep::set_error("mrep_monotonic_split: null pointer, surface geometry, negative n or unknown method");
        return MREP_E_INVALID_ARG;
    }
    if (n == 0) return MREP_OK;
    const mrep::DevGeom G = mrep::dev_view(geom->g);
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (method == MREP_ROOTS_FERRARI)
        hipLaunchKernelGGL(mrep::k_split<false>, grid, block, 0, (hipStream_t)stream, G, n, curve_id, piece, q_xyz,
                           roots_out, count_out);
    else
        hipLaunchKernelGGL(mrep::k_split<true>, grid, block, 0, (hipStream_t)stream, G, n, curve_id, piece, q_xyz,
                           roots_out, count_out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        mrep::set_error(std::string("mrep_monotonic_split: ") + hipGetErrorString(e));
        return MREP_E_HIP;
    }
    return MREP_OK;
}
