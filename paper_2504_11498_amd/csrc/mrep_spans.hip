// Exact Bezier form of every knot interval of a batch of B-spline curves, on
// the device (the span decomposition of Sec. 5.2.1, done for the whole batch
// in one launch instead of on the host).
//
// The Bezier points of the span [a, b] = [U_q, U_{q+1}] of a degree-p curve
// are the blossom values b_j = P(a, .., a, b, .., b) with p - j arguments a
// and j arguments b.  Each is one de Boor triangle over the p + 1 control
// points P_{q-p} .. P_q, level k taking its own argument x_k:
//   d_r <- (1 - w) d_{r-1} + w d_r,  w = (x_k - U_i) / (U_{i+p+1-k} - U_i),
// r = p down to k, i = q - p + r.  Every w lies in [0, 1] (the knot interval
// [U_i, U_{i+p+1-k}] contains [a, b]), so the scheme is a chain of convex
// combinations.  It yields the same points as the product B_p^{-1} M A P of
// eqs. `decomposition` / `decomfinal` without the power basis in between,
// whose conversion back to Bernstein form grows rounding with the binomial
// coefficients of the degree.
//
// One thread per knot interval; the degree is a template parameter so that
// the control points and the 2p knots the triangle touches stay in registers,
// and the kernel is instantiated for the batch's largest degree (3, 5, 7, 9
// or 15) so that low-degree batches are not held to the registers of degree 15.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <string>

#include "../../include/mrep.h"
#include "mrep_internal.h"

namespace mrep {
namespace {

constexpr int kSpanBlock = 128;

// One interpolation level k of the triangle with argument x on points
// d[k..P] (d[r] for r < k is no longer needed).
template <int P, int K>
__device__ __forceinline__ void span_level(double (&d)[P + 1][3], const double (&kn)[2 * P + 1], double x)
{
#pragma unroll
    for (int r = P; r >= K; --r) {
        const double lo = kn[r];  // U_i, i = q - P + r
        const double w = (x - lo) / (kn[r + P + 1 - K] - lo);
#pragma unroll
        for (int e = 0; e < 3; ++e) d[r][e] = fma(w, d[r][e] - d[r - 1][e], d[r - 1][e]);
    }
}

// b_{P-M}: the state after M levels with argument a, then levels M+1 .. P with b.
template <int P, int M, int K>
__device__ __forceinline__ void span_b_levels(double (&e)[P + 1][3], const double (&kn)[2 * P + 1], double b)
{
    if constexpr (K <= P) {
        span_level<P, K>(e, kn, b);
        span_b_levels<P, M, K + 1>(e, kn, b);
    }
}

// The a-levels are shared by every point: after M levels with argument a the
// state d[M..P] is copied and finished with b for b_{P-M}, then level M + 1
// with a is applied.  p^3/6 interpolations instead of p^3/2 for one triangle
// per point.
template <int P, int M>
__device__ __forceinline__ void span_points(double (&d)[P + 1][3], const double (&kn)[2 * P + 1], double a, double b,
                                            double* __restrict__ out)
{
    double e[P + 1][3];
#pragma unroll
    for (int r = M; r <= P; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) e[r][c] = d[r][c];
    span_b_levels<P, M, M + 1>(e, kn, b);
#pragma unroll
    for (int c = 0; c < 3; ++c) out[3 * (P - M) + c] = e[P][c];
    if constexpr (M < P) {
        span_level<P, M + 1>(d, kn, a);
        span_points<P, M + 1>(d, kn, a, b, out);
    }
}

template <int P>
__device__ __forceinline__ void span_bezier(const double* __restrict__ U, const double* __restrict__ cp, int q,
                            double* __restrict__ out)
{
    double kn[2 * P + 1];  // kn[m] = U[q - P + m], m = 1 .. 2P used
    double d[P + 1][3];
    kn[0] = 0.0;
#pragma unroll
    for (int m = 1; m <= 2 * P; ++m) kn[m] = U[q - P + m];
#pragma unroll
    for (int r = 0; r <= P; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) d[r][c] = cp[3 * (q - P + r) + c];
    span_points<P, 0>(d, kn, kn[P], kn[P + 1], out);
}

template <int P, int PMAX>
__device__ __forceinline__ void span_bezier_dispatch(int p, const double* U, const double* cp, int q, double* out)
{
    if (p == P)
        span_bezier<P>(U, cp, q, out);
    else if constexpr (P < PMAX)
        span_bezier_dispatch<P + 1, PMAX>(p, U, cp, q, out);
}

// PMAX: the largest degree this instantiation handles; it sets the kernel's
// register allocation, so a batch of low-degree curves runs a smaller one.
template <int PMAX>
__global__ __launch_bounds__(kSpanBlock) void k_span_bezier(int32_t n_curves, int64_t n_iv,
                                                             const int32_t* __restrict__ degree,
                                                             const int64_t* __restrict__ cp_off,
                                                             const int64_t* __restrict__ knot_off,
                                                             const int64_t* __restrict__ iv_off,
                                                             const int64_t* __restrict__ pt_off,
                                                             const double* __restrict__ cp,
                                                             const double* __restrict__ knots,
                                                             double* __restrict__ bz, double* __restrict__ t_out)
{
    const int64_t g = (int64_t)blockIdx.x * kSpanBlock + threadIdx.x;
    if (g >= n_iv) return;
    // curve of interval g: the last c with iv_off[c] <= g
    int lo = 0, hi = n_curves;  // iv_off[lo] <= g < iv_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (iv_off[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    const int c = lo;
    const int p = degree[c];
    const int64_t n_pts = cp_off[c + 1] - cp_off[c];
    const int64_t k = g - iv_off[c];
    const bool ok = p >= 1 && p <= PMAX && n_pts >= p + 1 && k >= 0 && k < n_pts - p &&
                    knot_off[c + 1] - knot_off[c] == n_pts + p + 1 &&
                    pt_off[c] + (k + 1) * (p + 1) <= pt_off[c + 1] && iv_off[c + 1] - iv_off[c] == n_pts - p;
    if (!ok) {
        t_out[2 * g] = NAN;
        t_out[2 * g + 1] = NAN;
        return;
    }
    const double* U = knots + knot_off[c];
    const int q = (int)k + p;
    double* out = bz + 3 * (pt_off[c] + k * (p + 1));
    const double a = U[q], b = U[q + 1];
    t_out[2 * g] = a;
    t_out[2 * g + 1] = b;
    if (!(a < b)) {
        for (int j = 0; j < 3 * (p + 1); ++j) out[j] = NAN;
        return;
    }
    span_bezier_dispatch<1, PMAX>(p, U, cp + 3 * cp_off[c], q, out);
}

}  // namespace
}  // namespace mrep

extern "C" int32_t mrep_span_layout(int32_t n_curves, const int32_t* degree, const int64_t* cp_off,
                                    const int64_t* knot_off, int64_t* iv_off, int64_t* pt_off)
{
    if (n_curves < 0 || (n_curves > 0 && (!degree || !cp_off || !knot_off)) || !iv_off || !pt_off) {
        mrep::set_error("mrep_span_layout: null pointer or negative n_curves");
        return MREP_E_INVALID_ARG;
    }
    iv_off[0] = 0;
    pt_off[0] = 0;
    for (int32_t c = 0; c < n_curves; ++c) {
        const int p = degree[c];
        const int64_t n = cp_off[c + 1] - cp_off[c];
        if (p < 1 || p > MREP_SPAN_MAX_DEGREE) {
            mrep::set_error("mrep_span_layout: curve " + std::to_string(c) + ": degree out of range 1..15");
            return MREP_E_BAD_DEGREE;
        }
        if (n < p + 1) {
            mrep::set_error("mrep_span_layout: curve " + std::to_string(c) + ": fewer than p + 1 control points");
            return MREP_E_BAD_DEGREE;
        }
        if (knot_off[c + 1] - knot_off[c] != n + p + 1) {
            mrep::set_error("mrep_span_layout: curve " + std::to_string(c) + ": knot count is not #points + p + 1");
            return MREP_E_BAD_KNOTS;
        }
        iv_off[c + 1] = iv_off[c] + (n - p);
        pt_off[c + 1] = pt_off[c] + (n - p) * (p + 1);
    }
    return MREP_OK;
}

extern "C" int32_t mrep_span_bezier_curves(int32_t n_curves, int64_t n_intervals, int32_t max_degree,
                                           const int32_t* degree,
                                           const int64_t* cp_off, const int64_t* knot_off, const int64_t* iv_off,
                                           const int64_t* pt_off, const double* cp_xyz, const double* knots,
                                           double* bz_out, double* t_out, void* stream)
{
    if (n_curves < 0 || n_intervals < 0 || max_degree < 1 || max_degree > MREP_SPAN_MAX_DEGREE ||
        (n_intervals > 0 && (n_curves == 0 || !degree || !cp_off || !knot_off || !iv_off || !pt_off || !cp_xyz ||
                             !knots || !bz_out || !t_out))) {
        mrep::set_error("mrep_span_bezier_curves: null pointer, negative count or max_degree outside 1..15");
        return MREP_E_INVALID_ARG;
    }
    if (n_intervals == 0) return MREP_OK;
    const int64_t blocks = (n_intervals + mrep::kSpanBlock - 1) / mrep::kSpanBlock;
    if (blocks > INT32_MAX) {
        mrep::set_error("mrep_span_bezier_curves: too many intervals");
        return MREP_E_INVALID_ARG;
    }
    const dim3 grid((unsigned)blocks), block(mrep::kSpanBlock);
    const hipStream_t st = (hipStream_t)stream;
#define MREP_SPAN_LAUNCH(PM)                                                                                      \
    hipLaunchKernelGGL(mrep::k_span_bezier<PM>, grid, block, 0, st, n_curves, n_intervals, degree, cp_off, knot_off, \
                       iv_off, pt_off, cp_xyz, knots, bz_out, t_out)
    if (max_degree <= 3)
        MREP_SPAN_LAUNCH(3);
    else if (max_degree <= 5)
        MREP_SPAN_LAUNCH(5);
    else if (max_degree <= 7)
        MREP_SPAN_LAUNCH(7);
    else if (max_degree <= 9)
        MREP_SPAN_LAUNCH(9);
    else
        MREP_SPAN_LAUNCH(15);
#undef MREP_SPAN_LAUNCH
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        mrep::set_error(std::string("mrep_span_bezier_curves: ") + hipGetErrorString(e));
        return MREP_E_HIP;
    }
    return MREP_OK;
}
