// Device decomposition of a batch of polynomial B-spline curves: the exact
// span forms (Sec. 5.2.1, eqs. decomposition / decomfinal), the G1 cubic that
// minimises the L2 deviation with the preloaded Gram matrices (Sec. 5.2.2, eqs.
// gram / G1-condition / epsl), error-controlled splitting of the original
// degree-p piece (eqs. submatrix / subLandR), and the screen tables of every
// cubic piece, all on the GPU.
//
// The splitting is level-synchronous, as in the paper's subdivision figure:
// level L holds every piece still above its tolerance; one kernel reduces each
// of them and decides leaf or split, two prefix sums compact the leaves and
// the children, and a second kernel writes the children of level L + 1 (the
// two halves of the degree-p piece at the sample of largest deviation).  A
// span's leaves, which come from several levels, are put back in parameter
// order by one small sort per span, so the pieces come out in the order of the
// host decomposition.
//
// The arithmetic of every step is that of the host decomposition (the shared
// mrep_decomp.h; this file is compiled without floating-point contraction),
// so the pieces, breakpoints and tables equal the host's bit for bit.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mrep.h"
#include "mrep_decomp.h"
#include "mrep_dev.h"
#include "mrep_internal.h"

namespace mrep {

// Device-side result of mrep_decompose_curves_device, owned by its plan.
struct DevPlan {
    int64_t n_curves = 0, n_span = 0, n_seg = 0, n_coef = 0, n_clu = 0;
    int32_t max_degree = 0;
    double tol_rel = 0.0;
    GeomLayout layout;
    // per curve
    int32_t* deg = nullptr;
    double* diag = nullptr;
    double* origin = nullptr;   // [3]
    double* tol_eff = nullptr;
    int64_t* span_off = nullptr;  // [n_curves + 1]
    int64_t* coef_off = nullptr;  // [n_curves + 1]
    int64_t* seg_off = nullptr;   // [n_curves + 1]
    int64_t* clu_off = nullptr;   // [n_curves + 1]
    // per span
    int32_t* span_curve = nullptr;
    double* span_t = nullptr;     // [2]
    int32_t* span0 = nullptr;     // [n_span + 1]
    double* coef = nullptr;
    // per piece
    double* seg_cp = nullptr;     // [12]
    double* seg_t = nullptr;      // [2]
    int32_t* seg_span = nullptr;
    ~DevPlan();
};

namespace {

constexpr int kBlock = 256;

#define DD_HIP(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            set_error(std::string("mrep_decompose_curves_device: ") + hipGetErrorString(e_)); \
            return MREP_E_HIP;                                                      \
        }                                                                           \
    } while (0)

unsigned blocks_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <typename T>
hipError_t dmalloc(T** p, int64_t n)
{
    *p = nullptr;
    if (n <= 0) return hipSuccess;
    return hipMalloc((void**)p, sizeof(T) * (size_t)n);
}

template <typename T>
void dfree(T*& p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

// ---------------------------------------------------------------------------
// exclusive prefix sums (three passes: block sums, one block over the block
// sums, block-local scans plus offsets); total (nullable) gets the sum
// ---------------------------------------------------------------------------
constexpr int kScanItems = 4;                     // per thread
constexpr int kScanTile = kBlock * kScanItems;    // per block

template <typename T>
__device__ T block_exclusive(T v, T* sh, T& total)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const T a = tid >= off ? sh[tid - off] : (T)0;
        __syncthreads();
        sh[tid] += a;
        __syncthreads();
    }
    total = sh[kBlock - 1];
    const T incl = sh[tid];
    __syncthreads();
    return incl - v;
}

template <typename T, typename In>
__global__ __launch_bounds__(kBlock) void k_scan_sums(const In* __restrict__ in, int64_t n, T* __restrict__ sums)
{
    __shared__ T sh[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T v = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) v += (T)in[base + k];
    T tot;
    block_exclusive<T>(v, sh, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// one block: exclusive scan of m block sums in place, total to *total
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_top(T* __restrict__ sums, int64_t m, T* __restrict__ total)
{
    __shared__ T sh[kBlock];
    const int64_t per = (m + kBlock - 1) / kBlock;
    const int64_t a = (int64_t)threadIdx.x * per, b = std::min<int64_t>(a + per, m);
    T v = 0;
    for (int64_t i = a; i < b; ++i) v += sums[i];
    T tot;
    T run = block_exclusive<T>(v, sh, tot);
    for (int64_t i = a; i < b; ++i) {
        const T x = sums[i];
        sums[i] = run;
        run += x;
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

template <typename T, typename In>
__global__ __launch_bounds__(kBlock) void k_scan_out(const In* __restrict__ in, int64_t n, const T* __restrict__ sums,
                                                     T* __restrict__ out)
{
    __shared__ T sh[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T x[kScanItems], v = 0;
    for (int k = 0; k < kScanItems; ++k) {
        x[k] = base + k < n ? (T)in[base + k] : (T)0;
        v += x[k];
    }
    T tot;
    T run = block_exclusive<T>(v, sh, tot) + sums[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) {
            out[base + k] = run;
            run += x[k];
        }
}

template <typename T>
__global__ void k_zero1(T* p)
{
    *p = (T)0;
}

// Scratch of a scan over n items: ceil(n / kScanTile) block sums.
struct Scanner {
    void* sums = nullptr;
    int64_t cap = 0;  // bytes
    ~Scanner() { if (sums) (void)hipFree(sums); }
    template <typename T>
    hipError_t run(const T* in, int64_t n, T* out, T* total_dev, hipStream_t st)
    {
        const int64_t nb = std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile);
        if ((int64_t)sizeof(T) * nb > cap) {
            if (sums) (void)hipFree(sums);
            sums = nullptr;
            cap = (int64_t)sizeof(T) * nb * 2;
            hipError_t e = hipMalloc(&sums, (size_t)cap);
            if (e != hipSuccess) { cap = 0; return e; }
        }
        T* s = (T*)sums;
        if (n > 0) hipLaunchKernelGGL((k_scan_sums<T, T>), dim3((unsigned)nb), dim3(kBlock), 0, st, in, n, s);
        else hipLaunchKernelGGL(k_zero1<T>, dim3(1), dim3(1), 0, st, s);
        hipLaunchKernelGGL(k_scan_top<T>, dim3(1), dim3(kBlock), 0, st, s, nb, total_dev);
        if (n > 0) hipLaunchKernelGGL((k_scan_out<T, T>), dim3((unsigned)nb), dim3(kBlock), 0, st, in, n, (const T*)s, out);
        return hipGetLastError();
    }
};

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// 1. per curve: validation (the host decomposition's rules), box diagonal,
//    FP32-representable origin, tolerances
// ---------------------------------------------------------------------------
enum {
    kErrNonFinitePoint = 1,
    kErrNonFiniteKnot,
    kErrKnotOrder,
    kErrNotClamped,
    kErrEmptyDomain,
    kErrMultiplicity,
    kErrEndMultiplicity,
};

__global__ void k_dd_curve(int32_t n_curves, const int32_t* __restrict__ deg, const int64_t* __restrict__ cp_off,
                           const int64_t* __restrict__ knot_off, const double* __restrict__ cp,
                           const double* __restrict__ knots, double tol_rel, int32_t* __restrict__ err,
                           double* __restrict__ diag, double* __restrict__ origin, double* __restrict__ tol_abs,
                           double* __restrict__ tol_eff)
{
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n_curves) return;
    const int p = deg[c];
    const int64_t n = cp_off[c + 1] - cp_off[c];
    const double* P = cp + 3 * cp_off[c];
    const double* U = knots + knot_off[c];
    const int64_t m = n + p + 1;
    int e = 0;
    for (int64_t i = 0; i < 3 * n && !e; ++i)
        if (!isfinite(P[i])) e = kErrNonFinitePoint;
    for (int64_t i = 0; i < m && !e; ++i)
        if (!isfinite(U[i])) e = kErrNonFiniteKnot;
    for (int64_t i = 0; i + 1 < m && !e; ++i)
        if (U[i + 1] < U[i]) e = kErrKnotOrder;
    for (int i = 0; i < p && !e; ++i)
        if (U[i] != U[p] || U[m - 1 - i] != U[n]) e = kErrNotClamped;
    if (!e && !(U[p] < U[n])) e = kErrEmptyDomain;
    int run = 1;
    for (int64_t i = p + 2; i <= n - 1 && !e; ++i) {
        run = (U[i] == U[i - 1]) ? run + 1 : 1;
        if (run > p) e = kErrMultiplicity;
    }
    if (!e && n - 1 >= p + 1 && (U[p + 1] == U[p] || U[n - 1] == U[n])) e = kErrEndMultiplicity;
    err[c] = e;
    double lo[3] = {P[0], P[1], P[2]}, hi[3] = {P[0], P[1], P[2]};
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            lo[k] = dm::mn(lo[k], P[3 * i + k]);
            hi[k] = dm::mx(hi[k], P[3 * i + k]);
        }
    const double d = sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                          (hi[2] - lo[2]) * (hi[2] - lo[2]));
    diag[c] = d;
    for (int k = 0; k < 3; ++k) origin[3 * c + k] = (double)(float)(0.5 * (lo[k] + hi[k]));
    // the pieces of p <= 3 are exact: their deviation term is rounding only
    const double ta = p >= 4 ? tol_rel * d : 0.0;
    tol_abs[c] = ta;
    tol_eff[c] = p >= 4 ? dm::mx(ta, 1e-13 * d) : 1e-13 * d;
}

// curve of interval g: the last c with iv_off[c] <= g
__device__ __forceinline__ int curve_of(const int64_t* __restrict__ iv_off, int32_t n_curves, int64_t g)
{
    int lo = 0, hi = n_curves;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (iv_off[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// 2. non-empty knot intervals
__global__ void k_dd_nonempty(int32_t n_curves, int64_t n_iv, const int32_t* __restrict__ deg,
                              const int64_t* __restrict__ knot_off, const int64_t* __restrict__ iv_off,
                              const double* __restrict__ knots, int32_t* __restrict__ ne)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= n_iv) return;
    const int c = curve_of(iv_off, n_curves, g);
    const int q = (int)(g - iv_off[c]) + deg[c];
    const double* U = knots + knot_off[c];
    ne[g] = U[q] < U[q + 1] ? 1 : 0;
}

// per curve: first span, span count and exact-span doubles (for the scans)
__global__ void k_dd_curve_spans(int32_t n_curves, int64_t n_iv, const int32_t* __restrict__ deg,
                                 const int64_t* __restrict__ iv_off, const int32_t* __restrict__ sidx,
                                 const int32_t* __restrict__ n_span_total, int64_t* __restrict__ span_off,
                                 int64_t* __restrict__ coef_n)
{
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c > n_curves) return;
    const int64_t a = iv_off[c] < n_iv ? (int64_t)sidx[iv_off[c]] : (int64_t)*n_span_total;
    span_off[c] = a;
    if (c == n_curves) return;
    const int64_t b = iv_off[c + 1] < n_iv ? (int64_t)sidx[iv_off[c + 1]] : (int64_t)*n_span_total;
    coef_n[c] = (b - a) * 3 * (deg[c] + 1);
}

// Span forms and splits with the degree a compile-time constant (the shared
// functions inlined with p = P: unrolled loops, arrays in registers).  A wave
// holds the intervals or pieces of one or two curves, so its degree is nearly
// always uniform; a mixed wave takes the generic path.
template <int P>
__device__ __forceinline__ void span_forms_fixed(const dm::DegreeTables& T, const double* U, int q, const double* P_,
                                                 double* cf, double* o)
{
    double D[(P + 1) * 3], Q[(P + 1) * 3];
    dm::span_power_bezier<P>(P, T, U, q, P_, D, Q);
    for (int i = 0; i < 3 * (P + 1); ++i) cf[i] = D[i];
    for (int i = 0; i < 3 * (P + 1); ++i) o[i] = Q[i];
}

template <int MP, int P = 1>
__device__ __forceinline__ void span_forms_degree(int p, const dm::DegreeTables* tab, const double* U, int q,
                                                  const double* P_, double* cf, double* o)
{
    if constexpr (P < MP) {
        if (p != P) return span_forms_degree<MP, P + 1>(p, tab, U, q, P_, cf, o);
    }
    span_forms_fixed<P>(tab[P], U, q, P_, cf, o);
}

template <int P>
__device__ __forceinline__ void split_fixed(const double* Q, double z, double* Ql, double* Qr)
{
    double Lq[(P + 1) * 3], Rq[(P + 1) * 3], Qv[(P + 1) * 3];
    for (int k = 0; k < 3 * (P + 1); ++k) Qv[k] = Q[k];
    dm::split_piece(P, Qv, z, Lq, Rq);
    for (int k = 0; k < 3 * (P + 1); ++k) {
        Ql[k] = Lq[k];
        Qr[k] = Rq[k];
    }
}

template <int MP, int P = 4>
__device__ __forceinline__ void split_degree(int p, const double* Q, double z, double* Ql, double* Qr)
{
    if constexpr (P < MP) {
        if (p != P) return split_degree<MP, P + 1>(p, Q, z, Ql, Qr);
    }
    split_fixed<P>(Q, z, Ql, Qr);
}

// 3. exact span forms and the first level of pieces: one thread per interval.
//    MP bounds the batch's degree (array sizes only).
template <int MP>
__global__ __launch_bounds__(kBlock) void k_dd_spans(int32_t n_curves, int64_t n_iv, const int32_t* __restrict__ deg,
                                                     const int64_t* __restrict__ cp_off,
                                                     const int64_t* __restrict__ knot_off,
                                                     const int64_t* __restrict__ iv_off,
                                                     const double* __restrict__ cp, const double* __restrict__ knots,
                                                     const dm::DegreeTables* __restrict__ tab,
                                                     const int32_t* __restrict__ ne, const int32_t* __restrict__ sidx,
                                                     const int64_t* __restrict__ span_off,
                                                     const int64_t* __restrict__ coef_off, int32_t* __restrict__ span_curve,
                                                     double* __restrict__ span_t, double* __restrict__ coef,
                                                     int32_t* __restrict__ it_span, double* __restrict__ it_t,
                                                     double* __restrict__ it_Q, int32_t q_stride)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= n_iv || !ne[g]) return;
    const int c = curve_of(iv_off, n_curves, g);
    const int p = deg[c];
    const int q = (int)(g - iv_off[c]) + p;
    const double* U = knots + knot_off[c];
    const int64_t s = sidx[g];
    span_curve[s] = c;
    span_t[2 * s] = U[q];
    span_t[2 * s + 1] = U[q + 1];
    double* cf = coef + coef_off[c] + (s - span_off[c]) * 3 * (p + 1);
    it_span[s] = (int32_t)s;
    it_t[2 * s] = U[q];
    it_t[2 * s + 1] = U[q + 1];
    double* o = it_Q + s * (int64_t)q_stride;
    const double* P_ = cp + 3 * cp_off[c];
    const int p0 = __builtin_amdgcn_readfirstlane(p);
    if (__all(p == p0)) {
        span_forms_degree<MP>(p0, tab, U, q, P_, cf, o);
    } else {
        double D[(MP + 1) * 3], Q[(MP + 1) * 3];
        dm::span_power_bezier<MP>(p, tab[p], U, q, P_, D, Q);
        for (int i = 0; i < 3 * (p + 1); ++i) cf[i] = D[i];
        for (int i = 0; i < 3 * (p + 1); ++i) o[i] = Q[i];
    }
}

// The reduction and the deviation bound of one piece with the degree a
// compile-time constant: the shared (host) functions, inlined with p = P, so
// that the loops over the control points unroll and the piece's points are
// loaded once into registers instead of once per error sample.
template <int P>
__device__ __forceinline__ double reduce_fixed(const dm::DegreeTables& T, const double* Q, double* R, int* imax)
{
    dm::g1_reduce(P, T, Q, R);
    return dm::deviation_bound(P, T, Q, R, imax);
}

template <int MP, int P = 4>
__device__ __forceinline__ double reduce_degree(int p, const dm::DegreeTables* tab, const double* Q, double* R,
                                                int* imax)
{
    if constexpr (P < MP) {
        if (p != P) return reduce_degree<MP, P + 1>(p, tab, Q, R, imax);
    }
    return reduce_fixed<P>(tab[P], Q, R, imax);
}

// 4. one level: the cubic of every piece, and leaf (deviation bound within the
//    curve's tolerance, or an exact cubic) or split at the worst sample.
template <int MP>
__global__ __launch_bounds__(kBlock) void k_dd_level(int64_t n_items, const int32_t* __restrict__ deg,
                                                     const int32_t* __restrict__ span_curve,
                                                     const double* __restrict__ tol_abs,
                                                     const dm::DegreeTables* __restrict__ tab,
                                                     const int32_t* __restrict__ it_span, const double* __restrict__ it_Q,
                                                     int32_t q_stride, double* __restrict__ it_R,
                                                     int32_t* __restrict__ it_z, int32_t* __restrict__ is_leaf,
                                                     int32_t* __restrict__ is_split, int32_t* __restrict__ splits,
                                                     int32_t* __restrict__ fail)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_items) return;
    const int32_t s = it_span[i];
    const int c = span_curve[s];
    const int p = deg[c];
    const double* Q = it_Q + i * (int64_t)q_stride;
    double R[12];
    bool leaf = true;
    int iz = 0;
    if (p <= 3) {
        dm::elevate_to_cubic(p, Q, R);
    } else {
        int imax = 64;
        double e;
        // The pieces of one curve share its degree, so a wave is nearly always of one
        // degree: then the degree is wave-uniform and every table entry the reduction
        // and the deviation bound read is one scalar load for the whole wave.
        const int p0 = __builtin_amdgcn_readfirstlane(p);
        if (__all(p == p0)) {
            e = reduce_degree<MP>(p0, tab, Q, R, &imax);
        } else {
            dm::g1_reduce(p, tab[p], Q, R);
            e = dm::deviation_bound(p, tab[p], Q, R, &imax);
        }
        if (!(e <= tol_abs[c])) {
            leaf = false;
            iz = dm::mn(dm::mx(imax, 16), 112);
            if (atomicAdd(&splits[s], 1) + 1 >= MREP_MAX_PIECES_PER_SPAN) atomicOr(fail, 1);
        }
    }
    for (int k = 0; k < 12; ++k) it_R[12 * i + k] = R[k];
    it_z[i] = iz;
    is_leaf[i] = leaf ? 1 : 0;
    is_split[i] = leaf ? 0 : 1;
}

// 5. write the level's leaves (appended after leaf_base) and the two halves of
//    every split piece (the next level, in item order)
template <int MP>
__global__ __launch_bounds__(kBlock) void k_dd_emit(int64_t n_items, const int32_t* __restrict__ deg,
                                                    const int32_t* __restrict__ span_curve,
                                                    const int32_t* __restrict__ it_span, const double* __restrict__ it_t,
                                                    const double* __restrict__ it_Q, int32_t q_stride,
                                                    const double* __restrict__ it_R, const int32_t* __restrict__ it_z,
                                                    const int32_t* __restrict__ is_leaf, const int32_t* __restrict__ lpos,
                                                    const int32_t* __restrict__ cpos, int64_t leaf_base,
                                                    double* __restrict__ lf_R, double* __restrict__ lf_t,
                                                    int32_t* __restrict__ lf_span, int32_t* __restrict__ span_nleaf,
                                                    int32_t* __restrict__ nx_span, double* __restrict__ nx_t,
                                                    double* __restrict__ nx_Q)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_items) return;
    const int32_t s = it_span[i];
    const double ta = it_t[2 * i], tb = it_t[2 * i + 1];
    if (is_leaf[i]) {
        const int64_t L = leaf_base + lpos[i];
        for (int k = 0; k < 12; ++k) lf_R[12 * L + k] = it_R[12 * i + k];
        lf_t[2 * L] = ta;
        lf_t[2 * L + 1] = tb;
        lf_span[L] = s;
        atomicAdd(&span_nleaf[s], 1);
        return;
    }
    const int p = deg[span_curve[s]];
    const double z = (double)it_z[i] / 128.0;
    const double tm = ta + z * (tb - ta);
    const int64_t j = 2 * (int64_t)cpos[i];
    double* Ql = nx_Q + j * q_stride;
    double* Qr = Ql + q_stride;
    const int p0 = __builtin_amdgcn_readfirstlane(p);
    if (__all(p == p0)) {
        split_degree<MP>(p0, it_Q + i * (int64_t)q_stride, z, Ql, Qr);
    } else {
        double Lq[(MP + 1) * 3], Rq[(MP + 1) * 3];
        dm::split_piece(p, it_Q + i * (int64_t)q_stride, z, Lq, Rq);
        for (int k = 0; k < 3 * (p + 1); ++k) {
            Ql[k] = Lq[k];
            Qr[k] = Rq[k];
        }
    }
    nx_span[j] = s;
    nx_span[j + 1] = s;
    nx_t[2 * j] = ta;
    nx_t[2 * j + 1] = tm;
    nx_t[2 * j + 2] = tm;
    nx_t[2 * j + 3] = tb;
}

// 6. parameter order inside each span: slot of every leaf, then one insertion
//    sort per span by t_a (the breakpoints of a span are strictly increasing)
__global__ void k_dd_place(int64_t n_leaves, const int32_t* __restrict__ lf_span, const int32_t* __restrict__ span0,
                           int32_t* __restrict__ cursor, int32_t* __restrict__ perm)
{
    const int64_t L = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (L >= n_leaves) return;
    const int32_t s = lf_span[L];
    perm[span0[s] + atomicAdd(&cursor[s], 1)] = (int32_t)L;
}

__global__ void k_dd_sort(int64_t n_span, const int32_t* __restrict__ span0, const double* __restrict__ lf_t,
                          int32_t* __restrict__ perm)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n_span) return;
    const int32_t a = span0[s], b = span0[s + 1];
    for (int32_t k = a + 1; k < b; ++k) {
        const int32_t v = perm[k];
        const double key = lf_t[2 * (int64_t)v];
        int32_t m = k - 1;
        while (m >= a && lf_t[2 * (int64_t)perm[m]] > key) {
            perm[m + 1] = perm[m];
            --m;
        }
        perm[m + 1] = v;
    }
}

__global__ void k_dd_gather(int64_t n_seg, const int32_t* __restrict__ perm, const double* __restrict__ lf_R,
                            const double* __restrict__ lf_t, const int32_t* __restrict__ lf_span,
                            double* __restrict__ seg_cp, double* __restrict__ seg_t, int32_t* __restrict__ seg_span)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= n_seg) return;
    const int64_t L = perm[g];
    for (int k = 0; k < 12; ++k) seg_cp[12 * g + k] = lf_R[12 * L + k];
    seg_t[2 * g] = lf_t[2 * L];
    seg_t[2 * g + 1] = lf_t[2 * L + 1];
    seg_span[g] = lf_span[L];
}

// per curve: first piece and cluster counts
__global__ void k_dd_curve_segs(int32_t n_curves, const int64_t* __restrict__ span_off,
                                const int32_t* __restrict__ span0, int64_t* __restrict__ seg_off,
                                int32_t* __restrict__ n_clu)
{
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c > n_curves) return;
    seg_off[c] = span0[span_off[c]];
    if (c == n_curves) return;
    const int64_t ns = (int64_t)span0[span_off[c + 1]] - span0[span_off[c]];
    n_clu[c] = (int32_t)((ns + kCluPieces - 1) / kCluPieces);
}

// ---------------------------------------------------------------------------
// tables of the geometry buffer (the layout of mrep_upload)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_dd_pieces(int64_t n_seg, const int32_t* __restrict__ seg_span,
                                                      const int32_t* __restrict__ span_curve,
                                                      const double* __restrict__ origin,
                                                      const double* __restrict__ tol_eff,
                                                      const double* __restrict__ seg_cp, uint16_t* __restrict__ col,
                                                      float* __restrict__ aux, float* __restrict__ lcp,
                                                      float* __restrict__ sph)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= n_seg) return;
    const int c = span_curve[seg_span[g]];
    double R[12], o[3];
    for (int k = 0; k < 12; ++k) R[k] = seg_cp[12 * g + k];
    for (int k = 0; k < 3; ++k) o[k] = origin[3 * c + k];
    uint16_t cl[kScreenK];
    float ax[8], lc[12], sp[4];
    for (int k = 0; k < 8; ++k) ax[k] = 0.f;
    dm::piece_tables(R, o, tol_eff[c], cl, ax, lc);
    dm::piece_sphere(ax, lc, tol_eff[c], sp);
    for (int k = 0; k < kScreenK; ++k) col[kScreenK * g + k] = cl[k];
    for (int k = 0; k < 8; ++k) aux[8 * g + k] = ax[k];
    for (int k = 0; k < 12; ++k) lcp[12 * g + k] = lc[k];
    for (int k = 0; k < 4; ++k) sph[4 * g + k] = sp[k];
}

__global__ void k_dd_dcurve(int32_t n_curves, double tol_rel, const int32_t* __restrict__ deg,
                            const double* __restrict__ diag, const double* __restrict__ origin,
                            const double* __restrict__ tol_eff, const int64_t* __restrict__ span_off,
                            const int64_t* __restrict__ coef_off, const int64_t* __restrict__ seg_off,
                            const int64_t* __restrict__ clu_off, const float* __restrict__ aux,
                            const float* __restrict__ sph, float* __restrict__ csph, DCurve* __restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n_curves) return;
    DCurve d;
    d.seg_off = seg_off[c];
    d.span_off = span_off[c];
    d.coef_off = coef_off[c];
    d.n_seg = (int32_t)(seg_off[c + 1] - seg_off[c]);
    d.n_span = (int32_t)(span_off[c + 1] - span_off[c]);
    d.degree = deg[c];
    d.tol_eff = tol_eff[c];
    d.tol_user = tol_rel * diag[c];
    d.diag = diag[c];
    for (int k = 0; k < 3; ++k) d.origin[k] = origin[3 * c + k];
    d.clu_off = clu_off[c];
    d.n_clu = (int32_t)(clu_off[c + 1] - clu_off[c]);
    d.rational = 0;
    d.pad_ = 0;
    float es = 0.f;
    for (int64_t g = d.seg_off; g < d.seg_off + d.n_seg; ++g) es = dm::mx(es, aux[8 * g + AUX_ES]);
    d.es_max = es;
    double rsum = 0.0;
    for (int32_t k = 0; k < d.n_clu; ++k) {
        const int64_t a = d.seg_off + (int64_t)k * kCluPieces;
        const int64_t m = dm::mn<int64_t>(kCluPieces, d.n_seg - (int64_t)k * kCluPieces);
        float* cs = csph + 4 * (d.clu_off + k);
        dm::bounding_sphere(sph + 4 * a, m, cs);
        rsum += cs[3];
    }
    d.clu_use = d.n_clu >= 4 && d.n_clu < 65536 && rsum / d.n_clu <= 0.1 * d.diag ? 1 : 0;
    out[c] = d;
}

// Errors of k_dd_curve as the host decomposition reports them.
void curve_error(int e, int32_t& code, std::string& msg)
{
    code = MREP_E_BAD_KNOTS;
    switch (e) {
        case kErrNonFinitePoint: code = MREP_E_INVALID_ARG; msg = "non-finite control point"; break;
        case kErrNonFiniteKnot: msg = "non-finite knot"; break;
        case kErrKnotOrder: msg = "knots not non-decreasing"; break;
        case kErrNotClamped: msg = "knot vector not clamped"; break;
        case kErrEmptyDomain: msg = "empty parameter domain"; break;
        case kErrMultiplicity: msg = "interior knot multiplicity > degree"; break;
        default: msg = "knot vector not clamped (multiplicity > p+1 at an end)"; break;
    }
}

// Kernels instantiated for the batch's largest degree (their arrays).
template <int MP>
void launch_spans(unsigned grid, hipStream_t st, int32_t n_curves, int64_t n_iv, const int32_t* deg,
                  const int64_t* cp_off, const int64_t* knot_off, const int64_t* iv_off, const double* cp,
                  const double* knots, const dm::DegreeTables* tab, const int32_t* ne, const int32_t* sidx,
                  const int64_t* span_off, const int64_t* coef_off, int32_t* span_curve, double* span_t, double* coef,
                  int32_t* it_span, double* it_t, double* it_Q, int32_t q_stride)
{
    hipLaunchKernelGGL(k_dd_spans<MP>, dim3(grid), dim3(kBlock), 0, st, n_curves, n_iv, deg, cp_off, knot_off,
                       iv_off, cp, knots, tab, ne, sidx, span_off, coef_off, span_curve, span_t, coef, it_span, it_t,
                       it_Q, q_stride);
}

template <int MP>
void launch_emit(unsigned grid, hipStream_t st, int64_t n, const int32_t* deg, const int32_t* span_curve,
                 const int32_t* it_span, const double* it_t, const double* it_Q, int32_t q_stride, const double* it_R,
                 const int32_t* it_z, const int32_t* is_leaf, const int32_t* lpos, const int32_t* cpos,
                 int64_t leaf_base, double* lf_R, double* lf_t, int32_t* lf_span, int32_t* span_nleaf,
                 int32_t* nx_span, double* nx_t, double* nx_Q)
{
    hipLaunchKernelGGL(k_dd_emit<MP>, dim3(grid), dim3(kBlock), 0, st, n, deg, span_curve, it_span, it_t, it_Q,
                       q_stride, it_R, it_z, is_leaf, lpos, cpos, leaf_base, lf_R, lf_t, lf_span, span_nleaf,
                       nx_span, nx_t, nx_Q);
}

// degree bound of the instantiation used for a batch
int degree_class(int pmax) { return pmax <= 5 ? 5 : (pmax <= 9 ? 9 : 15); }

}  // namespace

DevPlan::~DevPlan()
{
    dfree(deg); dfree(diag); dfree(origin); dfree(tol_eff);
    dfree(span_off); dfree(coef_off); dfree(seg_off); dfree(clu_off);
    dfree(span_curve); dfree(span_t); dfree(span0); dfree(coef);
    dfree(seg_cp); dfree(seg_t); dfree(seg_span);
}

void devplan_free(DevPlan* d) { delete d; }

// Everything of one decomposition call that is freed when it returns.
struct DdTemps {
    int64_t* cp_off = nullptr;
    int64_t* knot_off = nullptr;
    int64_t* iv_off = nullptr;
    dm::DegreeTables* tab = nullptr;
    int32_t* err = nullptr;
    double* tol_abs = nullptr;
    int32_t* ne = nullptr;
    int32_t* sidx = nullptr;
    int32_t* cnt = nullptr;      // device counters: [0] spans, [1] leaves, [2] splits, [3] fail, [4] clusters
    int64_t* cnt64 = nullptr;    // [0] coef doubles
    int64_t* coef_n = nullptr;
    int32_t* splits = nullptr;
    int32_t* span_nleaf = nullptr;
    int32_t* n_clu = nullptr;
    int32_t* perm = nullptr;
    double* lf_R = nullptr;
    double* lf_t = nullptr;
    int32_t* lf_span = nullptr;
    int64_t lf_cap = 0;
    ~DdTemps()
    {
        dfree(cp_off); dfree(knot_off); dfree(iv_off); dfree(tab); dfree(err); dfree(tol_abs); dfree(ne);
        dfree(sidx); dfree(cnt); dfree(cnt64); dfree(coef_n); dfree(splits); dfree(span_nleaf); dfree(n_clu);
        dfree(perm); dfree(lf_R); dfree(lf_t); dfree(lf_span);
    }
};

// Items of one level.  The two level buffers are reused from level to level
// and only grow (by half again), so a decomposition makes a handful of
// allocations instead of a set per level.
struct Level {
    int32_t* span = nullptr;
    double* t = nullptr;
    double* Q = nullptr;
    double* R = nullptr;
    int32_t* z = nullptr;
    int32_t* leaf = nullptr;
    int32_t* split = nullptr;
    int32_t* lpos = nullptr;
    int32_t* cpos = nullptr;
    int64_t cap = 0;
    ~Level() { release(); }
    void release()
    {
        dfree(span); dfree(t); dfree(Q); dfree(R); dfree(z); dfree(leaf); dfree(split); dfree(lpos); dfree(cpos);
        cap = 0;
    }
    hipError_t ensure(int64_t n, int32_t stride)
    {
        if (n <= cap) return hipSuccess;
        release();
        return alloc(std::max<int64_t>(n, cap + cap / 2), stride);
    }
    hipError_t alloc(int64_t n, int32_t stride)
    {
        hipError_t e;
        cap = n;
        if ((e = dmalloc(&span, n)) != hipSuccess) return e;
        if ((e = dmalloc(&t, 2 * n)) != hipSuccess) return e;
        if ((e = dmalloc(&Q, n * stride)) != hipSuccess) return e;
        if ((e = dmalloc(&R, 12 * n)) != hipSuccess) return e;
        if ((e = dmalloc(&z, n)) != hipSuccess) return e;
        if ((e = dmalloc(&leaf, n)) != hipSuccess) return e;
        if ((e = dmalloc(&split, n)) != hipSuccess) return e;
        if ((e = dmalloc(&lpos, n)) != hipSuccess) return e;
        return dmalloc(&cpos, n);
    }
};

int device_decompose(int32_t n_curves, const int32_t* degree, const int64_t* cp_off, const int64_t* knot_off,
                     const double* cp_xyz, const double* knots, double tol_rel, hipStream_t st, DevPlan** out)
{
    // host checks (the host decomposition's, plus the device degree range)
    std::vector<int64_t> iv((size_t)n_curves + 1, 0);
    int pmax = 1;
    for (int32_t c = 0; c < n_curves; ++c) {
        const int64_t n = cp_off[c + 1] - cp_off[c], nk = knot_off[c + 1] - knot_off[c];
        const std::string who = "mrep_decompose_curves_device: curve " + std::to_string(c) + ": ";
        if (n < 0 || nk < 0) { set_error("mrep_decompose_curves_device: negative CSR extent"); return MREP_E_INVALID_ARG; }
        if (degree[c] < 1 || degree[c] > MREP_SPAN_MAX_DEGREE) {
            set_error(who + "degree outside 1..15 (higher degrees and rational curves: mrep_decompose_curves)");
            return MREP_E_BAD_DEGREE;
        }
        if (n < degree[c] + 1) { set_error(who + "fewer than p+1 control points"); return MREP_E_BAD_DEGREE; }
        if (nk != n + degree[c] + 1) { set_error(who + "knot count != points + p + 1"); return MREP_E_BAD_KNOTS; }
        if (n > (int64_t)1 << 24) { set_error(who + "curve too long"); return MREP_E_INVALID_ARG; }
        iv[(size_t)c + 1] = iv[(size_t)c] + (n - degree[c]);
        pmax = std::max(pmax, degree[c]);
    }
    const int64_t n_iv = iv[(size_t)n_curves];
    if (n_iv >= INT32_MAX) { set_error("mrep_decompose_curves_device: more than 2^31 knot intervals"); return MREP_E_INVALID_ARG; }
    const int mp = degree_class(pmax);
    const int32_t stride = 3 * (mp + 1);
    DdTemps T;
    DevPlan* D = new DevPlan();
    std::unique_ptr<DevPlan> hold(D);
    D->n_curves = n_curves;
    D->tol_rel = tol_rel;
    D->max_degree = pmax;
    DD_HIP(dmalloc(&D->deg, n_curves));
    DD_HIP(dmalloc(&T.cp_off, n_curves + 1));
    DD_HIP(dmalloc(&T.knot_off, n_curves + 1));
    DD_HIP(dmalloc(&T.iv_off, n_curves + 1));
    DD_HIP(dmalloc(&T.tab, dm::kMaxP + 1));
    DD_HIP(dmalloc(&T.err, n_curves));
    DD_HIP(dmalloc(&T.tol_abs, n_curves));
    DD_HIP(dmalloc(&D->diag, n_curves));
    DD_HIP(dmalloc(&D->origin, 3 * (int64_t)n_curves));
    DD_HIP(dmalloc(&D->tol_eff, n_curves));
    DD_HIP(dmalloc(&T.cnt, 8));
    DD_HIP(dmalloc(&T.cnt64, 2));
    DD_HIP(hipMemcpyAsync(D->deg, degree, sizeof(int32_t) * n_curves, hipMemcpyHostToDevice, st));
    DD_HIP(hipMemcpyAsync(T.cp_off, cp_off, sizeof(int64_t) * (n_curves + 1), hipMemcpyHostToDevice, st));
    DD_HIP(hipMemcpyAsync(T.knot_off, knot_off, sizeof(int64_t) * (n_curves + 1), hipMemcpyHostToDevice, st));
    DD_HIP(hipMemcpyAsync(T.iv_off, iv.data(), sizeof(int64_t) * (n_curves + 1), hipMemcpyHostToDevice, st));
    DD_HIP(hipMemcpyAsync(T.tab, dm::degree_tables_host(), sizeof(dm::DegreeTables) * (dm::kMaxP + 1),
                          hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(kBlock), 0, st, T.cnt, (int64_t)8, 0);
    // 1. curves
    hipLaunchKernelGGL(k_dd_curve, dim3(blocks_of(n_curves)), dim3(kBlock), 0, st, n_curves, D->deg, T.cp_off,
                       T.knot_off, cp_xyz, knots, tol_rel, T.err, D->diag, D->origin, T.tol_abs, D->tol_eff);
    DD_HIP(hipGetLastError());
    {
        std::vector<int32_t> err((size_t)n_curves);
        DD_HIP(hipMemcpyAsync(err.data(), T.err, sizeof(int32_t) * n_curves, hipMemcpyDeviceToHost, st));
        DD_HIP(hipStreamSynchronize(st));
        for (int32_t c = 0; c < n_curves; ++c)
            if (err[(size_t)c]) {
                int32_t code;
                std::string msg;
                curve_error(err[(size_t)c], code, msg);
                set_error("mrep_decompose_curves_device: curve " + std::to_string(c) + ": " + msg);
                return code;
            }
    }
    // 2. spans: non-empty intervals, their global index, per-curve offsets
    Scanner sc;
    DD_HIP(dmalloc(&T.ne, n_iv));
    DD_HIP(dmalloc(&T.sidx, n_iv));
    if (n_iv > 0)
        hipLaunchKernelGGL(k_dd_nonempty, dim3(blocks_of(n_iv)), dim3(kBlock), 0, st, n_curves, n_iv, D->deg,
                           T.knot_off, T.iv_off, knots, T.ne);
    DD_HIP(hipGetLastError());
    DD_HIP(sc.run(T.ne, n_iv, T.sidx, T.cnt + 0, st));
    DD_HIP(dmalloc(&D->span_off, n_curves + 1));
    DD_HIP(dmalloc(&D->coef_off, n_curves + 1));
    DD_HIP(dmalloc(&T.coef_n, n_curves + 1));
    hipLaunchKernelGGL(k_dd_curve_spans, dim3(blocks_of(n_curves + 1)), dim3(kBlock), 0, st, n_curves, n_iv, D->deg,
                       T.iv_off, T.sidx, T.cnt + 0, D->span_off, T.coef_n);
    DD_HIP(hipGetLastError());
    DD_HIP(sc.run(T.coef_n, n_curves, D->coef_off, T.cnt64 + 0, st));
    int32_t n_span = 0;
    int64_t n_coef = 0;
    DD_HIP(hipMemcpyAsync(&n_span, T.cnt + 0, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    DD_HIP(hipMemcpyAsync(&n_coef, T.cnt64 + 0, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    DD_HIP(hipStreamSynchronize(st));
    // the coef scan's last entry is the total
    DD_HIP(hipMemcpyAsync(D->coef_off + n_curves, T.cnt64 + 0, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    D->n_span = n_span;
    D->n_coef = n_coef;
    DD_HIP(dmalloc(&D->span_curve, n_span));
    DD_HIP(dmalloc(&D->span_t, 2 * (int64_t)n_span));
    DD_HIP(dmalloc(&D->coef, n_coef));
    DD_HIP(dmalloc(&D->span0, (int64_t)n_span + 1));
    DD_HIP(dmalloc(&T.splits, n_span));
    DD_HIP(dmalloc(&T.span_nleaf, (int64_t)n_span + 1));
    if (n_span > 0) {
        hipLaunchKernelGGL(k_fill<int32_t>, dim3(blocks_of(n_span)), dim3(kBlock), 0, st, T.splits, (int64_t)n_span, 0);
        hipLaunchKernelGGL(k_fill<int32_t>, dim3(blocks_of(n_span + 1)), dim3(kBlock), 0, st, T.span_nleaf,
                           (int64_t)n_span + 1, 0);
    }
    // 3. exact span forms; level 0 = every span
    Level cur, nxt;
    int64_t n_items = n_span;
    DD_HIP(cur.ensure(n_items, stride));
    if (n_iv > 0) {
        const unsigned g = blocks_of(n_iv);
        if (mp == 5)
            launch_spans<5>(g, st, n_curves, n_iv, D->deg, T.cp_off, T.knot_off, T.iv_off, cp_xyz, knots, T.tab, T.ne,
                            T.sidx, D->span_off, D->coef_off, D->span_curve, D->span_t, D->coef, cur.span, cur.t, cur.Q,
                            stride);
        else if (mp == 9)
            launch_spans<9>(g, st, n_curves, n_iv, D->deg, T.cp_off, T.knot_off, T.iv_off, cp_xyz, knots, T.tab, T.ne,
                            T.sidx, D->span_off, D->coef_off, D->span_curve, D->span_t, D->coef, cur.span, cur.t, cur.Q,
                            stride);
        else
            launch_spans<15>(g, st, n_curves, n_iv, D->deg, T.cp_off, T.knot_off, T.iv_off, cp_xyz, knots, T.tab, T.ne,
                             T.sidx, D->span_off, D->coef_off, D->span_curve, D->span_t, D->coef, cur.span, cur.t,
                             cur.Q, stride);
        DD_HIP(hipGetLastError());
    }
    dfree(T.ne);
    dfree(T.sidx);
    // 4-5. levels
    int64_t n_leaves = 0;
    while (n_items > 0) {
        const unsigned g = blocks_of(n_items);
#define DD_LEVEL(MPV)                                                                                              \
    hipLaunchKernelGGL(k_dd_level<MPV>, dim3(g), dim3(kBlock), 0, st, n_items, D->deg, D->span_curve, T.tol_abs, T.tab, \
                       cur.span, cur.Q, stride, cur.R, cur.z, cur.leaf, cur.split, T.splits, T.cnt + 3)
        if (mp == 5) DD_LEVEL(5);
        else if (mp == 9) DD_LEVEL(9);
        else DD_LEVEL(15);
#undef DD_LEVEL
        DD_HIP(hipGetLastError());
        DD_HIP(sc.run(cur.leaf, n_items, cur.lpos, T.cnt + 1, st));
        DD_HIP(sc.run(cur.split, n_items, cur.cpos, T.cnt + 2, st));
        int32_t h[4];
        DD_HIP(hipMemcpyAsync(h, T.cnt, sizeof(int32_t) * 4, hipMemcpyDeviceToHost, st));
        DD_HIP(hipStreamSynchronize(st));
        if (h[3]) {
            set_error("mrep_decompose_curves_device: a span needed more than MREP_MAX_PIECES_PER_SPAN pieces");
            return MREP_E_TOL;
        }
        const int64_t nl = h[1], ns = h[2];
        if (n_leaves + nl >= INT32_MAX || 2 * ns >= INT32_MAX) {
            set_error("mrep_decompose_curves_device: more than 2^31 pieces");
            return MREP_E_INVALID_ARG;
        }
        if (n_leaves + nl > T.lf_cap) {
            // grow the leaf arrays (geometric, from four pieces per span), keeping what is there
            const int64_t cap = std::max<int64_t>(std::max<int64_t>(n_leaves + nl, 2 * T.lf_cap), 4 * (int64_t)n_span);
            double *R2 = nullptr, *t2 = nullptr;
            int32_t* s2 = nullptr;
            DD_HIP(dmalloc(&R2, 12 * cap));
            DD_HIP(dmalloc(&t2, 2 * cap));
            DD_HIP(dmalloc(&s2, cap));
            if (n_leaves > 0) {
                DD_HIP(hipMemcpyAsync(R2, T.lf_R, sizeof(double) * 12 * n_leaves, hipMemcpyDeviceToDevice, st));
                DD_HIP(hipMemcpyAsync(t2, T.lf_t, sizeof(double) * 2 * n_leaves, hipMemcpyDeviceToDevice, st));
                DD_HIP(hipMemcpyAsync(s2, T.lf_span, sizeof(int32_t) * n_leaves, hipMemcpyDeviceToDevice, st));
                DD_HIP(hipStreamSynchronize(st));
            }
            dfree(T.lf_R); dfree(T.lf_t); dfree(T.lf_span);
            T.lf_R = R2; T.lf_t = t2; T.lf_span = s2;
            T.lf_cap = cap;
        }
        DD_HIP(nxt.ensure(2 * ns, stride));
        if (mp == 5)
            launch_emit<5>(g, st, n_items, D->deg, D->span_curve, cur.span, cur.t, cur.Q, stride, cur.R, cur.z, cur.leaf,
                           cur.lpos, cur.cpos, n_leaves, T.lf_R, T.lf_t, T.lf_span, T.span_nleaf, nxt.span, nxt.t, nxt.Q);
        else if (mp == 9)
            launch_emit<9>(g, st, n_items, D->deg, D->span_curve, cur.span, cur.t, cur.Q, stride, cur.R, cur.z, cur.leaf,
                           cur.lpos, cur.cpos, n_leaves, T.lf_R, T.lf_t, T.lf_span, T.span_nleaf, nxt.span, nxt.t, nxt.Q);
        else
            launch_emit<15>(g, st, n_items, D->deg, D->span_curve, cur.span, cur.t, cur.Q, stride, cur.R, cur.z,
                            cur.leaf, cur.lpos, cur.cpos, n_leaves, T.lf_R, T.lf_t, T.lf_span, T.span_nleaf, nxt.span,
                            nxt.t, nxt.Q);
        DD_HIP(hipGetLastError());
        DD_HIP(hipStreamSynchronize(st));
        n_leaves += nl;
        n_items = 2 * ns;
        std::swap(cur.span, nxt.span); std::swap(cur.t, nxt.t); std::swap(cur.Q, nxt.Q); std::swap(cur.R, nxt.R);
        std::swap(cur.z, nxt.z); std::swap(cur.leaf, nxt.leaf); std::swap(cur.split, nxt.split);
        std::swap(cur.lpos, nxt.lpos); std::swap(cur.cpos, nxt.cpos); std::swap(cur.cap, nxt.cap);
    }
    cur.release();
    nxt.release();
    D->n_seg = n_leaves;
    // 6. order: first piece of each span, slots, per-span sort, gather
    DD_HIP(sc.run(T.span_nleaf, (int64_t)n_span + 1, D->span0, (int32_t*)nullptr, st));
    DD_HIP(dmalloc(&T.perm, n_leaves));
    DD_HIP(dmalloc(&D->seg_cp, 12 * n_leaves));
    DD_HIP(dmalloc(&D->seg_t, 2 * n_leaves));
    DD_HIP(dmalloc(&D->seg_span, n_leaves));
    if (n_span > 0)
        hipLaunchKernelGGL(k_fill<int32_t>, dim3(blocks_of(n_span)), dim3(kBlock), 0, st, T.splits, (int64_t)n_span, 0);
    if (n_leaves > 0) {
        hipLaunchKernelGGL(k_dd_place, dim3(blocks_of(n_leaves)), dim3(kBlock), 0, st, n_leaves, T.lf_span, D->span0,
                           T.splits, T.perm);
        hipLaunchKernelGGL(k_dd_sort, dim3(blocks_of(n_span)), dim3(kBlock), 0, st, (int64_t)n_span, D->span0,
                           T.lf_t, T.perm);
        hipLaunchKernelGGL(k_dd_gather, dim3(blocks_of(n_leaves)), dim3(kBlock), 0, st, n_leaves, T.perm, T.lf_R,
                           T.lf_t, T.lf_span, D->seg_cp, D->seg_t, D->seg_span);
        DD_HIP(hipGetLastError());
    }
    // per curve: pieces and clusters
    DD_HIP(dmalloc(&D->seg_off, n_curves + 1));
    DD_HIP(dmalloc(&D->clu_off, n_curves + 1));
    DD_HIP(dmalloc(&T.n_clu, n_curves + 1));
    hipLaunchKernelGGL(k_dd_curve_segs, dim3(blocks_of(n_curves + 1)), dim3(kBlock), 0, st, n_curves, D->span_off,
                       D->span0, D->seg_off, T.n_clu);
    DD_HIP(hipGetLastError());
    DD_HIP(hipMemsetAsync(T.cnt64 + 1, 0, sizeof(int64_t), st));
    {
        // cluster offsets: int32 counts, int64 offsets
        std::vector<int32_t> ncl((size_t)n_curves);
        DD_HIP(hipMemcpyAsync(ncl.data(), T.n_clu, sizeof(int32_t) * n_curves, hipMemcpyDeviceToHost, st));
        DD_HIP(hipStreamSynchronize(st));
        std::vector<int64_t> off((size_t)n_curves + 1, 0);
        for (int32_t c = 0; c < n_curves; ++c) off[(size_t)c + 1] = off[(size_t)c] + ncl[(size_t)c];
        D->n_clu = off[(size_t)n_curves];
        DD_HIP(hipMemcpyAsync(D->clu_off, off.data(), sizeof(int64_t) * (n_curves + 1), hipMemcpyHostToDevice, st));
        DD_HIP(hipStreamSynchronize(st));
    }
    curve_layout(D->layout, n_curves, D->n_seg, D->n_span, D->n_coef, D->n_clu);
    D->layout.general = pmax > MREP_POWER_MAX_DEGREE ? 1 : 0;
    DD_HIP(hipStreamSynchronize(st));
    *out = hold.release();
    return MREP_OK;
}

int devplan_upload(const DevPlan& D, char* b, hipStream_t st)
{
    const GeomLayout& L = D.layout;
    auto cp = [&](int64_t off, const void* src, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        return hipMemcpyAsync(b + off, src, n, hipMemcpyDeviceToDevice, st);
    };
    DD_HIP(cp(L.off_gcp, D.seg_cp, sizeof(double) * 12 * D.n_seg));
    DD_HIP(cp(L.off_segt, D.seg_t, sizeof(double) * 2 * D.n_seg));
    DD_HIP(cp(L.off_segspan, D.seg_span, sizeof(int32_t) * D.n_seg));
    DD_HIP(cp(L.off_spant, D.span_t, sizeof(double) * 2 * D.n_span));
    DD_HIP(cp(L.off_span0, D.span0, sizeof(int32_t) * (D.n_span + 1)));
    DD_HIP(cp(L.off_coef, D.coef, sizeof(double) * D.n_coef));
    if (D.n_seg > 0)
        hipLaunchKernelGGL(k_dd_pieces, dim3(blocks_of(D.n_seg)), dim3(kBlock), 0, st, D.n_seg, D.seg_span,
                           D.span_curve, D.origin, D.tol_eff, D.seg_cp, (uint16_t*)(b + L.off_col),
                           (float*)(b + L.off_aux), (float*)(b + L.off_lcp), (float*)(b + L.off_sph));
    DD_HIP(hipGetLastError());
    if (D.n_curves > 0)
        hipLaunchKernelGGL(k_dd_dcurve, dim3(blocks_of(D.n_curves)), dim3(kBlock), 0, st, (int32_t)D.n_curves,
                           D.tol_rel, D.deg, D.diag, D.origin, D.tol_eff, D.span_off, D.coef_off, D.seg_off, D.clu_off,
                           (const float*)(b + L.off_aux), (const float*)(b + L.off_sph), (float*)(b + L.off_csph),
                           (DCurve*)(b + L.off_curve));
    DD_HIP(hipGetLastError());
    DD_HIP(hipStreamSynchronize(st));
    return MREP_OK;
}

int devplan_export(const DevPlan& D, int64_t* seg_off, double* seg_t, double* seg_cp, int32_t* seg_span)
{
    if (seg_off) DD_HIP(hipMemcpy(seg_off, D.seg_off, sizeof(int64_t) * (D.n_curves + 1), hipMemcpyDeviceToHost));
    if (seg_t && D.n_seg) DD_HIP(hipMemcpy(seg_t, D.seg_t, sizeof(double) * 2 * D.n_seg, hipMemcpyDeviceToHost));
    if (seg_cp && D.n_seg) DD_HIP(hipMemcpy(seg_cp, D.seg_cp, sizeof(double) * 12 * D.n_seg, hipMemcpyDeviceToHost));
    if (seg_span && D.n_seg) DD_HIP(hipMemcpy(seg_span, D.seg_span, sizeof(int32_t) * D.n_seg, hipMemcpyDeviceToHost));
    return MREP_OK;
}

const GeomLayout& devplan_layout(const DevPlan& D) { return D.layout; }
int32_t devplan_max_degree(const DevPlan& D) { return D.max_degree; }
double devplan_tol_rel(const DevPlan& D) { return D.tol_rel; }

}  // namespace mrep

extern "C" int32_t mrep_decompose_curves_device(int32_t n_curves, const int32_t* degree, const int64_t* cp_off,
                                                const double* cp_xyz, const int64_t* knot_off, const double* knots,
                                                double tol_rel, void* stream, mrep_plan** out)
{
    if (!out) {
        mrep::set_error("mrep_decompose_curves_device: null output");
        return MREP_E_INVALID_ARG;
    }
    *out = nullptr;
    if (n_curves <= 0 || !degree || !cp_off || !knot_off || !cp_xyz || !knots) {
        mrep::set_error("mrep_decompose_curves_device: null pointer or no curves");
        return MREP_E_INVALID_ARG;
    }
    if (!(tol_rel > 0.0) || !(tol_rel < 1.0)) {
        mrep::set_error("mrep_decompose_curves_device: tol_rel must be in (0, 1)");
        return MREP_E_INVALID_ARG;
    }
    int rc = mrep::check_device();
    if (rc) return rc;
    mrep::DevPlan* d = nullptr;
    rc = mrep::device_decompose(n_curves, degree, cp_off, knot_off, cp_xyz, knots, tol_rel, (hipStream_t)stream, &d);
    if (rc) return rc;
    mrep_plan* p = new mrep_plan();
    p->kind = MREP_GEOM_CURVES;
    p->dev = d;
    *out = p;
    return MREP_OK;
}
