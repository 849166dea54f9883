// Host-side M-rep decomposition of clamped B-spline curves (FP64).
//
// Each non-degenerate knot span q is converted to its exact Bezier form in the
// matrix form of Sec. 5.2.1:  Q_q = B_p^{-1} M_{q,p,T} A_{q,p,T} [P_{q-p} .. P_q]
// (eqs. bsplinematrix, Mqpt, decomposition, decomfinal).  A_{q,p,T} holds the
// power coefficients of the p+1 basis functions that live on the span; they are
// produced by running the Cox-de Boor recursion (eq. bsplinebasis) on
// polynomials.  We expand them in the span-local shifted variable s = t - t_q,
// which turns M_{q,p,T} into diag(h^j), h = t_{q+1} - t_q: the binomial terms
// t_q^{i-j} of the paper's M only move the origin of the power basis, and an
// origin at t = 0 would cost ~(t_q/h)^p of FP64 precision for short spans far
// from the origin.
//
// Cubic conversion (Sec. 5.2.2): p = 3 keeps Q, p <= 2 elevates it, p >= 4
// takes the G1-continuous cubic R (eq. G1-condition) whose (delta0, delta1)
// minimise the L2 deviation (eq. epsl), from the 2x2 system obtained by setting
// the derivatives of eqs. differentiatedelta0/1 to zero with the Gram matrices
// of eq. gram.  A cubic whose deviation bound exceeds the tolerance is replaced
// by splitting the ORIGINAL degree-p piece with the degree-p form of the
// subdivision matrix S(z) (eqs. submatrix, subLandR) at the sample of largest
// deviation and reducing both halves again, so that the split point lies on
// the original curve (the effect of the paper's control-polygon modification).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <thread>

#include "../../include/mrep.h"
#include "mrep_decomp.h"
#include "mrep_internal.h"

namespace mrep {

namespace {

// The arithmetic that the device decomposition repeats bit for bit lives in
// mrep_decomp.h; the host-only parts (degree > 15, rational spans) stay here.
using dm::binom;
using dm::bf16_to_f32;
using dm::bounding_sphere;
using dm::DegreeTables;
using dm::deviation_bound;
using dm::dot3;
using dm::g1_reduce;
using dm::ipow;
using dm::kErrSamples;
using dm::kMaxP;
using dm::piece_sphere;
using dm::piece_tables;
using dm::split_piece;

inline void span_basis_poly(int p, const double* U, int q, double* A) { dm::span_basis_poly<kMaxP>(p, U, q, A); }


DegreeTables g_tab[kMaxP + 1];
std::atomic<int> g_tab_ready{0};

void elevation_matrix(int p, double* E)  // (p+2) x (p+1): degree p -> p+1
{
    for (int i = 0; i <= p + 1; ++i)
        for (int j = 0; j <= p; ++j) {
            double a = (double)i / (double)(p + 1);
            double v = 0.0;
            if (j == i - 1) v += a;
            if (j == i) v += 1.0 - a;
            E[i * (p + 1) + j] = v;
        }
}

void init_tables()
{
    if (g_tab_ready.load(std::memory_order_acquire)) return;
    static std::atomic<int> once{0};
    int expected = 0;
    if (!once.compare_exchange_strong(expected, 1)) {
        while (!g_tab_ready.load(std::memory_order_acquire)) std::this_thread::yield();
        return;
    }
    for (int p = 1; p <= kMaxP; ++p) {
        DegreeTables& T = g_tab[p];
        T.p = p;
        bernstein_inverse(p, T.Bi);
        for (int i = 0; i < kErrSamples; ++i) {
            double u = (double)i / (double)(kErrSamples - 1);
            for (int k = 0; k <= p; ++k) T.Bq[i * (p + 1) + k] = binom(p, k) * ipow(u, k) * ipow(1.0 - u, p - k);
            for (int k = 0; k <= 3; ++k) T.B3[i * 4 + k] = binom(3, k) * ipow(u, k) * ipow(1.0 - u, 3 - k);
        }
        // E3p = E_{p-1} ... E_3 (identity for p <= 3)
        double cur[(kMaxP + 1) * 4], nxt[(kMaxP + 1) * 4], E[(kMaxP + 2) * (kMaxP + 1)];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) cur[i * 4 + j] = (i == j) ? 1.0 : 0.0;
        for (int d = 3; d < p; ++d) {
            elevation_matrix(d, E);
            for (int i = 0; i <= d + 1; ++i)
                for (int j = 0; j < 4; ++j) {
                    double s = 0.0;
                    for (int k = 0; k <= d; ++k) s += E[i * (d + 1) + k] * cur[k * 4 + j];
                    nxt[i * 4 + j] = s;
                }
            memcpy(cur, nxt, sizeof(double) * 4 * (size_t)(d + 2));
        }
        if (p >= 3) memcpy(T.E3p, cur, sizeof(double) * 4 * (size_t)(p + 1));
        gram_matrix(3, p, T.G3p);
        gram_matrix(3, 3, T.G33);
    }
    g_tab_ready.store(1, std::memory_order_release);
}

struct Piece {
    double R[12];
    double ta, tb;
    int32_t span;
};

struct CurveOut {
    std::vector<Piece> pieces;
    std::vector<double> span_t;
    std::vector<double> coef;   // (p+1)*3 per span
    std::vector<int32_t> span_first;  // first piece (local) of each span
    int rc = 0;
    std::string err;
    double diag = 0.0, tol_abs = 0.0;
};

bool reduce_span(int p, const DegreeTables& T, const double* Q, double ta, double tb, double tol, int32_t span,
                 std::vector<Piece>& out)
{
    struct Item { double Q[3 * (kMaxP + 1)]; double ta, tb; };
    std::vector<Item> stack;
    stack.reserve(64);
    Item first;
    memcpy(first.Q, Q, sizeof(double) * 3 * (size_t)(p + 1));
    first.ta = ta; first.tb = tb;
    stack.push_back(first);
    int splits = 0;
    while (!stack.empty()) {
        Item it = stack.back();
        stack.pop_back();
        Piece pc;
        g1_reduce(p, T, it.Q, pc.R);
        int imax = 64;
        double e = deviation_bound(p, T, it.Q, pc.R, &imax);
        if (e <= tol) {
            pc.ta = it.ta; pc.tb = it.tb; pc.span = span;
            out.push_back(pc);
            continue;
        }
        if (++splits >= MREP_MAX_PIECES_PER_SPAN) return false;
        int iz = std::min(std::max(imax, 16), 112);
        double z = (double)iz / 128.0;
        Item l, r;
        split_piece(p, it.Q, z, l.Q, r.Q);
        double tm = it.ta + z * (it.tb - it.ta);
        l.ta = it.ta; l.tb = tm;
        r.ta = tm; r.tb = it.tb;
        stack.push_back(r);  // left is processed first: pieces come out in order
        stack.push_back(l);
    }
    return true;
}

// Bezier points of span [a, b] = [U_q, U_q+1] of degree p as blossom values
// b_j = P(a^{p-j}, b^j): de Boor's triangle whose level k takes the argument a
// for k <= p - j and b after (every weight in [0, 1]: a chain of convex
// combinations, stable at any degree).  Q[3j + c].
void span_blossom(int p, const double* P, const double* U, int q, double* Q)
{
    const double a = U[q], b = U[q + 1];
    double d[(kMaxP + 1) * 3];
    for (int j = 0; j <= p; ++j) {
        for (int r = 0; r <= p; ++r)
            for (int c = 0; c < 3; ++c) d[3 * r + c] = P[3 * (q - p + r) + c];
        for (int k = 1; k <= p; ++k) {
            const double x = (k <= p - j) ? a : b;
            for (int r = p; r >= k; --r) {
                const int i = q - p + r;
                const double al = (x - U[i]) / (U[i + p - k + 1] - U[i]);
                for (int c = 0; c < 3; ++c) d[3 * r + c] = (1.0 - al) * d[3 * (r - 1) + c] + al * d[3 * r + c];
            }
        }
        for (int c = 0; c < 3; ++c) Q[3 * j + c] = d[3 * p + c];
    }
}

// Homogeneous Bezier points (w x, w y, w z, w) of span q of a rational curve:
// the blossom of the homogeneous control points, as span_blossom.
void span_blossom4(int p, const double* H, const double* U, int q, double* Q)
{
    const double a = U[q], b = U[q + 1];
    double d[(kMaxP + 1) * 4];
    for (int j = 0; j <= p; ++j) {
        for (int r = 0; r <= p; ++r)
            for (int c = 0; c < 4; ++c) d[4 * r + c] = H[4 * (q - p + r) + c];
        for (int k = 1; k <= p; ++k) {
            const double x = (k <= p - j) ? a : b;
            for (int r = p; r >= k; --r) {
                const int i = q - p + r;
                const double al = (x - U[i]) / (U[i + p - k + 1] - U[i]);
                for (int c = 0; c < 4; ++c) d[4 * r + c] = (1.0 - al) * d[4 * (r - 1) + c] + al * d[4 * r + c];
            }
        }
        for (int c = 0; c < 4; ++c) Q[4 * j + c] = d[4 * p + c];
    }
}

// de Casteljau split at z of a degree-p homogeneous Bezier piece (exact
// subdivision of the rational piece)
void split_piece4(int p, const double* G, double z, double* L, double* R)
{
    double w[(kMaxP + 1) * 4];
    memcpy(w, G, sizeof(double) * 4 * (size_t)(p + 1));
    for (int c = 0; c < 4; ++c) { L[c] = w[c]; R[4 * p + c] = w[4 * p + c]; }
    for (int r = 1; r <= p; ++r) {
        for (int j = 0; j <= p - r; ++j)
            for (int c = 0; c < 4; ++c) w[4 * j + c] = (1.0 - z) * w[4 * j + c] + z * w[4 * (j + 1) + c];
        for (int c = 0; c < 4; ++c) { L[4 * r + c] = w[c]; R[4 * (p - r) + c] = w[4 * (p - r) + c]; }
    }
}

// Cubic Hermite piece of a rational piece G (degree p, homogeneous): the end
// points and end derivatives of the rational curve, C'(0) = p (w1/w0)(P1 - P0)
// and C'(1) = p (w_{p-1}/w_p)(P_p - P_{p-1}) -- the G1 conditions of Sec. 5.2.2
// with delta0 = delta1 = 1 (the L2 optimum has no closed form for a rational
// piece).  Returns its deviation bound: the largest deviation on the error
// samples plus (1/256) times a bound on |(C - R)'|.  With N = X - W R (the
// numerator of C - R, degree p + 3, Bernstein coefficients by the product
// rule) and W >= w_min:  |(N/W)'| <= ((p+3) max|dN| + max|N| p max|dw| / w_min) / w_min.
double rational_cubic(int p, const DegreeTables& T, const double* G, double* R, int* imax)
{
    double P0[3], P1[3], Pq[3], Pq1[3];
    for (int c = 0; c < 3; ++c) {
        P0[c] = G[c] / G[3];
        P1[c] = G[4 + c] / G[7];
        Pq[c] = G[4 * p + c] / G[4 * p + 3];
        Pq1[c] = G[4 * (p - 1) + c] / G[4 * (p - 1) + 3];
    }
    const double s0 = (double)p * G[7] / G[3] / 3.0, s1 = (double)p * G[4 * (p - 1) + 3] / G[4 * p + 3] / 3.0;
    for (int c = 0; c < 3; ++c) {
        R[c] = P0[c];
        R[3 + c] = P0[c] + s0 * (P1[c] - P0[c]);
        R[6 + c] = Pq[c] - s1 * (Pq[c] - Pq1[c]);
        R[9 + c] = Pq[c];
    }
    double best = -1.0, ev[kErrSamples];
    for (int i = 0; i < kErrSamples; ++i) {
        double x[4] = {0, 0, 0, 0}, y[3] = {0, 0, 0};
        for (int k = 0; k <= p; ++k)
            for (int c = 0; c < 4; ++c) x[c] += T.Bq[i * (p + 1) + k] * G[4 * k + c];
        for (int k = 0; k < 4; ++k)
            for (int c = 0; c < 3; ++c) y[c] += T.B3[i * 4 + k] * R[3 * k + c];
        double e2 = 0.0;
        for (int c = 0; c < 3; ++c) e2 += (x[c] / x[3] - y[c]) * (x[c] / x[3] - y[c]);
        ev[i] = sqrt(e2);
        best = std::max(best, ev[i]);
    }
    int bi = 64;
    for (int i = 0; i < kErrSamples; ++i)
        if (ev[i] >= best * (1.0 - 1e-6)) { bi = i; break; }
    *imax = bi;
    double N[(kMaxP + 4) * 3];
    for (int k = 0; k <= p + 3; ++k)
        for (int c = 0; c < 3; ++c) N[3 * k + c] = 0.0;
    for (int i = 0; i <= p; ++i)
        for (int j = 0; j <= 3; ++j) {
            const double f = binom(p, i) * binom(3, j) / binom(p + 3, i + j);
            for (int c = 0; c < 3; ++c) N[3 * (i + j) + c] += f * (G[4 * i + c] - G[4 * i + 3] * R[3 * j + c]);
        }
    double nmax = 0.0, dn = 0.0, wmin = INFINITY, dw = 0.0;
    for (int k = 0; k <= p + 3; ++k) {
        nmax = std::max(nmax, sqrt(N[3 * k] * N[3 * k] + N[3 * k + 1] * N[3 * k + 1] + N[3 * k + 2] * N[3 * k + 2]));
        if (k < p + 3) {
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) d2 += (N[3 * (k + 1) + c] - N[3 * k + c]) * (N[3 * (k + 1) + c] - N[3 * k + c]);
            dn = std::max(dn, sqrt(d2));
        }
    }
    for (int k = 0; k <= p; ++k) {
        wmin = std::min(wmin, G[4 * k + 3]);
        if (k < p) dw = std::max(dw, fabs(G[4 * (k + 1) + 3] - G[4 * k + 3]));
    }
    const double lip = ((double)(p + 3) * dn + nmax * (double)p * dw / wmin) / wmin;
    return best + lip / 256.0;
}

// Polynomial cubic pieces within tol of the rational span G on [ta, tb]:
// split at the sample of largest deviation (clamped to [1/8, 7/8]) of the
// rational piece itself until every piece's bound holds, as reduce_span.
bool approx_rational_span(int p, const DegreeTables& T, const double* G, double ta, double tb, double tol,
                          int32_t span, std::vector<Piece>& out, double& worst)
{
    struct Item { double G[4 * (kMaxP + 1)]; double ta, tb; };
    std::vector<Item> stack;
    stack.reserve(64);
    Item first;
    memcpy(first.G, G, sizeof(double) * 4 * (size_t)(p + 1));
    first.ta = ta; first.tb = tb;
    stack.push_back(first);
    int splits = 0;
    while (!stack.empty()) {
        Item it = stack.back();
        stack.pop_back();
        Piece pc;
        int imax = 64;
        const double e = rational_cubic(p, T, it.G, pc.R, &imax);
        if (e <= tol) {
            pc.ta = it.ta; pc.tb = it.tb; pc.span = span;
            out.push_back(pc);
            worst = std::max(worst, e);
            continue;
        }
        if (++splits >= MREP_MAX_PIECES_PER_SPAN) return false;
        const int iz = std::min(std::max(imax, 16), 112);
        const double z = (double)iz / 128.0;
        Item l, r;
        split_piece4(p, it.G, z, l.G, r.G);
        const double tm = it.ta + z * (it.tb - it.ta);
        l.ta = it.ta; l.tb = tm;
        r.ta = tm; r.tb = it.tb;
        stack.push_back(r);
        stack.push_back(l);
    }
    return true;
}

bool validate_curve(int p, int n, const double* P, const double* U, std::string& err, int& code)
{
    if (p < 1 || p > kMaxP) { code = MREP_E_BAD_DEGREE; err = "degree out of range"; return false; }
    if (n < p + 1) { code = MREP_E_BAD_DEGREE; err = "fewer than p+1 control points"; return false; }
    int m = n + p + 1;
    for (int i = 0; i < 3 * n; ++i)
        if (!std::isfinite(P[i])) { code = MREP_E_INVALID_ARG; err = "non-finite control point"; return false; }
    for (int i = 0; i < m; ++i)
        if (!std::isfinite(U[i])) { code = MREP_E_BAD_KNOTS; err = "non-finite knot"; return false; }
    for (int i = 0; i + 1 < m; ++i)
        if (U[i + 1] < U[i]) { code = MREP_E_BAD_KNOTS; err = "knots not non-decreasing"; return false; }
    for (int i = 0; i < p; ++i)
        if (U[i] != U[p] || U[m - 1 - i] != U[n]) { code = MREP_E_BAD_KNOTS; err = "knot vector not clamped"; return false; }
    if (!(U[p] < U[n])) { code = MREP_E_BAD_KNOTS; err = "empty parameter domain"; return false; }
    // interior multiplicity (indices p+1 .. n-1) at most p
    int run = 1;
    for (int i = p + 2; i <= n - 1; ++i) {
        run = (U[i] == U[i - 1]) ? run + 1 : 1;
        if (run > p) { code = MREP_E_BAD_KNOTS; err = "interior knot multiplicity > degree"; return false; }
    }
    if (n - 1 >= p + 1 && U[p + 1] == U[p]) {
        // an interior knot equal to the clamped start would make multiplicity > p+1 at the end
        code = MREP_E_BAD_KNOTS; err = "knot vector not clamped (multiplicity > p+1 at an end)"; return false;
    }
    if (n - 1 >= p + 1 && U[n - 1] == U[n]) {
        code = MREP_E_BAD_KNOTS; err = "knot vector not clamped (multiplicity > p+1 at an end)"; return false;
    }
    return true;
}

// A rational curve: each non-degenerate span's homogeneous Bezier points are
// kept as its exact form, and polynomial cubic pieces within tol_rel * diag of
// the rational curve feed the screen and the refine (the pieces' deviation
// bound is the curve's tol_eff).
void decompose_curve_rational(int p, int n, const double* P, const double* w, const double* U, double tol_rel,
                              CurveOut& out)
{
    const DegreeTables& T = g_tab[p];
    double lo[3] = {P[0], P[1], P[2]}, hi[3] = {P[0], P[1], P[2]};
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) { lo[c] = std::min(lo[c], P[3 * i + c]); hi[c] = std::max(hi[c], P[3 * i + c]); }
    out.diag = sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) + (hi[2] - lo[2]) * (hi[2] - lo[2]));
    const double tol = tol_rel * out.diag;
    std::vector<double> H((size_t)4 * n);
    for (int i = 0; i < n; ++i) {
        for (int c = 0; c < 3; ++c) H[(size_t)4 * i + c] = w[i] * P[3 * i + c];
        H[(size_t)4 * i + 3] = w[i];
    }
    double G[(kMaxP + 1) * 4];
    double worst = 0.0;
    int32_t span_local = 0;
    for (int q = p; q <= n - 1; ++q) {
        if (!(U[q] < U[q + 1])) continue;
        span_blossom4(p, H.data(), U, q, G);
        out.span_t.push_back(U[q]);
        out.span_t.push_back(U[q + 1]);
        out.coef.insert(out.coef.end(), G, G + 4 * (p + 1));
        out.span_first.push_back((int32_t)out.pieces.size());
        if (!approx_rational_span(p, T, G, U[q], U[q + 1], tol, span_local, out.pieces, worst)) {
            out.rc = MREP_E_TOL;
            out.err = "a span needed more than MREP_MAX_PIECES_PER_SPAN pieces";
            return;
        }
        span_local++;
    }
    out.tol_abs = worst;
}

void decompose_curve(int p, int n, const double* P, const double* w, const double* U, double tol_rel, CurveOut& out)
{
    std::string err;
    int code = 0;
    if (!validate_curve(p, n, P, U, err, code)) { out.rc = code; out.err = err; return; }
    if (w) {
        for (int i = 0; i < n; ++i)
            if (!(w[i] > 0.0) || !std::isfinite(w[i])) {
                out.rc = MREP_E_INVALID_ARG;
                out.err = "weights must be positive and finite";
                return;
            }
        decompose_curve_rational(p, n, P, w, U, tol_rel, out);
        return;
    }
    const DegreeTables& T = g_tab[p];
    double lo[3] = {P[0], P[1], P[2]}, hi[3] = {P[0], P[1], P[2]};
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) { lo[c] = std::min(lo[c], P[3 * i + c]); hi[c] = std::max(hi[c], P[3 * i + c]); }
    out.diag = sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) + (hi[2] - lo[2]) * (hi[2] - lo[2]));
    out.tol_abs = tol_rel * out.diag;
    double D[(kMaxP + 1) * 3], Q[(kMaxP + 1) * 3];
    int32_t span_local = 0;
    for (int q = p; q <= n - 1; ++q) {
        if (!(U[q] < U[q + 1])) continue;
        if (p <= MREP_POWER_MAX_DEGREE) {
            // D = diag(h^j) A P_{q-p..q} (power coefficients in the local u), Q = B_p^{-1} D
            dm::span_power_bezier<kMaxP>(p, T, U, q, P, D, Q);
        } else {
            // the exact span is kept as its Bezier points (the polish evaluates them by de Casteljau)
            span_blossom(p, P, U, q, Q);
            memcpy(D, Q, sizeof(double) * 3 * (size_t)(p + 1));
        }
        out.span_t.push_back(U[q]);
        out.span_t.push_back(U[q + 1]);
        out.coef.insert(out.coef.end(), D, D + 3 * (p + 1));
        out.span_first.push_back((int32_t)out.pieces.size());
        if (p <= 3) {
            double Acur[12];
            dm::elevate_to_cubic(p, Q, Acur);
            Piece pc;
            memcpy(pc.R, Acur, sizeof(pc.R));
            pc.ta = U[q]; pc.tb = U[q + 1]; pc.span = span_local;
            out.pieces.push_back(pc);
        } else {
            if (!reduce_span(p, T, Q, U[q], U[q + 1], out.tol_abs, span_local, out.pieces)) {
                out.rc = MREP_E_TOL;
                out.err = "a span needed more than MREP_MAX_PIECES_PER_SPAN pieces";
                return;
            }
        }
        span_local++;
    }
    if (p <= 3) out.tol_abs = 0.0;
}





int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

}  // namespace

uint16_t f32_to_bf16_rne(float x) { return dm::f32_to_bf16_rne(x); }

void bernstein_matrix(int p, double* B)
{
    for (int j = 0; j <= p; ++j)
        for (int i = 0; i <= p; ++i) B[j * (p + 1) + i] = 0.0;
    for (int i = 0; i <= p; ++i)
        for (int k = 0; k <= p - i; ++k)
            B[(i + k) * (p + 1) + i] = binom(p, i) * binom(p - i, k) * ((k & 1) ? -1.0 : 1.0);
}

void bernstein_inverse(int p, double* Bi)
{
    for (int i = 0; i <= p; ++i)
        for (int j = 0; j <= p; ++j) Bi[i * (p + 1) + j] = (j <= i) ? binom(i, j) / binom(p, j) : 0.0;
}

void subdivision_matrix(int p, double z, double* S)
{
    int n = p + 1;
    for (int i = 0; i < 2 * n * n; ++i) S[i] = 0.0;
    for (int i = 0; i <= p; ++i)
        for (int j = 0; j <= i; ++j) S[i * n + j] = binom(i, j) * ipow(z, j) * ipow(1.0 - z, i - j);
    for (int i = 0; i <= p; ++i)
        for (int j = i; j <= p; ++j) S[(n + i) * n + j] = binom(p - i, j - i) * ipow(z, j - i) * ipow(1.0 - z, p - j);
}

void gram_matrix(int m, int n, double* G)
{
    for (int i = 0; i <= m; ++i)
        for (int j = 0; j <= n; ++j)
            G[i * (n + 1) + j] = binom(m, i) * binom(n, j) / ((double)(m + n + 1) * binom(m + n, i + j));
}

int build_plan(int32_t n_curves, const int32_t* degree, const int64_t* cp_off, const double* cp_xyz,
               const double* weights, const int64_t* knot_off, const double* knots, double tol_rel, int n_threads,
               Plan& plan, std::string& err)
{
    init_tables();
    std::vector<CurveOut> outs((size_t)n_curves);
    for (int32_t c = 0; c < n_curves; ++c) {
        int64_t n = cp_off[c + 1] - cp_off[c];
        int64_t nk = knot_off[c + 1] - knot_off[c];
        if (n < 0 || nk < 0) { err = "negative CSR extent"; return MREP_E_INVALID_ARG; }
        if (degree[c] < 1 || degree[c] > kMaxP) { err = "curve " + std::to_string(c) + ": degree out of range"; return MREP_E_BAD_DEGREE; }
        if (nk != n + degree[c] + 1) { err = "curve " + std::to_string(c) + ": knot count != points + p + 1"; return MREP_E_BAD_KNOTS; }
        if (n > (int64_t)1 << 24) { err = "curve too long"; return MREP_E_INVALID_ARG; }
    }
    int nt = n_threads > 0 ? n_threads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = std::min<int>(nt, std::max<int32_t>(1, n_curves));
    std::atomic<int32_t> next{0};
    auto worker = [&]() {
        for (;;) {
            int32_t c = next.fetch_add(1);
            if (c >= n_curves) break;
            decompose_curve(degree[c], (int)(cp_off[c + 1] - cp_off[c]), cp_xyz + 3 * cp_off[c],
                            weights ? weights + cp_off[c] : nullptr, knots + knot_off[c], tol_rel, outs[(size_t)c]);
        }
    };
    std::vector<std::thread> th;
    for (int i = 1; i < nt; ++i) th.emplace_back(worker);
    worker();
    for (auto& t : th) t.join();
    for (int32_t c = 0; c < n_curves; ++c)
        if (outs[(size_t)c].rc) {
            err = "curve " + std::to_string(c) + ": " + outs[(size_t)c].err;
            return outs[(size_t)c].rc;
        }
    // concatenate
    plan.n_curves = n_curves;
    plan.tol_rel = tol_rel;
    plan.max_degree = 0;
    plan.curves.resize((size_t)n_curves);
    int64_t nseg = 0, nspan = 0, ncoef = 0, nclu = 0;
    for (int32_t c = 0; c < n_curves; ++c) {
        const CurveOut& o = outs[(size_t)c];
        DCurve& d = plan.curves[(size_t)c];
        d.clu_off = nclu;
        d.n_clu = (int32_t)((o.pieces.size() + kCluPieces - 1) / kCluPieces);
        d.clu_use = 0;
        nclu += d.n_clu;
        d.seg_off = nseg;
        d.span_off = nspan;
        d.coef_off = ncoef;
        d.n_seg = (int32_t)o.pieces.size();
        d.n_span = (int32_t)(o.span_t.size() / 2);
        d.degree = degree[c];
        d.es_max = 0.f;
        d.rational = weights ? 1 : 0;
        d.pad_ = 0;
        d.tol_eff = (degree[c] >= 4 || weights) ? std::max(o.tol_abs, 1e-13 * o.diag) : 1e-13 * o.diag;
        d.tol_user = tol_rel * o.diag;
        d.diag = o.diag;
        {
            const double* P = cp_xyz + 3 * cp_off[c];
            int64_t n = cp_off[c + 1] - cp_off[c];
            for (int k = 0; k < 3; ++k) {
                double lo = P[k], hi = P[k];
                for (int64_t i = 0; i < n; ++i) { lo = std::min(lo, P[3 * i + k]); hi = std::max(hi, P[3 * i + k]); }
                d.origin[k] = (double)(float)(0.5 * (lo + hi));
            }
        }
        nseg += d.n_seg;
        nspan += d.n_span;
        ncoef += (int64_t)o.coef.size();
        plan.max_degree = std::max(plan.max_degree, degree[c]);
    }
    if (nseg >= ((int64_t)1 << 31)) { err = "more than 2^31 pieces"; return MREP_E_INVALID_ARG; }
    plan.seg_cp.resize((size_t)nseg * 12);
    plan.seg_t.resize((size_t)nseg * 2);
    plan.seg_span.resize((size_t)nseg);
    plan.span_t.resize((size_t)nspan * 2);
    plan.span0.resize((size_t)nspan + 1);
    plan.coef.resize((size_t)ncoef);
    plan.col.resize((size_t)nseg * kScreenK);
    plan.aux.resize((size_t)nseg * 8);
    plan.lcp.resize((size_t)nseg * 12);
    plan.sph.resize((size_t)nseg * 4);
    plan.csph.resize((size_t)nclu * 4);
    std::atomic<int32_t> next2{0};
    auto worker2 = [&]() {
        for (;;) {
            int32_t c = next2.fetch_add(1);
            if (c >= n_curves) break;
            const CurveOut& o = outs[(size_t)c];
            DCurve& d = plan.curves[(size_t)c];
            double tol_eff = d.tol_eff;
            float es_max = 0.f;
            for (int32_t s = 0; s < d.n_seg; ++s) {
                const Piece& pc = o.pieces[(size_t)s];
                int64_t g = d.seg_off + s;
                memcpy(&plan.seg_cp[(size_t)g * 12], pc.R, sizeof(double) * 12);
                plan.seg_t[(size_t)g * 2] = pc.ta;
                plan.seg_t[(size_t)g * 2 + 1] = pc.tb;
                plan.seg_span[(size_t)g] = (int32_t)(d.span_off + pc.span);
                piece_tables(pc.R, d.origin, tol_eff, &plan.col[(size_t)g * kScreenK], &plan.aux[(size_t)g * 8],
                             &plan.lcp[(size_t)g * 12]);
                es_max = std::max(es_max, plan.aux[(size_t)g * 8 + AUX_ES]);
                piece_sphere(&plan.aux[(size_t)g * 8], &plan.lcp[(size_t)g * 12], tol_eff, &plan.sph[(size_t)g * 4]);
            }
            d.es_max = es_max;
            double rsum = 0.0;
            for (int32_t k = 0; k < d.n_clu; ++k) {
                const int64_t a = d.seg_off + (int64_t)k * kCluPieces;
                const int64_t m = std::min<int64_t>(kCluPieces, d.n_seg - (int64_t)k * kCluPieces);
                bounding_sphere(&plan.sph[(size_t)a * 4], m, &plan.csph[(size_t)(d.clu_off + k) * 4]);
                rsum += plan.csph[(size_t)(d.clu_off + k) * 4 + 3];
            }
            // clusters pay off when they are small against the curve (a wandering
            // curve), not when consecutive pieces jump across its whole box
            d.clu_use = d.n_clu >= 4 && d.n_clu < 65536 && rsum / d.n_clu <= 0.1 * d.diag ? 1 : 0;
            for (int32_t j = 0; j < d.n_span; ++j) {
                plan.span_t[(size_t)(d.span_off + j) * 2] = o.span_t[(size_t)j * 2];
                plan.span_t[(size_t)(d.span_off + j) * 2 + 1] = o.span_t[(size_t)j * 2 + 1];
                plan.span0[(size_t)(d.span_off + j)] = (int32_t)(d.seg_off + o.span_first[(size_t)j]);
            }
            memcpy(&plan.coef[(size_t)d.coef_off], o.coef.data(), sizeof(double) * o.coef.size());
        }
    };
    th.clear();
    next2 = 0;
    for (int i = 1; i < nt; ++i) th.emplace_back(worker2);
    worker2();
    for (auto& t : th) t.join();
    plan.span0[(size_t)nspan] = (int32_t)nseg;

    curve_layout(plan.layout, n_curves, nseg, nspan, ncoef, nclu);
    plan.layout.general = (weights != nullptr || plan.max_degree > MREP_POWER_MAX_DEGREE) ? 1 : 0;
    return MREP_OK;
}

void curve_layout(GeomLayout& L, int64_t n_curves, int64_t nseg, int64_t nspan, int64_t ncoef, int64_t nclu)
{
    L.n_curves = n_curves;
    L.n_seg = nseg;
    L.n_span = nspan;
    L.n_coef = ncoef;
    int64_t off = 0;
    L.off_curve = off; off = align256(off + (int64_t)sizeof(DCurve) * n_curves);
    L.off_col = off; off = align256(off + 2 * kScreenK * nseg);
    L.off_aux = off; off = align256(off + 4 * 8 * nseg);
    L.off_lcp = off; off = align256(off + 4 * 12 * nseg);
    L.off_gcp = off; off = align256(off + 8 * 12 * nseg);
    L.off_segt = off; off = align256(off + 8 * 2 * nseg);
    L.off_segspan = off; off = align256(off + 4 * nseg);
    L.off_spant = off; off = align256(off + 8 * 2 * nspan);
    L.off_span0 = off; off = align256(off + 4 * (nspan + 1));
    L.off_coef = off; off = align256(off + 8 * ncoef);
    L.n_clu = nclu;
    L.off_sph = off; off = align256(off + 16 * nseg);
    L.off_csph = off; off = align256(off + 16 * nclu);
    L.total = off;
    L.general = 0;
}

const dm::DegreeTables* dm::degree_tables_host()
{
    init_tables();
    return g_tab;
}

}  // namespace mrep

// ---------------------------------------------------------------------------
// Surfaces.  A tensor-product span patch (span q_u in u, q_v in v) is the
// matrix form of Sec. 5.2.1 applied in both directions: power coefficients
// C = D_u P D_v^T (D = diag(h^j) A of the span, eq. Mqpt) and Bezier net
// N = B_p^{-1} D_u P D_v^T B_q^{-T}.  Degrees <= 3 are elevated to cubic
// exactly; a degree >= 4 direction is reduced with the curve's G1 L2 cubic
// (Sec. 5.2.2), rows in u first, then columns in v, and a patch whose error
// bound on a 32 x 32 grid exceeds the tolerance is split (on the exact net) in
// the direction whose hodograph bound of the error is larger, at the worst
// grid line clamped to [4/31, 27/31].
// ---------------------------------------------------------------------------
namespace mrep {
namespace {

constexpr int kSurfGrid = 32;

struct SPiece {
    double R[48];
    double ua, ub, va, vb;
    int32_t span;
};

struct SurfOut {
    std::vector<SPiece> pieces;
    std::vector<double> brk, coef;
    std::vector<int32_t> span_first;
    int n_su = 0, n_sv = 0;
    int rc = 0;
    std::string err;
    double diag = 0.0, tol_abs = 0.0;
};

// degree-d curve (d+1 points) -> cubic (4 points)
void curve_to_cubic(int d, const double* Q, double* R4)
{
    if (d == 3) { memcpy(R4, Q, sizeof(double) * 12); return; }
    if (d > 3) { g1_reduce(d, g_tab[d], Q, R4); return; }
    double A[12], B[12], E[5 * 4];
    memcpy(A, Q, sizeof(double) * 3 * (size_t)(d + 1));
    for (int e = d; e < 3; ++e) {
        elevation_matrix(e, E);
        for (int i = 0; i <= e + 1; ++i)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int k = 0; k <= e; ++k) s += E[i * (e + 1) + k] * A[3 * k + c];
                B[3 * i + c] = s;
            }
        memcpy(A, B, sizeof(double) * 3 * (size_t)(e + 2));
    }
    memcpy(R4, A, sizeof(double) * 12);
}

// (p+1) x (q+1) net (u-major) -> bicubic 4 x 4: rows in u, then columns in v
void net_to_bicubic(int p, int q, const double* N, double* R)
{
    double T[4 * (kMaxP + 1) * 3], col[(kMaxP + 1) * 3], r4[12];
    for (int j = 0; j <= q; ++j) {
        for (int i = 0; i <= p; ++i)
            for (int c = 0; c < 3; ++c) col[3 * i + c] = N[3 * (i * (q + 1) + j) + c];
        curve_to_cubic(p, col, r4);
        for (int k = 0; k < 4; ++k)
            for (int c = 0; c < 3; ++c) T[3 * (k * (q + 1) + j) + c] = r4[3 * k + c];
    }
    for (int k = 0; k < 4; ++k) {
        curve_to_cubic(q, &T[3 * (k * (q + 1))], r4);
        for (int l = 0; l < 4; ++l)
            for (int c = 0; c < 3; ++c) R[3 * (k * 4 + l) + c] = r4[3 * l + c];
    }
}

void bern_row(int d, double s, double* b)
{
    for (int i = 0; i <= d; ++i) b[i] = binom(d, i) * ipow(s, i) * ipow(1.0 - s, d - i);
}

// net of degree (a, b) written at degree (A, B) >= (a, b)
void elevate_net(int a, int b, const double* N, int A, int B, double* out)
{
    double cur[(kMaxP + 1) * (kMaxP + 1) * 3], nxt[(kMaxP + 1) * (kMaxP + 1) * 3], E[(kMaxP + 2) * (kMaxP + 1)];
    memcpy(cur, N, sizeof(double) * 3 * (size_t)(a + 1) * (b + 1));
    int ca = a, cb = b;
    while (ca < A) {
        elevation_matrix(ca, E);
        for (int i = 0; i <= ca + 1; ++i)
            for (int j = 0; j <= cb; ++j)
                for (int c = 0; c < 3; ++c) {
                    double s = 0.0;
                    for (int k = 0; k <= ca; ++k) s += E[i * (ca + 1) + k] * cur[3 * (k * (cb + 1) + j) + c];
                    nxt[3 * (i * (cb + 1) + j) + c] = s;
                }
        ++ca;
        memcpy(cur, nxt, sizeof(double) * 3 * (size_t)(ca + 1) * (cb + 1));
    }
    while (cb < B) {
        elevation_matrix(cb, E);
        for (int i = 0; i <= ca; ++i)
            for (int j = 0; j <= cb + 1; ++j)
                for (int c = 0; c < 3; ++c) {
                    double s = 0.0;
                    for (int k = 0; k <= cb; ++k) s += E[j * (cb + 1) + k] * cur[3 * (i * (cb + 1) + k) + c];
                    nxt[3 * (i * (cb + 2) + j) + c] = s;
                }
        ++cb;
        memcpy(cur, nxt, sizeof(double) * 3 * (size_t)(ca + 1) * (cb + 1));
    }
    memcpy(out, cur, sizeof(double) * 3 * (size_t)(A + 1) * (B + 1));
}

// Error bound of the bicubic R against the exact net N: the largest deviation
// on the 32 x 32 grid plus half a grid step times the hodograph bounds Ls, Lt
// of their difference.  (ki, kj): the first grid point (row-major) within
// 1e-6 relative of the largest deviation.
double bicubic_error(int p, int q, const double* N, const double* R, int* ki, int* kj, double* Ls, double* Lt)
{
    double bp[kSurfGrid][kMaxP + 1], bq[kSurfGrid][kMaxP + 1], b3[kSurfGrid][4];
    for (int k = 0; k < kSurfGrid; ++k) {
        const double s = (double)k / (kSurfGrid - 1);
        bern_row(p, s, bp[k]);
        bern_row(q, s, bq[k]);
        bern_row(3, s, b3[k]);
    }
    static thread_local std::vector<double> ev;
    ev.assign((size_t)kSurfGrid * kSurfGrid, 0.0);
    double best = 0.0;
    for (int k = 0; k < kSurfGrid; ++k) {
        // rows of N and R collapsed in u at s_k
        double nu[(kMaxP + 1) * 3], ru[4 * 3];
        for (int j = 0; j <= q; ++j)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int i = 0; i <= p; ++i) s += bp[k][i] * N[3 * (i * (q + 1) + j) + c];
                nu[3 * j + c] = s;
            }
        for (int l = 0; l < 4; ++l)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int i = 0; i < 4; ++i) s += b3[k][i] * R[3 * (i * 4 + l) + c];
                ru[3 * l + c] = s;
            }
        for (int l = 0; l < kSurfGrid; ++l) {
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                double x = 0.0, y = 0.0;
                for (int j = 0; j <= q; ++j) x += bq[l][j] * nu[3 * j + c];
                for (int j = 0; j < 4; ++j) y += b3[l][j] * ru[3 * j + c];
                d2 += (x - y) * (x - y);
            }
            const double e = sqrt(d2);
            ev[(size_t)k * kSurfGrid + l] = e;
            best = std::max(best, e);
        }
    }
    *ki = 0; *kj = 0;
    for (int k = 0, found = 0; k < kSurfGrid && !found; ++k)
        for (int l = 0; l < kSurfGrid; ++l)
            if (ev[(size_t)k * kSurfGrid + l] >= best * (1.0 - 1e-6)) { *ki = k; *kj = l; found = 1; break; }
    const int A = std::max(p, 3), B = std::max(q, 3);
    double Ne[(kMaxP + 1) * (kMaxP + 1) * 3], Re[(kMaxP + 1) * (kMaxP + 1) * 3];
    elevate_net(p, q, N, A, B, Ne);
    elevate_net(3, 3, R, A, B, Re);
    double ls = 0.0, lt = 0.0;
    for (int i = 0; i <= A; ++i)
        for (int j = 0; j <= B; ++j) {
            double du2 = 0.0, dv2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double d00 = Ne[3 * (i * (B + 1) + j) + c] - Re[3 * (i * (B + 1) + j) + c];
                if (i < A) {
                    const double d10 = Ne[3 * ((i + 1) * (B + 1) + j) + c] - Re[3 * ((i + 1) * (B + 1) + j) + c];
                    du2 += (d10 - d00) * (d10 - d00);
                }
                if (j < B) {
                    const double d01 = Ne[3 * (i * (B + 1) + j + 1) + c] - Re[3 * (i * (B + 1) + j + 1) + c];
                    dv2 += (d01 - d00) * (d01 - d00);
                }
            }
            ls = std::max(ls, (double)A * sqrt(du2));
            lt = std::max(lt, (double)B * sqrt(dv2));
        }
    *Ls = ls;
    *Lt = lt;
    return best + (ls + lt) / (2.0 * (kSurfGrid - 1));
}

// split an exact net at z in u (dir 0: every column curve) or v (dir 1: every row curve)
void split_net(int p, int q, const double* N, int dir, double z, double* A, double* B)
{
    double c[(kMaxP + 1) * 3], l[(kMaxP + 1) * 3], r[(kMaxP + 1) * 3];
    if (dir == 0) {
        for (int j = 0; j <= q; ++j) {
            for (int i = 0; i <= p; ++i)
                for (int k = 0; k < 3; ++k) c[3 * i + k] = N[3 * (i * (q + 1) + j) + k];
            split_piece(p, c, z, l, r);
            for (int i = 0; i <= p; ++i)
                for (int k = 0; k < 3; ++k) {
                    A[3 * (i * (q + 1) + j) + k] = l[3 * i + k];
                    B[3 * (i * (q + 1) + j) + k] = r[3 * i + k];
                }
        }
    } else {
        for (int i = 0; i <= p; ++i) {
            split_piece(q, &N[3 * (i * (q + 1))], z, l, r);
            memcpy(&A[3 * (i * (q + 1))], l, sizeof(double) * 3 * (size_t)(q + 1));
            memcpy(&B[3 * (i * (q + 1))], r, sizeof(double) * 3 * (size_t)(q + 1));
        }
    }
}

bool reduce_patch(int p, int q, const double* N0, double ua, double ub, double va, double vb, double tol, int32_t span,
                  std::vector<SPiece>& out)
{
    struct Item {
        double N[(kMaxP + 1) * (kMaxP + 1) * 3];
        double ua, ub, va, vb;
    };
    std::vector<Item> stack;
    Item first;
    memcpy(first.N, N0, sizeof(double) * 3 * (size_t)(p + 1) * (q + 1));
    first.ua = ua; first.ub = ub; first.va = va; first.vb = vb;
    stack.push_back(first);
    int splits = 0;
    while (!stack.empty()) {
        Item it = stack.back();
        stack.pop_back();
        SPiece pc;
        net_to_bicubic(p, q, it.N, pc.R);
        pc.ua = it.ua; pc.ub = it.ub; pc.va = it.va; pc.vb = it.vb; pc.span = span;
        if (p <= 3 && q <= 3) { out.push_back(pc); continue; }
        int ki = 0, kj = 0;
        double Ls = 0.0, Lt = 0.0;
        const double e = bicubic_error(p, q, it.N, pc.R, &ki, &kj, &Ls, &Lt);
        if (e <= tol) { out.push_back(pc); continue; }
        if (++splits >= MREP_MAX_PIECES_PER_SPAN) return false;
        const int dir = (p >= 4 && (q <= 3 || Ls >= Lt)) ? 0 : 1;
        const int k = std::min(std::max(dir == 0 ? ki : kj, 4), kSurfGrid - 1 - 4);
        const double z = (double)k / (kSurfGrid - 1);
        Item a, b;
        a.ua = b.ua = it.ua; a.ub = b.ub = it.ub; a.va = b.va = it.va; a.vb = b.vb = it.vb;
        split_net(p, q, it.N, dir, z, a.N, b.N);
        if (dir == 0) {
            const double um = it.ua + z * (it.ub - it.ua);
            a.ub = um; b.ua = um;
        } else {
            const double vm = it.va + z * (it.vb - it.va);
            a.vb = vm; b.va = vm;
        }
        stack.push_back(b);
        stack.push_back(a);
    }
    return true;
}

void decompose_surface(int p, int q, int nu, int nv, const double* P, const double* U, const double* V, double tol_rel,
                       SurfOut& out)
{
    std::string err;
    int code = 0;
    std::vector<double> zeros((size_t)3 * std::max(nu, nv), 0.0);
    if (!validate_curve(p, nu, zeros.data(), U, err, code) || !validate_curve(q, nv, zeros.data(), V, err, code)) {
        out.rc = code;
        out.err = err;
        return;
    }
    for (int64_t i = 0; i < (int64_t)3 * nu * nv; ++i)
        if (!std::isfinite(P[i])) { out.rc = MREP_E_INVALID_ARG; out.err = "non-finite control point"; return; }
    double lo[3] = {P[0], P[1], P[2]}, hi[3] = {P[0], P[1], P[2]};
    for (int i = 0; i < nu * nv; ++i)
        for (int c = 0; c < 3; ++c) { lo[c] = std::min(lo[c], P[3 * i + c]); hi[c] = std::max(hi[c], P[3 * i + c]); }
    out.diag = sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) + (hi[2] - lo[2]) * (hi[2] - lo[2]));
    out.tol_abs = tol_rel * out.diag;
    std::vector<int> su, sv;
    for (int k = p; k <= nu - 1; ++k) if (U[k] < U[k + 1]) su.push_back(k);
    for (int k = q; k <= nv - 1; ++k) if (V[k] < V[k + 1]) sv.push_back(k);
    out.n_su = (int)su.size();
    out.n_sv = (int)sv.size();
    for (int k : su) out.brk.push_back(U[k]);
    out.brk.push_back(U[su.back() + 1]);
    for (int k : sv) out.brk.push_back(V[k]);
    out.brk.push_back(V[sv.back() + 1]);
    const DegreeTables& Tp = g_tab[p];
    const DegreeTables& Tq = g_tab[q];
    double Au[(kMaxP + 1) * (kMaxP + 1)], Av[(kMaxP + 1) * (kMaxP + 1)];
    double Du[(kMaxP + 1) * (kMaxP + 1)], Dv[(kMaxP + 1) * (kMaxP + 1)];
    double Mu[(kMaxP + 1) * (kMaxP + 1)], Mv[(kMaxP + 1) * (kMaxP + 1)];
    std::vector<double> Cf((size_t)(p + 1) * (q + 1) * 3), Nz((size_t)(p + 1) * (q + 1) * 3);
    int32_t span = 0;
    for (int a = 0; a < out.n_su; ++a) {
        const int qu = su[(size_t)a];
        const double hu = U[qu + 1] - U[qu];
        span_basis_poly(p, U, qu, Au);
        double hj = 1.0;
        for (int j = 0; j <= p; ++j, hj *= hu)
            for (int r = 0; r <= p; ++r) Du[j * (p + 1) + r] = hj * Au[j * (p + 1) + r];
        for (int i = 0; i <= p; ++i)
            for (int r = 0; r <= p; ++r) {
                double s = 0.0;
                for (int j = 0; j <= i; ++j) s += Tp.Bi[i * (p + 1) + j] * Du[j * (p + 1) + r];
                Mu[i * (p + 1) + r] = s;
            }
        for (int b = 0; b < out.n_sv; ++b) {
            const int qv = sv[(size_t)b];
            const double hv = V[qv + 1] - V[qv];
            span_basis_poly(q, V, qv, Av);
            double hk = 1.0;
            for (int j = 0; j <= q; ++j, hk *= hv)
                for (int r = 0; r <= q; ++r) Dv[j * (q + 1) + r] = hk * Av[j * (q + 1) + r];
            for (int i = 0; i <= q; ++i)
                for (int r = 0; r <= q; ++r) {
                    double s = 0.0;
                    for (int j = 0; j <= i; ++j) s += Tq.Bi[i * (q + 1) + j] * Dv[j * (q + 1) + r];
                    Mv[i * (q + 1) + r] = s;
                }
            // C = Du P Dv^T and N = Mu P Mv^T over the span's control points
            for (int x = 0; x <= p; ++x)
                for (int y = 0; y <= q; ++y)
                    for (int c = 0; c < 3; ++c) {
                        double sc = 0.0, sn = 0.0;
                        for (int r = 0; r <= p; ++r)
                            for (int t = 0; t <= q; ++t) {
                                const double pv = P[3 * ((size_t)(qu - p + r) * nv + (qv - q + t)) + c];
                                sc += Du[x * (p + 1) + r] * Dv[y * (q + 1) + t] * pv;
                                sn += Mu[x * (p + 1) + r] * Mv[y * (q + 1) + t] * pv;
                            }
                        Cf[3 * (x * (q + 1) + y) + c] = sc;
                        Nz[3 * (x * (q + 1) + y) + c] = sn;
                    }
            out.coef.insert(out.coef.end(), Cf.begin(), Cf.end());
            out.span_first.push_back((int32_t)out.pieces.size());
            if (!reduce_patch(p, q, Nz.data(), U[qu], U[qu + 1], V[qv], V[qv + 1], out.tol_abs, span, out.pieces)) {
                out.rc = MREP_E_TOL;
                out.err = "a span patch needed more than MREP_MAX_PIECES_PER_SPAN pieces";
                return;
            }
            ++span;
        }
    }
    if (p <= 3 && q <= 3) out.tol_abs = 0.0;
}

// tables of one bicubic patch: FP32 centre relative to the origin (exact in
// FP64), radius bound, FP32 net relative to the centre
void patch_tables(const double* R, const double* o, double tol_eff, float* sph, float* lcp)
{
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
        lo[c] = hi[c] = R[c];
        for (int i = 1; i < 16; ++i) { lo[c] = std::min(lo[c], R[3 * i + c]); hi[c] = std::max(hi[c], R[3 * i + c]); }
    }
    float cf[3];
    double cd[3];
    for (int c = 0; c < 3; ++c) {
        cf[c] = (float)(0.5 * (lo[c] + hi[c]) - o[c]);
        cd[c] = o[c] + (double)cf[c];
    }
    double r = 0.0;
    for (int i = 0; i < 16; ++i) {
        double d2 = 0.0;
        for (int c = 0; c < 3; ++c) d2 += (R[3 * i + c] - cd[c]) * (R[3 * i + c] - cd[c]);
        r = std::max(r, sqrt(d2));
        for (int c = 0; c < 3; ++c) lcp[3 * i + c] = (float)(R[3 * i + c] - cd[c]);
    }
    sph[0] = cf[0];
    sph[1] = cf[1];
    sph[2] = cf[2];
    sph[3] = nextafterf((float)(r * (1.0 + 1e-6) + tol_eff * (1.0 + 1e-6)), INFINITY);
}

// Cluster = block of bs x bs exact spans of one surface, about 32 patches,
// at most 65535 clusters per surface.
int cluster_block(int64_t n_patch, int32_t n_su, int32_t n_sv)
{
    const double pps = (double)n_patch / std::max<int64_t>(1, (int64_t)n_su * n_sv);
    int bs = (int)std::max(1L, std::min(8L, lround(sqrt(32.0 / std::max(pps, 1e-9)))));
    while ((int64_t)((n_su + bs - 1) / bs) * ((n_sv + bs - 1) / bs) > 65535) ++bs;
    return bs;
}

// sphere (FP32 centre in the same frame, radius rounded up) containing the
// patch spheres sph[4k..] of the cluster's span rows: centre at the middle of
// their centres' box
void cluster_sphere(const float* sph, const int32_t* span0, const DSurf& d, int32_t c, float* out)
{
    const int bs = d.clu_bs, bu = c / d.n_cbv, bv = c % d.n_cbv;
    const int iu0 = bu * bs, iu1 = std::min(d.n_su, iu0 + bs), iv0 = bv * bs, iv1 = std::min(d.n_sv, iv0 + bs);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t end = d.span_off + (int64_t)d.n_su * d.n_sv;  // first span of the next surface
    auto rows = [&](auto&& f) {
        for (int iu = iu0; iu < iu1; ++iu) {
            const int64_t rs = d.span_off + (int64_t)iu * d.n_sv;
            const int64_t k1 = rs + iv1 == end ? d.patch_off + d.n_patch : span0[rs + iv1];
            for (int64_t k = span0[rs + iv0]; k < k1; ++k) f(k);
        }
    };
    rows([&](int64_t k) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], (double)sph[4 * k + a]);
            hi[a] = std::max(hi[a], (double)sph[4 * k + a]);
        }
    });
    float cf[3];
    for (int a = 0; a < 3; ++a) cf[a] = lo[a] <= hi[a] ? (float)(0.5 * (lo[a] + hi[a])) : 0.f;
    double r = 0.0;
    rows([&](int64_t k) {
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) d2 += ((double)sph[4 * k + a] - cf[a]) * ((double)sph[4 * k + a] - cf[a]);
        r = std::max(r, sqrt(d2) + (double)sph[4 * k + 3]);
    });
    for (int a = 0; a < 3; ++a) out[a] = cf[a];
    out[3] = nextafterf((float)(r * (1.0 + 1e-6)), INFINITY);
}

}  // namespace

int build_surf_plan(int32_t n_surf, const int32_t* deg_u, const int32_t* deg_v, const int32_t* n_u, const int32_t* n_v,
                    const int64_t* cp_off, const double* cp_xyz, const int64_t* ku_off, const double* ku,
                    const int64_t* kv_off, const double* kv, double tol_rel, int n_threads, SurfPlan& plan,
                    std::string& err)
{
    init_tables();
    for (int32_t s = 0; s < n_surf; ++s) {
        const std::string who = "surface " + std::to_string(s) + ": ";
        if (deg_u[s] < 1 || deg_u[s] > MREP_MAX_SURFACE_DEGREE || deg_v[s] < 1 || deg_v[s] > MREP_MAX_SURFACE_DEGREE) { err = who + "degree out of range"; return MREP_E_BAD_DEGREE; }
        if (n_u[s] < deg_u[s] + 1 || n_v[s] < deg_v[s] + 1) { err = who + "too few control points"; return MREP_E_BAD_DEGREE; }
        if (cp_off[s + 1] - cp_off[s] != (int64_t)n_u[s] * n_v[s]) { err = who + "net size != n_u * n_v"; return MREP_E_INVALID_ARG; }
        if (ku_off[s + 1] - ku_off[s] != n_u[s] + deg_u[s] + 1 || kv_off[s + 1] - kv_off[s] != n_v[s] + deg_v[s] + 1) {
            err = who + "knot count != points + degree + 1";
            return MREP_E_BAD_KNOTS;
        }
        if ((int64_t)n_u[s] * n_v[s] > ((int64_t)1 << 24)) { err = who + "net too large"; return MREP_E_INVALID_ARG; }
    }
    std::vector<SurfOut> outs((size_t)n_surf);
    int nt = n_threads > 0 ? n_threads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = std::min<int>(nt, std::max<int32_t>(1, n_surf));
    std::atomic<int32_t> next{0};
    auto worker = [&]() {
        for (;;) {
            const int32_t s = next.fetch_add(1);
            if (s >= n_surf) break;
            decompose_surface(deg_u[s], deg_v[s], n_u[s], n_v[s], cp_xyz + 3 * cp_off[s], ku + ku_off[s],
                              kv + kv_off[s], tol_rel, outs[(size_t)s]);
        }
    };
    std::vector<std::thread> th;
    for (int i = 1; i < nt; ++i) th.emplace_back(worker);
    worker();
    for (auto& t : th) t.join();
    for (int32_t s = 0; s < n_surf; ++s)
        if (outs[(size_t)s].rc) {
            err = "surface " + std::to_string(s) + ": " + outs[(size_t)s].err;
            return outs[(size_t)s].rc;
        }
    plan.n_surf = n_surf;
    plan.tol_rel = tol_rel;
    plan.surfs.resize((size_t)n_surf);
    int64_t npatch = 0, nspan = 0, ncoef = 0, nbrk = 0, nclu = 0;
    for (int32_t s = 0; s < n_surf; ++s) {
        const SurfOut& o = outs[(size_t)s];
        DSurf& d = plan.surfs[(size_t)s];
        d.patch_off = npatch;
        d.span_off = nspan;
        d.coef_off = ncoef;
        d.brk_off = nbrk;
        d.n_patch = (int32_t)o.pieces.size();
        d.n_su = o.n_su;
        d.n_sv = o.n_sv;
        d.deg_u = deg_u[s];
        d.deg_v = deg_v[s];
        d.clu_bs = cluster_block((int64_t)o.pieces.size(), o.n_su, o.n_sv);
        d.n_cbv = (o.n_sv + d.clu_bs - 1) / d.clu_bs;
        d.n_clu = ((o.n_su + d.clu_bs - 1) / d.clu_bs) * d.n_cbv;
        d.clu_off = nclu;
        nclu += d.n_clu;
        d.tol_eff = (deg_u[s] >= 4 || deg_v[s] >= 4) ? o.tol_abs : 1e-13 * o.diag;
        d.tol_user = tol_rel * o.diag;
        d.diag = o.diag;
        const double* P = cp_xyz + 3 * cp_off[s];
        const int64_t n = (int64_t)n_u[s] * n_v[s];
        for (int k = 0; k < 3; ++k) {
            double lo = P[k], hi = P[k];
            for (int64_t i = 0; i < n; ++i) { lo = std::min(lo, P[3 * i + k]); hi = std::max(hi, P[3 * i + k]); }
            d.origin[k] = (double)(float)(0.5 * (lo + hi));
        }
        npatch += d.n_patch;
        nspan += (int64_t)o.n_su * o.n_sv;
        ncoef += (int64_t)o.coef.size();
        nbrk += (int64_t)o.brk.size();
        plan.max_degree = std::max(plan.max_degree, std::max(deg_u[s], deg_v[s]));
    }
    if (npatch >= ((int64_t)1 << 31)) { err = "more than 2^31 patches"; return MREP_E_INVALID_ARG; }
    plan.gcp.resize((size_t)npatch * 48);
    plan.uv.resize((size_t)npatch * 4);
    plan.pspan.resize((size_t)npatch);
    plan.span0.resize((size_t)nspan + 1);
    plan.brk.resize((size_t)nbrk);
    plan.coef.resize((size_t)ncoef);
    plan.sph.resize((size_t)npatch * 4);
    plan.lcp.resize((size_t)npatch * 48);
    plan.csph.resize((size_t)nclu * 4);
    std::atomic<int32_t> next2{0};
    auto worker2 = [&]() {
        for (;;) {
            const int32_t s = next2.fetch_add(1);
            if (s >= n_surf) break;
            const SurfOut& o = outs[(size_t)s];
            const DSurf& d = plan.surfs[(size_t)s];
            for (int32_t k = 0; k < d.n_patch; ++k) {
                const SPiece& pc = o.pieces[(size_t)k];
                const int64_t g = d.patch_off + k;
                memcpy(&plan.gcp[(size_t)g * 48], pc.R, sizeof(double) * 48);
                plan.uv[(size_t)g * 4] = pc.ua;
                plan.uv[(size_t)g * 4 + 1] = pc.ub;
                plan.uv[(size_t)g * 4 + 2] = pc.va;
                plan.uv[(size_t)g * 4 + 3] = pc.vb;
                plan.pspan[(size_t)g] = (int32_t)(d.span_off + pc.span);
                patch_tables(pc.R, d.origin, d.tol_eff, &plan.sph[(size_t)g * 4], &plan.lcp[(size_t)g * 48]);
            }
            const int64_t ns_s = (int64_t)o.n_su * o.n_sv;
            for (int64_t j = 0; j < ns_s; ++j)
                plan.span0[(size_t)(d.span_off + j)] = (int32_t)(d.patch_off + o.span_first[(size_t)j]);
            for (int32_t c = 0; c < d.n_clu; ++c)
                cluster_sphere(plan.sph.data(), plan.span0.data(), d, c, &plan.csph[(size_t)(d.clu_off + c) * 4]);
            memcpy(&plan.brk[(size_t)d.brk_off], o.brk.data(), sizeof(double) * o.brk.size());
            memcpy(&plan.coef[(size_t)d.coef_off], o.coef.data(), sizeof(double) * o.coef.size());
        }
    };
    th.clear();
    for (int i = 1; i < nt; ++i) th.emplace_back(worker2);
    worker2();
    for (auto& t : th) t.join();
    plan.span0[(size_t)nspan] = (int32_t)npatch;
    SurfLayout& L = plan.layout;
    L.n_surf = n_surf;
    L.n_patch = npatch;
    L.n_span = nspan;
    L.n_coef = ncoef;
    L.n_brk = nbrk;
    int64_t off = 0;
    L.off_surf = off; off = align256(off + (int64_t)sizeof(DSurf) * n_surf);
    L.off_sph = off; off = align256(off + 16 * npatch);
    L.off_lcp = off; off = align256(off + 4 * 48 * npatch);
    L.off_gcp = off; off = align256(off + 8 * 48 * npatch);
    L.off_uv = off; off = align256(off + 8 * 4 * npatch);
    L.off_pspan = off; off = align256(off + 4 * npatch);
    L.off_span0 = off; off = align256(off + 4 * (nspan + 1));
    L.n_clu = nclu;
    L.off_csph = off; off = align256(off + 16 * nclu);
    L.off_brk = off; off = align256(off + 8 * nbrk);
    L.off_coef = off; off = align256(off + 8 * ncoef);
    L.total = off;
    return MREP_OK;
}

}  // namespace mrep
