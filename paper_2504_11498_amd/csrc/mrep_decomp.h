// Decomposition arithmetic shared by the host decomposition (g++) and the
// device decomposition (hipcc): one source compiled both ways, both without
// floating-point contraction and with correctly rounded division and square
// root, so that the host and the device produce the same bits.
// Sec. 5.2.1 (span forms, eqs. decomposition / decomfinal), Sec. 5.2.2 (G1/L2
// reduction, eqs. gram / G1-condition; error control, eq. epsl; splitting,
// eqs. submatrix / subLandR); the screen tables of a cubic piece.
#pragma once

#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/mrep.h"
#include "mrep_internal.h"

#if defined(__HIPCC__)
#define MREP_HD __host__ __device__
#else
#define MREP_HD
#endif

namespace mrep {
namespace dm {

constexpr int kMaxP = MREP_MAX_DEGREE;
constexpr int kErrSamples = 129;  // u_i = i / 128

// std::max / std::min semantics, usable on both sides
template <class T>
MREP_HD inline T mx(T a, T b) { return (a < b) ? b : a; }
template <class T>
MREP_HD inline T mn(T a, T b) { return (b < a) ? b : a; }
MREP_HD inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Constant tables per degree: Bernstein inverse, Bernstein values at the error
// samples, elevation of a cubic to degree p, Gram matrices (eq. gram).
struct DegreeTables {
    int p = 0;
    double Bi[(kMaxP + 1) * (kMaxP + 1)];                 // power -> Bernstein
    double Bq[kErrSamples * (kMaxP + 1)];                 // B_{k,p}(u_i)
    double B3[kErrSamples * 4];                           // B_{k,3}(u_i)
    double E3p[(kMaxP + 1) * 4];                          // cubic written at degree p
    double G3p[4 * (kMaxP + 1)];                          // Gram G_{3,p}
    double G33[16];
};

MREP_HD inline double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return round(r);
}

MREP_HD inline double ipow(double x, int k)
{
    double r = 1.0;
    for (int i = 0; i < k; ++i) r *= x;
    return r;
}

MREP_HD inline float bf16_to_f32(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// FP32 -> BF16, round to nearest even (NaN kept quiet)
MREP_HD inline uint16_t f32_to_bf16_rne(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    uint32_t r = 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)((u + r) >> 16);
}


// Power coefficients (in s = t - t_q) of N_{q-p+r, p} for r = 0..p on span q:
// A[j*(p+1) + r] = coefficient of s^j.  Cox-de Boor on polynomials.
// MP bounds the degree (the arrays' size only; the arithmetic does not depend on it).
template <int MP>
MREP_HD inline void span_basis_poly(int p, const double* U, int q, double* A)
{
    double N[MP + 2][MP + 2];  // N[r][j], r = i - (q - p)
    for (int r = 0; r <= p + 1; ++r)
        for (int j = 0; j <= p + 1; ++j) N[r][j] = 0.0;
    N[p][0] = 1.0;  // N_{q,0} = 1 on [t_q, t_q+1)
    const double tq = U[q];
    for (int k = 1; k <= p; ++k) {
        double M[MP + 2][MP + 2];
        for (int r = 0; r <= p + 1; ++r)
            for (int j = 0; j <= p + 1; ++j) M[r][j] = 0.0;
        for (int i = q - k; i <= q; ++i) {
            int r = i - (q - p);
            // (s + tq - U_i)/(U_{i+k} - U_i) * N_{i,k-1}
            double d1 = U[i + k] - U[i];
            if (d1 != 0.0) {
                double c0 = (tq - U[i]) / d1, c1 = 1.0 / d1;
                for (int j = 0; j < k; ++j) {
                    M[r][j] += c0 * N[r][j];
                    M[r][j + 1] += c1 * N[r][j];
                }
            }
            // (U_{i+k+1} - tq - s)/(U_{i+k+1} - U_{i+1}) * N_{i+1,k-1}
            double d2 = U[i + k + 1] - U[i + 1];
            if (d2 != 0.0 && r + 1 <= p) {
                double c0 = (U[i + k + 1] - tq) / d2, c1 = -1.0 / d2;
                for (int j = 0; j < k; ++j) {
                    M[r][j] += c0 * N[r + 1][j];
                    M[r][j + 1] += c1 * N[r + 1][j];
                }
            }
        }
        memcpy(N, M, sizeof(N));
    }
    for (int j = 0; j <= p; ++j)
        for (int r = 0; r <= p; ++r) A[j * (p + 1) + r] = N[r][j];
}

// G1 L2-optimal cubic of a degree-p piece (p >= 4).
MREP_HD inline void g1_reduce(int p, const DegreeTables& T, const double* Q, double* R)
{
    const double* Q0 = Q;
    const double* Qp = Q + 3 * p;
    double a[3], b[3], V1[3], V2[3];
    const double* g = T.G33;
    for (int c = 0; c < 3; ++c) {
        a[c] = (double)p / 3.0 * (Q[3 + c] - Q[c]);
        b[c] = (double)p / 3.0 * (Q[3 * p + c] - Q[3 * (p - 1) + c]);
        double s1 = 0.0, s2 = 0.0;
        for (int k = 0; k <= p; ++k) {
            s1 += T.G3p[1 * (p + 1) + k] * Q[3 * k + c];
            s2 += T.G3p[2 * (p + 1) + k] * Q[3 * k + c];
        }
        V1[c] = s1 - (g[4 + 0] + g[4 + 1]) * Q0[c] - (g[4 + 2] + g[4 + 3]) * Qp[c];
        V2[c] = s2 - (g[8 + 0] + g[8 + 1]) * Q0[c] - (g[8 + 2] + g[8 + 3]) * Qp[c];
    }
    double aa = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    double bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    double V1a = V1[0] * a[0] + V1[1] * a[1] + V1[2] * a[2];
    double V2b = V2[0] * b[0] + V2[1] * b[1] + V2[2] * b[2];
    double g11 = g[5], g12 = g[6], g21 = g[9], g22 = g[10];
    // g11 aa d0 - g12 ab d1 = V1a ;  g21 ab d0 - g22 bb d1 = V2b
    double d0 = 1.0, d1 = 1.0;
    if (aa > 0.0 && bb > 0.0) {
        double m11 = g11 * aa, m12 = -g12 * ab, m21 = g21 * ab, m22 = -g22 * bb;
        double det = m11 * m22 - m12 * m21;
        d0 = (V1a * m22 - m12 * V2b) / det;
        d1 = (m11 * V2b - m21 * V1a) / det;
    } else if (aa > 0.0) {
        d0 = (V1a + g12 * ab * d1) / (g11 * aa);
    } else if (bb > 0.0) {
        d1 = (g21 * ab * d0 - V2b) / (g22 * bb);
    }
    for (int c = 0; c < 3; ++c) {
        R[c] = Q0[c];
        R[3 + c] = Q0[c] + a[c] * d0;
        R[6 + c] = Qp[c] - b[c] * d1;
        R[9 + c] = Qp[c];
    }
}

// Deviation bound of R from Q: max over the error samples plus (1/256) times a
// bound on |Q' - R'| from the hodograph of Q - E3p R.
MREP_HD inline double deviation_bound(int p, const DegreeTables& T, const double* Q, const double* R, int* imax)
{
    // |Q(u_i) - R(u_i)| at error sample i (recomputed where needed: no per-sample array)
    auto ev = [&](int i) {
        double x[3] = {0, 0, 0}, y[3] = {0, 0, 0};
        for (int k = 0; k <= p; ++k)
            for (int c = 0; c < 3; ++c) x[c] += T.Bq[i * (p + 1) + k] * Q[3 * k + c];
        for (int k = 0; k < 4; ++k)
            for (int c = 0; c < 3; ++c) y[c] += T.B3[i * 4 + k] * R[3 * k + c];
        return sqrt((x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]) + (x[2] - y[2]) * (x[2] - y[2]));
    };
    double best = -1.0;
    int bi = 64;
    for (int i = 0; i < kErrSamples; ++i) best = mx(best, ev(i));
    // The deviation can peak at several parameters at once (the paper splits
    // all of them); samples within 1e-6 relative of the maximum count as tied
    // and the smallest parameter among them is split first, so that rounding
    // differences cannot move the split point.
    for (int i = 0; i < kErrSamples; ++i)
        if (ev(i) >= best * (1.0 - 1e-6)) { bi = i; break; }
    // hodograph bound of Q - E3p R (its control points D_i, recomputed per use)
    auto dcp = [&](int i, int c) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += T.E3p[i * 4 + k] * R[3 * k + c];
        return Q[3 * i + c] - s;
    };
    double L = 0.0;
    for (int i = 0; i < p; ++i) {
        double v2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            double d = dcp(i + 1, c) - dcp(i, c);
            v2 += d * d;
        }
        double v = (double)p * sqrt(v2);
        if (v > L) L = v;
    }
    *imax = bi;
    return best + L / 256.0;
}

// Split a degree-p Bezier piece at z with the entries of the subdivision
// matrix S(z) (eqs. submatrix, subLandR) computed where they are used; the
// zero entries are skipped, which leaves every sum unchanged.
MREP_HD inline void split_piece(int p, const double* Q, double z, double* L, double* R)
{
    for (int i = 0; i <= p; ++i)
        for (int c = 0; c < 3; ++c) {
            double l = 0.0, r = 0.0;
            for (int k = 0; k <= i; ++k) l += binom(i, k) * ipow(z, k) * ipow(1.0 - z, i - k) * Q[3 * k + c];
            for (int k = i; k <= p; ++k) r += binom(p - i, k - i) * ipow(z, k - i) * ipow(1.0 - z, p - k) * Q[3 * k + c];
            L[3 * i + c] = l;
            R[3 * i + c] = r;
        }
}


// sphere of one piece: its FP32 centre (aux) and the largest control-point
// distance from it plus the deviation bound, rounded up
MREP_HD inline void piece_sphere(const float* aux, const float* lcp, double tol_eff, float* out)
{
    double r2 = 0.0;
    for (int i = 0; i < 4; ++i) {
        const double x = lcp[3 * i], y = lcp[3 * i + 1], z = lcp[3 * i + 2];
        r2 = mx(r2, x * x + y * y + z * z);
    }
    out[0] = aux[AUX_CX];
    out[1] = aux[AUX_CY];
    out[2] = aux[AUX_CZ];
    out[3] = nextafterf((float)(sqrt(r2) * (1.0 + 2e-6) + tol_eff * (1.0 + 1e-6)), INFINITY);
}

// sphere containing the m spheres sph[4k..]: centre at the middle of their
// centres' box, radius rounded up
MREP_HD inline void bounding_sphere(const float* sph, int64_t m, float* out)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = 0; k < m; ++k)
        for (int a = 0; a < 3; ++a) {
            lo[a] = mn(lo[a], (double)sph[4 * k + a]);
            hi[a] = mx(hi[a], (double)sph[4 * k + a]);
        }
    float cf[3];
    for (int a = 0; a < 3; ++a) cf[a] = m > 0 ? (float)(0.5 * (lo[a] + hi[a])) : 0.f;
    double r = 0.0;
    for (int64_t k = 0; k < m; ++k) {
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) d2 += ((double)sph[4 * k + a] - cf[a]) * ((double)sph[4 * k + a] - cf[a]);
        r = mx(r, sqrt(d2) + (double)sph[4 * k + 3]);
    }
    for (int a = 0; a < 3; ++a) out[a] = cf[a];
    out[3] = nextafterf((float)(r * (1.0 + 1e-6)), INFINITY);
}

// Screen and refine tables of one piece.  The centre c = o + c_rel with c_rel
// rounded to FP32, o the curve origin, so that c is exact in FP64.
MREP_HD inline void piece_tables(const double* R, const double* o, double tol_eff, uint16_t* col, float* aux, float* lcp)
{
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
        lo[c] = mn(mn(R[c], R[3 + c]), mn(R[6 + c], R[9 + c]));
        hi[c] = mx(mx(R[c], R[3 + c]), mx(R[6 + c], R[9 + c]));
    }
    float cf[3];
    double cd[3];
    for (int c = 0; c < 3; ++c) {
        cf[c] = (float)(0.5 * (lo[c] + hi[c]) - o[c]);
        cd[c] = o[c] + (double)cf[c];
    }
    double crel[3] = {(double)cf[0], (double)cf[1], (double)cf[2]};
    double a[4][3];
    for (int c = 0; c < 3; ++c) {
        a[0][c] = R[c] - cd[c];
        a[1][c] = 3.0 * (R[3 + c] - R[c]);
        a[2][c] = 3.0 * (R[6 + c] - 2.0 * R[3 + c] + R[c]);
        a[3][c] = R[9 + c] - 3.0 * R[6 + c] + 3.0 * R[3 + c] - R[c];
    }
    // the screen works in the centred parameter v = 2u - 1: b_m = sum_j a_j C(j,m) 2^-j
    double b[4][3];
    for (int m = 0; m < 4; ++m)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int j = m; j < 4; ++j) s += a[j][c] * binom(j, m) * ipow(0.5, j);
            b[m][c] = s;
        }
    double e[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 4; ++k) e[j + k] += dot3(b[j], b[k]);
    for (int m = 0; m < 4; ++m) e[m] += 2.0 * dot3(crel, b[m]);
    double colv[kScreenK];
    for (int i = 0; i < kScreenK; ++i) colv[i] = 0.0;
    for (int j = 0; j < 4; ++j)
        for (int c = 0; c < 3; ++c) colv[3 * j + c] = -2.0 * b[j][c];
    for (int m = 0; m < 7; ++m) colv[12 + m] = e[m];
    double As = 0.0, Es = 0.0, Cs = 0.0;
    for (int i = 0; i < 12; ++i) As += fabs(colv[i]);
    for (int m = 0; m < 7; ++m) Es += fabs(e[m]);
    for (int i = 0; i < kScreenK; ++i) col[i] = f32_to_bf16_rne((float)colv[i]);
    // entries 19..31: the piece's part of |q' - c|^2.  c_i = ch_i + cl_i (+ a
    // rest of <= 2^-16 |c_i|), both BF16; rows carry qh_i, qh_i, ql_i, Qh, Ql,
    // 1, 1 (see the screen kernel), so that the row . column sum adds
    // -2 (qh.ch + qh.cl + ql.ch) + (Qh + Ql) + (Ph + Pl) ~ |q' - c|^2 - beta - gamma.
    const double ccf = (double)cf[0] * cf[0] + (double)cf[1] * cf[1] + (double)cf[2] * cf[2];
    for (int c = 0; c < 3; ++c) {
        const uint16_t h = f32_to_bf16_rne(cf[c]);
        const float hf = bf16_to_f32(h);
        const uint16_t l = f32_to_bf16_rne(cf[c] - hf);  // cf - hf is exact in FP32
        col[19 + c] = f32_to_bf16_rne(-2.0f * hf);
        col[22 + c] = f32_to_bf16_rne(-2.0f * bf16_to_f32(l));
        col[25 + c] = col[19 + c];
        Cs += fabs((double)cf[c]);
    }
    col[28] = col[29] = f32_to_bf16_rne(1.0f);
    // Error of the screen's sum against D - beta_eff - gamma_eff (D the exact
    // squared sample distance), per (query, piece):
    //   qmax alpha + beta_req + gamma_req,
    //   alpha = kappa' A + 1.02e-4 sum|c_i|     (BF16 rounding of the first 19
    //           entries; the split cross term 6.03 * 2^-16 |q'_i||c_i|; the
    //           FP32 accumulation 62 * 2^-24 of |products| <= 2.05 qmax sum|c_i|)
    //   beta_req  = kappa' E + 4e-6 |c|^2       (accumulation of |Ph + Pl|)
    //   gamma_req = 4e-6 |q'|^2                 (per query, in the kernel)
    // The constant entry P = |c|^2 - beta_t is split into Ph + Pl, and
    // beta_eff = |c|^2 - (Ph + Pl) (exact in FP64 here) is checked to be at
    // least beta_req, so that the sum minus qmax alpha is a lower bound of D.
    const double kap = kScreenKappaBf16 * 1.01 + 1e-6;
    const double alpha = kap * As + 1.02e-4 * Cs;
    const double beta_req = kap * Es + 4e-6 * ccf + 1e-30;
    double beta_t = beta_req + 0x1p-15 * (ccf + beta_req);
    double beta_eff = 0.0;
    for (int tries = 0; tries < 4; ++tries) {
        const double P = ccf - beta_t;
        const uint16_t h = f32_to_bf16_rne((float)P);
        const double hd = (double)bf16_to_f32(h);
        const uint16_t l = f32_to_bf16_rne((float)(P - hd));
        col[30] = h;
        col[31] = l;
        beta_eff = ccf - (hd + (double)bf16_to_f32(l));
        if (beta_eff >= beta_req) break;
        beta_t += 2.0 * (beta_req - beta_eff);
    }
    double L = 0.0;
    for (int i = 0; i < 3; ++i) {
        double d[3] = {R[3 * (i + 1)] - R[3 * i], R[3 * (i + 1) + 1] - R[3 * i + 1], R[3 * (i + 1) + 2] - R[3 * i + 2]};
        L = mx(L, 3.0 * sqrt(dot3(d, d)));
    }
    aux[AUX_CX] = cf[0];
    aux[AUX_CY] = cf[1];
    aux[AUX_CZ] = cf[2];
    aux[AUX_CC] = (float)dot3(crel, crel);
    // rounded up from FP64 by a relative 1e-5
    aux[AUX_KA] = (float)(alpha * 1.00001);
    aux[AUX_KE] = (float)((beta_req + beta_eff * (1.0 + 1e-12) + 1e-30) * 1.00001);
    aux[AUX_ES] = (float)((L / (2.0 * (kSamples - 1)) + tol_eff) * 1.0001);
    aux[AUX_L] = (float)L;
    for (int i = 0; i < 4; ++i)
        for (int c = 0; c < 3; ++c) lcp[3 * i + c] = (float)(R[3 * i + c] - cd[c]);
}



// Elevation of a degree-(p+1) Bezier by one: E[i][j] (Sec. 5.2.2, p <= 2 pieces)
MREP_HD inline double elev(int p, int i, int j)
{
    double a = (double)i / (double)(p + 1);
    double v = 0.0;
    if (j == i - 1) v += a;
    if (j == i) v += 1.0 - a;
    return v;
}

// The cubic of a span of degree p <= 3: elevated to degree 3 (exact)
MREP_HD inline void elevate_to_cubic(int p, const double* Q, double* R)
{
    double Acur[3 * 4], Bn[3 * 4];
    for (int i = 0; i < 3 * (p + 1); ++i) Acur[i] = Q[i];
    for (int d = p; d < 3; ++d) {
        for (int i = 0; i <= d + 1; ++i)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int k = 0; k <= d; ++k) s += elev(d, i, k) * Acur[3 * k + c];
                Bn[3 * i + c] = s;
            }
        for (int i = 0; i < 3 * (d + 2); ++i) Acur[i] = Bn[i];
    }
    for (int i = 0; i < 12; ++i) R[i] = Acur[i];
}

// Span q of a degree-p curve in the matrix form of Sec. 5.2.1: D = diag(h^j)
// A P_{q-p..q} (power coefficients in the local u, eq. Mqpt with the origin at
// t_q) and its Bezier points Q = B_p^{-1} D (eq. decomfinal).  MP bounds p.
template <int MP>
MREP_HD inline void span_power_bezier(int p, const DegreeTables& T, const double* U, int q, const double* P, double* D,
                                      double* Q)
{
    double A[(MP + 1) * (MP + 1)];
    const double h = U[q + 1] - U[q];
    span_basis_poly<MP>(p, U, q, A);
    double hj = 1.0;
    for (int j = 0; j <= p; ++j) {
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int r = 0; r <= p; ++r) s += A[j * (p + 1) + r] * P[3 * (q - p + r) + c];
            D[3 * j + c] = hj * s;
        }
        hj *= h;
    }
    for (int i = 0; i <= p; ++i)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int j = 0; j <= i; ++j) s += T.Bi[i * (p + 1) + j] * D[3 * j + c];
            Q[3 * i + c] = s;
        }
}

// The per-degree tables of the host decomposition, index p = 0 .. kMaxP (host
// memory, built on first use): the device decomposition copies them.
const DegreeTables* degree_tables_host();

}  // namespace dm
}  // namespace mrep
