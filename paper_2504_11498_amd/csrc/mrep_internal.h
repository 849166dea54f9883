// Internal layout shared by the host decomposition and the HIP kernels of
// libmrep.  Not part of the public ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace mrep {

// Samples per cubic piece in the screen and in the per-candidate rescan: the
// local parameter u_k = k / (kSamples - 1), both ends included.
constexpr int kSamples = 32;
// Queries per screen workgroup tile.
#ifndef MREP_TILE_QUERIES
#define MREP_TILE_QUERIES 32
#endif
constexpr int kQueriesPerTile = MREP_TILE_QUERIES;
// accelerator complex dies of an MI355X, each with its own L2: tiled launches
// deal contiguous tile ranges to the dies
constexpr int kXcdCount = 8;
// Segments staged in LDS per chunk by the screen.
#ifndef MREP_SCREEN_CHUNK
#define MREP_SCREEN_CHUNK 256
#endif
constexpr int kChunk = MREP_SCREEN_CHUNK;
// Length of a screen row / column (MFMA K dimension, 19 entries used).
constexpr int kScreenK = 32;
// candidates a query may keep from the screen (16 lanes x 3 per lane at most)
constexpr int kMaxCand = 48;

// Per-curve record in device memory.
struct DCurve {
    int64_t seg_off;     // first piece (global index)
    int64_t span_off;    // first span (global index)
    int64_t coef_off;    // first double of this curve's exact spans (power coefficients, or Bezier points:
                         // 3 per point, 4 homogeneous ones for a rational curve)
    int32_t n_seg;
    int32_t n_span;
    int32_t degree;
    float es_max;        // largest sample-spacing term e = L/(2(S-1)) + tol of the curve's pieces
    double tol_eff;      // same-parameter deviation bound of the pieces (rounding level for p <= 3)
    double tol_user;     // tol_rel * diag: the caller's tolerance (inversion's on-curve test)
    double diag;         // control-point box diagonal
    double origin[3];    // FP32-representable box centre: screen coordinates are relative to it
    int64_t clu_off;     // first cluster (global): kCluPieces consecutive pieces each
    int32_t n_clu;
    int32_t clu_use;     // 1: the clusters are compact enough for the candidate sweep to use them
    int32_t rational;    // 1: a rational curve; its exact spans are homogeneous Bezier points (4 per point)
    int32_t pad_;
};
static_assert(sizeof(DCurve) == 112, "DCurve layout");
// 64-bit counters that follow the per-curve histogram at the start of a curve
// projection workspace (the sphere lists count their sphere tests there; one
// counter per workgroup slot modulo this, summed by mrep_workspace_counts)
constexpr int kWsCounters = 1024;
// pieces per cluster of a curve (the last one may hold fewer)
constexpr int kCluPieces = 32;

// Offsets (bytes) of each table inside the device buffer.
struct GeomLayout {
    int64_t n_curves = 0, n_seg = 0, n_span = 0, n_coef = 0;
    int64_t off_curve = 0;   // DCurve[n_curves]
    int64_t off_col = 0;     // uint16 (bf16 bits)[n_seg][32]   screen column
    int64_t off_aux = 0;     // float[n_seg][8]                 centre, bound terms
    int64_t off_lcp = 0;     // float[n_seg][12]                control points minus centre
    int64_t off_gcp = 0;     // double[n_seg][12]               control points (global)
    int64_t off_segt = 0;    // double[n_seg][2]                (t_a, t_b)
    int64_t off_segspan = 0; // int32[n_seg]                    span index (global)
    int64_t off_spant = 0;   // double[n_span][2]               (t_q, t_q+1)
    int64_t off_span0 = 0;   // int32[n_span + 1]               first piece of each span (global)
    int64_t off_coef = 0;    // double[n_coef]                  exact span power coefficients in local u
    int64_t n_clu = 0;
    int64_t off_sph = 0;     // float4[n_seg]                   piece sphere: centre (as aux), radius
    int64_t off_csph = 0;    // float4[n_clu]                   sphere around each cluster's piece spheres
    int64_t total = 0;
    int32_t general = 0;     // 1: some span is kept as (homogeneous) Bezier points, not in power form
};

// aux[8] per piece: cx, cy, cz (FP32 centre relative to the curve origin),
// |c|^2, then the screen's bound terms alpha (AUX_KA: the coefficient of
// max|q'_i| in the error of a screened squared distance) and K_B (AUX_KE: the
// piece's part of the upper bound's offset, beta_req + beta_eff), e = L/(2(S-1))
// + tol (sample spacing term), L (speed bound in u).  The screen reads the
// last four as one 16-byte record.
enum { AUX_CX = 0, AUX_CY, AUX_CZ, AUX_CC, AUX_KA, AUX_KE, AUX_ES, AUX_L };

// BF16 screen: |computed - exact| of a sample's squared distance is at most
// kappa * (max|q'_i| A + E).  BF16 rounds each row and column entry by <= 2^-8
// relative and the MFMA sums exact products in FP32 (<= 32 * 2^-24), so
// 2 * 2^-8 + 2^-16 + 32 * 2^-24 = 0.00783 is the bound; 0.0085 leaves margin.
constexpr double kScreenKappaBf16 = 0.0085;

struct Plan {
    int64_t n_curves = 0;
    double tol_rel = 0;
    int32_t max_degree = 0;
    std::vector<DCurve> curves;
    // pieces
    std::vector<double> seg_cp;   // 12 per piece (global FP64)
    std::vector<double> seg_t;    // 2 per piece
    std::vector<int32_t> seg_span;
    // spans
    std::vector<double> span_t;   // 2 per span
    std::vector<int32_t> span0;   // n_span + 1
    std::vector<double> coef;     // exact span power coefficients
    // derived screen tables
    std::vector<uint16_t> col;    // 32 per piece
    std::vector<float> aux;       // 8 per piece
    std::vector<float> lcp;       // 12 per piece
    std::vector<float> sph;       // 4 per piece
    std::vector<float> csph;      // 4 per cluster
    GeomLayout layout;
};

struct Geom {
    GeomLayout L;
    char* base = nullptr;
    int device = 0;
    const DCurve* curves() const { return reinterpret_cast<const DCurve*>(base + L.off_curve); }
};

// ---------------------------------------------------------------------------
// Surfaces: bicubic patches of tensor-product B-spline surfaces
// ---------------------------------------------------------------------------
// Per-surface record in device memory.
struct DSurf {
    int64_t patch_off;   // first bicubic patch (global)
    int64_t span_off;    // first exact span patch (global); u-span major, n_su x n_sv
    int64_t coef_off;    // first double of the exact span patches' power coefficients
    int64_t brk_off;     // first double of the breakpoints: n_su + 1 in u, then n_sv + 1 in v
    int32_t n_patch;
    int32_t n_su, n_sv;  // exact span grid
    int32_t deg_u, deg_v;
    int32_t clu_bs;      // cluster = block of clu_bs x clu_bs exact spans
    double tol_eff;      // deviation bound of the patches from the exact surface
    double tol_user;     // tol_rel * diag
    double diag;         // control-net box diagonal
    double origin[3];    // FP32-representable box centre
    int64_t clu_off;     // first cluster (global); clusters row-major over the span blocks
    int32_t n_clu, n_cbv;  // clusters, cluster columns (blocks along v)
};
static_assert(sizeof(DSurf) == 120, "DSurf layout");

struct SurfLayout {
    int64_t n_surf = 0, n_patch = 0, n_span = 0, n_coef = 0, n_brk = 0;
    int64_t off_surf = 0;   // DSurf[n_surf]
    int64_t off_sph = 0;    // float4[n_patch]      centre (relative to the surface origin), radius
    int64_t off_lcp = 0;    // float[n_patch][48]  control net minus centre (u-major, 4 x 4 x xyz)
    int64_t off_gcp = 0;    // double[n_patch][48] control net (global)
    int64_t off_uv = 0;     // double[n_patch][4]  (u_a, u_b, v_a, v_b)
    int64_t off_pspan = 0;  // int32[n_patch]      exact span patch (global)
    int64_t off_span0 = 0;  // int32[n_span + 1]   first patch of each exact span patch (global)
    int64_t n_clu = 0;
    int64_t off_csph = 0;   // float4[n_clu]       sphere around the spheres of each cluster's patches
    int64_t off_brk = 0;    // double[n_brk]
    int64_t off_coef = 0;   // double[n_coef]      exact span patches: power coefficients in local (s, t)
    int64_t total = 0;
};

struct SurfPlan {
    int64_t n_surf = 0;
    double tol_rel = 0;
    int32_t max_degree = 0;
    std::vector<DSurf> surfs;
    std::vector<double> gcp, uv, brk, coef;
    std::vector<int32_t> pspan, span0;
    std::vector<float> sph, lcp, csph;
    SurfLayout layout;
};

struct SurfGeom {
    SurfLayout L;
    char* base = nullptr;
    int device = 0;
};

// host decomposition (mrep_host.cpp)
// weights (nullable): per control point, > 0: rational curves
int build_plan(int32_t n_curves, const int32_t* degree, const int64_t* cp_off, const double* cp_xyz,
               const double* weights, const int64_t* knot_off, const double* knots, double tol_rel, int n_threads,
               Plan& plan, std::string& err);
int build_surf_plan(int32_t n_surf, const int32_t* deg_u, const int32_t* deg_v, const int32_t* n_u,
                    const int32_t* n_v, const int64_t* cp_off, const double* cp_xyz, const int64_t* ku_off,
                    const double* ku, const int64_t* kv_off, const double* kv, double tol_rel, int n_threads,
                    SurfPlan& plan, std::string& err);
void bernstein_matrix(int p, double* B);      // (p+1)^2, power coeffs of each Bernstein function
void bernstein_inverse(int p, double* Bi);    // power -> Bernstein
void subdivision_matrix(int p, double z, double* S);
void gram_matrix(int m, int n, double* G);
uint16_t f32_to_bf16_rne(float x);

// Byte offsets of a curve geometry with these counts (general = 0).
void curve_layout(GeomLayout& L, int64_t n_curves, int64_t n_seg, int64_t n_span, int64_t n_coef, int64_t n_clu);
void set_error(const std::string& msg);

}  // namespace mrep
