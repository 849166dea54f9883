// Device-side views shared by the HIP translation units of libmrep.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mrep.h"
#include "mrep_internal.h"

namespace mrep {

struct PairRes;  // one (query, piece) refine result (mrep_refine.h)

// ---------------------------------------------------------------------------
// device views
// ---------------------------------------------------------------------------
struct DevGeom {
    const DCurve* curves;
    const uint16_t* col;
    const float* aux;
    const float* lcp;
    const double* gcp;
    const double* segt;
    const int32_t* segspan;
    const double* spant;
    const int32_t* span0;
    const double* coef;
    const float4* sph;   // piece spheres
    const float4* csph;  // cluster spheres
    int32_t n_curves;
    int64_t n_seg;
    int32_t general;  // spans beyond the power form present (degree > MREP_POWER_MAX_DEGREE or rational)
};

inline DevGeom dev_view(const Geom& g)
{
    DevGeom d;
    d.curves = reinterpret_cast<const DCurve*>(g.base + g.L.off_curve);
    d.col = reinterpret_cast<const uint16_t*>(g.base + g.L.off_col);
    d.aux = reinterpret_cast<const float*>(g.base + g.L.off_aux);
    d.lcp = reinterpret_cast<const float*>(g.base + g.L.off_lcp);
    d.gcp = reinterpret_cast<const double*>(g.base + g.L.off_gcp);
    d.segt = reinterpret_cast<const double*>(g.base + g.L.off_segt);
    d.segspan = reinterpret_cast<const int32_t*>(g.base + g.L.off_segspan);
    d.spant = reinterpret_cast<const double*>(g.base + g.L.off_spant);
    d.span0 = reinterpret_cast<const int32_t*>(g.base + g.L.off_span0);
    d.coef = reinterpret_cast<const double*>(g.base + g.L.off_coef);
    d.sph = reinterpret_cast<const float4*>(g.base + g.L.off_sph);
    d.csph = reinterpret_cast<const float4*>(g.base + g.L.off_csph);
    d.n_curves = (int32_t)g.L.n_curves;
    d.n_seg = g.L.n_seg;
    d.general = g.L.general;
    return d;
}


// Outputs of the screen, per sorted query position j and per reserved
// (query, piece) pair p.  A workgroup reserves one contiguous block of pairs.
struct ScreenOut {
    int32_t* cand_n;      // [n] candidates of query j, or -1 when the list overflowed
    int32_t* pair_off;    // [n] first pair of query j
    int32_t* pair_seg;    // [cap] global piece index of pair p
    int32_t* pair_j;      // [cap] sorted query position of pair p
    int32_t* pair_count;  // pairs reserved so far (zero before the screen)
    int64_t pair_cap;     // capacity of the pair arrays; beyond it a query overflows
    float* ub;            // [n] a certified upper bound of query j's distance (the full scan starts from it)
};

// Launch the BF16 MFMA screen (mrep_screen.hip): one workgroup per tile of
// kQueriesPerTile queries of one curve, workgroup b taking tile_map[b];
// grid = screen_grid(n_curves, n).
hipError_t launch_screen_bf16(const DevGeom& G, int64_t grid, const int4* tile_map, const int32_t* perm,
                              const double* qxyz, int32_t kc, const ScreenOut& out, hipStream_t st);
// workgroup slots of a tiled launch over n queries in n_groups groups: an upper
// bound of the tile count plus room for the per-XCD rounding
inline int64_t screen_grid(int64_t n_groups, int64_t n)
{
    return n_groups + (n + kQueriesPerTile - 1) / kQueriesPerTile + kXcdCount;
}
// k_tile_map: slot -> {group, first sorted query, end of the group's queries, tile}
hipError_t launch_tile_map(const int32_t* tile_off, const int32_t* q_off, int64_t n_groups, int64_t grid,
                           int4* map, hipStream_t st);

// Output arrays of a projection call (indexed by the caller's query index).
struct Outs {
    double* t;
    double* d;
    int32_t* s;
    uint32_t* f;
};

// Shared host helpers (mrep_device.hip).
int check_device();
int check_opts(const mrep_opts* o);
// Stage timing of the calling thread: stage_begin records event 0, stage_mark(i)
// event i, stage_end(count) publishes the call's stage count.
int stage_begin(hipStream_t st);
int stage_mark(int i, hipStream_t st);
void stage_end(int count);

// Group n queries by curve (n_dev, nullable: actual count on the device):
// hist[n_curves + 2] zeroed and counted, q_off / tile_off exclusive scans,
// perm[sorted position] = query index.  Invalid ids get NaN / -1 /
// MREP_F_BAD_ID outputs when o.t is not null.
hipError_t launch_grouping(int64_t n_curves, int64_t n, const int32_t* n_dev, const int32_t* curve_id,
                           int32_t* hist, int32_t* q_off, int32_t* tile_off, int32_t* perm, const Outs& o,
                           hipStream_t st);

// Refine, finish and full-scan fallback over candidate pairs in ScreenOut form
// (k_pairs, k_finish, k_fullscan in FP32); pairs_mark >= 0 records that stage
// event after the pair refine.  n bounds the sorted query count;
// done (nullable) skips decided queries; flag_in is ORed into every flag word
// written; the overflow counter *ovf_count must be zero on entry.
hipError_t launch_refine(const DevGeom& G, int64_t n, const int32_t* curve_id, const double* q_xyz,
                         const int32_t* q_off, const int32_t* perm, const ScreenOut& so, PairRes* pair_res,
                         const uint8_t* done, uint32_t flag_in, double tie_rel, int invert, int32_t* ovf_list,
                         int32_t* ovf_count, const Outs& o, hipStream_t st, bool clip = false,
                         int pairs_mark = -1);
// k_pairs_clip (mrep_clip.hip): the paper's refinement path on every candidate pair
hipError_t launch_pairs_clip(const DevGeom& G, const int32_t* curve_id, const double* q_xyz, const int32_t* perm,
                             const ScreenOut& so, const uint8_t* done, PairRes* pair_res, hipStream_t st);

// The screened projection pipeline (grouping, screen, refine, finish) on a
// workspace of project_ws_bytes(n_curves, n, kc) bytes.  n bounds the query
// count; n_dev (nullable) holds the actual count on the device.  With timed,
// stage marks stage0 + 1 .. stage0 + 4 are recorded after grouping, screen,
// pair refine and finish.
int64_t project_ws_bytes(int64_t n_curves, int64_t n, int kc);
int project_core(const Geom& geom, const mrep_opts* opts, int64_t n, const int32_t* n_dev, const int32_t* curve_id,
                 const double* q_xyz, void* workspace, const Outs& o, hipStream_t st, int invert, bool timed,
                 int stage0);

// Network kind of a handle (-1 for NULL), and the fused inference kernel over
// the (sorted query, candidate patch) rows of a surface call: xb[n][4][64] BF16
// inputs, cand[n][4] global patch (or -1), out[n][4] = (s, t, logit, 0).
int nn_kind(const mrep_nn* nn);
int nn_score_surface_pairs(const mrep_nn* nn, const int32_t* q_off, int32_t n_surf, const int32_t* cand,
                           const uint16_t* xb, float4* out, int64_t n_rows, hipStream_t st);

}  // namespace mrep

namespace mrep {
// Result of the device decomposition (mrep_ddecomp.hip): device arrays owned by
// its plan; the geometry tables are built from them by mrep_upload.
struct DevPlan;
void devplan_free(DevPlan* d);
int devplan_upload(const DevPlan& d, char* buf, hipStream_t st);
int devplan_export(const DevPlan& d, int64_t* seg_off, double* seg_t, double* seg_cp, int32_t* seg_span);
const GeomLayout& devplan_layout(const DevPlan& d);
int32_t devplan_max_degree(const DevPlan& d);
double devplan_tol_rel(const DevPlan& d);
}  // namespace mrep

// Handles of the C ABI.  A plan (host tables, or device arrays for a device
// decomposition) and a geometry (non-owning device view of the caller's
// buffer) hold either curves or surfaces.
enum { MREP_GEOM_CURVES = 0, MREP_GEOM_SURFACES = 1 };
struct mrep_plan {
    int kind = MREP_GEOM_CURVES;
    mrep::Plan p;
    mrep::SurfPlan sp;
    mrep::DevPlan* dev = nullptr;  // set by mrep_decompose_curves_device
    ~mrep_plan() { mrep::devplan_free(dev); }
};
struct mrep_geom {
    int kind = MREP_GEOM_CURVES;
    int strategy = MREP_STRATEGY_SCREEN;  // chosen by mrep_tune_curves
    int box_lanes = 8;                    // schedule of the sphere-list kernel: lanes per query (4, 8, 16)
    int box_persist = 0;                  // 1: persistent grid over per-XCD tile queues, 0: tile map
    double box_ms[MREP_N_BOX_SCHEDULES] = {};  // the last tune's time of each schedule (ms)
    mrep::Geom g;
    mrep::SurfGeom sg;
};

namespace mrep {
// schedule s of the sphere-list kernel: 4 << (s % 3) lanes per query, persistent grid when s >= 3
inline void box_schedule(int s, int* lanes, int* persist)
{
    *lanes = 4 << (s % 3);
    *persist = s / 3;
}
// the seeded / sphere-pruned curve projection (nn == NULL: sphere-pruned)
int seeded_core(const char* fn, const mrep_geom* geom, const mrep_nn* nn, const mrep_opts* opts, int64_t n,
                const int32_t* curve_id, const double* q_xyz, void* workspace, int64_t ws_bytes, double* t_out,
                double* dist_out, int32_t* seg_out, uint32_t* flags_out, void* stream, int invert);
int64_t seeded_ws_bytes(const mrep_geom* geom, int64_t n);
}  // namespace mrep
