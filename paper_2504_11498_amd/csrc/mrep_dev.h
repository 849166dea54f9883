// Device-side views shared by the HIP translation units of libmrep.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mrep_internal.h"

namespace mrep {

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
    int32_t n_curves;
    int64_t n_seg;
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
    d.n_curves = (int32_t)g.L.n_curves;
    d.n_seg = g.L.n_seg;
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
    float* ub;            // [n] the certified upper bound of query j (diagnostic)
};

// Launch the BF16 MFMA screen (mrep_screen.hip): one workgroup per tile of
// kQueriesPerTile queries of one curve; grid = n_curves + ceil(n / tile).
hipError_t launch_screen_bf16(const DevGeom& G, int64_t grid, const int32_t* tile_off, const int32_t* q_off,
                              const int32_t* perm, const double* qxyz, int32_t kc, const ScreenOut& out,
                              hipStream_t st);

}  // namespace mrep
