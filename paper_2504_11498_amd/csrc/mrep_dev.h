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
    return d;
}


// Launch the BF16 MFMA screen (mrep_screen.hip): one workgroup per tile of
// kQueriesPerTile queries of one curve; grid = n_curves + ceil(n / tile).
hipError_t launch_screen_bf16(const DevGeom& G, int64_t grid, const int32_t* tile_off, const int32_t* q_off,
                              const int32_t* perm, const double* qxyz, int32_t kc, int32_t* cand, int32_t* cand_n,
                              float* ub_out, hipStream_t st);

}  // namespace mrep
