// Surface projection and inversion on gfx950: tensor-product B-spline surfaces
// decomposed (host, FP64) into bicubic Bezier patches, the surface case of the
// paper's matrix representation (Sec. 5.2.1 applied in u and in v).
//
// Pipeline for n queries, each onto its own surface:
//   1. group queries by surface (counting sort, shared with the curve path);
//   2. per query (one kernel): every patch lies in a sphere (centre, radius
//      bound incl. its deviation from the exact surface); the patches whose
//      lower bound |q - c| - r reaches the best upper bound |q - c| + r plus
//      the tie margin are listed, a 4 x 4 sample bound of each listed patch
//      (second-order, min(samples) - (M_ss + M_tt) / 72) is taken, the best
//      sample lowers the query's bound, and the patches whose sampled bound
//      still reaches it form the query's (query, patch) pairs;
//   3. per pair, the certified minimum of |S(s,t) - q|^2 over the patch in
//      FP32, capped at the query's bound plus the tie margin: a 7 x 7 sample
//      grid, box-constrained Newton on the stationarity conditions
//      (S - q).S_s = (S - q).S_t = 0 from its local minima, the four edge
//      curves by the curve path's certified 1D minimum, and a Newton solve in
//      every grid cell whose second-order lower bound
//      min(corner f) - (M_ss h^2 + M_tt h^2) / 8 still beats the best;
//   4. per query, the two best pairs; FP64 box-constrained Newton on the EXACT
//      span patch (power form of degree (p, q)) from the best, continuing into
//      a neighbouring span patch when the minimiser sits on a shared edge with
//      the gradient pointing across, and from the runner-up when it is within
//      the tie margin; write (u, v), distance, patch index and flags.
// Queries whose list overflows take a wave-per-query scan of all their patches.
//
// Seeded calls (learned seeding, an extension): a first sweep keeps each
// query's 4 patches with the smallest sphere lower bounds and writes their
// network inputs; the surface network scores them; Newton from the predicted
// (s, t) on the best-scored patch attains a first bound, which replaces the
// sphere upper bound of step 2; the rest of the pipeline is unchanged, so the
// answer is the certified global minimum whatever the network predicts.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "../../include/mrep.h"
#include "mrep_dev.h"
#include "mrep_refine.h"

using namespace mrep;

namespace {

constexpr int kSphSub = 8;
constexpr int kSphThreads = kQueriesPerTile * kSphSub;
// 192 listed patches per query keep the list kernel at 53 KB of LDS, 3
// workgroups per CU: on the batched surfaces the list stage takes 43 ms
// against 63 ms with 256 (2 workgroups), for 1.8% instead of 1.3% of the
// queries sent to the full scan; 160 sends 2.5% and is slower overall.
#ifndef MREP_SPH_CAP
#define MREP_SPH_CAP 192
#endif
constexpr int kSphCap = MREP_SPH_CAP;    // listed patches per query; more: the full scan
constexpr int kCluChunk = 8 * kSphCap;  // cluster spheres staged per round (shares LDS with the lists' bounds)
constexpr int kCluCap = 64;     // candidate clusters per query; more: the full scan
constexpr int kXcds = 8;
constexpr int64_t kSurfPairsPerQuery = 96;
constexpr int kGrid = 7;  // samples per direction in a patch
constexpr int kK = MREP_NN_K;  // candidate patches scored per query (seeded calls)
constexpr int kFeat = MREP_NN_SURFACE_IN;
static_assert(kSphThreads == 256, "sphere kernels: 32 queries x 8 lanes");
static_assert(sizeof(float4) * kCluChunk == sizeof(float) * kQueriesPerTile * kSphCap, "list kernel LDS union");

struct DevSurf {
    const DSurf* surfs;
    const float4* sph;
    const float* lcp;
    const double* gcp;
    const double* uv;
    const int32_t* pspan;
    const int32_t* span0;
    const float4* csph;
    const double* brk;
    const double* coef;
    int32_t n_surf;
    int64_t n_patch;
};

DevSurf surf_view(const SurfGeom& g)
{
    DevSurf d;
    d.surfs = reinterpret_cast<const DSurf*>(g.base + g.L.off_surf);
    d.sph = reinterpret_cast<const float4*>(g.base + g.L.off_sph);
    d.lcp = reinterpret_cast<const float*>(g.base + g.L.off_lcp);
    d.gcp = reinterpret_cast<const double*>(g.base + g.L.off_gcp);
    d.uv = reinterpret_cast<const double*>(g.base + g.L.off_uv);
    d.pspan = reinterpret_cast<const int32_t*>(g.base + g.L.off_pspan);
    d.span0 = reinterpret_cast<const int32_t*>(g.base + g.L.off_span0);
    d.csph = reinterpret_cast<const float4*>(g.base + g.L.off_csph);
    d.brk = reinterpret_cast<const double*>(g.base + g.L.off_brk);
    d.coef = reinterpret_cast<const double*>(g.base + g.L.off_coef);
    d.n_surf = (int32_t)g.L.n_surf;
    d.n_patch = g.L.n_patch;
    return d;
}

__device__ __forceinline__ float s_margin(float d, const DSurf& sf, float tie_rel)
{
    return 2.f * (float)sf.tol_eff + 4e-6f * (d + (float)sf.diag) + tie_rel * (float)sf.diag;
}

// ---------------------------------------------------------------------------
// 2. sphere candidate lists
// ---------------------------------------------------------------------------
// Seeded calls: candidate patches and their network inputs
struct SphTop {
    int32_t* cand;  // [n][kK] global patch index (-1: fewer patches)
    uint16_t* xb;   // [n][kK][64] BF16 network inputs (null: not written)
};

// float -> uint32 with the same order (negative values included)
__device__ __forceinline__ uint32_t ord_key(float x)
{
    const uint32_t b = __float_as_uint(x);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ord_val(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
__device__ __forceinline__ void cswap(uint64_t& a, uint64_t& b)
{
    const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    a = lo;
    b = hi;
}

// Network inputs of a (query, patch) pair: the 16 control points (row-major,
// i along u) and the query, minus the control points' centroid, over the
// diagonal of their box.
__device__ __forceinline__ void patch_features(const DevSurf& D, const DSurf& sf, int64_t k, const double* q,
                                               float* x)
{
    const float* lp = D.lcp + k * 48;
    const float4 c = D.sph[k];
    const float ql[3] = {(float)(q[0] - (sf.origin[0] + (double)c.x)), (float)(q[1] - (sf.origin[1] + (double)c.y)),
                         (float)(q[2] - (sf.origin[2] + (double)c.z))};
    float m[3], ext2 = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float sum = 0.f, lo = INFINITY, hi = -INFINITY;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float v = lp[3 * i + a];
            sum += v;
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
        m[a] = sum * (1.f / 16.f);
        ext2 += (hi - lo) * (hi - lo);
    }
    const float inv = ext2 > 0.f ? 1.f / sqrtf(ext2) : 1.f;
#pragma unroll
    for (int i = 0; i < 16; ++i)
#pragma unroll
        for (int a = 0; a < 3; ++a) x[3 * i + a] = (lp[3 * i + a] - m[a]) * inv;
#pragma unroll
    for (int a = 0; a < 3; ++a) x[48 + a] = (ql[a] - m[a]) * inv;
}

// ---------------------------------------------------------------------------
// Two-level sphere sweeps.  The exact spans of a surface are grouped into
// clusters (blocks of clu_bs x clu_bs spans, about 32 patches), each with a
// sphere around its patches' spheres, so for a query q and any patch p of
// cluster C
//     |q - c_p| - r_p >= |q - c_C| - r_C    and    |q - c_p| + r_p <= |q - c_C| + r_C.
// A query's 8 lanes test the surface's cluster spheres (staged in LDS) and then
// only the patches of the clusters whose lower bound reaches the threshold
// (read from global memory; one row of a cluster's spans holds contiguous
// patches).
// ---------------------------------------------------------------------------
// one staging round of cluster spheres; all threads of the block call it
__device__ __forceinline__ void stage_clusters(const DevSurf& D, const DSurf& sf, int c0, int cn, float4* st)
{
    __syncthreads();
    for (int i = threadIdx.x; i < cn; i += kSphThreads) st[i] = D.csph[sf.clu_off + c0 + i];
    __syncthreads();
}

// span rows of cluster c: rows iu in [iu0, iu1), each the patches
// [span0[r + iv0], span0[r + iv1]) with r = span_off + iu * n_sv
struct CluRows {
    int iu0, iu1, iv0, iv1;
};
__device__ __forceinline__ CluRows clu_rows(const DSurf& sf, int c)
{
    const int bs = sf.clu_bs, bu = c / sf.n_cbv, bv = c % sf.n_cbv;
    return CluRows{bu * bs, min(sf.n_su, bu * bs + bs), bv * bs, min(sf.n_sv, bv * bs + bs)};
}

// min over the patches of cluster c of |q - c_p| + r_p + eps (per lane)
constexpr int kBatch = 4;  // patch spheres a lane loads at once

// ... also keeping this lane's patch with the nearest centre (bd, bk: its
// centre distance and global index; ties to the lower index)
__device__ __forceinline__ float clu_patch_ub(const DevSurf& D, const DSurf& sf, int c, const float* ql, float eps,
                                              int sub, float ub, float& bd, int& bk)
{
    const CluRows R = clu_rows(sf, c);
    for (int iu = R.iu0; iu < R.iu1; ++iu) {
        const int64_t rs = sf.span_off + (int64_t)iu * sf.n_sv;
        const int k1 = D.span0[rs + R.iv1];
        // kBatch patches per lane loaded together, so that their latencies overlap
        for (int k = D.span0[rs + R.iv0] + sub; k < k1; k += kBatch * kSphSub) {
            float4 p[kBatch];
#pragma unroll
            for (int r = 0; r < kBatch; ++r)
                p[r] = k + r * kSphSub < k1 ? D.sph[k + r * kSphSub] : make_float4(0.f, 0.f, 0.f, INFINITY);
#pragma unroll
            for (int r = 0; r < kBatch; ++r) {
                const float dx = ql[0] - p[r].x, dy = ql[1] - p[r].y, dz = ql[2] - p[r].z;
                // the raw square root (<= 1 ulp) is inside the allowance eps
                const float d = __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz);
                ub = fminf(ub, d + p[r].w + eps);
                const int kk = k + r * kSphSub;
                if (kk < k1 && (d < bd || (d == bd && kk < bk))) {
                    bd = d;
                    bk = kk;
                }
            }
        }
    }
    return ub;
}

// An upper bound from points of the patch with the nearest centre among the
// query's 8 lanes' candidates (bd, bk; ties to the lower index): lanes 0..3
// take its corner control points, which are points of its FP32 Bezier form,
// lane 4 its centre B(1/2, 1/2); plus the patch's deviation bound tol_eff and
// 4e-6 r for the FP32 net and the evaluation.  INFINITY in the other lanes.
__device__ __forceinline__ float patch_point_bound(const DevSurf& D, const DSurf& sf, float bd, int bk, int sub,
                                                   bool active, const float* ql, float eps)
{
#pragma unroll
    for (int off = 1; off < kSphSub; off <<= 1) {
        const float od = __shfl_xor(bd, off, 64);
        const int ok = __shfl_xor(bk, off, 64);
        const bool take = od < bd || (od == bd && (unsigned)ok < (unsigned)bk);
        bk = take ? ok : bk;
        bd = take ? od : bd;
    }
    if (!active || bk < 0 || sub > 4) return INFINITY;
    const float4* lp = reinterpret_cast<const float4*>(D.lcp + (int64_t)bk * 48);
    const float4 c = D.sph[bk];
    float px, py, pz;
    if (sub < 4) {
        // P00 = lcp[0..2], P03 = lcp[9..11], P30 = lcp[36..38], P33 = lcp[45..47]
        const float4 v = lp[sub == 0 ? 0 : (sub == 1 ? 2 : (sub == 2 ? 9 : 11))];
        const bool hi = sub == 1 || sub == 3;
        px = hi ? v.y : v.x;
        py = hi ? v.z : v.y;
        pz = hi ? v.w : v.z;
    } else {
        const float w[4] = {0.125f, 0.375f, 0.375f, 0.125f};
        const float* l = D.lcp + (int64_t)bk * 48;
        px = py = pz = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float wij = w[i] * w[j];
                px += wij * l[3 * (4 * i + j)];
                py += wij * l[3 * (4 * i + j) + 1];
                pz += wij * l[3 * (4 * i + j) + 2];
            }
    }
    const float dx = ql[0] - (c.x + px), dy = ql[1] - (c.y + py), dz = ql[2] - (c.z + pz);
    return __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz) + 1.0001f * (float)sf.tol_eff + 4e-6f * c.w + eps;
}

// A first bound on the distance: min over clusters of |q - c_C| + r_C + eps,
// and over the patches of the kK clusters with the smallest lower bounds
// |q - c_C| - r_C of |q - c_p| + r_p + eps (same value in the query's 8 lanes).
__device__ float first_ub(const DevSurf& D, const DSurf& sf, float4* st, const float* ql, float eps, bool active,
                          int sub)
{
    float ub = INFINITY;
    uint64_t key[kK];  // (ordered lower bound, local cluster), sorted
#pragma unroll
    for (int k = 0; k < kK; ++k) key[k] = ~0ull;
    for (int c0 = 0; c0 < sf.n_clu; c0 += kCluChunk) {
        const int cn = min(kCluChunk, sf.n_clu - c0);
        stage_clusters(D, sf, c0, cn, st);
        if (!active) continue;
        for (int i = sub; i < cn; i += kSphSub) {
            const float4 p = st[i];
            const float dx = ql[0] - p.x, dy = ql[1] - p.y, dz = ql[2] - p.z;
            const float d = sqrtf(dx * dx + dy * dy + dz * dz);
            ub = fminf(ub, d + p.w + eps);
            uint64_t x = ((uint64_t)ord_key(d - p.w) << 32) | (uint32_t)(c0 + i);
            if (x < key[kK - 1]) {
#pragma unroll
                for (int k = 0; k < kK; ++k) cswap(key[k], x);
            }
        }
    }
#pragma unroll
    for (int off = 1; off < kSphSub; off <<= 1) {
        uint64_t o[kK];
#pragma unroll
        for (int k = 0; k < kK; ++k) o[k] = __shfl_xor(key[k], off, 64);
#pragma unroll
        for (int k = 0; k < kK; ++k) key[k] = min(key[k], o[kK - 1 - k]);
        cswap(key[0], key[2]);
        cswap(key[1], key[3]);
        cswap(key[0], key[1]);
        cswap(key[2], key[3]);
    }
    float bd = INFINITY;
    int bk = -1;
    if (active) {
#pragma unroll
        for (int m = 0; m < kK; ++m)
            if (key[m] != ~0ull) ub = clu_patch_ub(D, sf, (int)(uint32_t)key[m], ql, eps, sub, ub, bd, bk);
    }
    ub = fminf(ub, patch_point_bound(D, sf, bd, bk, sub, active, ql, eps));
#pragma unroll
    for (int off = 1; off < kSphSub; off <<= 1) ub = fminf(ub, __shfl_xor(ub, off, 64));
    return ub;
}

// clusters whose lower bound |q - c_C| - r_C - eps reaches thr, in index
// order, into list[0..kCluCap) as local indices; returns their count (more
// than kCluCap: overflow)
__device__ int clu_list(const DevSurf& D, const DSurf& sf, float4* st, const float* ql, float eps, float thr,
                        bool active, int lane, int sub, uint16_t* list)
{
    int cnt = 0;
    for (int c0 = 0; c0 < sf.n_clu; c0 += kCluChunk) {
        const int cn = min(kCluChunk, sf.n_clu - c0);
        stage_clusters(D, sf, c0, cn, st);
        if (!active) continue;
        // the 8 lanes of a query run the same trip count: the ballot sees all of them
        for (int i0 = 0; i0 < cn; i0 += kSphSub) {
            const int i = i0 + sub;
            bool hit = false;
            if (i < cn) {
                const float4 p = st[i];
                const float dx = ql[0] - p.x, dy = ql[1] - p.y, dz = ql[2] - p.z;
                const float tt = thr + p.w + eps;
                hit = tt >= 0.f && dx * dx + dy * dy + dz * dz <= tt * tt;
            }
            const uint32_t grp = (uint32_t)(__ballot(hit) >> (lane & 56)) & 0xffu;
            const int pos = cnt + __popc(grp & ((1u << sub) - 1u));
            if (hit && pos < kCluCap) list[pos] = (uint16_t)(c0 + i);  // a surface has < 65536 clusters
            cnt += __popc(grp);
        }
    }
    return cnt;
}

// Candidates of the seeded calls: per query, the kK patches with the smallest
// sphere lower bounds (ties to the lower index) among the clusters whose bound
// reaches the first bound plus the tie margin, their network inputs (BF16
// rows of 64, when top.xb is set) and the best patch sphere upper bound
// so.ub.  One workgroup per tile of kQueriesPerTile queries of one surface, 8
// lanes per query.  A query with more than kCluCap such clusters gets so.ub =
// +inf and candidates from the first kCluCap only.
__global__ __launch_bounds__(kSphThreads) void k_scand(DevSurf D, const int32_t* __restrict__ tile_off,
                                                       const int32_t* __restrict__ q_off,
                                                       const int32_t* __restrict__ perm,
                                                       const double* __restrict__ qxyz, float tie_rel, ScreenOut so,
                                                       SphTop top)
{
    __shared__ float4 s_st[kCluChunk];
    __shared__ uint16_t s_clu[kQueriesPerTile][kCluCap];
    const int n_tiles = tile_off[D.n_surf];
    const int per = (n_tiles + kXcds - 1) / kXcds;
    const int slot = (int)(blockIdx.x / kXcds);
    const int tile = (int)(blockIdx.x % kXcds) * per + slot;
    if (slot >= per || tile >= n_tiles) return;
    int lo_c = 0, hi_c = D.n_surf;
    while (hi_c - lo_c > 1) {
        const int mid = (lo_c + hi_c) >> 1;
        if (tile_off[mid] <= tile) lo_c = mid; else hi_c = mid;
    }
    const DSurf sf = D.surfs[lo_c];
    const int lane = threadIdx.x & 63;
    const int qs = threadIdx.x / kSphSub, sub = threadIdx.x % kSphSub;
    const int64_t j = (int64_t)q_off[lo_c] + (int64_t)(tile - tile_off[lo_c]) * kQueriesPerTile + qs;
    const bool active = j < q_off[lo_c + 1];
    float ql[3] = {0.f, 0.f, 0.f};
    if (active) {
        const int32_t qi = perm[j];
#pragma unroll
        for (int k = 0; k < 3; ++k) ql[k] = (float)(qxyz[3 * (int64_t)qi + k] - sf.origin[k]);
    }
    const float eps = 1e-6f * (sqrtf(ql[0] * ql[0] + ql[1] * ql[1] + ql[2] * ql[2]) + (float)sf.diag);
    const float ubs = first_ub(D, sf, s_st, ql, eps, active, sub);
    const float thr0 = ubs + s_margin(ubs, sf, tie_rel);
    const int ns = clu_list(D, sf, s_st, ql, eps, thr0, active, lane, sub, s_clu[qs]);
    float ub = INFINITY;
    uint64_t key[kK];
#pragma unroll
    for (int k = 0; k < kK; ++k) key[k] = ~0ull;
    if (active) {
        for (int m = 0; m < min(ns, kCluCap); ++m) {
            const CluRows R = clu_rows(sf, s_clu[qs][m]);
            for (int iu = R.iu0; iu < R.iu1; ++iu) {
                const int64_t rs = sf.span_off + (int64_t)iu * sf.n_sv;
                const int k1 = D.span0[rs + R.iv1];
                for (int k = D.span0[rs + R.iv0] + sub; k < k1; k += kSphSub) {
                    const float4 p = D.sph[k];
                    const float dx = ql[0] - p.x, dy = ql[1] - p.y, dz = ql[2] - p.z;
                    const float d = sqrtf(dx * dx + dy * dy + dz * dz);
                    const float re = p.w + eps;
                    ub = fminf(ub, d + re);
                    uint64_t x = ((uint64_t)ord_key(d - re) << 32) | (uint32_t)(k - sf.patch_off);
                    if (x < key[kK - 1]) {
#pragma unroll
                        for (int t = 0; t < kK; ++t) cswap(key[t], x);  // insertion into the sorted list
                    }
                }
            }
        }
    }
    // merge the lanes' sorted lists: exchange, keep the smaller half (bitonic)
#pragma unroll
    for (int off = 1; off < kSphSub; off <<= 1) {
        ub = fminf(ub, __shfl_xor(ub, off, 64));
        uint64_t o[kK];
#pragma unroll
        for (int k = 0; k < kK; ++k) o[k] = __shfl_xor(key[k], off, 64);
#pragma unroll
        for (int k = 0; k < kK; ++k) key[k] = min(key[k], o[kK - 1 - k]);
        cswap(key[0], key[2]);
        cswap(key[1], key[3]);
        cswap(key[0], key[1]);
        cswap(key[2], key[3]);
    }
    if (!active) return;
    if (sub == 0) so.ub[j] = ns <= kCluCap ? ub : INFINITY;
    if (sub < kK) {
        const uint64_t kk = sub == 0 ? key[0] : (sub == 1 ? key[1] : (sub == 2 ? key[2] : key[3]));
        const int64_t g = kk == ~0ull ? -1 : sf.patch_off + (int64_t)(uint32_t)kk;
        top.cand[j * kK + sub] = (int32_t)g;
        if (top.xb) {
            float f[kFeat];
#pragma unroll
            for (int k = 0; k < kFeat; ++k) f[k] = 0.f;
            if (g >= 0) {
                const int32_t qi = perm[j];
                const double q[3] = {qxyz[3 * (int64_t)qi], qxyz[3 * (int64_t)qi + 1], qxyz[3 * (int64_t)qi + 2]};
                patch_features(D, sf, g, q, f);
            }
            uint4* dst = reinterpret_cast<uint4*>(top.xb + (j * kK + sub) * 64);
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                uint32_t w[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k0 = 8 * c + 2 * e;
                    const uint16_t lo = k0 < kFeat ? __builtin_bit_cast(uint16_t, (__bf16)f[k0]) : (uint16_t)0;
                    const uint16_t hi = k0 + 1 < kFeat ? __builtin_bit_cast(uint16_t, (__bf16)f[k0 + 1]) : (uint16_t)0;
                    w[e] = (uint32_t)lo | ((uint32_t)hi << 16);
                }
                dst[c] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 3. certified minimum of one bicubic patch (FP32, local frame)
// ---------------------------------------------------------------------------
// Power form relative to the query: S(s,t) - q = sum_{a,b} C[a][b] s^a t^b.
struct Bicubic {
    float C[4][4][3];
    float Ls, Lt, Lss, Ltt, far;  // |S_s|, |S_t|, |S_ss|, |S_tt| bounds; max |P - q|
};

__device__ __forceinline__ void load_bicubic(const DevSurf& D, const DSurf& sf, int64_t k, const double* q, Bicubic& B)
{
    const float* lp = D.lcp + k * 48;
    const float4 c = D.sph[k];
    const float ql[3] = {(float)(q[0] - (sf.origin[0] + (double)c.x)), (float)(q[1] - (sf.origin[1] + (double)c.y)),
                         (float)(q[2] - (sf.origin[2] + (double)c.z))};
    float P[4][4][3];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int x = 0; x < 3; ++x) P[i][j][x] = lp[3 * (4 * i + j) + x] - ql[x];
    // hodograph bounds
    float ls = 0.f, lt = 0.f, lss = 0.f, ltt = 0.f, far = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            far = fmaxf(far, P[i][j][0] * P[i][j][0] + P[i][j][1] * P[i][j][1] + P[i][j][2] * P[i][j][2]);
            if (i < 3) {
                const float a = P[i + 1][j][0] - P[i][j][0], b = P[i + 1][j][1] - P[i][j][1], e = P[i + 1][j][2] - P[i][j][2];
                ls = fmaxf(ls, a * a + b * b + e * e);
            }
            if (j < 3) {
                const float a = P[i][j + 1][0] - P[i][j][0], b = P[i][j + 1][1] - P[i][j][1], e = P[i][j + 1][2] - P[i][j][2];
                lt = fmaxf(lt, a * a + b * b + e * e);
            }
            if (i < 2) {
                const float a = P[i + 2][j][0] - 2.f * P[i + 1][j][0] + P[i][j][0];
                const float b = P[i + 2][j][1] - 2.f * P[i + 1][j][1] + P[i][j][1];
                const float e = P[i + 2][j][2] - 2.f * P[i + 1][j][2] + P[i][j][2];
                lss = fmaxf(lss, a * a + b * b + e * e);
            }
            if (j < 2) {
                const float a = P[i][j + 2][0] - 2.f * P[i][j + 1][0] + P[i][j][0];
                const float b = P[i][j + 2][1] - 2.f * P[i][j + 1][1] + P[i][j][1];
                const float e = P[i][j + 2][2] - 2.f * P[i][j + 1][2] + P[i][j][2];
                ltt = fmaxf(ltt, a * a + b * b + e * e);
            }
        }
    B.Ls = 3.f * sqrtf(ls);
    B.Lt = 3.f * sqrtf(lt);
    B.Lss = 6.f * sqrtf(lss);
    B.Ltt = 6.f * sqrtf(ltt);
    B.far = sqrtf(far);
    // Bernstein -> power in each direction: rows of M are (1,0,0,0) (-3,3,0,0) (3,-6,3,0) (-1,3,-3,1)
    const float M[4][4] = {{1.f, 0.f, 0.f, 0.f}, {-3.f, 3.f, 0.f, 0.f}, {3.f, -6.f, 3.f, 0.f}, {-1.f, 3.f, -3.f, 1.f}};
    float T[4][4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                float s = 0.f;
#pragma unroll
                for (int i = 0; i < 4; ++i) s += M[a][i] * P[i][j][x];
                T[a][j][x] = s;
            }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                float s = 0.f;
#pragma unroll
                for (int j = 0; j < 4; ++j) s += M[b][j] * T[a][j][x];
                B.C[a][b][x] = s;
            }
}

__device__ __forceinline__ float bc_f(const Bicubic& B, float s, float t)
{
    float r = 0.f;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        float acc = 0.f;
#pragma unroll
        for (int a = 3; a >= 0; --a) {
            const float d = B.C[a][0][x] + t * (B.C[a][1][x] + t * (B.C[a][2][x] + t * B.C[a][3][x]));
            acc = acc * s + d;
        }
        r += acc * acc;
    }
    return r;
}

// value, gradient of f/2 = (S-q).S_s, (S-q).S_t, Hessian of f/2, metric
struct BcEval {
    float f, gs, gt, h11, h12, h22, g11, g12, g22;
};

__device__ __forceinline__ BcEval bc_eval(const Bicubic& B, float s, float t)
{
    float r[3], Ss[3], St[3], Sss[3], Sst[3], Stt[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        float D[4], D1[4], D2[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            D[a] = B.C[a][0][x] + t * (B.C[a][1][x] + t * (B.C[a][2][x] + t * B.C[a][3][x]));
            D1[a] = B.C[a][1][x] + t * (2.f * B.C[a][2][x] + t * 3.f * B.C[a][3][x]);
            D2[a] = 2.f * B.C[a][2][x] + t * 6.f * B.C[a][3][x];
        }
        r[x] = D[0] + s * (D[1] + s * (D[2] + s * D[3]));
        Ss[x] = D[1] + s * (2.f * D[2] + s * 3.f * D[3]);
        Sss[x] = 2.f * D[2] + s * 6.f * D[3];
        St[x] = D1[0] + s * (D1[1] + s * (D1[2] + s * D1[3]));
        Sst[x] = D1[1] + s * (2.f * D1[2] + s * 3.f * D1[3]);
        Stt[x] = D2[0] + s * (D2[1] + s * (D2[2] + s * D2[3]));
    }
    BcEval e;
    e.f = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    e.gs = r[0] * Ss[0] + r[1] * Ss[1] + r[2] * Ss[2];
    e.gt = r[0] * St[0] + r[1] * St[1] + r[2] * St[2];
    e.g11 = Ss[0] * Ss[0] + Ss[1] * Ss[1] + Ss[2] * Ss[2];
    e.g12 = Ss[0] * St[0] + Ss[1] * St[1] + Ss[2] * St[2];
    e.g22 = St[0] * St[0] + St[1] * St[1] + St[2] * St[2];
    e.h11 = e.g11 + r[0] * Sss[0] + r[1] * Sss[1] + r[2] * Sss[2];
    e.h12 = e.g12 + r[0] * Sst[0] + r[1] * Sst[1] + r[2] * Sst[2];
    e.h22 = e.g22 + r[0] * Stt[0] + r[1] * Stt[1] + r[2] * Stt[2];
    return e;
}

// smallest eigenvalue of the Hessian of f/2 relative to the metric (1 if degenerate)
template <typename T>
__device__ __forceinline__ T rel_curv(T h11, T h12, T h22, T g11, T g12, T g22)
{
    const T dg = g11 * g22 - g12 * g12;
    if (!(dg > (T)0)) return (T)1;
    const T tr = (g22 * h11 - (T)2 * g12 * h12 + g11 * h22) / dg;
    const T dt = (h11 * h22 - h12 * h12) / dg;
    const T disc = tr * tr - (T)4 * dt;
    return (T)0.5 * (tr - sqrt(disc > (T)0 ? disc : (T)0));
}

// The patch minimum and the second best distinct local minimum found (s2, t2,
// f2: a tie between two minima of one patch needs it).
struct PatchMin {
    float s, t, f, kappa;
    float s2, t2, f2;
    int loc;  // the best is a local minimum of the patch (not an edge point the distance leaves inward)
};
// patch parameters closer than this (|ds| + |dt|) are one minimum, not two
constexpr float kDistinctST = 1e-4f;

// Only a local minimum of the patch (loc) can become the second: the minimum
// of an edge where the distance falls into the patch is a bound, not a minimum.
// Two points are two minima only with a barrier between them (the distance at
// their midpoint above both): FP32 Newton solves that stop at different points
// of one shallow minimum are one minimum.
__device__ __forceinline__ void pm_take(const Bicubic& B, PatchMin& best, float s, float t, float f, float k,
                                        bool loc = true)
{
    bool apart = fabsf(s - best.s) + fabsf(t - best.t) > kDistinctST;
    if (apart && best.f < INFINITY)
        apart = bc_f(B, 0.5f * (s + best.s), 0.5f * (t + best.t)) > fmaxf(f, best.f) * (1.f + 4e-6f);
    if (f < best.f) {
        if (apart && best.loc) { best.s2 = best.s; best.t2 = best.t; best.f2 = best.f; }
        best.s = s; best.t = t; best.f = f; best.kappa = k; best.loc = loc;
    } else if (loc && f < best.f2 && apart) {
        best.s2 = s; best.t2 = t; best.f2 = f;
    }
}

// Box-constrained Newton on [lo_s, hi_s] x [lo_t, hi_t] from (s, t): a
// coordinate on a side with the gradient pointing outward is held there.
__device__ void bc_newton(const Bicubic& B, float s, float t, float lo_s, float hi_s, float lo_t, float hi_t,
                          PatchMin& best)
{
    BcEval e = bc_eval(B, s, t);
    for (int it = 0; it < 16; ++it) {
        // active set: a coordinate on a side whose gradient points outward stays there
        const bool fs = (s == lo_s && e.gs > 0.f) || (s == hi_s && e.gs < 0.f);
        const bool ft = (t == lo_t && e.gt > 0.f) || (t == hi_t && e.gt < 0.f);
        if (fs && ft) break;
        float ds = 0.f, dt = 0.f;
        if (!fs && !ft) {
            // where the distance is not convex, shift the Hessian by a multiple of the
            // metric (Levenberg-Marquardt) so that its smallest relative curvature is 1e-3
            float h11 = e.h11, h12 = e.h12, h22 = e.h22;
            const float lam = rel_curv(h11, h12, h22, e.g11, e.g12, e.g22);
            if (lam < 1e-3f) {
                const float mu = 1e-3f - lam;
                h11 += mu * e.g11; h12 += mu * e.g12; h22 += mu * e.g22;
            }
            const float det = h11 * h22 - h12 * h12;
            if (det > 0.f && h11 > 0.f) {
                ds = -(h22 * e.gs - h12 * e.gt) / det;
                dt = -(h11 * e.gt - h12 * e.gs) / det;
            } else {
                ds = -e.gs / (e.g11 + 1e-30f);
                dt = -e.gt / (e.g22 + 1e-30f);
            }
        } else if (!fs) {
            ds = -e.gs / fmaxf(e.h11, 1e-3f * e.g11 + 1e-30f);
        } else {
            dt = -e.gt / fmaxf(e.h22, 1e-3f * e.g22 + 1e-30f);
        }
        const float lim = 0.25f;
        const float m = fmaxf(fabsf(ds), fabsf(dt));
        if (m > lim) { ds *= lim / m; dt *= lim / m; }
        float sn = fminf(fmaxf(s + ds, lo_s), hi_s), tn = fminf(fmaxf(t + dt, lo_t), hi_t);
        BcEval en = bc_eval(B, sn, tn);
        for (int bt = 0; bt < 4 && en.f > e.f; ++bt) {
            ds *= 0.5f;
            dt *= 0.5f;
            sn = fminf(fmaxf(s + ds, lo_s), hi_s);
            tn = fminf(fmaxf(t + dt, lo_t), hi_t);
            en = bc_eval(B, sn, tn);
        }
        if (en.f > e.f) break;
        const float step = fabsf(sn - s) + fabsf(tn - t);
        s = sn;
        t = tn;
        e = en;
        if (step <= 1e-7f) break;
    }
    const bool interior = s > 0.f && s < 1.f && t > 0.f && t < 1.f;
    pm_take(B, best, s, t, e.f, interior ? rel_curv(e.h11, e.h12, e.h22, e.g11, e.g12, e.g22) : 1.f);
}

// one edge of the patch as a cubic curve relative to the query
__device__ __forceinline__ void bc_edge(const Bicubic& B, int which, Cubic<float>& E)
{
    float c[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            float v = 0.f;
            if (which == 0) v = B.C[0][k][x];                                                       // s = 0, along t
            else if (which == 1) v = B.C[0][k][x] + B.C[1][k][x] + B.C[2][k][x] + B.C[3][k][x];     // s = 1
            else if (which == 2) v = B.C[k][0][x];                                                  // t = 0, along s
            else v = B.C[k][0][x] + B.C[k][1][x] + B.C[k][2][x] + B.C[k][3][x];                     // t = 1
            c[k][x] = v;
        }
    E.a0 = {c[0][0], c[0][1], c[0][2]};
    E.a1 = {c[1][0], c[1][1], c[1][2]};
    E.a2 = {c[2][0], c[2][1], c[2][2]};
    E.a3 = {c[3][0], c[3][1], c[3][2]};
}

// Minimum of f = |S - q|^2 over the patch, or f = +inf when the patch holds no
// value below `cap` (a value known to be attained elsewhere, plus the tie
// margin; +inf: no cap).  The 7 x 7 samples give second-order bounds
// min(corner f) - M h^2 / 8 on every cell and along every edge; an edge or a
// cell whose bound reaches the best value so far is skipped.
__device__ PatchMin patch_min(const Bicubic& B, float cap)
{
    constexpr int kC = kGrid - 1;  // cells per direction
    static_assert(kC * kC <= 64 && (kGrid - 2) * (kGrid - 2) <= 32, "cell and sample masks fit their words");
    const float h = 1.f / kC;
    const float Mss = 2.f * (B.Ls * B.Ls + B.far * B.Lss), Mtt = 2.f * (B.Lt * B.Lt + B.far * B.Ltt);
    const float gap = (Mss + Mtt) * h * h * 0.125f;
    // Phase 1, on the samples (all loops unrolled, so they stay in registers
    // and are dead afterwards): interior local minima below the cap, each
    // edge's smallest sample, and the cells whose bound is below the cap.
    uint32_t lmin = 0;   // bit (i-1)*(kGrid-2)+(j-1)
    uint64_t cells = 0;  // bit i*kC+j: cell (i, j)
    float emn[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    {
        float F[kGrid][kGrid];
#pragma unroll
        for (int i = 0; i < kGrid; ++i)
#pragma unroll
            for (int j = 0; j < kGrid; ++j) F[i][j] = bc_f(B, i * h, j * h);
#pragma unroll
        for (int i = 1; i < kGrid - 1; ++i)
#pragma unroll
            for (int j = 1; j < kGrid - 1; ++j) {
                const float v = F[i][j];
                bool m = v < cap;
#pragma unroll
                for (int a = -1; a <= 1; ++a)
#pragma unroll
                    for (int b = -1; b <= 1; ++b)
                        if (a || b) m = m && !(F[i + a][j + b] < v);
                lmin |= (uint32_t)m << ((i - 1) * (kGrid - 2) + (j - 1));
            }
#pragma unroll
        for (int k = 0; k < kGrid; ++k) {
            emn[0] = fminf(emn[0], F[0][k]);
            emn[1] = fminf(emn[1], F[kGrid - 1][k]);
            emn[2] = fminf(emn[2], F[k][0]);
            emn[3] = fminf(emn[3], F[k][kGrid - 1]);
        }
#pragma unroll
        for (int i = 0; i < kC; ++i)
#pragma unroll
            for (int j = 0; j < kC; ++j) {
                const float mn = fminf(fminf(F[i][j], F[i + 1][j]), fminf(F[i][j + 1], F[i + 1][j + 1]));
                cells |= (uint64_t)(mn - gap < cap) << (i * kC + j);
            }
    }
    PatchMin best{0.f, 0.f, cap, 1.f, 0.f, 0.f, cap, 0};
    // Phase 2: Newton from each local minimum; the four cells around such a
    // sample count as covered
    uint64_t covered = 0;
    for (uint32_t m = lmin; m; m &= m - 1) {
        const int k = __ffs(m) - 1;
        const int i = k / (kGrid - 2) + 1, j = k % (kGrid - 2) + 1;
        bc_newton(B, i * h, j * h, 0.f, 1.f, 0.f, 1.f, best);
        covered |= (3ull << ((i - 1) * kC + (j - 1))) | (3ull << (i * kC + (j - 1)));
    }
    // Phase 3: certified 1D minima of the boundary curves whose sampled bound
    // (second-order along the edge) reaches below the best
    for (int w = 0; w < 4; ++w) {
        const float e = w == 0 ? emn[0] : (w == 1 ? emn[1] : (w == 2 ? emn[2] : emn[3]));
        if (!(e - (w < 2 ? Mtt : Mss) * h * h * 0.125f < best.f * (1.f + 8e-6f))) continue;
        Cubic<float> E;
        bc_edge(B, w, E);
        float u, d, k;
        piece_min(E, u, d, k);
        const float s = w == 0 ? 0.f : (w == 1 ? 1.f : u);
        const float t = w == 2 ? 0.f : (w == 3 ? 1.f : u);
        // a local minimum of the patch only where the distance does not fall
        // into the patch across this edge (up to rounding)
        const BcEval ev = bc_eval(B, s, t);
        const float g = w < 2 ? ev.gs : ev.gt, tol = 1e-5f * sqrtf(ev.f * (w < 2 ? ev.g11 : ev.g22));
        const bool loc = (w == 0 || w == 2) ? g >= -tol : g <= tol;
        pm_take(B, best, s, t, d, 1.f, loc);
    }
    // Phase 4: a Newton solve in every uncovered cell whose second-order bound
    // min(corner f) - (M_ss + M_tt) h^2 / 8 is still below the best (corners
    // evaluated again)
    for (uint64_t m = cells & ~covered; m; m &= m - 1) {
        const int c = __ffsll((unsigned long long)m) - 1;
        const int i = c / kC, j = c % kC;
        const float mn = fminf(fminf(bc_f(B, i * h, j * h), bc_f(B, (i + 1) * h, j * h)),
                               fminf(bc_f(B, i * h, (j + 1) * h), bc_f(B, (i + 1) * h, (j + 1) * h)));
        if (mn - gap < best.f * (1.f - 8e-6f))
            bc_newton(B, (i + 0.5f) * h, (j + 0.5f) * h, i * h, (i + 1) * h, j * h, (j + 1) * h, best);
    }
    if (!(best.f < cap)) best = PatchMin{0.f, 0.f, INFINITY, 1.f, 0.f, 0.f, INFINITY, 0};
    if (!(best.f2 < cap)) best.f2 = INFINITY;
    return best;
}

// ---------------------------------------------------------------------------
// 2 + 3a. per query, the patches that can hold its minimum
// ---------------------------------------------------------------------------
// One workgroup per tile of kQueriesPerTile queries of one surface, 8 lanes per
// query:
//   a. threshold: a first bound from the cluster spheres and the patches of
//      the nearest clusters, then the best patch sphere upper bound over the
//      clusters that reach it (plain calls), each sharpened by points of the
//      nearest-centre patch (patch_point_bound), or the seed's value (seeded
//      calls, in fub); plus the tie margin;
//   b. list the patches of those clusters whose sphere lower bound reaches the
//      threshold (at most kSphCap, and at most kCluCap clusters; more: the
//      query takes the full scan);
//   c. a 4 x 4 sample bound of every listed patch: lb = min(samples) -
//      (M_ss + M_tt) h^2 / 8 with h = 1/3 (second-order bound of f = |S - q|^2),
//      and the best sample value lowers the query's bound;
//   d. keep the patches whose lb reaches the final threshold, compacted into
//      the query's pair list (one atomic per workgroup); fub = final bound.
template <bool kSeeded>
__global__ __launch_bounds__(kSphThreads) void k_slist(DevSurf D, const int32_t* __restrict__ tile_off,
                                                       const int32_t* __restrict__ q_off,
                                                       const int32_t* __restrict__ perm,
                                                       const double* __restrict__ qxyz, float tie_rel, ScreenOut so,
                                                       uint32_t* __restrict__ fub)
{
    // the sampled bounds reuse the cluster staging area once the sweeps are done
    __shared__ union {
        float4 st[kCluChunk];
        float lb[kQueriesPerTile][kSphCap];
    } s_u;
    __shared__ int32_t s_list[kQueriesPerTile][kSphCap];
    __shared__ uint16_t s_clu[kQueriesPerTile][kCluCap];
    __shared__ int32_t s_base[kQueriesPerTile];
    const int n_tiles = tile_off[D.n_surf];
    const int per = (n_tiles + kXcds - 1) / kXcds;
    const int slot = (int)(blockIdx.x / kXcds);
    const int tile = (int)(blockIdx.x % kXcds) * per + slot;
    if (slot >= per || tile >= n_tiles) return;
    int lo_c = 0, hi_c = D.n_surf;
    while (hi_c - lo_c > 1) {
        const int mid = (lo_c + hi_c) >> 1;
        if (tile_off[mid] <= tile) lo_c = mid; else hi_c = mid;
    }
    const DSurf sf = D.surfs[lo_c];
    const int lane = threadIdx.x & 63;
    const int qs = threadIdx.x / kSphSub, sub = threadIdx.x % kSphSub;
    const int64_t j = (int64_t)q_off[lo_c] + (int64_t)(tile - tile_off[lo_c]) * kQueriesPerTile + qs;
    const bool active = j < q_off[lo_c + 1];
    double q[3] = {0.0, 0.0, 0.0};
    if (active) {
        const int32_t qi = perm[j];
#pragma unroll
        for (int k = 0; k < 3; ++k) q[k] = qxyz[3 * (int64_t)qi + k];
    }
    const float ql[3] = {(float)(q[0] - sf.origin[0]), (float)(q[1] - sf.origin[1]), (float)(q[2] - sf.origin[2])};
    const float eps = 1e-6f * (sqrtf(ql[0] * ql[0] + ql[1] * ql[1] + ql[2] * ql[2]) + (float)sf.diag);
    // a. threshold and candidate clusters
    float ub = INFINITY, fq = INFINITY;
    int ns;
    if (kSeeded) {
        if (active) fq = __uint_as_float(fub[j]);
        ub = sqrtf(fq);
        ns = clu_list(D, sf, s_u.st, ql, eps, ub + s_margin(ub, sf, tie_rel), active, lane, sub, s_clu[qs]);
    } else {
        const float ubs = first_ub(D, sf, s_u.st, ql, eps, active, sub);
        ns = clu_list(D, sf, s_u.st, ql, eps, ubs + s_margin(ubs, sf, tie_rel), active, lane, sub, s_clu[qs]);
        // the best patch sphere upper bound over the candidate clusters
        float bd = INFINITY;
        int bk = -1;
        if (active && ns <= kCluCap)
            for (int m = 0; m < ns; ++m) ub = clu_patch_ub(D, sf, s_clu[qs][m], ql, eps, sub, ub, bd, bk);
        // and the point bound of the nearest-centre patch over all of them (the
        // first bound holds too)
        ub = fminf(fminf(ub, ubs), patch_point_bound(D, sf, bd, bk, sub, active && ns <= kCluCap, ql, eps));
#pragma unroll
        for (int off = 1; off < kSphSub; off <<= 1) ub = fminf(ub, __shfl_xor(ub, off, 64));
    }
    const float thr = ub + s_margin(ub, sf, tie_rel);
    // b. list the patches of the candidate clusters whose sphere bound reaches thr
    int cnt = 0;  // same value in the query's 8 lanes
    if (active && ns <= kCluCap) {
        for (int m = 0; m < ns; ++m) {
            const CluRows R = clu_rows(sf, s_clu[qs][m]);
            for (int iu = R.iu0; iu < R.iu1; ++iu) {
                const int64_t rs = sf.span_off + (int64_t)iu * sf.n_sv;
                const int k0 = D.span0[rs + R.iv0], k1 = D.span0[rs + R.iv1];
                for (int i0 = k0; i0 < k1; i0 += kBatch * kSphSub) {
                    float4 p[kBatch];
#pragma unroll
                    for (int r = 0; r < kBatch; ++r) {
                        const int k = i0 + r * kSphSub + sub;
                        p[r] = k < k1 ? D.sph[k] : make_float4(0.f, 0.f, 0.f, 0.f);
                    }
#pragma unroll
                    for (int r = 0; r < kBatch; ++r) {
                        const int k = i0 + r * kSphSub + sub;
                        bool hit = false;
                        if (k < k1) {
                            const float dx = ql[0] - p[r].x, dy = ql[1] - p[r].y, dz = ql[2] - p[r].z;
                            const float tt = thr + p[r].w + eps;
                            hit = tt >= 0.f && dx * dx + dy * dy + dz * dz <= tt * tt;
                        }
                        const uint32_t grp = (uint32_t)(__ballot(hit) >> (lane & 56)) & 0xffu;
                        const int pos = cnt + __popc(grp & ((1u << sub) - 1u));
                        if (hit && pos < kSphCap) s_list[qs][pos] = k - (int)sf.patch_off;
                        cnt += __popc(grp);
                    }
                }
            }
        }
    } else if (active) {
        cnt = kSphCap + 1;  // too many clusters: the full scan
    }
    const bool listed = active && cnt <= kSphCap;
    __syncthreads();  // every wave is done with the staged spheres
    // c. sampled bounds
    if (listed) {
        for (int k = sub; k < cnt; k += kSphSub) {
            Bicubic B;
            load_bicubic(D, sf, sf.patch_off + s_list[qs][k], q, B);
            float mn = INFINITY;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) mn = fminf(mn, bc_f(B, a * (1.f / 3.f), b * (1.f / 3.f)));
            const float Mss = 2.f * (B.Ls * B.Ls + B.far * B.Lss), Mtt = 2.f * (B.Lt * B.Lt + B.far * B.Ltt);
            s_u.lb[qs][k] = mn * (1.f - 4e-6f) - (Mss + Mtt) * (1.f / 72.f) * 1.0001f;
            fq = fminf(fq, mn * (1.f + 4e-6f));
        }
    }
#pragma unroll
    for (int off = 1; off < kSphSub; off <<= 1) fq = fminf(fq, __shfl_xor(fq, off, 64));
    __syncthreads();
    // d. gate: compaction in place (a kept entry moves to a position at most its own)
    int live = 0;
    if (listed) {
        const float u = sqrtf(fq);
        const float t = u + s_margin(u, sf, tie_rel);
        const float t2 = t * t;
        for (int i0 = 0; i0 < cnt; i0 += kSphSub) {
            const int k = i0 + sub;
            const bool keep = k < cnt && s_u.lb[qs][k] <= t2;
            const int32_t v = keep ? s_list[qs][k] : 0;
            const uint32_t grp = (uint32_t)(__ballot(keep) >> (lane & 56)) & 0xffu;
            const int pos = live + __popc(grp & ((1u << sub) - 1u));
            if (keep) s_list[qs][pos] = v;
            live += __popc(grp);
        }
    }
    // reserve the workgroup's pairs with one atomic
    if (sub == 0) s_base[qs] = listed ? live : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < kQueriesPerTile; ++k) {
            const int v = s_base[k];
            s_base[k] = tot;
            tot += v;
        }
        const int base = tot > 0 ? atomicAdd(so.pair_count, tot) : 0;
        for (int k = 0; k < kQueriesPerTile; ++k) s_base[k] += base;
    }
    __syncthreads();
    if (!active) return;
    const int64_t b = s_base[qs];
    const bool fits = listed && b + live <= so.pair_cap;
    if (sub == 0) {
        so.cand_n[j] = fits ? live : -1;
        so.pair_off[j] = (int32_t)b;
        so.ub[j] = ub;
        fub[j] = __float_as_uint(fq);
    }
    if (listed) {
        for (int k = sub; k < live; k += kSphSub) {
            if (b + k >= so.pair_cap) break;
            so.pair_seg[b + k] = fits ? (int32_t)(sf.patch_off + s_list[qs][k]) : 0;
            so.pair_j[b + k] = fits ? (int32_t)j : -1;  // a slot past the capacity stays unused
        }
    }
}

// 3b. One thread per listed pair: the certified patch minimum below the
// query's threshold.
// Occupancy of the patch kernels (waves per SIMD; the register limit makes the
// compiler spill some temporaries): measured on the batched surfaces,
// patch minima 40.9 -> 31.2 ms with k_spairs at 4 (256 VGPRs -> 128), polish
// and write 26.8 -> 23.5 ms with k_sfinish at 3 and k_sfull at 2.
#ifndef MREP_SPAIRS_MIN_WAVES
#define MREP_SPAIRS_MIN_WAVES 4
#endif
#ifndef MREP_SFINISH_MIN_WAVES
#define MREP_SFINISH_MIN_WAVES 3
#endif
#ifndef MREP_SFULL_MIN_WAVES
#define MREP_SFULL_MIN_WAVES 2
#endif
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MREP_SPAIRS_MIN_WAVES, 8))) void k_spairs(DevSurf D, const int32_t* __restrict__ sid,
                                                const double* __restrict__ qxyz, const int32_t* __restrict__ perm,
                                                ScreenOut so, const uint32_t* __restrict__ fub, float tie_rel,
                                                float4* __restrict__ res)
{
    const int64_t total = min((int64_t)*so.pair_count, so.pair_cap);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t jj = so.pair_j[p];
        if (jj < 0) continue;
        const int64_t k = so.pair_seg[p];
        const int32_t qi = perm[jj];
        const DSurf sf = D.surfs[sid[qi]];
        const double q[3] = {qxyz[3 * (int64_t)qi], qxyz[3 * (int64_t)qi + 1], qxyz[3 * (int64_t)qi + 2]};
        Bicubic B;
        load_bicubic(D, sf, k, q, B);
        const float ub = sqrtf(__uint_as_float(fub[jj]));
        const float thr = ub + s_margin(ub, sf, tie_rel);
        const PatchMin m = patch_min(B, thr * thr * (1.f + 1e-5f));
        res[2 * p] = make_float4(m.s, m.t, m.f, m.kappa);
        res[2 * p + 1] = make_float4(m.s2, m.t2, m.f2, 1.f);
    }
}

// Seeded calls, one thread per query: Newton from the network's (s, t) on the
// best-scored candidate patch; the attained value (with the same rounding
// allowance as a sample), or the square of the best sphere upper bound when
// that is smaller, is the query's first bound.
__global__ __launch_bounds__(256) void k_sseed(DevSurf D, const int32_t* __restrict__ sid,
                                               const double* __restrict__ qxyz, const int32_t* __restrict__ q_off,
                                               const int32_t* __restrict__ perm, const int32_t* __restrict__ cand,
                                               const float4* __restrict__ score, const float* __restrict__ ub,
                                               uint32_t* __restrict__ fub, int32_t* __restrict__ seed_patch)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q_off[D.n_surf]) return;
    int best = -1;
    float z = -INFINITY;
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        const float zk = score[j * kK + k].z;
        if (cand[j * kK + k] >= 0 && (best < 0 || zk > z)) { best = k; z = zk; }
    }
    const float u2 = ub[j] * ub[j];
    if (best < 0) {
        fub[j] = __float_as_uint(u2);
        seed_patch[j] = -1;
        return;
    }
    const int64_t k = cand[j * kK + best];
    const float4 sc = score[j * kK + best];
    const int32_t qi = perm[j];
    const DSurf sf = D.surfs[sid[qi]];
    const double q[3] = {qxyz[3 * (int64_t)qi], qxyz[3 * (int64_t)qi + 1], qxyz[3 * (int64_t)qi + 2]};
    Bicubic B;
    load_bicubic(D, sf, k, q, B);
    // a prediction that is not a number starts from the patch centre
    const float s0 = sc.x == sc.x ? fminf(fmaxf(sc.x, 0.f), 1.f) : 0.5f;
    const float t0 = sc.y == sc.y ? fminf(fmaxf(sc.y, 0.f), 1.f) : 0.5f;
    PatchMin m{0.f, 0.f, INFINITY, 1.f, 0.f, 0.f, INFINITY};
    bc_newton(B, s0, t0, 0.f, 1.f, 0.f, 1.f, m);
    const float f = m.f * (1.f + 4e-6f);
    fub[j] = __float_as_uint(f < u2 ? f : u2);
    seed_patch[j] = (int32_t)k;
}

// ---------------------------------------------------------------------------
// 4. FP64 polish on the exact span patch, finish
// ---------------------------------------------------------------------------
struct SCand {
    double u, v, d2, kappa;
    int64_t patch;
    int32_t edge;  // bit 0: on the boundary of its patch's rectangle; bit 1: the patch's second
                   // local minimum, not its minimum
};

// lexicographic (d2, u, v); bitwise operators keep it free of branches
__device__ __forceinline__ bool s_better(const SCand& a, const SCand& b)
{
    return (a.d2 < b.d2) | ((a.d2 == b.d2) & ((a.u < b.u) | ((a.u == b.u) & (a.v < b.v))));
}

// x sits on the boundary of the closed rectangle of another patch whose
// minimum is y (false when y is empty or a second minimum)
__device__ __forceinline__ bool s_on(const DevSurf& D, const SCand& x, const SCand& y)
{
    if (!(x.edge & 1) || (y.edge & 2) || !(y.d2 < INFINITY) || x.patch == y.patch) return false;
    const double* r = D.uv + 4 * y.patch;
    const double eps = 1e-12 * (fabs(r[0]) + fabs(r[1]) + fabs(r[2]) + fabs(r[3]) + 1e-300);
    return x.u >= r[0] - eps && x.u <= r[1] + eps && x.v >= r[2] - eps && x.v <= r[3] + eps;
}

__device__ __forceinline__ void s_select(bool c, const SCand& a, SCand& dst)
{
    dst.u = c ? a.u : dst.u;
    dst.v = c ? a.v : dst.v;
    dst.d2 = c ? a.d2 : dst.d2;
    dst.kappa = c ? a.kappa : dst.kappa;
    dst.patch = c ? a.patch : dst.patch;
    dst.edge = c ? a.edge : dst.edge;
}

// (b1, b2) <- the two best of (b1, b2, x), field by field so that the
// candidates stay in registers.  A candidate on the boundary of the patch whose
// minimum is the best is no lower than that minimum and no other local minimum
// of the surface (a genuine one there is that patch's second minimum): it is
// dropped, and when the best lies on the patch whose minimum the new candidate
// is, the new one replaces it without becoming the runner-up.  Otherwise the
// copies of one minimum held by the patches around it would fill both places
// and push a genuine second minimum out of the tie test.
__device__ __forceinline__ void s_top2(const DevSurf& D, const SCand& x, SCand& b1, SCand& b2)
{
    const bool live = x.d2 < INFINITY && !s_on(D, x, b1);
    const bool repl = live && s_on(D, b1, x);
    const bool first = live && (repl || s_better(x, b1));
    const bool second = live && !first && !s_on(D, x, b2) && s_better(x, b2);
    if (repl && s_on(D, b2, x)) b2.d2 = INFINITY;
    s_select(first && !repl, b1, b2);
    s_select(second, x, b2);
    s_select(first, x, b1);
}

__device__ __forceinline__ SCand s_empty()
{
    SCand c;
    c.u = c.v = 0.0;
    c.d2 = INFINITY;
    c.kappa = 1.0;
    c.patch = -1;
    c.edge = 0;
    return c;
}

__device__ __forceinline__ SCand s_make(const DevSurf& D, int64_t k, float s, float t, float f, float kap)
{
    const double* r = D.uv + 4 * k;
    SCand c;
    c.u = s == 1.f ? r[1] : r[0] + (double)s * (r[1] - r[0]);
    c.v = t == 1.f ? r[3] : r[2] + (double)t * (r[3] - r[2]);
    c.d2 = (double)f;
    c.kappa = (double)kap;
    c.patch = k;
    c.edge = s == 0.f || s == 1.f || t == 0.f || t == 1.f;
    return c;
}

// Exact span patch (degree p x q, power form in local (s, t)) minus the query.
struct ExactEval {
    double f, gs, gt, h11, h12, h22, g11, g12, g22;
};

// P, Q > 0: degrees fixed at compile time (loops unrolled, coefficient loads
// issued together); P = Q = 0: the degrees p, q given at run time.
template <int P, int Q>
__device__ __forceinline__ ExactEval exact_eval_deg(const double* cf, int p, int q, const double* x, double s,
                                                    double t)
{
    if (P > 0) {
        p = P;
        q = Q;
    }
    double r[3], Ss[3], St[3], Sss[3], Sst[3], Stt[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // Horner in s of D_a(t), D_a'(t), D_a''(t)
        double v = 0, vs = 0, vss = 0, vt = 0, vst = 0, vtt = 0;
#pragma unroll 1
        for (int a = p; a >= 0; --a) {
            double d = 0, d1 = 0, d2 = 0;
#pragma unroll
            for (int b = q; b >= 0; --b) {
                const double cc = cf[3 * (a * (q + 1) + b) + c];
                d2 = d2 * t + 2.0 * d1;
                d1 = d1 * t + d;
                d = d * t + cc;
            }
            vss = vss * s + 2.0 * vs;
            vs = vs * s + v;
            v = v * s + d;
            vst = vst * s + vt;
            vt = vt * s + d1;
            vtt = vtt * s + d2;
        }
        r[c] = v - x[c];
        Ss[c] = vs;
        Sss[c] = vss;
        St[c] = vt;
        Sst[c] = vst;
        Stt[c] = vtt;
    }
    ExactEval e;
    e.f = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    e.gs = r[0] * Ss[0] + r[1] * Ss[1] + r[2] * Ss[2];
    e.gt = r[0] * St[0] + r[1] * St[1] + r[2] * St[2];
    e.g11 = Ss[0] * Ss[0] + Ss[1] * Ss[1] + Ss[2] * Ss[2];
    e.g12 = Ss[0] * St[0] + Ss[1] * St[1] + Ss[2] * St[2];
    e.g22 = St[0] * St[0] + St[1] * St[1] + St[2] * St[2];
    e.h11 = e.g11 + r[0] * Sss[0] + r[1] * Sss[1] + r[2] * Sss[2];
    e.h12 = e.g12 + r[0] * Sst[0] + r[1] * Sst[1] + r[2] * Sst[2];
    e.h22 = e.g22 + r[0] * Stt[0] + r[1] * Stt[1] + r[2] * Stt[2];
    return e;
}

// the degrees of the benchmark surfaces (3 x 3 and 5 x 5) get unrolled code
__device__ __forceinline__ ExactEval exact_eval(const double* cf, int p, int q, const double* x, double s, double t)
{
    if (p == 3 && q == 3) return exact_eval_deg<3, 3>(cf, p, q, x, s, t);
    if (p == 5 && q == 5) return exact_eval_deg<5, 5>(cf, p, q, x, s, t);
    return exact_eval_deg<0, 0>(cf, p, q, x, s, t);
}

// span index of parameter w among n spans with breakpoints b[0..n]
__device__ __forceinline__ int span_of(const double* b, int n, double w)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (b[mid] <= w) lo = mid; else hi = mid;
    }
    return lo;
}

struct Polished {
    double u, v, dist, kappa;
};

// FP64 box-constrained Newton on the exact span patch holding (u, v); moves to
// the neighbouring span patch (at most 4 times) when it stops on a shared edge
// with the gradient pointing across it.
__device__ Polished s_polish(const DevSurf& D, const DSurf& sf, double u, double v, const double* x)
{
    const double* bu = D.brk + sf.brk_off;
    const double* bv = bu + sf.n_su + 1;
    int iu = span_of(bu, sf.n_su, u), iv = span_of(bv, sf.n_sv, v);
    const int p = sf.deg_u, q = sf.deg_v;
    double s = 0, t = 0;
    ExactEval e;
    for (int hop = 0; hop < 5; ++hop) {
        const double ua = bu[iu], ub = bu[iu + 1], va = bv[iv], vb = bv[iv + 1];
        const double* cf = D.coef + sf.coef_off + (int64_t)(iu * sf.n_sv + iv) * 3 * (p + 1) * (q + 1);
        s = fmin(fmax((u - ua) / (ub - ua), 0.0), 1.0);
        t = fmin(fmax((v - va) / (vb - va), 0.0), 1.0);
        e = exact_eval(cf, p, q, x, s, t);
        for (int it = 0; it < 60; ++it) {
            // active set: a coordinate on a side whose gradient points outward stays there
            const bool fs = (s == 0.0 && e.gs > 0.0) || (s == 1.0 && e.gs < 0.0);
            const bool ft = (t == 0.0 && e.gt > 0.0) || (t == 1.0 && e.gt < 0.0);
            if (fs && ft) break;
            double ds = 0, dt = 0;
            if (!fs && !ft) {
                double h11 = e.h11, h12 = e.h12, h22 = e.h22;
                const double lam = rel_curv(h11, h12, h22, e.g11, e.g12, e.g22);
                if (lam < 1e-3) {  // Levenberg-Marquardt shift where the distance is not convex
                    const double mu = 1e-3 - lam;
                    h11 += mu * e.g11; h12 += mu * e.g12; h22 += mu * e.g22;
                }
                const double det = h11 * h22 - h12 * h12;
                if (det > 0.0 && h11 > 0.0) {
                    ds = -(h22 * e.gs - h12 * e.gt) / det;
                    dt = -(h11 * e.gt - h12 * e.gs) / det;
                } else {
                    ds = -e.gs / (e.g11 + 1e-300);
                    dt = -e.gt / (e.g22 + 1e-300);
                }
            } else if (!fs) {
                ds = -e.gs / fmax(e.h11, 1e-3 * e.g11 + 1e-300);
            } else {
                dt = -e.gt / fmax(e.h22, 1e-3 * e.g22 + 1e-300);
            }
            const double m = fmax(fabs(ds), fabs(dt));
            if (m > 0.25) { ds *= 0.25 / m; dt *= 0.25 / m; }
            double sn = fmin(fmax(s + ds, 0.0), 1.0), tn = fmin(fmax(t + dt, 0.0), 1.0);
            ExactEval en = exact_eval(cf, p, q, x, sn, tn);
            for (int bt = 0; bt < 12 && en.f > e.f; ++bt) {
                ds *= 0.5;
                dt *= 0.5;
                sn = fmin(fmax(s + ds, 0.0), 1.0);
                tn = fmin(fmax(t + dt, 0.0), 1.0);
                en = exact_eval(cf, p, q, x, sn, tn);
            }
            if (en.f > e.f) break;  // no decrease above rounding: converged
            const double step = fabs(sn - s) + fabs(tn - t);
            s = sn;
            t = tn;
            e = en;
            // the error after a Newton step is of the order of its square
            if (step <= 1e-10) break;
        }
        u = s == 1.0 ? ub : ua + s * (ub - ua);
        v = t == 1.0 ? vb : va + t * (vb - va);
        // continue across a shared edge when the gradient points across it
        int niu = iu, niv = iv;
        if (s == 0.0 && e.gs > 0.0 && iu > 0) niu = iu - 1;
        else if (s == 1.0 && e.gs < 0.0 && iu < sf.n_su - 1) niu = iu + 1;
        if (t == 0.0 && e.gt > 0.0 && iv > 0) niv = iv - 1;
        else if (t == 1.0 && e.gt < 0.0 && iv < sf.n_sv - 1) niv = iv + 1;
        if (niu == iu && niv == iv) break;
        iu = niu;
        iv = niv;
    }
    Polished r;
    r.u = u;
    r.v = v;
    r.dist = sqrt(e.f);
    const bool interior = s > 0.0 && s < 1.0 && t > 0.0 && t < 1.0;
    r.kappa = interior ? rel_curv(e.h11, e.h12, e.h22, e.g11, e.g12, e.g22) : 1.0;
    return r;
}

struct SOuts {
    double* uv;
    double* d;
    int32_t* patch;
    uint32_t* f;
};

__device__ void s_finish(const DevSurf& D, const DSurf& sf, const double* x, const SCand& b1, const SCand& b2,
                         uint32_t flags, double tie_rel, int invert, int32_t qi, const SOuts& o)
{
    const double d1 = sqrt(b1.d2), d2 = sqrt(b2.d2);
    const double margin = 2.0 * sf.tol_eff + 2e-6 * (d1 + sf.diag) + tie_rel * sf.diag;
    const bool tie = b2.d2 < INFINITY && (d2 - d1) <= margin;
    flags |= MREP_F_POLISHED;
    Polished r = s_polish(D, sf, b1.u, b1.v, x);
    // A runner-up needs no polish of its own when it is the point the polish of
    // the best already reached, or when it lies on the closed rectangle of the
    // best's patch: that patch's minimum (the best) is then no larger, and a
    // descent from the runner-up can only end lower by entering a patch whose
    // minimum would have ranked above it.
    const double* bu0 = D.brk + sf.brk_off;
    const double* bv0 = bu0 + sf.n_su + 1;
    const double span = fmax(bu0[sf.n_su] - bu0[0], bv0[sf.n_sv] - bv0[0]);
    const double* r1 = D.uv + 4 * b1.patch;
    const double eps = 1e-12 * span;
    // (a second minimum of the best's own patch is a distinct local minimum: it is polished)
    const bool on_best = b2.patch != b1.patch && b2.u >= r1[0] - eps && b2.u <= r1[1] + eps && b2.v >= r1[2] - eps &&
                         b2.v <= r1[3] + eps;
    if (tie && !on_best && fabs(b2.u - r.u) + fabs(b2.v - r.v) > 1e-6 * span) {
        const Polished r2 = s_polish(D, sf, b2.u, b2.v, x);
        const bool take = r2.dist < r.dist || (r2.dist == r.dist && (r2.u < r.u || (r2.u == r.u && r2.v < r.v)));
        const double sep = fabs(r2.u - r.u) + fabs(r2.v - r.v);
        if (fabs(r2.dist - r.dist) <= tie_rel * sf.diag && sep > 1e-6) flags |= MREP_F_NEAR_TIE;
        if (take) r = r2;
    }
    if (r.kappa < 1e-2) flags |= MREP_F_ILL_COND;
    // patch holding (u, v): among the pieces of its exact span patch, half-open
    // rectangles closed at the surface's far sides
    const double* bu = D.brk + sf.brk_off;
    const double* bv = bu + sf.n_su + 1;
    const int iu = span_of(bu, sf.n_su, r.u), iv = span_of(bv, sf.n_sv, r.v);
    const int64_t sp = sf.span_off + (int64_t)iu * sf.n_sv + iv;
    int64_t patch = D.span0[sp];
    for (int64_t k = D.span0[sp]; k < D.span0[sp + 1]; ++k) {
        const double* rc = D.uv + 4 * k;
        const bool in_u = r.u >= rc[0] && (r.u < rc[1] || (rc[1] == bu[sf.n_su] && r.u <= rc[1]));
        const bool in_v = r.v >= rc[2] && (r.v < rc[3] || (rc[3] == bv[sf.n_sv] && r.v <= rc[3]));
        if (in_u && in_v) { patch = k; break; }
    }
    const double u0 = bu[0], u1 = bu[sf.n_su], v0 = bv[0], v1 = bv[sf.n_sv];
    if (r.u <= u0 + 1e-12 * (u1 - u0) || r.u >= u1 - 1e-12 * (u1 - u0) || r.v <= v0 + 1e-12 * (v1 - v0) ||
        r.v >= v1 - 1e-12 * (v1 - v0))
        flags |= MREP_F_ENDPOINT;
    if (invert && r.dist > sf.tol_user) flags |= MREP_F_OFFCURVE;
    o.uv[2 * (int64_t)qi] = r.u;
    o.uv[2 * (int64_t)qi + 1] = r.v;
    o.d[qi] = r.dist;
    o.patch[qi] = (int32_t)(patch - sf.patch_off);
    o.f[qi] = flags;
}

__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(MREP_SFINISH_MIN_WAVES, 8))) void k_sfinish(DevSurf D, const int32_t* __restrict__ sid,
                                                 const double* __restrict__ qxyz, const int32_t* __restrict__ q_off,
                                                 const int32_t* __restrict__ perm, ScreenOut so,
                                                 const float4* __restrict__ res, double tie_rel, int32_t invert,
                                                 int32_t* __restrict__ ovf_list, int32_t* __restrict__ ovf_count,
                                                 const int32_t* __restrict__ seed_patch, SOuts o)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q_off[D.n_surf]) return;
    const int n_list = so.cand_n[j];
    if (n_list <= 0) {
        ovf_list[atomicAdd(ovf_count, 1)] = (int32_t)j;
        return;
    }
    const int32_t qi = perm[j];
    const DSurf sf = D.surfs[sid[qi]];
    const double x[3] = {qxyz[3 * (int64_t)qi], qxyz[3 * (int64_t)qi + 1], qxyz[3 * (int64_t)qi + 2]};
    SCand b1 = s_empty(), b2 = b1;
    const int64_t p0 = so.pair_off[j];
    for (int i = 0; i < n_list; ++i) {
        const float4 r = res[2 * (p0 + i)], r2 = res[2 * (p0 + i) + 1];
        if (r.z < INFINITY) s_top2(D, s_make(D, so.pair_seg[p0 + i], r.x, r.y, r.z, r.w), b1, b2);
        if (r2.z < INFINITY) {
            SCand c2 = s_make(D, so.pair_seg[p0 + i], r2.x, r2.y, r2.z, r2.w);
            c2.edge |= 2;  // the patch's second local minimum
            s_top2(D, c2, b1, b2);
        }
    }
    if (!(b1.d2 < INFINITY)) {
        // no pair reached below its cap (FP32 rounding at the threshold): full scan
        ovf_list[atomicAdd(ovf_count, 1)] = (int32_t)j;
        return;
    }
    // seeded calls: the network's patch did not hold the minimum
    const bool missed = seed_patch && b1.patch != seed_patch[j];
    s_finish(D, sf, x, b1, b2, missed ? (uint32_t)MREP_F_NN_FALLBACK : 0u, tie_rel, invert, qi, o);
}

// Overflowed lists: one wave per query, three traversals of the clusters whose
// sphere reaches the current threshold (the lanes test 64 clusters at a time,
// then stride over the patches of each hit whose own sphere reaches it):
//   A. the best patch sphere upper bound;
//   B. the 4 x 4 sample bounds, whose best sample lowers the bound;
//   C. the capped patch minimum of every patch whose sampled bound reaches it.
template <typename F>
__device__ void wave_patches(const DevSurf& D, const DSurf& sf, const float* ql, float eps, float thr, int lane,
                             F&& f)
{
    for (int c0 = 0; c0 < sf.n_clu; c0 += 64) {
        const int c = c0 + lane;
        bool hit = false;
        if (c < sf.n_clu) {
            const float4 p = D.csph[sf.clu_off + c];
            const float dx = ql[0] - p.x, dy = ql[1] - p.y, dz = ql[2] - p.z;
            const float tt = thr + p.w + eps;
            hit = tt >= 0.f && dx * dx + dy * dy + dz * dz <= tt * tt;
        }
        for (uint64_t m = __ballot(hit); m; m &= m - 1) {
            const CluRows R = clu_rows(sf, c0 + __ffsll((unsigned long long)m) - 1);
            for (int iu = R.iu0; iu < R.iu1; ++iu) {
                const int64_t rs = sf.span_off + (int64_t)iu * sf.n_sv;
                const int k1 = D.span0[rs + R.iv1];
                for (int k = D.span0[rs + R.iv0] + lane; k < k1; k += 64) {
                    const float4 p = D.sph[k];
                    const float dx = ql[0] - p.x, dy = ql[1] - p.y, dz = ql[2] - p.z;
                    const float d = sqrtf(dx * dx + dy * dy + dz * dz);
                    if (d - p.w - eps <= thr) f(k, d + p.w + eps);
                }
            }
        }
    }
}

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MREP_SFULL_MIN_WAVES, 8))) void k_sfull(DevSurf D, const int32_t* __restrict__ sid,
                                               const double* __restrict__ qxyz, const int32_t* __restrict__ perm,
                                               const int32_t* __restrict__ list, const int32_t* __restrict__ count,
                                               double tie_rel, int32_t invert, uint32_t extra, SOuts o)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t total = *count;
    const float tr = (float)tie_rel;
    for (int64_t item = wave; item < total; item += nwaves) {
        const int32_t qi = perm[list[item]];
        const DSurf sf = D.surfs[sid[qi]];
        const double x[3] = {qxyz[3 * (int64_t)qi], qxyz[3 * (int64_t)qi + 1], qxyz[3 * (int64_t)qi + 2]};
        const float ql[3] = {(float)(x[0] - sf.origin[0]), (float)(x[1] - sf.origin[1]), (float)(x[2] - sf.origin[2])};
        const float eps = 1e-6f * (sqrtf(ql[0] * ql[0] + ql[1] * ql[1] + ql[2] * ql[2]) + (float)sf.diag);
        float ub = INFINITY;
        for (int c = lane; c < sf.n_clu; c += 64) {
            const float4 p = D.csph[sf.clu_off + c];
            const float dx = ql[0] - p.x, dy = ql[1] - p.y, dz = ql[2] - p.z;
            ub = fminf(ub, sqrtf(dx * dx + dy * dy + dz * dz) + p.w + eps);
        }
        ub = wave_min(ub);
        // A
        float ubp = ub;
        wave_patches(D, sf, ql, eps, ub + s_margin(ub, sf, tr), lane, [&](int, float u) { ubp = fminf(ubp, u); });
        ub = wave_min(ubp);
        // B
        float fq = ub * ub;
        wave_patches(D, sf, ql, eps, ub + s_margin(ub, sf, tr), lane, [&](int k, float) {
            Bicubic B;
            load_bicubic(D, sf, k, x, B);
            float mn = INFINITY;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) mn = fminf(mn, bc_f(B, a * (1.f / 3.f), b * (1.f / 3.f)));
            fq = fminf(fq, mn * (1.f + 4e-6f));
        });
        fq = wave_min(fq);
        // C
        const float u = sqrtf(fq);
        const float thr = u + s_margin(u, sf, tr);
        const float thr2 = thr * thr;
        SCand b1 = s_empty(), b2 = b1;
        wave_patches(D, sf, ql, eps, thr, lane, [&](int k, float) {
            Bicubic B;
            load_bicubic(D, sf, k, x, B);
            float mn = INFINITY;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) mn = fminf(mn, bc_f(B, a * (1.f / 3.f), b * (1.f / 3.f)));
            const float Mss = 2.f * (B.Ls * B.Ls + B.far * B.Lss), Mtt = 2.f * (B.Lt * B.Lt + B.far * B.Ltt);
            if (mn * (1.f - 4e-6f) - (Mss + Mtt) * (1.f / 72.f) * 1.0001f > thr2) return;
            const PatchMin m = patch_min(B, thr2 * (1.f + 1e-5f));
            if (m.f < INFINITY) s_top2(D, s_make(D, k, m.s, m.t, m.f, m.kappa), b1, b2);
            if (m.f2 < INFINITY) {
                SCand c2 = s_make(D, k, m.s2, m.t2, m.f2, 1.f);
                c2.edge |= 2;
                s_top2(D, c2, b1, b2);
            }
        });
        // wave top-2
        for (int off = 32; off > 0; off >>= 1) {
            SCand o1, o2;
            o1.u = __shfl_xor(b1.u, off, 64); o1.v = __shfl_xor(b1.v, off, 64); o1.d2 = __shfl_xor(b1.d2, off, 64);
            o1.kappa = __shfl_xor(b1.kappa, off, 64); o1.patch = __shfl_xor(b1.patch, off, 64);
            o2.u = __shfl_xor(b2.u, off, 64); o2.v = __shfl_xor(b2.v, off, 64); o2.d2 = __shfl_xor(b2.d2, off, 64);
            o2.kappa = __shfl_xor(b2.kappa, off, 64); o2.patch = __shfl_xor(b2.patch, off, 64);
            o1.edge = __shfl_xor(b1.edge, off, 64); o2.edge = __shfl_xor(b2.edge, off, 64);
            s_top2(D, o1, b1, b2);
            s_top2(D, o2, b1, b2);
        }
        if (lane == 0) s_finish(D, sf, x, b1, b2, (uint32_t)MREP_F_FULLSCAN | extra, tie_rel, invert, qi, o);
    }
}

__global__ void k_seval(DevSurf D, int64_t n, const int32_t* __restrict__ sid, const double* __restrict__ uv,
                        double* __restrict__ xyz)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = sid[i];
    if (c < 0 || c >= D.n_surf) {
        xyz[3 * i] = xyz[3 * i + 1] = xyz[3 * i + 2] = __builtin_nan("");
        return;
    }
    const DSurf sf = D.surfs[c];
    const double* bu = D.brk + sf.brk_off;
    const double* bv = bu + sf.n_su + 1;
    const double u = fmin(fmax(uv[2 * i], bu[0]), bu[sf.n_su]);
    const double v = fmin(fmax(uv[2 * i + 1], bv[0]), bv[sf.n_sv]);
    const int iu = span_of(bu, sf.n_su, u), iv = span_of(bv, sf.n_sv, v);
    const int p = sf.deg_u, q = sf.deg_v;
    const double* cf = D.coef + sf.coef_off + (int64_t)(iu * sf.n_sv + iv) * 3 * (p + 1) * (q + 1);
    const double s = (u - bu[iu]) / (bu[iu + 1] - bu[iu]), t = (v - bv[iv]) / (bv[iv + 1] - bv[iv]);
    for (int x = 0; x < 3; ++x) {
        double acc = 0.0;
        for (int a = p; a >= 0; --a) {
            double d = 0.0;
            for (int b = q; b >= 0; --b) d = d * t + cf[3 * (a * (q + 1) + b) + x];
            acc = acc * s + d;
        }
        xyz[3 * i + x] = acc;
    }
}

// Training-data export: the candidates and their FP32 inputs, by query
__global__ void k_sfeat_write(DevSurf D, const int32_t* __restrict__ sid, const double* __restrict__ qxyz,
                              const int32_t* __restrict__ q_off, const int32_t* __restrict__ perm,
                              const int32_t* __restrict__ cand, int32_t* __restrict__ patch_out,
                              float* __restrict__ x_out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q_off[D.n_surf]) return;
    const int32_t qi = perm[j];
    const DSurf sf = D.surfs[sid[qi]];
    const double q[3] = {qxyz[3 * (int64_t)qi], qxyz[3 * (int64_t)qi + 1], qxyz[3 * (int64_t)qi + 2]};
    for (int k = 0; k < kK; ++k) {
        const int64_t g = cand[j * kK + k];
        float f[kFeat];
        for (int i = 0; i < kFeat; ++i) f[i] = 0.f;
        if (g >= 0) patch_features(D, sf, g, q, f);
        patch_out[(int64_t)qi * kK + k] = g >= 0 ? (int32_t)(g - sf.patch_off) : -1;
        for (int i = 0; i < kFeat; ++i) x_out[((int64_t)qi * kK + k) * kFeat + i] = f[i];
    }
}

__global__ void k_sfeat_fill(int64_t n, int32_t* __restrict__ patch_out, float* __restrict__ x_out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * kK) return;
    patch_out[i] = -1;
    for (int k = 0; k < kFeat; ++k) x_out[i * kFeat + k] = 0.f;
}

struct SWork {
    int32_t *hist, *q_off, *tile_off, *perm, *ovf_list, *ovf_count;
    ScreenOut so;     // per query: its pairs (patches that can hold its minimum)
    float4* res;      // [2 cap] per pair: (s, t, f, kappa) of the patch minimum, then (s, t, f) of a second one
    uint32_t* fub;    // [n] bound on each query's squared distance (float bits)
    // seeded calls
    SphTop top;          // [n][kK] candidates, [n][kK][64] BF16 inputs
    float4* score;       // [n][kK] network outputs
    int32_t* seed_patch; // [n] seeded patch (global) or -1
};

int64_t s_layout(int64_t ns, int64_t n, bool seeded, char* base, SWork* w)
{
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t o = off;
        off = (off + bytes + 255) & ~(int64_t)255;
        return o;
    };
    const int64_t cap = std::min<int64_t>(kSurfPairsPerQuery * n + 1024, (int64_t)INT32_MAX);
    const int64_t oh = take(4 * (ns + 2)), oq = take(4 * (ns + 1)), ot = take(4 * (ns + 1)), op = take(4 * n);
    const int64_t oov = take(4 * n), ocn = take(4 * n), opo = take(4 * n), oub = take(4 * n);
    const int64_t ops = take(4 * cap), opj = take(4 * cap), ors = take(32 * cap);
    const int64_t ofu = take(4 * n);
    const int64_t m = seeded ? n : 0;
    const int64_t oca = take(4 * kK * m), oxb = take(128 * kK * m), osc = take(16 * kK * m), osp = take(4 * m);
    if (w) {
        w->top.cand = seeded ? (int32_t*)(base + oca) : nullptr;
        w->top.xb = seeded ? (uint16_t*)(base + oxb) : nullptr;
        w->score = seeded ? (float4*)(base + osc) : nullptr;
        w->seed_patch = seeded ? (int32_t*)(base + osp) : nullptr;
        w->hist = (int32_t*)(base + oh); w->q_off = (int32_t*)(base + oq); w->tile_off = (int32_t*)(base + ot);
        w->perm = (int32_t*)(base + op); w->ovf_list = (int32_t*)(base + oov);
        w->ovf_count = w->hist + ns;
        w->so.cand_n = (int32_t*)(base + ocn);
        w->so.pair_off = (int32_t*)(base + opo);
        w->so.ub = (float*)(base + oub);
        w->so.pair_seg = (int32_t*)(base + ops);
        w->so.pair_j = (int32_t*)(base + opj);
        w->so.pair_count = w->hist + ns + 1;
        w->so.pair_cap = cap;
        w->res = (float4*)(base + ors);
        w->fub = (uint32_t*)(base + ofu);
    }
    return off;
}

#define S_HIP(expr)                                                               \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));        \
            return MREP_E_HIP;                                                    \
        }                                                                         \
    } while (0)

int32_t run_surf(const char* fn, const mrep_geom* geom, const mrep_nn* nn, const mrep_opts* opts, int64_t n,
                 const int32_t* sid, const double* q, void* ws, int64_t ws_bytes, double* uv_out, double* dist_out,
                 int32_t* patch_out, uint32_t* flags_out, void* stream, int invert)
{
    const std::string f(fn);
    if (!geom || n < 0) {
        set_error(f + ": null geometry or negative n");
        return MREP_E_INVALID_ARG;
    }
    if (geom->kind != MREP_GEOM_SURFACES) {
        set_error(f + ": the geometry holds curves");
        return MREP_E_INVALID_ARG;
    }
    int rc = check_opts(opts);
    if (rc) return rc;
    if (n == 0) return MREP_OK;
    if (n * kSurfPairsPerQuery >= (int64_t)INT32_MAX) {
        set_error(f + ": n must be < 2^31 / 96");
        return MREP_E_INVALID_ARG;
    }
    if (!sid || !q || !ws || !uv_out || !dist_out || !patch_out || !flags_out) {
        set_error(f + ": null pointer");
        return MREP_E_INVALID_ARG;
    }
    const int64_t ns = geom->sg.L.n_surf;
    if (ns == 0) {
        set_error(f + ": geometry has no surfaces");
        return MREP_E_INVALID_ARG;
    }
    const bool seeded = nn != nullptr;
    SWork w;
    if (ws_bytes < s_layout(ns, n, seeded, (char*)ws, &w)) {
        set_error(f + (seeded ? ": workspace smaller than mrep_surface_seeded_workspace_bytes"
                              : ": workspace smaller than mrep_surface_workspace_bytes"));
        return MREP_E_SMALL_BUFFER;
    }
    if (((uintptr_t)ws & 255) != 0) {
        set_error(f + ": workspace not 256-byte aligned");
        return MREP_E_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    const bool timed = (opts->flags & MREP_OPT_TIME_STAGES) != 0;
    if (timed && (rc = stage_begin(st))) return rc;
    int stage = 0;
    const DevSurf D = surf_view(geom->sg);
    const float tie = (float)opts->tie_rel;
    // invalid surface ids are skipped by the grouping and written by k_sbad
    S_HIP(launch_grouping(ns, n, nullptr, sid, w.hist, w.q_off, w.tile_off, w.perm,
                          Outs{nullptr, nullptr, nullptr, nullptr}, st));
    const int64_t tiles = ns + (n + kQueriesPerTile - 1) / kQueriesPerTile + kXcds;
    const int32_t* tq[3] = {w.tile_off, w.q_off, w.perm};
    if (seeded) {
        hipLaunchKernelGGL(k_scand, dim3((unsigned)tiles), dim3(kSphThreads), 0, st, D, tq[0], tq[1], tq[2], q, tie,
                           w.so, w.top);
        S_HIP(hipGetLastError());
        if (timed && (rc = stage_mark(++stage, st))) return rc;
        if ((rc = nn_score_surface_pairs(nn, w.q_off, (int32_t)ns, w.top.cand, w.top.xb, w.score, n * kK, st)))
            return rc;
        if (timed && (rc = stage_mark(++stage, st))) return rc;
        hipLaunchKernelGGL(k_sseed, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, D, sid, q, tq[1], tq[2],
                           (const int32_t*)w.top.cand, (const float4*)w.score, (const float*)w.so.ub, w.fub,
                           w.seed_patch);
        hipLaunchKernelGGL(k_slist<true>, dim3((unsigned)tiles), dim3(kSphThreads), 0, st, D, tq[0], tq[1], tq[2], q,
                           tie, w.so, w.fub);
    } else {
        hipLaunchKernelGGL(k_slist<false>, dim3((unsigned)tiles), dim3(kSphThreads), 0, st, D, tq[0], tq[1], tq[2], q,
                           tie, w.so, w.fub);
        S_HIP(hipGetLastError());
        if (timed && (rc = stage_mark(++stage, st))) return rc;
    }
    const unsigned pb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((w.so.pair_cap + 255) / 256, 8192));
    hipLaunchKernelGGL(k_spairs, dim3(pb), dim3(256), 0, st, D, sid, q, tq[2], w.so, (const uint32_t*)w.fub, tie,
                       w.res);
    S_HIP(hipGetLastError());
    if (timed && (rc = stage_mark(++stage, st))) return rc;
    SOuts o{uv_out, dist_out, patch_out, flags_out};
    hipLaunchKernelGGL(k_sfinish, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, D, sid, q,
                       (const int32_t*)w.q_off, (const int32_t*)w.perm, w.so, (const float4*)w.res, opts->tie_rel,
                       invert, w.ovf_list, w.ovf_count, (const int32_t*)w.seed_patch, o);
    const unsigned fb = (unsigned)std::min<int64_t>((n + 3) / 4, 2048);
    hipLaunchKernelGGL(k_sfull, dim3(fb), dim3(256), 0, st, D, sid, q, (const int32_t*)w.perm,
                       (const int32_t*)w.ovf_list, (const int32_t*)w.ovf_count, opts->tie_rel, invert,
                       seeded ? (uint32_t)MREP_F_NN_FALLBACK : 0u, o);
    S_HIP(hipGetLastError());
    if (timed) {
        if ((rc = stage_mark(++stage, st))) return rc;
        stage_end(stage);
    }
    return MREP_OK;
}

}  // namespace

// invalid surface ids: written before grouping (grouping skips them)
__global__ void k_sbad(int64_t n, int32_t n_surf, const int32_t* __restrict__ sid, double* __restrict__ uv,
                       double* __restrict__ d, int32_t* __restrict__ patch, uint32_t* __restrict__ f)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = sid[i];
    if (c >= 0 && c < n_surf) return;
    const double nan = __builtin_nan("");
    uv[2 * i] = uv[2 * i + 1] = nan;
    d[i] = nan;
    patch[i] = -1;
    f[i] = MREP_F_BAD_ID;
}

extern "C" {

static int32_t surf_ws_bytes(const char* fn, const mrep_geom* geom, int64_t n, const mrep_opts* opts,
                             bool seeded, int64_t* bytes)
{
    if (!geom || !bytes || n < 0) {
        set_error(std::string(fn) + ": null pointer or negative n");
        return MREP_E_INVALID_ARG;
    }
    if (geom->kind != MREP_GEOM_SURFACES) {
        set_error(std::string(fn) + ": the geometry holds curves");
        return MREP_E_INVALID_ARG;
    }
    int rc = check_opts(opts);
    if (rc) return rc;
    *bytes = s_layout(geom->sg.L.n_surf, n, seeded, nullptr, nullptr);
    return MREP_OK;
}

int32_t mrep_surface_workspace_bytes(const mrep_geom* geom, int64_t n, const mrep_opts* opts, int64_t* bytes)
{
    return surf_ws_bytes("mrep_surface_workspace_bytes", geom, n, opts, false, bytes);
}

int32_t mrep_surface_seeded_workspace_bytes(const mrep_geom* geom, int64_t n, const mrep_opts* opts, int64_t* bytes)
{
    return surf_ws_bytes("mrep_surface_seeded_workspace_bytes", geom, n, opts, true, bytes);
}

static int32_t surf_entry(const char* fn, const mrep_geom* geom, const mrep_nn* nn, const mrep_opts* opts, int64_t n,
                          const int32_t* sid, const double* q, void* ws, int64_t ws_bytes, double* uv_out,
                          double* dist_out, int32_t* patch_out, uint32_t* flags_out, void* stream, int invert)
{
    int rc = run_surf(fn, geom, nn, opts, n, sid, q, ws, ws_bytes, uv_out, dist_out, patch_out, flags_out, stream,
                      invert);
    if (rc || n == 0) return rc;
    hipLaunchKernelGGL(k_sbad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n,
                       (int32_t)geom->sg.L.n_surf, sid, uv_out, dist_out, patch_out, flags_out);
    S_HIP(hipGetLastError());
    return MREP_OK;
}

int32_t mrep_project_surfaces(const mrep_geom* geom, const mrep_opts* opts, int64_t n, const int32_t* surface_id,
                              const double* q_xyz, void* workspace, int64_t ws_bytes, double* uv_out,
                              double* dist_out, int32_t* patch_out, uint32_t* flags_out, void* stream)
{
    return surf_entry("mrep_project_surfaces", geom, nullptr, opts, n, surface_id, q_xyz, workspace, ws_bytes, uv_out,
                      dist_out, patch_out, flags_out, stream, 0);
}

int32_t mrep_invert_surfaces(const mrep_geom* geom, const mrep_opts* opts, int64_t n, const int32_t* surface_id,
                             const double* q_xyz, void* workspace, int64_t ws_bytes, double* uv_out, double* dist_out,
                             int32_t* patch_out, uint32_t* flags_out, void* stream)
{
    return surf_entry("mrep_invert_surfaces", geom, nullptr, opts, n, surface_id, q_xyz, workspace, ws_bytes, uv_out,
                      dist_out, patch_out, flags_out, stream, 1);
}

int32_t mrep_project_surfaces_seeded(const mrep_geom* geom, const mrep_nn* nn, const mrep_opts* opts, int64_t n,
                                     const int32_t* surface_id, const double* q_xyz, void* workspace,
                                     int64_t ws_bytes, double* uv_out, double* dist_out, int32_t* patch_out,
                                     uint32_t* flags_out, void* stream)
{
    if (nn_kind(nn) != MREP_NN_SURFACE) {
        set_error("mrep_project_surfaces_seeded: the network is missing or not of kind MREP_NN_SURFACE");
        return MREP_E_INVALID_ARG;
    }
    return surf_entry("mrep_project_surfaces_seeded", geom, nn, opts, n, surface_id, q_xyz, workspace, ws_bytes,
                      uv_out, dist_out, patch_out, flags_out, stream, 0);
}

int32_t mrep_nn_surface_features(const mrep_geom* geom, int64_t n, const int32_t* surface_id, const double* q_xyz,
                                 int32_t* patch_out, float* x_out, void* workspace, int64_t ws_bytes, void* stream)
{
    if (!geom || n < 0 || geom->kind != MREP_GEOM_SURFACES) {
        set_error("mrep_nn_surface_features: null or curve geometry, or negative n");
        return MREP_E_INVALID_ARG;
    }
    if (n == 0) return MREP_OK;
    if (!surface_id || !q_xyz || !patch_out || !x_out || !workspace) {
        set_error("mrep_nn_surface_features: null pointer");
        return MREP_E_INVALID_ARG;
    }
    const int64_t ns = geom->sg.L.n_surf;
    if (n * kSurfPairsPerQuery >= (int64_t)INT32_MAX || ns == 0) {
        set_error("mrep_nn_surface_features: n must be < 2^31 / 96 and the geometry non-empty");
        return MREP_E_INVALID_ARG;
    }
    SWork w;
    if (ws_bytes < s_layout(ns, n, true, (char*)workspace, &w)) {
        set_error("mrep_nn_surface_features: workspace smaller than mrep_surface_seeded_workspace_bytes");
        return MREP_E_SMALL_BUFFER;
    }
    if (((uintptr_t)workspace & 255) != 0) {
        set_error("mrep_nn_surface_features: workspace not 256-byte aligned");
        return MREP_E_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    const DevSurf D = surf_view(geom->sg);
    hipLaunchKernelGGL(k_sfeat_fill, dim3((unsigned)((n * kK + 255) / 256)), dim3(256), 0, st, n, patch_out, x_out);
    S_HIP(launch_grouping(ns, n, nullptr, surface_id, w.hist, w.q_off, w.tile_off, w.perm,
                          Outs{nullptr, nullptr, nullptr, nullptr}, st));
    const int64_t tiles = ns + (n + kQueriesPerTile - 1) / kQueriesPerTile + kXcds;
    hipLaunchKernelGGL(k_scand, dim3((unsigned)tiles), dim3(kSphThreads), 0, st, D, (const int32_t*)w.tile_off,
                       (const int32_t*)w.q_off, (const int32_t*)w.perm, q_xyz, 2e-6f, w.so,
                       SphTop{w.top.cand, nullptr});
    hipLaunchKernelGGL(k_sfeat_write, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, D, surface_id, q_xyz,
                       (const int32_t*)w.q_off, (const int32_t*)w.perm, (const int32_t*)w.top.cand, patch_out, x_out);
    S_HIP(hipGetLastError());
    return MREP_OK;
}

int32_t mrep_eval_surfaces(const mrep_geom* geom, int64_t n, const int32_t* surface_id, const double* uv,
                           double* xyz_out, void* stream)
{
    if (!geom || n < 0 || (n > 0 && (!surface_id || !uv || !xyz_out))) {
        set_error("mrep_eval_surfaces: null pointer or negative n");
        return MREP_E_INVALID_ARG;
    }
    if (geom->kind != MREP_GEOM_SURFACES) {
        set_error("mrep_eval_surfaces: the geometry holds curves");
        return MREP_E_INVALID_ARG;
    }
    if (n == 0) return MREP_OK;
    hipLaunchKernelGGL(k_seval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       surf_view(geom->sg), n, surface_id, uv, xyz_out);
    S_HIP(hipGetLastError());
    return MREP_OK;
}

}  // extern "C"
