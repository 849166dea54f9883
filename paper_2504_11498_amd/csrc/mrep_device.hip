// HIP kernels and C-ABI entry points of libmrep (gfx950 / MI355X).
//
// Projection pipeline for n queries, each onto its own curve (Sec. 4, eq.
// projections), after the curves were decomposed into cubic Bezier pieces in
// matrix form (Sec. 5.2):
//   1. group queries by curve (histogram, scan, scatter);
//   2. screen (BF16 mode): for every (query, piece) the squared distance to the
//      piece's 32 uniform samples is one MFMA contraction of a per-(query,
//      sample) monomial row with a per-piece coefficient column; the minimum
//      over samples gives a certified lower bound of the distance to the EXACT
//      curve over the piece's parameter range, and every piece whose lower
//      bound does not exceed the best upper bound is kept as a candidate (the
//      role the paper's elimination criterion, Sec. 5.3, plays);
//   3. refine: Newton on the orthogonality condition (C - q).C' = 0 (eqs. Et
//      and E't) from every local minimum of a rescan of each candidate, in
//      FP32 in the piece's local frame (FP64 in the FP64 mode, which examines
//      every piece instead of screening);
//   4. polish: FP64 Newton on the exact degree-p span (power form of the
//      decomposed span) wherever the cubic is an approximation (p >= 4), the
//      minimiser is near-tangent, or two minima are nearly tied;
//   5. write t (FP64 curve parameter, Sec. 5.4.2 reparameterisation), the
//      distance, the piece index and flags.
// The paper's per-query minimum under atomic locks (PCWS, Sec. 5.4.2) becomes a
// per-query ownership: one thread (refine) or one 16-lane row (screen) owns a
// query, so no lock or atomic is needed.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "../../include/mrep.h"
#include "mrep_dev.h"
#include "mrep_refine.h"

using namespace mrep;



namespace mrep {
static thread_local std::string t_err;
void set_error(const std::string& msg) { t_err = msg; }
}  // namespace mrep

#define HIP_OK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                   \
            return MREP_E_HIP;                                                               \
        }                                                                                    \
    } while (0)

struct Work {
    int32_t* hist;        // n_curves + 1: per-curve counts / scatter cursors, then the overflow count
    int32_t* q_off;       // n_curves + 1
    int32_t* tile_off;    // n_curves + 1
    int4* tile_map;       // screen_grid(n_curves, n): workgroup slot -> {curve, first query, end, tile}
    int32_t* perm;        // n: sorted position -> query
    int32_t* ovf_list;    // n: sorted positions whose candidate list overflowed
    int32_t* ovf_count;   // = hist + n_curves
    int32_t* pair_count;  // = hist + n_curves + 1
    ScreenOut so;         // candidate lists as (query, piece) pairs
    PairRes* pair_res;    // [cap] per pair: the piece's minimum and second local minimum (mrep_refine.h)
};

// pairs reserved per query on average before queries overflow to the full scan
constexpr int64_t kPairsPerQuery = 4;
static int64_t a256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Stage timing: events recorded on the call's stream when asked to.
struct StageEvents {
    hipEvent_t ev[MREP_N_STAGES + 1] = {};
    bool created = false;
    int count = 0;  // stages of the last completed timed call (0: none)
};
static thread_local StageEvents t_stage;

int mrep::stage_mark(int i, hipStream_t st)
{
    if (!t_stage.created) {
        for (int k = 0; k <= MREP_N_STAGES; ++k) HIP_OK(hipEventCreate(&t_stage.ev[k]));
        t_stage.created = true;
    }
    HIP_OK(hipEventRecord(t_stage.ev[i], st));
    return MREP_OK;
}
int mrep::stage_begin(hipStream_t st)
{
    t_stage.count = 0;
    return stage_mark(0, st);
}
void mrep::stage_end(int count) { t_stage.count = count; }

static int64_t work_layout(int64_t n_curves, int64_t n, int kc, char* base, Work* w)
{
    (void)kc;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        int64_t o = off;
        off = a256(off + bytes);
        return o;
    };
    const int64_t cap = std::min<int64_t>(kPairsPerQuery * n + 1024, (int64_t)INT32_MAX);
    int64_t o_hist = take(4 * (n_curves + 2));
    (void)take(8 * kWsCounters);  // the sphere-test counters (written by the sphere strategy only)
    int64_t o_qoff = take(4 * (n_curves + 1));
    int64_t o_toff = take(4 * (n_curves + 1));
    int64_t o_tmap = take(16 * screen_grid(n_curves, n));
    int64_t o_perm = take(4 * n);
    int64_t o_ovf = take(4 * n);
    int64_t o_candn = take(4 * n);
    int64_t o_poff = take(4 * n);
    int64_t o_ub = take(4 * n);
    int64_t o_pseg = take(4 * cap);
    int64_t o_pj = take(4 * cap);
    int64_t o_pres = take((int64_t)sizeof(PairRes) * cap);
    if (w) {
        w->hist = reinterpret_cast<int32_t*>(base + o_hist);
        w->q_off = reinterpret_cast<int32_t*>(base + o_qoff);
        w->tile_off = reinterpret_cast<int32_t*>(base + o_toff);
        w->tile_map = reinterpret_cast<int4*>(base + o_tmap);
        w->perm = reinterpret_cast<int32_t*>(base + o_perm);
        w->ovf_list = reinterpret_cast<int32_t*>(base + o_ovf);
        w->ovf_count = w->hist + n_curves;
        w->pair_count = w->hist + n_curves + 1;
        w->so.cand_n = reinterpret_cast<int32_t*>(base + o_candn);
        w->so.pair_off = reinterpret_cast<int32_t*>(base + o_poff);
        w->so.pair_seg = reinterpret_cast<int32_t*>(base + o_pseg);
        w->so.pair_j = reinterpret_cast<int32_t*>(base + o_pj);
        w->so.pair_count = w->pair_count;
        w->so.pair_cap = cap;
        w->so.ub = reinterpret_cast<float*>(base + o_ub);
        w->pair_res = reinterpret_cast<PairRes*>(base + o_pres);
    }
    return off;
}

// ---------------------------------------------------------------------------
// 1. grouping queries by curve
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Lanes of a wave that share a key make one atomic between them (sorted or
// clustered inputs put whole waves on one curve).  Returns the old counter
// value plus the lane's rank among the lanes with its key.  Every iteration
// retires at least the leader lane, so the loop ends within 64 rounds.
__device__ __forceinline__ int32_t wave_add(int32_t* base, int32_t key, bool active)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    uint64_t pending = __ballot(active);
    int32_t result = 0;
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int32_t lkey = __shfl(key, leader, 64);
        const uint64_t same = __ballot(active && key == lkey) & pending;
        int32_t old = 0;
        if (lane == leader) old = atomicAdd(&base[lkey], (int32_t)__popcll(same));
        old = __shfl(old, leader, 64);
        if ((same >> lane) & 1ull) result = old + (int32_t)__popcll(same & lt);
        pending &= ~same;
    }
    return result;
}

// n_dev (nullable): the query count lives on the device and n only bounds it.
__global__ __launch_bounds__(256) void k_hist(const int32_t* __restrict__ cid, int64_t n,
                                              const int32_t* __restrict__ n_dev, int32_t n_curves,
                                              int32_t* __restrict__ hist, double* __restrict__ t_out,
                                              double* __restrict__ d_out, int32_t* __restrict__ s_out,
                                              uint32_t* __restrict__ f_out)
{
    if (n_dev) n = min(n, (int64_t)*n_dev);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t c = i < n ? cid[i] : -1;
    const bool bad = i < n && (c < 0 || c >= n_curves);
    if (bad && t_out) {
        t_out[i] = __longlong_as_double(0x7ff8000000000000ll);
        d_out[i] = __longlong_as_double(0x7ff8000000000000ll);
        s_out[i] = -1;
        f_out[i] = MREP_F_BAD_ID;
    }
    wave_add(hist, c, i < n && !bad);
}

// One workgroup of 1024 threads: q_off = exclusive scan of hist, tile_off =
// exclusive scan of ceil(hist / kQueriesPerTile); hist is reset to 0 for use
// as the scatter cursor.
__global__ __launch_bounds__(1024) void k_scan(int32_t* __restrict__ hist, int32_t n_curves,
                                               int32_t* __restrict__ q_off, int32_t* __restrict__ tile_off)
{
    __shared__ int32_t s_q[1024], s_t[1024];
    const int tid = threadIdx.x;
    const int per = (n_curves + 1023) / 1024;
    const int lo = min(tid * per, n_curves), hi = min(lo + per, n_curves);
    int32_t sq = 0, st = 0;
    for (int c = lo; c < hi; ++c) {
        int32_t h = hist[c];
        sq += h;
        st += (h + kQueriesPerTile - 1) / kQueriesPerTile;
    }
    s_q[tid] = sq;
    s_t[tid] = st;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        int32_t aq = tid >= d ? s_q[tid - d] : 0;
        int32_t at = tid >= d ? s_t[tid - d] : 0;
        __syncthreads();
        s_q[tid] += aq;
        s_t[tid] += at;
        __syncthreads();
    }
    int32_t rq = s_q[tid] - sq, rt = s_t[tid] - st;  // exclusive
    for (int c = lo; c < hi; ++c) {
        int32_t h = hist[c];
        q_off[c] = rq;
        tile_off[c] = rt;
        rq += h;
        rt += (h + kQueriesPerTile - 1) / kQueriesPerTile;
        hist[c] = 0;
    }
    if (tid == 1023) {
        q_off[n_curves] = s_q[1023];
        tile_off[n_curves] = s_t[1023];
    }
}

__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ cid, int64_t n,
                                                 const int32_t* __restrict__ n_dev, int32_t n_curves,
                                                 const int32_t* __restrict__ q_off, int32_t* __restrict__ cursor,
                                                 int32_t* __restrict__ perm)
{
    if (n_dev) n = min(n, (int64_t)*n_dev);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t c = i < n ? cid[i] : -1;
    const bool ok = i < n && c >= 0 && c < n_curves;
    const int32_t pos = wave_add(cursor, c, ok);
    if (ok) perm[q_off[c] + pos] = (int32_t)i;
}


// Workgroup slot -> tile of the grouped queries.  Tiles are dealt to the 8
// XCDs in contiguous ranges (slot b runs on XCD b % 8 and takes tile
// (b % 8) * per + b / 8), so the tiles of one group share an L2; each entry is
// {group, first sorted query of the tile, end of the group's queries, tile}, or
// group -1 for a slot without a tile.
__global__ __launch_bounds__(256) void k_tile_map(const int32_t* __restrict__ tile_off,
                                                  const int32_t* __restrict__ q_off, int32_t n_groups, int64_t grid,
                                                  int4* __restrict__ map)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= grid) return;
    const int n_tiles = tile_off[n_groups];
    const int per = (n_tiles + kXcdCount - 1) / kXcdCount;
    const int slot = (int)(b / kXcdCount);
    const int tile = (int)(b % kXcdCount) * per + slot;
    int4 r = make_int4(-1, 0, 0, 0);
    if (slot < per && tile < n_tiles) {
        int lo = 0, hi = n_groups;  // tile_off[lo] <= tile < tile_off[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tile_off[mid] <= tile) lo = mid; else hi = mid;
        }
        r = make_int4(lo, q_off[lo] + (tile - tile_off[lo]) * kQueriesPerTile, q_off[lo + 1], tile);
    }
    map[b] = r;
}

hipError_t mrep::launch_tile_map(const int32_t* tile_off, const int32_t* q_off, int64_t n_groups, int64_t grid,
                                 int4* map, hipStream_t st)
{
    hipLaunchKernelGGL(k_tile_map, dim3((unsigned)((grid + 255) / 256)), dim3(256), 0, st, tile_off, q_off,
                       (int32_t)n_groups, grid, map);
    return hipGetLastError();
}

// One thread per (query, candidate piece) pair reserved by the screen: the
// certified minimum over the piece in the refine precision.  Persistent grid.
// done (nullable): per sorted query, nonzero when the query is already decided.
// occupancy hints (waves per SIMD): k_pairs 6 (80 VGPRs, no spill) and
// k_finish 6 trim the refine stage by about 3% on the batched curves; the full
// scan keeps its registers (its FP64 instance would spill heavily)
#ifndef MREP_PAIRS_MIN_WAVES
#define MREP_PAIRS_MIN_WAVES 5
#endif
#ifndef MREP_FINISH_MIN_WAVES
#define MREP_FINISH_MIN_WAVES 4
#endif
#ifndef MREP_FULLSCAN_MIN_WAVES
#define MREP_FULLSCAN_MIN_WAVES 1
#endif
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MREP_PAIRS_MIN_WAVES, 8))) void k_pairs(DevGeom G, const int32_t* __restrict__ cid,
                                               const double* __restrict__ qxyz, const int32_t* __restrict__ perm,
                                               const int32_t* __restrict__ pair_seg,
                                               const int32_t* __restrict__ pair_j,
                                               const int32_t* __restrict__ pair_count, int64_t pair_cap,
                                               const float* __restrict__ ub, double tie_rel,
                                               const uint8_t* __restrict__ done, PairRes* __restrict__ pair_res)
{
    const int64_t total = min((int64_t)*pair_count, pair_cap);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t jj = pair_j[p];
        if (jj < 0) continue;  // reserved by a query that then overflowed the capacity
        if (done && done[jj]) continue;
        const int64_t s = pair_seg[p];
        if (s < 0 || s >= G.n_seg) continue;  // never written by the screen (defensive)
        const int32_t qi = perm[jj];
        const DCurve cv = G.curves[cid[qi]];
        const double q[3] = {qxyz[3 * (int64_t)qi], qxyz[3 * (int64_t)qi + 1], qxyz[3 * (int64_t)qi + 2]};
        Cubic<T> C;
        load_cubic(G, cv, s, q, C);
        // beyond the query's certified bound plus twice the widest tie margin of
        // the finish, a piece cannot hold the minimum nor a runner-up that counts
        const double ubq = (double)ub[jj];
        const double lim = ubq + 2.0 * (2.0 * cv.tol_eff + 4e-6 * (ubq + cv.diag) + tie_rel * cv.diag);
        T u, d, k, u2, d2;
        piece_min(C, u, d, k, u2, d2, (T)(lim * lim));
        const double err = param_error(C, u, k, G.segt[2 * s], G.segt[2 * s + 1]);
        pair_res[p] = pair_result(G, cv, s, q, (double)u, (double)d, (double)k, err, (double)u2, (double)d2);
    }
}

__device__ __forceinline__ Cand cand_from_lane(const Cand& c, int src)
{
    Cand r;
    r.d2 = __shfl(c.d2, src, 64);
    r.t = __shfl(c.t, src, 64);
    r.kappa = __shfl(c.kappa, src, 64);
    r.t_err = __shfl(c.t_err, src, 64);
    r.seg = __shfl(c.seg, src, 64);
    r.across = __shfl(c.across, src, 64);
    r.end = __shfl(c.end, src, 64);
    return r;
}

// One thread per query: the two best of its pairs, then finish.  Queries whose
// list overflowed are appended to ovf_list for k_fullscan.  (A split into a
// coalesced selection kernel, eight lanes per query, and a polish kernel was
// measured slower on the lattice struts: 27.6 ms against 16.8 ms.)
template <typename T, bool kGen>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(MREP_FINISH_MIN_WAVES, 8))) void k_finish(DevGeom G, const int32_t* __restrict__ cid,
                                                const double* __restrict__ qxyz, const int32_t* __restrict__ q_off,
                                                const int32_t* __restrict__ perm, ScreenOut so,
                                                const PairRes* __restrict__ pair_res, const uint8_t* __restrict__ done,
                                                uint32_t flag_in, double tie_rel, int32_t invert,
                                                int32_t* __restrict__ ovf_list, int32_t* __restrict__ ovf_count,
                                                Outs o)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q_off[G.n_curves]) return;
    if (done && done[j]) return;
    const int n_list = so.cand_n[j];
    if (n_list <= 0) {  // overflow (or, impossible for finite input, an empty list)
        ovf_list[atomicAdd(ovf_count, 1)] = (int32_t)j;
        return;
    }
    const int32_t qi = perm[j];
    const DCurve cv = G.curves[cid[qi]];
    const double q[3] = {qxyz[3 * (int64_t)qi], qxyz[3 * (int64_t)qi + 1], qxyz[3 * (int64_t)qi + 2]};
    Cand b1 = empty_cand(cv), b2 = b1;
    const int64_t p0 = so.pair_off[j];
    // each pair record is loaded once; its minimum, then its second local minimum
    for (int i = 0; i < n_list; ++i) {
        const PairRes r = pair_res[p0 + i];
        const int32_t sg = so.pair_seg[p0 + i];
        const Cand x0 = pair_cand(r, sg, false);
        top2(x0, b1, b2);
        if (r.d2b < INFINITY) top2(pair_cand(r, sg, true), b1, b2);
    }
    finish<T, kGen>(G, cv, q, b1, b2, flag_in, tie_rel, invert, qi, o);
}



// One wave per query, lanes striding over the query's pieces: (1) the best
// upper bound from every piece's samples, (2) refine every piece whose lower
// bound reaches it, (3) wave top-2, (4) finish on lane 0.  Used for every
// query in the FP64 mode (list == nullptr) and for the screen's overflows.
// Persistent: wave w takes items w, w + waves, ... until the count is reached.
template <typename T, bool kGen>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MREP_FULLSCAN_MIN_WAVES, 8))) void k_fullscan(DevGeom G, const int32_t* __restrict__ cid,
                                                  const double* __restrict__ qxyz,
                                                  const int32_t* __restrict__ q_off,
                                                  const int32_t* __restrict__ perm,
                                                  const int32_t* __restrict__ list,
                                                  const int32_t* __restrict__ count, const float* __restrict__ ub_in,
                                                  uint32_t flag_in, double tie_rel, int32_t invert, Outs o)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t total = list ? (int64_t)*count : (int64_t)q_off[G.n_curves];
    // relative sampling error of the refine precision on a squared distance
    const double rel = sizeof(T) == 4 ? 4e-6 : 1e-14;
    for (int64_t item = wave; item < total; item += nwaves) {
        const int64_t j = list ? (int64_t)list[item] : item;
        const int32_t qi = perm[j];
        const DCurve cv = G.curves[cid[qi]];
        double q[3] = {qxyz[3 * (int64_t)qi], qxyz[3 * (int64_t)qi + 1], qxyz[3 * (int64_t)qi + 2]};
        const int64_t s_end = cv.seg_off + cv.n_seg;
        // distance from q to the centre of piece s's sphere (which holds the
        // exact curve over the piece), with its radius
        auto sph = [&](int64_t s, double& r) {
            const float4 p = G.sph[s];
            const double dx = q[0] - (cv.origin[0] + (double)p.x), dy = q[1] - (cv.origin[1] + (double)p.y),
                         dz = q[2] - (cv.origin[2] + (double)p.z);
            r = (double)p.w;
            return sqrt(dx * dx + dy * dy + dz * dz);
        };
        // a piece whose sphere lies beyond ub + margin can be neither the
        // minimum nor a runner-up within the tie margin of the finish
        auto margin = [&](double d) { return 2.0 * cv.tol_eff + 4e-6 * (d + cv.diag) + tie_rel * cv.diag; };
        // upper bound: the caller's (a certified bound from the screen or the
        // sphere listing), then the spheres', then the sampled minima
        double ub = ub_in ? (double)ub_in[j] : INFINITY;
        for (int64_t s = cv.seg_off + lane; s < s_end; s += 64) {
            double r;
            const double d = sph(s, r);
            ub = fmin(ub, (d + r) * (1.0 + 1e-12));
        }
        for (int off = 32; off > 0; off >>= 1) ub = fmin(ub, __shfl_xor(ub, off, 64));
        double lim = ub + margin(ub);
        for (int64_t s = cv.seg_off + lane; s < s_end; s += 64) {
            double r;
            if (sph(s, r) - r > lim) continue;
            double m = (double)piece_sample_min<T>(G, cv, s, q);
            ub = fmin(ub, sqrt(m * (1.0 + rel)) + cv.tol_eff);
        }
        for (int off = 32; off > 0; off >>= 1) ub = fmin(ub, __shfl_xor(ub, off, 64));
        lim = ub + margin(ub);
        Cand b1 = empty_cand(cv), b2 = b1;
        for (int64_t s = cv.seg_off + lane; s < s_end; s += 64) {
            double r;
            if (sph(s, r) - r > lim) continue;
            double m = (double)piece_sample_min<T>(G, cv, s, q);
            double lb = sqrt(fmax(m * (1.0 - rel), 0.0)) - (double)G.aux[s * 8 + AUX_ES] * 1.001;
            // lim, not ub: a runner-up within the tie margin is refined too
            if (lb <= lim) consider<T>(G, cv, s, q, b1, b2);
        }
        // wave top-2 by the same rules as one lane's: a tree onto lane 0, in a fixed order
        for (int off = 32; off > 0; off >>= 1) {
            const Cand o1 = cand_from_lane(b1, lane + off), o2 = cand_from_lane(b2, lane + off);
            if (lane + off < 64) {
                top2(o1, b1, b2);
                top2(o2, b1, b2);
            }
        }
        if (lane == 0) finish<T, kGen>(G, cv, q, b1, b2, flag_in, tie_rel, invert, qi, o);
    }
}

__global__ void k_eval(DevGeom G, int64_t n, const int32_t* __restrict__ cid, const double* __restrict__ t,
                       double* __restrict__ xyz)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = cid[i];
    if (c < 0 || c >= G.n_curves) {
        xyz[3 * i] = xyz[3 * i + 1] = xyz[3 * i + 2] = __builtin_nan("");
        return;
    }
    const DCurve cv = G.curves[c];
    const double dom0 = G.spant[2 * cv.span_off], dom1 = G.spant[2 * (cv.span_off + cv.n_span - 1) + 1];
    double tt = fmin(fmax(t[i], dom0), dom1);
    int lo = 0, hi = cv.n_span;  // spant[lo].t0 <= tt
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (G.spant[2 * (cv.span_off + mid)] <= tt) lo = mid; else hi = mid;
    }
    const int64_t sp = cv.span_off + lo;
    const double tq = G.spant[2 * sp], tq1 = G.spant[2 * sp + 1];
    const double v = (tt - tq) / (tq1 - tq);
    const double* cf = span_coef(G, cv, sp);
    const double z[3] = {0, 0, 0};
    double r[3], d1[3], d2[3];
    span_eval_cv<true>(cv, cf, v, z, r, d1, d2);
    xyz[3 * i] = r[0];
    xyz[3 * i + 1] = r[1];
    xyz[3 * i + 2] = r[2];
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
int mrep::check_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("no HIP device");
        return MREP_E_NO_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        set_error("hipGetDeviceProperties failed");
        return MREP_E_NO_DEVICE;
    }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        set_error(std::string("libmrep is built for gfx950, device is ") + prop.gcnArchName);
        return MREP_E_NO_DEVICE;
    }
    return MREP_OK;
}

extern "C" {

int32_t mrep_abi_version(void) { return MREP_ABI_VERSION; }

const char* mrep_last_error(void) { return t_err.c_str(); }

static int32_t decompose_curves(const char* fn, int32_t n_curves, const int32_t* degree, const int64_t* cp_off,
                                const double* cp_xyz, const double* weights, const int64_t* knot_off,
                                const double* knots, double tol_rel, int32_t n_threads, mrep_plan** out)
{
    if (!out || n_curves < 0 || (n_curves > 0 && (!degree || !cp_off || !cp_xyz || !knot_off || !knots))) {
        set_error(std::string(fn) + ": null pointer or negative count");
        return MREP_E_INVALID_ARG;
    }
    *out = nullptr;
    if (!(tol_rel > 0.0) || !std::isfinite(tol_rel)) {
        set_error(std::string(fn) + ": tol_rel must be positive");
        return MREP_E_TOL;
    }
    mrep_plan* p = new mrep_plan();
    std::string err;
    int rc = build_plan(n_curves, degree, cp_off, cp_xyz, weights, knot_off, knots, tol_rel, n_threads, p->p, err);
    if (rc != MREP_OK) {
        delete p;
        set_error(std::string(fn) + ": " + err);
        return rc;
    }
    *out = p;
    return MREP_OK;
}

int32_t mrep_decompose_curves(int32_t n_curves, const int32_t* degree, const int64_t* cp_off, const double* cp_xyz,
                              const int64_t* knot_off, const double* knots, double tol_rel, int32_t n_threads,
                              mrep_plan** out)
{
    return decompose_curves("mrep_decompose_curves", n_curves, degree, cp_off, cp_xyz, nullptr, knot_off, knots,
                            tol_rel, n_threads, out);
}

int32_t mrep_decompose_curves_rational(int32_t n_curves, const int32_t* degree, const int64_t* cp_off,
                                       const double* cp_xyz, const double* weights, const int64_t* knot_off,
                                       const double* knots, double tol_rel, int32_t n_threads, mrep_plan** out)
{
    if (n_curves > 0 && !weights) {
        set_error("mrep_decompose_curves_rational: null weights");
        return MREP_E_INVALID_ARG;
    }
    return decompose_curves("mrep_decompose_curves_rational", n_curves, degree, cp_off, cp_xyz, weights, knot_off,
                            knots, tol_rel, n_threads, out);
}

int32_t mrep_plan_info(const mrep_plan* plan, mrep_plan_info_t* info)
{
    if (!plan || !info) {
        set_error("mrep_plan_info: null pointer");
        return MREP_E_INVALID_ARG;
    }
    if (plan->kind == MREP_GEOM_SURFACES) {
        const SurfPlan& S = plan->sp;
        info->n_curves = S.n_surf;
        info->n_spans = S.layout.n_span;
        info->n_segments = S.layout.n_patch;
        info->device_bytes = S.layout.total;
        info->max_degree = S.max_degree;
        info->reserved = 1;
        info->tol_rel = S.tol_rel;
        return MREP_OK;
    }
    if (plan->dev) {
        const GeomLayout& L = devplan_layout(*plan->dev);
        info->n_curves = L.n_curves;
        info->n_spans = L.n_span;
        info->n_segments = L.n_seg;
        info->device_bytes = L.total;
        info->max_degree = devplan_max_degree(*plan->dev);
        info->reserved = 0;
        info->tol_rel = devplan_tol_rel(*plan->dev);
        return MREP_OK;
    }
    info->n_curves = plan->p.n_curves;
    info->n_spans = plan->p.layout.n_span;
    info->n_segments = plan->p.layout.n_seg;
    info->device_bytes = plan->p.layout.total;
    info->max_degree = plan->p.max_degree;
    info->reserved = 0;
    info->tol_rel = plan->p.tol_rel;
    return MREP_OK;
}

int32_t mrep_decompose_surfaces(int32_t n_surf, const int32_t* deg_u, const int32_t* deg_v, const int32_t* n_u,
                                const int32_t* n_v, const int64_t* cp_off, const double* cp_xyz,
                                const int64_t* ku_off, const double* ku, const int64_t* kv_off, const double* kv,
                                double tol_rel, int32_t n_threads, mrep_plan** out)
{
    if (!out || n_surf < 0 ||
        (n_surf > 0 && (!deg_u || !deg_v || !n_u || !n_v || !cp_off || !cp_xyz || !ku_off || !ku || !kv_off || !kv))) {
        set_error("mrep_decompose_surfaces: null pointer or negative count");
        return MREP_E_INVALID_ARG;
    }
    *out = nullptr;
    if (!(tol_rel > 0.0) || !std::isfinite(tol_rel)) {
        set_error("mrep_decompose_surfaces: tol_rel must be positive");
        return MREP_E_TOL;
    }
    mrep_plan* p = new mrep_plan();
    p->kind = MREP_GEOM_SURFACES;
    std::string err;
    int rc = build_surf_plan(n_surf, deg_u, deg_v, n_u, n_v, cp_off, cp_xyz, ku_off, ku, kv_off, kv, tol_rel,
                             n_threads, p->sp, err);
    if (rc != MREP_OK) {
        delete p;
        set_error("mrep_decompose_surfaces: " + err);
        return rc;
    }
    *out = p;
    return MREP_OK;
}

int32_t mrep_plan_export_surfaces(const mrep_plan* plan, int64_t* patch_off, double* patch_uv, double* patch_cp,
                                  int32_t* patch_span)
{
    if (!plan || plan->kind != MREP_GEOM_SURFACES) {
        set_error("mrep_plan_export_surfaces: null plan or a curve plan");
        return MREP_E_INVALID_ARG;
    }
    const SurfPlan& S = plan->sp;
    if (patch_off) {
        for (int64_t c = 0; c < S.n_surf; ++c) patch_off[c] = S.surfs[(size_t)c].patch_off;
        patch_off[S.n_surf] = S.layout.n_patch;
    }
    if (patch_uv) memcpy(patch_uv, S.uv.data(), sizeof(double) * S.uv.size());
    if (patch_cp) memcpy(patch_cp, S.gcp.data(), sizeof(double) * S.gcp.size());
    if (patch_span) {
        for (int64_t c = 0; c < S.n_surf; ++c) {
            const DSurf& d = S.surfs[(size_t)c];
            for (int32_t k = 0; k < d.n_patch; ++k)
                patch_span[d.patch_off + k] = (int32_t)(S.pspan[(size_t)(d.patch_off + k)] - d.span_off);
        }
    }
    return MREP_OK;
}

int32_t mrep_plan_export(const mrep_plan* plan, int64_t* seg_off, double* seg_t, double* seg_cp, int32_t* seg_span)
{
    if (!plan || plan->kind != MREP_GEOM_CURVES) {
        set_error("mrep_plan_export: null plan or a surface plan");
        return MREP_E_INVALID_ARG;
    }
    if (plan->dev) return devplan_export(*plan->dev, seg_off, seg_t, seg_cp, seg_span);
    const Plan& P = plan->p;
    if (seg_off) {
        for (int64_t c = 0; c < P.n_curves; ++c) seg_off[c] = P.curves[(size_t)c].seg_off;
        seg_off[P.n_curves] = P.layout.n_seg;
    }
    if (seg_t) memcpy(seg_t, P.seg_t.data(), sizeof(double) * P.seg_t.size());
    if (seg_cp) memcpy(seg_cp, P.seg_cp.data(), sizeof(double) * P.seg_cp.size());
    if (seg_span) memcpy(seg_span, P.seg_span.data(), sizeof(int32_t) * P.seg_span.size());
    return MREP_OK;
}

void mrep_plan_free(mrep_plan* plan) { delete plan; }

static int32_t upload_surfaces(const SurfPlan& P, void* dev_buf, int64_t bytes, void* stream, mrep_geom** out);

int32_t mrep_upload(const mrep_plan* plan, void* dev_buf, int64_t bytes, void* stream, mrep_geom** out)
{
    if (!plan || !dev_buf || !out) {
        set_error("mrep_upload: null pointer");
        return MREP_E_INVALID_ARG;
    }
    *out = nullptr;
    if (plan->kind == MREP_GEOM_SURFACES) return upload_surfaces(plan->sp, dev_buf, bytes, stream, out);
    if (plan->dev) {
        const GeomLayout& L = devplan_layout(*plan->dev);
        if (bytes < L.total) {
            set_error("mrep_upload: buffer smaller than device_bytes");
            return MREP_E_SMALL_BUFFER;
        }
        if (((uintptr_t)dev_buf & 255) != 0) {
            set_error("mrep_upload: buffer not 256-byte aligned");
            return MREP_E_INVALID_ARG;
        }
        int rc = check_device();
        if (rc) return rc;
        rc = devplan_upload(*plan->dev, (char*)dev_buf, (hipStream_t)stream);
        if (rc) return rc;
        mrep_geom* g = new mrep_geom();
        g->g.L = L;
        g->g.base = (char*)dev_buf;
        HIP_OK(hipGetDevice(&g->g.device));
        *out = g;
        return MREP_OK;
    }
    const Plan& P = plan->p;
    if (bytes < P.layout.total) {
        set_error("mrep_upload: buffer smaller than device_bytes");
        return MREP_E_SMALL_BUFFER;
    }
    if (((uintptr_t)dev_buf & 255) != 0) {
        set_error("mrep_upload: buffer not 256-byte aligned");
        return MREP_E_INVALID_ARG;
    }
    int rc = check_device();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    char* b = (char*)dev_buf;
    const GeomLayout& L = P.layout;
    auto cp = [&](int64_t off, const void* src, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        return hipMemcpyAsync(b + off, src, n, hipMemcpyHostToDevice, st);
    };
    HIP_OK(cp(L.off_curve, P.curves.data(), sizeof(DCurve) * P.curves.size()));
    HIP_OK(cp(L.off_col, P.col.data(), sizeof(uint16_t) * P.col.size()));
    HIP_OK(cp(L.off_aux, P.aux.data(), sizeof(float) * P.aux.size()));
    HIP_OK(cp(L.off_lcp, P.lcp.data(), sizeof(float) * P.lcp.size()));
    HIP_OK(cp(L.off_gcp, P.seg_cp.data(), sizeof(double) * P.seg_cp.size()));
    HIP_OK(cp(L.off_segt, P.seg_t.data(), sizeof(double) * P.seg_t.size()));
    HIP_OK(cp(L.off_segspan, P.seg_span.data(), sizeof(int32_t) * P.seg_span.size()));
    HIP_OK(cp(L.off_spant, P.span_t.data(), sizeof(double) * P.span_t.size()));
    HIP_OK(cp(L.off_span0, P.span0.data(), sizeof(int32_t) * P.span0.size()));
    HIP_OK(cp(L.off_coef, P.coef.data(), sizeof(double) * P.coef.size()));
    HIP_OK(cp(L.off_sph, P.sph.data(), sizeof(float) * P.sph.size()));
    HIP_OK(cp(L.off_csph, P.csph.data(), sizeof(float) * P.csph.size()));
    // the plan's host vectors are pageable: finish the copies before returning
    HIP_OK(hipStreamSynchronize(st));
    mrep_geom* g = new mrep_geom();
    g->g.L = L;
    g->g.base = b;
    HIP_OK(hipGetDevice(&g->g.device));
    *out = g;
    return MREP_OK;
}

void mrep_geom_release(mrep_geom* geom) { delete geom; }

static int32_t upload_surfaces(const SurfPlan& P, void* dev_buf, int64_t bytes, void* stream, mrep_geom** out)
{
    if (bytes < P.layout.total) {
        set_error("mrep_upload: buffer smaller than device_bytes");
        return MREP_E_SMALL_BUFFER;
    }
    if (((uintptr_t)dev_buf & 255) != 0) {
        set_error("mrep_upload: buffer not 256-byte aligned");
        return MREP_E_INVALID_ARG;
    }
    int rc = check_device();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    char* b = (char*)dev_buf;
    const SurfLayout& L = P.layout;
    auto cp = [&](int64_t off, const void* src, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        return hipMemcpyAsync(b + off, src, n, hipMemcpyHostToDevice, st);
    };
    HIP_OK(cp(L.off_surf, P.surfs.data(), sizeof(DSurf) * P.surfs.size()));
    HIP_OK(cp(L.off_sph, P.sph.data(), sizeof(float) * P.sph.size()));
    HIP_OK(cp(L.off_lcp, P.lcp.data(), sizeof(float) * P.lcp.size()));
    HIP_OK(cp(L.off_gcp, P.gcp.data(), sizeof(double) * P.gcp.size()));
    HIP_OK(cp(L.off_uv, P.uv.data(), sizeof(double) * P.uv.size()));
    HIP_OK(cp(L.off_pspan, P.pspan.data(), sizeof(int32_t) * P.pspan.size()));
    HIP_OK(cp(L.off_span0, P.span0.data(), sizeof(int32_t) * P.span0.size()));
    HIP_OK(cp(L.off_csph, P.csph.data(), sizeof(float) * P.csph.size()));
    HIP_OK(cp(L.off_brk, P.brk.data(), sizeof(double) * P.brk.size()));
    HIP_OK(cp(L.off_coef, P.coef.data(), sizeof(double) * P.coef.size()));
    // the plan's host vectors are pageable: finish the copies before returning
    HIP_OK(hipStreamSynchronize(st));
    mrep_geom* g = new mrep_geom();
    g->kind = MREP_GEOM_SURFACES;
    g->sg.L = L;
    g->sg.base = b;
    HIP_OK(hipGetDevice(&g->sg.device));
    *out = g;
    return MREP_OK;
}

int32_t mrep_opts_default(mrep_opts* o)
{
    if (!o) {
        set_error("mrep_opts_default: null pointer");
        return MREP_E_INVALID_ARG;
    }
    o->struct_size = (int32_t)sizeof(mrep_opts);
    o->precision = MREP_PREC_BF16;
    o->max_candidates = 32;
    o->flags = 0;
    o->tie_rel = 2e-6;
    return MREP_OK;
}

}  // extern "C"

int mrep::check_opts(const mrep_opts* o)
{
    if (!o || o->struct_size != (int32_t)sizeof(mrep_opts)) {
        set_error("mrep_opts: null or struct_size mismatch");
        return MREP_E_INVALID_ARG;
    }
    if (o->precision != MREP_PREC_FP64 && o->precision != MREP_PREC_FP32 && o->precision != MREP_PREC_BF16) {
        set_error("mrep_opts: unsupported precision");
        return MREP_E_INVALID_ARG;
    }
    if (o->max_candidates < 1 || o->max_candidates > kMaxCand) {
        set_error("mrep_opts: max_candidates out of range 1..48");
        return MREP_E_INVALID_ARG;
    }
    if (!(o->tie_rel >= 0.0)) {
        set_error("mrep_opts: tie_rel must be >= 0");
        return MREP_E_INVALID_ARG;
    }
    return MREP_OK;
}

extern "C" {

int32_t mrep_workspace_bytes(const mrep_geom* geom, int64_t n, const mrep_opts* opts, int64_t* bytes)
{
    if (!geom || !bytes || n < 0 || geom->kind != MREP_GEOM_CURVES) {
        set_error("mrep_workspace_bytes: null pointer, surface geometry or negative n");
        return MREP_E_INVALID_ARG;
    }
    int rc = check_opts(opts);
    if (rc) return rc;
    *bytes = work_layout(geom->g.L.n_curves, n, opts->max_candidates, nullptr, nullptr);
    if (opts->flags & MREP_OPT_TUNED) *bytes = std::max<int64_t>(*bytes, seeded_ws_bytes(geom, n));
    return MREP_OK;
}

}  // extern "C"

extern "C" int32_t mrep_workspace_counts(const mrep_geom* geom, const void* workspace, int64_t* counts_out,
                                         void* stream)
{
    if (!geom || !workspace || !counts_out || geom->kind != MREP_GEOM_CURVES) {
        set_error("mrep_workspace_counts: null pointer or surface geometry");
        return MREP_E_INVALID_ARG;
    }
    // both workspace layouts start with the per-curve histogram, then the overflow
    // and pair counters, then (256-byte aligned) the sphere-test counters
    int32_t c[2] = {0, 0};
    const int64_t nc = geom->g.L.n_curves;
    const char* at = (const char*)workspace + 4 * nc;
    std::vector<unsigned long long> tests(kWsCounters);
    HIP_OK(hipMemcpyAsync(c, at, sizeof(c), hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIP_OK(hipMemcpyAsync(tests.data(), (const char*)workspace + ((4 * (nc + 2) + 255) & ~(int64_t)255),
                          sizeof(unsigned long long) * kWsCounters, hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    counts_out[0] = c[0];
    counts_out[1] = c[1];
    unsigned long long t = 0;
    for (unsigned long long v : tests) t += v;
    counts_out[2] = (int64_t)t;
    return MREP_OK;
}

hipError_t mrep::launch_grouping(int64_t nc, int64_t n, const int32_t* n_dev, const int32_t* curve_id,
                                 int32_t* hist, int32_t* q_off, int32_t* tile_off, int32_t* perm, const Outs& o,
                                 hipStream_t st)
{
    const int T = 256;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((nc + 2 + T - 1) / T)), dim3(T), 0, st, hist, nc + 2, 0);
    hipLaunchKernelGGL(k_hist, dim3((unsigned)((n + T - 1) / T)), dim3(T), 0, st, curve_id, n, n_dev, (int32_t)nc,
                       hist, o.t, o.d, o.s, o.f);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, hist, (int32_t)nc, q_off, tile_off);
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)((n + T - 1) / T)), dim3(T), 0, st, curve_id, n, n_dev,
                       (int32_t)nc, q_off, hist, perm);
    return hipGetLastError();
}

int mrep::project_core(const Geom& geom, const mrep_opts* opts, int64_t n, const int32_t* n_dev, const int32_t* curve_id,
                 const double* q_xyz, void* workspace, const Outs& o, hipStream_t st, int invert, bool timed,
                 int stage0)
{
    const int64_t nc = geom.L.n_curves;
    const int kc = opts->max_candidates;
    Work w;
    work_layout(nc, n, kc, (char*)workspace, &w);
    DevGeom G = dev_view(geom);
    int rc;
    HIP_OK(launch_grouping(nc, n, n_dev, curve_id, w.hist, w.q_off, w.tile_off, w.perm, o, st));
    // the sphere-test counters after the histogram: none in this strategy
    hipLaunchKernelGGL(k_fill_i32, dim3(2 * kWsCounters / 256), dim3(256), 0, st,
                       (int32_t*)((char*)workspace + a256(4 * (nc + 2))), (int64_t)(2 * kWsCounters), 0);
    if (timed && (rc = stage_mark(stage0 + 1, st))) return rc;
    if (opts->precision == MREP_PREC_BF16) {
        const int64_t grid = screen_grid(nc, n);
        HIP_OK(launch_tile_map(w.tile_off, w.q_off, nc, grid, w.tile_map, st));
        HIP_OK(launch_screen_bf16(G, grid, w.tile_map, w.perm, q_xyz, (int32_t)kc, w.so, st));
    }
    if (timed && (rc = stage_mark(stage0 + 2, st))) return rc;
    if (opts->precision == MREP_PREC_BF16) {
        HIP_OK(launch_refine(G, n, curve_id, q_xyz, w.q_off, w.perm, w.so, w.pair_res, nullptr, 0u, opts->tie_rel,
                             invert, w.ovf_list, w.ovf_count, o, st, (opts->flags & MREP_OPT_CLIP) != 0,
                             timed ? stage0 + 3 : -1));
    } else {
        if (timed && (rc = stage_mark(stage0 + 3, st))) return rc;
        const unsigned fs_blocks = (unsigned)std::min<int64_t>((n + 3) / 4, 2048);  // 4 waves per block, persistent
        // every query examined over all its pieces, in FP64 or FP32
        const bool f32 = opts->precision == MREP_PREC_FP32;
        if (G.general && f32)
            hipLaunchKernelGGL((k_fullscan<float, true>), dim3(fs_blocks), dim3(256), 0, st, G, curve_id, q_xyz,
                               w.q_off, w.perm, (const int32_t*)nullptr, (const int32_t*)nullptr, (const float*)nullptr,
                               0u, opts->tie_rel, invert, o);
        else if (f32)
            hipLaunchKernelGGL((k_fullscan<float, false>), dim3(fs_blocks), dim3(256), 0, st, G, curve_id, q_xyz,
                               w.q_off, w.perm, (const int32_t*)nullptr, (const int32_t*)nullptr, (const float*)nullptr,
                               0u, opts->tie_rel, invert, o);
        else if (G.general)
            hipLaunchKernelGGL((k_fullscan<double, true>), dim3(fs_blocks), dim3(256), 0, st, G, curve_id, q_xyz,
                               w.q_off, w.perm, (const int32_t*)nullptr, (const int32_t*)nullptr, (const float*)nullptr,
                               0u, opts->tie_rel, invert, o);
        else
            hipLaunchKernelGGL((k_fullscan<double, false>), dim3(fs_blocks), dim3(256), 0, st, G, curve_id, q_xyz,
                               w.q_off, w.perm, (const int32_t*)nullptr, (const int32_t*)nullptr, (const float*)nullptr,
                               0u, opts->tie_rel, invert, o);
    }
    HIP_OK(hipGetLastError());
    if (timed && (rc = stage_mark(stage0 + 4, st))) return rc;
    return MREP_OK;
}

hipError_t mrep::launch_refine(const DevGeom& G, int64_t n, const int32_t* curve_id, const double* q_xyz,
                               const int32_t* q_off, const int32_t* perm, const ScreenOut& so, PairRes* pair_res,
                               const uint8_t* done, uint32_t flag_in, double tie_rel, int invert, int32_t* ovf_list,
                               int32_t* ovf_count, const Outs& o, hipStream_t st, bool clip, int pairs_mark)
{
    const int RT = 128;
    // the full scan of overflowed queries: a persistent grid sized for about one
    // overflow in 256 queries (an empty launch of the wide grid cost 38 us on
    // 4,096-query calls; a grid that is too small stays correct, only slower)
    const unsigned fs_blocks = (unsigned)std::max<int64_t>(16, std::min<int64_t>((n + 63) / 64, 2048));
    const unsigned pr_blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((so.pair_cap + 255) / 256, 8192));
    if (clip) {
        const hipError_t e = launch_pairs_clip(G, curve_id, q_xyz, perm, so, done, pair_res, st);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(k_pairs<float>, dim3(pr_blocks), dim3(256), 0, st, G, curve_id, q_xyz, perm,
                           (const int32_t*)so.pair_seg, (const int32_t*)so.pair_j, (const int32_t*)so.pair_count,
                           so.pair_cap, (const float*)so.ub, tie_rel, done, pair_res);
    }
    if (pairs_mark >= 0 && stage_mark(pairs_mark, st) != MREP_OK) return hipErrorUnknown;
    // the general instances evaluate Bezier and rational spans as well (geometries that hold them)
    if (G.general) {
        hipLaunchKernelGGL((k_finish<float, true>), dim3((unsigned)((n + RT - 1) / RT)), dim3(RT), 0, st, G, curve_id,
                           q_xyz, q_off, perm, so, (const PairRes*)pair_res, done, flag_in, tie_rel, invert, ovf_list,
                           ovf_count, o);
        hipLaunchKernelGGL((k_fullscan<float, true>), dim3(fs_blocks), dim3(256), 0, st, G, curve_id, q_xyz, q_off,
                           perm, (const int32_t*)ovf_list, (const int32_t*)ovf_count, (const float*)so.ub,
                           (uint32_t)MREP_F_FULLSCAN | flag_in, tie_rel, invert, o);
    } else {
        hipLaunchKernelGGL((k_finish<float, false>), dim3((unsigned)((n + RT - 1) / RT)), dim3(RT), 0, st, G, curve_id,
                           q_xyz, q_off, perm, so, (const PairRes*)pair_res, done, flag_in, tie_rel, invert, ovf_list,
                           ovf_count, o);
        hipLaunchKernelGGL((k_fullscan<float, false>), dim3(fs_blocks), dim3(256), 0, st, G, curve_id, q_xyz, q_off,
                           perm, (const int32_t*)ovf_list, (const int32_t*)ovf_count, (const float*)so.ub,
                           (uint32_t)MREP_F_FULLSCAN | flag_in, tie_rel, invert, o);
    }
    return hipGetLastError();
}

int64_t mrep::project_ws_bytes(int64_t n_curves, int64_t n, int kc) { return work_layout(n_curves, n, kc, nullptr, nullptr); }

// Scratch of the allocation-free entry point: one fixed array per GPU, held
// until the process ends.  Host code must never pass `scratch` itself to a
// kernel (in host code it names a host-side stand-in); it uses the device
// address hipGetSymbolAddress returns, looked up once per device with that
// device current.  Every call on a GPU shares that GPU's array, so calls that
// may overlap on one GPU race; each call clears what it needs cleared with its
// own fill kernels, like a call on caller-owned workspace.
constexpr int64_t kNoAllocScratchBytes = MREP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];
constexpr int kNoAllocMaxDevices = 64;
static char* g_scratch_dev[kNoAllocMaxDevices] = {};
static std::mutex g_scratch_mu;

static int noalloc_scratch(char** out)
{
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices) {
        set_error("mrep_project_curves_noalloc: device ordinal beyond the scratch table");
        return MREP_E_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255) != 0) {
            set_error("mrep_project_curves_noalloc: scratch symbol address missing or misaligned");
            return MREP_E_HIP;
        }
        g_scratch_dev[dev] = (char*)p;
    }
    *out = g_scratch_dev[dev];
    return MREP_OK;
}

static int32_t run_project(const mrep_geom* geom, const mrep_opts* opts, int64_t n, const int32_t* curve_id,
                           const double* q_xyz, void* workspace, int64_t ws_bytes, double* t_out, double* dist_out,
                           int32_t* seg_out, uint32_t* flags_out, void* stream, int invert, int strategy = -1)
{
    if (!geom || n < 0 || geom->kind != MREP_GEOM_CURVES) {
        set_error("mrep_project_curves: null or surface geometry, or negative n");
        return MREP_E_INVALID_ARG;
    }
    int rc = check_opts(opts);
    if (rc) return rc;
    if (strategy < 0) strategy = (opts->flags & MREP_OPT_TUNED) ? geom->strategy : MREP_STRATEGY_SCREEN;
    if (strategy == MREP_STRATEGY_SPHERES && opts->precision == MREP_PREC_BF16)
        return seeded_core(invert ? "mrep_invert_curves" : "mrep_project_curves", geom, nullptr, opts, n, curve_id,
                           q_xyz, workspace, ws_bytes, t_out, dist_out, seg_out, flags_out, stream, invert);
    if (n == 0) return MREP_OK;
    // the screen's pair counter is 32-bit: n * max_candidates must stay below 2^31
    if (n * (int64_t)opts->max_candidates >= (int64_t)INT32_MAX) {
        set_error("mrep_project_curves: n * max_candidates must be < 2^31");
        return MREP_E_INVALID_ARG;
    }
    if (!curve_id || !q_xyz || !workspace || !t_out || !dist_out || !seg_out || !flags_out) {
        set_error("mrep_project_curves: null pointer");
        return MREP_E_INVALID_ARG;
    }
    const int64_t nc = geom->g.L.n_curves;
    if (ws_bytes < project_ws_bytes(nc, n, opts->max_candidates)) {
        set_error("mrep_project_curves: workspace smaller than mrep_workspace_bytes");
        return MREP_E_SMALL_BUFFER;
    }
    if (((uintptr_t)workspace & 255) != 0) {
        set_error("mrep_project_curves: workspace not 256-byte aligned");
        return MREP_E_INVALID_ARG;
    }
    if (nc == 0) {
        set_error("mrep_project_curves: geometry has no curves");
        return MREP_E_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    const bool timed = (opts->flags & MREP_OPT_TIME_STAGES) != 0;
    if (timed && (rc = stage_begin(st))) return rc;
    Outs o{t_out, dist_out, seg_out, flags_out};
    rc = project_core(geom->g, opts, n, nullptr, curve_id, q_xyz, workspace, o, st, invert, timed, 0);
    if (rc) return rc;
    if (timed) stage_end(4);
    return MREP_OK;
}

extern "C" {

int32_t mrep_project_curves(const mrep_geom* geom, const mrep_opts* opts, int64_t n, const int32_t* curve_id,
                            const double* q_xyz, void* workspace, int64_t ws_bytes, double* t_out, double* dist_out,
                            int32_t* seg_out, uint32_t* flags_out, void* stream)
{
    return run_project(geom, opts, n, curve_id, q_xyz, workspace, ws_bytes, t_out, dist_out, seg_out, flags_out,
                       stream, 0);
}

int32_t mrep_invert_curves(const mrep_geom* geom, const mrep_opts* opts, int64_t n, const int32_t* curve_id,
                           const double* q_xyz, void* workspace, int64_t ws_bytes, double* t_out, double* dist_out,
                           int32_t* seg_out, uint32_t* flags_out, void* stream)
{
    return run_project(geom, opts, n, curve_id, q_xyz, workspace, ws_bytes, t_out, dist_out, seg_out, flags_out,
                       stream, 1);
}

int32_t mrep_project_curves_noalloc(const mrep_geom* geom, const mrep_opts* opts, int64_t n, const int32_t* curve_id,
                                    const double* q_xyz, double* t_out, double* dist_out, int32_t* seg_out,
                                    uint32_t* flags_out, void* stream)
{
    const char* fn = "mrep_project_curves_noalloc";
    if (!geom || n < 0 || geom->kind != MREP_GEOM_CURVES) {
        set_error(std::string(fn) + ": null or surface geometry, or negative n");
        return MREP_E_INVALID_ARG;
    }
    int rc = check_opts(opts);
    if (rc) return rc;
    if (opts->flags & MREP_OPT_TIME_STAGES) {
        set_error(std::string(fn) + ": MREP_OPT_TIME_STAGES creates events; use mrep_project_curves to time stages");
        return MREP_E_INVALID_ARG;
    }
    int64_t need = 0;
    if ((rc = mrep_workspace_bytes(geom, n, opts, &need))) return rc;
    if (need > kNoAllocScratchBytes) {
        set_error(std::string(fn) + ": " + std::to_string(n) + " queries need " + std::to_string(need) +
                  " bytes of scratch, more than the library's fixed " + std::to_string(kNoAllocScratchBytes) +
                  " (MREP_NOALLOC_SCRATCH_BYTES); split the batch or use mrep_project_curves");
        return MREP_E_SMALL_BUFFER;
    }
    if (n == 0) return MREP_OK;
    char* ws = nullptr;
    if ((rc = noalloc_scratch(&ws))) return rc;
    return run_project(geom, opts, n, curve_id, q_xyz, ws, kNoAllocScratchBytes, t_out, dist_out, seg_out, flags_out,
                       stream, 0);
}

int32_t mrep_tune_curves(mrep_geom* geom, const mrep_opts* opts, int64_t n, const int32_t* curve_id,
                         const double* q_xyz, void* workspace, int64_t ws_bytes, double* t_out, double* dist_out,
                         int32_t* seg_out, uint32_t* flags_out, int32_t* strategy_out, double* ms_out, void* stream)
{
    if (!geom || geom->kind != MREP_GEOM_CURVES) {
        set_error("mrep_tune_curves: null or surface geometry");
        return MREP_E_INVALID_ARG;
    }
    int rc = check_opts(opts);
    if (rc) return rc;
    if (opts->precision != MREP_PREC_BF16) {
        set_error("mrep_tune_curves: the strategies differ in the BF16 mode only");
        return MREP_E_INVALID_ARG;
    }
    int64_t need = 0;
    mrep_opts o2 = *opts;
    o2.flags = (opts->flags | MREP_OPT_TUNED) & ~MREP_OPT_TIME_STAGES;
    if ((rc = mrep_workspace_bytes(geom, n, &o2, &need))) return rc;
    if (ws_bytes < need) {
        set_error("mrep_tune_curves: workspace smaller than mrep_workspace_bytes with MREP_OPT_TUNED");
        return MREP_E_SMALL_BUFFER;
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    // runs 0..MREP_N_BOX_SCHEDULES-1: the sphere strategy in each schedule; the last: the screen
    double tms[MREP_N_BOX_SCHEDULES + 1] = {};
    for (int run = 0; run <= MREP_N_BOX_SCHEDULES && rc == MREP_OK; ++run) {
        const int strat = run < MREP_N_BOX_SCHEDULES ? MREP_STRATEGY_SPHERES : MREP_STRATEGY_SCREEN;
        if (strat == MREP_STRATEGY_SPHERES) box_schedule(run, &geom->box_lanes, &geom->box_persist);
        for (int it = 0; it < 3 && rc == MREP_OK; ++it) {
            if (it == 1) rc = hipEventRecord(e0, st) == hipSuccess ? MREP_OK : MREP_E_HIP;
            if (rc == MREP_OK)
                rc = run_project(geom, &o2, n, curve_id, q_xyz, workspace, ws_bytes, t_out, dist_out, seg_out,
                                 flags_out, stream, 0, strat);
        }
        float t = 0.f;
        if (rc == MREP_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&t, e0, e1) != hipSuccess)) {
            set_error("mrep_tune_curves: event timing failed");
            rc = MREP_E_HIP;
        }
        tms[run] = 0.5 * (double)t;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    int best = 0;
    for (int s = 0; s < MREP_N_BOX_SCHEDULES; ++s) {
        geom->box_ms[s] = tms[s];
        if (tms[s] < tms[best]) best = s;
    }
    box_schedule(best, &geom->box_lanes, &geom->box_persist);
    const double ms[2] = {tms[MREP_N_BOX_SCHEDULES], tms[best]};
    geom->strategy = ms[MREP_STRATEGY_SPHERES] < ms[MREP_STRATEGY_SCREEN] ? MREP_STRATEGY_SPHERES : MREP_STRATEGY_SCREEN;
    // leave the chosen strategy's answers in the outputs (the screen ran last)
    if (geom->strategy == MREP_STRATEGY_SPHERES &&
        (rc = run_project(geom, &o2, n, curve_id, q_xyz, workspace, ws_bytes, t_out, dist_out, seg_out, flags_out,
                          stream, 0, MREP_STRATEGY_SPHERES)))
        return rc;
    HIP_OK(hipStreamSynchronize(st));
    if (strategy_out) *strategy_out = geom->strategy;
    if (ms_out) { ms_out[0] = ms[0]; ms_out[1] = ms[1]; }
    return MREP_OK;
}

int32_t mrep_set_curve_strategy(mrep_geom* geom, int32_t strategy)
{
    if (!geom || geom->kind != MREP_GEOM_CURVES ||
        (strategy != MREP_STRATEGY_SCREEN && strategy != MREP_STRATEGY_SPHERES)) {
        set_error("mrep_set_curve_strategy: null or surface geometry, or unknown strategy");
        return MREP_E_INVALID_ARG;
    }
    geom->strategy = strategy;
    return MREP_OK;
}

int32_t mrep_curve_schedule(const mrep_geom* geom, int32_t* lanes_out, int32_t* persistent_out, double* ms_out)
{
    if (!geom || geom->kind != MREP_GEOM_CURVES || !lanes_out || !persistent_out) {
        set_error("mrep_curve_schedule: null or surface geometry, or null outputs");
        return MREP_E_INVALID_ARG;
    }
    *lanes_out = geom->box_lanes;
    *persistent_out = geom->box_persist;
    if (ms_out)
        for (int s = 0; s < MREP_N_BOX_SCHEDULES; ++s) ms_out[s] = geom->box_ms[s];
    return MREP_OK;
}

int32_t mrep_set_curve_schedule(mrep_geom* geom, int32_t lanes, int32_t persistent)
{
    if (!geom || geom->kind != MREP_GEOM_CURVES || (lanes != 4 && lanes != 8 && lanes != 16) ||
        (persistent != 0 && persistent != 1)) {
        set_error("mrep_set_curve_schedule: null or surface geometry, lanes not 4, 8 or 16, or persistent not 0/1");
        return MREP_E_INVALID_ARG;
    }
    geom->box_lanes = lanes;
    geom->box_persist = persistent;
    return MREP_OK;
}

int32_t mrep_eval_curves(const mrep_geom* geom, int64_t n, const int32_t* curve_id, const double* t, double* xyz_out,
                         void* stream)
{
    if (!geom || n < 0 || (n > 0 && (!curve_id || !t || !xyz_out)) || geom->kind != MREP_GEOM_CURVES) {
        set_error("mrep_eval_curves: null pointer, surface geometry or negative n");
        return MREP_E_INVALID_ARG;
    }
    if (n == 0) return MREP_OK;
    DevGeom G = dev_view(geom->g);
    hipLaunchKernelGGL(k_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, G, n, curve_id, t,
                       xyz_out);
    HIP_OK(hipGetLastError());
    return MREP_OK;
}

int32_t mrep_last_stage_times(double* ms_out, int32_t n)
{
    const int cnt = t_stage.count;
    if (!ms_out || cnt == 0 || n < cnt) {
        set_error("mrep_last_stage_times: no timed call on this thread, or n too small");
        return MREP_E_INVALID_ARG;
    }
    HIP_OK(hipEventSynchronize(t_stage.ev[cnt]));
    for (int k = 0; k < cnt; ++k) {
        float ms = 0.f;
        HIP_OK(hipEventElapsedTime(&ms, t_stage.ev[k], t_stage.ev[k + 1]));
        ms_out[k] = (double)ms;
    }
    return cnt;
}

int32_t mrep_bernstein_matrix(int32_t p, int32_t inverse, double* out)
{
    if (p < 1 || p > MREP_MAX_DEGREE || !out) {
        set_error("mrep_bernstein_matrix: bad degree or null");
        return MREP_E_INVALID_ARG;
    }
    if (inverse) bernstein_inverse(p, out); else bernstein_matrix(p, out);
    return MREP_OK;
}

int32_t mrep_subdivision_matrix(int32_t p, double z, double* out)
{
    if (p < 1 || p > MREP_MAX_DEGREE || !out) {
        set_error("mrep_subdivision_matrix: bad degree or null");
        return MREP_E_INVALID_ARG;
    }
    subdivision_matrix(p, z, out);
    return MREP_OK;
}

int32_t mrep_gram_matrix(int32_t m, int32_t n, double* out)
{
    if (m < 0 || n < 0 || m > 2 * MREP_MAX_DEGREE || n > 2 * MREP_MAX_DEGREE || !out) {
        set_error("mrep_gram_matrix: bad degree or null");
        return MREP_E_INVALID_ARG;
    }
    gram_matrix(m, n, out);
    return MREP_OK;
}

}  // extern "C"
