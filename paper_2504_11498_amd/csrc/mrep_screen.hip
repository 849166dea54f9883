// BF16 MFMA screen of libmrep (gfx950).
//
// This translation unit is compiled with -fno-honor-nans (its inputs are
// finite: NaN query coordinates are outside the contract) so that the minimum
// over MFMA results needs no canonicalisation, and with MFMA results in VGPRs
// (no AGPR round trip): two v_min3 per MFMA is then the whole reduction.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/mrep.h"
#include "mrep_dev.h"

namespace mrep {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// 2. BF16 MFMA screen
// ---------------------------------------------------------------------------
// Row of a (query, sample) pair, length 32, in the centred sample parameter
// v = 2u - 1 in [-1, 1]:
//   [v^j q'_x, v^j q'_y, v^j q'_z  (j = 0..3) | v^m (m = 0..6) |
//    qh (3) | qh (3) | ql (3) | Qh, Ql | 1, 1]
// Column of a piece C = c + sum_j b_j v^j (centre c relative to the curve
// origin o, q' = q - o):
//   [-2 b_j (12) | e_m (7) | -2 ch (3) | -2 cl (3) | -2 ch (3) | 1, 1 | Ph, Pl]
// with e(v) = |C - c|^2 + 2 c.(C - c), q'_i ~ qh_i + ql_i and c_i ~ ch_i + cl_i
// split into two BF16 each, Qh + Ql ~ |q'|^2 - gamma and Ph + Pl ~ |c|^2 - beta.
// The first 19 products give |q - C|^2 - |q' - c|^2 and the last 13 give
// |q' - c|^2 - beta - gamma, so the MFMA result is the squared sample distance
// minus two small per-piece and per-query offsets, and the epilogue is one FMA
// and one compare.  The centred basis keeps |b_j| near the piece's half-chord
// and curvature terms, which is what the BF16 rounding bound scales with.
//
// v_mfma_f32_16x16x32_bf16 operand layout (wave64): lane l supplies row
// (l & 15) of A and column (l & 15) of B, each with K entries 8*(l>>4) .. +7;
// the 16x16 FP32 result gives lane l column (l & 15), rows 4*(l>>4) .. +3.
// Rows of one MFMA are (query g = row>>2, sample 4i + (row&3)) for i = 0..7,
// so lane l ends up with 4 samples of query (l>>4) against piece (l&15) per
// MFMA, and 8 MFMAs cover all 32 samples without any cross-lane reduction.
//
// Screen bound: the sum S of a sample differs from D - beta_eff - gamma_eff
// (D the exact squared distance, beta_eff = |c|^2 - (Ph + Pl), gamma_eff =
// |q'|^2 - (Qh + Ql)) by at most qmax alpha + beta_req + gamma_req, qmax =
// max|q'_i|: alpha and beta_req (per piece, from the host) cover the BF16
// rounding of the first 19 entries (kScreenKappaBf16), the dropped parts of the
// split cross term and the FP32 accumulation; gamma_req = 4e-6 |q'|^2.  With
// beta_eff >= beta_req and gamma_eff >= gamma_req:
//   D >= S - qmax alpha                          (lower bound X)
//   D <= X + 2 qmax alpha + K_B + K_G            (K_B = beta_req + beta_eff,
//                                                 K_G >= gamma_req + gamma_eff)
// Qh + Ql = Qt (1 +- 2^-16) with Qt = |q'|^2 (1 - 2e-5) in FP32 gives
// gamma_eff in |q'|^2 [4.3e-6, 3.57e-5]: K_G = 4.2e-5 |q'|^2.
constexpr float kGammaT = 2e-5f;
constexpr float kGammaUb = 4.2e-5f;
constexpr unsigned kBf16Inf = 0x7F80u;  // +inf in the low half of a column's last uint4 (entry 30)

// round to the nearest BF16 value (ties to even), returned as FP32
__device__ __forceinline__ float bf16_round(float x) { return (float)(__bf16)x; }

// Sample factors of the rows: entry k of lane l in MFMA i (sample 4i + (l & 3),
// K block l >> 4) is a power of the sample's v, multiplied in the kernel by
// the query factor of that entry (1 where the entry is a pure power):
//   K block 0: [1 1 1 v v v v^2 v^2]      K block 1: [v^2 v^3 v^3 v^3 1 v v^2 v^3]
//   K block 2: [v^4 v^5 v^6 1 1 1 1 1]    K block 3: [1 1 1 1 1 1 1 1]
// v = 2u - 1 for u = k / (kSamples - 1) is rounded once to FP32 (so the first
// and last samples are exactly -1 and 1), its powers are FP32 products.
struct RowM {
    float m[8 * 64 * 8];
};
constexpr RowM make_row_m()
{
    RowM t{};
    for (int i = 0; i < 8; ++i)
        for (int l = 0; l < 64; ++l) {
            const int kb = l >> 4;
            const float v = (float)(-1.0 + 2.0 * (double)(4 * i + (l & 3)) / (double)(kSamples - 1));
            const float v2 = v * v, v3 = v2 * v, v4 = v2 * v2, v5 = v4 * v, v6 = v3 * v3;
            const float r[4][8] = {{1.f, 1.f, 1.f, v, v, v, v2, v2},
                                   {v2, v3, v3, v3, 1.f, v, v2, v3},
                                   {v4, v5, v6, 1.f, 1.f, 1.f, 1.f, 1.f},
                                   {1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f}};
            for (int k = 0; k < 8; ++k) t.m[(i * 64 + l) * 8 + k] = r[kb][k];
        }
    return t;
}
__device__ constexpr RowM kRowM = make_row_m();
static_assert(kSamples == 32, "8 MFMAs of 4 samples per piece");

// minimum over the 16 lanes of a DPP row (the 16 lanes of one query)
template <int Ctrl>
__device__ __forceinline__ float dpp_f(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), Ctrl, 0xF, 0xF, false));
}
__device__ __forceinline__ float min16(float u)
{
    u = fminf(u, dpp_f<0xB1>(u));   // quad_perm [1,0,3,2]
    u = fminf(u, dpp_f<0x4E>(u));   // quad_perm [2,3,0,1]
    u = fminf(u, dpp_f<0x141>(u));  // row_half_mirror: lane i <-> 7 - i within 8
    u = fminf(u, dpp_f<0x140>(u));  // row_mirror: lane i <-> 15 - i within 16
    return u;
}

#ifndef MREP_SCREEN_WAVES
#define MREP_SCREEN_WAVES 4
#endif
#ifndef MREP_SCREEN_SETS
#define MREP_SCREEN_SETS 2
#endif
constexpr int kWaves = MREP_SCREEN_WAVES;  // waves per workgroup
constexpr int kSets = MREP_SCREEN_SETS;    // query sets of 4 per wave
constexpr int kThreads = 64 * kWaves;
constexpr int kDepth = 3;   // lower bounds kept per lane and query
static_assert(4 * kSets * kWaves == kQueriesPerTile, "tile = waves x sets x 4 queries");
// margins that make the raw hardware square root (<= 1 ulp) safe for the
// certified bounds, with room for the FP32 rounding of the epilogue
constexpr float kSqrtLo = 1.0f - 0x1p-20f;
constexpr float kSqrtHi = 1.0f + 0x1p-20f;
// lb <= U implies D - delta <= ((U + e) / kSqrtLo)^2 <= ((U + e_max) / kSqrtLo)^2;
// the threshold is computed with a relative margin of 2^-18 so that FP32
// rounding can only let more pieces through
#ifndef MREP_CHUNK_AHEAD
#define MREP_CHUNK_AHEAD 0  // 1: the next chunk's loads are issued before the current chunk is screened
#endif
#ifndef MREP_SHARE_EVERY
#define MREP_SHARE_EVERY 8
#endif
constexpr int kShareEvery = MREP_SHARE_EVERY;  // tiles between refreshes of a query's shared upper bound

// Staging of one chunk of kChunk pieces as 80-byte LDS records: the column
// (64 B) and the bound terms (16 B) of each piece.  Each thread loads
// kColLoads column quarters and one bound record into registers; pieces past
// the curve's end get columns whose constant entry is +inf (every sum is +inf:
// never a candidate, never an upper bound).
constexpr int kColLoads = kChunk * 4 / kThreads;
constexpr int kAuxLoads = kChunk / kThreads;
static_assert(kChunk % kThreads == 0, "whole bound records per thread");
__device__ __forceinline__ void load_chunk(const DevGeom& G, const DCurve& cv, int base, uint4* cr, uint4* ar)
{
    const int cn = min(kChunk, cv.n_seg - base);
    const uint4* gc = reinterpret_cast<const uint4*>(G.col + (cv.seg_off + base) * kScreenK);
    const uint4* ga = reinterpret_cast<const uint4*>(G.aux + (cv.seg_off + base) * 8);
#pragma unroll
    for (int k = 0; k < kColLoads; ++k) {
        const int i = threadIdx.x + k * kThreads;
        cr[k] = (i < cn * 4) ? gc[i] : ((i & 3) == 3 ? make_uint4(0, 0, 0, kBf16Inf) : make_uint4(0, 0, 0, 0));
    }
#pragma unroll
    for (int k = 0; k < kAuxLoads; ++k) {
        const int i = threadIdx.x + k * kThreads;
        ar[k] = (i < cn) ? ga[2 * i + 1] : make_uint4(0, 0, 0, 0);
    }
}

// 4 waves per SIMD (at most 128 VGPRs; one value spills, stored in the
// prologue and read back in the candidate output): the MFMA-to-reduction
// latency and the per-tile row building and staging are hidden by the other
// waves.  Measured on the batched curves: 3 waves (with the next chunk's loads
// issued ahead, 163 VGPRs) 1.03 ms, 4 waves 0.96 ms; 2 waves lose a fifth.
#ifndef MREP_SCREEN_MIN_WAVES
#define MREP_SCREEN_MIN_WAVES 4
#endif
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(MREP_SCREEN_MIN_WAVES, 8))) void k_screen_bf16(
    DevGeom G, const int4* __restrict__ tile_map, const int32_t* __restrict__ perm, const double* __restrict__ qxyz,
    int32_t kc, ScreenOut out)
{
    __shared__ uint4 s_rec[kChunk * 5];
    __shared__ int32_t s_off[kWaves * kSets * 4];
    __shared__ int32_t s_base;

    // this workgroup's tile (XCD-aware order: the tiles of one curve run on one
    // XCD and share its L2 for the curve's pieces)
    const int4 tm = tile_map[blockIdx.x];
    if (tm.x < 0) return;
    const int c = tm.x;
    const DCurve cv = G.curves[c];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int qbase = tm.y + wave * (4 * kSets);
    const int qend = tm.z;

    // the first chunk's loads are in flight while the rows are built
    const int nseg = cv.n_seg;
    uint4 cr[kColLoads], ar[kAuxLoads];
    if (MREP_CHUNK_AHEAD) load_chunk(G, cv, 0, cr, ar);

    // A fragments (rows), built once per query set: entry k of lane l is
    // kRowM[i][l][k] (the sample's power) times the query factor w[k].
    const int arow = lane & 15;
    const int kb = lane >> 4;
    bf16x8 A[kSets][8];
    // epilogue terms of this lane's query (query lane>>4 of each set)
    float qmax[kSets], kg[kSets], eq[kSets];
    bool pvalid[kSets];
    float w[kSets][8];
    for (int s = 0; s < kSets; ++s) {
        int ja = qbase + 4 * s + (arow >> 2);
        float qx = 0.f, qy = 0.f, qz = 0.f;
        if (ja < qend) {
            const double* q = qxyz + 3 * (int64_t)perm[ja];
            qx = (float)(q[0] - cv.origin[0]);
            qy = (float)(q[1] - cv.origin[1]);
            qz = (float)(q[2] - cv.origin[2]);
        }
        // the query's part of |q' - c|^2: q'_i = qh_i + ql_i (+ <= 2^-16 |q'_i|)
        // and Q = |q'|^2 - gamma_t = Qh + Ql, all BF16
        const float qhx = bf16_round(qx), qhy = bf16_round(qy), qhz = bf16_round(qz);
        const float qlx = bf16_round(qx - qhx), qly = bf16_round(qy - qhy), qlz = bf16_round(qz - qhz);
        const float qqa = fmaf(qz, qz, fmaf(qy, qy, qx * qx));
        const float Qt = qqa - kGammaT * qqa;
        const float Qh = bf16_round(Qt), Ql = bf16_round(Qt - Qh);
        // query factors by K block (kb): [q q q q q q q q] [q q q q 1 1 1 1]
        // [1 1 1 qh qh qh qh qh] [qh ql ql ql Qh Ql 1 1]
        const bool k0 = kb == 0, k1 = kb == 1, k2 = kb == 2;
        w[s][0] = k0 ? qx : (k1 ? qz : (k2 ? 1.f : qhz));
        w[s][1] = k0 ? qy : (k1 ? qx : (k2 ? 1.f : qlx));
        w[s][2] = k0 ? qz : (k1 ? qy : (k2 ? 1.f : qly));
        w[s][3] = k0 ? qx : (k1 ? qz : (k2 ? qhx : qlz));
        w[s][4] = k0 ? qy : (k1 ? 1.f : (k2 ? qhy : Qh));
        w[s][5] = k0 ? qz : (k1 ? 1.f : (k2 ? qhz : Ql));
        w[s][6] = k0 ? qx : (k1 ? 1.f : (k2 ? qhx : 1.f));
        w[s][7] = k0 ? qy : (k1 ? 1.f : (k2 ? qhy : 1.f));
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float4* mp = reinterpret_cast<const float4*>(&kRowM.m[(i * 64 + lane) * 8]);
        const float4 m0 = mp[0], m1 = mp[1];
        const float m[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
#pragma unroll
        for (int s = 0; s < kSets; ++s) {
            bf16x8 a;
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] = (__bf16)(m[k] * w[s][k]);  // v_cvt_pk_bf16_f32, round to nearest even
            A[s][i] = a;
        }
    }
    for (int s = 0; s < kSets; ++s) {
        const int jp = qbase + 4 * s + (lane >> 4);
        pvalid[s] = jp < qend;
        float px = 0.f, py = 0.f, pz = 0.f;
        if (pvalid[s]) {
            const double* q = qxyz + 3 * (int64_t)perm[jp];
            px = (float)(q[0] - cv.origin[0]);
            py = (float)(q[1] - cv.origin[1]);
            pz = (float)(q[2] - cv.origin[2]);
        }
        const float qq = fmaf(pz, pz, fmaf(py, py, px * px));
        kg[s] = kGammaUb * qq;
        qmax[s] = fmaxf(fabsf(px), fmaxf(fabsf(py), fabsf(pz)));
        // rounding q - o to FP32 moves the query by <= 2^-24 |q - o| per axis
        // (the origin is exact in FP32): 2.4e-7 |q'| bounds the distance change
        eq[s] = __builtin_amdgcn_sqrtf(qq) * 2.4e-7f + 1e-30f;
    }

    // per lane and query set: running upper bound (squared), the kDepth smallest
    // lower bounds (sorted) with their pieces, the smallest discarded bound.
    // Lower bounds here leave out the per-query term eq, added at the end.
    // xth: from the query's upper bound shared among its 16 lanes every
    // kShareEvery tiles; a piece whose lower bound is above it can be neither a
    // candidate nor a better upper bound, and skips the list and bound update.
    float ubsq[kSets], lbk[kSets][kDepth], disc[kSets], xth[kSets];
    int sk[kSets][kDepth];
    for (int s = 0; s < kSets; ++s) {
        ubsq[s] = INFINITY;
        disc[s] = INFINITY;
        xth[s] = INFINITY;
        for (int k = 0; k < kDepth; ++k) { lbk[s][k] = INFINITY; sk[s][k] = -1; }
    }
    const float tol = (float)cv.tol_eff;
    const float es_max = cv.es_max;
    int it = 0;

    for (int base = 0; base < nseg; base += kChunk) {
        const int cn = min(kChunk, nseg - base);
        const int cn16 = (cn + 15) & ~15;
        __syncthreads();  // every wave is done with the previous chunk
        if (!MREP_CHUNK_AHEAD) load_chunk(G, cv, base, cr, ar);
#pragma unroll
        for (int k = 0; k < kColLoads; ++k) {
            const int i = threadIdx.x + k * kThreads;
            s_rec[(i >> 2) * 5 + (i & 3)] = cr[k];
        }
#pragma unroll
        for (int k = 0; k < kAuxLoads; ++k) s_rec[(threadIdx.x + k * kThreads) * 5 + 4] = ar[k];
        __syncthreads();
        // the next chunk's loads are in flight while this one is screened
        if (MREP_CHUNK_AHEAD && base + kChunk < nseg) load_chunk(G, cv, base + kChunk, cr, ar);
        for (int tb = 0; tb < cn16; tb += 16) {
            const int sl = tb + (lane & 15);
            const bf16x8 B = __builtin_bit_cast(bf16x8, s_rec[sl * 5 + kb]);
            const float4 x1 = __builtin_bit_cast(float4, s_rec[sl * 5 + 4]);  // alpha, K_B, e, L
            // the sets' MFMAs are interleaved and each result is reduced one
            // step later, so that no reduction waits on the MFMA just issued
            float accs[kSets];
            static_assert(kSets == 2, "two query sets alternate");
            {
                // fenced order: the MFMA of one set, then the reduction of that
                // set's previous result (two MFMAs old), alternating the sets, so
                // that every MFMA is followed by this wave's own VALU work
                const floatx4 z = {0.f, 0.f, 0.f, 0.f};
                floatx4 p0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0][0], B, z, 0, 0, 0);
                floatx4 p1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1][0], B, z, 0, 0, 0);
                accs[0] = INFINITY;
                accs[1] = INFINITY;
#pragma unroll
                for (int i = 1; i < 8; ++i) {
                    __builtin_amdgcn_sched_barrier(0);
                    const floatx4 c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0][i], B, z, 0, 0, 0);
                    accs[0] = __builtin_fminf(__builtin_fminf(accs[0], p0[0]), p0[1]);
                    accs[0] = __builtin_fminf(__builtin_fminf(accs[0], p0[2]), p0[3]);
                    __builtin_amdgcn_sched_barrier(0);
                    const floatx4 c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1][i], B, z, 0, 0, 0);
                    accs[1] = __builtin_fminf(__builtin_fminf(accs[1], p1[0]), p1[1]);
                    accs[1] = __builtin_fminf(__builtin_fminf(accs[1], p1[2]), p1[3]);
                    p0 = c0;
                    p1 = c1;
                }
                __builtin_amdgcn_sched_barrier(0);
                accs[0] = __builtin_fminf(__builtin_fminf(accs[0], p0[0]), p0[1]);
                accs[0] = __builtin_fminf(__builtin_fminf(accs[0], p0[2]), p0[3]);
                accs[1] = __builtin_fminf(__builtin_fminf(accs[1], p1[0]), p1[1]);
                accs[1] = __builtin_fminf(__builtin_fminf(accs[1], p1[2]), p1[3]);
            }
            // X = min over the samples of (sum - qmax alpha) <= the smallest squared
            // sample distance (query lane>>4 of set s, piece sl)
            float X[kSets];
            bool any = false;
#pragma unroll
            for (int s = 0; s < kSets; ++s) {
                X[s] = fmaf(-qmax[s], x1.x, accs[s]);
                any |= X[s] <= xth[s];
            }
            if (any) {
                const int gseg = (int)(cv.seg_off + base + sl);
#pragma unroll
                for (int s = 0; s < kSets; ++s) {
                    if (!(X[s] <= xth[s])) continue;
                    // squared sample distance <= X + 2 qmax alpha + K_B + K_G; the
                    // last term covers this sum's FP32 rounding
                    const float t = fmaf(2.f * qmax[s], x1.x, X[s]) + (x1.y + kg[s]);
                    const float ub2 = fmaf(0x1p-21f, fabsf(X[s]) + fmaf(2.f * qmax[s], x1.x, x1.y + kg[s]), t);
                    ubsq[s] = fminf(ubsq[s], ub2);
                    // raw v_sqrt_f32 (<= 1 ulp): the lower bound is shrunk by 2^-20 relative
                    const float lb = fmaf(__builtin_amdgcn_sqrtf(fmaxf(X[s], 0.f)), kSqrtLo, -x1.z);
                    const float l3 = lbk[s][kDepth - 1];
                    disc[s] = fminf(disc[s], fmaxf(lb, l3));  // the value that leaves the list
                    if (lb < l3) {  // insert into the sorted list
                        float v = lb;
                        int g = gseg;
#pragma unroll
                        for (int k = 0; k < kDepth; ++k) {
                            const bool sw = v < lbk[s][k];
                            const float tv = sw ? lbk[s][k] : v;
                            const int tg = sw ? sk[s][k] : g;
                            lbk[s][k] = sw ? v : lbk[s][k];
                            sk[s][k] = sw ? g : sk[s][k];
                            v = tv;
                            g = tg;
                        }
                    }
                }
            }
            if (++it % kShareEvery == 0 || it == 1) {  // first refresh after one tile
                for (int s = 0; s < kSets; ++s) {
                    const float u = min16(ubsq[s]);
                    const float w = (__builtin_amdgcn_sqrtf(u) * kSqrtHi + tol + 2.f * eq[s] + es_max) *
                                     (1.0f / kSqrtLo);
                    xth[s] = w * w * (1.0f + 0x1p-18f);
                }
            }
        }
    }
    // per query (16 lanes): upper bound and candidate count; then one atomic
    // per workgroup reserves the pairs of all its queries
    const int g = lane >> 4;
    const uint64_t gm = 0xFFFFull << (16 * g);
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int tot[kSets], pos[kSets];
    bool ovf[kSets];
    float UBv[kSets];
    bool ck[kSets][kDepth];
    for (int s = 0; s < kSets; ++s) {
        const float u = min16(ubsq[s]);
        UBv[s] = __builtin_amdgcn_sqrtf(u) * kSqrtHi + (float)cv.tol_eff + eq[s];
        // lower bounds carry eq only here: lb - eq <= UB  <=>  lb <= UB + eq
        const float cmp = UBv[s] + eq[s];
        tot[s] = 0;
        pos[s] = 0;
#pragma unroll
        for (int k = 0; k < kDepth; ++k) {
            ck[s][k] = sk[s][k] >= 0 && lbk[s][k] <= cmp;  // an unfilled slot is never a candidate
            const uint64_t m = __ballot(ck[s][k]);
            tot[s] += __popcll(m & gm);
            pos[s] += __popcll(m & gm & below);
        }
        ovf[s] = tot[s] > kc || (__ballot(disc[s] <= cmp) & gm) != 0ull || !pvalid[s];
        if ((lane & 15) == 0) s_off[(wave * kSets + s) * 4 + g] = ovf[s] ? 0 : tot[s];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int sum = 0;
        for (int i = 0; i < kWaves * kSets * 4; ++i) {
            const int v = s_off[i];
            s_off[i] = sum;
            sum += v;
        }
        s_base = sum > 0 ? atomicAdd(out.pair_count, sum) : 0;
    }
    __syncthreads();
    for (int s = 0; s < kSets; ++s) {
        if (!pvalid[s]) continue;
        const int jp = qbase + 4 * s + g;
        const int64_t first = (int64_t)s_base + s_off[(wave * kSets + s) * 4 + g];
        const bool over = ovf[s] || first + tot[s] > out.pair_cap;
        if (!ovf[s]) {
            // every reserved slot below the capacity is written; a query cut by
            // the capacity marks its slots unused (-1) and takes the full scan
#pragma unroll
            for (int k = 0; k < kDepth; ++k)
                if (ck[s][k]) {
                    const int64_t p = first + pos[s] + k;
                    if (p < out.pair_cap) {
                        out.pair_seg[p] = sk[s][k];
                        out.pair_j[p] = over ? -1 : jp;
                    }
                }
        }
        if ((lane & 15) == 0) {
            out.cand_n[jp] = over ? -1 : tot[s];
            out.pair_off[jp] = (int32_t)(over ? 0 : first);
            out.ub[jp] = UBv[s];
        }
    }
}

hipError_t launch_screen_bf16(const DevGeom& G, int64_t grid, const int4* tile_map, const int32_t* perm,
                              const double* qxyz, int32_t kc, const ScreenOut& out, hipStream_t st)
{
    hipLaunchKernelGGL(k_screen_bf16, dim3((unsigned)grid), dim3(kThreads), 0, st, G, tile_map, perm, qxyz, kc, out);
    return hipGetLastError();
}

}  // namespace mrep
