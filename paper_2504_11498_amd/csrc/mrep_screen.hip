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
//   [v^j q'_x, v^j q'_y, v^j q'_z  (j = 0..3) | v^m (m = 0..6) | 0 x 13]
// Column of a piece C = c + sum_j b_j v^j (centre c relative to the curve
// origin o, q' = q - o):
//   [-2 b_j (12) | e_m (7) | 0 x 13],  e(v) = |C - c|^2 + 2 c.(C - c)
// row . col + |q' - c|^2 = |q - C|^2.  The centred basis keeps |b_j| near the
// piece's half-chord and curvature terms (the u-basis coefficients are several
// times the chord), which is what the BF16 rounding bound scales with.
//
// v_mfma_f32_16x16x32_bf16 operand layout (wave64): lane l supplies row
// (l & 15) of A and column (l & 15) of B, each with K entries 8*(l>>4) .. +7;
// the 16x16 FP32 result gives lane l column (l & 15), rows 4*(l>>4) .. +3.
// Rows of one MFMA are (query g = row>>2, sample 4i + (row&3)) for i = 0..7,
// so lane l ends up with 4 samples of query (l>>4) against piece (l&15) per
// MFMA, and 8 MFMAs cover all 32 samples without any cross-lane reduction.


// Screen bound: |computed - exact| of a squared sample distance.  BF16 rounds
// each row and column entry by <= 2^-8 relative, products are exact in FP32
// and the FP32 sum adds <= 32 * 2^-24; kScreenKappaBf16 (folded into the
// stored bound terms A and E) covers 2 * 2^-8 + both with margin.  The
// epilogue's FP32 terms add <= 1e-6 (|q'|^2 + |c|^2 + |acc|).

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
constexpr int kXcds = 8;    // accelerator complex dies of an MI355X, each with its own L2
static_assert(4 * kSets * kWaves == kQueriesPerTile, "tile = waves x sets x 4 queries");
static_assert(kChunk * 4 % kThreads == 0 && kChunk * 2 % kThreads == 0, "full-chunk staging");
// margins that make the raw hardware square root (<= 1 ulp) safe for the
// certified bounds, with room for the FP32 rounding of the epilogue
constexpr float kSqrtLo = 1.0f - 0x1p-20f;
constexpr float kSqrtHi = 1.0f + 0x1p-20f;
// lb <= U implies D - delta <= ((U + e) / kSqrtLo)^2 <= ((U + e_max) / kSqrtLo)^2;
// the threshold is computed with a relative margin of 2^-18 so that FP32
// rounding can only let more pieces through
constexpr int kShareEvery = 4;  // tiles between refreshes of a query's shared upper bound

// 3 waves per SIMD (at most 168 VGPRs): the MFMA-to-reduction latency is
// hidden by the other waves; 2 waves per SIMD lose a fifth of the throughput
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_screen_bf16(DevGeom G, const int32_t* __restrict__ tile_off,
                                                          const int32_t* __restrict__ q_off,
                                                          const int32_t* __restrict__ perm,
                                                          const double* __restrict__ qxyz, int32_t kc,
                                                          ScreenOut out)
{
    __shared__ __attribute__((aligned(16))) unsigned short s_col[kChunk * kScreenK];
    __shared__ __attribute__((aligned(16))) float s_aux[kChunk * 8];
    __shared__ int32_t s_off[kWaves * kSets * 4];
    __shared__ int32_t s_base;

    const int n_curves = G.n_curves;
    // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs
    // (blockIdx % 8), so XCD x takes the contiguous tile range [x*per, (x+1)*per)
    // and the tiles of one curve share that XCD's L2 for the curve's pieces.
    const int n_tiles = tile_off[n_curves];
    const int per = (n_tiles + kXcds - 1) / kXcds;
    const int slot = (int)(blockIdx.x / kXcds);
    const int tile = (int)(blockIdx.x % kXcds) * per + slot;
    if (slot >= per || tile >= n_tiles) return;
    // curve owning this tile: last c with tile_off[c] <= tile
    int lo = 0, hi = n_curves;  // tile_off[lo] <= tile < tile_off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (tile_off[mid] <= tile) lo = mid; else hi = mid;
    }
    const int c = lo;
    const DCurve cv = G.curves[c];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int qbase = q_off[c] + (tile - tile_off[c]) * kQueriesPerTile + wave * (4 * kSets);
    const int qend = q_off[c + 1];

    // A fragments (rows), built once per query set.
    const int arow = lane & 15;
    const int kb = lane >> 4;
    bf16x8 A[kSets][8];
    // epilogue query of this lane (query lane>>4 of each set): -2 q', |q'|^2, max |q'_i|
    float m2q[kSets][3], qq[kSets], qq6[kSets], qmax[kSets], eq[kSets];
    bool pvalid[kSets];
    for (int s = 0; s < kSets; ++s) {
        int ja = qbase + 4 * s + (arow >> 2);
        float qx = 0.f, qy = 0.f, qz = 0.f;
        if (ja < qend) {
            const double* q = qxyz + 3 * (int64_t)perm[ja];
            qx = (float)(q[0] - cv.origin[0]);
            qy = (float)(q[1] - cv.origin[1]);
            qz = (float)(q[2] - cv.origin[2]);
        }
        for (int i = 0; i < 8; ++i) {
            // centred sample parameter v = 2u - 1 in [-1, 1]
            float u = -1.0f + 2.0f * (float)(4 * i + (arow & 3)) / (float)(kSamples - 1);
            float u2 = u * u, u3 = u2 * u, u4 = u2 * u2, u5 = u4 * u, u6 = u3 * u3;
            float v[8];
            if (kb == 0) {
                v[0] = qx; v[1] = qy; v[2] = qz; v[3] = u * qx; v[4] = u * qy; v[5] = u * qz; v[6] = u2 * qx; v[7] = u2 * qy;
            } else if (kb == 1) {
                v[0] = u2 * qz; v[1] = u3 * qx; v[2] = u3 * qy; v[3] = u3 * qz; v[4] = 1.f; v[5] = u; v[6] = u2; v[7] = u3;
            } else if (kb == 2) {
                v[0] = u4; v[1] = u5; v[2] = u6; v[3] = 0.f; v[4] = 0.f; v[5] = 0.f; v[6] = 0.f; v[7] = 0.f;
            } else {
                for (int k = 0; k < 8; ++k) v[k] = 0.f;
            }
            bf16x8 a;
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] = (__bf16)v[k];  // v_cvt_pk_bf16_f32, round to nearest even
            A[s][i] = a;
        }
        const int jp = qbase + 4 * s + (lane >> 4);
        pvalid[s] = jp < qend;
        float px = 0.f, py = 0.f, pz = 0.f;
        if (pvalid[s]) {
            const double* q = qxyz + 3 * (int64_t)perm[jp];
            px = (float)(q[0] - cv.origin[0]);
            py = (float)(q[1] - cv.origin[1]);
            pz = (float)(q[2] - cv.origin[2]);
        }
        m2q[s][0] = -2.f * px; m2q[s][1] = -2.f * py; m2q[s][2] = -2.f * pz;
        qq[s] = px * px + py * py + pz * pz;
        qq6[s] = 1.02e-6f * qq[s];  // the epilogue's FP32 rounding, query part
        qmax[s] = fmaxf(fabsf(px), fmaxf(fabsf(py), fabsf(pz)));
        // rounding q - o to FP32 moves the query by <= 2^-24 |q - o| per axis
        // (the origin is exact in FP32): 2.4e-7 |q'| bounds the distance change
        eq[s] = __builtin_amdgcn_sqrtf(qq[s]) * 2.4e-7f + 1e-30f;
    }

    // per lane and query set: running upper bound (squared), the kDepth smallest
    // lower bounds (sorted) with their pieces, the smallest discarded bound.
    // Lower bounds here leave out the per-query term eq, added at the end.
    // ush: the query's upper bound shared among its 16 lanes every kShareEvery
    // tiles, in the form the final candidate test uses; a piece whose lower
    // bound is above it can never be a candidate and skips the list update.
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

    const int nseg = cv.n_seg;
    for (int base = 0; base < nseg; base += kChunk) {
        const int cn = min(kChunk, nseg - base);
        const int cn16 = (cn + 15) & ~15;
        __syncthreads();
        // stage columns (64 B each) and aux (32 B each).  The ragged tail gets
        // zero columns and aux that force an infinite lower and upper bound.
        {
            const uint4* gc = reinterpret_cast<const uint4*>(G.col + (cv.seg_off + base) * kScreenK);
            uint4* sc = reinterpret_cast<uint4*>(s_col);
            const float4* ga = reinterpret_cast<const float4*>(G.aux + (cv.seg_off + base) * 8);
            float4* sa = reinterpret_cast<float4*>(s_aux);
            if (cn == kChunk) {
                uint4 cr[kChunk * 4 / kThreads];
                float4 ar[kChunk * 2 / kThreads];
#pragma unroll
                for (int k = 0; k < kChunk * 4 / kThreads; ++k) cr[k] = gc[threadIdx.x + k * kThreads];
#pragma unroll
                for (int k = 0; k < kChunk * 2 / kThreads; ++k) ar[k] = ga[threadIdx.x + k * kThreads];
#pragma unroll
                for (int k = 0; k < kChunk * 4 / kThreads; ++k) sc[threadIdx.x + k * kThreads] = cr[k];
#pragma unroll
                for (int k = 0; k < kChunk * 2 / kThreads; ++k) sa[threadIdx.x + k * kThreads] = ar[k];
            } else {
                for (int i = threadIdx.x; i < cn16 * 4; i += kThreads) sc[i] = (i < cn * 4) ? gc[i] : make_uint4(0, 0, 0, 0);
                for (int i = threadIdx.x; i < cn16 * 2; i += kThreads)
                    sa[i] = (i < cn * 2) ? ga[i] : ((i & 1) ? make_float4(0.f, INFINITY, -INFINITY, 0.f)
                                                            : make_float4(0.f, 0.f, 0.f, 0.f));
            }
        }
        __syncthreads();
        for (int tb = 0; tb < cn16; tb += 16) {
            const int sl = tb + (lane & 15);
            const bf16x8 B = *reinterpret_cast<const bf16x8*>(&s_col[sl * kScreenK + kb * 8]);
            const float4 x0 = *reinterpret_cast<const float4*>(&s_aux[sl * 8]);      // c, |c|^2
            const float4 x1 = *reinterpret_cast<const float4*>(&s_aux[sl * 8 + 4]);  // kappa A, kappa E, e
            const int gseg = (int)(cv.seg_off + base + sl);
            // the sets' MFMAs are interleaved and each result is reduced one
            // step later, so that no reduction waits on the MFMA just issued
            float accs[kSets];
            {
                const floatx4 z = {0.f, 0.f, 0.f, 0.f};
                floatx4 prev[kSets];
#pragma unroll
                for (int s = 0; s < kSets; ++s) {
                    accs[s] = INFINITY;
                    prev[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[s][0], B, z, 0, 0, 0);
                }
#pragma unroll
                for (int i = 1; i <= 8; ++i) {
                    floatx4 cur[kSets];
#pragma unroll
                    for (int s = 0; s < kSets; ++s)
                        if (i < 8) cur[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[s][i], B, z, 0, 0, 0);
#pragma unroll
                    for (int s = 0; s < kSets; ++s) {
                        accs[s] = __builtin_fminf(__builtin_fminf(accs[s], prev[s][0]), prev[s][1]);
                        accs[s] = __builtin_fminf(__builtin_fminf(accs[s], prev[s][2]), prev[s][3]);
                        if (i < 8) prev[s] = cur[s];
                    }
                }
            }
            for (int s = 0; s < kSets; ++s) {
                const float acc = accs[s];
                // epilogue for (query lane>>4 of set s, piece sl).  The FP32
                // rounding term 1e-6 (|q'|^2 + |c|^2 + |acc|) is folded into the
                // stored A and E terms and qq6 (|acc| <= max|q'_i| A + E).
                const float d2c = fmaf(m2q[s][0], x0.x, fmaf(m2q[s][1], x0.y, fmaf(m2q[s][2], x0.z, qq[s] + x0.w)));
                const float D = acc + d2c;
                const float delta = fmaf(qmax[s], x1.x, x1.y) + qq6[s];
                ubsq[s] = fminf(ubsq[s], D + delta);
                const float X = D - delta;
                if (!(X <= xth[s])) continue;  // above the query's bound: never a candidate
                // raw v_sqrt_f32 (<= 1 ulp): the lower bound is shrunk by 2^-20 relative
                const float lb = fmaf(__builtin_amdgcn_sqrtf(fmaxf(X, 0.f)), kSqrtLo, -x1.z);
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
            if (++it % kShareEvery == 0) {
                for (int s = 0; s < kSets; ++s) {
                    float u = ubsq[s];
                    for (int off = 1; off < 16; off <<= 1) u = fminf(u, __shfl_xor(u, off, 64));
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
        float u = ubsq[s];
        for (int off = 1; off < 16; off <<= 1) u = fminf(u, __shfl_xor(u, off, 64));
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

hipError_t launch_screen_bf16(const DevGeom& G, int64_t grid, const int32_t* tile_off, const int32_t* q_off,
                              const int32_t* perm, const double* qxyz, int32_t kc, const ScreenOut& out,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_screen_bf16, dim3((unsigned)grid), dim3(kThreads), 0, st, G, tile_off, q_off, perm, qxyz, kc,
                       out);
    return hipGetLastError();
}

}  // namespace mrep
