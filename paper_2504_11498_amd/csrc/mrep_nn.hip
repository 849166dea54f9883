// Learned seeding: a small MLP proposes, for a (query, candidate piece) pair,
// the local parameter(s) of the closest point on the piece and a logit that
// the projection lies on that piece; a certificate then decides whether the
// seeded answer is the global minimum, and the screened pipeline takes every
// query whose certificate fails.  (The paper has no learned part; this is an
// extension built around its piecewise-cubic matrix representation, Sec. 5.2,
// and its Newton step on (C - q).C' = 0, eqs. Et and E't.)
//
// Networks (exact-erf GELU, FP32 master weights, BF16 MFMA products with FP32
// accumulation), inputs translated by the control points' centroid and scaled
// by 1 / their box diagonal:
//   curve kind:   x (15: a piece's 4 control points and the query)
//                 -> Linear(15, 128) -> GELU -> Linear(128, 128) -> GELU
//                 -> Linear(128, 2) = (u, logit);
//   surface kind: x (51: a bicubic patch's 16 control points and the query)
//                 -> Linear(51, 128) -> GELU -> Linear(128, 128) -> GELU
//                 -> Linear(128, 3) = (s, t, logit).
// Parameter layout (FP32, row-major W[out][in]): W1 | b1 | W2 | b2 | W3 | b3.
// This file holds both kinds' training and inference kernels and the curve
// path; the surface path lives with the other surface kernels.
//
// Seeded projection of one query onto a curve:
//   1. candidates: every piece of the query's curve is bounded by a sphere
//      around its control points; the K pieces with the smallest sphere lower
//      bound, the smallest sphere upper bound UB, and the index range [lo, hi]
//      of pieces whose lower bound reaches UB plus the tie margin;
//   2. the MLP scores the K candidates;
//   3. Newton from the predicted u on the best-scored piece, after walking to a
//      neighbour while the piece is monotone in the distance (at most 4 hops).
//      The piece minimum is certified by the Bernstein coefficients of
//      f(u) = (C(u) - q).C'(u): one sign change means exactly one critical
//      point;
//   4. certificate over [lo, hi]: every other piece has a sphere lower bound
//      above d* + margin, or a minimum above it: an endpoint distance where f
//      keeps one sign on the piece (again read off its Bernstein coefficients),
//      else the piece's certified minimum;
//   5. certified queries finish as in the screened pipeline (FP64 polish rules,
//      reparameterisation, flags); the others are compacted and projected by
//      the screened pipeline, flagged MREP_F_NN_FALLBACK.
// Without a network the same kernels give a sphere-pruned projection: every
// piece in [lo, hi] whose lower bound reaches UB + margin is refined.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <string>
#include <vector>

#include "../../include/mrep.h"
#include "mrep_dev.h"
#include "mrep_refine.h"

using namespace mrep;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kH = MREP_NN_HIDDEN, kK = MREP_NN_K;
constexpr int kRowW2 = 272;  // 128 bf16 + 16 bytes pad
constexpr int kCurveIn = MREP_NN_CURVE_IN;
static_assert(kH == 128 && kK == 4, "kernel tiling assumes 128 hidden units and 4 candidates");

int64_t a256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Sizes of one network kind.  BF16 weight image copied into LDS by the
// inference kernel: W1 rows of k1 (inputs padded to a multiple of 32) bf16 plus
// 16 bytes, so that the 16 rows one MFMA operand load touches start in
// different banks; W2 rows of 128 and W3 rows of 128 (16 rows, out used) with
// their columns stored in the order in which the previous layer's MFMA output
// already sits in the lanes (see k_mlp); FP32 biases.
template <int KB1>
struct Img {
    static constexpr int row1 = 64 * KB1 + 16;
    static constexpr int w2 = kH * row1;
    static constexpr int w3 = w2 + kH * kRowW2;
    static constexpr int b1 = w3 + 16 * kRowW2;
    static constexpr int b2 = b1 + 4 * kH;
    static constexpr int b3 = b2 + 4 * kH;
    static constexpr int bytes = b3 + 64;
    static_assert(bytes % 16 == 0, "image copied in 16-byte units");
};
static_assert(Img<1>::bytes == 50496 && Img<2>::bytes == 58688, "image sizes");

struct NetDims {
    int in, out, k1;
    int64_t oW1, oB1, oW2, oB2, oW3, oB3, n;
    int row1, img_w2, img_w3, img_b1, img_b2, img_b3, img_bytes;
    int64_t param_bytes, state_bytes;
};

NetDims net_dims(int kind)
{
    NetDims d;
    d.in = kind == MREP_NN_SURFACE ? MREP_NN_SURFACE_IN : MREP_NN_CURVE_IN;
    d.out = kind == MREP_NN_SURFACE ? MREP_NN_SURFACE_OUT : MREP_NN_CURVE_OUT;
    d.k1 = ((d.in + 31) / 32) * 32;
    d.oW1 = 0;
    d.oB1 = d.oW1 + (int64_t)kH * d.in;
    d.oW2 = d.oB1 + kH;
    d.oB2 = d.oW2 + (int64_t)kH * kH;
    d.oW3 = d.oB2 + kH;
    d.oB3 = d.oW3 + (int64_t)d.out * kH;
    d.n = d.oB3 + d.out;
    const bool two = d.k1 == 64;
    d.row1 = two ? Img<2>::row1 : Img<1>::row1;
    d.img_w2 = two ? Img<2>::w2 : Img<1>::w2;
    d.img_w3 = two ? Img<2>::w3 : Img<1>::w3;
    d.img_b1 = two ? Img<2>::b1 : Img<1>::b1;
    d.img_b2 = two ? Img<2>::b2 : Img<1>::b2;
    d.img_b3 = two ? Img<2>::b3 : Img<1>::b3;
    d.img_bytes = two ? Img<2>::bytes : Img<1>::bytes;
    d.param_bytes = a256(4 * d.n);
    d.state_bytes = 4 * d.param_bytes + a256(d.img_bytes);
    return d;
}

#define NN_HIP(expr)                                                              \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));        \
            return MREP_E_HIP;                                                    \
        }                                                                         \
    } while (0)

unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

// ---------------------------------------------------------------------------
// Training-form kernels: a strided BF16 MFMA GEMM and elementwise passes.
// ---------------------------------------------------------------------------
// C[M x N] = sum_k A(m, k) B(k, n) with A, B FP32 in memory (any strides),
// rounded to BF16 in registers; v_mfma_f32_16x16x32_bf16, FP32 accumulation.
// One wave per 16x16 tile of C and K range; out-of-range rows, columns and k
// read as zero.  Split K (the weight gradients, K = batch rows): blockIdx.y
// takes rows [y kc, (y+1) kc) and writes a dense M x N partial to parts + y M N,
// which k_sum_parts adds in a fixed order (deterministic).
struct GemmArgs {
    int M, N, K;
    const float* A;
    int64_t sam, sak;
    const float* B;
    int64_t sbk, sbn;
    float* C;
    int64_t scm, scn;
};

__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g, int kc, float* __restrict__ parts)
{
    const int lane = threadIdx.x & 63;
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int tiles_n = (g.N + 15) / 16;
    const int64_t tiles = (int64_t)((g.M + 15) / 16) * tiles_n;
    if (tile >= tiles) return;
    const int m0 = (int)(tile / tiles_n) * 16, n0 = (int)(tile % tiles_n) * 16;
    const int r = lane & 15, kb = lane >> 4;
    const int am = m0 + r, bn = n0 + r;
    const int kbeg = (int)blockIdx.y * kc, kend = min(g.K, kbeg + kc);
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    // A with unit stride along k and 16-byte rows: a lane's 8 k values as two
    // float4 loads (k is a multiple of 8, so they stay inside the row)
    const bool a_vec = g.sak == 1 && g.sam % 4 == 0 && ((uintptr_t)g.A & 15u) == 0;
    for (int k0 = kbeg; k0 < kend; k0 += 32) {
        bf16x8 a, b;
        const int kl = k0 + kb * 8;
        if (a_vec && kl + 8 <= kend && am < g.M) {
            const float4* ap = reinterpret_cast<const float4*>(g.A + (int64_t)am * g.sam + kl);
            const float4 lo = ap[0], hi = ap[1];
            a[0] = (__bf16)lo.x; a[1] = (__bf16)lo.y; a[2] = (__bf16)lo.z; a[3] = (__bf16)lo.w;
            a[4] = (__bf16)hi.x; a[5] = (__bf16)hi.y; a[6] = (__bf16)hi.z; a[7] = (__bf16)hi.w;
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = kl + j;
                a[j] = (__bf16)((k < kend && am < g.M) ? g.A[am * g.sam + k * g.sak] : 0.f);
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = kl + j;
            b[j] = (__bf16)((k < kend && bn < g.N) ? g.B[k * g.sbk + bn * g.sbn] : 0.f);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    const int cn = n0 + r;
    float* part = parts ? parts + (int64_t)blockIdx.y * g.M * g.N : nullptr;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int cm = m0 + 4 * kb + i;
        if (cm < g.M && cn < g.N) {
            if (part) part[(int64_t)cm * g.N + cn] = acc[i];
            else g.C[cm * g.scm + cn * g.scn] = acc[i];
        }
    }
}

// C = sum over the splits of the dense M x N partials, in split order
__global__ void k_sum_parts(int M, int N, int splits, const float* __restrict__ parts, float* __restrict__ C,
                            int64_t scm, int64_t scn)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)M * N) return;
    // sixteen loads in flight, added in split order
    const int64_t mn = (int64_t)M * N;
    float acc = 0.f;
    int s = 0;
    for (; s + 16 <= splits; s += 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = parts[(int64_t)(s + u) * mn + i];
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += v[u];
    }
    for (; s < splits; ++s) acc += parts[(int64_t)s * mn + i];
    C[(i / N) * scm + (i % N) * scn] = acc;
}

// FP32-compute debug form of the same product: one thread per element of C,
// FP32 fused multiply-adds in k order, no BF16 rounding.
__global__ void k_gemm_f32(GemmArgs g)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)g.M * g.N) return;
    const int m = (int)(i / g.N), n = (int)(i % g.N);
    float acc = 0.f;
    for (int k = 0; k < g.K; ++k) acc = fmaf(g.A[m * g.sam + k * g.sak], g.B[k * g.sbk + n * g.sbn], acc);
    g.C[m * g.scm + n * g.scn] = acc;
}

// splits of a long K and the dense partials they need (parts holds kMaxSplits x M x N floats)
// (64 rows: the weight gradients have only 8 to 64 output tiles, so the splits
// are what fills the chip)
constexpr int kMaxSplits = 128;
constexpr int kSplitRows = 64;  // K rows per split

// the training kernels' products in FP32 instead of BF16 MFMA (mrep_nn_set_compute; debug)
static thread_local bool t_gemm_fp32 = false;

hipError_t gemm(const GemmArgs& a, hipStream_t st, float* parts = nullptr)
{
    const int64_t tiles = (int64_t)((a.M + 15) / 16) * ((a.N + 15) / 16);
    if (tiles == 0) return hipSuccess;
    if (t_gemm_fp32) {
        hipLaunchKernelGGL(k_gemm_f32, dim3(blocks_for((int64_t)a.M * a.N)), dim3(256), 0, st, a);
        return hipGetLastError();
    }
    int splits = 1, kc = a.K;
    if (parts && a.K > 2 * kSplitRows) {
        splits = std::min(kMaxSplits, (a.K + kSplitRows - 1) / kSplitRows);
        kc = ((a.K + splits - 1) / splits + 31) / 32 * 32;
        splits = (a.K + kc - 1) / kc;
    }
    hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)((tiles + 3) / 4), (unsigned)splits), dim3(256), 0, st, a, kc,
                       splits > 1 ? parts : (float*)nullptr);
    if (splits > 1)
        hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for((int64_t)a.M * a.N)), dim3(256), 0, st, a.M, a.N, splits,
                           (const float*)parts, a.C, a.scm, a.scn);
    return hipGetLastError();
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float dgelu(float z)
{
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// Z += b (per column); H = GELU(Z) when H is not null
__global__ void k_bias_act(int64_t M, int N, float* __restrict__ Z, const float* __restrict__ b, float* __restrict__ H)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * N) return;
    const float z = Z[i] + b[i % N];
    Z[i] = z;
    if (H) H[i] = gelu(z);
}

// dZ = dH * GELU'(Z)
__global__ void k_gelu_back(int64_t n, const float* __restrict__ dH, const float* __restrict__ Z, float* __restrict__ dZ)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dZ[i] = dH[i] * dgelu(Z[i]);
}

// out[n] = sum_m X[m][n]: one block per column, fixed-order tree (deterministic)
__global__ __launch_bounds__(256) void k_colsum(int64_t M, int N, const float* __restrict__ X, float* __restrict__ out)
{
    __shared__ float s[256];
    const int n = blockIdx.x;
    float a = 0.f;
    for (int64_t m = threadIdx.x; m < M; m += 256) a += X[m * N + n];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = s[0];
}

// Loss a |y_param - t|^2 + BCE(y_logit, a) per row (outputs: out - 1 parameters, then the logit)
// and dL/dY of the batch mean.
__global__ void k_loss_grad(int64_t B, int out, const float* __restrict__ Y, const float* __restrict__ T,
                            const float* __restrict__ acc, float* __restrict__ dY, float* __restrict__ row_loss)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    const float a = acc[i], z = Y[i * out + out - 1];
    float mse = 0.f;
    for (int o = 0; o < out - 1; ++o) {
        const float du = Y[i * out + o] - T[i * (out - 1) + o];
        mse += du * du;
        dY[i * out + o] = 2.f * a * du / (float)B;
    }
    row_loss[i] = a * mse + fmaxf(z, 0.f) - z * a + log1pf(expf(-fabsf(z)));
    dY[i * out + out - 1] = (1.f / (1.f + expf(-z)) - a) / (float)B;
}

// mean of x[0..n) into *out (one block, fixed order)
__global__ __launch_bounds__(256) void k_mean(int64_t n, const float* __restrict__ x, float* __restrict__ out)
{
    __shared__ float s[256];
    float a = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += 256) a += x[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0] / (float)(n > 0 ? n : 1);
}

// Minibatch gather: rows[i] selects the training row of batch row i; a row
// outside [0, n_rows) becomes an all-zero row.
__global__ void k_gather(int64_t B, const int32_t* __restrict__ rows, int64_t n_rows, int in, int nt,
                         const float* __restrict__ x, const float* __restrict__ t, const float* __restrict__ acc,
                         float* __restrict__ xb, float* __restrict__ tb, float* __restrict__ accb)
{
    // one thread per (batch row, column) of the in + nt + 1 columns
    const int w = in + nt + 1;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * w) return;
    const int64_t i = e / w;
    const int k = (int)(e - i * w);
    const int64_t r = rows[i];
    const bool ok = r >= 0 && r < n_rows;
    if (k < in) xb[i * in + k] = ok ? x[r * in + k] : 0.f;
    else if (k < in + nt) tb[i * nt + (k - in)] = ok ? t[r * nt + (k - in)] : 0.f;
    else accb[i] = ok ? acc[r] : 0.f;
}

// Adam with bias correction c1 = 1 - b1^t, c2 = 1 - b2^t on FP32 master weights.
__global__ void k_adam(int64_t n, float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// FP32 master weights -> BF16 LDS image (one thread per 2-byte slot; the FP32
// bias slots are written by the thread of their first half).
__global__ void k_pack(NetDims d, const float* __restrict__ P, uint8_t* __restrict__ img)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.img_bytes / 2) return;
    const int off = 2 * i;
    if (off >= d.img_b1) {
        if (off & 2) return;
        float v = 0.f;
        if (off < d.img_b2) v = P[d.oB1 + (off - d.img_b1) / 4];
        else if (off < d.img_b3) v = P[d.oB2 + (off - d.img_b2) / 4];
        else if ((off - d.img_b3) / 4 < d.out) v = P[d.oB3 + (off - d.img_b3) / 4];
        *reinterpret_cast<float*>(img + off) = v;
        return;
    }
    float v = 0.f;
    if (off < d.img_w2) {
        const int h = off / d.row1, k = (off % d.row1) / 2;
        if (k < d.in) v = P[d.oW1 + h * d.in + k];
    } else {
        const bool l3 = off >= d.img_w3;
        const int base = l3 ? d.img_w3 : d.img_w2;
        const int h = (off - base) / kRowW2, p = ((off - base) % kRowW2) / 2;
        if (p < kH && (!l3 || h < d.out)) {
            // K position p = (kb, g, j) holds hidden unit 32 kb + 16 (j >> 2) + 4 g + (j & 3)
            const int kb = p >> 5, g = (p >> 3) & 3, j = p & 7;
            const int src = 32 * kb + 16 * (j >> 2) + 4 * g + (j & 3);
            v = l3 ? P[d.oW3 + h * kH + src] : P[d.oW2 + h * kH + src];
        }
    }
    *reinterpret_cast<__bf16*>(img + off) = (__bf16)v;
}

struct TrainWork {
    float *Xb, *Tb, *Ab, *Z1, *H1, *Z2, *H2, *Y, *dY, *dH, *dZ, *rowl;
    float* parts;  // split-K partials of the weight gradients: kMaxSplits x kH x kH
};

int64_t train_layout(const NetDims& d, int64_t B, char* base, TrainWork* w)
{
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        int64_t o = off;
        off = a256(off + bytes);
        return o;
    };
    int64_t oXb = take(4 * B * d.in), oT = take(4 * B * (d.out - 1)), oA = take(4 * B);
    int64_t oZ1 = take(4 * B * kH), oH1 = take(4 * B * kH), oZ2 = take(4 * B * kH), oH2 = take(4 * B * kH);
    int64_t oY = take(4 * B * d.out), odY = take(4 * B * d.out), odH = take(4 * B * kH), odZ = take(4 * B * kH);
    int64_t orl = take(4 * B);
    int64_t opt = take(4 * (int64_t)kMaxSplits * kH * std::max(kH, d.k1));
    if (w) {
        w->parts = (float*)(base + opt);
        w->Xb = (float*)(base + oXb); w->Tb = (float*)(base + oT); w->Ab = (float*)(base + oA);
        w->Z1 = (float*)(base + oZ1); w->H1 = (float*)(base + oH1); w->Z2 = (float*)(base + oZ2);
        w->H2 = (float*)(base + oH2); w->Y = (float*)(base + oY); w->dY = (float*)(base + odY);
        w->dH = (float*)(base + odH); w->dZ = (float*)(base + odZ); w->rowl = (float*)(base + orl);
    }
    return off;
}

int forward(const NetDims& d, const float* P, int64_t B, const float* X, const TrainWork& w, hipStream_t st)
{
    NN_HIP(gemm(GemmArgs{(int)B, kH, d.in, X, d.in, 1, P + d.oW1, 1, d.in, w.Z1, kH, 1}, st));
    hipLaunchKernelGGL(k_bias_act, dim3(blocks_for(B * kH)), dim3(256), 0, st, B, kH, w.Z1, P + d.oB1, w.H1);
    NN_HIP(gemm(GemmArgs{(int)B, kH, kH, w.H1, kH, 1, P + d.oW2, 1, kH, w.Z2, kH, 1}, st));
    hipLaunchKernelGGL(k_bias_act, dim3(blocks_for(B * kH)), dim3(256), 0, st, B, kH, w.Z2, P + d.oB2, w.H2);
    NN_HIP(gemm(GemmArgs{(int)B, d.out, kH, w.H2, kH, 1, P + d.oW3, 1, kH, w.Y, d.out, 1}, st));
    hipLaunchKernelGGL(k_bias_act, dim3(blocks_for(B * d.out)), dim3(256), 0, st, B, d.out, w.Y, P + d.oB3,
                       (float*)nullptr);
    NN_HIP(hipGetLastError());
    return MREP_OK;
}

int backward(const NetDims& d, const float* P, int64_t B, const float* X, const float* T, const float* acc,
             const TrainWork& w, float* G, float* loss_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_loss_grad, dim3(blocks_for(B)), dim3(256), 0, st, B, d.out, w.Y, T, acc, w.dY, w.rowl);
    if (loss_out) hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, st, B, w.rowl, loss_out);
    // layer 3: dW3 = dY^T H2, db3 = colsum dY, dH2 = dY W3
    NN_HIP(gemm(GemmArgs{d.out, kH, (int)B, w.dY, 1, d.out, w.H2, kH, 1, G + d.oW3, kH, 1}, st, w.parts));
    hipLaunchKernelGGL(k_colsum, dim3(d.out), dim3(256), 0, st, B, d.out, w.dY, G + d.oB3);
    NN_HIP(gemm(GemmArgs{(int)B, kH, d.out, w.dY, d.out, 1, P + d.oW3, kH, 1, w.dH, kH, 1}, st));
    hipLaunchKernelGGL(k_gelu_back, dim3(blocks_for(B * kH)), dim3(256), 0, st, B * kH, w.dH, w.Z2, w.dZ);
    // layer 2: dW2 = dZ2^T H1, db2, dH1 = dZ2 W2
    NN_HIP(gemm(GemmArgs{kH, kH, (int)B, w.dZ, 1, kH, w.H1, kH, 1, G + d.oW2, kH, 1}, st, w.parts));
    hipLaunchKernelGGL(k_colsum, dim3(kH), dim3(256), 0, st, B, kH, w.dZ, G + d.oB2);
    NN_HIP(gemm(GemmArgs{(int)B, kH, kH, w.dZ, kH, 1, P + d.oW2, kH, 1, w.dH, kH, 1}, st));
    hipLaunchKernelGGL(k_gelu_back, dim3(blocks_for(B * kH)), dim3(256), 0, st, B * kH, w.dH, w.Z1, w.dZ);
    // layer 1: dW1 = dZ1^T X, db1
    NN_HIP(gemm(GemmArgs{kH, d.in, (int)B, w.dZ, 1, kH, X, d.in, 1, G + d.oW1, d.in, 1}, st, w.parts));
    hipLaunchKernelGGL(k_colsum, dim3(kH), dim3(256), 0, st, B, kH, w.dZ, G + d.oB1);
    NN_HIP(hipGetLastError());
    return MREP_OK;
}

// splitmix64 (Steele, Lea and Flood, 2014): the initialisation generator
uint64_t splitmix64(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// Features of a (query, piece) pair of a curve, shared by training-data export
// and the fused inference kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pair_features(const DevGeom& G, const DCurve& cv, int64_t s, const double* q, float* x)
{
    const float* lp = G.lcp + s * 12;
    const float* ax = G.aux + s * 8;
    float P[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) P[i] = lp[i];
    const float ql[3] = {(float)(q[0] - (cv.origin[0] + (double)ax[AUX_CX])),
                         (float)(q[1] - (cv.origin[1] + (double)ax[AUX_CY])),
                         (float)(q[2] - (cv.origin[2] + (double)ax[AUX_CZ]))};
    float m[3], ext2 = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        m[c] = 0.25f * (P[c] + P[3 + c] + P[6 + c] + P[9 + c]);
        const float lo = fminf(fminf(P[c], P[3 + c]), fminf(P[6 + c], P[9 + c]));
        const float hi = fmaxf(fmaxf(P[c], P[3 + c]), fmaxf(P[6 + c], P[9 + c]));
        ext2 += (hi - lo) * (hi - lo);
    }
    const float inv = ext2 > 0.f ? 1.f / sqrtf(ext2) : 1.f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) x[3 * i + c] = (P[3 * i + c] - m[c]) * inv;
#pragma unroll
    for (int c = 0; c < 3; ++c) x[12 + c] = (ql[c] - m[c]) * inv;
}

// ---------------------------------------------------------------------------
// Fused inference: one wave runs 16 rows through the three layers with the
// weights' BF16 image in LDS.  The products are computed transposed
// (Z^T = W X^T): weights are the MFMA A operand, rows the B operand, so each
// layer's output already sits in the lanes as the next layer's B operand (lane
// (g, r) holds units 16 t + 4 g + i of row r); the image stores layer 2 and 3
// weight columns in that order.  Layer 1 takes KB1 K-blocks of 32 inputs.
// Persistent grid; 4 waves per block.
// Rows interface: KB1, count(), operand(row, g, kb) = inputs 32 kb + 8 g ..
// + 7 of the row as BF16, write(row, acc) with acc[o] = output o.
// ---------------------------------------------------------------------------
template <int IN, int OUT>
struct RowsFromMemory {
    static constexpr int KB1 = (IN + 31) / 32;
    int64_t n;
    const float* x;
    float* y;
    __device__ int64_t count() const { return n; }
    __device__ bf16x8 operand(int64_t row, int g, int kb) const
    {
        bf16x8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (__bf16)0.f;
        const int k0 = 32 * kb + 8 * g;
        if (row < n && k0 < IN) {
            const float* r = x + row * IN + k0;
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (__bf16)((k0 + j < IN) ? r[j] : 0.f);
        }
        return v;
    }
    __device__ void write(int64_t row, const floatx4& acc) const
    {
        if (row < n) {
#pragma unroll
            for (int o = 0; o < OUT; ++o) y[OUT * row + o] = acc[o];
        }
    }
};

// Rows = (sorted query, candidate piece) pairs of curves; inputs prepared by
// k_box as BF16 rows of 16.
struct RowsFromCandidates {
    static constexpr int KB1 = 1;
    const int32_t* q_off;
    int32_t n_curves;
    const int32_t* cand;  // [n][kK] global piece index or -1
    const uint16_t* xb;   // [n][kK][16] BF16 inputs
    float2* out;          // [n][kK] (u, logit)
    __device__ int64_t count() const { return (int64_t)q_off[n_curves] * kK; }
    __device__ bf16x8 operand(int64_t row, int g, int) const
    {
        bf16x8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (__bf16)0.f;
        if (g < 2 && row < count() && cand[row] >= 0) v = *reinterpret_cast<const bf16x8*>(xb + row * 16 + 8 * g);
        return v;
    }
    __device__ void write(int64_t row, const floatx4& acc) const
    {
        if (row < count()) out[row] = make_float2(acc[0], cand[row] >= 0 ? acc[1] : -INFINITY);
    }
};

// Rows = (sorted query, candidate patch) pairs of surfaces; BF16 rows of 64
// (51 inputs, zero padded).
struct RowsFromSurfCandidates {
    static constexpr int KB1 = 2;
    const int32_t* q_off;
    int32_t n_surf;
    const int32_t* cand;  // [n][kK] global patch index or -1
    const uint16_t* xb;   // [n][kK][64] BF16 inputs
    float4* out;          // [n][kK] (s, t, logit, 0)
    __device__ int64_t count() const { return (int64_t)q_off[n_surf] * kK; }
    __device__ bf16x8 operand(int64_t row, int g, int kb) const
    {
        bf16x8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (__bf16)0.f;
        if (row < count() && cand[row] >= 0) v = *reinterpret_cast<const bf16x8*>(xb + row * 64 + 32 * kb + 8 * g);
        return v;
    }
    __device__ void write(int64_t row, const floatx4& acc) const
    {
        if (row < count()) out[row] = make_float4(acc[0], acc[1], cand[row] >= 0 ? acc[2] : -INFINITY, 0.f);
    }
};

__device__ __forceinline__ bf16x8 pack8(const floatx4& a, const floatx4& b)
{
    bf16x8 r;
    r[0] = (__bf16)a[0]; r[1] = (__bf16)a[1]; r[2] = (__bf16)a[2]; r[3] = (__bf16)a[3];
    r[4] = (__bf16)b[0]; r[5] = (__bf16)b[1]; r[6] = (__bf16)b[2]; r[7] = (__bf16)b[3];
    return r;
}

// GELU for inference: erf by Abramowitz and Stegun, Handbook of Mathematical
// Functions, formula 7.1.28 (erf a = 1 - (1 + a1 a + ... + a6 a^6)^-16 for
// a >= 0, |error| <= 3e-7), so GELU is within 1e-6 absolute of the erf form --
// far below the BF16 rounding of the next layer's operands.  No exp and one
// reciprocal, against libm's erf in the training kernels.
__device__ __forceinline__ float gelu_inf(float z)
{
    const float x = z * 0.70710678118654752f;
    const float a = fabsf(x);
    const float p = 1.f + a * (0.0705230784f + a * (0.0422820123f + a * (0.0092705272f +
                    a * (0.0001520143f + a * (0.0002765672f + a * 0.0000430638f)))));
    const float r = __builtin_amdgcn_rcpf(p);
    const float r2 = r * r, r4 = r2 * r2, r8 = r4 * r4;
    const float h = 0.5f * z * (r8 * r8);  // 0.5 z erfc(a)
    return x >= 0.f ? z - h : h;
}

__device__ __forceinline__ floatx4 gelu4(floatx4 z)
{
    floatx4 h;
#pragma unroll
    for (int i = 0; i < 4; ++i) h[i] = gelu_inf(z[i]);
    return h;
}

template <typename Rows>
__global__ __launch_bounds__(256) void k_mlp(Rows rows, const uint8_t* __restrict__ img)
{
    constexpr int KB1 = Rows::KB1;
    using I = Img<KB1>;
    __shared__ __attribute__((aligned(16))) uint8_t s_img[I::bytes];
    for (int i = threadIdx.x; i < I::bytes / 16; i += 256)
        reinterpret_cast<uint4*>(s_img)[i] = reinterpret_cast<const uint4*>(img)[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    const int64_t n_tiles = (rows.count() + 15) / 16;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < n_tiles; tile += nwaves) {
        const int64_t row = tile * 16 + r;
        bf16x8 xb[KB1];
#pragma unroll
        for (int kb = 0; kb < KB1; ++kb) xb[kb] = rows.operand(row, g, kb);
        // layer 1
        floatx4 h[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            floatx4 acc = *reinterpret_cast<const floatx4*>(s_img + I::b1 + 4 * (16 * t + 4 * g));
#pragma unroll
            for (int kb = 0; kb < KB1; ++kb) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(s_img + (16 * t + r) * I::row1 + 64 * kb + 16 * g);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, xb[kb], acc, 0, 0, 0);
            }
            h[t] = gelu4(acc);
        }
        // layer 2
        bf16x8 hb[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) hb[kb] = pack8(h[2 * kb], h[2 * kb + 1]);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            floatx4 acc = *reinterpret_cast<const floatx4*>(s_img + I::b2 + 4 * (16 * t + 4 * g));
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const bf16x8 a =
                    *reinterpret_cast<const bf16x8*>(s_img + I::w2 + (16 * t + r) * kRowW2 + 64 * kb + 16 * g);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hb[kb], acc, 0, 0, 0);
            }
            h[t] = gelu4(acc);
            // keeps the scheduler from hoisting every output tile's weight loads
            // (which took all 512 registers and left one wave per SIMD)
            __builtin_amdgcn_sched_barrier(0);
        }
        // layer 3 (the first rows of the 16-row weight tile are the outputs)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) hb[kb] = pack8(h[2 * kb], h[2 * kb + 1]);
        floatx4 acc = *reinterpret_cast<const floatx4*>(s_img + I::b3 + 16 * g);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(s_img + I::w3 + r * kRowW2 + 64 * kb + 16 * g);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hb[kb], acc, 0, 0, 0);
        }
        if (g == 0) rows.write(row, acc);
    }
}

// ---------------------------------------------------------------------------
// Candidates by sphere bounds.  Piece s lies in the sphere of radius r_s
// (largest control-point distance from its box centre c_s, plus the piece's
// deviation bound tol_eff) around c_s, so for the query q
//     |q - c_s| - r_s  <=  dist(q, piece s)  <=  |q - c_s| + r_s,
// and a cluster of kCluPieces consecutive pieces lies in a sphere around
// theirs.  One workgroup per tile of kQueriesPerTile queries of one curve, 8
// lanes per query.  Curves whose clusters are compact (clu_use):
//   a. a first bound: the best cluster upper bound, the piece upper bounds of
//      the cluster with the smallest lower bound (clusters staged in LDS,
//      pieces read from global memory), and the distances to four points of
//      its piece with the nearest centre;
//   b. the clusters whose lower bound reaches it plus the tie margin;
//   c. over their pieces: UB = the smallest upper bound and the K pieces with
//      the smallest lower bounds (ties to the lower index), and every piece
//      whose lower bound reaches the running UB + margin (a superset of the
//      list, since UB only falls);
//   d. the list: those of them whose lower bounds, the sphere's and the
//      capsule's around the chord P0P3 (capsule_lb), both reach UB + margin(UB)
//      (a second pass over the clusters' pieces when the superset overflows).
// The lanes of a query load all of their pieces of a cluster at once, so the
// loads' latencies overlap.  Other curves: the same UB, K nearest and list from two passes over all the
// curve's piece spheres staged in LDS.  Bounds carry a rounding allowance of 1e-6 (|q'| + diag).  More than
// kBoxCluCap clusters or kBoxCap pieces: the query takes the full scan.
//
// Schedules (chosen per geometry by the autotuner): L = 4, 8 or 16 lanes per
// query (workgroups of 32 L threads), and either one workgroup per tile in
// XCD-aware order (tile map) or a persistent grid that takes tiles from one
// queue per XCD and, once its own is empty, from the others.  Every schedule
// gives the same bounds, keys and lists in the same order.
// ---------------------------------------------------------------------------
constexpr int kBoxChunk = 768;   // cluster or piece spheres staged per round (LDS for 6 workgroups per CU)
constexpr int kBoxCluCap = 64;   // candidate clusters per query
constexpr int kBoxCap = 64;      // listed pieces per query; more: the query goes to the full scan
constexpr int kXcds = 8;

struct BoxOut {
    int32_t* cand;  // [n][kK] global piece index (-1: fewer pieces)
    uint16_t* xb;   // [n][kK][16] BF16 network inputs of the candidates (null: not written)
    ScreenOut so;   // per query: the pieces whose lower bound reaches UB + margin; so.ub = UB
    unsigned long long* tests;  // [kWsCounters] sphere tests, per workgroup slot modulo kWsCounters (zeroed)
    int32_t* queue;             // [kXcds] next tile of each XCD's range (persistent schedules; zeroed)
    int32_t* tile_curve;        // [tiles] the curve of each tile (k_box_tiles)
};

// float -> uint32 with the same order (negative values included), and back
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
// merge the L lanes' sorted lists of kK keys: exchange, keep the smaller half (bitonic)
template <int L>
__device__ __forceinline__ void merge_keys(uint64_t* key)
{
#pragma unroll
    for (int off = 1; off < L; off <<= 1) {
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
}
__device__ __forceinline__ void insert_key(uint64_t* key, uint64_t x)
{
    if (x < key[kK - 1]) {
#pragma unroll
        for (int k = 0; k < kK; ++k) cswap(key[k], x);
    }
}
template <int L>
__device__ __forceinline__ float min_lanes(float v)
{
#pragma unroll
    for (int off = 1; off < L; off <<= 1) v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}
// the hits of the L lanes of this lane's query, bit i = lane i of the query
template <int L>
__device__ __forceinline__ uint32_t group_hits(bool hit, int lane)
{
    return (uint32_t)(__ballot(hit) >> (lane & (64 - L))) & (uint32_t)((1ull << L) - 1ull);
}

__device__ __forceinline__ float tie_margin(float d, const DCurve& cv, float tie_rel)
{
    return 2.f * (float)cv.tol_eff + 4e-6f * (d + (float)cv.diag) + tie_rel * (float)cv.diag;
}

// Distance from v to the segment [0, a] (inv = 1 / |a|^2, or 0 for a point).
// An inexact inv moves the foot along the segment: the result can only grow,
// by at most 2e-7 |a|.
__device__ __forceinline__ float chord_dist(float vx, float vy, float vz, float ax, float ay, float az, float inv)
{
    const float t = fminf(fmaxf((vx * ax + vy * ay + vz * az) * inv, 0.f), 1.f);
    const float x = vx - t * ax, y = vy - t * ay, z = vz - t * az;
    return __builtin_amdgcn_sqrtf(x * x + y * y + z * z);
}
// A second lower bound of the distance from the query to piece k's span (c: the
// piece's sphere).  The FP32 control points lie within rho of the chord P0P3,
// so the Bezier piece (inside their convex hull) lies in the capsule of radius
// rho around the chord, and the span within tol_eff of the piece; 8e-6 w covers
// the FP32 control points and this arithmetic.  Far tighter than the sphere for
// the long, nearly straight pieces beside the nearest one.
__device__ __forceinline__ float capsule_lb(const DevGeom& G, const DCurve& cv, int k, const float4& c, const float* ql)
{
    const float4* lp = reinterpret_cast<const float4*>(G.lcp + 12 * (cv.seg_off + (int64_t)k));
    const float4 a = lp[0], b = lp[1], e = lp[2];
    // P0 = (a.x, a.y, a.z), P1 = (a.w, b.x, b.y), P2 = (b.z, b.w, e.x), P3 = (e.y, e.z, e.w)
    const float ax = e.y - a.x, ay = e.z - a.y, az = e.w - a.z;
    const float aa = ax * ax + ay * ay + az * az;
    const float inv = aa > 1e-30f ? __builtin_amdgcn_rcpf(aa) : 0.f;
    const float rho = fmaxf(chord_dist(a.w - a.x, b.x - a.y, b.y - a.z, ax, ay, az, inv),
                            chord_dist(b.z - a.x, b.w - a.y, e.x - a.z, ax, ay, az, inv));
    const float d = chord_dist(ql[0] - c.x - a.x, ql[1] - c.y - a.y, ql[2] - c.z - a.z, ax, ay, az, inv);
    return d - rho - 1.0001f * (float)cv.tol_eff - 8e-6f * c.w;
}

// The piece with the nearest centre among the L lanes' candidates (bd, bw, bk:
// centre distance, radius, index; ties to the lower index, so the same piece
// for every lane count), and an upper bound from points of it, far tighter
// than its sphere's: lanes 0..3 take B(0), B(1/3), B(2/3), B(1) of its FP32
// Bezier form (the span lies within tol_eff of it; 4e-6 w covers the FP32
// control points and the evaluation).  INFINITY in the other lanes.
template <int L>
__device__ __forceinline__ float point_bound(const DevGeom& G, const DCurve& cv, float bd, float bw, int bk, int sub,
                                             bool active, const float* ql, float eps)
{
#pragma unroll
    for (int off = 1; off < L; off <<= 1) {
        const float od = __shfl_xor(bd, off, 64), ow = __shfl_xor(bw, off, 64);
        const int ok = __shfl_xor(bk, off, 64);
        const bool take = od < bd || (od == bd && (unsigned)ok < (unsigned)bk);
        bk = take ? ok : bk;
        bw = take ? ow : bw;
        bd = take ? od : bd;
    }
    if (!active || bk < 0 || sub >= 4) return INFINITY;
    const float4* lp = reinterpret_cast<const float4*>(G.lcp + 12 * (cv.seg_off + (int64_t)bk));
    const float4 a = lp[0], b = lp[1], e = lp[2];
    const float4 c = G.sph[cv.seg_off + bk];
    const float t = (float)sub * (1.f / 3.f), s = 1.f - t;
    const float w0 = s * s * s, w1 = 3.f * t * s * s, w2 = 3.f * t * t * s, w3 = t * t * t;
    const float dx = ql[0] - (c.x + (w0 * a.x + w1 * a.w + w2 * b.z + w3 * e.y));
    const float dy = ql[1] - (c.y + (w0 * a.y + w1 * b.x + w2 * b.w + w3 * e.z));
    const float dz = ql[2] - (c.z + (w0 * a.z + w1 * b.y + w2 * e.x + w3 * e.w));
    return __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz) + 1.0001f * (float)cv.tol_eff + 4e-6f * bw + eps;
}

template <int T>
__device__ __forceinline__ void stage_clusters(const DevGeom& G, const DCurve& cv, int c0, int cn, float4* st)
{
    __syncthreads();
    for (int i = threadIdx.x; i < cn; i += T) st[i] = G.csph[cv.clu_off + c0 + i];
    __syncthreads();
}

// The pieces of cluster cl that lane `sub` of a query visits (k = cl*kCluPieces
// + sub + r*L), loaded together so that their latencies overlap; ok[r] marks
// the ones inside the curve.
template <int L>
__device__ __forceinline__ void load_cluster(const DevGeom& G, const DCurve& cv, int cl, int sub, float4* p, bool* ok)
{
    static_assert(kCluPieces % L == 0, "whole pieces per lane and cluster");
#pragma unroll
    for (int r = 0; r < kCluPieces / L; ++r) {
        const int k = cl * kCluPieces + sub + r * L;
        ok[r] = cl >= 0 && k < cv.n_seg;
        p[r] = ok[r] ? G.sph[cv.seg_off + k] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

struct BoxShared {
    float4 st[kBoxChunk];
    uint16_t clu[kQueriesPerTile][kBoxCluCap];  // a curve using clusters has < 65536
    int32_t list[kQueriesPerTile][kBoxCap];
    int32_t base[kQueriesPerTile];
    int32_t next;
};

// One tile of kQueriesPerTile queries of one curve, L lanes per query.  kKeys:
// also find the K pieces with the smallest lower bounds (the network's
// candidates); the sphere-pruned call needs only the bound and the list.
template <bool kKeys, int L>
__device__ __forceinline__ void box_tile(const DevGeom& G, int tile, const int32_t* __restrict__ tile_off,
                                         const int32_t* __restrict__ q_off, const int32_t* __restrict__ perm,
                                         const double* __restrict__ qxyz, float tie_rel, const BoxOut& out,
                                         BoxShared& sh)
{
    constexpr int T = kQueriesPerTile * L;  // threads
    constexpr int kPer = kCluPieces / L;    // pieces of a cluster per lane
    static_assert(L >= kK && L <= 16 && (L & (L - 1)) == 0, "4, 8 or 16 lanes per query");
    float4* const s_st = sh.st;
    const int c = out.tile_curve[tile];
    const DCurve cv = G.curves[c];
    const int lane = threadIdx.x & 63;
    const int qs = threadIdx.x / L, sub = threadIdx.x % L;
    const int64_t j = (int64_t)q_off[c] + (int64_t)(tile - tile_off[c]) * kQueriesPerTile + qs;
    const bool active = j < q_off[c + 1];
    const int32_t qi = active ? perm[j] : 0;
    float ql[3] = {0.f, 0.f, 0.f};
    if (active) {
#pragma unroll
        for (int k = 0; k < 3; ++k) ql[k] = (float)(qxyz[3 * (int64_t)qi + k] - cv.origin[k]);
    }
    const float eps = 1e-6f * (sqrtf(ql[0] * ql[0] + ql[1] * ql[1] + ql[2] * ql[2]) + (float)cv.diag);
    // the raw hardware square root (<= 1 ulp) is inside the allowance eps
    auto dist = [&](const float4& p) {
        const float dx = ql[0] - p.x, dy = ql[1] - p.y, dz = ql[2] - p.z;
        return __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz);
    };
    float ub = INFINITY;
    uint64_t key[kK];
    int cnt = 0;  // pieces listed (same value in the query's 8 lanes)
    uint32_t nt = 0;  // sphere tests of this lane (the algorithmic work the bench reports)
    if (cv.clu_use) {
        // a. first bound: the best cluster upper bound, sharpened by the pieces
        // of the cluster with the smallest lower bound
        // this lane's nearest-bound cluster (ties to the lower index: the lane
        // visits its clusters in increasing order), then the query's
        float near_lb = INFINITY;
        int near_c = -1;
        for (int c0 = 0; c0 < cv.n_clu; c0 += kBoxChunk) {
            const int cn = min(kBoxChunk, cv.n_clu - c0);
            stage_clusters<T>(G, cv, c0, cn, s_st);
            if (!active) continue;
            for (int i = sub; i < cn; i += L) {
                const float4 p = s_st[i];
                const float d = dist(p);
                ub = fminf(ub, d + p.w + eps);
                const float v = d - p.w;
                near_c = v < near_lb ? c0 + i : near_c;
                near_lb = fminf(near_lb, v);
                ++nt;
            }
        }
#pragma unroll
        for (int off = 1; off < L; off <<= 1) {
            const float ov = __shfl_xor(near_lb, off, 64);
            const int oc = __shfl_xor(near_c, off, 64);
            const bool take = ov < near_lb || (ov == near_lb && (unsigned)oc < (unsigned)near_c);
            near_c = take ? oc : near_c;
            near_lb = take ? ov : near_lb;
        }
        // the piece of that cluster whose centre is nearest (ties to the lower
        // index, so the same piece for every lane count)
        float bd = INFINITY, bw = 0.f;
        int bk = -1;
        if (active) {
            float4 p[kPer];
            bool ok[kPer];
            load_cluster<L>(G, cv, near_c, sub, p, ok);
#pragma unroll
            for (int r = 0; r < kPer; ++r)
                if (ok[r]) {
                    const float d = dist(p[r]);
                    ub = fminf(ub, d + p[r].w + eps);
                    ++nt;
                    if (d < bd) {
                        bd = d;
                        bw = p[r].w;
                        bk = near_c * kCluPieces + sub + r * L;
                    }
                }
        }
        ub = min_lanes<L>(fminf(ub, point_bound<L>(G, cv, bd, bw, bk, sub, active, ql, eps)));
        // b. candidate clusters
        const float thr0 = ub + tie_margin(ub, cv, tie_rel);
        int ncl = 0;  // same value in the query's 8 lanes
        for (int c0 = 0; c0 < cv.n_clu; c0 += kBoxChunk) {
            const int cn = min(kBoxChunk, cv.n_clu - c0);
            stage_clusters<T>(G, cv, c0, cn, s_st);
            if (!active) continue;
            // the L lanes of a query run the same trip count: the ballot below sees all of them
            for (int i0 = 0; i0 < cn; i0 += L) {
                const int i = i0 + sub;
                bool hit = false;
                if (i < cn) {
                    const float4 p = s_st[i];
                    const float dx = ql[0] - p.x, dy = ql[1] - p.y, dz = ql[2] - p.z;
                    const float tt = thr0 + eps + p.w;  // >= 0
                    hit = dx * dx + dy * dy + dz * dz <= tt * tt;
                    ++nt;
                }
                const uint32_t grp = group_hits<L>(hit, lane);
                const int pos = ncl + __popc(grp & ((1u << sub) - 1u));
                if (hit && pos < kBoxCluCap) sh.clu[qs][pos] = (uint16_t)(c0 + i);
                ncl += __popc(grp);
            }
        }
        // c. UB and the K nearest-bound pieces over the candidate clusters, and
        // every piece whose lower bound reaches the running UB + margin (UB
        // only falls, so this holds the final list)
        const bool clus_ok = ncl <= kBoxCluCap;
#pragma unroll
        for (int k = 0; k < kK; ++k) key[k] = ~0ull;
        int pre = 0;  // pieces kept so far (same value in the query's 8 lanes)
        bd = INFINITY;
        bk = -1;
        if (active && clus_ok) {
            for (int m = 0; m < ncl; ++m) {
                const int cl = sh.clu[qs][m];
                float4 p[kPer];
                bool ok[kPer];
                load_cluster<L>(G, cv, cl, sub, p, ok);
                float lbv[kPer];
#pragma unroll
                for (int r = 0; r < kPer; ++r) {
                    const float d = dist(p[r]), re = p[r].w + eps;
                    lbv[r] = d - p[r].w - eps;
                    if (ok[r]) {
                        ub = fminf(ub, d + re);
                        if (d < bd) {
                            bd = d;
                            bw = p[r].w;
                            bk = cl * kCluPieces + sub + r * L;
                        }
                        if constexpr (kKeys)
                            insert_key(key, ((uint64_t)ord_key(d - re) << 32) | (uint32_t)(cl * kCluPieces + sub + r * L));
                        ++nt;
                    }
                }
                ub = min_lanes<L>(ub);
                const float thr_run = ub + tie_margin(ub, cv, tie_rel);
                bool any = false;
#pragma unroll
                for (int r = 0; r < kPer; ++r) any |= ok[r] && lbv[r] <= thr_run;
                if (group_hits<L>(any, lane) == 0u) continue;  // most clusters add no piece
#pragma unroll
                for (int r = 0; r < kPer; ++r) {
                    const bool hit = ok[r] && lbv[r] <= thr_run;
                    const uint32_t grp = group_hits<L>(hit, lane);
                    const int pos = pre + __popc(grp & ((1u << sub) - 1u));
                    if (hit && pos < kBoxCap) sh.list[qs][pos] = cl * kCluPieces + sub + r * L;
                    pre += __popc(grp);
                }
            }
        }
        // the same point bound for the nearest-centre piece of all candidate clusters
        ub = min_lanes<L>(fminf(ub, point_bound<L>(G, cv, bd, bw, bk, sub, active && clus_ok, ql, eps)));
        if constexpr (kKeys) merge_keys<L>(key);
        // d. the list: the kept pieces whose lower bound reaches the final UB +
        // margin, in visiting order; if more than kBoxCap were kept, a second
        // pass over the candidate clusters
        const float thr = ub + tie_margin(ub, cv, tie_rel);
        if (active && clus_ok && pre <= kBoxCap) {
            for (int i0 = 0; i0 < pre; i0 += L) {
                const int i = i0 + sub;
                bool hit = false;
                int k = 0;
                if (i < pre) {
                    k = sh.list[qs][i];
                    const float4 p = G.sph[cv.seg_off + k];
                    hit = dist(p) - p.w - eps <= thr;
                    if (hit) hit = capsule_lb(G, cv, k, p, ql) - eps <= thr;
                    ++nt;
                }
                // every lane has read its entry before any is overwritten: the
                // write position is below i0 + L
                const uint32_t grp = group_hits<L>(hit, lane);
                const int pos = cnt + __popc(grp & ((1u << sub) - 1u));
                if (hit) sh.list[qs][pos] = k;
                cnt += __popc(grp);
            }
        } else if (active && clus_ok) {
            for (int m = 0; m < ncl; ++m) {
                const int cl = sh.clu[qs][m];
                float4 p[kPer];
                bool ok[kPer];
                load_cluster<L>(G, cv, cl, sub, p, ok);
#pragma unroll
                for (int r = 0; r < kPer; ++r) {
                    bool hit = ok[r] && dist(p[r]) - p[r].w - eps <= thr;
                    if (hit) hit = capsule_lb(G, cv, cl * kCluPieces + sub + r * L, p[r], ql) - eps <= thr;
                    nt += ok[r];
                    const uint32_t grp = group_hits<L>(hit, lane);
                    const int pos = cnt + __popc(grp & ((1u << sub) - 1u));
                    if (hit && pos < kBoxCap) sh.list[qs][pos] = cl * kCluPieces + sub + r * L;
                    cnt += __popc(grp);
                }
            }
        } else if (active) {
            cnt = kBoxCap + 1;  // too many clusters: the full scan
        }
    } else {
        // one pass over the curve's piece spheres staged in LDS for the bound and
        // the K nearest, a second one for the list
#pragma unroll
        for (int k = 0; k < kK; ++k) key[k] = ~0ull;
        float thr = 0.f;
        for (int pass = 0; pass < 2; ++pass) {
            for (int c0 = 0; c0 < cv.n_seg; c0 += kBoxChunk) {
                const int cn = min(kBoxChunk, cv.n_seg - c0);
                __syncthreads();
                for (int i = threadIdx.x; i < cn; i += T) s_st[i] = G.sph[cv.seg_off + c0 + i];
                __syncthreads();
                if (!active) continue;
                if (pass == 0) {
                    for (int i = sub; i < cn; i += L) {
                        const float4 p = s_st[i];
                        const float dx = ql[0] - p.x, dy = ql[1] - p.y, dz = ql[2] - p.z;
                        const float d2 = dx * dx + dy * dy + dz * dz;
                        const float re = p.w + eps;
                        ++nt;
                        const float t4 = ord_val((uint32_t)(key[kK - 1] >> 32)) + re;
                        const float tu = ub - re;
                        const bool c4 = kKeys && (key[kK - 1] == ~0ull || (t4 > 0.f && d2 < t4 * t4));
                        const bool cu = tu > 0.f && d2 < tu * tu;
                        if (c4 || cu) {
                            const float d = __builtin_amdgcn_sqrtf(d2);
                            ub = fminf(ub, d + re);
                            uint64_t x = ((uint64_t)ord_key(d - re) << 32) | (uint32_t)(c0 + i);
#pragma unroll
                            for (int k = 0; k < kK; ++k) cswap(key[k], x);  // insertion into the sorted list
                        }
                    }
                } else {
                    // the L lanes of a query run the same trip count: the ballot sees all of them
                    for (int i0 = 0; i0 < cn; i0 += L) {
                        const int i = i0 + sub;
                        bool hit = false;
                        if (i < cn) {
                            const float4 p = s_st[i];
                            const float dx = ql[0] - p.x, dy = ql[1] - p.y, dz = ql[2] - p.z;
                            const float tt = thr + p.w + eps;
                            hit = tt >= 0.f && dx * dx + dy * dy + dz * dz <= tt * tt;
                            if (hit) hit = capsule_lb(G, cv, c0 + i, p, ql) - eps <= thr;
                            ++nt;
                        }
                        const uint32_t grp = group_hits<L>(hit, lane);
                        const int pos = cnt + __popc(grp & ((1u << sub) - 1u));
                        if (hit && pos < kBoxCap) sh.list[qs][pos] = c0 + i;
                        cnt += __popc(grp);
                    }
                }
            }
            if (pass == 0) {
                merge_keys<L>(key);
                ub = min_lanes<L>(ub);
                thr = ub + tie_margin(ub, cv, tie_rel);
            }
        }
    }
    // the workgroup's sphere tests: one atomic per wave into a counter chosen by the slot
    {
        unsigned long long w = nt;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off, 64);
        if (lane == 0 && out.tests) atomicAdd(&out.tests[blockIdx.x % kWsCounters], w);
    }
    // reserve the workgroup's pairs with one atomic
    const bool listed = active && cnt <= kBoxCap;
    if (sub == 0) sh.base[qs] = listed ? cnt : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < kQueriesPerTile; ++k) {
            const int v = sh.base[k];
            sh.base[k] = tot;
            tot += v;
        }
        const int base = tot > 0 ? atomicAdd(out.so.pair_count, tot) : 0;
        for (int k = 0; k < kQueriesPerTile; ++k) sh.base[k] += base;
    }
    __syncthreads();
    if (!active) return;
    const int64_t b = sh.base[qs];
    const bool fits = listed && b + cnt <= out.so.pair_cap;
    if (sub == 0) {
        out.so.cand_n[j] = fits ? cnt : -1;
        out.so.pair_off[j] = (int32_t)b;
        out.so.ub[j] = ub;
        if constexpr (kKeys) {
#pragma unroll
            for (int k = 0; k < kK; ++k)
                out.cand[j * kK + k] = key[k] == ~0ull ? -1 : (int32_t)(cv.seg_off + (uint32_t)key[k]);
        }
    }
    if (listed) {
        for (int k = sub; k < cnt; k += L) {
            if (b + k >= out.so.pair_cap) break;
            out.so.pair_seg[b + k] = fits ? (int32_t)(cv.seg_off + sh.list[qs][k]) : 0;
            out.so.pair_j[b + k] = fits ? (int32_t)j : -1;  // a slot past the capacity stays unused
        }
    }
    if (kKeys && out.xb && sub < kK) {
        const uint64_t kk = sub == 0 ? key[0] : (sub == 1 ? key[1] : (sub == 2 ? key[2] : key[3]));
        float f[kCurveIn];
#pragma unroll
        for (int k = 0; k < kCurveIn; ++k) f[k] = 0.f;
        if (kk != ~0ull) {
            const double q[3] = {qxyz[3 * (int64_t)qi], qxyz[3 * (int64_t)qi + 1], qxyz[3 * (int64_t)qi + 2]};
            pair_features(G, cv, cv.seg_off + (uint32_t)kk, q, f);
        }
        uint32_t w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint16_t lo = __builtin_bit_cast(uint16_t, (__bf16)f[2 * k]);
            const uint16_t hi = 2 * k + 1 < kCurveIn ? __builtin_bit_cast(uint16_t, (__bf16)f[2 * k + 1]) : (uint16_t)0;
            w[k] = (uint32_t)lo | ((uint32_t)hi << 16);
        }
        uint4* dst = reinterpret_cast<uint4*>(out.xb + (j * kK + sub) * 16);
        dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
        dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
    }
}

template <bool kKeys, int L, bool kPersist>
__global__ __launch_bounds__(kQueriesPerTile * L) void k_box(DevGeom G, const int32_t* __restrict__ tile_off,
                                                             const int32_t* __restrict__ q_off,
                                                             const int32_t* __restrict__ perm,
                                                             const double* __restrict__ qxyz, float tie_rel, BoxOut out)
{
    __shared__ BoxShared sh;
    const int n_tiles = tile_off[G.n_curves];
    const int per = (n_tiles + kXcds - 1) / kXcds;  // tiles of each XCD's contiguous range
    if constexpr (!kPersist) {
        // workgroups are dispatched to the XCDs in turn: workgroup b runs on XCD b % kXcds
        const int slot = (int)(blockIdx.x / kXcds);
        const int tile = (int)(blockIdx.x % kXcds) * per + slot;
        if (slot >= per || tile >= n_tiles) return;
        box_tile<kKeys, L>(G, tile, tile_off, q_off, perm, qxyz, tie_rel, out, sh);
    } else {
        // the next tile of this XCD's range, then of the others in turn; every
        // workgroup leaves once all kXcds queues are past their ranges
        int x = (int)(blockIdx.x % kXcds);
        for (int hop = 0; hop < kXcds;) {
            __syncthreads();  // the previous tile is done with sh
            if (threadIdx.x == 0) sh.next = atomicAdd(&out.queue[x], 1);
            __syncthreads();
            const int t = sh.next;
            const int tile = x * per + t;
            if (t >= per || tile >= n_tiles) {
                ++hop;
                x = (x + 1) % kXcds;
                continue;
            }
            box_tile<kKeys, L>(G, tile, tile_off, q_off, perm, qxyz, tie_rel, out, sh);
        }
    }
}

// ---------------------------------------------------------------------------
// Certificate helpers
// ---------------------------------------------------------------------------
// Piece s relative to the query in its local frame: R_i = P_i - q (Bernstein
// control points of C - q), D_j = 3 (P_{j+1} - P_j) (of C').
struct BezQ {
    float R[4][3];
    float D[3][3];
    float qn;   // |q - c_s|
    float rad;  // max |P_i - c_s|
};

__device__ __forceinline__ void load_bezq(const DevGeom& G, const DCurve& cv, int64_t s, const double* q, BezQ& b)
{
    const float* lp = G.lcp + s * 12;
    const float* ax = G.aux + s * 8;
    const float ql[3] = {(float)(q[0] - (cv.origin[0] + (double)ax[AUX_CX])),
                         (float)(q[1] - (cv.origin[1] + (double)ax[AUX_CY])),
                         (float)(q[2] - (cv.origin[2] + (double)ax[AUX_CZ]))};
    float P[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) P[i] = lp[i];
    float r2 = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        r2 = fmaxf(r2, P[3 * i] * P[3 * i] + P[3 * i + 1] * P[3 * i + 1] + P[3 * i + 2] * P[3 * i + 2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) b.R[i][c] = P[3 * i + c] - ql[c];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) b.D[i][c] = 3.f * (P[3 * (i + 1) + c] - P[3 * i + c]);
    b.qn = sqrtf(ql[0] * ql[0] + ql[1] * ql[1] + ql[2] * ql[2]);
    b.rad = sqrtf(r2);
}

// Sphere lower bound of the distance from q to the exact curve over piece s.
__device__ __forceinline__ float sphere_lb(const BezQ& b, const DCurve& cv)
{
    return b.qn * (1.f - 1e-6f) - b.rad * (1.f + 1e-6f) - (float)(cv.tol_eff * 1.000001);
}

__device__ __forceinline__ float dot3f(const float* a, const float* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
__device__ __forceinline__ float norm3f(const float* a) { return sqrtf(dot3f(a, a)); }

// Bernstein coefficients beta_k (k = 0..5) of f(u) = (C(u) - q).C'(u) and a
// bound e_k on their rounding: B^3_i B^2_j = C(3,i) C(2,j) / C(5,i+j) B^5_{i+j}.
// Returns the sign class: +1 every beta_k > e_k, -1 every beta_k < -e_k,
// 2 one sign change from clearly negative to clearly positive, 0 otherwise.
// relax0 / relax5 let beta_0 / beta_5 sit within its rounding band (a piece
// adjacent to the chosen one shares that endpoint with it).
__device__ __forceinline__ int fprime_class(const BezQ& b, bool relax0, bool relax5)
{
    float dd[4][3], aa[4][3];
    float nR[4], nD[3];
#pragma unroll
    for (int i = 0; i < 4; ++i) nR[i] = norm3f(b.R[i]) + b.qn;
#pragma unroll
    for (int j = 0; j < 3; ++j) nD[j] = norm3f(b.D[j]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            dd[i][j] = dot3f(b.R[i], b.D[j]);
            aa[i][j] = nR[i] * nD[j];
        }
    float be[6], er[6];
    be[0] = dd[0][0];
    be[1] = 0.6f * dd[1][0] + 0.4f * dd[0][1];
    be[2] = 0.3f * dd[2][0] + 0.6f * dd[1][1] + 0.1f * dd[0][2];
    be[3] = 0.1f * dd[3][0] + 0.6f * dd[2][1] + 0.3f * dd[1][2];
    be[4] = 0.4f * dd[3][1] + 0.6f * dd[2][2];
    be[5] = dd[3][2];
    er[0] = aa[0][0];
    er[1] = 0.6f * aa[1][0] + 0.4f * aa[0][1];
    er[2] = 0.3f * aa[2][0] + 0.6f * aa[1][1] + 0.1f * aa[0][2];
    er[3] = 0.1f * aa[3][0] + 0.6f * aa[2][1] + 0.3f * aa[1][2];
    er[4] = 0.4f * aa[3][1] + 0.6f * aa[2][2];
    er[5] = aa[3][2];
    bool pos = true, neg = true, amb = false;
    int changes = 0, prev = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float e = 1e-6f * er[k];
        const bool relaxed = (k == 0 && relax0) || (k == 5 && relax5);
        const int sg = be[k] > e ? 1 : (be[k] < -e ? -1 : 0);
        pos = pos && (sg > 0 || (relaxed && be[k] >= -e));
        neg = neg && (sg < 0 || (relaxed && be[k] <= e));
        if (sg == 0) amb = true;
        if (sg != 0) {
            if (prev != 0 && sg != prev) ++changes;
            prev = sg;
        }
    }
    if (pos) return 1;
    if (neg) return -1;
    if (!amb && changes == 1 && be[0] < 0.f) return 2;
    return 0;
}

__device__ __forceinline__ float end_dist(const BezQ& b, int i) { return norm3f(b.R[i]); }

// ---------------------------------------------------------------------------
// Seed + certificate: one thread per sorted query position.  Certified queries
// are finished and marked done; the others are left to the refine over their
// sphere lists (k_pairs / k_finish), which also covers list overflows.
// ---------------------------------------------------------------------------
// 4 waves per SIMD (128 VGPRs from 183): the certificate stage on the batched
// curves 3.23 -> 2.69 ms
#ifndef MREP_DECIDE_MIN_WAVES
#define MREP_DECIDE_MIN_WAVES 4
#endif
template <bool kGen>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(MREP_DECIDE_MIN_WAVES, 8))) void k_decide(DevGeom G, const int32_t* __restrict__ cid,
                                                const double* __restrict__ qxyz, const int32_t* __restrict__ q_off,
                                                const int32_t* __restrict__ perm, BoxOut box,
                                                const float2* __restrict__ scores, float tie_rel, int32_t invert,
                                                uint8_t* __restrict__ done, Outs o)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q_off[G.n_curves]) return;
    const int n_list = box.so.cand_n[j];
    if (n_list <= 0) {
        done[j] = 0;
        return;
    }
    const int32_t qi = perm[j];
    const DCurve cv = G.curves[cid[qi]];
    const double q[3] = {qxyz[3 * (int64_t)qi], qxyz[3 * (int64_t)qi + 1], qxyz[3 * (int64_t)qi + 2]};
    const int64_t p0 = box.so.pair_off[j];
    const int64_t s_first = cv.seg_off, s_last = cv.seg_off + cv.n_seg - 1;
    // 1. best-scored candidate
    int64_t s = -1;
    float best = -INFINITY, u0 = 0.5f;
#pragma unroll
    for (int k = 0; k < kK; ++k) {
        const int32_t sk = box.cand[j * kK + k];
        const float2 y = scores[j * kK + k];
        if (sk >= 0 && (s < 0 || y.y > best)) { s = sk; best = y.y; u0 = y.x; }
    }
    bool ok = s >= 0, certified = false;
    float u = 0.f, d2 = INFINITY, kap = 1.f;
    float u_sec = 0.f, d_sec = INFINITY;  // a second distinct local minimum of the chosen piece
    Cubic<float> C;
    Cand b2 = empty_cand(cv);
    // at most 3 attempts: a failed certificate that found a strictly closer piece restarts there
    for (int attempt = 0; ok && !certified && attempt < 3; ++attempt) {
        u0 = fminf(fmaxf(u0, 0.f), 1.f);
        // 2. walk to the piece holding the minimum, then its certified minimum
        int cls = 0;
        for (int hop = 0; ok; ++hop) {
            BezQ bq;
            load_bezq(G, cv, s, q, bq);
            cls = fprime_class(bq, false, false);
            if (cls == 1 && s > s_first) {
                if (hop == 4) ok = false;
                else { --s; u0 = 1.f; }
            } else if (cls == -1 && s < s_last) {
                if (hop == 4) ok = false;
                else { ++s; u0 = 0.f; }
            } else {
                break;
            }
        }
        if (!ok) break;
        load_cubic(G, cv, s, q, C);
        kap = 1.f;
        d_sec = INFINITY;
        if (cls == 1) { u = 0.f; d2 = C.dist2(0.f); }
        else if (cls == -1) { u = 1.f; d2 = C.dist2(1.f); }
        else {
            if (cls == 2) {
                newton_min(C, 0.f, 1.f, u0, u, d2, kap);
                // orthogonality residual of the Newton point: cosine <= 1e-4, or coincidence
                V3<float> r, d1, dd2;
                C.eval(u, r, d1, dd2);
                const float rn = sqrtf(dot(r, r)), sp = sqrtf(dot(d1, d1));
                const bool conv = u > 0.f && u < 1.f &&
                                  (fabsf(dot(r, d1)) <= 1e-4f * rn * sp || rn <= 1e-7f * (float)cv.diag);
                if (!conv) cls = 0;
            }
            if (cls == 0) piece_min(C, u, d2, kap, u_sec, d_sec);
        }
        const float ds = sqrtf(d2);
        // 3. certificate over the listed pieces (an unlisted piece's sphere lower bound
        // exceeds UB + margin >= d* + margin): each other piece whose sphere reaches
        // lim must have a certified minimum above lim.  A monotone piece's minimum is
        // an endpoint distance, any other piece's is its certified piece minimum.  The
        // neighbour whose minimum is the endpoint it shares with the chosen piece is
        // kept as the runner-up for the tie test instead.
        const float lim = ds + tie_margin(ds, cv, tie_rel);
        b2 = empty_cand(cv);
        bool fail = false;
        int64_t better = -1;
        float better_d = ds * (1.f - 1e-5f), better_u = 0.5f;
        for (int i = 0; i < n_list; ++i) {
            const int64_t s2 = box.so.pair_seg[p0 + i];
            if (s2 == s) continue;
            BezQ n;
            load_bezq(G, cv, s2, q, n);
            if (sphere_lb(n, cv) > lim) continue;
            const bool adj_r = s2 == s + 1, adj_l = s2 == s - 1;
            const int c2 = fprime_class(n, adj_r, adj_l);
            float mn, um;
            int end = -1;
            if (c2 == 1) { mn = end_dist(n, 0); end = 0; um = 0.f; }
            else if (c2 == -1) { mn = end_dist(n, 3); end = 3; um = 1.f; }
            else {
                Cubic<float> C2;
                load_cubic(G, cv, s2, q, C2);
                float dd, kk;
                piece_min(C2, um, dd, kk);
                mn = sqrtf(dd) * (1.f - 8e-6f);
            }
            if (mn > lim) continue;
            if ((adj_r && end == 0) || (adj_l && end == 3)) {
                const Cand e = make_cand(G, s2, end == 0 ? 0.0 : 1.0, (double)mn * mn, 1.0, 0.0);
                if (e.d2 < b2.d2) b2 = e;
                continue;
            }
            fail = true;
            if (mn < better_d) { better_d = mn; better = s2; better_u = um; }
        }
        if (!fail) { certified = true; break; }
        if (better < 0) ok = false;
        else { s = better; u0 = better_u; }
    }
    if (!certified) {
        done[j] = 0;
        return;
    }
    done[j] = 1;
    const double ta = G.segt[2 * s], tb = G.segt[2 * s + 1];
    const Cand b1 = make_cand(G, s, (double)u, (double)d2, (double)kap, param_error(C, u, kap, ta, tb));
    if (d_sec < INFINITY) {  // two minima on the chosen piece: the second is the tie test's runner-up
        const Cand c2 = make_cand_q(G, cv, s, (double)u_sec, (double)d_sec, 1.0, 0.0, q);
        if (!c2.across && c2.d2 < b2.d2) b2 = c2;
    }
    finish<float, kGen>(G, cv, q, b1, b2, 0u, (double)tie_rel, invert, qi, o);
}

// Training-data export: candidates and features in the caller's query order.
__global__ void k_feat_write(DevGeom G, const int32_t* __restrict__ cid, const double* __restrict__ qxyz,
                             const int32_t* __restrict__ q_off, const int32_t* __restrict__ perm,
                             const int32_t* __restrict__ cand, int32_t* __restrict__ seg_out, float* __restrict__ x_out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q_off[G.n_curves]) return;
    const int32_t qi = perm[j];
    const DCurve cv = G.curves[cid[qi]];
    const double q[3] = {qxyz[3 * (int64_t)qi], qxyz[3 * (int64_t)qi + 1], qxyz[3 * (int64_t)qi + 2]};
    for (int k = 0; k < kK; ++k) {
        const int32_t s = cand[j * kK + k];
        float f[kCurveIn];
        for (int i = 0; i < kCurveIn; ++i) f[i] = 0.f;
        if (s >= 0) pair_features(G, cv, s, q, f);
        seg_out[(int64_t)qi * kK + k] = s >= 0 ? (int32_t)(s - cv.seg_off) : -1;
        for (int i = 0; i < kCurveIn; ++i) x_out[((int64_t)qi * kK + k) * kCurveIn + i] = f[i];
    }
}

__global__ void k_fill_feat(int64_t n, int32_t* __restrict__ seg_out, float* __restrict__ x_out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * kK) return;
    seg_out[i] = -1;
    for (int k = 0; k < kCurveIn; ++k) x_out[i * kCurveIn + k] = 0.f;
}


// Workspace of the seeded call.
constexpr int64_t kSpherePairsPerQuery = 24;  // average listed pieces per query the pair arrays hold
struct SeedWork {
    int32_t *hist, *q_off, *tile_off, *perm, *ovf_list, *ovf_count;
    BoxOut box;
    PairRes* pair_res;
    float2* scores;
    uint8_t* done;
};

int64_t seed_layout(int64_t nc, int64_t n, char* base, SeedWork* w)
{
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        int64_t o = off;
        off = a256(off + bytes);
        return o;
    };
    const int64_t cap = std::min<int64_t>(kSpherePairsPerQuery * n + 1024, (int64_t)INT32_MAX);
    const int64_t oh = take(4 * (nc + 2)), otc = take(8 * kWsCounters), oq = take(4 * (nc + 1)),
                  ot = take(4 * (nc + 1)), op = take(4 * n);
    const int64_t oov = take(4 * n), oc = take(4 * n * kK), oxb = take(32 * n * kK), ocn = take(4 * n);
    const int64_t opo = take(4 * n), oub = take(4 * n), ops = take(4 * cap), opj = take(4 * cap);
    const int64_t opr = take((int64_t)sizeof(PairRes) * cap), osc = take(8 * n * kK), odn = take(n);
    const int64_t oqu = take(4 * kXcds), otcv = take(4 * (nc + (n + kQueriesPerTile - 1) / kQueriesPerTile + kXcds));
    if (w) {
        w->hist = (int32_t*)(base + oh); w->q_off = (int32_t*)(base + oq); w->tile_off = (int32_t*)(base + ot);
        w->perm = (int32_t*)(base + op); w->ovf_list = (int32_t*)(base + oov);
        w->ovf_count = w->hist + nc;  // zeroed by the grouping, like the pair counter after it
        w->box.cand = (int32_t*)(base + oc);
        w->box.tests = (unsigned long long*)(base + otc);
        w->box.queue = (int32_t*)(base + oqu);
        w->box.tile_curve = (int32_t*)(base + otcv);
        w->box.xb = (uint16_t*)(base + oxb);
        w->box.so.cand_n = (int32_t*)(base + ocn);
        w->box.so.pair_off = (int32_t*)(base + opo);
        w->box.so.ub = (float*)(base + oub);
        w->box.so.pair_seg = (int32_t*)(base + ops);
        w->box.so.pair_j = (int32_t*)(base + opj);
        w->box.so.pair_count = w->hist + nc + 1;
        w->box.so.pair_cap = cap;
        w->pair_res = (PairRes*)(base + opr);
        w->scores = (float2*)(base + osc);
        w->done = (uint8_t*)(base + odn);
    }
    return off;
}

}  // namespace

struct mrep_nn {
    uint8_t* base = nullptr;  // device: params | m | v | grad | image
    int64_t step = 0;
    int kind = MREP_NN_CURVE;
    int compute = MREP_NN_COMPUTE_BF16;  // products of mrep_nn_forward / mrep_nn_train_step
    NetDims d;
    float* params() const { return (float*)base; }
    float* m() const { return (float*)(base + d.param_bytes); }
    float* v() const { return (float*)(base + 2 * d.param_bytes); }
    float* grad() const { return (float*)(base + 3 * d.param_bytes); }
    uint8_t* img() const { return base + 4 * d.param_bytes; }
};

static bool known_kind(int32_t kind) { return kind == MREP_NN_CURVE || kind == MREP_NN_SURFACE; }

static int pack_image(const mrep_nn* nn, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack, dim3(blocks_for(nn->d.img_bytes / 2)), dim3(256), 0, st, nn->d,
                       (const float*)nn->params(), nn->img());
    NN_HIP(hipGetLastError());
    return MREP_OK;
}

// grouping + sphere candidates shared by the seeded call and the feature export
__global__ void k_zero_counters(unsigned long long* __restrict__ p, int64_t n, int32_t* __restrict__ queue)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
    if (i < kXcds) queue[i] = 0;
}

constexpr int kMaxDevices = 64;

// the curve of every tile: one thread per curve writes its tiles
__global__ __launch_bounds__(256) void k_box_tiles(const int32_t* __restrict__ tile_off, int32_t n_curves,
                                                  int32_t* __restrict__ tile_curve)
{
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= n_curves) return;
    for (int t = tile_off[c]; t < tile_off[c + 1]; ++t) tile_curve[t] = c;
}

// one schedule of the box kernel; a persistent grid holds as many workgroups
// as the device keeps resident at once (the occupancy is queried once per
// device and schedule)
template <bool kKeys, int L, bool kPersist>
static hipError_t launch_box_t(const mrep_geom* geom, int64_t tiles, const SeedWork& w, const double* q_xyz,
                               float tie_rel, hipStream_t st)
{
    constexpr int T = kQueriesPerTile * L;
    int64_t grid = tiles;
    if (kPersist) {
        static std::atomic<int> cap[kMaxDevices];  // resident workgroups of the device (0: not queried yet)
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
        int c = cap[dev].load(std::memory_order_relaxed);
        if (c == 0) {
            int cus = 0, per_cu = 0;
            if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
            if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_box<kKeys, L, kPersist>, T, 0)) !=
                hipSuccess)
                return e;
            c = std::max(1, cus) * std::max(1, per_cu);
            cap[dev].store(c, std::memory_order_relaxed);
        }
        grid = std::min<int64_t>(tiles, c);
    }
    hipLaunchKernelGGL((k_box<kKeys, L, kPersist>), dim3((unsigned)grid), dim3(T), 0, st, dev_view(geom->g),
                       (const int32_t*)w.tile_off, (const int32_t*)w.q_off, (const int32_t*)w.perm, q_xyz, tie_rel,
                       w.box);
    return hipGetLastError();
}

template <bool kKeys>
static hipError_t launch_box(const mrep_geom* geom, int64_t tiles, const SeedWork& w, const double* q_xyz,
                             float tie_rel, hipStream_t st)
{
    const bool p = geom->box_persist != 0;
    switch (geom->box_lanes) {
    case 4: return p ? launch_box_t<kKeys, 4, true>(geom, tiles, w, q_xyz, tie_rel, st)
                     : launch_box_t<kKeys, 4, false>(geom, tiles, w, q_xyz, tie_rel, st);
    case 16: return p ? launch_box_t<kKeys, 16, true>(geom, tiles, w, q_xyz, tie_rel, st)
                      : launch_box_t<kKeys, 16, false>(geom, tiles, w, q_xyz, tie_rel, st);
    default: return p ? launch_box_t<kKeys, 8, true>(geom, tiles, w, q_xyz, tie_rel, st)
                      : launch_box_t<kKeys, 8, false>(geom, tiles, w, q_xyz, tie_rel, st);
    }
}

static int candidates(const mrep_geom* geom, int64_t n, const int32_t* curve_id, const double* q_xyz, float tie_rel,
                      SeedWork& w, const Outs& o, hipStream_t st, bool keys, bool timed)
{
    const int64_t nc = geom->g.L.n_curves;
    NN_HIP(launch_grouping(nc, n, nullptr, curve_id, w.hist, w.q_off, w.tile_off, w.perm, o, st));
    int rc;
    if (timed && (rc = stage_mark(1, st))) return rc;
    hipLaunchKernelGGL(k_zero_counters, dim3(kWsCounters / 256), dim3(256), 0, st, w.box.tests, (int64_t)kWsCounters,
                       w.box.queue);
    // an upper bound of the tile count (tiles of a curve: ceil(its queries / kQueriesPerTile)), plus one per XCD
    const int64_t tiles = nc + (n + kQueriesPerTile - 1) / kQueriesPerTile + kXcds;
    hipLaunchKernelGGL(k_box_tiles, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, (const int32_t*)w.tile_off,
                       (int32_t)nc, w.box.tile_curve);
    NN_HIP(keys ? launch_box<true>(geom, tiles, w, q_xyz, tie_rel, st)
                : launch_box<false>(geom, tiles, w, q_xyz, tie_rel, st));
    return MREP_OK;
}

namespace mrep {

int nn_kind(const mrep_nn* nn) { return nn ? nn->kind : -1; }

int nn_score_surface_pairs(const mrep_nn* nn, const int32_t* q_off, int32_t n_surf, const int32_t* cand,
                           const uint16_t* xb, float4* out, int64_t n_rows, hipStream_t st)
{
    int rc = pack_image(nn, st);
    if (rc) return rc;
    RowsFromSurfCandidates rows{q_off, n_surf, cand, xb, out};
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n_rows + 63) / 64, 2048));
    hipLaunchKernelGGL(k_mlp<RowsFromSurfCandidates>, dim3(nb), dim3(256), 0, st, rows, (const uint8_t*)nn->img());
    NN_HIP(hipGetLastError());
    return MREP_OK;
}

}  // namespace mrep

extern "C" {

int32_t mrep_nn_param_count(int32_t kind) { return known_kind(kind) ? (int32_t)net_dims(kind).n : -1; }

int32_t mrep_nn_bytes(int32_t kind, int64_t batch, int64_t* state_bytes, int64_t* work_bytes)
{
    if (!known_kind(kind) || batch < 0 || (!state_bytes && !work_bytes)) {
        set_error("mrep_nn_bytes: unknown kind, negative batch or no output");
        return MREP_E_INVALID_ARG;
    }
    const NetDims d = net_dims(kind);
    if (state_bytes) *state_bytes = d.state_bytes;
    if (work_bytes) *work_bytes = train_layout(d, batch, nullptr, nullptr);
    return MREP_OK;
}

int32_t mrep_nn_bind(int32_t kind, void* dev_state, int64_t bytes, mrep_nn** out)
{
    if (!dev_state || !out || !known_kind(kind)) {
        set_error("mrep_nn_bind: null pointer or unknown kind");
        return MREP_E_INVALID_ARG;
    }
    *out = nullptr;
    const NetDims d = net_dims(kind);
    if (bytes < d.state_bytes) {
        set_error("mrep_nn_bind: buffer smaller than mrep_nn_bytes' state size");
        return MREP_E_SMALL_BUFFER;
    }
    if (((uintptr_t)dev_state & 255) != 0) {
        set_error("mrep_nn_bind: buffer not 256-byte aligned");
        return MREP_E_INVALID_ARG;
    }
    int rc = check_device();
    if (rc) return rc;
    mrep_nn* n = new mrep_nn();
    n->base = (uint8_t*)dev_state;
    n->kind = kind;
    n->d = d;
    *out = n;
    return MREP_OK;
}

void mrep_nn_release(mrep_nn* nn) { delete nn; }

int32_t mrep_nn_set_params(mrep_nn* nn, const float* host, int64_t n, void* stream)
{
    if (!nn || !host || n != nn->d.n) {
        set_error("mrep_nn_set_params: null pointer or wrong parameter count");
        return MREP_E_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    const int64_t np = nn->d.n;
    std::vector<float> zero((size_t)np, 0.f);
    NN_HIP(hipMemcpyAsync(nn->params(), host, 4 * np, hipMemcpyHostToDevice, st));
    NN_HIP(hipMemcpyAsync(nn->m(), zero.data(), 4 * np, hipMemcpyHostToDevice, st));
    NN_HIP(hipMemcpyAsync(nn->v(), zero.data(), 4 * np, hipMemcpyHostToDevice, st));
    NN_HIP(hipMemcpyAsync(nn->grad(), zero.data(), 4 * np, hipMemcpyHostToDevice, st));
    // pageable host sources: complete before returning
    NN_HIP(hipStreamSynchronize(st));
    nn->step = 0;
    return MREP_OK;
}

int32_t mrep_nn_get_params(const mrep_nn* nn, float* host, int64_t n, void* stream)
{
    if (!nn || !host || n != nn->d.n) {
        set_error("mrep_nn_get_params: null pointer or wrong parameter count");
        return MREP_E_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    NN_HIP(hipMemcpyAsync(host, nn->params(), 4 * nn->d.n, hipMemcpyDeviceToHost, st));
    NN_HIP(hipStreamSynchronize(st));
    return MREP_OK;
}

int32_t mrep_nn_init(mrep_nn* nn, uint64_t seed, void* stream)
{
    if (!nn) {
        set_error("mrep_nn_init: null pointer");
        return MREP_E_INVALID_ARG;
    }
    // weights uniform in +-1/sqrt(fan_in), biases zero
    const NetDims& d = nn->d;
    std::vector<float> p((size_t)d.n, 0.f);
    uint64_t s = seed;
    auto fill = [&](int64_t off, int64_t count, int fan_in) {
        const double a = 1.0 / sqrt((double)fan_in);
        for (int64_t i = 0; i < count; ++i) {
            const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
            p[(size_t)(off + i)] = (float)((2.0 * u - 1.0) * a);
        }
    };
    fill(d.oW1, (int64_t)kH * d.in, d.in);
    fill(d.oW2, (int64_t)kH * kH, kH);
    fill(d.oW3, (int64_t)d.out * kH, kH);
    return mrep_nn_set_params(nn, p.data(), d.n, stream);
}

int32_t mrep_nn_forward(const mrep_nn* nn, int64_t n, const float* x, float* y, void* work, int64_t work_bytes,
                        void* stream)
{
    if (!nn || n < 0 || (n > 0 && (!x || !y || !work))) {
        set_error("mrep_nn_forward: null pointer or negative n");
        return MREP_E_INVALID_ARG;
    }
    if (n == 0) return MREP_OK;
    if (n > INT32_MAX / kH) {
        set_error("mrep_nn_forward: n too large for one call");
        return MREP_E_INVALID_ARG;
    }
    TrainWork w;
    if (work_bytes < train_layout(nn->d, n, (char*)work, &w)) {
        set_error("mrep_nn_forward: work buffer smaller than mrep_nn_bytes(kind, n)");
        return MREP_E_SMALL_BUFFER;
    }
    hipStream_t st = (hipStream_t)stream;
    t_gemm_fp32 = nn->compute == MREP_NN_COMPUTE_FP32;
    int rc = forward(nn->d, nn->params(), n, x, w, st);
    t_gemm_fp32 = false;
    if (rc) return rc;
    NN_HIP(hipMemcpyAsync(y, w.Y, 4 * n * nn->d.out, hipMemcpyDeviceToDevice, st));
    return MREP_OK;
}

int32_t mrep_nn_set_compute(mrep_nn* nn, int32_t compute)
{
    if (!nn || (compute != MREP_NN_COMPUTE_BF16 && compute != MREP_NN_COMPUTE_FP32)) {
        set_error("mrep_nn_set_compute: null network or unknown compute mode");
        return MREP_E_INVALID_ARG;
    }
    nn->compute = compute;
    return MREP_OK;
}

int32_t mrep_nn_infer(const mrep_nn* nn, int64_t n, const float* x, float* y, void* stream)
{
    if (!nn || n < 0 || (n > 0 && (!x || !y))) {
        set_error("mrep_nn_infer: null pointer or negative n");
        return MREP_E_INVALID_ARG;
    }
    if (n == 0) return MREP_OK;
    hipStream_t st = (hipStream_t)stream;
    int rc = pack_image(nn, st);
    if (rc) return rc;
    const unsigned nb = (unsigned)std::min<int64_t>((n + 63) / 64, 2048);
    if (nn->kind == MREP_NN_SURFACE) {
        using R = RowsFromMemory<MREP_NN_SURFACE_IN, MREP_NN_SURFACE_OUT>;
        hipLaunchKernelGGL(k_mlp<R>, dim3(nb), dim3(256), 0, st, R{n, x, y}, (const uint8_t*)nn->img());
    } else {
        using R = RowsFromMemory<MREP_NN_CURVE_IN, MREP_NN_CURVE_OUT>;
        hipLaunchKernelGGL(k_mlp<R>, dim3(nb), dim3(256), 0, st, R{n, x, y}, (const uint8_t*)nn->img());
    }
    NN_HIP(hipGetLastError());
    return MREP_OK;
}

int32_t mrep_nn_train_step(mrep_nn* nn, int64_t n_rows, const float* x, const float* target, const float* accept,
                           int64_t batch, const int32_t* rows, float lr, float* loss_out, float* grad_out,
                           void* work, int64_t work_bytes, void* stream)
{
    if (!nn || batch <= 0 || !x || !target || !accept || !work || (!rows && n_rows < batch)) {
        set_error("mrep_nn_train_step: null pointer or empty batch");
        return MREP_E_INVALID_ARG;
    }
    if (batch > INT32_MAX / kH || !(lr >= 0.f)) {
        set_error("mrep_nn_train_step: batch too large or negative learning rate");
        return MREP_E_INVALID_ARG;
    }
    const NetDims& d = nn->d;
    TrainWork w;
    if (work_bytes < train_layout(d, batch, (char*)work, &w)) {
        set_error("mrep_nn_train_step: work buffer smaller than mrep_nn_bytes(kind, batch)");
        return MREP_E_SMALL_BUFFER;
    }
    hipStream_t st = (hipStream_t)stream;
    const float *X = x, *T = target, *A = accept;
    if (rows) {
        hipLaunchKernelGGL(k_gather, dim3(blocks_for(batch * (d.in + d.out))), dim3(256), 0, st, batch, rows, n_rows, d.in, d.out - 1,
                           x, target, accept, w.Xb, w.Tb, w.Ab);
        X = w.Xb; T = w.Tb; A = w.Ab;
    }
    t_gemm_fp32 = nn->compute == MREP_NN_COMPUTE_FP32;
    int rc = forward(d, nn->params(), batch, X, w, st);
    if (rc == MREP_OK) rc = backward(d, nn->params(), batch, X, T, A, w, nn->grad(), loss_out, st);
    t_gemm_fp32 = false;
    if (rc) return rc;
    if (grad_out) NN_HIP(hipMemcpyAsync(grad_out, nn->grad(), 4 * d.n, hipMemcpyDeviceToDevice, st));
    if (lr > 0.f) {
        nn->step += 1;
        const float c1 = (float)(1.0 - pow(0.9, (double)nn->step)), c2 = (float)(1.0 - pow(0.999, (double)nn->step));
        hipLaunchKernelGGL(k_adam, dim3(blocks_for(d.n)), dim3(256), 0, st, d.n, nn->params(), nn->m(), nn->v(),
                           (const float*)nn->grad(), lr, 0.9f, 0.999f, 1e-8f, c1, c2);
        NN_HIP(hipGetLastError());
    }
    return MREP_OK;
}

int32_t mrep_seeded_workspace_bytes(const mrep_geom* geom, int64_t n, const mrep_opts* opts, int64_t* bytes)
{
    if (!geom || !bytes || n < 0 || geom->kind != MREP_GEOM_CURVES) {
        set_error("mrep_seeded_workspace_bytes: null pointer, surface geometry or negative n");
        return MREP_E_INVALID_ARG;
    }
    int rc = check_opts(opts);
    if (rc) return rc;
    *bytes = seed_layout(geom->g.L.n_curves, n, nullptr, nullptr);
    return MREP_OK;
}

int32_t mrep_nn_features(const mrep_geom* geom, int64_t n, const int32_t* curve_id, const double* q_xyz,
                         int32_t* seg_out, float* x_out, void* workspace, int64_t ws_bytes, void* stream)
{
    if (!geom || n < 0 || geom->kind != MREP_GEOM_CURVES) {
        set_error("mrep_nn_features: null or surface geometry, or negative n");
        return MREP_E_INVALID_ARG;
    }
    if (n == 0) return MREP_OK;
    if (!curve_id || !q_xyz || !seg_out || !x_out || !workspace) {
        set_error("mrep_nn_features: null pointer");
        return MREP_E_INVALID_ARG;
    }
    if (n * kK >= (int64_t)INT32_MAX || geom->g.L.n_curves == 0) {
        set_error("mrep_nn_features: n * 4 must be < 2^31 and the geometry non-empty");
        return MREP_E_INVALID_ARG;
    }
    const int64_t nc = geom->g.L.n_curves;
    SeedWork w;
    if (ws_bytes < seed_layout(nc, n, (char*)workspace, &w)) {
        set_error("mrep_nn_features: workspace smaller than mrep_seeded_workspace_bytes");
        return MREP_E_SMALL_BUFFER;
    }
    if (((uintptr_t)workspace & 255) != 0) {
        set_error("mrep_nn_features: workspace not 256-byte aligned");
        return MREP_E_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill_feat, dim3(blocks_for(n * kK)), dim3(256), 0, st, n, seg_out, x_out);
    // grouping writes nothing for invalid ids when the outputs are null
    const Outs none{nullptr, nullptr, nullptr, nullptr};
    w.box.xb = nullptr;
    int rc = candidates(geom, n, curve_id, q_xyz, 2e-6f, w, none, st, true, false);
    if (rc) return rc;
    hipLaunchKernelGGL(k_feat_write, dim3(blocks_for(n, 128)), dim3(128), 0, st, dev_view(geom->g), curve_id, q_xyz,
                       (const int32_t*)w.q_off, (const int32_t*)w.perm, (const int32_t*)w.box.cand, seg_out, x_out);
    NN_HIP(hipGetLastError());
    return MREP_OK;
}

int32_t mrep_project_curves_seeded(const mrep_geom* geom, const mrep_nn* nn, const mrep_opts* opts, int64_t n,
                                   const int32_t* curve_id, const double* q_xyz, void* workspace, int64_t ws_bytes,
                                   double* t_out, double* dist_out, int32_t* seg_out, uint32_t* flags_out, void* stream)
{
    return seeded_core("mrep_project_curves_seeded", geom, nn, opts, n, curve_id, q_xyz, workspace, ws_bytes, t_out,
                       dist_out, seg_out, flags_out, stream, 0);
}

}  // extern "C"

int64_t mrep::seeded_ws_bytes(const mrep_geom* geom, int64_t n)
{
    return seed_layout(geom->g.L.n_curves, n, nullptr, nullptr);
}

int mrep::seeded_core(const char* fn_, const mrep_geom* geom, const mrep_nn* nn, const mrep_opts* opts, int64_t n,
                      const int32_t* curve_id, const double* q_xyz, void* workspace, int64_t ws_bytes,
                      double* t_out, double* dist_out, int32_t* seg_out, uint32_t* flags_out, void* stream,
                      int invert)
{
    const std::string fn(fn_);
    if (!geom || n < 0 || geom->kind != MREP_GEOM_CURVES) {
        set_error(fn + ": null or surface geometry, or negative n");
        return MREP_E_INVALID_ARG;
    }
    if (nn && nn->kind != MREP_NN_CURVE) {
        set_error(fn + ": the network is not of kind MREP_NN_CURVE");
        return MREP_E_INVALID_ARG;
    }
    int rc = check_opts(opts);
    if (rc) return rc;
    if (opts->precision != MREP_PREC_BF16) {
        set_error(fn + ": the seeded path runs in the BF16 mode (FP32 refine)");
        return MREP_E_INVALID_ARG;
    }
    if (n == 0) return MREP_OK;
    if (n * (int64_t)std::max(opts->max_candidates, kK) >= (int64_t)INT32_MAX) {
        set_error(fn + ": n * max(max_candidates, 4) must be < 2^31");
        return MREP_E_INVALID_ARG;
    }
    if (!curve_id || !q_xyz || !workspace || !t_out || !dist_out || !seg_out || !flags_out) {
        set_error(fn + ": null pointer");
        return MREP_E_INVALID_ARG;
    }
    const int64_t nc = geom->g.L.n_curves;
    if (nc == 0) {
        set_error(fn + ": geometry has no curves");
        return MREP_E_INVALID_ARG;
    }
    SeedWork w;
    if (ws_bytes < seed_layout(nc, n, (char*)workspace, &w)) {
        set_error(fn + ": workspace smaller than mrep_seeded_workspace_bytes");
        return MREP_E_SMALL_BUFFER;
    }
    if (((uintptr_t)workspace & 255) != 0) {
        set_error(fn + ": workspace not 256-byte aligned");
        return MREP_E_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    const bool timed = (opts->flags & MREP_OPT_TIME_STAGES) != 0;
    if (timed && (rc = stage_begin(st))) return rc;
    const Outs o{t_out, dist_out, seg_out, flags_out};
    const DevGeom G = dev_view(geom->g);
    const float tie = (float)opts->tie_rel;
    if (!nn) w.box.xb = nullptr;
    rc = candidates(geom, n, curve_id, q_xyz, tie, w, o, st, nn != nullptr, timed);
    if (rc) return rc;
    if (timed && (rc = stage_mark(2, st))) return rc;
    if (nn) {
        rc = pack_image(nn, st);
        if (rc) return rc;
        const RowsFromCandidates rows{w.q_off, (int32_t)nc, w.box.cand, w.box.xb, w.scores};
        const unsigned nb = (unsigned)std::min<int64_t>((n * kK + 63) / 64, 2048);
        hipLaunchKernelGGL(k_mlp<RowsFromCandidates>, dim3(nb), dim3(256), 0, st, rows, (const uint8_t*)nn->img());
        NN_HIP(hipGetLastError());
    }
    if (timed && (rc = stage_mark(3, st))) return rc;
    if (nn) {
        if (G.general)
            hipLaunchKernelGGL((k_decide<true>), dim3(blocks_for(n, 128)), dim3(128), 0, st, G, curve_id, q_xyz,
                               (const int32_t*)w.q_off, (const int32_t*)w.perm, w.box, (const float2*)w.scores, tie,
                               (int32_t)invert, w.done, o);
        else
            hipLaunchKernelGGL((k_decide<false>), dim3(blocks_for(n, 128)), dim3(128), 0, st, G, curve_id, q_xyz,
                               (const int32_t*)w.q_off, (const int32_t*)w.perm, w.box, (const float2*)w.scores, tie,
                               (int32_t)invert, w.done, o);
        NN_HIP(hipGetLastError());
    }
    if (timed && (rc = stage_mark(4, st))) return rc;
    NN_HIP(launch_refine(G, n, curve_id, q_xyz, w.q_off, w.perm, w.box.so, w.pair_res, nn ? w.done : nullptr,
                         nn ? (uint32_t)MREP_F_NN_FALLBACK : 0u, opts->tie_rel, invert, w.ovf_list, w.ovf_count, o, st,
                         (opts->flags & MREP_OPT_CLIP) != 0, timed ? 5 : -1));
    if (timed) {
        if ((rc = stage_mark(6, st))) return rc;
        stage_end(6);
    }
    return MREP_OK;
}
