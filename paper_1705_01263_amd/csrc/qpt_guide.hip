// The learned proposal on gfx950: a 32-64-64-64-40 ReLU network in BF16 on
// MFMA with FP32 accumulation, mapping an encoded hit position and outgoing
// direction to an 8-lobe von Mises-Fisher mixture; trained online from the
// renderer's own radiance samples with Adam on FP32 master weights. The
// operand layout of the MFMA tiles and the inference path are in
// qpt_guide_mlp.h; this file holds training, the fragment builder and the
// standalone inference kernel.
#include <hip/hip_runtime.h>

#include "qpt_guide_dev.h"
#include "qpt_guide_mlp.h"
#include "qpt_internal.h"
#include "qpt_state_dev.h"

namespace qpt {
namespace {

using namespace mlp;

constexpr int kGB[4] = {0, 0, 16, 32};         // first transposed fragment (layers 1..3)
constexpr int kOffW[4] = {0, 2112, 6272, 10432};
constexpr int kOffB[4] = {2048, 6208, 10368, 12992};
constexpr int kTrainBlock = 512;               // 8 waves: two row halves of the four gradient-tile owners
static_assert(kTrainBlock == 512, "the per-block weight and loss sums add eight waves");

// ReLU, its mask (bit 16t + v), and the BF16 B operands of the next layer
__device__ __forceinline__ void relu_pack(const v16f *acc, v4s *out, uint32_t &mask)
{
    mask = 0;
    float a[32];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            float z = acc[t][v];
            bool p = z > 0.0f;
            mask |= (uint32_t)p << (16 * t + v);
            a[16 * t + v] = p ? z : 0.0f;
        }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        int b = 16 * (s / 4) + 4 * (s % 4);
        out[s] = pack4(a[b], a[b + 1], a[b + 2], a[b + 3]);
    }
}

// B operands of layer 0 from a row's 32 features (each lane takes its half)
__device__ __forceinline__ void input_frags(const float *f, v4s *a0)
{
    const bool hi = lane_id() >= 32;
#pragma unroll
    for (int s = 0; s < 4; ++s)
        a0[s] = hi ? pack4(f[8 * s + 4], f[8 * s + 5], f[8 * s + 6], f[8 * s + 7])
                   : pack4(f[8 * s], f[8 * s + 1], f[8 * s + 2], f[8 * s + 3]);
}

struct Act {
    v4s a1[8], a2[8], a3[8];
    uint32_t m0, m1, m2;
};

__device__ __forceinline__ void mlp_forward(const uint2 *sfrag, const float *sbias, const v4s *a0, Act &A, v16f *out)
{
    v16f acc[2];
    layer_fwd<0>(sfrag, sbias, a0, acc);
    relu_pack(acc, A.a1, A.m0);
    layer_fwd<1>(sfrag, sbias, A.a1, acc);
    relu_pack(acc, A.a2, A.m1);
    layer_fwd<2>(sfrag, sbias, A.a2, acc);
    relu_pack(acc, A.a3, A.m2);
    layer_fwd<3>(sfrag, sbias, A.a3, out);
}

// all 40 outputs of the lane's row: half from itself, half from lane ^ 32
__device__ __forceinline__ void gather40(const v16f *acc, float *o)
{
    const bool hi = lane_id() >= 32;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        float mine = acc[0][v];
        float other = guide::xor32(mine);
        int f = 8 * (v / 4) + (v % 4);
        o[f] = hi ? other : mine;       // features with 4(l/32) = 0
        o[f + 4] = hi ? mine : other;   // features with 4(l/32) = 4
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        float mine = acc[1][v];
        float other = guide::xor32(mine);
        o[32 + v] = hi ? other : mine;
        o[36 + v] = hi ? mine : other;
    }
}

// Gradient of -w log q(w_dir) w.r.t. the 40 outputs, through the decode,
// with lobe responsibilities g_k = pi_k f_k / q (stable in log space):
//   logit: -w (g_k - pi_k); mu_raw: -w g_k kappa (w - (mu.w) mu) / |mu_raw|;
//   kappa_raw: -w g_k (1/kappa - 2/expm1(2 kappa) + mu.w - 1) sigmoid(kappa_raw)
// (zero where kappa is clamped), and -w log q in `loss`. The outputs are in
// the fragments' order (frag_out_row): lane half h holds the five parameters
// of lobes 4h + j in out[0][j], out[0][4 + j], out[0][8 + j], out[0][12 + j]
// and out[1][j], computes their gradient in the same registers of dz (the
// padding rows get 0), and exchanges only the softmax's and the mixture's
// normalisers with its partner lane. With e = expm1(-2 kappa), the vMF
// normaliser kappa / (2 pi (1 - exp(-2 kappa))) is kappa / (2 pi (-e)) and
// 2 / expm1(2 kappa) = -2 (1 + e) / e: one expm1 per lobe, accurate for the
// smallest kappa (1e-3), where the two terms of the kappa gradient cancel.
__device__ __forceinline__ void pair_loss_grad(const v16f *out, guide::V3 wd, float w, v16f *dz, float &loss)
{
    float mx = fmaxf(fmaxf(out[0][0], out[0][1]), fmaxf(out[0][2], out[0][3]));
    mx = fmaxf(mx, guide::xor32(mx));
    float se = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) se += __expf(out[0][j] - mx);
    se += guide::xor32(se);
    const float lse = __logf(se);
    float lp[4], kap[4], inv_mn[4], cw[4], mu[4][3], em[4], lf[4];
    bool clamped[4];
    float lmax = -INFINITY;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        lp[j] = out[0][j] - mx - lse;
        const float x = out[0][4 + j], y = out[0][8 + j], z = out[0][12 + j];
        inv_mn[j] = 1.0f / fmaxf(sqrtf(x * x + y * y + z * z), 1e-12f);
        mu[j][0] = x * inv_mn[j];
        mu[j][1] = y * inv_mn[j];
        mu[j][2] = z * inv_mn[j];
        const float kk = guide::softplus(out[1][j]) + 1e-3f;
        clamped[j] = kk >= 1e4f;
        kap[j] = fminf(kk, 1e4f);
        cw[j] = mu[j][0] * wd.x + mu[j][1] * wd.y + mu[j][2] * wd.z;
        em[j] = expm1f(-2.0f * kap[j]);
        lf[j] = lp[j] + __logf(kap[j] / (2.0f * guide::kPiF * -em[j])) + kap[j] * (cw[j] - 1.0f);
        lmax = fmaxf(lmax, lf[j]);
    }
    lmax = fmaxf(lmax, guide::xor32(lmax));
    float g[4], sg = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        g[j] = __expf(lf[j] - lmax);
        sg += g[j];
    }
    sg += guide::xor32(sg);
    loss = -w * (lmax + __logf(sg));
    const float inv = 1.0f / sg;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float gk = g[j] * inv;
        dz[0][j] = -w * (gk - __expf(lp[j]));
        const float c = -w * gk * kap[j] * inv_mn[j];
        dz[0][4 + j] = c * (wd.x - cw[j] * mu[j][0]);
        dz[0][8 + j] = c * (wd.y - cw[j] * mu[j][1]);
        dz[0][12 + j] = c * (wd.z - cw[j] * mu[j][2]);
        const float dk = 1.0f / kap[j] + 2.0f * (1.0f + em[j]) / em[j] + cw[j] - 1.0f;
        const float sgm = 1.0f / (1.0f + __expf(-out[1][j]));
        dz[1][j] = clamped[j] ? 0.0f : -w * gk * dk * sgm;
    }
#pragma unroll
    for (int v = 4; v < 16; ++v) dz[1][v] = 0.0f;
}

// Training backward, block-cooperative. A block of eight waves takes 256
// rows (32 per wave) per iteration, two waves per SIMD to hide the MFMA and
// LDS latencies of each other. For each layer, every wave stages its rows'
// BF16 pre-activation gradients dZ and layer inputs A in LDS, transposed
// ([feature][row], 256 rows plus padding per feature), then waves w and
// w + 4 multiply the same 32 x 32 tile of dW^T = dZ^T A, over rows 0-127 and
// 128-255 respectively (the rows are the MFMA reduction dimension), into
// accumulators they keep across iterations, and waves L and 4 + L sum the
// two halves' rows of dZ for layer L's bias gradient (a product with a
// column of ones on 16 x 16 x 32 MFMA). Nothing is added atomically: the
// halves are combined in a fixed order and each gradient value is written
// once per block at the end.
constexpr int kRowsPerIter = 256;
constexpr int kRowsPerOwner = 128;  // rows of an iteration in one wave's gradient tiles
constexpr int kStageRow = 260;   // BF16 per staged feature: 256 rows + 4 (bank-conflict-free b64 reads)

typedef float v4f __attribute__((ext_vector_type(4)));

// 16 x 16 x 32: the same pairing of two 4-element fragments per operand
__device__ __forceinline__ v4f mfma16x2(v4s a0, v4s a1, v4s b0, v4s b1, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(cat8(a0, a1), cat8(b0, b1), c, 0, 0, 0);
}

__device__ __forceinline__ v4s lds_b64(const uint16_t *p) { return __builtin_bit_cast(v4s, *(const uint2 *)p); }

struct GradAcc {
    v16f w[4];  // this wave's dW^T tile of each layer over its row half (layer 0: owners 0 and 1 only)
    v4f b[4];   // bias gradient of layer `wave & 3` over its row half, four 16-output tiles
};

// the dW^T tile of layer L owned by wave wv (both row halves): owner
// u = wv & 3, output tile to = u & 1, input tile tk = u >> 1 (layer 0 has
// one input tile: owners 2 and 3 have none)
template <int L>
__device__ __forceinline__ bool owns_tile(uint32_t wv, int &to, int &tk)
{
    const uint32_t u = wv & 3u;
    to = (int)(u & 1u);
    tk = (int)(u >> 1);
    return tk < kKS[L] / 4;
}

template <int L>
__device__ __forceinline__ void layer_bwd(const v16f *dz, const v4s *in, const uint2 *sfragT, uint32_t mask_prev,
                                          uint16_t *sZ, uint16_t *sA, uint32_t wv, GradAcc &acc, v16f *dz_prev)
{
    const uint32_t lane = lane_id(), half = lane >> 5, row = lane & 31;
    const uint32_t R = wv * 32 + row;  // the lane's row within the block's 128
    constexpr int KS = kKS[L], N = kN[L];
    // BF16 operands: zf[s] = dZ[row][8s + 4 half + e] (the data-gradient B operand)
    v4s zf[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        int t = s / 4, b = 4 * (s % 4);
        zf[s] = pack4(dz[t][b], dz[t][b + 1], dz[t][b + 2], dz[t][b + 3]);
    }
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int e = 0; e < 4; ++e) sZ[(8 * s + 4 * half + e) * kStageRow + R] = (uint16_t)zf[s][e];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int e = 0; e < 4; ++e) sA[(8 * s + 4 * half + e) * kStageRow + R] = (uint16_t)in[s][e];
    __syncthreads();
    int to, tk;
    const uint32_t r0 = kRowsPerOwner * (wv >> 2);  // this wave's row half
    if (owns_tile<L>(wv, to, tk) && !(to == 1 && N <= 32)) {
        const uint16_t *za = sZ + (32 * to + row) * kStageRow + r0 + 4 * half;
        const uint16_t *aa = sA + (32 * tk + row) * kStageRow + r0 + 4 * half;
        v16f c = acc.w[L];
#pragma unroll
        for (int s = 0; s < kRowsPerOwner / 8; s += 2)
            c = mfma2(lds_b64(za + 8 * s), lds_b64(za + 8 * s + 8), lds_b64(aa + 8 * s), lds_b64(aa + 8 * s + 8), c);
        acc.w[L] = c;
    }
    if ((wv & 3u) == (uint32_t)L) {
        const v4s ones = {(short)0x3F80, (short)0x3F80, (short)0x3F80, (short)0x3F80};
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            if (16 * ot >= N) continue;
            const uint16_t *za = sZ + (16 * ot + (lane & 15)) * kStageRow + r0 + 4 * (lane >> 4);
            v4f c = acc.b[ot];
#pragma unroll
            for (int s = 0; s < kRowsPerOwner / 16; s += 2) c = mfma16x2(lds_b64(za + 16 * s), lds_b64(za + 16 * s + 16), ones, ones, c);
            acc.b[ot] = c;
        }
    }
    __syncthreads();
    if constexpr (L > 0) {
        // dA^T[k][row] = sum_o W[k][o] dZ^T[o][row], then the ReLU mask of layer L-1
#pragma unroll
        for (int tkk = 0; tkk < 2; ++tkk) {
            v16f c = {};
#pragma unroll
            for (int s = 0; s < 8; s += 2) {
                const uint2 *f = sfragT + (kGB[L] + tkk * 8 + s) * 64 + lane;
                c = mfma2(as_v4s(f[0]), as_v4s(f[64]), zf[s], zf[s + 1], c);
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) c[v] = ((mask_prev >> (16 * tkk + v)) & 1u) ? c[v] : 0.0f;
            dz_prev[tkk] = c;
        }
    }
}

// ------------------------------------------------------------- kernels

// BF16 fragments and biases from the FP32 master parameters
// the BF16 operand tiles of the FP32 master weights, for training (T.frag,
// T.fragT, T.bias) and, where given, for the renderer's published copies
__global__ void k_guide_frag(GuideTrain T, uint2 *pub_a, float *pub_ab, uint2 *pub_b, float *pub_bb)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nf = kGuideFrags * 64, nt = kGuideFragsT * 64;
    auto w_at = [&](int L, int k, int o) -> float { return o < kN[L] ? T.master[kOffW[L] + k * kN[L] + o] : 0.0f; };
    auto pack2 = [](float a, float b) { return bf16_rne(a) | (bf16_rne(b) << 16); };
    if (i < nf) {
        uint32_t f = i / 64, lane = i % 64, half = lane / 32;
        int L = f < 8 ? 0 : (f < 24 ? 1 : (f < 40 ? 2 : 3));
        int r = f - kFB[L], t = r / kKS[L], s = r % kKS[L];
        int k = 8 * s + 4 * half, o = 32 * t + lane % 32;
        auto frag = [&](int oo) {
            return make_uint2(pack2(w_at(L, k, oo), w_at(L, k + 1, oo)), pack2(w_at(L, k + 2, oo), w_at(L, k + 3, oo)));
        };
        const uint2 v = frag(L == 3 ? frag_out_row(o) : o);
        T.frag[i] = v;
        if (pub_a) pub_a[i] = v;
        if (pub_b) pub_b[i] = v;
    } else if (i < nf + nt) {
        uint32_t j = i - nf, g = j / 64, lane = j % 64, half = lane / 32;
        int L = 1 + g / 16;
        int r = g % 16, tk = r / 8, s = r % 8;
        int k = 32 * tk + lane % 32, o = 8 * s + 4 * half;
        auto w_row = [&](int r) { return w_at(L, k, L == 3 ? frag_out_row(r) : r); };
        T.fragT[j] = make_uint2(pack2(w_row(o), w_row(o + 1)), pack2(w_row(o + 2), w_row(o + 3)));
    } else if (i < nf + nt + 256) {
        uint32_t j = i - nf - nt;
        int L = j / 64, o = j % 64;
        auto bias = [&](int oo) { return __uint_as_float(bf16_rne(oo < kN[L] ? T.master[kOffB[L] + oo] : 0.0f) << 16); };
        const float bq = bias(L == 3 ? frag_out_row(o) : o);
        T.bias[j] = bq;
        if (pub_ab) pub_ab[j] = bq;
        if (pub_bb) pub_bb[j] = bq;
    }
}

// rows of the inference parity hook: n positions and outgoing directions (n x 3
// each) and n output rows of 10 uint4 (the first 5 hold the packed mixture)
struct EvalSrc {
    const float *x, *wo;
    uint32_t n;
    uint4 *out;
};

// mixture of every row: each lane of a pair encodes its half of the inputs
// and decodes four of the eight lobes
// the mixture of every row (parity hook: explicit positions and directions)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_guide_eval(Frame F, EvalSrc src)
{
    __shared__ uint2 sfrag[kGuideFrags * 64];
    __shared__ __align__(16) float sbias[256];
    const uint32_t n = src.n;
    if ((size_t)blockIdx.x * (blockDim.x / 2) >= n) return;  // uniform per block
    load_weights(F.guide.frag, F.guide.bias, sfrag, sbias);
    __syncthreads();
    const uint32_t lane = lane_id();
    const uint32_t wave = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const uint32_t waves = gridDim.x * (blockDim.x / 64);
    for (uint32_t base = wave * 32; base < n; base += waves * 32) {
        // keeps the weight reads inside the loop: hoisted, they would pin
        // ~240 registers and leave one wave per SIMD
        asm volatile("" ::: "memory");
        const uint32_t i = base + (lane & 31);
        const bool valid = i < n;
        guide::V3 x = {0.0f, 0.0f, 0.0f}, wo = {0.0f, 1.0f, 0.0f};
        if (valid) {
            x = {src.x[3 * (size_t)i], src.x[3 * (size_t)i + 1], src.x[3 * (size_t)i + 2]};
            wo = {src.wo[3 * (size_t)i], src.wo[3 * (size_t)i + 1], src.wo[3 * (size_t)i + 2]};
        }
        infer_pair(sfrag, sbias, x, wo, F.guide.bmin, F.guide.binv, valid,
                   src.out + (size_t)(valid ? i : 0) * 2 * guide::kMixU4);
    }
}

// training records -> replay samples with a positive loss weight: the
// luminance of the sample's own estimate f cos L_i / p of the scattering
// integral, so that the network learns a density proportional to the
// integrand. Samples are appended to a ring that keeps the newest ring_cap;
// a weight estimated under an older proposal is still an estimate of the
// same integrand, so older samples remain valid training data.
__global__ void k_rec_finalize(Frame F, Pool P, GuideTrain T)
{
    uint32_t cnt = min(*F.guide.rec_count, F.guide.rec_cap);
    for (uint32_t base = blockIdx.x * blockDim.x; base < cnt; base += gridDim.x * blockDim.x) {
        uint32_t i = base + threadIdx.x;
        bool ok = false;
        if (i < cnt) {
            float4 *r = F.guide.rec + (size_t)i * kRecF4;
            const float w = guide::record_weight(r[3], r[4], r[5], P.rad[__float_as_uint(r[2].w)]);
            ok = w > 0.0f && w < INFINITY;
            if (ok) {
                r[1].w = w;
            }
        }
        unsigned long long mask = __ballot(ok);
        uint32_t b = 0;
        if (mask) {
            uint32_t leader = __ffsll((long long)mask) - 1;
            if (lane_id() == leader) b = atomicAdd(T.ring_head, (uint32_t)__popcll(mask));
            b = __shfl(b, (int)leader);
        }
        uint32_t off = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        if (ok) {
            const float4 *r = F.guide.rec + (size_t)i * kRecF4;
            float4 *q = T.ring + (size_t)((b + off) & (T.ring_cap - 1u)) * kRingF4;
            float4 r0 = r[0], r1 = r[1], r2 = r[2];
            q[0] = make_float4(r0.x, r0.y, r0.z, r1.w);
            q[1] = make_float4(r1.x, r1.y, r1.z, 0.0f);
            q[2] = make_float4(r2.x, r2.y, r2.z, 0.0f);
        }
    }
}

struct RowSrc {
    // records (debug == false) or explicit arrays (debug == true)
    bool debug;
    const float *x, *dirs, *w;  // debug: n x 32 features, n x 3, n
    uint32_t n;                  // debug: rows; replay: the batch size
    const uint32_t *count;       // replay: samples ever appended to the ring (device)
    float u;                     // stratification offset in [0, 1)
};

__global__ __launch_bounds__(kTrainBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_guide_train(Frame F, GuideTrain T, RowSrc src)
{
    extern __shared__ unsigned char smem[];
    uint2 *sfrag = (uint2 *)smem;
    uint2 *sfragT = sfrag + kGuideFrags * 64;
    float *sbias = (float *)(sfragT + kGuideFragsT * 64);
    uint16_t *sZ = (uint16_t *)(sbias + 256);
    uint16_t *sA = sZ + 64 * kStageRow;
    for (uint32_t i = threadIdx.x; i < kGuideFrags * 64; i += blockDim.x) sfrag[i] = T.frag[i];
    for (uint32_t i = threadIdx.x; i < kGuideFragsT * 64; i += blockDim.x) sfragT[i] = T.fragT[i];
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) sbias[i] = T.bias[i];
    __syncthreads();
    const uint32_t lane = lane_id(), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);  // uniform per wave
    // replay: a batch of min(batch, samples held) rows, a stratified subset
    const uint32_t count = src.debug ? src.n : min(*src.count, T.ring_cap);
    const uint32_t nrows = min(src.n, count);
    const uint32_t iters = (nrows + kRowsPerIter - 1) / kRowsPerIter;
    GradAcc acc;
#pragma unroll
    for (int L = 0; L < 4; ++L) {
        acc.w[L] = (v16f){};
        acc.b[L] = (v4f){};
    }
    float wsum = 0.0f, lsum = 0.0f;
    // every wave of a block runs the same iterations (block-wide barriers inside)
    for (uint32_t it = blockIdx.x; it < iters; it += gridDim.x) {
        asm volatile("" ::: "memory");  // weight reads stay in the loop
        uint32_t row = it * kRowsPerIter + wv * 32 + (lane & 31);
        bool valid = row < nrows;
        float f[32];
        guide::V3 wd = {0.0f, 0.0f, 1.0f}, xs = {0.0f, 0.0f, 0.0f}, wos = {0.0f, 1.0f, 0.0f};
        float wt = 0.0f;
        for (int j = 0; j < 32; ++j) f[j] = 0.0f;
        if (valid) {
            if (src.debug) {
                for (int j = 0; j < 32; ++j) f[j] = src.x[(size_t)row * 32 + j];
                wd = {src.dirs[3 * (size_t)row], src.dirs[3 * (size_t)row + 1], src.dirs[3 * (size_t)row + 2]};
                wt = src.w[row];
            } else {
                // stratified subset of the ring's samples
                uint32_t c = (uint32_t)(((double)row + src.u) * (double)count / (double)nrows);
                c = min(c, count - 1);
                const float4 *r = T.ring + (size_t)c * kRingF4;
                float4 r0 = r[0], r1 = r[1], r2 = r[2];
                xs = {r0.x, r0.y, r0.z};
                wos = {r1.x, r1.y, r1.z};
                wd = {r2.x, r2.y, r2.z};
                wt = r0.w;
            }
        }
        v4s a0[4];
        if (src.debug) input_frags(f, a0);
        else encode_half(xs, wos, F.guide.bmin, F.guide.binv, a0);
        Act A;
        v16f out[2];
        mlp_forward(sfrag, sbias, a0, A, out);
        v16f dz[2], dzp[2];
        float lv;
        pair_loss_grad(out, wd, wt, dz, lv);
        if (valid && lane < 32) {
            wsum += wt;
            lsum += lv;
        }
        layer_bwd<3>(dz, A.a3, sfragT, A.m2, sZ, sA, wv, acc, dzp);
        layer_bwd<2>(dzp, A.a2, sfragT, A.m1, sZ, sA, wv, acc, dz);
        layer_bwd<1>(dz, A.a1, sfragT, A.m0, sZ, sA, wv, acc, dzp);
        layer_bwd<0>(dzp, a0, sfragT, 0u, sZ, sA, wv, acc, dz);
    }
    for (int off = 32; off > 0; off >>= 1) {
        wsum += __shfl_xor(wsum, off);
        lsum += __shfl_xor(lsum, off);
    }
    // the block's weight and loss sums, in wave order (no atomics: the step
    // is a deterministic function of its rows)
    __shared__ float swl[2][kTrainBlock / 64];
    if (lane == 0) {
        swl[0][wv] = wsum;
        swl[1][wv] = lsum;
    }
    // the staged weights and rows are done with: the LDS holds the upper row
    // halves' partial gradients from here on
    __syncthreads();
    if (threadIdx.x == 0) {
        T.scalars[2 + 2 * blockIdx.x] = ((swl[0][0] + swl[0][1]) + (swl[0][2] + swl[0][3])) +
                                        ((swl[0][4] + swl[0][5]) + (swl[0][6] + swl[0][7]));
        T.scalars[3 + 2 * blockIdx.x] = ((swl[1][0] + swl[1][1]) + (swl[1][2] + swl[1][3])) +
                                        ((swl[1][4] + swl[1][5]) + (swl[1][6] + swl[1][7]));
    }
    // this block's gradient sums: the lower half's partial plus the upper
    // half's, every parameter written by exactly one lane
    float *comb = (float *)smem;  // 4 owners x 64 lanes x 16 floats
    float *mine = comb + ((wv & 3u) * 64 + lane) * 16;
    const bool upper = wv >= 4;
    float *out_p = T.partial + (size_t)blockIdx.x * kGuideParams;
    const uint32_t half = lane >> 5;
#pragma unroll
    for (int L = 0; L < 4; ++L) {
        int to, tk;
        bool own;
        switch (L) {
        case 0: own = owns_tile<0>(wv, to, tk); break;
        case 1: own = owns_tile<1>(wv, to, tk); break;
        case 2: own = owns_tile<2>(wv, to, tk); break;
        default: own = owns_tile<3>(wv, to, tk); break;
        }
        if (own && upper)
#pragma unroll
            for (int v = 0; v < 16; ++v) mine[v] = acc.w[L][v];
        __syncthreads();
        if (own && !upper) {
            const int N = kN[L];
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                int o = 32 * to + 8 * (v / 4) + 4 * (int)half + (v % 4);  // accumulator row
                int k = 32 * tk + (int)(lane & 31);
                if (o < N) out_p[kOffW[L] + k * N + (L == 3 ? frag_out_row(o) : o)] = acc.w[L][v] + mine[v];
            }
        }
        __syncthreads();
    }
    if (upper)
#pragma unroll
        for (int ot = 0; ot < 4; ++ot)
#pragma unroll
            for (int v = 0; v < 4; ++v) mine[4 * ot + v] = acc.b[ot][v];
    __syncthreads();
    if (!upper && (lane & 15) == 0) {
        const int N = kN[wv];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int o = 16 * ot + 4 * (int)(lane >> 4) + v;  // accumulator row
                if (o < N) out_p[kOffB[wv] + (wv == 3 ? frag_out_row(o) : o)] = acc.b[ot][v] + mine[4 * ot + v];
            }
    }
}

constexpr uint32_t kReduceParams = 64;
// Where master parameter p sits in the BF16 copies (the inverse of the
// fragment builder's map): the 16-bit element of the forward fragments, of
// the transposed ones (layers 1-3; -1 otherwise) and of the bias table.
struct FragSlot {
    int fwd, tr, bias;
};

__device__ __forceinline__ FragSlot frag_slot(uint32_t p)
{
    FragSlot r{-1, -1, -1};
#pragma unroll
    for (int L = 0; L < 4; ++L) {
        const int N = kN[L];
        const int q = (int)p - kOffW[L];
        if (q < 0) break;
        if (q < kOffB[L] - kOffW[L]) {  // weight W_L[k][o]
            const int k = q / N, o = q % N;
            const int row = L == 3 ? frag_in_row(o) : o;  // accumulator row of output o
            const int f = kFB[L] + (row / 32) * kKS[L] + k / 8;
            r.fwd = (f * 64 + 32 * ((k % 8) / 4) + row % 32) * 4 + k % 4;
            if (L > 0) {
                const int g = kGB[L] + (k / 32) * 8 + row / 8;
                r.tr = (g * 64 + 32 * ((row % 8) / 4) + k % 32) * 4 + row % 4;
            }
            return r;
        }
        if (q < kOffB[L] - kOffW[L] + N) {  // bias b_L[o]
            const int o = q - (kOffB[L] - kOffW[L]);
            r.bias = L * 64 + (L == 3 ? frag_in_row(o) : o);
            return r;
        }
    }
    return r;
}

// sum the block partials, normalise by the weight sum; then Adam or a plain
// copy. With Adam, the updated parameter also goes straight into the BF16
// copies training reads (and, where given, the renderer's published copies):
// no separate pass over the parameters per step. A block owns 64
// parameters; its four waves each sum every fourth partial (coalesced
// 256-byte rows), then wave 0 combines the four sums.
__global__ __launch_bounds__(256) void k_guide_reduce(GuideTrain T, uint32_t blocks, int adam, uint32_t step,
                                                      float lr, float *grad_out, uint2 *pub_a, float *pub_ab,
                                                      uint2 *pub_b, float *pub_bb)
{
    __shared__ float part[4][kReduceParams];
    const uint32_t lane = threadIdx.x & 63u, grp = threadIdx.x >> 6;
    const uint32_t p = blockIdx.x * kReduceParams + lane;
    // the weight and loss sums over the training blocks: each thread loads
    // those of the blocks t, t + 256, ... (every load at once), then a fixed
    // pairwise tree in LDS (every block forms the same sums)
    __shared__ float swl[2][256];
    {
        float w = 0.0f, l = 0.0f;
        for (uint32_t b = threadIdx.x; b < blocks; b += 256) {
            w += T.scalars[2 + 2 * b];
            l += T.scalars[3 + 2 * b];
        }
        swl[0][threadIdx.x] = w;
        swl[1][threadIdx.x] = l;
    }
    // every fourth partial from grp on, into four running sums (partial
    // grp + 4 i goes to sum i mod 4), thirty-two loads in flight per lane
    // (the partials come from L2 or HBM: a chain of dependent loads would pay
    // their latency once per partial); a fixed order, so the step stays a
    // deterministic function of its rows
    float g4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (p < kGuideParams) {
        uint32_t b = grp;
        for (; b + 124 < blocks; b += 128) {
            float t[32];
#pragma unroll
            for (int j = 0; j < 32; ++j) t[j] = T.partial[(size_t)(b + 4 * j) * kGuideParams + p];
#pragma unroll
            for (int j = 0; j < 32; ++j) g4[j & 3] += t[j];
        }
        for (int j = 0; b < blocks; b += 4, ++j) g4[j & 3] += T.partial[(size_t)b * kGuideParams + p];
    }
    float g = (g4[0] + g4[1]) + (g4[2] + g4[3]);
    part[grp][lane] = g;
    for (uint32_t h = 128; h > 0; h >>= 1) {
        __syncthreads();
        if (threadIdx.x < h) {
            swl[0][threadIdx.x] += swl[0][threadIdx.x + h];
            swl[1][threadIdx.x] += swl[1][threadIdx.x + h];
        }
    }
    __syncthreads();
    if (grp != 0 || p >= kGuideParams) return;
    g = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    const float ws = swl[0][0], ls = swl[1][0];
    if (blockIdx.x == 0 && lane == 0) {
        T.scalars[0] = ws;
        T.scalars[1] = ls;
    }
    g = ws > 0.0f ? g / ws : 0.0f;
    if (grad_out) grad_out[p] = g;
    if (!adam || !(ws > 0.0f)) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float m = b1 * T.m[p] + (1.0f - b1) * g;
    float v = b2 * T.v[p] + (1.0f - b2) * g * g;
    T.m[p] = m;
    T.v[p] = v;
    float mh = m / (1.0f - powf(b1, (float)step));
    float vh = v / (1.0f - powf(b2, (float)step));
    const float w = T.master[p] - lr * mh / (sqrtf(vh) + eps);
    T.master[p] = w;
    const FragSlot fs = frag_slot(p);
    const uint16_t h = (uint16_t)bf16_rne(w);
    if (fs.fwd >= 0) {
        ((uint16_t *)T.frag)[fs.fwd] = h;
        if (pub_a) ((uint16_t *)pub_a)[fs.fwd] = h;
        if (pub_b) ((uint16_t *)pub_b)[fs.fwd] = h;
    }
    if (fs.tr >= 0) ((uint16_t *)T.fragT)[fs.tr] = h;
    if (fs.bias >= 0) {
        const float bq = __uint_as_float((uint32_t)h << 16);
        T.bias[fs.bias] = bq;
        if (pub_ab) pub_ab[fs.bias] = bq;
        if (pub_bb) pub_bb[fs.bias] = bq;
    }
}

__global__ void k_fill_u32_1(uint32_t *p) { *p = 0u; }

// forward on given features (parity hook; outputs in the network's order)
__global__ __launch_bounds__(256) void k_guide_fwd_debug(Frame F, const float *x, uint32_t n, float *out)
{
    __shared__ uint2 sfrag[kGuideFrags * 64];
    __shared__ __align__(16) float sbias[256];
    load_weights(F.guide.frag, F.guide.bias, sfrag, sbias);
    __syncthreads();
    const uint32_t lane = lane_id();
    const uint32_t wave = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const uint32_t waves = gridDim.x * (blockDim.x / 64);
    for (uint32_t base = wave * 32; base < n; base += waves * 32) {
        uint32_t row = base + (lane & 31);
        float f[32];
        for (int j = 0; j < 32; ++j) f[j] = row < n ? x[(size_t)row * 32 + j] : 0.0f;
        v4s a0[4];
        input_frags(f, a0);
        Act A;
        v16f o2[2];
        mlp_forward(sfrag, sbias, a0, A, o2);
        float o[40];
        gather40(o2, o);  // accumulator rows: row r holds network output frag_out_row(r)
        if (row < n)
            for (int r = 20 * (lane >> 5); r < 20 * (lane >> 5) + 20; ++r) out[(size_t)row * 40 + frag_out_row(r)] = o[r];
    }
}

// decode, pdf at given directions and samples from given numbers (parity hook)
__global__ void k_guide_mix_debug(const float *out40, const float *dirs, const float *u, uint32_t n, float *pdf,
                                  float *sample)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    guide::Mix m;
    guide::decode(out40 + (size_t)i * 40, m);
    guide::V3 w = {dirs[3 * (size_t)i], dirs[3 * (size_t)i + 1], dirs[3 * (size_t)i + 2]};
    pdf[i] = guide::mixture_pdf(m, w);
    guide::V3 s = guide::mixture_sample(m, u[3 * (size_t)i], u[3 * (size_t)i + 1], u[3 * (size_t)i + 2]);
    sample[3 * (size_t)i] = s.x;
    sample[3 * (size_t)i + 1] = s.y;
    sample[3 * (size_t)i + 2] = s.z;
}

size_t train_smem()
{
    return kGuideFrags * 64 * 8 + kGuideFragsT * 64 * 8 + 256 * 4 + 2 * 64 * kStageRow * 2;
}

inline uint32_t nblocks(size_t n, uint32_t bs, uint32_t cap)
{
    size_t b = (n + bs - 1) / bs;
    return (uint32_t)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

hipError_t launch_guide_frag(const GuideTrain &T, hipStream_t s, uint2 *pub_a, float *pub_ab, uint2 *pub_b,
                             float *pub_bb)
{
    uint32_t n = (kGuideFrags + kGuideFragsT) * 64 + 256;
    hipLaunchKernelGGL(k_guide_frag, dim3(nblocks(n, 256, 1u << 20)), dim3(256), 0, s, T, pub_a, pub_ab, pub_b,
                       pub_bb);
    return hipGetLastError();
}

// packed mixtures (first 80 bytes of each 160-byte row) -> the decoded FP32
// values the renderer uses, in place: 8 x (mu.xyz, kappa), then 8 weights
__global__ void k_mix_unpack_debug(uint4 *rows, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint4 *row = rows + (size_t)i * 2 * guide::kMixU4;
    uint4 packed[guide::kMixU4];
    for (int j = 0; j < guide::kMixU4; ++j) packed[j] = row[j];
    guide::Mix m;
    guide::unpack_mix(packed, m);
    float4 *out = (float4 *)row;
    for (int k = 0; k < guide::kLobes; ++k) out[k] = m.lobe[k];
    out[8] = m.w0;
    out[9] = m.w1;
}

hipError_t launch_guide_debug_eval(const Frame &f, const Pool &pool, const float *x, const float *wo, uint32_t n,
                                   float *mix, hipStream_t s)
{
    EvalSrc src{x, wo, n, (uint4 *)mix};
    hipLaunchKernelGGL(k_guide_eval, dim3(nblocks(((size_t)n + 31) / 32, 4, 2048)), dim3(256), 0, s, f, src);
    hipLaunchKernelGGL(k_mix_unpack_debug, dim3(nblocks(n, 256, 1u << 20)), dim3(256), 0, s, (uint4 *)mix, n);
    return hipGetLastError();
}

static hipError_t run_train(const Frame &f, const GuideTrain &T, const RowSrc &src, hipStream_t s, uint32_t *blocks_out)
{
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_guide_train, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)train_smem());
        if (e != hipSuccess) return e;
        attr = true;
    }
    uint32_t blocks = nblocks(((size_t)src.n + 31) / 32, kTrainBlock / 64, T.max_blocks);
    hipLaunchKernelGGL(k_guide_train, dim3(blocks), dim3(kTrainBlock), train_smem(), s, f, T, src);
    *blocks_out = blocks;
    return hipGetLastError();
}

hipError_t launch_guide_finalize(const Frame &f, const Pool &pool, const GuideTrain &T, hipStream_t s)
{
    hipLaunchKernelGGL(k_rec_finalize, dim3(nblocks(f.guide.rec_cap, 256, 4096)), dim3(256), 0, s, f, pool, T);
    return hipGetLastError();
}

hipError_t launch_guide_ring_clear(const GuideTrain &T, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u32_1, dim3(1), dim3(1), 0, s, T.ring_head);
    return hipGetLastError();
}

hipError_t launch_guide_train_steps(const Frame &f, const GuideTrain &T, uint32_t batch, uint32_t step0,
                                    uint32_t nsteps, float lr, uint32_t seed, hipStream_t s, uint2 *pub_frag,
                                    float *pub_bias)
{
    hipError_t e = hipSuccess;
    for (uint32_t k = 0; k < nsteps && e == hipSuccess; ++k) {
        const uint32_t step = step0 + k;
        // stratification offset from the step and seed (splitmix64 finaliser):
        // each step of one batch sees a different subset of its records
        uint64_t z = ((uint64_t)seed << 32) + step + 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        RowSrc src{false, nullptr, nullptr, nullptr, batch, T.ring_head, (float)((z >> 40) * 0x1p-24)};
        uint32_t blocks = 0;
        e = run_train(f, T, src, s, &blocks);
        if (e != hipSuccess) break;
        // the last step of the batch also publishes the weights for the renderer
        const bool last = k + 1 == nsteps;
        hipLaunchKernelGGL(k_guide_reduce, dim3((kGuideParams + kReduceParams - 1) / kReduceParams), dim3(256), 0, s,
                           T, blocks, 1, step, lr, (float *)nullptr, last ? pub_frag : nullptr,
                           last ? pub_bias : nullptr, (uint2 *)nullptr, (float *)nullptr);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_guide_debug_forward(const Frame &f, const float *x, uint32_t n, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_guide_fwd_debug, dim3(nblocks(((size_t)n + 31) / 32, 4, 2048)), dim3(256), 0, s, f, x, n,
                       out);
    return hipGetLastError();
}

hipError_t launch_guide_debug_grad(const Frame &f, const GuideTrain &T, const float *x, const float *dirs,
                                   const float *w, uint32_t n, float *grad, int adam, uint32_t step, float lr,
                                   hipStream_t s, uint2 *pub_a, float *pub_ab, uint2 *pub_b, float *pub_bb)
{
    RowSrc src{true, x, dirs, w, n, nullptr, 0.0f};
    uint32_t blocks = 0;
    hipError_t e = run_train(f, T, src, s, &blocks);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_guide_reduce, dim3((kGuideParams + kReduceParams - 1) / kReduceParams), dim3(256), 0, s, T, blocks, adam,
                       step, lr, grad, pub_a, pub_ab, pub_b, pub_bb);
    return hipGetLastError();
}

hipError_t launch_guide_debug_mixture(const float *out40, const float *dirs, const float *u, uint32_t n, float *pdf,
                                      float *sample, hipStream_t s)
{
    hipLaunchKernelGGL(k_guide_mix_debug, dim3(nblocks(n, 256, 1u << 20)), dim3(256), 0, s, out40, dirs, u, n, pdf,
                       sample);
    return hipGetLastError();
}

}  // namespace qpt
