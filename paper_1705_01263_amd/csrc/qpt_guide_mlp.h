// Inference of the learned proposal on gfx950's matrix cores, shared by the
// standalone inference kernel and the shading kernel of the guided vertices:
// BF16 MFMA forward of the 32-64-64-64-40 network with FP32 accumulation,
// the half-row input encoding per lane, and the decode of the 8-lobe mixture
// into its packed form.
//
// MFMA mapping (v_mfma_f32_32x32x16_bf16, D = A x B + C, 32x32x16).
// Operands are kept as 4-element fragments of 8-wide k-blocks s:
//   A fragment = weights:     lane l holds W[k = 8s + 4(l/32) + e][o = 32t + l%32], e = 0..3
//   B fragment = activations: lane l holds act[row = l%32][k = 8s + 4(l/32) + e]
//   D:                        lane l, register v holds Z[o = 32t + 8(v/4) + 4(l/32) + v%4][row = l%32]
// so registers 4s'..4s'+3 of the output tile s'/4 are exactly the B fragment
// of block s' of the next layer: layers chain in registers. One 16-deep MFMA
// takes fragments 2s and 2s + 1 of both operands as its 8 elements per lane:
// the hardware pairs element e of A and B lanes for one reduction index, and
// both operands map (lane half, e) to the same k = 16s + 8(e/4) + 4(l/32) +
// e%4, so the product is the sum over the 16 k of the block in another order.
// Each row (a path vertex or a training sample) is handled by the lane pair
// (l, l + 32); a wave works on 32 rows at a time.
#pragma once

#include <hip/hip_runtime.h>

#include "qpt_guide_dev.h"
#include "qpt_internal.h"

namespace qpt {
namespace mlp {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef short v2s __attribute__((ext_vector_type(2)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kKS[4] = {4, 8, 8, 8};          // k-steps of 8 per layer
constexpr int kN[4] = {64, 64, 64, 40};        // true output widths
constexpr int kFB[4] = {0, 8, 24, 40};         // first forward fragment of each layer

// round to the nearest BF16, ties to even (v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ uint32_t bf16_rne(float f)
{
    return (uint32_t)__builtin_bit_cast(unsigned short, (__bf16)f);
}

typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

// four floats -> four BF16 (round to nearest even), two per conversion
__device__ __forceinline__ v4s pack4(float a, float b, float c, float d)
{
    uint32_t lo = __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f){a, b}, v2bf));
    uint32_t hi = __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f){c, d}, v2bf));
    return __builtin_bit_cast(v4s, make_uint2(lo, hi));
}

// the four BF16 of a fragment word pair, low half first (a reinterpretation:
// building the vector from shifted halves costs a bitfield insert each)
__device__ __forceinline__ v4s as_v4s(uint2 u) { return __builtin_bit_cast(v4s, u); }

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v8bf cat8(v4s lo, v4s hi)
{
    return __builtin_bit_cast(v8bf, (v8s){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]});
}

// D += A B over a 16-deep block given as two 8-deep fragments of each operand
__device__ __forceinline__ v16f mfma2(v4s a0, v4s a1, v4s b0, v4s b1, v16f c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(cat8(a0, a1), cat8(b0, b1), c, 0, 0, 0);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// one layer: acc[t] = W_L^T x in + b for the two 32-wide output tiles
template <int L>
__device__ __forceinline__ void layer_fwd(const uint2 *sfrag, const float *sbias, const v4s *in, v16f *acc)
{
    const uint32_t lane = lane_id(), half = lane >> 5;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        // the bias is the accumulator's initial value (four float4 reads)
        v16f c;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float4 b = *(const float4 *)&sbias[L * 64 + 32 * t + 8 * q + 4 * half];
            c[4 * q] = b.x;
            c[4 * q + 1] = b.y;
            c[4 * q + 2] = b.z;
            c[4 * q + 3] = b.w;
        }
#pragma unroll
        for (int s = 0; s < kKS[L]; s += 2) {
            const uint2 *f = sfrag + (kFB[L] + t * kKS[L] + s) * 64 + lane;
            c = mfma2(as_v4s(f[0]), as_v4s(f[64]), in[s], in[s + 1], c);
        }
        acc[t] = c;
    }
}

__device__ __forceinline__ void load_weights(const uint2 *frag, const float *bias, uint2 *sfrag, float *sbias)
{
    for (uint32_t i = threadIdx.x; i < kGuideFrags * 64; i += blockDim.x) sfrag[i] = frag[i];
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) sbias[i] = bias[i];
}

// ReLU and BF16 operands without the mask (inference): round to BF16 first,
// then a 16-bit signed max with 0 per half word (a BF16 value is negative
// exactly when its sign bit is set, and rounding keeps the sign), the same
// bits as rounding max(z, 0)
__device__ __forceinline__ void relu_pack_infer(const v16f *acc, v4s *out)
{
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int t = s / 4, b = 4 * (s % 4);
        const uint2 u = __builtin_bit_cast(uint2, pack4(acc[t][b], acc[t][b + 1], acc[t][b + 2], acc[t][b + 3]));
        const v2s lo = __builtin_elementwise_max(__builtin_bit_cast(v2s, u.x), (v2s){0, 0});
        const v2s hi = __builtin_elementwise_max(__builtin_bit_cast(v2s, u.y), (v2s){0, 0});
        out[s] = __builtin_bit_cast(v4s, make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi)));
    }
}

// inference forward: only the running B operands, no stored activations
__device__ __forceinline__ void mlp_infer(const uint2 *sfrag, const float *sbias, const v4s *a0, v16f *out)
{
    v16f acc[2];
    v4s cur[8];
    layer_fwd<0>(sfrag, sbias, a0, acc);
    relu_pack_infer(acc, cur);
    layer_fwd<1>(sfrag, sbias, cur, acc);
    relu_pack_infer(acc, cur);
    layer_fwd<2>(sfrag, sbias, cur, acc);
    relu_pack_infer(acc, cur);
    layer_fwd<3>(sfrag, sbias, cur, out);
}

// the B operands of layer 0 for this lane's half of the row: half h needs
// features 8s + 4h .. 8s + 4h + 3, i.e. octaves 2h and 2h + 1 of axis s
// (s < 3), then the polar (h = 0) or azimuthal (h = 1) terms; the same
// values as the full encoding, computed once per lane
__device__ __forceinline__ void encode_half(guide::V3 x, guide::V3 wo, const float *bmin, const float *binv, v4s *a0)
{
    const uint32_t h = lane_id() >> 5;
    float xh[3] = {(x.x - bmin[0]) * binv[0], (x.y - bmin[1]) * binv[1], (x.z - bmin[2]) * binv[2]};
    const float m0 = 0.5f * guide::kOct[2 * h], m1 = 0.5f * guide::kOct[2 * h + 1];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float s0, c0, s1, c1;
        guide::sincos_rev(m0 * xh[a], &s0, &c0);
        guide::sincos_rev(m1 * xh[a], &s1, &c1);
        a0[a] = pack4(s0, c0, s1, c1);
    }
    // lane half 0: th (one atan2 of (sin th, cos th)); half 1: ph -- one
    // atan2 per lane with lane-dependent arguments, no divergence
    float y = fminf(1.0f, fmaxf(-1.0f, wo.y));
    float ay = h ? wo.x : sqrtf(fmaxf(0.0f, 1.0f - y * y));
    float ax = h ? -wo.z : y;
    float ang = guide::atan2_enc(ay, ax);
    if (h && ang < 0.0f) ang += 2.0f * guide::kPiF;
    float r1 = ang * (h ? 1.0f / (2.0f * guide::kPiF) : 1.0f / guide::kPiF);
    float r0 = h ? r1 : 0.5f * r1;
    r1 = h ? 2.0f * r1 : r1;
    float s0, c0, s1, c1;
    guide::sincos_rev(r0, &s0, &c0);
    guide::sincos_rev(r1, &s1, &c1);
    a0[3] = pack4(s0, c0, s1, c1);
}

// Every BF16 copy of the weights (training's and the renderer's) orders the
// last layer's outputs by parameter, then lobe: accumulator row 8c + k holds
// parameter c (0: weight logit, 1-3: mean direction, 4: concentration) of
// lobe k, which is network output 5k + c (the FP32 master parameters keep
// the network's order). A lane of the 32 x 32 output tile holds rows
// 8q + 4h + r (h its lane half), so each lane ends up with all five
// parameters of lobes 4h .. 4h + 3 and decodes them, or takes their
// gradient, without exchanging outputs with its partner lane.
__host__ __device__ constexpr int frag_out_row(int r) { return r < 40 ? 5 * (r % 8) + r / 8 : r; }
// and its inverse: the accumulator row of network output o
__host__ __device__ constexpr int frag_in_row(int o) { return o < 40 ? 8 * (o % 5) + o / 5 : o; }

// The mixture of the lane pair's row (both lanes of the pair pass the row's
// hit point x and outgoing direction wo) in its packed form at dst (kMixU4
// uint4: lane half h stores lobes 4h .. 4h + 3 and their weights). Every lane
// of the wave takes part (MFMA and the exchange between the pair); a row
// with valid false is computed and not stored. The weights' softmax takes its
// maximum and sum over both halves; the concentration is softplus(raw) +
// 1e-3, at most 1e4; the mean direction is normalised.
__device__ __forceinline__ void infer_pair(const uint2 *sfrag, const float *sbias, guide::V3 x, guide::V3 wo,
                                           const float *bmin, const float *binv, bool valid, uint4 *dst)
{
    const uint32_t h = lane_id() >> 5;
    v4s a0[4];
    encode_half(x, wo, bmin, binv, a0);
    v16f out[2];
    mlp_infer(sfrag, sbias, a0, out);
    // this lane's lobes 4h + j (the fragments' output order, frag_out_row):
    // logit out[0][j], mean direction out[0][4 + j], out[0][8 + j],
    // out[0][12 + j], concentration out[1][j]
    float mx = fmaxf(fmaxf(out[0][0], out[0][1]), fmaxf(out[0][2], out[0][3]));
    mx = fmaxf(mx, guide::xor32(mx));
    float e[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) e[j] = __expf(out[0][j] - mx);
    float se = (e[0] + e[1]) + (e[2] + e[3]);
    se += guide::xor32(se);
    if (!valid) return;
    const float inv = 1.0f / se;
    uint32_t q[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float ox = out[0][4 + j], oy = out[0][8 + j], oz = out[0][12 + j], ok = out[1][j];
        const float in = rsqrtf(fmaxf(ox * ox + oy * oy + oz * oz, 1e-24f));
        const float sp = ok > 20.0f ? ok : __logf(1.0f + __expf(ok));
        const float kap = fminf(sp + 1e-3f, 1e4f);
        q[2 * j] = guide::pack_h2(ox * in, oy * in);
        q[2 * j + 1] = guide::pack_h2(oz * in, kap);
    }
    // lobes 4h .. 4h + 3 are uint4 2h and 2h + 1; weights 4h .. 4h + 3 half of uint4 4
    dst[2 * h] = make_uint4(q[0], q[1], q[2], q[3]);
    dst[2 * h + 1] = make_uint4(q[4], q[5], q[6], q[7]);
    ((uint2 *)(dst + 4))[h] = make_uint2(guide::pack_h2(e[0] * inv, e[1] * inv), guide::pack_h2(e[2] * inv, e[3] * inv));
}

// The mixtures of a wave's 64 rows, one per lane (x, wo and valid of the
// lane's own row), into rows[0 .. 63]: rows 0-31 in one pass of the lane
// pairs, rows 32-63 in a second. Every lane of the wave takes part.
__device__ __forceinline__ void infer_wave64(const uint2 *sfrag, const float *sbias, guide::V3 x, guide::V3 wo,
                                             bool valid, const float *bmin, const float *binv, uint4 *rows)
{
    const uint32_t lane = lane_id(), h = lane >> 5;
    const guide::V3 xp = {guide::xor32(x.x), guide::xor32(x.y), guide::xor32(x.z)};
    const guide::V3 wp = {guide::xor32(wo.x), guide::xor32(wo.y), guide::xor32(wo.z)};
    const bool vp = guide::xor32_u32(valid ? 1u : 0u) != 0u;
    infer_pair(sfrag, sbias, h ? xp : x, h ? wp : wo, bmin, binv, h ? vp : valid, rows + (lane & 31u) * guide::kMixU4);
    // the second pass reads the weights from LDS again: shared between the
    // passes, the 56 fragments would stay live in registers
    asm volatile("" ::: "memory");
    infer_pair(sfrag, sbias, h ? x : xp, h ? wo : wp, bmin, binv, h ? valid : vp,
               rows + (32u + (lane & 31u)) * guide::kMixU4);
}

}  // namespace mlp
}  // namespace qpt
