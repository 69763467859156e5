// Device-side pieces of the learned proposal shared by the shading kernel and
// the network kernels: the 8-lobe von Mises-Fisher mixture (decode, pdf,
// sampling) and the input encoding. FP32 throughout.
#pragma once

#include <hip/hip_runtime.h>

#include "qpt_internal.h"

namespace qpt {
namespace guide {

constexpr float kPiF = 3.14159265358979323846f;
constexpr int kLobes = 8;
// frequency multipliers of the four position octaves
#ifndef QPT_GUIDE_OCT
#define QPT_GUIDE_OCT 0
#endif
#if QPT_GUIDE_OCT == 1
__device__ constexpr float kOct[4] = {1.0f, 4.0f, 16.0f, 64.0f};
#elif QPT_GUIDE_OCT == 2
__device__ constexpr float kOct[4] = {2.0f, 8.0f, 32.0f, 128.0f};
#else
__device__ constexpr float kOct[4] = {1.0f, 2.0f, 4.0f, 8.0f};
#endif

struct V3 {
    float x, y, z;
};

// the value of lane l ^ 32 (the other half of the wave), by gfx950's
// v_permlane32_swap, which exchanges one register's upper half with another
// register's lower half: given the value twice, one of the two results
// holds the partner's value on each lane and the other the lane's own, so
// XOR-ing both with the own value leaves the partner's bits whichever of
// the two results it is in (no LDS crossbar round trip as with a shuffle)
__device__ __forceinline__ uint32_t xor32_u32(uint32_t v)
{
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return r[0] ^ r[1] ^ v;
}
__device__ __forceinline__ float xor32(float v) { return __uint_as_float(xor32_u32(__float_as_uint(v))); }
__device__ __forceinline__ float dot3(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// sin and cos of 2 pi r for an angle r given in revolutions (hardware
// v_sin_f32 / v_cos_f32: about 1e-7 absolute error for |r| <= 4)
__device__ __forceinline__ void sincos_rev(float r, float *s, float *c)
{
    *s = __builtin_amdgcn_sinf(r);
    *c = __builtin_amdgcn_cosf(r);
}

// atan2 with C's quadrant and signed-zero conventions, from a least-squares
// polynomial for atan on [0, 1] fitted for this library (degree 6 in a^2,
// |error| < 4e-7 rad in FP32); the encoding only feeds it to sin and cos
__device__ __forceinline__ float atan2_enc(float y, float x)
{
    float ax = fabsf(x), ay = fabsf(y);
    float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    float a = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    a = fminf(a, 1.0f);
    float q = a * a;
    float r = 0.006812187377363443f;
    r = fmaf(r, q, -0.03360540792346001f);
    r = fmaf(r, q, 0.07962503284215927f);
    r = fmaf(r, q, -0.1323341578245163f);
    r = fmaf(r, q, 0.19807834923267365f);
    r = fmaf(r, q, -0.3331736922264099f);
    r = fmaf(r, q, 0.9999961256980896f);
    r *= a;
    if (ay > ax) r = 0.5f * kPiF - r;
    if (__builtin_signbit(x)) r = kPiF - r;
    return __builtin_signbit(y) ? -r : r;
}

// encoding angles of an outgoing direction: th = polar angle from +y over
// pi, ph = atan2(x, -z) over 2 pi in [0, 1)
__device__ __forceinline__ float enc_theta(V3 wo)
{
    float y = fminf(1.0f, fmaxf(-1.0f, wo.y));
    return atan2_enc(sqrtf(fmaxf(0.0f, 1.0f - y * y)), y) * (1.0f / kPiF);
}

__device__ __forceinline__ float enc_phi(V3 wo)
{
    float ph = atan2_enc(wo.x, -wo.z);
    if (ph < 0.0f) ph += 2.0f * kPiF;
    return ph * (1.0f / (2.0f * kPiF));
}

// the decoded mixture as stored per path slot: lobe k = (mu.xyz, kappa), then
// the 8 weights in two float4
struct Mix {
    float4 lobe[kLobes];
    float4 w0, w1;
};

__device__ __forceinline__ float weight(const Mix &m, int k)
{
    const float4 &w = k < 4 ? m.w0 : m.w1;
    int j = k & 3;
    return j == 0 ? w.x : (j == 1 ? w.y : (j == 2 ? w.z : w.w));
}
__device__ __forceinline__ float4 lobe(const Mix &m, int k) { return m.lobe[k]; }

__device__ __forceinline__ float softplus(float r) { return r > 20.0f ? r : log1pf(expf(r)); }

// The mixture as stored per path slot, 80 bytes: uint4 j < 4 holds lobes 2j
// and 2j + 1 as FP16 (mu.x, mu.y, mu.z, kappa); uint4 4 holds the eight
// weights as FP16. The density the renderer samples and evaluates is the one
// these stored values define, decoded by unpack_mix (means and weights
// renormalised in FP32), so rounding to FP16 leaves the estimator unbiased.
constexpr int kMixU4 = 5;

typedef float v2f_ __attribute__((ext_vector_type(2)));
typedef _Float16 v2h_ __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_h2(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f_){a, b}, v2h_));
}

__device__ __forceinline__ float2 unpack_h2(uint32_t u)
{
    v2f_ f = __builtin_convertvector(__builtin_bit_cast(v2h_, u), v2f_);
    return make_float2(f.x, f.y);
}

__device__ __forceinline__ float4 unit_lobe(float2 a, float2 b)
{
    float in = rsqrtf(fmaxf(a.x * a.x + a.y * a.y + b.x * b.x, 1e-24f));
    return make_float4(a.x * in, a.y * in, b.x * in, b.y);
}

// a stored mixture read in place, lobe by lobe (keeps the shading kernel's
// registers free); decodes exactly as unpack_mix does
struct MixRef {
    const uint4 *p;
    float winv;  // 1 / sum of the stored weights
};

__device__ __forceinline__ MixRef mix_ref(const uint4 *p)
{
    uint4 w = p[4];
    float2 w01 = unpack_h2(w.x), w23 = unpack_h2(w.y), w45 = unpack_h2(w.z), w67 = unpack_h2(w.w);
    return {p, 1.0f / (((w01.x + w01.y) + (w23.x + w23.y)) + ((w45.x + w45.y) + (w67.x + w67.y)))};
}

__device__ __forceinline__ float weight(const MixRef &m, int k)
{
    const uint32_t *w = (const uint32_t *)(m.p + 4);
    float2 h = unpack_h2(w[k >> 1]);
    return (k & 1 ? h.y : h.x) * m.winv;
}

__device__ __forceinline__ float4 lobe(const MixRef &m, int k)
{
    uint2 u = ((const uint2 *)m.p)[k];
    return unit_lobe(unpack_h2(u.x), unpack_h2(u.y));
}

__device__ inline void unpack_mix(const uint4 *src, Mix &m)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint4 u = src[j];
        m.lobe[2 * j] = unit_lobe(unpack_h2(u.x), unpack_h2(u.y));
        m.lobe[2 * j + 1] = unit_lobe(unpack_h2(u.z), unpack_h2(u.w));
    }
    uint4 w = src[4];
    float2 w01 = unpack_h2(w.x), w23 = unpack_h2(w.y), w45 = unpack_h2(w.z), w67 = unpack_h2(w.w);
    float inv = 1.0f / (((w01.x + w01.y) + (w23.x + w23.y)) + ((w45.x + w45.y) + (w67.x + w67.y)));
    m.w0 = make_float4(w01.x * inv, w01.y * inv, w23.x * inv, w23.y * inv);
    m.w1 = make_float4(w45.x * inv, w45.y * inv, w67.x * inv, w67.y * inv);
}

// outputs 5k..5k+4 of lobe k: logit, mu_raw xyz, kappa_raw
__device__ inline void decode(const float *o, Mix &m)
{
    float mx = o[0];
    for (int k = 1; k < kLobes; ++k) mx = fmaxf(mx, o[5 * k]);
    float e[kLobes], sum = 0.0f;
    for (int k = 0; k < kLobes; ++k) {
        e[k] = expf(o[5 * k] - mx);
        sum += e[k];
    }
    float inv = 1.0f / sum;
    m.w0 = make_float4(e[0] * inv, e[1] * inv, e[2] * inv, e[3] * inv);
    m.w1 = make_float4(e[4] * inv, e[5] * inv, e[6] * inv, e[7] * inv);
    for (int k = 0; k < kLobes; ++k) {
        float x = o[5 * k + 1], y = o[5 * k + 2], z = o[5 * k + 3];
        float n = fmaxf(sqrtf(x * x + y * y + z * z), 1e-12f);
        float kap = fminf(softplus(o[5 * k + 4]) + 1e-3f, 1e4f);
        m.lobe[k] = make_float4(x / n, y / n, z / n, kap);
    }
}

// 1 - e^-x for x >= 0: a Taylor polynomial below 0.1, where the subtraction
// would cancel (truncation below 2e-7 relative), else the hardware exponential
__device__ __forceinline__ float one_minus_exp_neg(float x)
{
    const float p = x * (1.0f - x * (0.5f - x * (1.0f / 6.0f - x * (1.0f / 24.0f - x * (1.0f / 120.0f)))));
    return x < 0.1f ? p : 1.0f - __expf(-x);
}

// vMF density on the unit sphere, kappa / (2 pi (1 - e^-2 kappa)) e^(kappa (mu.w - 1)),
// with the hardware's exponential and reciprocal (evaluated at every lobe
// for each density the guided shading needs, twice per vertex)
__device__ __forceinline__ float vmf_pdf(float4 l, V3 w)
{
    float c = l.x * w.x + l.y * w.y + l.z * w.z;
    return l.w * __builtin_amdgcn_rcpf(2.0f * kPiF * one_minus_exp_neg(2.0f * l.w)) * __expf(l.w * (c - 1.0f));
}

// the eight lobes' weights times their vMF normalisers, formed once per
// mixture for the densities evaluated at several directions
struct MixCoef {
    float c[kLobes];
};

template <class M>
__device__ __forceinline__ MixCoef mixture_coef(const M &m)
{
    MixCoef mc;
#pragma unroll
    for (int k = 0; k < kLobes; ++k) {
        const float kap = lobe(m, k).w;
        mc.c[k] = weight(m, k) * (kap * __builtin_amdgcn_rcpf(2.0f * kPiF * one_minus_exp_neg(2.0f * kap)));
    }
    return mc;
}

// the mixture's density at w, sum_k c_k e^(kappa_k (mu_k.w - 1)) (the same
// value as the sum of weight times vmf_pdf, up to the order of the products)
template <class M>
__device__ __forceinline__ float mixture_pdf(const M &m, const MixCoef &mc, V3 w)
{
    float q = 0.0f;
#pragma unroll
    for (int k = 0; k < kLobes; ++k) {
        const float4 l = lobe(m, k);
        q += mc.c[k] * __expf(l.w * ((l.x * w.x + l.y * w.y + l.z * w.z) - 1.0f));
    }
    return q;
}

template <class M>
__device__ __forceinline__ float mixture_pdf(const M &m, V3 w)
{
    return mixture_pdf(m, mixture_coef(m), w);
}

// lobe: first k with u < cumulative weight; direction by stable vMF sampling
// (Jakob 2012) in a Duff et al. 2017 frame around mu
template <class M>
__device__ inline V3 mixture_sample(const M &m, float u_lobe, float u1, float u2)
{
    int k = kLobes - 1;
    float c = 0.0f;
    for (int j = 0; j < kLobes - 1; ++j) {
        c += weight(m, j);
        if (u_lobe < c) {
            k = j;
            break;
        }
    }
    float4 l = lobe(m, k);
    float w = 1.0f + logf(u1 + (1.0f - u1) * expf(-2.0f * l.w)) / l.w;
    w = fminf(1.0f, fmaxf(-1.0f, w));
    float s = copysignf(1.0f, l.z);
    float a = -1.0f / (s + l.z);
    float b = l.x * l.y * a;
    V3 t1 = {1.0f + s * l.x * l.x * a, s * b, -s * l.x};
    V3 t2 = {b, s + l.y * l.y * a, -l.y};
    float r = sqrtf(fmaxf(0.0f, 1.0f - w * w));
    float sp, cp;
    sincos_rev(u2, &sp, &cp);
    return {w * l.x + r * (cp * t1.x + sp * t2.x), w * l.y + r * (cp * t1.y + sp * t2.y),
            w * l.z + r * (cp * t1.z + sp * t2.z)};
}

// Weight of a training record once its path has ended with radiance L: the
// luminance of (L - radiance before the vertex's NEE - that NEE) / the
// throughput before the scattering (roulette folded in), per channel where
// that throughput is positive, each channel clamped at 0: the sample's own
// estimate f cos L_i / p of the scattering integral. r3 = radiance before
// the NEE, r4 = throughput before the scattering, r5 = the NEE (0 if occluded).
__device__ __forceinline__ float record_weight(float4 r3, float4 r4, float4 r5, float4 L)
{
    // what the path gained after the vertex: its final radiance less the
    // radiance right after the vertex's own next-event estimate, formed by
    // the same addition the occlusion kernel made (r5 is zero when occluded),
    // so a path that gains nothing afterwards weighs exactly zero
    const float li[3] = {L.x - (r3.x + r5.x), L.y - (r3.y + r5.y), L.z - (r3.z + r5.z)};
    const float tb[3] = {r4.x, r4.y, r4.z};
    const float wl[3] = {0.2126f, 0.7152f, 0.0722f};
    float w = 0.0f;
    for (int c = 0; c < 3; ++c) w += tb[c] > 0.0f ? wl[c] * fmaxf(0.0f, li[c] / tb[c]) : 0.0f;
    return w;
}

// the 32 input features: sin/cos of 2^o pi x_hat per axis and octave, then
// sin/cos of pi th, 2 pi th, 2 pi ph, 4 pi ph of the outgoing direction
// (th = polar angle from +y over pi, ph = atan2(x, -z) over 2 pi in [0, 1))
__device__ inline void encode(V3 x, V3 wo, const float *bmin, const float *binv, float *f)
{
    float xh[3] = {(x.x - bmin[0]) * binv[0], (x.y - bmin[1]) * binv[1], (x.z - bmin[2]) * binv[2]};
    for (int a = 0; a < 3; ++a)
        for (int o = 0; o < 4; ++o) sincos_rev(0.5f * kOct[o] * xh[a], &f[8 * a + 2 * o], &f[8 * a + 2 * o + 1]);
    float th = enc_theta(wo), ph = enc_phi(wo);
    float rev[4] = {0.5f * th, th, ph, 2.0f * ph};
    for (int j = 0; j < 4; ++j) sincos_rev(rev[j], &f[24 + 2 * j], &f[25 + 2 * j]);
}

}  // namespace guide
}  // namespace qpt
