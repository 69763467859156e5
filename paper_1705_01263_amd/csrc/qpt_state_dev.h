// Path state in one of two layouts (device code). The full layout keeps the
// direction, the throughput and the hit record as float4 each; the compressed
// one (render option compress_state; Sec. 3.1.1: unit vectors as octahedral
// 2 x 16 bits, unit floats as 16-bit fixed point, limited-range floats as
// half precision) keeps the direction and the previous vertex in 8 bytes,
// the throughput and the last sampling density in 8 and the hit record in
// 12. Both live in the same arrays (the compressed records packed densely
// from the start). A direction is quantised where it is sampled, so tracing,
// the BSDF and the densities all see the direction the state holds.
#pragma once

#include <hip/hip_runtime.h>

#include "qpt_internal.h"

namespace qpt {
namespace state {

// octahedral map of a unit vector onto two signed 16-bit integers
__device__ __forceinline__ uint32_t oct_encode(float x, float y, float z)
{
    const float s = 1.0f / (fabsf(x) + fabsf(y) + fabsf(z));
    float u = x * s, v = y * s;
    if (z < 0.0f) {
        const float uu = (1.0f - fabsf(v)) * copysignf(1.0f, u);
        v = (1.0f - fabsf(u)) * copysignf(1.0f, v);
        u = uu;
    }
    const int qu = (int)rintf(fminf(fmaxf(u, -1.0f), 1.0f) * 32767.0f);
    const int qv = (int)rintf(fminf(fmaxf(v, -1.0f), 1.0f) * 32767.0f);
    return ((uint32_t)qu & 0xffffu) | (((uint32_t)qv & 0xffffu) << 16);
}

__device__ __forceinline__ void oct_decode(uint32_t e, float &x, float &y, float &z)
{
    float u = (float)(int16_t)(e & 0xffffu) * (1.0f / 32767.0f);
    float v = (float)(int16_t)(e >> 16) * (1.0f / 32767.0f);
    const float w = 1.0f - fabsf(u) - fabsf(v);
    if (w < 0.0f) {
        const float uu = (1.0f - fabsf(v)) * copysignf(1.0f, u);
        v = (1.0f - fabsf(u)) * copysignf(1.0f, v);
        u = uu;
    }
    const float r = 1.0f / sqrtf(u * u + v * v + w * w);
    x = u * r;
    y = v * r;
    z = w * r;
}

__device__ __forceinline__ uint32_t half_bits(float f)
{
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)fminf(f, 65504.0f));
}

__device__ __forceinline__ float half_value(uint32_t b)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(b & 0xffffu));
}

// the direction the state will hold (unchanged in the full layout)
__device__ __forceinline__ void quantise_dir(const Frame &F, float &x, float &y, float &z)
{
    if (F.compress) oct_decode(oct_encode(x, y, z), x, y, z);
}

// next ray's direction (xyz) and the previous vertex (w, as bits)
__device__ __forceinline__ float4 load_dir(const Frame &F, const Pool &P, uint32_t s)
{
    if (!F.compress) return P.ray_d[s];
    const uint2 c = ((const uint2 *)P.ray_d)[s];
    float x, y, z;
    oct_decode(c.x, x, y, z);
    return make_float4(x, y, z, __uint_as_float(c.y));
}

__device__ __forceinline__ void store_dir(const Frame &F, const Pool &P, uint32_t s, float4 d)
{
    if (!F.compress) {
        P.ray_d[s] = d;
        return;
    }
    ((uint2 *)P.ray_d)[s] = make_uint2(oct_encode(d.x, d.y, d.z), __float_as_uint(d.w));
}

// throughput (xyz) and the density of the last sampled direction (w)
__device__ __forceinline__ float4 load_thr(const Frame &F, const Pool &P, uint32_t s)
{
    if (!F.compress) return P.thr[s];
    const uint2 c = ((const uint2 *)P.thr)[s];
    return make_float4(half_value(c.x), half_value(c.x >> 16), half_value(c.y), half_value(c.y >> 16));
}

__device__ __forceinline__ void store_thr(const Frame &F, const Pool &P, uint32_t s, float4 t)
{
    if (!F.compress) {
        P.thr[s] = t;
        return;
    }
    ((uint2 *)P.thr)[s] = make_uint2(half_bits(t.x) | (half_bits(t.y) << 16), half_bits(t.z) | (half_bits(t.w) << 16));
}

// hit record: t, triangle (bits), barycentrics b1, b2
__device__ __forceinline__ float4 load_hit(const Frame &F, const Pool &P, uint32_t s)
{
    if (!F.compress) return P.hit[s];
    const float *h = (const float *)P.hit + 3 * (size_t)s;
    const uint32_t b = __float_as_uint(h[2]);
    return make_float4(h[0], h[1], (float)(b & 0xffffu) * (1.0f / 65535.0f), (float)(b >> 16) * (1.0f / 65535.0f));
}

__device__ __forceinline__ void store_hit(const Frame &F, const Pool &P, uint32_t s, float4 hv)
{
    if (!F.compress) {
        P.hit[s] = hv;
        return;
    }
    float *h = (float *)P.hit + 3 * (size_t)s;
    const uint32_t q1 = (uint32_t)rintf(fminf(fmaxf(hv.z, 0.0f), 1.0f) * 65535.0f);
    const uint32_t q2 = (uint32_t)rintf(fminf(fmaxf(hv.w, 0.0f), 1.0f) * 65535.0f);
    h[0] = hv.x;
    h[1] = hv.y;
    h[2] = __uint_as_float(q1 | (q2 << 16));
}

}  // namespace state
}  // namespace qpt
