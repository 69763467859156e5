// HIP kernels of libqpt for gfx950 (CDNA4, wave64).
//
// One pass = one sample per pixel over the frame (Sec. 3.2.2). A batch of
// passes (or of pixels) is rendered as a wavefront (Sec. 3.1): a generation
// kernel fills the path pool, then for every depth v a closest-hit kernel, a
// shading kernel (emission + MIS, next-event estimation, BSDF sampling,
// roulette) and an occlusion kernel run over compact queues of path slots;
// queues are rebuilt just in time by wave-level appends (Sec. 3.1.2); state
// stays in place as structures of arrays (Sec. 3.1.1). A final kernel adds
// the batch into the FP64 framebuffer in pass order and bumps the per-pixel
// sample counts (Appendix A.4).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "qpt_guide_dev.h"
#include "qpt_guide_mlp.h"
#include "qpt_internal.h"
#include "qpt_state_dev.h"

namespace qpt {

namespace {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kInvPi = 0.318309886183790671538f;

// ---------------------------------------------------------------- vectors

struct f3 {
    float x, y, z;
};
__device__ __forceinline__ f3 mk(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ f3 xyz(float4 v) { return {v.x, v.y, v.z}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator*(f3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ f3 operator*(f3 a, f3 b) { return {a.x * b.x, a.y * b.y, a.z * b.z}; }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float length(f3 a) { return sqrtf(dot(a, a)); }
__device__ __forceinline__ f3 normalize(f3 a) { return a * (1.0f / length(a)); }
__device__ __forceinline__ float maxc(f3 a) { return fmaxf(a.x, fmaxf(a.y, a.z)); }
__device__ __forceinline__ float lum(f3 c) { return 0.2126f * c.x + 0.7152f * c.y + 0.0722f * c.z; }
__device__ __forceinline__ float4 f4(f3 a, float w) { return make_float4(a.x, a.y, a.z, w); }
__device__ __forceinline__ float ubits(uint32_t u) { return __uint_as_float(u); }
__device__ __forceinline__ uint32_t fbits(float f) { return __float_as_uint(f); }

// ------------------------------------------------------- wave primitives

// Append to a queue from a whole wave with one atomic: ballot the lanes
// that append, the first of them reserves popcount slots, every lane finds
// its offset with mbcnt. All 64 lanes must call it.
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool pred)
{
    unsigned long long mask = __ballot(pred);
    uint32_t base = 0;
    if (mask) {
        uint32_t lane = __lane_id();
        uint32_t leader = __ffsll((long long)mask) - 1;
        if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
        base = __shfl(base, (int)leader);
    }
    uint32_t lo = (uint32_t)mask, hi = (uint32_t)(mask >> 32);
    return base + __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
}

// Appends of a whole block to three counters with one atomic per counter
// and block (a device-wide atomic on one address is served one at a time, so
// every wave of a large launch taking its own slots serialised on it): each
// wave ballots its lanes, the waves' counts meet in LDS, three lanes turn them
// into offsets and reserve the block's totals, and every lane finds its place
// from its wave's offset and mbcnt. Every thread of the block calls it, with
// no lane of a wave inactive (two block barriers); s holds 3 x (waves + 1)
// words of LDS. A wave writes only its own counts and reads only its own
// offsets and the totals, which change only after the next call's first
// barrier, so calls in a loop need no further barrier.
constexpr uint32_t kAppendWaves = 8;  // the most waves per block that append
static_assert(kShadeBlock / 64 <= kAppendWaves && kBlock / 64 <= kAppendWaves && kShadeGuidedBlock / 64 <= kAppendWaves,
              "appending blocks fit the LDS counts");
__device__ __forceinline__ void block_append3(uint32_t *c0, bool p0, uint32_t *c1, bool p1, uint32_t *c2, bool p2,
                                              uint32_t *s, uint32_t &o0, uint32_t &o1, uint32_t &o2)
{
    constexpr uint32_t S = kAppendWaves + 1;
    const unsigned long long m[3] = {__ballot(p0), __ballot(p1), __ballot(p2)};
    const uint32_t waves = blockDim.x >> 6, w = threadIdx.x >> 6, lane = __lane_id();
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < 3; ++j) s[j * S + w] = (uint32_t)__popcll(m[j]);
    __syncthreads();
    if (threadIdx.x < 3) {
        uint32_t *a = s + threadIdx.x * S;
        uint32_t *ctr = threadIdx.x == 0 ? c0 : (threadIdx.x == 1 ? c1 : c2);
        uint32_t tot = 0;
        for (uint32_t k = 0; k < waves; ++k) {
            const uint32_t c = a[k];
            a[k] = tot;
            tot += c;
        }
        a[kAppendWaves] = tot ? atomicAdd(ctr, tot) : 0u;
    }
    __syncthreads();
    uint32_t r[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const uint32_t lo = (uint32_t)m[j], hi = (uint32_t)(m[j] >> 32);
        r[j] = s[j * S + kAppendWaves] + s[j * S + w] + __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
    }
    o0 = r[0];
    o1 = r[1];
    o2 = r[2];
}

// ----------------------------------------------------------------- Halton

__device__ __forceinline__ uint32_t div_b(uint32_t n, uint32_t m, uint32_t sh)
{
    uint32_t t = __umulhi(m, n);
    return (t + ((n - t) >> 1)) >> sh;
}

__device__ __forceinline__ uint64_t div_B(uint64_t n, uint64_t m, uint32_t sh)
{
    uint64_t t = __umul64hi(m, n);
    return (t + ((n - t) >> 1)) >> sh;
}

// digits of an e-digit chunk c, scrambled and reversed: sum pi(d_m) b^(e-1-m)
__device__ __forceinline__ uint32_t chunk_reverse(uint32_t c, const HaltonBase &h, uint32_t f)
{
    uint32_t r = 0;
    for (uint32_t k = 0; k < h.e; ++k) {
        uint32_t q = div_b(c, h.m32, h.sh32);
        uint32_t d = c - q * h.b;
        c = q;
        uint32_t p = f * d;
        r = r * h.b + (p - div_b(p, h.m32, h.sh32) * h.b);
    }
    return r;
}

// one Horner step over a chunk in base B = b^e: floor((R 2^32 + Y) / B)
__device__ __forceinline__ uint32_t horner(uint32_t R, uint32_t Y, const HaltonBase &h)
{
    return (uint32_t)div_B(((uint64_t)R << 32) | Y, h.m64, h.shB);
}

// floor(2^32 * RI^pi_b(i)), exact: i is split into base-B chunks (B < 2^32,
// at most three for 64-bit indices); each chunk's digits are reversed with
// 32-bit strength-reduced divisions, the chunks are combined by Horner's
// rule from the most significant one, each step an exact 64-bit division.
__device__ uint32_t radical_inverse_bits(uint64_t i, const HaltonBase &h, uint32_t f)
{
    uint64_t q1 = div_B(i, h.m64, h.shB);
    uint32_t c0 = (uint32_t)(i - q1 * h.B);
    uint32_t Y = 0;
    if (q1) {
        uint64_t q2 = div_B(q1, h.m64, h.shB);
        uint32_t c1 = (uint32_t)(q1 - q2 * h.B);
        if (q2) Y = horner(chunk_reverse((uint32_t)q2, h, f), 0u, h);
        Y = horner(chunk_reverse(c1, h, f), Y, h);
    }
    return horner(chunk_reverse(c0, h, f), Y, h);
}

// 32-bit sample of dimension d for Halton index i; dims 0/1 are the film
// offsets (digits left after the pixel's own base-2 / base-3 digits)
__device__ __forceinline__ uint32_t sample_bits(const Frame &F, uint64_t i, uint32_t d, uint32_t scramble)
{
    if (d == 0) return __brev((uint32_t)(i >> F.k2));
    if (d == 1) {
        uint64_t q = F.p3 > 1 ? div_B(i, F.m_p3, F.sh_p3) : i;
        return radical_inverse_bits(q, F.bases[1], 1u);
    }
    const HaltonBase &h = F.bases[d];
    return radical_inverse_bits(i, h, scramble ? h.f : 1u);
}

__device__ __forceinline__ float u24(uint32_t bits) { return (float)(bits >> 8) * 0x1p-24f; }

// full-screen enumeration: the index in [0, 2^k 3^l) whose first k binary and
// l ternary digits reversed are (x, y), plus pass * 2^k 3^l
__device__ uint64_t pixel_index(const Frame &F, uint32_t px, uint32_t py, uint64_t pass)
{
    uint32_t a = F.k2 ? (__brev(px) >> (32 - F.k2)) : 0u;
    uint32_t c = 0, y = py;
    for (uint32_t m = 0; m < F.l3; ++m) {
        c = c * 3u + y % 3u;
        y /= 3u;
    }
    uint32_t p3 = (uint32_t)F.p3;
    uint32_t diff = (c + p3 - a % p3) % p3;
    uint32_t t = (uint32_t)(((uint64_t)diff * F.inv2k_mod_p3) % p3);
    uint64_t i0 = (uint64_t)a + ((uint64_t)t << F.k2);
    return i0 + pass * F.S;
}

// ---------------------------------------------------------- intersection

struct RayPre {
    f3 o;
    float Sx, Sy, Sz;
    int kx, ky, kz;
    f3 inv;  // reciprocal direction for slab tests
};

__device__ __forceinline__ float comp(f3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

__device__ __forceinline__ RayPre prepare(f3 o, f3 d)
{
    RayPre r;
    r.o = o;
    int kz = 0;
    if (fabsf(d.y) > fabsf(comp(d, kz))) kz = 1;
    if (fabsf(d.z) > fabsf(comp(d, kz))) kz = 2;
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    float dz = comp(d, kz);
    if (dz < 0.0f) {
        int s = kx;
        kx = ky;
        ky = s;
    }
    r.kx = kx;
    r.ky = ky;
    r.kz = kz;
    r.Sx = comp(d, kx) / dz;
    r.Sy = comp(d, ky) / dz;
    r.Sz = 1.0f / dz;
    auto safe = [](float x) { return fabsf(x) < 1e-20f ? copysignf(1e-20f, x) : x; };
    r.inv = mk(1.0f / safe(d.x), 1.0f / safe(d.y), 1.0f / safe(d.z));
    return r;
}

// Watertight ray/triangle test (Woop, Benthin, Wald 2013) in FP32. The edge
// functions use separately rounded products so a shared edge evaluates to
// exactly opposite values in its two triangles; an exact zero is re-evaluated
// in FP64. Hit iff 0 < t < tmax.
__device__ __forceinline__ bool tri_test(const RayPre &r, float4 v0, float4 v1, float4 v2, float tmax,
                                         float &t_out, float &b1, float &b2)
{
#pragma clang fp contract(off)
    f3 A = xyz(v0) - r.o, B = xyz(v1) - r.o, C = xyz(v2) - r.o;
    float Akz = comp(A, r.kz), Bkz = comp(B, r.kz), Ckz = comp(C, r.kz);
    float Ax = fmaf(-r.Sx, Akz, comp(A, r.kx)), Ay = fmaf(-r.Sy, Akz, comp(A, r.ky));
    float Bx = fmaf(-r.Sx, Bkz, comp(B, r.kx)), By = fmaf(-r.Sy, Bkz, comp(B, r.ky));
    float Cx = fmaf(-r.Sx, Ckz, comp(C, r.kx)), Cy = fmaf(-r.Sy, Ckz, comp(C, r.ky));
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    float det = (U + V) + W;
    if (det == 0.0f) return false;
    float Az = r.Sz * Akz, Bz = r.Sz * Bkz, Cz = r.Sz * Ckz;
    float T = fmaf(U, Az, fmaf(V, Bz, W * Cz));
    float t = T / det;
    if (!(t > 0.0f && t < tmax)) return false;
    t_out = t;
    b1 = V / det;
    b2 = W / det;
    return true;
}

// slab test of child c against [0, tlim] from the distances to its six
// planes: a sort key (entry distance with the child slot in the two low bits;
// entry distances are >= 0, so unsigned order is distance order) or ~0 for a
// miss or an unused slot
__device__ __forceinline__ uint32_t key_from_t(float lx, float hx, float ly, float hy, float lz, float hz,
                                               int32_t ref, float tlim, uint32_t c)
{
    float tn = fmaxf(fmaxf(fminf(lx, hx), fminf(ly, hy)), fmaxf(fminf(lz, hz), 0.0f));
    float tf = fminf(fminf(fmaxf(lx, hx), fmaxf(ly, hy)), fminf(fmaxf(lz, hz), tlim));
    // the padded boxes make a relative slack of a few ulps harmless
    bool hit = ref != kEmptyChild && tn <= tf * 1.0000005f;
    return hit ? ((__float_as_uint(tn) & ~3u) | c) : ~0u;
}

__device__ __forceinline__ uint32_t child_key(float lox, float loy, float loz, float hix, float hiy, float hiz,
                                              int32_t ref, const RayPre &r, f3 oi, float tlim, uint32_t c)
{
    return key_from_t(fmaf(lox, r.inv.x, -oi.x), fmaf(hix, r.inv.x, -oi.x), fmaf(loy, r.inv.y, -oi.y),
                      fmaf(hiy, r.inv.y, -oi.y), fmaf(loz, r.inv.z, -oi.z), fmaf(hiz, r.inv.z, -oi.z), ref, tlim, c);
}

// the four children of a quantised node: plane distances as q s + b per axis,
// with s = grid step / direction and b = (corner - origin) / direction
__device__ __forceinline__ void qnode_keys(const QNode &n, const RayPre &r, float tlim, uint32_t k[4], int32_t ref[4])
{
    const float sx = __uint_as_float((n.w0.w & 0xffu) << 23) * r.inv.x;
    const float sy = __uint_as_float(((n.w0.w >> 8) & 0xffu) << 23) * r.inv.y;
    const float sz = __uint_as_float(((n.w0.w >> 16) & 0xffu) << 23) * r.inv.z;
    const float bx = (__uint_as_float(n.w0.x) - r.o.x) * r.inv.x;
    const float by = (__uint_as_float(n.w0.y) - r.o.y) * r.inv.y;
    const float bz = (__uint_as_float(n.w0.z) - r.o.z) * r.inv.z;
    ref[0] = (int32_t)n.w2.z;
    ref[1] = (int32_t)n.w2.w;
    ref[2] = (int32_t)n.w3.x;
    ref[3] = (int32_t)n.w3.y;
#pragma unroll
    for (uint32_t c = 0; c < 4; ++c) {
        const uint32_t sh = 8 * c;
        const float lx = fmaf((float)((n.w1.x >> sh) & 0xffu), sx, bx), hx = fmaf((float)((n.w1.w >> sh) & 0xffu), sx, bx);
        const float ly = fmaf((float)((n.w1.y >> sh) & 0xffu), sy, by), hy = fmaf((float)((n.w2.x >> sh) & 0xffu), sy, by);
        const float lz = fmaf((float)((n.w1.z >> sh) & 0xffu), sz, bz), hz = fmaf((float)((n.w2.y >> sh) & 0xffu), sz, bz);
        k[c] = key_from_t(lx, hx, ly, hy, lz, hz, ref[c], tlim, c);
    }
}

__device__ __forceinline__ void cswap(uint32_t &a, uint32_t &b)
{
    uint32_t lo = min(a, b), hi = max(a, b);
    a = lo;
    b = hi;
}

__device__ __forceinline__ int32_t child_ref(const int4 &ref, uint32_t c)
{
    return c == 0 ? ref.x : (c == 1 ? ref.y : (c == 2 ? ref.z : ref.w));
}

struct HitRec {
    float t, b1, b2;
    uint32_t tri;   // BVH-order index
    uint32_t id;    // input id (tie-break)
    uint32_t nodes, tests;  // traversal work: node fetches, triangle tests
    uint32_t depth;         // deepest traversal stack (DEPTH = true only)
};

// sum of a per-lane count over the wave (every lane active): within each
// row of 16 lanes by DPP moves (pairs and quads by quad permutes, then the
// half-row and row mirrors, each lane adding its image), then the four row
// sums read by the scalar unit -- no LDS round trips
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm 1, 0, 3, 2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm 2, 3, 0, 1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
           (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

// sum a per-lane count over the wave and add it to a 64-bit counter once
// (called with every lane of the wave active)
__device__ __forceinline__ void wave_count(unsigned long long *ctr, uint32_t v)
{
    v = wave_sum_u32(v);
    if (__lane_id() == 0 && v) atomicAdd(ctr, (unsigned long long)v);
}

// Closest hit (ANY = false) or occlusion (ANY = true) through the 4-wide BVH
// (Sec. 2.3: watertight traversal). At each node the four slab tests give
// sort keys; a 5-comparator network orders them, the nearest hit child is
// visited next and the others are pushed farthest first. The stack keeps
// kShortStack entries per thread in LDS, laid out [entry][thread] (bank-
// conflict free), and spills deeper entries to a per-thread global area
// (stride gs) sized by the host for the tree's depth (at most 3 pushes per
// level). Children are culled against the current closest t with a closed
// interval, so the result does not depend on the visiting order.
//
// With TOP, the nodes below F.top_nodes (the tree's top levels) come from the
// block's copy in LDS (`top`, filled by stage_top) instead of global memory:
// every ray starts at the root, so these few nodes are fetched by every ray
// and their copy in LDS takes them off the chain of dependent global loads.
//
// Inner nodes and leaves are processed in separate loops so that a wave runs
// either kind of work with most lanes active: a lane that reaches a leaf
// postpones it and keeps descending, and the wave leaves the node loop only
// when a vote (ballot over the lanes still in it) finds that every one of them
// holds a leaf; then the postponed leaves, and any leaves that follow them on
// the stack, are tested. Postponing only delays the updates of the closest t,
// which cull later children, so the hit is the same.
template <bool ANY, bool QN, bool DEPTH = false, bool TOP = false>
__device__ bool traverse(const Frame &F, const RayPre &r, float tmax, HitRec &h, int *stk, int *gstk, size_t gs,
                         const QNode *top = nullptr)
{
    h.t = tmax;
    h.tri = kNoHit;
    h.id = kNoHit;
    h.nodes = 0;
    h.tests = 0;
    h.depth = 0;
    int sp = 0;
    const int step = (int)blockDim.x;
    const f3 oi = r.o * r.inv;
    // the empty stack pops a reference no child carries
    constexpr int32_t kDone = kEmptyChild;
    auto push = [&](int v) {
        if (sp < (int)kShortStack) stk[sp * step] = v;
        else gstk[(sp - kShortStack) * gs] = v;
        ++sp;
        if (DEPTH) h.depth = max(h.depth, (uint32_t)sp);
    };
    auto pop = [&]() -> int32_t {
        if (sp == 0) return kDone;
        --sp;
        return sp < (int)kShortStack ? stk[sp * step] : gstk[(sp - kShortStack) * gs];
    };
    int32_t ref = 0;       // next inner node (>= 0) or leaf (< 0, not kDone), or kDone
    int32_t leaf = 0;      // the postponed leaf, valid while has_leaf
    bool has_leaf = false;
    while (ref != kDone) {
        while (ref >= 0) {
            ++h.nodes;
            uint32_t k0, k1, k2, k3;
            int4 nref;
            if (QN) {
                const QNode n = (TOP && (uint32_t)ref < F.top_nodes) ? top[ref] : F.qnodes[ref];
                uint32_t k[4];
                int32_t rf[4];
                qnode_keys(n, r, h.t, k, rf);
                k0 = k[0];
                k1 = k[1];
                k2 = k[2];
                k3 = k[3];
                nref = make_int4(rf[0], rf[1], rf[2], rf[3]);
            } else {
                const Node n = F.nodes[ref];
                k0 = child_key(n.lox.x, n.loy.x, n.loz.x, n.hix.x, n.hiy.x, n.hiz.x, n.ref.x, r, oi, h.t, 0);
                k1 = child_key(n.lox.y, n.loy.y, n.loz.y, n.hix.y, n.hiy.y, n.hiz.y, n.ref.y, r, oi, h.t, 1);
                k2 = child_key(n.lox.z, n.loy.z, n.loz.z, n.hix.z, n.hiy.z, n.hiz.z, n.ref.z, r, oi, h.t, 2);
                k3 = child_key(n.lox.w, n.loy.w, n.loz.w, n.hix.w, n.hiy.w, n.hiz.w, n.ref.w, r, oi, h.t, 3);
                nref = n.ref;
            }
            cswap(k0, k1);
            cswap(k2, k3);
            cswap(k0, k2);
            cswap(k1, k3);
            cswap(k1, k2);
            if (k0 != ~0u) {
                if (k3 != ~0u) push(child_ref(nref, k3 & 3u));
                if (k2 != ~0u) push(child_ref(nref, k2 & 3u));
                if (k1 != ~0u) push(child_ref(nref, k1 & 3u));
                ref = child_ref(nref, k0 & 3u);
            } else {
                ref = pop();
            }
            if (ref < 0 && ref != kDone && !has_leaf) {
                leaf = ref;
                has_leaf = true;
                ref = pop();
            }
            if (__ballot(!has_leaf) == 0ull) break;
        }
        while (has_leaf) {
            const uint32_t payload = ~(uint32_t)leaf;
            const uint32_t first = payload >> 3, cnt = (payload & 7u) + 1u;
            for (uint32_t k = 0; k < cnt; ++k) {
                const Tri tr = F.tris[first + k];
                float t, b1, b2;
                ++h.tests;
                if (!tri_test(r, tr.v0, tr.v1, tr.v2, tmax, t, b1, b2)) continue;
                if (ANY) {
                    h.tri = first + k;
                    return true;
                }
                const uint32_t id = fbits(tr.v1.w);
                if (t < h.t || (t == h.t && id < h.id)) {
                    h.t = t;
                    h.b1 = b1;
                    h.b2 = b2;
                    h.tri = first + k;
                    h.id = id;
                }
            }
            // a leaf that follows on the stack is tested right away
            if (ref < 0 && ref != kDone) {
                leaf = ref;
                ref = pop();
            } else {
                has_leaf = false;
            }
        }
    }
    return h.tri != kNoHit;
}

template <bool ANY>
__device__ bool brute_force(const Frame &F, const RayPre &r, float tmax, HitRec &h)
{
    h.t = tmax;
    h.tri = kNoHit;
    h.id = kNoHit;
    for (uint32_t k = 0; k < F.num_tris; ++k) {
        const Tri tr = F.tris[k];
        float t, b1, b2;
        if (!tri_test(r, tr.v0, tr.v1, tr.v2, tmax, t, b1, b2)) continue;
        if (ANY) {
            h.tri = k;
            return true;
        }
        uint32_t id = fbits(tr.v1.w);
        if (t < h.t || (t == h.t && id < h.id)) {
            h.t = t;
            h.b1 = b1;
            h.b2 = b2;
            h.tri = k;
            h.id = id;
        }
    }
    return h.tri != kNoHit;
}

// -------------------------------------------------------------- shading

__device__ __forceinline__ f3 emission_at(const Material &m, f3 x)
{
    f3 E = xyz(m.emission_flags);
    if (fbits(m.emission_flags.w) & 2u) E = E * (0.55f + 0.45f * sinf(2.0f * kPi * 4.0f * (x.x + x.z)));
    return E;
}

__device__ __forceinline__ float fresnel(float c)
{
    float m = fmaxf(0.0f, 1.0f - c);
    float m2 = m * m;
    return 0.04f + 0.96f * m2 * m2 * m;
}

__device__ __forceinline__ float ggx_D(float ch, float a2)
{
    float k = ch * ch * (a2 - 1.0f) + 1.0f;
    return a2 / (kPi * k * k);
}

__device__ __forceinline__ float ggx_lambda(float c, float a2)
{
    float c2 = c * c;
    return 0.5f * (-1.0f + sqrtf(1.0f + a2 * (1.0f - c2) / c2));
}

// probability of the specular lobe as realised by u < p on the 2^-24 grid
__device__ __forceinline__ float spec_prob(const Material &m, float co)
{
    float F = fresnel(co);
    float p = F / (F + (1.0f - F) * lum(xyz(m.albedo_rough)));
    p = fminf(0.9f, fmaxf(0.1f, p));
    return ceilf(p * 16777216.0f) * 0x1p-24f;
}

// f (no cosine) and sampling pdf for reflection on the side of n (n . wo > 0)
__device__ void bsdf_eval(const Material &m, f3 n, f3 wo, f3 wi, f3 &f, float &pdf)
{
    float co = dot(n, wo), ci = dot(n, wi);
    f = mk(0.f, 0.f, 0.f);
    pdf = 0.0f;
    if (co <= 0.0f || ci <= 0.0f) return;
    f3 rho = xyz(m.albedo_rough);
    if (!(fbits(m.emission_flags.w) & 1u)) {
        f = rho * kInvPi;
        pdf = ci * kInvPi;
        return;
    }
    float a = m.albedo_rough.w, a2 = a * a;
    f3 h = normalize(wo + wi);
    float D = ggx_D(dot(n, h), a2);
    float lo = ggx_lambda(co, a2), li = ggx_lambda(ci, a2);
    float spec = D * fresnel(dot(wo, h)) / ((1.0f + lo + li) * 4.0f * co * ci);
    float kd = (1.0f - fresnel(co)) * (1.0f - fresnel(ci)) * kInvPi;
    f = mk(spec, spec, spec) + rho * kd;
    float ps = spec_prob(m, co);
    pdf = ps * D / ((1.0f + lo) * 4.0f * co) + (1.0f - ps) * ci * kInvPi;
}

// orthonormal basis around unit n (Duff et al. 2017)
__device__ __forceinline__ void onb(f3 n, f3 &b1, f3 &b2)
{
    float s = copysignf(1.0f, n.z);
    float a = -1.0f / (s + n.z);
    float b = n.x * n.y * a;
    b1 = mk(1.0f + s * n.x * n.x * a, s * b, -s * n.x);
    b2 = mk(b, s + n.y * n.y * a, -n.y);
}

// sample wi: lobe by u3, direction by (u4, u5); false below the surface
__device__ bool bsdf_sample(const Material &m, f3 n, f3 wo, float u3, float u4, float u5, f3 &wi)
{
    f3 b1, b2;
    onb(n, b1, b2);
    float co = dot(n, wo);
    bool spec = (fbits(m.emission_flags.w) & 1u) && u3 < spec_prob(m, co);
    float r = sqrtf(u4);
    float s, c;
    sincosf(2.0f * kPi * u5, &s, &c);
    if (!spec) {
        float z = sqrtf(fmaxf(0.0f, 1.0f - u4));
        wi = b1 * (r * c) + b2 * (r * s) + n * z;
        return true;
    }
    // visible-normal sampling of GGX (Heitz 2018) in the local frame
    float a = m.albedo_rough.w;
    f3 vh = normalize(mk(a * dot(wo, b1), a * dot(wo, b2), co));
    float l2 = vh.x * vh.x + vh.y * vh.y;
    f3 T1 = l2 > 0.0f ? mk(-vh.y, vh.x, 0.0f) * (1.0f / sqrtf(l2)) : mk(1.0f, 0.0f, 0.0f);
    f3 T2 = cross(vh, T1);
    float t1 = r * c, t2 = r * s;
    float sh = 0.5f * (1.0f + vh.z);
    t2 = (1.0f - sh) * sqrtf(fmaxf(0.0f, 1.0f - t1 * t1)) + sh * t2;
    f3 nh = T1 * t1 + T2 * t2 + vh * sqrtf(fmaxf(0.0f, 1.0f - t1 * t1 - t2 * t2));
    f3 ne = normalize(mk(a * nh.x, a * nh.y, fmaxf(0.0f, nh.z)));
    f3 hw = b1 * ne.x + b2 * ne.y + n * ne.z;
    wi = hw * (2.0f * dot(wo, hw)) - wo;
    return dot(n, wi) > 0.0f;
}

// origin offset (Waechter and Binder 2019): trunc(256 n) ulps per coordinate,
// n / 65536 within 1/32 of the origin
__device__ __forceinline__ float offset1(float p, float n)
{
    int k = (int)(256.0f * n);
    float pi = __int_as_float(__float_as_int(p) + (p < 0.0f ? -k : k));
    return fabsf(p) < 1.0f / 32.0f ? p + n * (1.0f / 65536.0f) : pi;
}
__device__ __forceinline__ f3 offset_ray(f3 p, f3 n) { return mk(offset1(p.x, n.x), offset1(p.y, n.y), offset1(p.z, n.z)); }

__device__ __forceinline__ float mis2(float a, float b)
{
    // a^2 / (a^2 + b^2), safe for infinities and zeros
    if (!(a > 0.0f)) return 0.0f;
    float q = b / a;
    return 1.0f / (1.0f + q * q);
}

__device__ void env_texel_of(const Frame &F, f3 w, uint32_t &row, uint32_t &col)
{
    float th = acosf(fminf(1.0f, fmaxf(-1.0f, w.y)));
    float ph = atan2f(w.x, -w.z);
    if (ph < 0.0f) ph += 2.0f * kPi;
    int r = (int)floorf(th / kPi * (float)F.env_h);
    int c = (int)floorf(ph / (2.0f * kPi) * (float)F.env_w);
    row = (uint32_t)min(max(r, 0), (int)F.env_h - 1);
    col = (uint32_t)min(max(c, 0), (int)F.env_w - 1);
}

__device__ float4 env_lookup(const Frame &F, f3 w)
{
    uint32_t r, c;
    env_texel_of(F, w, r, c);
    return F.env_texel[(size_t)r * F.env_w + c];
}

// largest k in [0, n) with q[k] <= s (q[0] == 0, non-decreasing)
__device__ __forceinline__ uint32_t upper_search(const uint32_t *q, uint32_t n, uint32_t s)
{
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (q[mid] <= s) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Unit geometric normal of a triangle and twice its area, each product and
// sum rounded once: shading and the light tree's re-descent at a later
// vertex must see the same bits.
__device__ __forceinline__ f3 unit_normal(f3 a, f3 b, f3 c, float &area2)
{
#pragma clang fp contract(off)
    const f3 e1 = b - a, e2 = c - a;
    const f3 n = mk(e1.y * e2.z - e1.z * e2.y, e1.z * e2.x - e1.x * e2.z, e1.x * e2.y - e1.y * e2.x);
    area2 = sqrtf((n.x * n.x + n.y * n.y) + n.z * n.z);
    const float inv = 1.0f / area2;
    return mk(n.x * inv, n.y * inv, n.z * inv);
}

// ------------------------------------------------------------ light tree
//
// Selection of a triangle light through the hierarchy of Sec. 2.1.1. A node's
// importance at a shading point x with normal n is its flux towards the
// emission region holding the direction from its centre to x, times an upper
// bound of the cosine at x over its bounding sphere, over max(d^2, r^2); each
// step rounds once, so the choice does not depend on the compiler's fusing.
__device__ float lt_importance(const LtNode *nd, f3 x, f3 n)
{
#pragma clang fp contract(off)
    const float4 sp = nd->sphere;
    const float dx = sp.x - x.x, dy = sp.y - x.y, dz = sp.z - x.z;
    const float d2 = (dx * dx + dy * dy) + dz * dz;
    const float r = sp.w, r2 = r * r;
    // region of the emission direction x - c: dominant axis (ties to the
    // lower axis) and its sign
    const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    int k = 0;
    float m = ax, ek = -dx;
    if (ay > m) {
        k = 1;
        m = ay;
        ek = -dy;
    }
    if (az > m) {
        k = 2;
        ek = -dz;
    }
    const float flux = nd->flux[2 * k + (ek < 0.0f ? 1 : 0)];
    float cosx = 1.0f;
    if (d2 > r2) {
        const float d = sqrtf(d2);
        const float sinb = r / d;
        const float cosb = sqrtf(1.0f - sinb * sinb);
        const float cosa = ((n.x * dx + n.y * dy) + n.z * dz) / d;
        if (cosa < cosb) {
            const float sina = sqrtf(fmaxf(0.0f, 1.0f - cosa * cosa));
            cosx = fmaxf(0.0f, cosa * cosb + sina * sinb);
        }
    }
    return flux * cosx / fmaxf(d2, r2);
}

// probability of the first child of the pair at `l`, in 24 bits, within [1/16, 15/16]
__device__ uint32_t lt_left_q(const Frame &F, int32_t l, f3 x, f3 n)
{
#pragma clang fp contract(off)
    const float el = lt_importance(F.lt_nodes + l, x, n), er = lt_importance(F.lt_nodes + l + 1, x, n);
    const float sum = el + er;
    float p = (sum > 0.0f && isfinite(sum)) ? el / sum : 0.5f;
    p = fminf(fmaxf(p, 0.0625f), 0.9375f);
    return (uint32_t)(p * 16777216.0f + 0.5f);
}

// floor(R q / 2^24) exactly (R < 2^63, q <= 2^24)
__device__ __forceinline__ uint64_t lt_split(uint64_t R, uint32_t q)
{
    return (R >> 24) * q + (((R & 0xFFFFFFull) * q) >> 24);
}

// the first child's share of an interval of size R, kept inside [1, R - 1]
__device__ __forceinline__ uint64_t lt_cut(uint64_t R, uint32_t q)
{
    const uint64_t T = lt_split(R, q);
    return T < 1 ? 1 : (T > R - 1 ? R - 1 : T);
}

// Emitter chosen by the 63-bit sample S: the descent narrows [0, 2^63) to
// the chosen leaf, whose cumulative weights split what is left. size = the
// emitter's interval, its selection probability times 2^63.
__device__ uint32_t lt_sample(const Frame &F, uint64_t S, f3 x, f3 n, uint64_t &size)
{
    uint64_t R = 1ull << 63;
    int32_t node = 0, l = F.lt_nodes[0].left;
    while (l >= 0) {
        const uint64_t T = lt_cut(R, lt_left_q(F, l, x, n));
        if (S < T) {
            R = T;
            node = l;
        } else {
            S -= T;
            R -= T;
            node = l + 1;
        }
        l = F.lt_nodes[node].left;
    }
    const uint32_t f = F.lt_nodes[node].first, c = F.lt_nodes[node].count;
    uint32_t j = 0;  // weights rise within a leaf: count the bounds at or below S
    for (uint32_t q = 1; q < c; ++q) j += S >= lt_split(R, F.lt_w[f + q]) ? 1u : 0u;
    const uint64_t a = lt_split(R, F.lt_w[f + j]);
    const uint64_t z = j + 1 < c ? lt_split(R, F.lt_w[f + j + 1]) : R;
    size = z - a;
    return F.lt_emit[f + j];
}

// the interval size of emitter e, by the same descent steered to its leaf
__device__ uint64_t lt_size_of(const Frame &F, uint32_t e, f3 x, f3 n)
{
    const uint32_t pos = F.lt_pos[e];
    uint64_t R = 1ull << 63;
    int32_t node = 0, l = F.lt_nodes[0].left;
    while (l >= 0) {
        const uint64_t T = lt_cut(R, lt_left_q(F, l, x, n));
        if (pos < F.lt_nodes[l + 1].first) {
            R = T;
            node = l;
        } else {
            R -= T;
            node = l + 1;
        }
        l = F.lt_nodes[node].left;
    }
    const uint32_t c = F.lt_nodes[node].count, j = pos - F.lt_nodes[node].first;
    const uint64_t a = lt_split(R, F.lt_w[pos]);
    const uint64_t z = j + 1 < c ? lt_split(R, F.lt_w[pos + 1]) : R;
    return z - a;
}

// the oriented normal of the previous vertex (its triangle and side bits, as
// kept in the ray direction's spare word), rounded as shading rounded it there
__device__ __forceinline__ f3 prev_normal(const Frame &F, float bits)
{
    const uint32_t pv = fbits(bits);
    const Tri pt = F.tris[pv & 0x7fffffffu];
    float a2;
    const f3 n = unit_normal(xyz(pt.v0), xyz(pt.v1), xyz(pt.v2), a2);
    return (pv >> 31) ? n * -1.0f : n;
}

// ------------------------------------------------- environment pyramid
//
// Hierarchical sampling of the environment (Sec. 2.1.2): from the two halves
// of the sphere down to the texels, each step picks the child column by the
// columns' shares of intensity x solid angle, then the row within it, as
// 24-bit probabilities narrowing two 32-bit samples (u columns, v rows) as
// integer intervals; a texel's probability is exactly the product of its two
// final interval sizes over 2^64. With a normal bin, the top levels use the
// bin's cosine-weighted splits.
__device__ __forceinline__ uint32_t ep_nodes_above(uint32_t k)
{
    return (uint32_t)((2ull * ((1ull << (2 * k)) - 1)) / 3);
}

// normal bin: 16 x 16 cells of the octahedral map (+y up), each step rounded once
__device__ uint32_t ep_bin(f3 n)
{
#pragma clang fp contract(off)
    const float a = (fabsf(n.x) + fabsf(n.y)) + fabsf(n.z);
    float px = n.x / a, pz = n.z / a;
    if (n.y < 0.0f) {
        const float fx = (1.0f - fabsf(pz)) * (px >= 0.0f ? 1.0f : -1.0f);
        const float fz = (1.0f - fabsf(px)) * (pz >= 0.0f ? 1.0f : -1.0f);
        px = fx;
        pz = fz;
    }
    const int i = min(max((int)floorf((px + 1.0f) * 8.0f), 0), 15);
    const int j = min(max((int)floorf((pz + 1.0f) * 8.0f), 0), 15);
    return (uint32_t)(j * 16 + i);
}

// the first child's part of an interval of size R for a 24-bit share q
// (0 and 2^24: a child without weight gets nothing)
__device__ __forceinline__ uint64_t ep_split(uint64_t R, uint32_t q)
{
    if (q == 0) return 0;
    if (q >= (1u << 24)) return R;
    const uint64_t T = (R >> 24) * q + (((R & 0xFFFFFFull) * q) >> 24);
    return R < 2 ? T : (T < 1 ? 1 : (T > R - 1 ? R - 1 : T));
}

// Sample the pyramid with (u, v), or with `steer` follow texel (row, col);
// bin < 0 uses the shared splits only. Returns the texel and the final
// intervals (sizes ru, rv; offsets su, sv inside them).
__device__ void ep_descend(const Frame &F, int bin, uint32_t u, uint32_t v, bool steer, uint32_t &row,
                           uint32_t &col, uint64_t &ru, uint64_t &su, uint64_t &rv, uint64_t &sv)
{
    const uint32_t m = F.ep_m;
    const uint4 *oq = bin >= 0 ? F.ep_oq + (size_t)bin * F.ep_stride : nullptr;
    ru = 1ull << 32;
    su = u;
    rv = 1ull << 32;
    sv = v;
    uint64_t T = ep_split(ru, oq ? oq[0].x : F.ep_root);
    const bool right = steer ? ((col >> m) & 1u) != 0 : su >= T;
    if (right) {
        su -= T;
        ru -= T;
    } else {
        ru = T;
    }
    uint32_t x = right ? 1u : 0u, y = 0;
    for (uint32_t k = 0; k < m; ++k) {
        const size_t at = (size_t)ep_nodes_above(k) + (size_t)y * (2u << k) + x;
        const uint4 q = (oq && k < F.ep_top) ? oq[1 + at] : F.ep_q[at];
        T = ep_split(ru, q.x);
        const bool cx = steer ? ((col >> (m - 1 - k)) & 1u) != 0 : su >= T;
        if (cx) {
            su -= T;
            ru -= T;
        } else {
            ru = T;
        }
        T = ep_split(rv, cx ? q.z : q.y);
        const bool cy = steer ? ((row >> (m - 1 - k)) & 1u) != 0 : sv >= T;
        if (cy) {
            sv -= T;
            rv -= T;
        } else {
            rv = T;
        }
        x = 2 * x + (cx ? 1u : 0u);
        y = 2 * y + (cy ? 1u : 0u);
    }
    row = y;
    col = x;
}

// solid-angle density of a texel of row `row` chosen with interval sizes ru, rv
__device__ __forceinline__ float ep_pdf(const Frame &F, uint32_t row, uint64_t ru, uint64_t rv)
{
#pragma clang fp contract(off)
    const float omega = (2.0f * kPi / (float)F.env_w) * (F.env_cos[row] - F.env_cos[row + 1]);
    return ((float)ru * (float)rv * 0x1p-64f) / omega;
}

// ---------------------------------------------------------------- kernels

__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_f64(double *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// Start of a batch: clear the lane's counters; the batch that starts a pass
// (its first pixel chunk) latches the caller's abort word, and every chunk of
// the pass renders nothing when it was set, so a pass is done whole or not at all.
__global__ void k_batch_begin(Pool P, const uint32_t *abort_word, uint32_t first_chunk)
{
    const uint32_t t = threadIdx.x;
    if (t < kCounters && t != kPassLatch && t != kSkip) P.counters[t] = 0;
    if (t == 0) {
        if (first_chunk)
            P.counters[kPassLatch] =
                abort_word ? __hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : 0u;
        P.counters[kSkip] = P.counters[kPassLatch];
    }
}

// Position q of a whole frame in 8 x 8 tile order -> row-major pixel. Bands of
// eight rows follow each other; inside a band the tiles go left to right and a
// tile's pixels row by row; the last band and the last tile of a band are
// narrower when H or W is not a multiple of 8. A bijection of [0, W H), so a
// wave's 64 camera rays leave one compact block of the image.
__device__ __forceinline__ uint32_t tile_pixel(uint32_t q, uint32_t W, uint32_t H)
{
    const uint32_t band = q / (8u * W);
    const uint32_t r = q - band * 8u * W;
    const uint32_t hy = min(8u, H - 8u * band);
    const uint32_t tx = min(r / (8u * hy), (W - 1u) / 8u);
    const uint32_t rem = r - tx * 8u * hy;
    const uint32_t tw = min(8u, W - 8u * tx);
    const uint32_t y = rem / tw;
    return (8u * band + y) * W + 8u * tx + (rem - y * tw);
}

// Slots of a batch -> (position q in [0, npix), pass j in [0, npass)). A
// whole-frame batch takes its positions in 8 x 8 tile order in groups of 64
// (one wave) and lays out each group's npass passes next to each other: slot
// = group * 64 npass + j * 64 + lane, the last group narrower when 64 does not
// divide npix. Launches that stride over the slots then work on one band of
// the image at a time, across every pass of the batch. Pixel chunks of a pass
// larger than the pool (npass = 1) keep scanline order.
struct SlotMap {
    uint32_t full;  // complete groups of 64 positions
    uint32_t tail;  // positions in the last, narrower group
    uint32_t npass;
};

__device__ __forceinline__ SlotMap slot_map(uint32_t npix, uint32_t npass)
{
    return {npix / 64u, npix % 64u, npass};
}

__device__ __forceinline__ uint32_t slot_of(const SlotMap &m, uint32_t q, uint32_t j)
{
    const uint32_t g = q / 64u, lane = q % 64u;
    const uint32_t w = g < m.full ? 64u : m.tail;
    return g * 64u * m.npass + j * w + lane;
}

__device__ __forceinline__ void position_of(const SlotMap &m, uint32_t s, uint32_t &q, uint32_t &j)
{
    const uint32_t g = s / (64u * m.npass);
    const uint32_t r = s - g * 64u * m.npass;
    const uint32_t w = g < m.full ? 64u : m.tail;
    j = r / w;
    q = g * 64u + (r - j * w);
}

__device__ __forceinline__ bool whole_frame(const Frame &F, uint32_t npix) { return npix == F.W * F.H; }

// The camera path with id `pid` of a batch of npass passes over npix pixels
// (pid -> (position, pass) as above; pixel tile_pixel(position) of a whole
// frame, else pix0 + position), started in state slot s: its camera ray,
// unit throughput, its Halton index, and zero radiance at rad[pid].
__device__ __forceinline__ void start_path(const Frame &F, const Pool &P, uint32_t s, uint32_t pid, uint32_t pix0,
                                           uint32_t npix, uint32_t npass, uint64_t pass0)
{
    uint32_t pl, j, p;
    if (whole_frame(F, npix)) {
        position_of(slot_map(npix, npass), pid, pl, j);
        p = tile_pixel(pl, F.W, F.H);
    } else {
        pl = pid % npix;
        j = pid / npix;
        p = pix0 + pl;
    }
    uint32_t px = p % F.W, py = p / F.W;
    uint64_t i = pixel_index(F, px, py, pass0 + j);
    const float u0 = u24(sample_bits(F, i, 0, 0)), u1 = u24(sample_bits(F, i, 1, 0));
    float fx = (float)px + u0, fy = (float)py + u1;
    if (F.gauss_filter) {
        // filter importance sampling (Appendix A.1): Gaussian of sigma 1/2 pixel
        // around the centre, untruncated, by Box-Muller (1 - u0 is exact and > 0)
        const float r = 0.5f * sqrtf(-2.0f * logf(1.0f - u0));
        float sn, cs;
        sincospif(2.0f * u1, &sn, &cs);
        fx = (float)px + 0.5f + r * cs;
        fy = (float)py + 0.5f + r * sn;
    }
    float sx = (2.0f * fx / (float)F.W - 1.0f) * F.cam.tan_half * F.cam.aspect;
    float sy = (1.0f - 2.0f * fy / (float)F.H) * F.cam.tan_half;
    f3 fwd = mk(F.cam.fwd[0], F.cam.fwd[1], F.cam.fwd[2]);
    f3 rt = mk(F.cam.right[0], F.cam.right[1], F.cam.right[2]);
    f3 up = mk(F.cam.up[0], F.cam.up[1], F.cam.up[2]);
    f3 d = normalize(fwd + (rt * sx + up * sy));
    state::quantise_dir(F, d.x, d.y, d.z);
    P.ray_o[s] = make_float4(F.cam.eye[0], F.cam.eye[1], F.cam.eye[2], INFINITY);
    state::store_dir(F, P, s, f4(d, 0.0f));
    state::store_thr(F, P, s, make_float4(1.0f, 1.0f, 1.0f, 0.0f));
    P.rad[pid] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    P.idx[s] = i;
}

// camera rays for slots [0, n), n = npix npass, one path per slot
__global__ __launch_bounds__(kBlock) void k_generate(Frame F, Pool P, uint32_t pix0, uint32_t npix, uint64_t pass0,
                                                     uint32_t n)
{
    if (P.counters[kSkip]) return;  // aborted: no paths, every later stage sees empty queues
    uint32_t s = blockIdx.x * kBlock + threadIdx.x;
    if (s == 0) P.counters[1] = n;
    if (s >= n) return;
    start_path(F, P, s, s, pix0, npix, n / npix, pass0);
    P.q_ext[1][s] = s;
}

// the tree's first F.top_nodes nodes into the block's LDS copy; every thread
// of the block calls it (it ends with the block barrier)
__device__ __forceinline__ void stage_top(const Frame &F, QNode *top)
{
    const uint4 *src = (const uint4 *)F.qnodes;
    uint4 *dst = (uint4 *)top;
    for (uint32_t i = threadIdx.x; i < 4 * F.top_nodes; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

// closest hit for the extension rays of queue q_ext[qsel] (counters[cnt]
// entries: the queue of one depth, or of one iteration when regenerating);
// the grid holds twice what is resident on the chip (a block that finishes
// early makes room for one that has not started) and strides over the queue
template <bool QN>
__global__ __launch_bounds__(kBlock, 8) void k_trace(Frame F, Pool P, uint32_t cnt, uint32_t qsel)
{
    __shared__ int stk[kShortStack * kBlock];
    __shared__ QNode top[QN ? kTopNodes : 1];
    const uint32_t n = P.counters[cnt];
    // blocks without rays leave before staging (uniform per block)
    if ((size_t)blockIdx.x * kBlock >= n) return;
    if (QN) stage_top(F, top);
    const uint32_t *q = P.q_ext[qsel];
    int *gstk = P.gstack + (size_t)(blockIdx.x * kBlock + threadIdx.x);
    uint32_t nodes = 0, tests = 0;
    for (uint32_t base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        uint32_t i = base + threadIdx.x;
        if (i >= n) break;
        uint32_t slot = q[i];
        float4 o = P.ray_o[slot], d = state::load_dir(F, P, slot);
        RayPre r = prepare(xyz(o), xyz(d));
        HitRec h;
        traverse<false, QN, false, QN>(F, r, o.w, h, stk + threadIdx.x, gstk, P.trav_threads, top);
        state::store_hit(F, P, slot, make_float4(h.t, ubits(h.tri), h.b1, h.b2));
        nodes += h.nodes;
        tests += h.tests;
    }
    wave_count(&P.stats[4], nodes);
    wave_count(&P.stats[5], tests);
}

// occlusion test of the counters[cnt] shadow rays of a depth (or iteration);
// add unoccluded contributions to the radiance of their paths
template <bool QN>
__global__ __launch_bounds__(kBlock) void k_shadow(Frame F, Pool P, uint32_t cnt)
{
    __shared__ int stk[kShortStack * kBlock];
    __shared__ QNode top[QN ? kTopNodes : 1];
    const uint32_t n = P.counters[cnt];
    if ((size_t)blockIdx.x * kBlock >= n) return;
    if (QN) stage_top(F, top);
    int *gstk = P.gstack + (size_t)(blockIdx.x * kBlock + threadIdx.x);
    uint32_t nodes = 0, tests = 0;
    for (uint32_t base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        uint32_t i = base + threadIdx.x;
        if (i >= n) break;
        float4 o = P.sh_o[i], d = P.sh_d[i];
        RayPre r = prepare(xyz(o), xyz(d));
        HitRec h;
        bool occluded = traverse<true, QN, false, QN>(F, r, o.w, h, stk + threadIdx.x, gstk, P.trav_threads, top);
        nodes += h.nodes;
        tests += h.tests;
        if (!occluded) {
            uint32_t rs = fbits(d.w);
            float4 c = P.sh_c[i];
            float4 L = P.rad[rs];
            P.rad[rs] = make_float4(L.x + c.x, L.y + c.y, L.z + c.z, L.w);
            uint32_t rec = fbits(c.w);
            if (rec != kNoHit) F.guide.rec[(size_t)rec * kRecF4 + 5] = make_float4(c.x, c.y, c.z, 0.0f);
        }
    }
    wave_count(&P.stats[6], nodes);
    wave_count(&P.stats[7], tests);
}

// which vertices leave a training record: a hash of the path's sample index
// and the depth (splitmix64 finaliser), uniform over the batch
__device__ __forceinline__ uint32_t rec_hash(uint64_t idx, uint32_t v)
{
    uint64_t z = idx * 0x9E3779B97F4A7C15ull + (uint64_t)v * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return (uint32_t)((z ^ (z >> 31)) >> 32);
}

// what shading one path vertex produces besides the slot's own state: a
// shadow ray with its pending contribution, whether the path continues, and
// a training record
struct ShadeOut {
    bool alive, shadow, record;
    float4 sh_o, sh_d, sh_c;
    float4 rec[5];
};

// emission with MIS, next-event estimation, BSDF (or guide) sampling and
// roulette at vertex v of the path in `slot` (its hit already traced): updates
// the slot's ray and throughput and the path's radiance rad[rs] (rs = the
// path's id in the batch; the NEE contribution stays pending in o.sh_c until
// its shadow ray is traced). mix_row: the vertex's packed mixture (a guided
// vertex), or null (BSDF sampling alone)
__device__ __forceinline__ void shade_slot(const Frame &F, const Pool &P, uint32_t v, uint32_t slot, uint32_t rs,
                                           ShadeOut &o, const uint4 *mix_row = nullptr)
{
    const uint32_t base_dim = 2 + 8 * (v - 1);
    o.alive = o.shadow = o.record = false;
    float4 hv = state::load_hit(F, P, slot);
    const float4 d4 = state::load_dir(F, P, slot);
    f3 d = xyz(d4);
    float4 T4 = state::load_thr(F, P, slot);
    f3 T = xyz(T4);
    float prev_pdf = T4.w;
    f3 L = xyz(P.rad[rs]);
    uint32_t tri = fbits(hv.y);
    if (tri == kNoHit) {
        if (F.env_w && (v == 1 || F.mode != 2)) {
            uint32_t er, ec;
            env_texel_of(F, d, er, ec);
            const float4 e = F.env_texel[(size_t)er * F.env_w + ec];
            float pe = e.w;
            if (v > 1 && F.mode == 0 && F.env_pyramid) {
                // the pyramid's density of this texel from the previous vertex
                const int bin = F.env_pyramid == 2 ? (int)ep_bin(prev_normal(F, d4.w)) : -1;
                uint64_t ru, su, rv, sv;
                ep_descend(F, bin, 0u, 0u, true, er, ec, ru, su, rv, sv);
                pe = ep_pdf(F, er, ru, rv);
            }
            float w = (v > 1 && F.mode == 0) ? mis2(prev_pdf, F.p_env * pe) : 1.0f;
            L = L + T * xyz(e) * w;
        }
    } else {
        const Tri tr = F.tris[tri];
        const Material m = F.mats[fbits(tr.v0.w)];
        f3 a = xyz(tr.v0), b = xyz(tr.v1), c = xyz(tr.v2);
        f3 x = a + ((b - a) * hv.z + (c - a) * hv.w);
        float area2;
        f3 ng = unit_normal(a, b, c, area2);
        float dn = dot(d, ng);
        bool front = dn < 0.0f;
        uint32_t em = fbits(tr.v2.w);
        if (front && em != kNoHit && !(v > 1 && F.mode == 2)) {
            f3 Le = emission_at(m, x);
            float w = 1.0f;
            if (v > 1 && F.mode == 0) {
                float pe;
                if (F.light_tree) {
                    // the tree's probability of this emitter from the previous
                    // vertex: its ray origin and oriented normal, as its NEE saw them
                    const uint64_t z = lt_size_of(F, em, xyz(P.ray_o[slot]), prev_normal(F, d4.w));
                    pe = (1.0f - F.p_env) * ((float)z * 0x1p-63f);
                } else {
                    pe = F.emit_pmf[em];
                }
                float pl = pe / (0.5f * area2) * hv.x * hv.x / (-dn);
                w = mis2(prev_pdf, pl);
            }
            L = L + T * Le * w;
        }
        bool scatters = maxc(xyz(m.albedo_rough)) > 0.0f || (fbits(m.emission_flags.w) & 1u);
        if (v < F.max_depth && scatters) {
            f3 nn = front ? ng : ng * -1.0f;
            f3 wo = d * -1.0f;
            f3 xo = offset_ray(x, nn);
            uint64_t idx = P.idx[slot];
            // learned proposal: this vertex's mixture (given only at the guided
            // vertices, and only with alpha > 0)
            const bool guided = mix_row != nullptr;
            guide::MixRef mix{nullptr, 0.0f};
            guide::MixCoef mc{};
            if (guided) {
                mix = guide::mix_ref(mix_row);
                mc = guide::mixture_coef(mix);
            }
            const float alpha = F.guide.alpha;
            // next-event estimation
            if (F.mode != 1 && (F.num_emit || F.env_w)) {
                uint32_t s0 = sample_bits(F, idx, base_dim + 0, F.scramble);
                bool use_env = F.env_w != 0;
                uint64_t rr = s0, R = 1ull << 32;
                if (F.env_w && F.num_emit) {
                    use_env = s0 < 0x80000000u;
                    rr = s0 - 0x80000000u;
                    R = 1ull << 31;
                }
                f3 wi, Le;
                float pl = 0.0f, tmax = INFINITY;
                bool ok = false;
                if (use_env) {
                    uint32_t s1 = sample_bits(F, idx, base_dim + 1, F.scramble);
                    uint32_t s2 = sample_bits(F, idx, base_dim + 2, F.scramble);
                    uint32_t row, col;
                    float fx, fy, pt = 0.0f;
                    if (F.env_pyramid) {
                        // pyramid: slot 2 narrows the columns, slot 1 the rows
                        const int bin = F.env_pyramid == 2 ? (int)ep_bin(nn) : -1;
                        uint64_t ru, su, rv, sv;
                        ep_descend(F, bin, s2, s1, false, row, col, ru, su, rv, sv);
                        fx = (float)su / (float)ru;
                        fy = (float)sv / (float)rv;
                        pt = ep_pdf(F, row, ru, rv);
                    } else {
                        row = upper_search(F.env_row, F.env_h, s1);
                        const uint32_t *cq = F.env_col + (size_t)row * F.env_w;
                        col = upper_search(cq, F.env_w, s2);
                        uint64_t r0 = F.env_row[row], r1 = row + 1 < F.env_h ? F.env_row[row + 1] : (1ull << 32);
                        uint64_t c0 = cq[col], c1 = col + 1 < F.env_w ? cq[col + 1] : (1ull << 32);
                        fy = (float)(s1 - r0) / (float)(r1 - r0);
                        fx = (float)(s2 - c0) / (float)(c1 - c0);
                    }
                    float ct = F.env_cos[row], cb = F.env_cos[row + 1];
                    float cth = ct + fy * (cb - ct);
                    float sth = sqrtf(fmaxf(0.0f, 1.0f - cth * cth));
                    float sp, cp;
                    sincosf(2.0f * kPi * ((float)col + fx) / (float)F.env_w, &sp, &cp);
                    wi = mk(sth * sp, cth, -sth * cp);
                    float4 e = F.env_texel[(size_t)row * F.env_w + col];
                    Le = xyz(e);
                    pl = F.p_env * (F.env_pyramid ? pt : e.w);
                    ok = pl > 0.0f;
                } else {
                    uint32_t s7 = sample_bits(F, idx, base_dim + 7, F.scramble);
                    uint32_t e;
                    float pe;
                    if (F.light_tree) {
                        // 63-bit sample: what slot 0 leaves after the environment
                        // choice (its top 31 bits without an environment), then slot 7
                        const uint64_t hi = F.env_w ? rr : (uint64_t)(s0 >> 1);
                        uint64_t z;
                        e = lt_sample(F, (hi << 32) | s7, xo, nn, z);
                        pe = (1.0f - F.p_env) * ((float)z * 0x1p-63f);
                    } else {
                        // rr < R <= 2^32 and num_emit < 2^27: the product fits 64 bits
                        uint32_t col =
                            (uint32_t)((rr * (uint64_t)F.num_emit) >> (R == (1ull << 31) ? 31 : 32));
                        e = (unsigned long long)s7 < F.alias_thr[col] ? col : F.alias_idx[col];
                        pe = F.emit_pmf[e];
                    }
                    const Tri lt = F.tris[F.emit_tri[e]];
                    float q1 = u24(sample_bits(F, idx, base_dim + 1, F.scramble));
                    float q2 = u24(sample_bits(F, idx, base_dim + 2, F.scramble));
                    float su = sqrtf(q1);
                    float b0 = 1.0f - su, bb1 = q2 * su, bb2 = su * (1.0f - q2);
                    f3 la = xyz(lt.v0), lb = xyz(lt.v1), lc = xyz(lt.v2);
                    f3 y = la * b0 + lb * bb1 + lc * bb2;
                    f3 nl = cross(lb - la, lc - la);
                    float la2 = length(nl);
                    nl = nl * (1.0f / la2);
                    f3 dv = y - xo;
                    float d2 = dot(dv, dv);
                    float dist = sqrtf(d2);
                    wi = dv * (1.0f / dist);
                    float cl = -dot(nl, wi);
                    if (cl > 0.0f) {
                        Le = emission_at(F.mats[fbits(lt.v0.w)], y);
                        pl = pe / (0.5f * la2) * d2 / cl;
                        ok = pl > 0.0f;
                        tmax = dist * (1.0f - 1e-4f);
                    }
                }
                if (ok) {
                    float ci = dot(nn, wi);
                    if (ci > 0.0f) {
                        f3 fb;
                        float pb;
                        bsdf_eval(m, nn, wo, wi, fb, pb);
                        if (guided) pb = alpha * guide::mixture_pdf(mix, mc, {wi.x, wi.y, wi.z}) + (1.0f - alpha) * pb;
                        float w = F.mode == 2 ? 1.0f : mis2(pl, pb);
                        f3 contrib = T * fb * Le * (ci * w / pl);
                        if (maxc(contrib) > 0.0f) {
                            o.shadow = true;
                            o.sh_o = f4(xo, tmax);
                            o.sh_d = f4(wi, ubits(rs));
                            o.sh_c = f4(contrib, 0.0f);
                        }
                    }
                }
            }
            // continue the path: slot 3 picks guide or BSDF (guide iff the 32-bit
            // sample < alpha 2^32) and, rescaled to [0, 2^32), the lobe; slots 4-5
            // the direction. The density is the one-sample mixture
            // alpha q + (1 - alpha) p_bsdf, so the estimator stays unbiased.
            uint32_t s3 = sample_bits(F, idx, base_dim + 3, F.scramble);
            bool use_guide = guided && s3 < F.guide.alpha_thr;
            uint32_t r3 = s3;
            if (guided) {
                uint64_t lo = use_guide ? 0ull : F.guide.alpha_thr;
                uint64_t range = use_guide ? F.guide.alpha_thr : (1ull << 32) - F.guide.alpha_thr;
                r3 = (uint32_t)((((uint64_t)s3 - lo) << 32) / range);
            }
            float u3 = u24(r3);
            float u4 = u24(sample_bits(F, idx, base_dim + 4, F.scramble));
            float u5 = u24(sample_bits(F, idx, base_dim + 5, F.scramble));
            f3 wi;
            bool ok;
            if (use_guide) {
                guide::V3 g = guide::mixture_sample(mix, u3, u4, u5);
                wi = mk(g.x, g.y, g.z);
                ok = dot(nn, wi) > 0.0f;
            } else {
                ok = bsdf_sample(m, nn, wo, u3, u4, u5, wi);
            }
            if (ok && F.compress) {
                // the direction the compressed state holds is the one sampled
                state::quantise_dir(F, wi.x, wi.y, wi.z);
                ok = dot(nn, wi) > 0.0f;
            }
            if (ok) {
                f3 fb;
                float pb;
                bsdf_eval(m, nn, wo, wi, fb, pb);
                if (guided) pb = alpha * guide::mixture_pdf(mix, mc, {wi.x, wi.y, wi.z}) + (1.0f - alpha) * pb;
                if (pb > 0.0f) {
                    f3 Tb = T;  // throughput before this vertex's scattering
                    T = T * fb * (dot(nn, wi) / pb);
                    if (maxc(T) > 0.0f) {
                        o.alive = true;
                        if (F.rr && v >= 3) {
                            float qq = fminf(0.95f, maxc(T));
                            qq = ceilf(qq * 16777216.0f) * 0x1p-24f;
                            float u6 = u24(sample_bits(F, idx, base_dim + 6, F.scramble));
                            if (u6 < qq) {
                                T = T * (1.0f / qq);
                                Tb = Tb * (1.0f / qq);
                            } else {
                                o.alive = false;
                            }
                        }
                        if (o.alive) {
                            P.ray_o[slot] = f4(xo, INFINITY);
                            state::store_dir(F, P, slot, f4(wi, ubits(tri | (front ? 0u : 0x80000000u))));
                            state::store_thr(F, P, slot, f4(T, pb));
                            if (F.guide.record && v <= F.guide.max_vertex &&
                                (F.guide.rec_thr == 0xffffffffu || rec_hash(idx, v) < F.guide.rec_thr)) {
                                // training record: (final - (now + this vertex's NEE)) /
                                // T_before is this sample's estimate f cos L_i / p of
                                // the scattering integral (roulette folded into T_before)
                                o.record = true;
                                o.rec[0] = f4(x, pb);
                                o.rec[1] = f4(wo, 0.0f);
                                o.rec[2] = f4(wi, ubits(rs));
                                o.rec[3] = f4(L, ubits(v));
                                o.rec[4] = f4(Tb, 0.0f);
                            }
                        }
                    }
                }
            }
        }
    }
    P.rad[rs] = f4(L, 0.0f);
}

// emission with MIS, next-event estimation, BSDF sampling and roulette at depth v
// (four blocks per CU: at most 128 VGPRs, four waves per SIMD, no spills)
// a shaded vertex's outputs: its training record, its shadow ray and its
// place in the next depth's queue (wave-aggregated appends)
__device__ __forceinline__ void shade_emit(const Frame &F, const Pool &P, uint32_t v, uint32_t slot, ShadeOut &o,
                                           uint32_t *qn, uint32_t *s_app)
{
    uint32_t rec_idx = kNoHit;
    const bool rec = F.guide.record && o.record;
    uint32_t pr, ps, pe;
    block_append3(&P.counters[127], rec, &P.counters[64 + v], o.shadow, &P.counters[v + 1], o.alive, s_app, pr, ps,
                  pe);
    if (F.guide.record) {
        if (rec && pr < F.guide.rec_cap) {
            float4 *r = F.guide.rec + (size_t)pr * kRecF4;
            r[0] = o.rec[0];
            r[1] = o.rec[1];
            r[2] = o.rec[2];
            r[3] = o.rec[3];
            r[4] = o.rec[4];
            r[5] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            rec_idx = pr;
        }
    }
    if (o.shadow) {
        o.sh_c.w = ubits(rec_idx);
        P.sh_o[ps] = o.sh_o;
        P.sh_d[ps] = o.sh_d;
        P.sh_c[ps] = o.sh_c;
    }
    if (o.alive) qn[pe] = slot;
}

__device__ __forceinline__ void shade_out_init(ShadeOut &o)
{
    // zero-initialised: the outputs stay in registers (no spills at 128 VGPRs)
    o.alive = o.shadow = o.record = false;
    o.sh_o = o.sh_d = o.sh_c = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int k = 0; k < 5; ++k) o.rec[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

__global__ __launch_bounds__(kShadeBlock, 4) void k_shade(Frame F, Pool P, uint32_t v)
{
    __shared__ uint32_t s_app[3 * (kAppendWaves + 1)];
    const uint32_t n = P.counters[v];
    const uint32_t *q = P.q_ext[v & 1];
    uint32_t *qn = P.q_ext[(v + 1) & 1];
    for (uint32_t base = blockIdx.x * kShadeBlock; base < n; base += gridDim.x * kShadeBlock) {
        uint32_t i = base + threadIdx.x;
        uint32_t slot = 0;
        ShadeOut o;
        shade_out_init(o);
        if (i < n) {
            slot = q[i];
            shade_slot(F, P, v, slot, slot, o);
        }
        shade_emit(F, P, v, slot, o, qn, s_app);
    }
}

// Shading of a guided vertex with the network's inference in the same
// launch: the block's weights in LDS, each wave's 64 mixtures computed on the
// matrix cores into LDS (packed, 80 bytes a row) and read there by the lane
// that shades the row -- the mixture never goes through HBM, and the hit and
// direction loads serve both. Blocks of 8 waves share one copy of the weights
// (69 KB of LDS a block, two blocks and 16 waves per CU, as many as the
// plain shading kernel keeps). A wave touches only its own 64 rows of the
// mixtures, so after the weights are staged the waves synchronise with
// themselves only. Blocks without rows leave before staging the weights
// (uniform per block, so the one block barrier is reached by all).
__global__ __launch_bounds__(kShadeGuidedBlock, kShadeGuidedWavesPerSIMD) void k_shade_guided(Frame F, Pool P, uint32_t v)
{
    __shared__ uint2 sfrag[kGuideFrags * 64];
    __shared__ __align__(16) float sbias[256];
    __shared__ uint4 smix[kShadeGuidedBlock * guide::kMixU4];
    __shared__ uint32_t s_app[3 * (kAppendWaves + 1)];
    const uint32_t n = P.counters[v];
    if ((size_t)blockIdx.x * kShadeGuidedBlock >= n) return;
    mlp::load_weights(F.guide.frag, F.guide.bias, sfrag, sbias);
    __syncthreads();
    const uint32_t *q = P.q_ext[v & 1];
    uint32_t *qn = P.q_ext[(v + 1) & 1];
    uint4 *wave_rows = smix + (threadIdx.x & ~63u) * guide::kMixU4;
    // the wave's rows are written by the lane pairs and read by their own
    // lanes: ordered within the wave (fences at wavefront scope and a wave
    // barrier, also before the next pass overwrites them)
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    for (uint32_t base = blockIdx.x * kShadeGuidedBlock; base < n; base += gridDim.x * kShadeGuidedBlock) {
        const uint32_t i = base + threadIdx.x;
        uint32_t slot = 0;
        bool valid = false;
        guide::V3 x = {0.0f, 0.0f, 0.0f}, wo = {0.0f, 1.0f, 0.0f};
        if (i < n) {
            slot = q[i];
            const float4 hv = state::load_hit(F, P, slot);
            const uint32_t tri = fbits(hv.y);
            if (tri != kNoHit) {
                const Tri tr = F.tris[tri];
                const float4 d = state::load_dir(F, P, slot);
                x = {tr.v0.x + ((tr.v1.x - tr.v0.x) * hv.z + (tr.v2.x - tr.v0.x) * hv.w),
                     tr.v0.y + ((tr.v1.y - tr.v0.y) * hv.z + (tr.v2.y - tr.v0.y) * hv.w),
                     tr.v0.z + ((tr.v1.z - tr.v0.z) * hv.z + (tr.v2.z - tr.v0.z) * hv.w)};
                wo = {-d.x, -d.y, -d.z};
                valid = true;
            }
        }
        wave_sync();
        mlp::infer_wave64(sfrag, sbias, x, wo, valid, F.guide.bmin, F.guide.binv, wave_rows);
        wave_sync();
        ShadeOut o;
        shade_out_init(o);
        if (i < n) shade_slot(F, P, v, slot, slot, o, smix + threadIdx.x * guide::kMixU4);
        shade_emit(F, P, v, slot, o, qn, s_app);
    }
}

// ---- regeneration (Sec. 3.1.3: terminated sample states are restarted with
// new samples once more than half of the states in memory are free). A
// whole-frame batch of N = npix npass paths runs through L state slots: slot
// s holds path pv[s].x (its id in the batch, the slot it would have without
// regeneration) at vertex pv[s].y. The path's radiance stays at rad[id], so
// the accumulation in pass order is unchanged and every path computes the
// same bits as without regeneration. Iteration t traces and shades the queue
// q_ext[t & 1] (counters[rg_queue_count(t)]) whatever the depth of each path in it.

// the first min(L, N) paths of the batch into slots [0, min(L, N))
__global__ __launch_bounds__(kBlock) void k_regen_init(Frame F, Pool P, uint32_t npix, uint64_t pass0,
                                                       uint32_t npass, uint32_t L)
{
    const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
    const bool skip = P.counters[kSkip] != 0;  // aborted: nothing to render
    const uint32_t N = npix * npass;
    const uint32_t n = skip ? 0u : min(L, N);
    if (s == 0) {
        P.counters[kRgQ0] = n;
        P.counters[kRgQ1] = 0;
        P.counters[kRgSh] = 0;
        P.counters[kRgDead] = 0;
        P.counters[kRgNext] = n;
        P.counters[kRgLeft] = skip ? 0u : N;
    }
    if (s >= n) return;
    start_path(F, P, s, s, 0, npix, npass, pass0);
    P.pv[s] = make_uint2(s, 1u);
    P.q_ext[0][s] = s;
}

// shading of iteration t: each slot at its own vertex; continuing paths join
// the next iteration's queue, terminated slots the dead list (plain
// rendering: no guide, no training records)
__global__ __launch_bounds__(kBlock, 4) void k_shade_regen(Frame F, Pool P, uint32_t t)
{
    __shared__ uint32_t s_app[3 * (kAppendWaves + 1)];
    const uint32_t n = P.counters[rg_queue_count(t)];
    const uint32_t *q = P.q_ext[t & 1];
    uint32_t *qn = P.q_ext[(t + 1) & 1];
    uint32_t *cn = &P.counters[rg_queue_count(t + 1)];
    for (uint32_t base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        const uint32_t i = base + threadIdx.x;
        const bool active = i < n;
        uint32_t slot = 0;
        ShadeOut o;
        o.alive = o.shadow = o.record = false;
        o.sh_o = o.sh_d = o.sh_c = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        for (int k = 0; k < 5; ++k) o.rec[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (active) {
            slot = q[i];
            const uint2 pv = P.pv[slot];
            shade_slot(F, P, pv.y, slot, pv.x, o);
            if (o.alive) P.pv[slot] = make_uint2(pv.x, pv.y + 1u);
        }
        const bool dead = active && !o.alive;
        uint32_t ps, pe, pd;
        block_append3(&P.counters[kRgSh], o.shadow, cn, o.alive, &P.counters[kRgDead], dead, s_app, ps, pe, pd);
        if (o.shadow) {
            o.sh_c.w = ubits(kNoHit);
            P.sh_o[ps] = o.sh_o;
            P.sh_d[ps] = o.sh_d;
            P.sh_c[ps] = o.sh_c;
        }
        if (o.alive) qn[pe] = slot;
        if (dead) P.q_dead[pd] = slot;
    }
}

// paths to start after an iteration: the free slots once more than half of
// the L slots are free, as long as paths of the batch remain to start
__device__ __forceinline__ uint32_t regen_count(const Pool &P, uint32_t L, uint32_t N)
{
    const uint32_t dead = P.counters[kRgDead], next = P.counters[kRgNext];
    return (2ull * dead > L && next < N) ? min(dead, N - next) : 0u;
}

// restart free slot k with path next + k, appended to the next iteration's
// queue after the paths that continue (counters updated by k_regen_commit)
__global__ __launch_bounds__(kBlock) void k_regen(Frame F, Pool P, uint32_t t, uint32_t npix, uint64_t pass0,
                                                  uint32_t npass, uint32_t L)
{
    const uint32_t N = npix * npass;
    const uint32_t k = regen_count(P, L, N);
    const uint32_t next = P.counters[kRgNext];
    const uint32_t at = P.counters[rg_queue_count(t + 1)];
    uint32_t *qn = P.q_ext[(t + 1) & 1];
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
        const uint32_t s = P.q_dead[i];
        start_path(F, P, s, next + i, 0, npix, npass, pass0);
        P.pv[s] = make_uint2(next + i, 1u);
        qn[at + i] = s;
    }
}

// one thread after iteration t and its regeneration: the iteration's rays
// into the statistics, the next queue's length, the dead list emptied (slots
// left over once every path has started are never needed again), the current
// queue's and the shadow count cleared for reuse, and the paths left
__global__ void k_regen_commit(Pool P, uint32_t t, uint32_t N, uint32_t L)
{
    const uint32_t k = regen_count(P, L, N);
    const uint32_t ci = rg_queue_count(t), cn = rg_queue_count(t + 1);
    P.stats[0] += P.counters[ci];
    P.stats[1] += P.counters[kRgSh];
    if (k) {
        P.counters[kRgDead] = 0;
        P.counters[kRgNext] += k;
    }
    P.counters[cn] += k;
    P.counters[ci] = 0;
    P.counters[kRgSh] = 0;
    P.counters[kRgLeft] = P.counters[cn] + (N - P.counters[kRgNext]);
}

// The tail of a batch in one launch (Sec. 3.1.3: a megakernel once few
// paths are left): every path still queued at depth v0 runs to its end in one
// thread -- closest hit, shading, its shadow ray, depth after depth -- with
// the same device code as the per-depth kernels, so its radiance is the same
// bit for bit. Rays of deeper vertices are added to the per-depth counters as
// the per-depth kernels would count them. With the guide on it starts past
// the guided vertices (records and mixtures stay in the per-depth kernels).
template <bool QN>
__global__ __launch_bounds__(kBlock, 4) void k_tail(Frame F, Pool P, uint32_t v0)
{
    __shared__ int stk[kShortStack * kBlock];
    __shared__ QNode top[QN ? kTopNodes : 1];
    __shared__ uint32_t cnt_ext[64], cnt_sh[64];
    if (threadIdx.x < 64) {
        cnt_ext[threadIdx.x] = 0;
        cnt_sh[threadIdx.x] = 0;
    }
    if (QN) stage_top(F, top);
    __syncthreads();
    const uint32_t n = P.counters[v0];
    const uint32_t *q = P.q_ext[v0 & 1];
    int *gstk = P.gstack + (size_t)(blockIdx.x * kBlock + threadIdx.x);
    uint32_t en = 0, et = 0, sn = 0, st = 0;
    for (uint32_t base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        const uint32_t i = base + threadIdx.x;
        if (i >= n) break;
        const uint32_t slot = q[i];
        for (uint32_t v = v0;; ++v) {
            const float4 o4 = P.ray_o[slot], d4 = state::load_dir(F, P, slot);
            RayPre r = prepare(xyz(o4), xyz(d4));
            HitRec h;
            traverse<false, QN, false, QN>(F, r, o4.w, h, stk + threadIdx.x, gstk, P.trav_threads, top);
            state::store_hit(F, P, slot, make_float4(h.t, ubits(h.tri), h.b1, h.b2));
            en += h.nodes;
            et += h.tests;
            ShadeOut o;
            o.sh_o = o.sh_d = o.sh_c = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            for (int k = 0; k < 5; ++k) o.rec[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            shade_slot(F, P, v, slot, slot, o);
            if (o.shadow) {
                atomicAdd(&cnt_sh[v], 1u);
                RayPre rs = prepare(xyz(o.sh_o), xyz(o.sh_d));
                HitRec hs;
                const bool occluded =
                    traverse<true, QN, false, QN>(F, rs, o.sh_o.w, hs, stk + threadIdx.x, gstk, P.trav_threads, top);
                sn += hs.nodes;
                st += hs.tests;
                if (!occluded) {
                    const float4 L = P.rad[slot];
                    P.rad[slot] = make_float4(L.x + o.sh_c.x, L.y + o.sh_c.y, L.z + o.sh_c.z, L.w);
                }
            }
            if (!o.alive) break;
            atomicAdd(&cnt_ext[v + 1], 1u);
        }
    }
    wave_count(&P.stats[4], en);
    wave_count(&P.stats[5], et);
    wave_count(&P.stats[6], sn);
    wave_count(&P.stats[7], st);
    __syncthreads();
    if (threadIdx.x < 64) {
        if (cnt_ext[threadIdx.x]) atomicAdd(&P.counters[threadIdx.x], cnt_ext[threadIdx.x]);
        if (cnt_sh[threadIdx.x]) atomicAdd(&P.counters[64 + threadIdx.x], cnt_sh[threadIdx.x]);
    }
}

// FP64 accumulation in pass order and sample counts
__global__ __launch_bounds__(kBlock) void k_accumulate(Frame F, Pool P, uint32_t pix0, uint32_t npix, uint32_t npass)
{
    if (P.counters[kSkip]) return;  // an aborted batch adds neither sums nor counts
    uint32_t q = blockIdx.x * kBlock + threadIdx.x;
    if (q == 0) {
        unsigned long long ext = 0, sh = 0;
        for (uint32_t v = 1; v <= F.max_depth; ++v) {
            ext += P.counters[v];
            sh += P.counters[64 + v];
        }
        P.stats[0] += ext;
        P.stats[1] += sh;
        P.stats[2] += (unsigned long long)npix * npass;
    }
    if (q >= npix) return;
    const bool whole = whole_frame(F, npix);
    const SlotMap m = slot_map(npix, npass);
    const uint32_t p = whole ? tile_pixel(q, F.W, F.H) : pix0 + q;
    double sx = P.fb_sum[3 * (size_t)p], sy = P.fb_sum[3 * (size_t)p + 1], sz = P.fb_sum[3 * (size_t)p + 2];
    for (uint32_t j = 0; j < npass; ++j) {
        float4 L = P.rad[whole ? slot_of(m, q, j) : (size_t)j * npix + q];
        sx += (double)L.x;
        sy += (double)L.y;
        sz += (double)L.z;
    }
    P.fb_sum[3 * (size_t)p] = sx;
    P.fb_sum[3 * (size_t)p + 1] = sy;
    P.fb_sum[3 * (size_t)p + 2] = sz;
    P.fb_count[p] += npass;
}

// per-wave sums of in[0 .. n) (n a multiple of 64, so a wave is either
// wholly in range, every lane active, or wholly out)
__global__ __launch_bounds__(kBlock) void k_debug_wave_sum(const uint32_t *in, uint32_t n, uint32_t *out)
{
    const size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    const uint32_t s = wave_sum_u32(in[q]);
    if (__lane_id() == 0) out[q / 64] = s;
}

__global__ void k_debug_sample_bits(Frame F, const uint64_t *idx, const uint32_t *dim, uint32_t n, int scramble,
                                    uint32_t *out)
{
    uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    uint32_t d = dim[q];
    out[q] = d < kMaxDims ? sample_bits(F, idx[q], d, (uint32_t)scramble) : 0u;
}

__global__ void k_debug_pixel_index(Frame F, uint64_t pass, uint64_t *out)
{
    uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= F.W * F.H) return;
    out[q] = pixel_index(F, q % F.W, q / F.W, pass);
}

template <bool ANY>
__global__ __launch_bounds__(kBlock) void k_debug_trace(Frame F, Pool P, const float *rays, uint32_t n, float *t,
                                                        uint32_t *tri, float *b12, uint32_t *depth)
{
    __shared__ int stk[kShortStack * kBlock];
    __shared__ QNode top[kTopNodes];
    if ((size_t)blockIdx.x * kBlock >= n) return;
    const bool qn = F.node_format == kNodeQuant;
    if (qn) stage_top(F, top);
    int *gstk = P.gstack + (size_t)(blockIdx.x * kBlock + threadIdx.x);
    for (uint32_t base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        uint32_t q = base + threadIdx.x;
        if (q >= n) break;
        const float *ry = rays + 8 * (size_t)q;
        RayPre r = prepare(mk(ry[0], ry[1], ry[2]), mk(ry[4], ry[5], ry[6]));
        HitRec h;
        bool hit = qn ? traverse<ANY, true, true, true>(F, r, ry[3], h, stk + threadIdx.x, gstk, P.trav_threads, top)
                      : traverse<ANY, false, true>(F, r, ry[3], h, stk + threadIdx.x, gstk, P.trav_threads);
        if (depth) depth[q] = h.depth;
        if (ANY) {
            tri[q] = hit ? 1u : 0u;
            continue;
        }
        tri[q] = hit ? h.id : kNoHit;
        t[q] = hit ? h.t : INFINITY;
        b12[2 * (size_t)q] = hit ? h.b1 : 0.0f;
        b12[2 * (size_t)q + 1] = hit ? h.b2 : 0.0f;
    }
}

template <bool ANY>
__global__ __launch_bounds__(kBlock) void k_debug_brute(Frame F, const float *rays, uint32_t n, float *t,
                                                        uint32_t *tri, float *b12)
{
    uint32_t q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    const float *ry = rays + 8 * (size_t)q;
    RayPre r = prepare(mk(ry[0], ry[1], ry[2]), mk(ry[4], ry[5], ry[6]));
    HitRec h;
    bool hit = brute_force<ANY>(F, r, ry[3], h);
    if (ANY) {
        tri[q] = hit ? 1u : 0u;
        return;
    }
    tri[q] = hit ? h.id : kNoHit;
    t[q] = hit ? h.t : INFINITY;
    b12[2 * (size_t)q] = hit ? h.b1 : 0.0f;
    b12[2 * (size_t)q + 1] = hit ? h.b2 : 0.0f;
}

inline uint32_t blocks_for(size_t n, uint32_t cap)
{
    size_t b = (n + kBlock - 1) / kBlock;
    return (uint32_t)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 4096)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(n, 4096)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

// one kernel launch; when profiling, the dispatch itself records the start
// and stop events (the kernel's own execution time, as a kernel trace
// measures it, without the event packets' overhead around it)
template <typename Kern, typename... Args>
static inline void launch_timed(Profiler *prof, int kind, Kern kernel, dim3 grid, dim3 block, hipStream_t s,
                                Args... args)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (prof) prof->kernel_events(kind, &a, &b);
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, b, 0, args...);
}

hipError_t launch_render_paths(const Frame &F, const Pool &P, uint32_t pix0, uint32_t npix, uint64_t pass0,
                               uint32_t npass, hipStream_t s, Profiler *prof)
{
    uint32_t n = npix * npass;
    launch_timed(prof, K_CLEAR, k_batch_begin, dim3(1), dim3(kCounters), s, P, F.abort_word, pix0 == 0 ? 1u : 0u);
    launch_timed(prof, K_GENERATE, k_generate, dim3(blocks_for(n, 1u << 30)), dim3(kBlock), s, F, P, pix0, npix, pass0,
                 n);
    uint32_t g = blocks_for(n, 8192);
    const uint32_t gs = (uint32_t)std::max<size_t>(1, (size_t)g * kBlock / kShadeBlock);  // k_shade: the same threads
    uint32_t gt = blocks_for(n, P.trav_threads / kBlock);
    // guided shading: four times the blocks resident at once, each staging
    // the weights once (a grid of only the resident blocks balances badly
    // when the other batch in flight holds part of the GPU)
    uint32_t gg = (uint32_t)std::min<size_t>(((size_t)n + kShadeGuidedBlock - 1) / kShadeGuidedBlock,
                                             P.trav_threads / kBlock / kTravBlocksPerCU * kShadeGuidedGridPerCU);
    // with the guide on, the tail may start only past its last guided
    // vertex: the mixtures and the training records belong to the per-depth
    // kernels, while the tail's vertices sample the BSDF alone (their MIS
    // reads the previous vertex's sampling density from the path state)
    const bool guide_on = F.guide.alpha_thr || F.guide.record;
    const bool tail_ok = F.tail_depth >= 1 && (!guide_on || F.tail_depth > F.guide.max_vertex);
    for (uint32_t v = 1; v <= F.max_depth; ++v) {
        if (tail_ok && v == F.tail_depth) {
            // the rest of the batch's paths in one launch (traversal grid, four blocks per CU resident)
            if (F.node_format == kNodeQuant) launch_timed(prof, K_TAIL, k_tail<true>, dim3(gt), dim3(kBlock), s, F, P, v);
            else launch_timed(prof, K_TAIL, k_tail<false>, dim3(gt), dim3(kBlock), s, F, P, v);
            break;
        }
        if (F.node_format == kNodeQuant)
            launch_timed(prof, K_TRACE, k_trace<true>, dim3(gt), dim3(kBlock), s, F, P, v, v & 1u);
        else
            launch_timed(prof, K_TRACE, k_trace<false>, dim3(gt), dim3(kBlock), s, F, P, v, v & 1u);
        if (F.guide.alpha_thr && v < F.max_depth && v <= F.guide.max_vertex)
            launch_timed(prof, K_SHADE_GUIDED, k_shade_guided, dim3(gg), dim3(kShadeGuidedBlock), s, F, P, v);
        else
            launch_timed(prof, K_SHADE, k_shade, dim3(gs), dim3(kShadeBlock), s, F, P, v);
        if (F.node_format == kNodeQuant)
            launch_timed(prof, K_SHADOW, k_shadow<true>, dim3(gt), dim3(kBlock), s, F, P, 64u + v);
        else
            launch_timed(prof, K_SHADOW, k_shadow<false>, dim3(gt), dim3(kBlock), s, F, P, 64u + v);
    }
    return hipGetLastError();
}

hipError_t launch_render_regen(const Frame &F, const Pool &P, uint32_t npix, uint64_t pass0, uint32_t npass,
                               hipStream_t s, Profiler *prof, uint32_t *left, hipEvent_t ev[2])
{
    const uint32_t N = npix * npass, L = std::min(F.regen, N);
    auto timed = [&](int kind, auto &&launch) {
        if (prof) prof->begin(kind, s);
        launch();
        if (prof) prof->end(kind, s);
    };
    timed(K_CLEAR, [&] { hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(kCounters), 0, s, P, F.abort_word, 1u); });
    timed(K_GENERATE, [&] {
        hipLaunchKernelGGL(k_regen_init, dim3(blocks_for(L, 1u << 30)), dim3(kBlock), 0, s, F, P, npix, pass0, npass, L);
    });
    const uint32_t g = blocks_for(L, 8192), gt = blocks_for(L, P.trav_threads / kBlock);
    auto iteration = [&](uint32_t t) {
        const uint32_t c = rg_queue_count(t);
        timed(K_TRACE, [&] {
            if (F.node_format == kNodeQuant) hipLaunchKernelGGL(k_trace<true>, dim3(gt), dim3(kBlock), 0, s, F, P, c, t & 1);
            else hipLaunchKernelGGL(k_trace<false>, dim3(gt), dim3(kBlock), 0, s, F, P, c, t & 1);
        });
        timed(K_SHADE, [&] { hipLaunchKernelGGL(k_shade_regen, dim3(g), dim3(kBlock), 0, s, F, P, t); });
        timed(K_SHADOW, [&] {
            if (F.node_format == kNodeQuant) hipLaunchKernelGGL(k_shadow<true>, dim3(gt), dim3(kBlock), 0, s, F, P, kRgSh);
            else hipLaunchKernelGGL(k_shadow<false>, dim3(gt), dim3(kBlock), 0, s, F, P, kRgSh);
        });
        timed(K_GENERATE, [&] {
            hipLaunchKernelGGL(k_regen, dim3(g), dim3(kBlock), 0, s, F, P, t, npix, pass0, npass, L);
            hipLaunchKernelGGL(k_regen_commit, dim3(1), dim3(1), 0, s, P, t, N, L);
        });
    };
    // Each iteration advances every live path by one vertex; one that leaves
    // more than half of the slots free is followed by a regeneration that
    // fills them, so at most every other iteration has fewer than L / 2 paths
    // while paths remain to start, and once all have started the last ones
    // end within max_depth iterations.
    const uint64_t bound = 4ull * (uint64_t)N * F.max_depth / L + 2ull * F.max_depth + 16;
    // Iterations go out in chunks; after each chunk the paths left are copied
    // to host memory, and the chunk before the previous one is checked before
    // the next goes out, so the queue never runs dry while the host waits.
    constexpr uint32_t kChunk = 4;
    uint32_t t = 0;
    for (uint64_t chunk = 0;; ++chunk) {
        if (chunk >= 2) {
            hipError_t e = hipEventSynchronize(ev[chunk & 1]);
            if (e != hipSuccess) return e;
            if (__atomic_load_n(&left[chunk & 1], __ATOMIC_ACQUIRE) == 0) break;
        }
        if (t > bound) return hipErrorUnknown;
        for (uint32_t k = 0; k < kChunk; ++k) iteration(t++);
        hipError_t e = hipMemcpyAsync(&left[chunk & 1], P.counters + kRgLeft, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipEventRecord(ev[chunk & 1], s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t launch_accumulate(const Frame &F, const Pool &P, uint32_t pix0, uint32_t npix, uint32_t npass,
                             hipStream_t s, Profiler *prof)
{
    launch_timed(prof, K_ACCUMULATE, k_accumulate, dim3(blocks_for(npix, 1u << 30)), dim3(kBlock), s, F, P, pix0, npix,
                 npass);
    return hipGetLastError();
}

hipError_t launch_render_batch(const Frame &F, const Pool &P, uint32_t pix0, uint32_t npix, uint64_t pass0,
                               uint32_t npass, hipStream_t s, Profiler *prof)
{
    hipError_t e = launch_render_paths(F, P, pix0, npix, pass0, npass, s, prof);
    if (e != hipSuccess) return e;
    return launch_accumulate(F, P, pix0, npix, npass, s, prof);
}

// the training records of a lane's last batch with their identity: pixel,
// pass and vertex of each, position, directions, density and the weight its
// finalisation gives (the same device function), for parity checks
__global__ void k_debug_records(Frame F, Pool P, uint32_t pix0, uint32_t npix, uint64_t pass0, uint32_t npass,
                                uint32_t n, uint32_t *ident, float *out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 *r = F.guide.rec + (size_t)i * kRecF4;
    const float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
    const uint32_t slot = fbits(r2.w);
    uint32_t pl, j, p;
    if (whole_frame(F, npix)) {
        position_of(slot_map(npix, npass), slot, pl, j);
        p = tile_pixel(pl, F.W, F.H);
    } else {
        pl = slot % npix;
        j = slot / npix;
        p = pix0 + pl;
    }
    ident[3 * (size_t)i] = p;
    ident[3 * (size_t)i + 1] = (uint32_t)(pass0 + j);
    ident[3 * (size_t)i + 2] = fbits(r3.w);
    float *o = out + 11 * (size_t)i;
    o[0] = r0.x; o[1] = r0.y; o[2] = r0.z;
    o[3] = r1.x; o[4] = r1.y; o[5] = r1.z;
    o[6] = r2.x; o[7] = r2.y; o[8] = r2.z;
    o[9] = r0.w;
    o[10] = guide::record_weight(r3, r[4], r[5], P.rad[slot]);
}

hipError_t launch_debug_records(const Frame &F, const Pool &P, uint32_t pix0, uint32_t npix, uint64_t pass0,
                                uint32_t npass, uint32_t n, uint32_t *ident, float *out, hipStream_t s)
{
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_debug_records, dim3((n + 255) / 256), dim3(256), 0, s, F, P, pix0, npix, pass0, npass, n,
                       ident, out);
    return hipGetLastError();
}

hipError_t launch_debug_wave_sum(const uint32_t *in, uint32_t n, uint32_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_wave_sum, dim3(blocks_for(n, 1u << 30)), dim3(kBlock), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_debug_sample_bits(const Frame &F, const uint64_t *idx, const uint32_t *dim, uint32_t n,
                                    int scramble, uint32_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_sample_bits, dim3(blocks_for(n, 1u << 30)), dim3(kBlock), 0, s, F, idx, dim, n,
                       scramble, out);
    return hipGetLastError();
}

__global__ void k_debug_env_sample(Frame F, const uint32_t *uv, const float *nrm, uint32_t n, uint32_t mode,
                                   uint32_t *texel, uint64_t *iv, uint64_t *iv_hit)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int bin = mode == 2 ? (int)ep_bin(mk(nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2])) : -1;
    uint32_t row, col;
    uint64_t ru, su, rv, sv;
    ep_descend(F, bin, uv[2 * i], uv[2 * i + 1], false, row, col, ru, su, rv, sv);
    texel[i] = row * F.env_w + col;
    iv[4 * i] = ru;
    iv[4 * i + 1] = su;
    iv[4 * i + 2] = rv;
    iv[4 * i + 3] = sv;
    ep_descend(F, bin, 0u, 0u, true, row, col, ru, su, rv, sv);
    iv_hit[2 * i] = ru;
    iv_hit[2 * i + 1] = rv;
}

hipError_t launch_debug_env_sample(const Frame &F, const uint32_t *uv, const float *nrm, uint32_t n, uint32_t mode,
                                   uint32_t *texel, uint64_t *iv, uint64_t *iv_hit, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_env_sample, dim3(blocks_for(n, 1u << 30)), dim3(kBlock), 0, s, F, uv, nrm, n, mode,
                       texel, iv, iv_hit);
    return hipGetLastError();
}

__global__ void k_debug_light_sample(Frame F, const uint64_t *S, const float *x, const float *nrm, uint32_t n,
                                     uint32_t *emitter, uint64_t *size, uint64_t *size_hit)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const f3 xp = mk(x[3 * i], x[3 * i + 1], x[3 * i + 2]), np = mk(nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]);
    uint64_t z;
    const uint32_t e = lt_sample(F, S[i] & 0x7fffffffffffffffull, xp, np, z);
    emitter[i] = e;
    size[i] = z;
    size_hit[i] = lt_size_of(F, e, xp, np);
}

hipError_t launch_debug_light_sample(const Frame &F, const uint64_t *S, const float *x, const float *nrm, uint32_t n,
                                     uint32_t *emitter, uint64_t *size, uint64_t *size_hit, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_light_sample, dim3(blocks_for(n, 1u << 30)), dim3(kBlock), 0, s, F, S, x, nrm, n,
                       emitter, size, size_hit);
    return hipGetLastError();
}

hipError_t launch_debug_pixel_index(const Frame &F, uint64_t pass, uint64_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_pixel_index, dim3(blocks_for((size_t)F.W * F.H, 1u << 30)), dim3(kBlock), 0, s, F,
                       pass, out);
    return hipGetLastError();
}

hipError_t launch_debug_trace(const Frame &F, const Pool &P, const float *rays, uint32_t n, int any_hit,
                              int brute, float *t, uint32_t *tri, float *b12, uint32_t *depth, hipStream_t s)
{
    dim3 b(kBlock);
    if (brute) {
        dim3 g(blocks_for(n, 1u << 30));
        if (any_hit) hipLaunchKernelGGL((k_debug_brute<true>), g, b, 0, s, F, rays, n, t, tri, b12);
        else hipLaunchKernelGGL((k_debug_brute<false>), g, b, 0, s, F, rays, n, t, tri, b12);
        return hipGetLastError();
    }
    dim3 g(blocks_for(n, P.trav_threads / kBlock));
    if (any_hit) hipLaunchKernelGGL((k_debug_trace<true>), g, b, 0, s, F, P, rays, n, t, tri, b12, depth);
    else hipLaunchKernelGGL((k_debug_trace<false>), g, b, 0, s, F, P, rays, n, t, tri, b12, depth);
    return hipGetLastError();
}
}  // namespace qpt
