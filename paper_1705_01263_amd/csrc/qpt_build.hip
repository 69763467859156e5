// GPU BVH builder: a linear BVH (Karras 2012, "Maximizing parallelism in the
// construction of BVHs, octrees, and k-d trees") over Morton-ordered triangle
// centroids, refitted bottom-up and collapsed top-down into the renderer's
// 4-wide node format. The paper builds on the GPU where it can (Sec. 3.1
// cites rapid GPU construction); the binned-SAH host builder stays the
// default, this one trades tree quality for build time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "qpt_internal.h"

namespace qpt {
namespace {

constexpr uint32_t kB = 256;

inline uint32_t grid_for(size_t n) { return (uint32_t)std::max<size_t>(1, std::min<size_t>((n + kB - 1) / kB, 1u << 20)); }

// triangle boxes, and per block the box of the centroids
__global__ void k_prim_boxes(const float *pos, const uint32_t *idx, uint32_t nt, float4 *blo, float4 *bhi,
                             float *cpart)
{
    __shared__ float red[6][kB];
    float c_lo[3] = {INFINITY, INFINITY, INFINITY}, c_hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t t = blockIdx.x * kB + threadIdx.x; t < nt; t += gridDim.x * kB) {
        float lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            const float v0 = pos[3 * (size_t)idx[3 * (size_t)t] + a], v1 = pos[3 * (size_t)idx[3 * (size_t)t + 1] + a];
            const float v2 = pos[3 * (size_t)idx[3 * (size_t)t + 2] + a];
            lo[a] = fminf(v0, fminf(v1, v2));
            hi[a] = fmaxf(v0, fmaxf(v1, v2));
            const float cc = 0.5f * (lo[a] + hi[a]);
            c_lo[a] = fminf(c_lo[a], cc);
            c_hi[a] = fmaxf(c_hi[a], cc);
        }
        blo[t] = make_float4(lo[0], lo[1], lo[2], 0.0f);
        bhi[t] = make_float4(hi[0], hi[1], hi[2], 0.0f);
    }
    for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = c_lo[a];
        red[3 + a][threadIdx.x] = c_hi[a];
    }
    __syncthreads();
    for (uint32_t w = kB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + w]);
                red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) cpart[6 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__device__ __forceinline__ uint32_t spread10(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// 30-bit Morton code of the centroid in the upper word, the triangle id in the
// lower: keys are distinct, so the hierarchy below is well defined
__global__ void k_morton(const float4 *blo, const float4 *bhi, uint32_t nt, float3 cmin, float3 cscale,
                         unsigned long long *keys)
{
    for (uint32_t t = blockIdx.x * kB + threadIdx.x; t < nt; t += gridDim.x * kB) {
        const float4 lo = blo[t], hi = bhi[t];
        const float c[3] = {0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z)};
        const float m[3] = {cmin.x, cmin.y, cmin.z}, s[3] = {cscale.x, cscale.y, cscale.z};
        uint32_t q[3];
        for (int a = 0; a < 3; ++a) q[a] = (uint32_t)fminf(fmaxf((c[a] - m[a]) * s[a], 0.0f), 1023.0f);
        const uint32_t code = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
        keys[t] = ((unsigned long long)code << 32) | t;
    }
}

__device__ __forceinline__ int common_prefix(const unsigned long long *k, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    return __clzll(k[i] ^ k[j]);
}

// Internal node i of n - 1 (node ids: internal 0..n-2, leaf j is n - 1 + j):
// its key range by the sign of the neighbouring prefixes, then the split at
// the highest differing bit (the construction of Karras 2012, Sec. 4).
__global__ void k_hierarchy(const unsigned long long *k, int n, int2 *child, int *parent, uint2 *range)
{
    for (int i = blockIdx.x * kB + threadIdx.x; i < n - 1; i += gridDim.x * kB) {
        const int d = common_prefix(k, n, i, i + 1) - common_prefix(k, n, i, i - 1) >= 0 ? 1 : -1;
        const int dmin = common_prefix(k, n, i, i - d);
        int lmax = 2;
        while (common_prefix(k, n, i, i + lmax * d) > dmin) lmax *= 2;
        int l = 0;
        for (int t = lmax / 2; t >= 1; t /= 2)
            if (common_prefix(k, n, i, i + (l + t) * d) > dmin) l += t;
        const int j = i + l * d;
        const int dnode = common_prefix(k, n, i, j);
        int s = 0, t = l;
        do {
            t = (t + 1) >> 1;
            if (common_prefix(k, n, i, i + (s + t) * d) > dnode) s += t;
        } while (t > 1);
        const int g = i + s * d + min(d, 0);
        const int lo = min(i, j), hi = max(i, j);
        const int left = lo == g ? (n - 1 + g) : g;
        const int right = hi == g + 1 ? (n - 1 + g + 1) : g + 1;
        child[i] = make_int2(left, right);
        range[i] = make_uint2((uint32_t)lo, (uint32_t)hi);
        parent[left] = i;
        parent[right] = i;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) parent[0] = -1;
}

__device__ __forceinline__ float ld_acquire(const float *p)
{
    return __int_as_float(__hip_atomic_load((const int *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Boxes bottom-up: each leaf climbs; at every inner node the second of its
// two children to arrive (counted with an atomic) merges both boxes and goes
// on, the first stops. No thread waits for another.
__global__ void k_refit(const unsigned long long *k, const float4 *blo, const float4 *bhi, int n, const int2 *child,
                        const int *parent, uint32_t *visits, float *box)
{
    for (int j = blockIdx.x * kB + threadIdx.x; j < n; j += gridDim.x * kB) {
        const uint32_t t = (uint32_t)(k[j] & 0xffffffffull);
        int node = n - 1 + j;
        const float4 lo = blo[t], hi = bhi[t];
        float *b = box + 6 * (size_t)node;
        b[0] = lo.x;
        b[1] = lo.y;
        b[2] = lo.z;
        b[3] = hi.x;
        b[4] = hi.y;
        b[5] = hi.z;
        for (;;) {
            const int p = parent[node];
            if (p < 0) break;
            __threadfence();
            if (atomicAdd(&visits[p], 1u) == 0u) break;
            __threadfence();
            const int2 ch = child[p];
            const float *a = box + 6 * (size_t)ch.x, *c = box + 6 * (size_t)ch.y;
            float *o = box + 6 * (size_t)p;
            for (int q = 0; q < 3; ++q) {
                o[q] = fminf(ld_acquire(a + q), ld_acquire(c + q));
                o[3 + q] = fmaxf(ld_acquire(a + 3 + q), ld_acquire(c + 3 + q));
            }
            node = p;
        }
    }
}

__device__ __forceinline__ uint32_t node_count(int id, int n, const uint2 *range)
{
    return id >= n - 1 ? 1u : range[id].y - range[id].x + 1u;
}

__device__ __forceinline__ float box_area(const float *b)
{
    const float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return 2.0f * (dx * dy + dy * dz + dz * dx);
}

// One level of the collapse: each queued binary node becomes a 4-wide node
// holding its two children and, while fewer than four, the children of its
// largest-area child that is not a leaf range; inner children get adjacent
// slots and go to the next level's queue.
__global__ void k_collapse(const uint2 *qin, const uint32_t *nin, uint2 *qout, uint32_t *nout, uint32_t *nodes_used,
                           int n, uint32_t leaf, float pad, const int2 *child, const uint2 *range, const float *box,
                           Node *out)
{
    const uint32_t count = *nin;
    for (uint32_t i = blockIdx.x * kB + threadIdx.x; i < count; i += gridDim.x * kB) {
        const uint2 w = qin[i];
        const int b = (int)w.x;
        int kids[4];
        int nk = 2;
        kids[0] = child[b].x;
        kids[1] = child[b].y;
        while (nk < 4) {
            int best = -1;
            float ba = -1.0f;
            for (int q = 0; q < nk; ++q) {
                if (node_count(kids[q], n, range) <= leaf) continue;
                const float a = box_area(box + 6 * (size_t)kids[q]);
                if (a > ba) {
                    ba = a;
                    best = q;
                }
            }
            if (best < 0) break;
            const int2 ch = child[kids[best]];
            kids[best] = ch.x;
            kids[nk++] = ch.y;
        }
        uint32_t inner = 0;
        for (int q = 0; q < nk; ++q) inner += node_count(kids[q], n, range) > leaf ? 1u : 0u;
        const uint32_t slot0 = inner ? atomicAdd(nodes_used, inner) : 0u;
        const uint32_t at0 = inner ? atomicAdd(nout, inner) : 0u;
        float bx[6][4];
        int ref[4];
        uint32_t used = 0;
        for (int q = 0; q < 4; ++q) {
            if (q >= nk) {
                for (int a = 0; a < 6; ++a) bx[a][q] = 0.0f;
                ref[q] = kEmptyChild;
                continue;
            }
            const float *cb = box + 6 * (size_t)kids[q];
            for (int a = 0; a < 3; ++a) {
                bx[a][q] = cb[a] - pad;
                bx[3 + a][q] = cb[3 + a] + pad;
            }
            const uint32_t cnt = node_count(kids[q], n, range);
            if (cnt > leaf) {
                ref[q] = (int)(slot0 + used);
                qout[at0 + used] = make_uint2((uint32_t)kids[q], slot0 + used);
                ++used;
            } else {
                const uint32_t first = kids[q] >= n - 1 ? (uint32_t)(kids[q] - (n - 1)) : range[kids[q]].x;
                ref[q] = ~(int)((first << 3) | (cnt - 1));
            }
        }
        Node nd;
        nd.lox = make_float4(bx[0][0], bx[0][1], bx[0][2], bx[0][3]);
        nd.loy = make_float4(bx[1][0], bx[1][1], bx[1][2], bx[1][3]);
        nd.loz = make_float4(bx[2][0], bx[2][1], bx[2][2], bx[2][3]);
        nd.hix = make_float4(bx[3][0], bx[3][1], bx[3][2], bx[3][3]);
        nd.hiy = make_float4(bx[4][0], bx[4][1], bx[4][2], bx[4][3]);
        nd.hiz = make_float4(bx[5][0], bx[5][1], bx[5][2], bx[5][3]);
        nd.ref = make_int4(ref[0], ref[1], ref[2], ref[3]);
        nd.pad = make_int4(nk, 0, 0, 0);
        out[w.y] = nd;
    }
}

// ---- stable LSD radix sort of the 64-bit keys by their upper 30 bits (the
// Morton code). The keys enter in triangle order (the id is the lower word),
// so a stable sort by the code leaves equal codes in id order: the result is
// the keys sorted as 64-bit integers. Each pass sorts by one 8-bit digit:
// tiles of kTile keys count their digits, each digit's column of tile counts
// is scanned, and the tiles scatter their keys to the digit's base plus the
// tile's prefix plus the key's rank among equal digits in the tile.

constexpr uint32_t kRadixItems = 16;                 // keys per thread and tile
constexpr uint32_t kTile = kB * kRadixItems;         // 4096 keys per tile

__device__ __forceinline__ uint32_t digit_of(unsigned long long key, uint32_t shift)
{
    return (uint32_t)(key >> shift) & 0xffu;
}

// hist[d * tiles + t] = keys of tile t with digit d
__global__ __launch_bounds__(kB) void k_radix_hist(const unsigned long long *keys, uint32_t n, uint32_t shift,
                                                   uint32_t tiles, uint32_t *hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * kTile;
    for (uint32_t c = 0; c < kRadixItems; ++c) {
        const size_t i = base + c * kB + threadIdx.x;
        if (i < n) atomicAdd(&h[digit_of(keys[i], shift)], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// block d: exclusive scan of digit d's column of tile counts (in place) and
// the digit's total
__global__ __launch_bounds__(kB) void k_radix_colscan(uint32_t *hist, uint32_t tiles, uint32_t *total)
{
    __shared__ uint32_t part[kB];
    uint32_t *col = hist + (size_t)blockIdx.x * tiles;
    const uint32_t per = (tiles + kB - 1) / kB;
    const uint32_t lo = min(tiles, threadIdx.x * per), hi = min(tiles, lo + per);
    uint32_t sum = 0;
    for (uint32_t t = lo; t < hi; ++t) sum += col[t];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < kB; off <<= 1) {   // inclusive scan of the partial sums
        const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - sum;
    for (uint32_t t = lo; t < hi; ++t) {
        const uint32_t v = col[t];
        col[t] = run;
        run += v;
    }
    if (threadIdx.x == kB - 1) total[blockIdx.x] = part[kB - 1];
}

// stable scatter: within a tile the keys keep their order per digit (chunks
// of kB keys in order; inside a chunk, waves in order, lanes in order)
__global__ __launch_bounds__(kB) void k_radix_scatter(const unsigned long long *keys, unsigned long long *out,
                                                      uint32_t n, uint32_t shift, uint32_t tiles, const uint32_t *hist,
                                                      const uint32_t *total)
{
    constexpr uint32_t kWaves = kB / 64;
    __shared__ uint32_t base[256];           // digit base + this tile's prefix + keys of the digit so far
    __shared__ uint32_t wcount[kWaves][256]; // keys per wave and digit in the current chunk
    __shared__ uint32_t scan[256];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    // digit bases: exclusive scan of the digit totals
    scan[tid] = total[tid];
    __syncthreads();
    for (uint32_t off = 1; off < 256; off <<= 1) {
        const uint32_t v = tid >= off ? scan[tid - off] : 0u;
        __syncthreads();
        scan[tid] += v;
        __syncthreads();
    }
    base[tid] = scan[tid] - total[tid] + hist[(size_t)tid * tiles + blockIdx.x];
    for (uint32_t w = 0; w < kWaves; ++w) wcount[w][tid] = 0;
    __syncthreads();
    const size_t t0 = (size_t)blockIdx.x * kTile;
    const unsigned long long below = (lane ? ~0ull >> (64 - lane) : 0ull);
    for (uint32_t c = 0; c < kRadixItems; ++c) {
        const size_t i = t0 + c * kB + tid;
        const bool valid = i < n;
        const unsigned long long key = valid ? keys[i] : 0ull;
        const uint32_t d = valid ? digit_of(key, shift) : 256u;
        // lanes of this wave with the same digit
        unsigned long long peers = __ballot(valid);
        for (uint32_t b = 0; b < 8; ++b) {
            const unsigned long long m = __ballot(valid && ((d >> b) & 1u));
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        const bool leader = valid && rank == 0;
        if (leader) wcount[wv][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = base[d] + rank;
            for (uint32_t w = 0; w < wv; ++w) off += wcount[w][d];
            out[off] = key;
        }
        __syncthreads();
        uint32_t add = 0;
        for (uint32_t w = 0; w < kWaves; ++w) {
            add += wcount[w][tid];
            wcount[w][tid] = 0;
        }
        base[tid] += add;
        __syncthreads();
    }
}

__global__ void k_fill32(uint32_t *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)kB + threadIdx.x; i < n; i += (size_t)gridDim.x * kB) p[i] = 0u;
}

__global__ void k_order(const unsigned long long *k, uint32_t n, uint32_t *order)
{
    for (uint32_t j = blockIdx.x * kB + threadIdx.x; j < n; j += gridDim.x * kB) order[j] = (uint32_t)(k[j] & 0xffffffffull);
}

// the builder's temporaries, carved from one caller-provided device region
struct Scratch {
    float *pos;
    uint32_t *idx;
    float4 *blo, *bhi;
    float *cpart;
    unsigned long long *keys, *sorted;
    uint32_t *hist, *total;
    int2 *child;
    int *parent;
    uint2 *range;
    uint32_t *visits;
    float *box;
    Node *nodes;
    uint2 *q0, *q1;
    uint32_t *cnt;
    uint32_t *order;
};

struct Carver {
    char *base;
    size_t off;
    template <class T> T *take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = (T *)(base ? base + off : nullptr);
        off += std::max<size_t>(count * sizeof(T), 16);
        return p;
    }
};

size_t carve(char *base, uint32_t nv, uint32_t nt, Scratch &S)
{
    const size_t g = grid_for(nt), tiles = (nt + kTile - 1) / kTile, nn = 2 * (size_t)nt - 1;
    Carver c{base, 0};
    S.pos = c.take<float>((size_t)nv * 3);
    S.idx = c.take<uint32_t>((size_t)nt * 3);
    S.blo = c.take<float4>(nt);
    S.bhi = c.take<float4>(nt);
    S.cpart = c.take<float>(g * 6);
    S.keys = c.take<unsigned long long>(nt);
    S.sorted = c.take<unsigned long long>(nt);
    S.hist = c.take<uint32_t>(256 * tiles);
    S.total = c.take<uint32_t>(256);
    S.child = c.take<int2>(nt);
    S.parent = c.take<int>(nn);
    S.range = c.take<uint2>(nt);
    S.visits = c.take<uint32_t>(nt);
    S.box = c.take<float>(nn * 6);
    S.nodes = c.take<Node>(nt);
    S.q0 = c.take<uint2>(nt);
    S.q1 = c.take<uint2>(nt);
    S.cnt = c.take<uint32_t>(4);
    S.order = c.take<uint32_t>(nt);
    return c.off;
}

}  // namespace

#define BT(x)                                        \
    do {                                             \
        hipError_t e_ = (x);                         \
        if (e_ != hipSuccess) return e_;             \
    } while (0)

size_t gpu_build_scratch_bytes(uint32_t nv, uint32_t nt)
{
    Scratch S;
    return carve(nullptr, nv, nt, S);
}

hipError_t gpu_build_bvh(const float *pos, uint32_t nv, const uint32_t *idx, uint32_t nt, uint32_t leaf, float pad,
                         void *scratch, size_t scratch_bytes, hipStream_t s, std::vector<Node> &nodes,
                         std::vector<uint32_t> &order, uint32_t &depth)
{
    const int n = (int)nt;
    Scratch S;
    if (!scratch || carve(nullptr, nv, nt, S) > scratch_bytes) return hipErrorInvalidValue;
    carve((char *)scratch, nv, nt, S);
    const uint32_t g = grid_for(nt);
    BT(hipMemcpyAsync(S.pos, pos, (size_t)nv * 12, hipMemcpyHostToDevice, s));
    BT(hipMemcpyAsync(S.idx, idx, (size_t)nt * 12, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_prim_boxes, dim3(g), dim3(kB), 0, s, S.pos, S.idx, nt, S.blo, S.bhi, S.cpart);
    BT(hipGetLastError());
    std::vector<float> part((size_t)g * 6);
    BT(hipMemcpyAsync(part.data(), S.cpart, part.size() * 4, hipMemcpyDeviceToHost, s));
    BT(hipStreamSynchronize(s));
    float cmin[3] = {INFINITY, INFINITY, INFINITY}, cmax[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t b = 0; b < g; ++b)
        for (int a = 0; a < 3; ++a) {
            cmin[a] = std::min(cmin[a], part[6 * b + a]);
            cmax[a] = std::max(cmax[a], part[6 * b + 3 + a]);
        }
    float sc[3];
    for (int a = 0; a < 3; ++a) sc[a] = cmax[a] > cmin[a] ? 1024.0f / (cmax[a] - cmin[a]) : 0.0f;
    hipLaunchKernelGGL(k_morton, dim3(g), dim3(kB), 0, s, S.blo, S.bhi, nt, make_float3(cmin[0], cmin[1], cmin[2]),
                       make_float3(sc[0], sc[1], sc[2]), S.keys);
    BT(hipGetLastError());
    // four stable passes over the 30-bit code (bits 32..61 of the keys)
    const uint32_t tiles = (nt + kTile - 1) / kTile;
    unsigned long long *kin = S.keys, *kout = S.sorted;
    for (uint32_t shift = 32; shift < 64; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(tiles), dim3(kB), 0, s, kin, nt, shift, tiles, S.hist);
        BT(hipGetLastError());
        hipLaunchKernelGGL(k_radix_colscan, dim3(256), dim3(kB), 0, s, S.hist, tiles, S.total);
        BT(hipGetLastError());
        hipLaunchKernelGGL(k_radix_scatter, dim3(tiles), dim3(kB), 0, s, kin, kout, nt, shift, tiles, S.hist, S.total);
        BT(hipGetLastError());
        std::swap(kin, kout);
    }
    const unsigned long long *sorted = kin;
    hipLaunchKernelGGL(k_fill32, dim3(grid_for(nt)), dim3(kB), 0, s, S.visits, (size_t)nt);
    BT(hipGetLastError());
    hipLaunchKernelGGL(k_hierarchy, dim3(g), dim3(kB), 0, s, sorted, n, S.child, S.parent, S.range);
    BT(hipGetLastError());
    hipLaunchKernelGGL(k_refit, dim3(g), dim3(kB), 0, s, sorted, S.blo, S.bhi, n, S.child, S.parent, S.visits, S.box);
    BT(hipGetLastError());
    // collapse, one level per launch; a 4-wide node takes at least one binary
    // inner node, so n - 1 slots suffice
    const uint2 root = make_uint2(0u, 0u);
    const uint32_t init[4] = {1u, 0u, 1u, 0u};  // queue 0 count, queue 1 count, nodes used, -
    BT(hipMemcpyAsync(S.q0, &root, 8, hipMemcpyHostToDevice, s));
    BT(hipMemcpyAsync(S.cnt, init, 16, hipMemcpyHostToDevice, s));
    uint32_t pending = 1, levels = 0;
    while (pending) {
        uint2 *qin = (levels & 1) ? S.q1 : S.q0;
        uint2 *qout = (levels & 1) ? S.q0 : S.q1;
        uint32_t *nin = S.cnt + (levels & 1), *nout = S.cnt + ((levels + 1) & 1);
        const uint32_t zero = 0;
        BT(hipMemcpyAsync(nout, &zero, 4, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_collapse, dim3(grid_for(pending)), dim3(kB), 0, s, qin, nin, qout, nout, S.cnt + 2, n,
                           leaf, pad, S.child, S.range, S.box, S.nodes);
        BT(hipGetLastError());
        BT(hipMemcpyAsync(&pending, nout, 4, hipMemcpyDeviceToHost, s));
        BT(hipStreamSynchronize(s));
        ++levels;
        if (levels > 128) return hipErrorUnknown;  // a key tree of 62 bits is far shallower
    }
    uint32_t used = 0;
    BT(hipMemcpyAsync(&used, S.cnt + 2, 4, hipMemcpyDeviceToHost, s));
    hipLaunchKernelGGL(k_order, dim3(g), dim3(kB), 0, s, sorted, nt, S.order);
    BT(hipGetLastError());
    BT(hipStreamSynchronize(s));
    nodes.resize(used);
    order.resize(nt);
    BT(hipMemcpyAsync(nodes.data(), S.nodes, (size_t)used * sizeof(Node), hipMemcpyDeviceToHost, s));
    BT(hipMemcpyAsync(order.data(), S.order, (size_t)nt * 4, hipMemcpyDeviceToHost, s));
    BT(hipStreamSynchronize(s));
    depth = levels - 1;
    return hipSuccess;
}

// ---- a build scratch region that needs no allocation: a file-scope device
// array of kStaticScratch bytes, resident on every GPU that loads the library
// until the process ends. Host code never passes the array's name to a
// kernel: its device address is looked up once per device.
namespace {
__device__ __align__(256) unsigned char scratch[kStaticScratch];
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};
}  // namespace

hipError_t static_scratch(int device, void **ptr)
{
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        BT(hipGetDevice(&cur));
        if (cur != device) BT(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace qpt
