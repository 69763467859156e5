// GPU BVH builder: a linear BVH (Karras 2012, "Maximizing parallelism in the
// construction of BVHs, octrees, and k-d trees") over Morton-ordered triangle
// centroids, refitted bottom-up and collapsed top-down into the renderer's
// 4-wide node format. The paper builds on the GPU where it can (Sec. 3.1
// cites rapid GPU construction); the binned-SAH host builder stays the
// default, this one trades tree quality for build time.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
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

__global__ void k_order(const unsigned long long *k, uint32_t n, uint32_t *order)
{
    for (uint32_t j = blockIdx.x * kB + threadIdx.x; j < n; j += gridDim.x * kB) order[j] = (uint32_t)(k[j] & 0xffffffffull);
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, std::max<size_t>(bytes, 16)); }
    template <class T> T *as() const { return (T *)p; }
};

}  // namespace

#define BT(x)                                        \
    do {                                             \
        hipError_t e_ = (x);                         \
        if (e_ != hipSuccess) return e_;             \
    } while (0)

hipError_t gpu_build_bvh(const float *pos, uint32_t nv, const uint32_t *idx, uint32_t nt, uint32_t leaf, float pad,
                         hipStream_t s, std::vector<Node> &nodes, std::vector<uint32_t> &order, uint32_t &depth)
{
    const int n = (int)nt;
    DevBuf d_pos, d_idx, d_blo, d_bhi, d_cpart, d_keys, d_sorted, d_tmp, d_child, d_parent, d_range, d_visits, d_box,
        d_q0, d_q1, d_cnt, d_nodes, d_order;
    const uint32_t g = grid_for(nt);
    BT(d_pos.alloc((size_t)nv * 12));
    BT(d_idx.alloc((size_t)nt * 12));
    BT(d_blo.alloc((size_t)nt * 16));
    BT(d_bhi.alloc((size_t)nt * 16));
    BT(d_cpart.alloc((size_t)g * 24));
    BT(hipMemcpyAsync(d_pos.p, pos, (size_t)nv * 12, hipMemcpyHostToDevice, s));
    BT(hipMemcpyAsync(d_idx.p, idx, (size_t)nt * 12, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_prim_boxes, dim3(g), dim3(kB), 0, s, d_pos.as<float>(), d_idx.as<uint32_t>(), nt,
                       d_blo.as<float4>(), d_bhi.as<float4>(), d_cpart.as<float>());
    BT(hipGetLastError());
    std::vector<float> part((size_t)g * 6);
    BT(hipMemcpyAsync(part.data(), d_cpart.p, part.size() * 4, hipMemcpyDeviceToHost, s));
    BT(hipStreamSynchronize(s));
    float cmin[3] = {INFINITY, INFINITY, INFINITY}, cmax[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t b = 0; b < g; ++b)
        for (int a = 0; a < 3; ++a) {
            cmin[a] = std::min(cmin[a], part[6 * b + a]);
            cmax[a] = std::max(cmax[a], part[6 * b + 3 + a]);
        }
    float sc[3];
    for (int a = 0; a < 3; ++a) sc[a] = cmax[a] > cmin[a] ? 1024.0f / (cmax[a] - cmin[a]) : 0.0f;
    BT(d_keys.alloc((size_t)nt * 8));
    BT(d_sorted.alloc((size_t)nt * 8));
    hipLaunchKernelGGL(k_morton, dim3(g), dim3(kB), 0, s, d_blo.as<float4>(), d_bhi.as<float4>(), nt,
                       make_float3(cmin[0], cmin[1], cmin[2]), make_float3(sc[0], sc[1], sc[2]),
                       d_keys.as<unsigned long long>());
    BT(hipGetLastError());
    size_t tmp_bytes = 0;
    BT(hipcub::DeviceRadixSort::SortKeys(nullptr, tmp_bytes, d_keys.as<unsigned long long>(),
                                         d_sorted.as<unsigned long long>(), n, 0, 62, s));
    BT(d_tmp.alloc(tmp_bytes));
    BT(hipcub::DeviceRadixSort::SortKeys(d_tmp.p, tmp_bytes, d_keys.as<unsigned long long>(),
                                         d_sorted.as<unsigned long long>(), n, 0, 62, s));
    const size_t nn = 2 * (size_t)nt - 1;
    BT(d_child.alloc((size_t)nt * 8));
    BT(d_parent.alloc(nn * 4));
    BT(d_range.alloc((size_t)nt * 8));
    BT(d_visits.alloc((size_t)nt * 4));
    BT(d_box.alloc(nn * 24));
    BT(hipMemsetAsync(d_visits.p, 0, (size_t)nt * 4, s));
    hipLaunchKernelGGL(k_hierarchy, dim3(g), dim3(kB), 0, s, d_sorted.as<unsigned long long>(), n, d_child.as<int2>(),
                       d_parent.as<int>(), d_range.as<uint2>());
    BT(hipGetLastError());
    hipLaunchKernelGGL(k_refit, dim3(g), dim3(kB), 0, s, d_sorted.as<unsigned long long>(), d_blo.as<float4>(),
                       d_bhi.as<float4>(), n, d_child.as<int2>(), d_parent.as<int>(), d_visits.as<uint32_t>(),
                       d_box.as<float>());
    BT(hipGetLastError());
    // collapse, one level per launch; a 4-wide node takes at least one binary
    // inner node, so n - 1 slots suffice
    BT(d_nodes.alloc((size_t)nt * sizeof(Node)));
    BT(d_q0.alloc((size_t)nt * 8));
    BT(d_q1.alloc((size_t)nt * 8));
    BT(d_cnt.alloc(16));
    const uint2 root = make_uint2(0u, 0u);
    const uint32_t init[4] = {1u, 0u, 1u, 0u};  // queue 0 count, queue 1 count, nodes used, -
    BT(hipMemcpyAsync(d_q0.p, &root, 8, hipMemcpyHostToDevice, s));
    BT(hipMemcpyAsync(d_cnt.p, init, 16, hipMemcpyHostToDevice, s));
    uint32_t *cnt = d_cnt.as<uint32_t>();
    uint32_t pending = 1, levels = 0;
    while (pending) {
        uint2 *qin = (levels & 1) ? d_q1.as<uint2>() : d_q0.as<uint2>();
        uint2 *qout = (levels & 1) ? d_q0.as<uint2>() : d_q1.as<uint2>();
        uint32_t *nin = cnt + (levels & 1), *nout = cnt + ((levels + 1) & 1);
        const uint32_t zero = 0;
        BT(hipMemcpyAsync(nout, &zero, 4, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_collapse, dim3(grid_for(pending)), dim3(kB), 0, s, qin, nin, qout, nout, cnt + 2, n, leaf,
                           pad, d_child.as<int2>(), d_range.as<uint2>(), d_box.as<float>(), d_nodes.as<Node>());
        BT(hipGetLastError());
        BT(hipMemcpyAsync(&pending, nout, 4, hipMemcpyDeviceToHost, s));
        BT(hipStreamSynchronize(s));
        ++levels;
        if (levels > 128) return hipErrorUnknown;  // a key tree of 62 bits is far shallower
    }
    uint32_t used = 0;
    BT(hipMemcpyAsync(&used, cnt + 2, 4, hipMemcpyDeviceToHost, s));
    BT(d_order.alloc((size_t)nt * 4));
    hipLaunchKernelGGL(k_order, dim3(g), dim3(kB), 0, s, d_sorted.as<unsigned long long>(), nt, d_order.as<uint32_t>());
    BT(hipGetLastError());
    BT(hipStreamSynchronize(s));
    nodes.resize(used);
    order.resize(nt);
    BT(hipMemcpyAsync(nodes.data(), d_nodes.p, (size_t)used * sizeof(Node), hipMemcpyDeviceToHost, s));
    BT(hipMemcpyAsync(order.data(), d_order.p, (size_t)nt * 4, hipMemcpyDeviceToHost, s));
    BT(hipStreamSynchronize(s));
    depth = levels - 1;
    return hipSuccess;
}

}  // namespace qpt
