// Host side of libqpt: context, scene ingest, light and environment tables,
// Halton constant tables, BVH construction, workspace layout and the C-ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <future>
#include <string>
#include <thread>
#include <vector>

#include "qpt.h"
#include "qpt_internal.h"

using namespace qpt;

namespace {

typedef unsigned __int128 u128;

struct Vec3 {
    double x, y, z;
};
inline Vec3 vsub(Vec3 a, Vec3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline Vec3 vadd(Vec3 a, Vec3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline Vec3 vscale(Vec3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline Vec3 vcross(Vec3 a, Vec3 b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double vlen(Vec3 a) { return std::sqrt(a.x * a.x + a.y * a.y + a.z * a.z); }
inline double luminance(double r, double g, double b) { return 0.2126 * r + 0.7152 * g + 0.0722 * b; }

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- Halton

std::vector<uint32_t> first_primes(uint32_t n)
{
    std::vector<uint32_t> p;
    for (uint32_t c = 2; p.size() < n; ++c) {
        bool prime = true;
        for (uint32_t q : p) {
            if (q * q > c) break;
            if (c % q == 0) { prime = false; break; }
        }
        if (prime) p.push_back(c);
    }
    return p;
}

// Granlund-Montgomery round-up multiplier for unsigned division by d of
// N-bit dividends: q = (t + ((n - t) >> 1)) >> (l - 1), t = mulhi(m, n),
// l = ceil(log2 d) >= 1, m = floor(2^N (2^l - d) / d) + 1.
void magic32(uint32_t d, uint32_t *m, uint32_t *sh)
{
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    uint64_t mm = (((uint64_t)1 << 32) * ((1ull << l) - d)) / d + 1;
    *m = (uint32_t)mm;
    *sh = l - 1;
}

void magic64(uint64_t d, uint64_t *m, uint32_t *sh)
{
    uint32_t l = 0;
    while (l < 64 && ((u128)1 << l) < d) ++l;
    u128 mm = (((u128)1 << 64) * (((u128)1 << l) - d)) / d + 1;
    *m = (uint64_t)mm;
    *sh = l - 1;
}

uint32_t scramble_multiplier(uint32_t b)
{
    // round(0.618034 b), kept in [1, b - 1]
    uint64_t f = ((uint64_t)b * 618034u + 500000u) / 1000000u;
    if (f < 1) f = 1;
    if (f > b - 1) f = b - 1;
    return (uint32_t)f;
}

std::vector<HaltonBase> make_bases()
{
    std::vector<uint32_t> pr = first_primes(kMaxDims);
    std::vector<HaltonBase> out(kMaxDims);
    for (uint32_t d = 0; d < kMaxDims; ++d) {
        HaltonBase h{};
        h.b = pr[d];
        h.f = scramble_multiplier(h.b);
        uint64_t B = h.b;
        uint32_t e = 1;
        while (B * h.b < (1ull << 32)) { B *= h.b; ++e; }
        h.e = e;
        h.B = B;
        magic32(h.b, &h.m32, &h.sh32);
        magic64(B, &h.m64, &h.shB);
        out[d] = h;
    }
    return out;
}

// ------------------------------------------------------------------- BVH

struct BuildNode {
    float lo[3], hi[3];
    int32_t left = -1, right = -1;  // inner: child indices
    uint32_t first = 0, count = 0;  // leaf: primitive range
    uint32_t depth = 0;
};

struct PrimInfo {
    float lo[3], hi[3];
    float c[3];
};

struct Builder {
    const std::vector<PrimInfo> &prim;
    std::vector<uint32_t> &order;
    std::vector<BuildNode> nodes;
    std::atomic<uint32_t> next{0};
    uint32_t leaf_size, bins;
    std::atomic<uint32_t> max_depth{0};

    Builder(const std::vector<PrimInfo> &p, std::vector<uint32_t> &o, uint32_t ls, uint32_t nb)
        : prim(p), order(o), leaf_size(ls), bins(nb)
    {
        nodes.resize(std::max<size_t>(2 * p.size(), 2));
    }

    static float area(const float lo[3], const float hi[3])
    {
        float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        if (dx < 0 || dy < 0 || dz < 0) return 0.0f;
        return 2.0f * (dx * dy + dy * dz + dz * dx);
    }

    uint32_t build(uint32_t first, uint32_t count, uint32_t depth, int spawn_budget)
    {
        uint32_t me = next.fetch_add(1);
        BuildNode &nd = nodes[me];
        nd.depth = depth;
        uint32_t md = max_depth.load();
        while (depth > md && !max_depth.compare_exchange_weak(md, depth)) {
        }
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (uint32_t q = first; q < first + count; ++q) {
            const PrimInfo &p = prim[order[q]];
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], p.lo[a]);
                hi[a] = std::max(hi[a], p.hi[a]);
                clo[a] = std::min(clo[a], p.c[a]);
                chi[a] = std::max(chi[a], p.c[a]);
            }
        }
        std::memcpy(nd.lo, lo, sizeof lo);
        std::memcpy(nd.hi, hi, sizeof hi);
        if (count <= leaf_size) {
            nd.first = first;
            nd.count = count;
            return me;
        }
        // levels a balanced split still needs below this node
        uint32_t need = 0;
        while (((uint64_t)leaf_size << need) < count) ++need;
        bool force_median = depth + need + 1 >= kMaxTreeDepth - 1;

        int best_axis = -1;
        uint32_t best_split = 0;
        float best_cost = INFINITY;
        if (!force_median) {
            std::vector<uint32_t> cnt(bins);
            std::vector<float> blo(bins * 3), bhi(bins * 3);
            std::vector<float> rarea(bins);
            std::vector<uint32_t> rcnt(bins);
            for (int a = 0; a < 3; ++a) {
                float ext = chi[a] - clo[a];
                if (!(ext > 0.0f)) continue;
                std::fill(cnt.begin(), cnt.end(), 0u);
                for (uint32_t b = 0; b < bins; ++b)
                    for (int k = 0; k < 3; ++k) { blo[b * 3 + k] = INFINITY; bhi[b * 3 + k] = -INFINITY; }
                float scale = bins / ext;
                for (uint32_t q = first; q < first + count; ++q) {
                    const PrimInfo &p = prim[order[q]];
                    uint32_t b = std::min(bins - 1, (uint32_t)((p.c[a] - clo[a]) * scale));
                    cnt[b]++;
                    for (int k = 0; k < 3; ++k) {
                        blo[b * 3 + k] = std::min(blo[b * 3 + k], p.lo[k]);
                        bhi[b * 3 + k] = std::max(bhi[b * 3 + k], p.hi[k]);
                    }
                }
                float rl[3] = {INFINITY, INFINITY, INFINITY}, rh[3] = {-INFINITY, -INFINITY, -INFINITY};
                uint32_t rc = 0;
                for (uint32_t b = bins - 1; b > 0; --b) {
                    for (int k = 0; k < 3; ++k) {
                        rl[k] = std::min(rl[k], blo[b * 3 + k]);
                        rh[k] = std::max(rh[k], bhi[b * 3 + k]);
                    }
                    rc += cnt[b];
                    rarea[b] = area(rl, rh);
                    rcnt[b] = rc;
                }
                float ll[3] = {INFINITY, INFINITY, INFINITY}, lh[3] = {-INFINITY, -INFINITY, -INFINITY};
                uint32_t lc = 0;
                for (uint32_t b = 0; b + 1 < bins; ++b) {
                    for (int k = 0; k < 3; ++k) {
                        ll[k] = std::min(ll[k], blo[b * 3 + k]);
                        lh[k] = std::max(lh[k], bhi[b * 3 + k]);
                    }
                    lc += cnt[b];
                    if (lc == 0 || rcnt[b + 1] == 0) continue;
                    float cost = area(ll, lh) * lc + rarea[b + 1] * rcnt[b + 1];
                    if (cost < best_cost) { best_cost = cost; best_axis = a; best_split = b + 1; }
                }
            }
        }
        uint32_t mid;
        if (best_axis >= 0) {
            float ext = chi[best_axis] - clo[best_axis];
            float scale = bins / ext;
            int a = best_axis;
            float c0 = clo[a];
            uint32_t nb = bins, sp = best_split;
            auto it = std::partition(order.begin() + first, order.begin() + first + count,
                                     [&](uint32_t q) {
                                         uint32_t b = std::min(nb - 1, (uint32_t)((prim[q].c[a] - c0) * scale));
                                         return b < sp;
                                     });
            mid = (uint32_t)(it - order.begin());
            if (mid == first || mid == first + count) mid = first + count / 2;
        } else {
            // object median on the widest centroid axis (or plain index median)
            int a = 0;
            for (int k = 1; k < 3; ++k)
                if (chi[k] - clo[k] > chi[a] - clo[a]) a = k;
            mid = first + count / 2;
            std::nth_element(order.begin() + first, order.begin() + mid, order.begin() + first + count,
                             [&](uint32_t x, uint32_t y) {
                                 if (prim[x].c[a] != prim[y].c[a]) return prim[x].c[a] < prim[y].c[a];
                                 return x < y;
                             });
        }
        uint32_t l, r;
        if (spawn_budget > 0 && count > 100000) {
            auto fut = std::async(std::launch::async, [&]() {
                return build(first, mid - first, depth + 1, spawn_budget - 1);
            });
            r = build(mid, first + count - mid, depth + 1, spawn_budget - 1);
            l = fut.get();
        } else {
            l = build(first, mid - first, depth + 1, 0);
            r = build(mid, first + count - mid, depth + 1, 0);
        }
        nodes[me].left = (int32_t)l;
        nodes[me].right = (int32_t)r;
        return me;
    }
};

// ------------------------------------------------------------ the context

struct Layout {
    size_t nodes, tris, mats, emit_tri, alias_idx, alias_thr, emit_pmf, lt_nodes, lt_emit, lt_pos, lt_w,
        ep_q, ep_oq, env_texel, env_row,
        env_col, env_cos, bases;
    // per batch lane (two batches in flight): path state, queues, shadow rays, counters, stack
    struct Lane {
        size_t ray_o, ray_d, hit, thr, rad, idx, q0, q1, qdead, pv, sh_o, sh_d, sh_c, counters, gstack;
    } lane[2];
    size_t stats;
    size_t fb_sum, fb_count;
    size_t g_frag, g_fragT, g_bias, g_rec[2], g_ring, g_ring_head, g_master, g_m, g_v, g_partial, g_scalars;
    size_t g_pub_frag[2], g_pub_bias[2];
    size_t total;
};

}  // namespace

namespace {
// events bracketing each kernel launch, read back once at the end
struct EventProfiler : qpt::Profiler {
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    hipEvent_t take()
    {
        if (used == pool.size()) {
            hipEvent_t e;
            // timing only: without the system-scope fence an event costs no
            // cache writeback and invalidation between the kernels it brackets
            // (with it, a launch's event span came out 11% longer than the
            // kernel's own duration in a kernel trace of the same run)
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    void begin(int kind, hipStream_t s) override
    {
        hipEvent_t e = take();
        if (e) (void)hipEventRecord(e, s);
        recs.push_back({kind, e, nullptr});
    }
    void end(int, hipStream_t s) override
    {
        hipEvent_t e = take();
        if (e) (void)hipEventRecord(e, s);
        recs.back().b = e;
    }
    void kernel_events(int kind, hipEvent_t *start, hipEvent_t *stop) override
    {
        *start = take();
        *stop = *start ? take() : nullptr;
        if (!*stop) *start = nullptr;
        recs.push_back({kind, *start, *stop});
    }
    void clear()
    {
        recs.clear();
        used = 0;
    }
    ~EventProfiler() override
    {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};
}  // namespace

struct qpt_ctx {
    int device = -1;
    uint32_t trav_threads = 0;  // traversal grid: CUs x resident blocks per CU x block size
    uint32_t guide_blocks = 256;  // training blocks (one per CU)
    GuideTrain gt{};
    qpt_guide_opts gopts{0.0f, 1e-3f, 1u << 18, 0, 1, 0, 0};
    bool guide_weights = false;
    uint32_t guide_steps = 0;
    uint32_t stack_need = 3;      // traversal stack entries per ray the BVH can require
    // training runs on the lane that rendered the batch, right after it
    bool own_lstream = false;                        // created here (else the caller's, not destroyed)
    void *static_scratch = nullptr;                  // this device's allocation-free build region
    hipEvent_t ev_train[2] = {nullptr, nullptr};  // the step publishing into buffer k has finished
    hipEvent_t ev_tdone = nullptr;                // the latest batch's samples and steps are done
    bool train_pending[2] = {false, false};
    bool tdone_pending = false;
    uint64_t gbatch = 0;   // training batches issued
    int last_buf = 0;      // buffer of the newest published weights
    uint2 *pub_frag[2] = {nullptr, nullptr};
    float *pub_bias[2] = {nullptr, nullptr};
    double bbox[6] = {0, 0, 0, 1, 1, 1};
    EventProfiler prof;
    bool profiling = false;
    hipStream_t stream = nullptr;
    std::string err;
    bool scene_ok = false, bvh_ok = false, bound = false;
    // scene (host copies)
    uint32_t W = 0, H = 0;
    std::vector<float> pos;
    std::vector<uint32_t> idx, tri_mat;
    std::vector<qpt_material> mats;
    uint32_t ew = 0, eh = 0;
    std::vector<float> env;
    qpt_camera cam{};
    // lights (emitter order: ascending input triangle id)
    std::vector<uint32_t> emit_input_tri;
    std::vector<double> emit_flux, alias_prob, emit_pmf;
    std::vector<uint32_t> alias_idx;
    std::vector<unsigned long long> alias_thr;
    std::vector<int32_t> tri_emit;
    double p_env = 0.0;
    // light tree (node 0 = root) and its leaf order of the emitters
    std::vector<LtNode> lt_nodes;
    std::vector<uint32_t> lt_emit, lt_pos, lt_w;
    // environment tables
    std::vector<uint32_t> env_row, env_col;
    std::vector<float4> env_texel;
    std::vector<float> env_cos;
    // environment pyramid: finest level (0 = none), normal-weighted levels,
    // left-root probability, 4 words per node (shared; then per normal bin)
    uint32_t ep_m = 0, ep_top = 0, ep_root = 0;
    std::vector<uint32_t> ep_q, ep_oq;
    // Halton + enumeration
    std::vector<HaltonBase> bases;
    Frame frame{};
    // BVH in GPU layout
    std::vector<Node> gnodes;
    uint32_t node_format = kNodeQuant;   // of the device tree (qpt_bvh_opts.node_format)
    std::vector<Tri> gtris;
    std::vector<Material> gmats;
    std::vector<uint32_t> emit_tri_bvh;
    // workspace
    uint8_t *ws = nullptr;
    size_t ws_bytes = 0;
    uint32_t pool_cap = 0;
    Layout lay{};
    Pool pool{};     // lane 0 (the caller's stream); the guide, debug hooks and readback use it
    Pool pool_b{};   // lane 1 (the library's second stream)
    // two batches in flight: lane 1's stream, and the events that order the
    // lanes against the caller's stream and the framebuffer updates in pass order
    hipStream_t lstream = nullptr;
    hipEvent_t ev_lane_in = nullptr, ev_lane_out = nullptr, ev_acc = nullptr;
    hipEvent_t ev_regen[2] = {nullptr, nullptr};  // regeneration: a chunk of iterations has copied its paths left
    uint32_t *abort_host = nullptr;              // pinned, mapped: the caller's stop request (word 0)
    uint32_t *abort_dev = nullptr;               // its device address
    float4 *lane_rec[2] = {nullptr, nullptr};    // per lane: training records
    uint64_t batches = 0;
    // the most recent batch (for the record hook): its lane, pixel range and passes
    struct {
        bool valid = false;
        int lane = 0;
        uint32_t p0 = 0, np = 0, nb = 0;
        uint64_t pass0 = 0;
    } last_batch;
};

namespace {

int fail(qpt_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

// Make ctx->device current for the duration of a call and restore the caller's.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (dev < 0) return;
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

#define HIP_TRY(ctx, expr)                                                              \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(ctx, QPT_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

Vec3 corner(const qpt_ctx *c, uint32_t t, int k)
{
    const float *p = &c->pos[3 * (size_t)c->idx[3 * (size_t)t + k]];
    return {p[0], p[1], p[2]};
}

// emission of material m at x (front face)
Vec3 emission_at(const qpt_material &m, Vec3 x)
{
    Vec3 E = {m.emission[0], m.emission[1], m.emission[2]};
    if (m.flags & QPT_MAT_EMIT_TEXTURE) {
        double k = 0.55 + 0.45 * std::sin(2.0 * kPi * 4.0 * (x.x + x.z));
        E = vscale(E, k);
    }
    return E;
}

// pi * area * lum(mean emission); mean over the 16 cell centroids of the
// 4x4 split, upright cell (i, j) then inverted cell (i, j), i outer, j inner
double triangle_flux(const qpt_ctx *c, uint32_t t)
{
    Vec3 a = corner(c, t, 0), b = corner(c, t, 1), d = corner(c, t, 2);
    const qpt_material &m = c->mats[c->tri_mat[t]];
    double area = 0.5 * vlen(vcross(vsub(b, a), vsub(d, a)));
    const int n = 4;
    double acc = 0.0;
    auto point = [&](double u, double v) { return vadd(a, vadd(vscale(vsub(b, a), u), vscale(vsub(d, a), v))); };
    for (int i = 0; i < n; ++i)
        for (int j = 0; i + j < n; ++j) {
            Vec3 E = emission_at(m, point((i + 1.0 / 3.0) / n, (j + 1.0 / 3.0) / n));
            acc += luminance(E.x, E.y, E.z);
            if (i + j < n - 1) {
                E = emission_at(m, point((i + 2.0 / 3.0) / n, (j + 2.0 / 3.0) / n));
                acc += luminance(E.x, E.y, E.z);
            }
        }
    return kPi * area * acc / (double)(n * n);
}

// Vose alias table with index-ordered FIFO worklists (FP64)
void build_alias(const std::vector<double> &w, std::vector<double> &prob, std::vector<uint32_t> &alias)
{
    size_t n = w.size();
    prob.assign(n, 1.0);
    alias.resize(n);
    double sum = 0.0;
    for (double x : w) sum += x;
    std::vector<double> q(n);
    std::vector<uint32_t> small, large;
    small.reserve(n);
    large.reserve(n);
    for (size_t i = 0; i < n; ++i) {
        q[i] = (w[i] * (double)n) / sum;
        (q[i] < 1.0 ? small : large).push_back((uint32_t)i);
        alias[i] = (uint32_t)i;
    }
    size_t sh = 0, lh = 0;
    while (sh < small.size() && lh < large.size()) {
        uint32_t s = small[sh++], l = large[lh];
        prob[s] = q[s];
        alias[s] = l;
        q[l] = (q[l] + q[s]) - 1.0;
        if (q[l] < 1.0) {
            ++lh;
            small.push_back(l);
        }
    }
    // leftovers keep prob 1 and alias = self
}

void build_lights(qpt_ctx *c)
{
    uint32_t nt = (uint32_t)c->tri_mat.size();
    c->emit_input_tri.clear();
    c->tri_emit.assign(nt, -1);
    for (uint32_t t = 0; t < nt; ++t) {
        const qpt_material &m = c->mats[c->tri_mat[t]];
        if (m.emission[0] > 0 || m.emission[1] > 0 || m.emission[2] > 0) {
            c->tri_emit[t] = (int32_t)c->emit_input_tri.size();
            c->emit_input_tri.push_back(t);
        }
    }
    size_t ne = c->emit_input_tri.size();
    c->emit_flux.resize(ne);
    for (size_t e = 0; e < ne; ++e) c->emit_flux[e] = triangle_flux(c, c->emit_input_tri[e]);
    c->alias_prob.clear();
    c->alias_idx.clear();
    c->alias_thr.clear();
    c->emit_pmf.assign(ne, 0.0);
    if (!ne) return;
    build_alias(c->emit_flux, c->alias_prob, c->alias_idx);
    c->alias_thr.resize(ne);
    for (size_t e = 0; e < ne; ++e)
        c->alias_thr[e] = (unsigned long long)std::ceil(c->alias_prob[e] * 4294967296.0);
}

// Light tree over the emitters (the hierarchy of Sec. 2.1.1). Each node takes
// its emitter range in the order its parent's sort left it, accumulates its
// corner box, centroid box and region fluxes over that range in FP64, then
// sorts the range by centroid along the centroid box's longest axis (ties:
// emitter index) and hands the lower half to the first of two adjacent
// children. Nodes are numbered in depth-first order, left subtree first.
// The importance estimate on the device bounds the emission cosine of a
// region's triangles by the cone of half-angle acos(1/sqrt 3) that holds
// the region.
double region_cos_bound(Vec3 n, int region)
{
    double s = (region & 1) ? -1.0 : 1.0;
    double c = s * (region < 2 ? n.x : region < 4 ? n.y : n.z);
    double ang = std::acos(std::max(-1.0, std::min(1.0, c)));
    double half = std::acos(1.0 / std::sqrt(3.0));
    if (ang <= half) return 1.0;
    return std::max(0.0, std::cos(ang - half));
}

void build_light_tree(qpt_ctx *c)
{
    const uint32_t ne = (uint32_t)c->emit_input_tri.size();
    c->lt_nodes.clear();
    c->lt_emit.clear();
    c->lt_pos.clear();
    c->lt_w.clear();
    if (!ne) return;
    std::vector<Vec3> cen(ne), nrm(ne);
    for (uint32_t e = 0; e < ne; ++e) {
        uint32_t t = c->emit_input_tri[e];
        Vec3 a = corner(c, t, 0), b = corner(c, t, 1), d = corner(c, t, 2);
        cen[e] = vscale(vadd(vadd(a, b), d), 1.0 / 3.0);
        Vec3 n = vcross(vsub(b, a), vsub(d, a));
        double l = vlen(n);
        nrm[e] = l > 0.0 ? vscale(n, 1.0 / l) : Vec3{0.0, 0.0, 1.0};
    }
    std::vector<uint32_t> &ord = c->lt_emit;
    ord.resize(ne);
    for (uint32_t e = 0; e < ne; ++e) ord[e] = e;
    c->lt_w.assign(ne, 0);
    c->lt_nodes.assign(2 * (size_t)ne, LtNode{});
    struct Work {
        uint32_t node, first, count;
    };
    std::vector<Work> todo{{0, 0, ne}};
    uint32_t next = 1;
    while (!todo.empty()) {
        Work wk = todo.back();
        todo.pop_back();
        const uint32_t first = wk.first, count = wk.count, end = first + count;
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double fl[6] = {0, 0, 0, 0, 0, 0};
        for (uint32_t q = first; q < end; ++q) {
            uint32_t e = ord[q], t = c->emit_input_tri[e];
            for (int k = 0; k < 3; ++k) {
                Vec3 p = corner(c, t, k);
                const double pv[3] = {p.x, p.y, p.z};
                for (int a = 0; a < 3; ++a) {
                    lo[a] = std::fmin(lo[a], pv[a]);
                    hi[a] = std::fmax(hi[a], pv[a]);
                }
            }
            const double cv[3] = {cen[e].x, cen[e].y, cen[e].z};
            for (int a = 0; a < 3; ++a) {
                clo[a] = std::fmin(clo[a], cv[a]);
                chi[a] = std::fmax(chi[a], cv[a]);
            }
            for (int r = 0; r < 6; ++r) fl[r] += c->emit_flux[e] * region_cos_bound(nrm[e], r);
        }
        LtNode &nd = c->lt_nodes[wk.node];
        Vec3 mid = vscale(vadd(Vec3{lo[0], lo[1], lo[2]}, Vec3{hi[0], hi[1], hi[2]}), 0.5);
        double radius = 0.5 * vlen(vsub(Vec3{hi[0], hi[1], hi[2]}, Vec3{lo[0], lo[1], lo[2]}));
        nd.sphere = make_float4((float)mid.x, (float)mid.y, (float)mid.z, (float)radius);
        for (int r = 0; r < 6; ++r) nd.flux[r] = (float)fl[r];
        nd.first = first;
        nd.count = count;
        if (count <= kLtLeaf) {
            // cumulative flux fractions in 24 bits (equal shares if the leaf has none)
            nd.left = -1;
            double total = 0.0, run = 0.0;
            for (uint32_t q = first; q < end; ++q) total += c->emit_flux[ord[q]];
            for (uint32_t q = first; q < end; ++q) {
                double frac = total > 0.0 ? run / total : (double)(q - first) / (double)count;
                c->lt_w[q] = (uint32_t)std::nearbyint(frac * 16777216.0);
                run += c->emit_flux[ord[q]];
            }
            continue;
        }
        const double ext[3] = {chi[0] - clo[0], chi[1] - clo[1], chi[2] - clo[2]};
        int axis = ext[1] > ext[0] ? 1 : 0;
        if (ext[2] > ext[axis]) axis = 2;
        auto key = [&](uint32_t e) { return axis == 0 ? cen[e].x : axis == 1 ? cen[e].y : cen[e].z; };
        std::sort(ord.begin() + first, ord.begin() + end, [&](uint32_t x, uint32_t y) {
            double kx = key(x), ky = key(y);
            return kx != ky ? kx < ky : x < y;
        });
        const uint32_t half = count / 2, l = next;
        next += 2;
        nd.left = (int32_t)l;
        todo.push_back({l + 1, first + half, count - half});
        todo.push_back({l, first, half});
    }
    c->lt_nodes.resize(next);
    c->lt_pos.assign(ne, 0);
    for (uint32_t q = 0; q < ne; ++q) c->lt_pos[ord[q]] = q;
}

// probability the integer light-selection rule realises for each emitter
void build_light_pmf(qpt_ctx *c)
{
    size_t ne = c->emit_input_tri.size();
    if (!ne) return;
    uint64_t R = c->ew ? (1ull << 31) : (1ull << 32);
    double ptri = 1.0 - c->p_env;
    for (size_t col = 0; col < ne; ++col) {
        // #{r in [0, R) : floor(r ne / R) == col}
        u128 hi = ((u128)(col + 1) * R + ne - 1) / ne, lo = ((u128)col * R + ne - 1) / ne;
        double pc = (double)(uint64_t)(hi - lo) / (double)R;
        double take = (double)c->alias_thr[col] / 4294967296.0;
        c->emit_pmf[col] += ptri * pc * take;
        c->emit_pmf[c->alias_idx[col]] += ptri * pc * (1.0 - take);
    }
}

// ------------------------------------------------- environment pyramid
//
// Hierarchical sampling of the lat-long map (Sec. 2.1.2). Level m holds the
// texels' intensity x solid angle (W = 2^(m+1), H = 2^m), level k < m the
// sums ((a + b) + c) + d of its 2 x 2 children (a, b the upper row, left
// first); a node's split is its children's column share, then the row share
// within the chosen column, each a 24-bit probability. Per normal bin (16 x 16
// octahedral cells, +y up) the levels above kEpTop use weights of the
// level-kEpTop cells scaled by a bound of the cosine between any normal of
// the bin and any direction of the cell, from bounding cones of both.
constexpr uint32_t kEpBins = 16, kEpTop = 5;

uint32_t ep_nodes_above(uint32_t k) { return (uint32_t)((2ull * ((1ull << (2 * k)) - 1)) / 3); }

uint32_t ep_share(double l, double r)
{
    if (!(l + r > 0.0)) return 1u << 23;
    double q = std::nearbyint(l / (l + r) * 16777216.0);
    if (l > 0.0 && q < 1.0) q = 1.0;
    if (r > 0.0 && q > 16777215.0) q = 16777215.0;
    return (uint32_t)q;
}

// splits of levels 0..top-1 from the weights of level `top` (2^(top+1) x 2^top, row-major)
void ep_fill_splits(const std::vector<double> &level_top, uint32_t top, uint32_t &root, uint32_t *q)
{
    std::vector<double> fine = level_top, coarse;
    for (uint32_t k = top; k-- > 0;) {
        const uint32_t w = 2u << k, h = 1u << k, fw = 2 * w;
        coarse.assign((size_t)w * h, 0.0);
        for (uint32_t y = 0; y < h; ++y)
            for (uint32_t x = 0; x < w; ++x) {
                const double a = fine[(size_t)(2 * y) * fw + 2 * x], b = fine[(size_t)(2 * y) * fw + 2 * x + 1];
                const double cc = fine[(size_t)(2 * y + 1) * fw + 2 * x];
                const double d = fine[(size_t)(2 * y + 1) * fw + 2 * x + 1];
                uint32_t *o = q + 4 * ((size_t)ep_nodes_above(k) + (size_t)y * w + x);
                o[0] = ep_share(a + cc, b + d);
                o[1] = ep_share(a, cc);
                o[2] = ep_share(b, d);
                o[3] = 0;
                coarse[(size_t)y * w + x] = ((a + b) + cc) + d;
            }
        fine.swap(coarse);
    }
    root = ep_share(fine[0], fine[1]);
}

Vec3 ep_direction(double theta, double phi)
{
    return {std::sin(theta) * std::sin(phi), std::cos(theta), -std::sin(theta) * std::cos(phi)};
}

double ep_angle(Vec3 a, Vec3 b)
{
    double d = a.x * b.x + a.y * b.y + a.z * b.z;
    return std::acos(std::max(-1.0, std::min(1.0, d)));
}

Vec3 ep_from_octahedral(double px, double pz)
{
    double y = 1.0 - std::fabs(px) - std::fabs(pz);
    if (y < 0.0) {
        const double fx = (1.0 - std::fabs(pz)) * (px >= 0.0 ? 1.0 : -1.0);
        const double fz = (1.0 - std::fabs(px)) * (pz >= 0.0 ? 1.0 : -1.0);
        px = fx;
        pz = fz;
    }
    Vec3 n{px, y, pz};
    return vscale(n, 1.0 / vlen(n));
}

void build_env_pyramid(qpt_ctx *c)
{
    c->ep_m = c->ep_top = c->ep_root = 0;
    c->ep_q.clear();
    c->ep_oq.clear();
    const uint32_t W = c->ew, H = c->eh;
    uint32_t m = 0;
    while ((1u << m) < H) ++m;
    if (m < 1 || H != (1u << m) || W != 2 * H) return;
    const uint32_t top = std::min(m, kEpTop);
    // texel weights, then sums down to level `top`
    std::vector<double> lvl((size_t)W * H);
    for (uint32_t r = 0; r < H; ++r) {
        const double om = (2.0 * kPi / W) * (std::cos(kPi * r / H) - std::cos(kPi * (r + 1) / H));
        for (uint32_t x = 0; x < W; ++x) {
            const float *L = &c->env[3 * ((size_t)r * W + x)];
            lvl[(size_t)r * W + x] = luminance(L[0], L[1], L[2]) * om;
        }
    }
    c->ep_q.assign(4 * (size_t)ep_nodes_above(m), 0);
    ep_fill_splits(lvl, m, c->ep_root, c->ep_q.data());
    for (uint32_t k = m; k > top; --k) {
        const uint32_t w = 1u << k, h = 1u << (k - 1), fw = 2 * w;
        std::vector<double> up((size_t)w * h);
        for (uint32_t y = 0; y < h; ++y)
            for (uint32_t x = 0; x < w; ++x) {
                const double a = lvl[(size_t)(2 * y) * fw + 2 * x], b = lvl[(size_t)(2 * y) * fw + 2 * x + 1];
                const double cc = lvl[(size_t)(2 * y + 1) * fw + 2 * x];
                const double d = lvl[(size_t)(2 * y + 1) * fw + 2 * x + 1];
                up[(size_t)y * w + x] = ((a + b) + cc) + d;
            }
        lvl.swap(up);
    }
    // bounding cones of the level-`top` cells
    const uint32_t tw = 2u << top, th = 1u << top;
    std::vector<Vec3> cell_axis((size_t)tw * th);
    std::vector<double> cell_half((size_t)tw * th);
    for (uint32_t y = 0; y < th; ++y)
        for (uint32_t x = 0; x < tw; ++x) {
            const double t0 = kPi * y / th, t1 = kPi * (y + 1) / th;
            const double p0 = 2.0 * kPi * x / tw, p1 = 2.0 * kPi * (x + 1) / tw;
            const Vec3 a = ep_direction(0.5 * (t0 + t1), 0.5 * (p0 + p1));
            const double h0 = std::max(ep_angle(a, ep_direction(t0, p0)), ep_angle(a, ep_direction(t0, p1)));
            const double h1 = std::max(ep_angle(a, ep_direction(t1, p0)), ep_angle(a, ep_direction(t1, p1)));
            cell_axis[(size_t)y * tw + x] = a;
            cell_half[(size_t)y * tw + x] = std::max(h0, h1) + 0.01;
        }
    const size_t per = 4 * (1 + (size_t)ep_nodes_above(top));
    c->ep_oq.assign((size_t)kEpBins * kEpBins * per, 0);
    std::vector<double> scaled((size_t)tw * th);
    const double side = 2.0 / kEpBins;
    for (uint32_t b = 0; b < kEpBins * kEpBins; ++b) {
        const double x0 = -1.0 + side * (b % kEpBins), z0 = -1.0 + side * (b / kEpBins);
        const Vec3 axis = ep_from_octahedral(x0 + 0.5 * side, z0 + 0.5 * side);
        double half = 0.0;
        for (int e = 0; e <= 16; ++e) {
            const double f = e / 16.0;
            half = std::max(half, ep_angle(axis, ep_from_octahedral(x0 + f * side, z0)));
            half = std::max(half, ep_angle(axis, ep_from_octahedral(x0 + f * side, z0 + side)));
            half = std::max(half, ep_angle(axis, ep_from_octahedral(x0, z0 + f * side)));
            half = std::max(half, ep_angle(axis, ep_from_octahedral(x0 + side, z0 + f * side)));
        }
        half += 0.02;
        for (size_t q = 0; q < scaled.size(); ++q) {
            const double gap = ep_angle(axis, cell_axis[q]) - half - cell_half[q];
            const double bound = gap <= 0.0 ? 1.0 : (gap >= 0.5 * kPi ? 0.0 : std::cos(gap));
            scaled[q] = lvl[q] * bound;
        }
        uint32_t *o = c->ep_oq.data() + (size_t)b * per;
        ep_fill_splits(scaled, top, o[0], o + 4);
    }
    c->ep_m = m;
    c->ep_top = top;
}

void build_env(qpt_ctx *c)
{
    uint32_t W = c->ew, H = c->eh;
    c->env_row.assign(H, 0);
    c->env_col.assign((size_t)W * H, 0);
    c->env_texel.resize((size_t)W * H);
    c->env_cos.resize(H + 1);
    for (uint32_t r = 0; r <= H; ++r) c->env_cos[r] = (float)std::cos(kPi * r / H);
    std::vector<double> rowsum(H), cdf(W + 1), omega(H);
    std::vector<uint64_t> colq((size_t)H * (W + 1));
    for (uint32_t r = 0; r < H; ++r) {
        double om = (2.0 * kPi / W) * (std::cos(kPi * r / H) - std::cos(kPi * (r + 1) / H));
        omega[r] = om;
        cdf[0] = 0.0;
        for (uint32_t x = 0; x < W; ++x) {
            const float *L = &c->env[((size_t)r * W + x) * 3];
            cdf[x + 1] = cdf[x] + luminance(L[0], L[1], L[2]) * om;
        }
        rowsum[r] = cdf[W];
        uint64_t *q = &colq[(size_t)r * (W + 1)];
        for (uint32_t x = 0; x < W; ++x)
            q[x] = cdf[W] > 0.0 ? (uint64_t)std::floor(cdf[x] / cdf[W] * 4294967296.0)
                                : (uint64_t)(((u128)x << 32) / W);
        q[W] = 1ull << 32;
    }
    std::vector<double> C(H + 1);
    C[0] = 0.0;
    for (uint32_t r = 0; r < H; ++r) C[r + 1] = C[r] + rowsum[r];
    std::vector<uint64_t> rowq(H + 1);
    for (uint32_t r = 0; r < H; ++r) rowq[r] = (uint64_t)std::floor(C[r] / C[H] * 4294967296.0);
    rowq[H] = 1ull << 32;
    for (uint32_t r = 0; r < H; ++r) {
        c->env_row[r] = (uint32_t)rowq[r];
        double pr = (double)(rowq[r + 1] - rowq[r]) / 4294967296.0;
        const uint64_t *q = &colq[(size_t)r * (W + 1)];
        for (uint32_t x = 0; x < W; ++x) {
            c->env_col[(size_t)r * W + x] = (uint32_t)q[x];
            double pc = (double)(q[x + 1] - q[x]) / 4294967296.0;
            const float *L = &c->env[((size_t)r * W + x) * 3];
            c->env_texel[(size_t)r * W + x] = make_float4(L[0], L[1], L[2], (float)(pr * pc / omega[r]));
        }
    }
}

void set_frame_constants(qpt_ctx *c)
{
    Frame &f = c->frame;
    f.W = c->W;
    f.H = c->H;
    uint32_t k = 0, l = 0;
    uint64_t p2 = 1, p3 = 1;
    while (p2 < c->W) { p2 *= 2; ++k; }
    while (p3 < c->H) { p3 *= 3; ++l; }
    f.k2 = k;
    f.l3 = l;
    f.p3 = p3;
    f.S = p2 * p3;
    if (p3 > 1) magic64(p3, &f.m_p3, &f.sh_p3);
    else { f.m_p3 = 0; f.sh_p3 = 0; }
    // (2^k)^-1 mod 3^l by search (3^l is small)
    f.inv2k_mod_p3 = 0;
    for (uint64_t x = 0; x < p3; ++x)
        if ((p2 % p3) * x % p3 == 1 % p3) { f.inv2k_mod_p3 = (uint32_t)x; break; }
    // camera basis in FP64, rounded once
    Vec3 eye = {c->cam.eye[0], c->cam.eye[1], c->cam.eye[2]};
    Vec3 look = {c->cam.look[0], c->cam.look[1], c->cam.look[2]};
    Vec3 up = {c->cam.up[0], c->cam.up[1], c->cam.up[2]};
    Vec3 fwd = vsub(look, eye);
    fwd = vscale(fwd, 1.0 / vlen(fwd));
    Vec3 right = vcross(fwd, up);
    right = vscale(right, 1.0 / vlen(right));
    Vec3 u = vcross(right, fwd);
    float *dst[4] = {f.cam.eye, f.cam.fwd, f.cam.right, f.cam.up};
    Vec3 src[4] = {eye, fwd, right, u};
    for (int q = 0; q < 4; ++q) {
        dst[q][0] = (float)src[q].x;
        dst[q][1] = (float)src[q].y;
        dst[q][2] = (float)src[q].z;
    }
    f.cam.tan_half = (float)std::tan(0.5 * c->cam.vfov_deg * kPi / 180.0);
    f.cam.aspect = (float)((double)c->W / (double)c->H);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// paths per batch when the caller leaves it to the library: sixteen frames'
// worth (a power of two in [2^16, 2^27]; two such pools take 16 GB at 1080p
// and 40 GB at 4K with the guide's buffers); batches of several one-sample
// passes keep the short queues of deep vertices full
uint32_t default_pool(const qpt_ctx *c)
{
    uint64_t want = 16ull * c->W * c->H, cap = 1u << 16;
    while (cap < want && cap < (1u << 27)) cap <<= 1;
    return (uint32_t)cap;
}

// training records per batch (vertices 1..max_vertex of each path, or a
// hashed subset of the vertices when that would overflow)
size_t guide_rec_cap(uint32_t cap) { return std::min<size_t>((size_t)1 << 22, (size_t)cap * 2); }
constexpr uint32_t kGuideRing = 1u << 20;   // replay samples kept

Layout make_layout(const qpt_ctx *c, uint32_t cap)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + std::max<size_t>(bytes, 1));
        return at;
    };
    L.nodes = take(c->gnodes.size() * (c->node_format == kNodeQuant ? sizeof(QNode) : sizeof(Node)));
    L.tris = take(c->gtris.size() * sizeof(Tri));
    L.mats = take(c->gmats.size() * sizeof(Material));
    size_t ne = c->emit_input_tri.size();
    L.emit_tri = take(ne * 4);
    L.alias_idx = take(ne * 4);
    L.alias_thr = take(ne * 8);
    L.emit_pmf = take(ne * 4);
    L.lt_nodes = take(c->lt_nodes.size() * sizeof(LtNode));
    L.lt_emit = take(ne * 4);
    L.lt_pos = take(ne * 4);
    L.lt_w = take(ne * 4);
    L.ep_q = take(c->ep_q.size() * 4);
    L.ep_oq = take(c->ep_oq.size() * 4);
    L.env_texel = take(c->env_texel.size() * sizeof(float4));
    L.env_row = take(c->env_row.size() * 4);
    L.env_col = take(c->env_col.size() * 4);
    L.env_cos = take(c->env_cos.size() * 4);
    L.bases = take(kMaxDims * sizeof(HaltonBase));
    for (int lane = 0; lane < 2; ++lane) {
        Layout::Lane &ln = L.lane[lane];
        ln.ray_o = take((size_t)cap * 16);
        ln.ray_d = take((size_t)cap * 16);
        ln.hit = take((size_t)cap * 16);
        ln.thr = take((size_t)cap * 16);
        ln.rad = take((size_t)cap * 16);
        ln.idx = take((size_t)cap * 8);
        ln.q0 = take((size_t)cap * 4);
        ln.q1 = take((size_t)cap * 4);
        ln.qdead = take((size_t)cap * 4);
        ln.pv = take(lane == 0 ? (size_t)cap * 8 : 0);   // regeneration runs on the first lane only
        ln.sh_o = take((size_t)cap * 16);
        ln.sh_d = take((size_t)cap * 16);
        ln.sh_c = take((size_t)cap * 16);
        ln.counters = take(kCounters * 4);
        ln.gstack = take((size_t)c->trav_threads * (c->stack_need > kShortStack ? c->stack_need - kShortStack : 1u) * 4);
    }
    L.stats = take(8 * 8);
    L.fb_sum = take((size_t)c->W * c->H * 3 * 8);
    L.fb_count = take((size_t)c->W * c->H * 4);
    // learned proposal: weights, training records, the
    // replay ring and optimiser state; the renderer's copy of the weights is
    // double-buffered so a training step overlaps the next batch
    size_t rec_cap = guide_rec_cap(cap);
    L.g_frag = take(kGuideFrags * 64 * 8);
    L.g_fragT = take(kGuideFragsT * 64 * 8);
    L.g_bias = take(256 * 4);
    for (int k = 0; k < 2; ++k) L.g_rec[k] = take(rec_cap * kRecF4 * 16);  // per lane: its training records
    L.g_ring = take((size_t)kGuideRing * kRingF4 * 16);
    L.g_ring_head = take(4);
    for (int k = 0; k < 2; ++k) {
        L.g_pub_frag[k] = take(kGuideFrags * 64 * 8);
        L.g_pub_bias[k] = take(256 * 4);
    }
    L.g_master = take(kGuideParams * 4);
    L.g_m = take(kGuideParams * 4);
    L.g_v = take(kGuideParams * 4);
    L.g_partial = take((size_t)c->guide_blocks * kGuideParams * 4);
    L.g_scalars = take((2 + 2 * (size_t)c->guide_blocks) * 4);  // totals, then per training block
    L.total = o;
    return L;
}

}  // namespace

// ================================================================== C-ABI

extern "C" {

int qpt_create(int hip_device, void *hip_stream, qpt_ctx **out)
{
    if (!out) return QPT_E_INVALID;
    *out = nullptr;
    qpt_ctx *c = new (std::nothrow) qpt_ctx();
    if (!c) return QPT_E_NOMEM;
    c->device = hip_device;
    c->stream = (hipStream_t)hip_stream;
    c->bases = make_bases();
    c->trav_threads = 256 * kTravBlocksPerCU * kBlock;  // host-only contexts: sizing only
    if (hip_device >= 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
            delete c;
            return QPT_E_HIP;
        }
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            delete c;
            return QPT_E_UNSUPPORTED;
        }
        c->trav_threads = (uint32_t)prop.multiProcessorCount * kTravBlocksPerCU * kBlock;
        c->guide_blocks = (uint32_t)prop.multiProcessorCount;
        // this device's address of the allocation-free build region (looked up once per device)
        if (static_scratch(hip_device, &c->static_scratch) != hipSuccess) {
            delete c;
            return QPT_E_HIP;
        }
    }
    *out = c;
    return QPT_OK;
}

void qpt_destroy(qpt_ctx *ctx)
{
    if (!ctx) return;
    for (int k = 0; k < 2; ++k) {
        DeviceGuard g(ctx->device);
        if (ctx->ev_train[k]) (void)hipEventDestroy(ctx->ev_train[k]);
    }
    if (ctx->ev_tdone) {
        DeviceGuard g(ctx->device);
        (void)hipEventDestroy(ctx->ev_tdone);
    }
    if (ctx->ev_lane_in) {
        DeviceGuard g(ctx->device);
        if (ctx->lstream) (void)hipStreamSynchronize(ctx->lstream);
        (void)hipEventDestroy(ctx->ev_lane_in);
        (void)hipEventDestroy(ctx->ev_lane_out);
        (void)hipEventDestroy(ctx->ev_acc);
        for (int k = 0; k < 2; ++k)
            if (ctx->ev_regen[k]) (void)hipEventDestroy(ctx->ev_regen[k]);
        if (ctx->abort_host) (void)hipHostFree(ctx->abort_host);
    }
    if (ctx->lstream && ctx->own_lstream) {
        DeviceGuard g(ctx->device);
        (void)hipStreamDestroy(ctx->lstream);
    }
    delete ctx;
}

int qpt_set_streams(qpt_ctx *c, void *lane_stream)
{
    if (!c || !lane_stream) return QPT_E_INVALID;
    if (c->device < 0) return fail(c, QPT_E_STATE, "context has no device");
    if (c->ev_lane_in) return fail(c, QPT_E_STATE, "set_streams after the first bind_workspace");
    if ((hipStream_t)lane_stream == c->stream) return fail(c, QPT_E_INVALID, "the second lane needs a stream of its own");
    c->lstream = (hipStream_t)lane_stream;
    c->own_lstream = false;
    return QPT_OK;
}

const char *qpt_last_error(const qpt_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int qpt_build_scene(qpt_ctx *c, const qpt_scene_desc *d)
{
    if (!c || !d) return QPT_E_INVALID;
    c->scene_ok = c->bvh_ok = c->bound = false;
    c->err.clear();
    if (!d->positions || !d->indices || !d->tri_material || !d->materials)
        return fail(c, QPT_E_INVALID, "null scene array");
    if (!d->num_vertices || !d->num_triangles || !d->num_materials)
        return fail(c, QPT_E_INVALID, "empty scene");
    if (!d->width || !d->height || d->width > 16384 || d->height > 16384)
        return fail(c, QPT_E_INVALID, "framebuffer %ux%u out of range", d->width, d->height);
    if (d->num_triangles > (1u << 27)) return fail(c, QPT_E_INVALID, "too many triangles");
    for (uint64_t q = 0; q < 3ull * d->num_vertices; ++q)
        if (!std::isfinite(d->positions[q])) return fail(c, QPT_E_INVALID, "non-finite position");
    for (uint64_t q = 0; q < 3ull * d->num_triangles; ++q)
        if (d->indices[q] >= d->num_vertices) return fail(c, QPT_E_INVALID, "index out of range");
    for (uint64_t q = 0; q < d->num_triangles; ++q)
        if (d->tri_material[q] >= d->num_materials) return fail(c, QPT_E_INVALID, "material out of range");
    for (uint32_t m = 0; m < d->num_materials; ++m) {
        const qpt_material &mm = d->materials[m];
        for (int k = 0; k < 3; ++k)
            if (!(mm.albedo[k] >= 0 && mm.albedo[k] <= 1) || !(mm.emission[k] >= 0) ||
                !std::isfinite(mm.emission[k]))
                return fail(c, QPT_E_INVALID, "material %u out of range", m);
        if ((mm.flags & QPT_MAT_GGX) && !(mm.roughness > 0 && mm.roughness <= 1))
            return fail(c, QPT_E_INVALID, "material %u roughness out of (0, 1]", m);
    }
    if ((d->env_width || d->env_height) && (!d->env_rgb || !d->env_width || !d->env_height))
        return fail(c, QPT_E_INVALID, "bad environment");
    c->W = d->width;
    c->H = d->height;
    c->pos.assign(d->positions, d->positions + 3ull * d->num_vertices);
    c->idx.assign(d->indices, d->indices + 3ull * d->num_triangles);
    c->tri_mat.assign(d->tri_material, d->tri_material + d->num_triangles);
    c->mats.assign(d->materials, d->materials + d->num_materials);
    c->ew = d->env_width;
    c->eh = d->env_height;
    c->env.assign(d->env_rgb ? d->env_rgb : nullptr,
                  d->env_rgb ? d->env_rgb + 3ull * c->ew * c->eh : nullptr);
    c->cam = d->camera;
    build_lights(c);
    build_light_tree(c);
    c->env_row.clear();
    c->env_col.clear();
    c->env_texel.clear();
    c->env_cos.clear();
    if (c->ew) build_env(c);
    build_env_pyramid(c);
    c->p_env = c->ew ? (c->emit_input_tri.empty() ? 1.0 : 0.5) : 0.0;
    build_light_pmf(c);
    if (c->emit_input_tri.empty() && !c->ew) {
        // a scene without light renders black; still valid
    }
    set_frame_constants(c);
    // scene box for the guide's position encoding
    for (int a = 0; a < 3; ++a) {
        double lo = INFINITY, hi = -INFINITY;
        for (uint64_t q = 0; q < d->num_vertices; ++q) {
            lo = std::min(lo, (double)d->positions[3 * q + a]);
            hi = std::max(hi, (double)d->positions[3 * q + a]);
        }
        c->bbox[a] = lo;
        c->bbox[3 + a] = std::max(hi - lo, 1e-6);
    }
    c->guide_weights = false;
    c->guide_steps = 0;
    c->gmats.resize(c->mats.size());
    for (size_t m = 0; m < c->mats.size(); ++m) {
        const qpt_material &mm = c->mats[m];
        uint32_t fl = mm.flags;
        float flf;
        std::memcpy(&flf, &fl, 4);
        c->gmats[m].albedo_rough = make_float4(mm.albedo[0], mm.albedo[1], mm.albedo[2], mm.roughness);
        c->gmats[m].emission_flags = make_float4(mm.emission[0], mm.emission[1], mm.emission[2], flf);
    }
    c->scene_ok = true;
    return QPT_OK;
}

// A full-precision 4-wide node -> its 64-byte quantised form: per axis the
// smallest power-of-two step 2^e with 255 steps spanning the union of the
// used children's boxes; each child's box rounded outwards to whole steps
// from the union's lower corner (exact in FP64, so the quantised box holds
// the full one). Unused slots keep an empty reference (and an inverted box).
static QNode quantize_node(const Node &n)
{
    const float lo[3][4] = {{n.lox.x, n.lox.y, n.lox.z, n.lox.w}, {n.loy.x, n.loy.y, n.loy.z, n.loy.w},
                            {n.loz.x, n.loz.y, n.loz.z, n.loz.w}};
    const float hi[3][4] = {{n.hix.x, n.hix.y, n.hix.z, n.hix.w}, {n.hiy.x, n.hiy.y, n.hiy.z, n.hiy.w},
                            {n.hiz.x, n.hiz.y, n.hiz.z, n.hiz.w}};
    const int32_t ref[4] = {n.ref.x, n.ref.y, n.ref.z, n.ref.w};
    float org[3] = {INFINITY, INFINITY, INFINITY}, top[3] = {-INFINITY, -INFINITY, -INFINITY};
    uint32_t used = 0;
    for (int q = 0; q < 4; ++q) {
        if (ref[q] == kEmptyChild) continue;
        ++used;
        for (int a = 0; a < 3; ++a) {
            org[a] = std::min(org[a], lo[a][q]);
            top[a] = std::max(top[a], hi[a][q]);
        }
    }
    uint32_t ebias[3], qlo[3] = {0, 0, 0}, qhi[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        if (!used) org[a] = top[a] = 0.0f;
        const double ext = (double)top[a] - (double)org[a];
        int e = -126;
        if (ext > 0.0) {
            e = std::max(-126, (int)std::ceil(std::log2(ext / 255.0)));
            while (e > -126 && std::ldexp(255.0, e - 1) >= ext) --e;
            while (std::ldexp(255.0, e) < ext) ++e;
        }
        ebias[a] = (uint32_t)(e + 127);
        for (int q = 0; q < 4; ++q) {
            uint32_t l = 255, h = 0;  // unused: an inverted box
            if (ref[q] != kEmptyChild) {
                l = (uint32_t)std::floor(std::ldexp((double)lo[a][q] - (double)org[a], -e));
                h = (uint32_t)std::ceil(std::ldexp((double)hi[a][q] - (double)org[a], -e));
                l = std::min(l, 255u);
                h = std::min(h, 255u);
            }
            qlo[a] |= l << (8 * q);
            qhi[a] |= h << (8 * q);
        }
    }
    QNode out;
    uint32_t ox, oy, oz;
    std::memcpy(&ox, &org[0], 4);
    std::memcpy(&oy, &org[1], 4);
    std::memcpy(&oz, &org[2], 4);
    out.w0 = make_uint4(ox, oy, oz, ebias[0] | (ebias[1] << 8) | (ebias[2] << 16) | (used << 24));
    out.w1 = make_uint4(qlo[0], qlo[1], qlo[2], qhi[0]);
    out.w2 = make_uint4(qhi[1], qhi[2], (uint32_t)ref[0], (uint32_t)ref[1]);
    out.w3 = make_uint4((uint32_t)ref[2], (uint32_t)ref[3], 0u, 0u);
    return out;
}

// after either builder: overflow stack size, triangles in leaf order, the
// emitters' leaf-order triangles
static void finish_bvh(qpt_ctx *c, const std::vector<uint32_t> &order, uint32_t depth4)
{
    const uint32_t nt = (uint32_t)order.size();
    // a ray at a node of depth d holds at most 3 (d + 1) stack entries
    c->stack_need = 3 * (depth4 + 1);
    c->gtris.resize(nt);
    c->emit_tri_bvh.assign(c->emit_input_tri.size(), 0);
    for (uint32_t k = 0; k < nt; ++k) {
        uint32_t t = order[k];
        const float *p0 = &c->pos[3 * (size_t)c->idx[3 * (size_t)t]];
        const float *p1 = &c->pos[3 * (size_t)c->idx[3 * (size_t)t + 1]];
        const float *p2 = &c->pos[3 * (size_t)c->idx[3 * (size_t)t + 2]];
        uint32_t m = c->tri_mat[t], e = c->tri_emit[t] >= 0 ? (uint32_t)c->tri_emit[t] : kNoHit;
        float mf, tf, ef;
        std::memcpy(&mf, &m, 4);
        std::memcpy(&tf, &t, 4);
        std::memcpy(&ef, &e, 4);
        c->gtris[k].v0 = make_float4(p0[0], p0[1], p0[2], mf);
        c->gtris[k].v1 = make_float4(p1[0], p1[1], p1[2], tf);
        c->gtris[k].v2 = make_float4(p2[0], p2[1], p2[2], ef);
        if (e != kNoHit) c->emit_tri_bvh[e] = k;
    }
    c->bvh_ok = true;
}

// the GPU builder (linear BVH, collapsed there into the 4-wide layout) with
// its temporaries in the device region [scratch, scratch + bytes)
static int build_bvh_gpu(qpt_ctx *c, uint32_t leaf, void *scratch, size_t bytes, qpt_bvh_stats *stats,
                         std::chrono::steady_clock::time_point t0)
{
    const uint32_t nt = (uint32_t)c->tri_mat.size(), nv = (uint32_t)(c->pos.size() / 3);
    const size_t need = gpu_build_scratch_bytes(nv, nt);
    if (bytes < need)
        return fail(c, QPT_E_NOMEM, "GPU BVH build needs %zu bytes of scratch, %zu given", need, bytes);
    double maxabs = 0.0;
    for (size_t q = 0; q < c->idx.size(); ++q)
        for (int a = 0; a < 3; ++a) maxabs = std::max(maxabs, (double)std::fabs(c->pos[3 * (size_t)c->idx[q] + a]));
    const float pad = (float)(std::ldexp(std::max(maxabs, 1e-3), -18));
    std::vector<uint32_t> order;
    uint32_t depth4 = 0;
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, QPT_E_HIP, "hipSetDevice failed");
    hipError_t e = gpu_build_bvh(c->pos.data(), nv, c->idx.data(), nt, leaf, pad, scratch, bytes, c->stream, c->gnodes,
                                 order, depth4);
    if (e != hipSuccess) return fail(c, QPT_E_HIP, "GPU BVH build: %s", hipGetErrorString(e));
    // leaves and the SAH cost of the 4-wide tree (node box = union of its slots)
    auto area = [](float dx, float dy, float dz) { return 2.0 * ((double)dx * dy + (double)dy * dz + (double)dz * dx); };
    uint32_t leaves = 0;
    double sah = 0.0, root_area = 0.0;
    for (size_t k = 0; k < c->gnodes.size(); ++k) {
        const Node &nd = c->gnodes[k];
        const float lo[3][4] = {{nd.lox.x, nd.lox.y, nd.lox.z, nd.lox.w}, {nd.loy.x, nd.loy.y, nd.loy.z, nd.loy.w},
                                {nd.loz.x, nd.loz.y, nd.loz.z, nd.loz.w}};
        const float hi[3][4] = {{nd.hix.x, nd.hix.y, nd.hix.z, nd.hix.w}, {nd.hiy.x, nd.hiy.y, nd.hiy.z, nd.hiy.w},
                                {nd.hiz.x, nd.hiz.y, nd.hiz.z, nd.hiz.w}};
        const int ref[4] = {nd.ref.x, nd.ref.y, nd.ref.z, nd.ref.w};
        float ulo[3] = {INFINITY, INFINITY, INFINITY}, uhi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int q = 0; q < nd.pad.x; ++q) {
            for (int a = 0; a < 3; ++a) {
                ulo[a] = std::min(ulo[a], lo[a][q]);
                uhi[a] = std::max(uhi[a], hi[a][q]);
            }
            if (ref[q] < 0) ++leaves;
        }
        const double na = area(uhi[0] - ulo[0], uhi[1] - ulo[1], uhi[2] - ulo[2]);
        if (k == 0) root_area = std::max(na, 1e-30);
        sah += na / root_area;
        for (int q = 0; q < nd.pad.x; ++q)
            if (ref[q] < 0)
                sah += area(hi[0][q] - lo[0][q], hi[1][q] - lo[1][q], hi[2][q] - lo[2][q]) / root_area *
                       (double)((~(uint32_t)ref[q] & 7u) + 1u);
    }
    finish_bvh(c, order, depth4);
    auto t1 = std::chrono::steady_clock::now();
    if (stats) {
        stats->num_nodes = (uint32_t)c->gnodes.size();
        stats->num_leaves = leaves;
        stats->max_depth = depth4;
        stats->node_bytes = c->node_format == kNodeQuant ? (uint32_t)sizeof(QNode) : (uint32_t)sizeof(Node);
        stats->sah_cost = sah;
        stats->build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    return QPT_OK;
}

static int bvh_opts(qpt_ctx *c, const qpt_bvh_opts *opts, uint32_t &leaf, uint32_t &bins, uint32_t &builder)
{
    // defaults: leaves of up to 3 triangles (measured: 2-3 trace 1-2% faster than 4, 6-8 up to
    // 12% slower on the grid and city workloads), 16 bins (32 and 64 made no difference)
    leaf = opts && opts->max_leaf_size ? opts->max_leaf_size : 3;
    bins = opts && opts->sah_bins ? opts->sah_bins : 16;
    builder = opts ? opts->builder : 0;
    if (leaf < 1 || leaf > 8 || bins < 4 || bins > 64 || builder > 1 || (opts && opts->node_format > 1))
        return fail(c, QPT_E_INVALID, "bad BVH options");
    return QPT_OK;
}

int qpt_bvh_scratch_size(qpt_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return QPT_E_INVALID;
    if (!c->scene_ok) return fail(c, QPT_E_STATE, "bvh_scratch_size before build_scene");
    *bytes = gpu_build_scratch_bytes((uint32_t)(c->pos.size() / 3), (uint32_t)c->tri_mat.size());
    return QPT_OK;
}

int qpt_build_bvh_noalloc(qpt_ctx *c, const qpt_bvh_opts *opts, qpt_bvh_stats *stats)
{
    if (!c) return QPT_E_INVALID;
    if (!c->scene_ok) return fail(c, QPT_E_STATE, "build_bvh before build_scene");
    if (c->device < 0) return fail(c, QPT_E_STATE, "the GPU builder needs a device context");
    uint32_t leaf, bins, builder;
    if (int rc = bvh_opts(c, opts, leaf, bins, builder)) return rc;
    const uint32_t nt = (uint32_t)c->tri_mat.size();
    if (nt <= leaf) return fail(c, QPT_E_INVALID, "the GPU builder needs more triangles than a leaf holds");
    c->node_format = opts ? opts->node_format : kNodeQuant;
    const size_t need = gpu_build_scratch_bytes((uint32_t)(c->pos.size() / 3), nt);
    if (need > kStaticScratch)
        return fail(c, QPT_E_INVALID, "scene too large for the allocation-free build: %zu bytes of scratch needed, "
                    "the library's static region holds %zu", need, kStaticScratch);
    if (!c->static_scratch) return fail(c, QPT_E_STATE, "no static scratch region on this device");
    c->bvh_ok = c->bound = false;
    return build_bvh_gpu(c, leaf, c->static_scratch, kStaticScratch, stats, std::chrono::steady_clock::now());
}

int qpt_build_bvh(qpt_ctx *c, const qpt_bvh_opts *opts, qpt_bvh_stats *stats)
{
    if (!c) return QPT_E_INVALID;
    if (!c->scene_ok) return fail(c, QPT_E_STATE, "build_bvh before build_scene");
    c->bvh_ok = c->bound = false;
    auto t0 = std::chrono::steady_clock::now();
    uint32_t leaf, bins, builder;
    if (int rc = bvh_opts(c, opts, leaf, bins, builder)) return rc;
    c->node_format = opts ? opts->node_format : kNodeQuant;
    uint32_t nt = (uint32_t)c->tri_mat.size();
    if (builder == 1 && c->device < 0) return fail(c, QPT_E_STATE, "the GPU builder needs a device context");
    if (builder == 1 && nt > leaf) {
        if (!opts->scratch) return fail(c, QPT_E_INVALID, "the GPU builder needs caller scratch (qpt_bvh_scratch_size)");
        return build_bvh_gpu(c, leaf, opts->scratch, opts->scratch_bytes, stats, t0);
    }
    std::vector<PrimInfo> prim(nt);
    double maxabs = 0.0;
    for (uint32_t t = 0; t < nt; ++t) {
        PrimInfo &p = prim[t];
        for (int a = 0; a < 3; ++a) {
            float v0 = c->pos[3 * (size_t)c->idx[3 * (size_t)t] + a];
            float v1 = c->pos[3 * (size_t)c->idx[3 * (size_t)t + 1] + a];
            float v2 = c->pos[3 * (size_t)c->idx[3 * (size_t)t + 2] + a];
            p.lo[a] = std::min(v0, std::min(v1, v2));
            p.hi[a] = std::max(v0, std::max(v1, v2));
            p.c[a] = 0.5f * (p.lo[a] + p.hi[a]);
            maxabs = std::max(maxabs, (double)std::max(std::fabs(p.lo[a]), std::fabs(p.hi[a])));
        }
    }
    std::vector<uint32_t> order(nt);
    for (uint32_t t = 0; t < nt; ++t) order[t] = t;
    Builder B(prim, order, leaf, bins);
    unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    int budget = 0;
    while ((1u << budget) < 2 * hw && budget < 6) ++budget;
    B.build(0, nt, 0, budget);
    if (B.max_depth.load() >= kMaxTreeDepth) return fail(c, QPT_E_INVALID, "binary BVH deeper than its limit");

    // boxes padded outward so that rounding in the slab test never culls a
    // triangle the exact triangle test would report
    float pad = (float)(std::ldexp(std::max(maxabs, 1e-3), -18));
    // collapse into a 4-wide tree: each node takes its binary node's two
    // children and keeps opening the inner child of largest surface area
    // until it has four; siblings are stored next to each other. Nodes are
    // numbered breadth-first until kTopNodes exist (the top levels, which
    // the traversal keeps in LDS, come first), depth-first after that.
    auto leaf_ref = [&](const BuildNode &bn) -> int32_t { return ~(int32_t)((bn.first << 3) | (bn.count - 1)); };
    c->gnodes.clear();
    uint32_t leaves = 0, depth4 = 0;
    double sah = 0.0;
    const BuildNode &root = B.nodes[0];
    const float root_area = std::max(Builder::area(root.lo, root.hi), 1e-30f);
    struct Item {
        uint32_t q, slot, depth;
    };
    std::vector<Item> work;
    size_t head = 0;  // breadth-first while head <= work.size() marks a queue
    bool bfs = true;
    c->gnodes.emplace_back();
    work.push_back({0u, 0u, 0u});
    while (head < work.size()) {
        if (bfs && c->gnodes.size() >= kTopNodes) {
            // the rest of the queue becomes the depth-first stack
            work.erase(work.begin(), work.begin() + (std::ptrdiff_t)head);
            head = 0;
            bfs = false;
        }
        Item it;
        if (bfs) {
            it = work[head++];
        } else {
            it = work.back();
            work.pop_back();
        }
        depth4 = std::max(depth4, it.depth);
        const BuildNode &bn = B.nodes[it.q];
        uint32_t kids[4];
        uint32_t nk = 0;
        if (bn.count) {
            kids[nk++] = it.q;  // the whole tree is one leaf
        } else {
            kids[nk++] = (uint32_t)bn.left;
            kids[nk++] = (uint32_t)bn.right;
            while (nk < 4) {
                int best = -1;
                float ba = -1.0f;
                for (uint32_t k = 0; k < nk; ++k) {
                    const BuildNode &ch = B.nodes[kids[k]];
                    if (ch.count) continue;
                    float a = Builder::area(ch.lo, ch.hi);
                    if (a > ba) {
                        ba = a;
                        best = (int)k;
                    }
                }
                if (best < 0) break;
                const BuildNode &op = B.nodes[kids[best]];
                kids[best] = (uint32_t)op.left;
                kids[nk++] = (uint32_t)op.right;
            }
        }
        sah += Builder::area(bn.lo, bn.hi) / root_area;
        float bx[6][4];
        int32_t ref[4];
        for (uint32_t k = 0; k < 4; ++k) {
            if (k >= nk) {
                for (int a = 0; a < 6; ++a) bx[a][k] = 0.0f;
                ref[k] = kEmptyChild;
                continue;
            }
            const BuildNode &ch = B.nodes[kids[k]];
            for (int a = 0; a < 3; ++a) {
                bx[a][k] = ch.lo[a] - pad;
                bx[3 + a][k] = ch.hi[a] + pad;
            }
            if (ch.count) {
                ref[k] = leaf_ref(ch);
                ++leaves;
                sah += Builder::area(ch.lo, ch.hi) / root_area * ch.count;
            } else {
                uint32_t slot = (uint32_t)c->gnodes.size();
                c->gnodes.emplace_back();
                ref[k] = (int32_t)slot;
                work.push_back({kids[k], slot, it.depth + 1});
            }
        }
        Node n;
        n.lox = make_float4(bx[0][0], bx[0][1], bx[0][2], bx[0][3]);
        n.loy = make_float4(bx[1][0], bx[1][1], bx[1][2], bx[1][3]);
        n.loz = make_float4(bx[2][0], bx[2][1], bx[2][2], bx[2][3]);
        n.hix = make_float4(bx[3][0], bx[3][1], bx[3][2], bx[3][3]);
        n.hiy = make_float4(bx[4][0], bx[4][1], bx[4][2], bx[4][3]);
        n.hiz = make_float4(bx[5][0], bx[5][1], bx[5][2], bx[5][3]);
        n.ref = make_int4(ref[0], ref[1], ref[2], ref[3]);
        n.pad = make_int4((int)nk, 0, 0, 0);
        c->gnodes[it.slot] = n;
    }
    finish_bvh(c, order, depth4);
    auto t1 = std::chrono::steady_clock::now();
    if (stats) {
        stats->num_nodes = (uint32_t)c->gnodes.size();
        stats->num_leaves = leaves;
        stats->max_depth = depth4;
        stats->node_bytes = c->node_format == kNodeQuant ? (uint32_t)sizeof(QNode) : (uint32_t)sizeof(Node);
        stats->sah_cost = sah;
        stats->build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    return QPT_OK;
}

int qpt_workspace_size(const qpt_ctx *c, uint32_t pool_paths, size_t *bytes)
{
    if (!c || !bytes) return QPT_E_INVALID;
    if (!c->scene_ok || !c->bvh_ok) return QPT_E_STATE;
    uint32_t cap = pool_paths ? pool_paths : default_pool(c);
    *bytes = make_layout(c, cap).total;
    return QPT_OK;
}

int qpt_bind_workspace(qpt_ctx *c, void *device_ptr, size_t bytes, uint32_t pool_paths)
{
    if (!c) return QPT_E_INVALID;
    if (c->device < 0) return fail(c, QPT_E_STATE, "context has no device");
    if (!c->scene_ok || !c->bvh_ok) return fail(c, QPT_E_STATE, "bind_workspace before build_scene/build_bvh");
    if (!device_ptr || ((uintptr_t)device_ptr & 255)) return fail(c, QPT_E_INVALID, "workspace must be 256-byte aligned");
    uint32_t cap = pool_paths ? pool_paths : default_pool(c);
    if (cap < 64 || cap > (1u << 28)) return fail(c, QPT_E_INVALID, "pool_paths out of range");
    Layout L = make_layout(c, cap);
    if (bytes < L.total) return fail(c, QPT_E_NOMEM, "workspace %zu bytes, need %zu", bytes, L.total);
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, QPT_E_HIP, "hipSetDevice failed");
    if (!c->ev_lane_in) {
        // the second lane's stream: the caller's (qpt_set_streams), else the
        // library's own, default priority, non-blocking so it can overlap a
        // caller's legacy stream. HIP places a new stream on its least-used
        // hardware queue, which keeps it off the caller's queue while the
        // device has queues to spare; two lanes sharing one queue would run
        // one after the other.
        if (!c->lstream) {
            HIP_TRY(c, hipStreamCreateWithFlags(&c->lstream, hipStreamNonBlocking));
            c->own_lstream = true;
        }
        for (int k = 0; k < 2; ++k) HIP_TRY(c, hipEventCreateWithFlags(&c->ev_train[k], hipEventDisableTiming));
        HIP_TRY(c, hipEventCreateWithFlags(&c->ev_tdone, hipEventDisableTiming));
        HIP_TRY(c, hipEventCreateWithFlags(&c->ev_lane_in, hipEventDisableTiming));
        HIP_TRY(c, hipEventCreateWithFlags(&c->ev_lane_out, hipEventDisableTiming));
        HIP_TRY(c, hipEventCreateWithFlags(&c->ev_acc, hipEventDisableTiming));
        for (int k = 0; k < 2; ++k) HIP_TRY(c, hipEventCreateWithFlags(&c->ev_regen[k], hipEventDisableTiming));
        // word 0: the stop request; words 8-9: regeneration's paths left per chunk
        HIP_TRY(c, hipHostMalloc((void **)&c->abort_host, 64, hipHostMallocMapped));
        HIP_TRY(c, hipHostGetDevicePointer((void **)&c->abort_dev, c->abort_host, 0));
        __atomic_store_n(c->abort_host, 0u, __ATOMIC_SEQ_CST);
    }
    c->ws = (uint8_t *)device_ptr;
    c->ws_bytes = bytes;
    c->pool_cap = cap;
    c->lay = L;
    uint8_t *w = c->ws;
    auto up = [&](size_t off, const void *src, size_t n) -> hipError_t {
        if (!n) return hipSuccess;
        return hipMemcpyAsync(w + off, src, n, hipMemcpyHostToDevice, c->stream);
    };
    std::vector<float> pmf32(c->emit_pmf.size());
    for (size_t e = 0; e < pmf32.size(); ++e) pmf32[e] = (float)c->emit_pmf[e];
    if (c->node_format == kNodeQuant) {
        std::vector<QNode> q(c->gnodes.size());
        for (size_t k = 0; k < q.size(); ++k) q[k] = quantize_node(c->gnodes[k]);
        HIP_TRY(c, up(L.nodes, q.data(), q.size() * sizeof(QNode)));
        HIP_TRY(c, hipStreamSynchronize(c->stream));  // q is freed on return
    } else {
        HIP_TRY(c, up(L.nodes, c->gnodes.data(), c->gnodes.size() * sizeof(Node)));
    }
    HIP_TRY(c, up(L.tris, c->gtris.data(), c->gtris.size() * sizeof(Tri)));
    HIP_TRY(c, up(L.mats, c->gmats.data(), c->gmats.size() * sizeof(Material)));
    HIP_TRY(c, up(L.emit_tri, c->emit_tri_bvh.data(), c->emit_tri_bvh.size() * 4));
    HIP_TRY(c, up(L.alias_idx, c->alias_idx.data(), c->alias_idx.size() * 4));
    HIP_TRY(c, up(L.alias_thr, c->alias_thr.data(), c->alias_thr.size() * 8));
    HIP_TRY(c, up(L.emit_pmf, pmf32.data(), pmf32.size() * 4));
    HIP_TRY(c, up(L.lt_nodes, c->lt_nodes.data(), c->lt_nodes.size() * sizeof(LtNode)));
    HIP_TRY(c, up(L.lt_emit, c->lt_emit.data(), c->lt_emit.size() * 4));
    HIP_TRY(c, up(L.lt_pos, c->lt_pos.data(), c->lt_pos.size() * 4));
    HIP_TRY(c, up(L.lt_w, c->lt_w.data(), c->lt_w.size() * 4));
    HIP_TRY(c, up(L.ep_q, c->ep_q.data(), c->ep_q.size() * 4));
    HIP_TRY(c, up(L.ep_oq, c->ep_oq.data(), c->ep_oq.size() * 4));
    HIP_TRY(c, up(L.env_texel, c->env_texel.data(), c->env_texel.size() * sizeof(float4)));
    HIP_TRY(c, up(L.env_row, c->env_row.data(), c->env_row.size() * 4));
    HIP_TRY(c, up(L.env_col, c->env_col.data(), c->env_col.size() * 4));
    HIP_TRY(c, up(L.env_cos, c->env_cos.data(), c->env_cos.size() * 4));
    HIP_TRY(c, up(L.bases, c->bases.data(), kMaxDims * sizeof(HaltonBase)));
    Frame &f = c->frame;
    f.nodes = (const Node *)(w + L.nodes);
    f.qnodes = (const QNode *)(w + L.nodes);
    f.node_format = c->node_format;
    f.top_nodes = c->node_format == kNodeQuant ? (uint32_t)std::min<size_t>(kTopNodes, c->gnodes.size()) : 0u;
    f.tris = (const Tri *)(w + L.tris);
    f.mats = (const Material *)(w + L.mats);
    f.num_tris = (uint32_t)c->gtris.size();
    f.num_emit = (uint32_t)c->emit_input_tri.size();
    f.emit_tri = (const uint32_t *)(w + L.emit_tri);
    f.alias_idx = (const uint32_t *)(w + L.alias_idx);
    f.alias_thr = (const unsigned long long *)(w + L.alias_thr);
    f.emit_pmf = (const float *)(w + L.emit_pmf);
    f.lt_nodes = (const LtNode *)(w + L.lt_nodes);
    f.lt_emit = (const uint32_t *)(w + L.lt_emit);
    f.lt_pos = (const uint32_t *)(w + L.lt_pos);
    f.lt_w = (const uint32_t *)(w + L.lt_w);
    f.env_w = c->ew;
    f.env_h = c->eh;
    f.env_texel = (const float4 *)(w + L.env_texel);
    f.env_row = (const uint32_t *)(w + L.env_row);
    f.env_col = (const uint32_t *)(w + L.env_col);
    f.env_cos = (const float *)(w + L.env_cos);
    f.p_env = (float)c->p_env;
    f.ep_q = (const uint4 *)(w + L.ep_q);
    f.ep_oq = (const uint4 *)(w + L.ep_oq);
    f.ep_m = c->ep_m;
    f.ep_top = c->ep_top;
    f.ep_root = c->ep_root;
    f.ep_stride = c->ep_m ? 1 + ep_nodes_above(c->ep_top) : 0;
    f.bases = (const HaltonBase *)(w + L.bases);
    for (int k = 0; k < 2; ++k) {
        const Layout::Lane &ln = L.lane[k];
        Pool &p = k ? c->pool_b : c->pool;
        p.cap = cap;
        p.ray_o = (float4 *)(w + ln.ray_o);
        p.ray_d = (float4 *)(w + ln.ray_d);
        p.hit = (float4 *)(w + ln.hit);
        p.thr = (float4 *)(w + ln.thr);
        p.rad = (float4 *)(w + ln.rad);
        p.idx = (unsigned long long *)(w + ln.idx);
        p.q_ext[0] = (uint32_t *)(w + ln.q0);
        p.q_ext[1] = (uint32_t *)(w + ln.q1);
        p.q_dead = (uint32_t *)(w + ln.qdead);
        p.pv = k ? nullptr : (uint2 *)(w + ln.pv);
        p.sh_o = (float4 *)(w + ln.sh_o);
        p.sh_d = (float4 *)(w + ln.sh_d);
        p.sh_c = (float4 *)(w + ln.sh_c);
        p.counters = (uint32_t *)(w + ln.counters);
        p.gstack = (int *)(w + ln.gstack);
        p.trav_threads = c->trav_threads;
        p.stats = (unsigned long long *)(w + L.stats);
        p.fb_sum = (double *)(w + L.fb_sum);
        p.fb_count = (uint32_t *)(w + L.fb_count);
    }
    GuideTrain &T = c->gt;
    T.master = (float *)(w + L.g_master);
    T.m = (float *)(w + L.g_m);
    T.v = (float *)(w + L.g_v);
    T.frag = (uint2 *)(w + L.g_frag);
    T.fragT = (uint2 *)(w + L.g_fragT);
    T.bias = (float *)(w + L.g_bias);
    for (int k = 0; k < 2; ++k) {
        c->pub_frag[k] = (uint2 *)(w + L.g_pub_frag[k]);
        c->pub_bias[k] = (float *)(w + L.g_pub_bias[k]);
    }
    c->gbatch = 0;
    c->last_buf = 0;
    T.ring = (float4 *)(w + L.g_ring);
    T.ring_head = (uint32_t *)(w + L.g_ring_head);
    T.ring_cap = kGuideRing;
    T.partial = (float *)(w + L.g_partial);
    T.scalars = (float *)(w + L.g_scalars);
    T.max_blocks = c->guide_blocks;
    GuideDev &G = f.guide;
    G.frag = T.frag;
    G.fragT = T.fragT;
    G.bias = T.bias;
    for (int k = 0; k < 2; ++k) {
        c->lane_rec[k] = (float4 *)(w + L.g_rec[k]);
    }
    for (int a = 0; a < 3; ++a) {
        G.bmin[a] = (float)c->bbox[a];
        G.binv[a] = (float)(1.0 / (double)(float)c->bbox[3 + a]);
    }
    G.alpha_thr = 0;
    G.alpha = 0.0f;
    G.record = 0;
    G.rec = (float4 *)(w + L.g_rec[0]);
    G.rec_cap = (uint32_t)guide_rec_cap(cap);
    G.rec_count = c->pool.counters + 127;
    c->guide_weights = false;
    c->guide_steps = 0;
    c->last_batch.valid = false;
    c->bound = true;
    int rc = qpt_reset_accum(c);
    if (rc) {
        c->bound = false;
        return rc;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return QPT_OK;
}

int qpt_load_accum(qpt_ctx *c, const double *sum_rgb, const uint32_t *counts, int src_is_device)
{
    if (!c || !sum_rgb || !counts) return QPT_E_INVALID;
    if (!c->bound) return fail(c, QPT_E_STATE, "load_accum before bind_workspace");
    DeviceGuard g(c->device);
    const size_t npix = (size_t)c->W * c->H;
    const hipMemcpyKind k = src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIP_TRY(c, hipMemcpyAsync(c->pool.fb_sum, sum_rgb, npix * 3 * 8, k, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->pool.fb_count, counts, npix * 4, k, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return QPT_OK;
}

int qpt_reset_accum(qpt_ctx *c)
{
    if (!c) return QPT_E_INVALID;
    if (!c->bound) return fail(c, QPT_E_STATE, "no workspace bound");
    DeviceGuard g(c->device);
    size_t npix = (size_t)c->W * c->H;
    HIP_TRY(c, launch_fill_f64(c->pool.fb_sum, npix * 3, c->stream));
    HIP_TRY(c, launch_fill_u32(c->pool.fb_count, npix, 0, c->stream));
    HIP_TRY(c, launch_fill_u32((uint32_t *)c->pool.stats, 16, 0, c->stream));
    return QPT_OK;
}

int qpt_render_pass(qpt_ctx *c, uint64_t first_pass, uint32_t num_passes, const qpt_render_opts *o)
{
    if (!c || !o) return QPT_E_INVALID;
    if (!c->bound) return fail(c, QPT_E_STATE, "render_pass before bind_workspace");
    if (o->max_depth < 1 || 2 + 8 * (o->max_depth - 1) > kMaxDims || o->mode > 2 || o->light_tree > 1 ||
        o->env_sampling > 2 || o->filter > 1 || o->tail_depth > o->max_depth ||
        (o->regen_paths && (o->regen_paths < 64 || o->regen_paths > c->pool_cap)) || o->compress_state > 1)
        return fail(c, QPT_E_INVALID, "bad render options (max_depth 1..32, mode 0..2, light_tree 0..1, "
                                      "env_sampling 0..2, filter 0..1, tail_depth 0..max_depth, regen_paths 0 or "
                                      "64..pool, compress_state 0..1)");
    if (o->env_sampling && c->ew && !c->ep_m)
        return fail(c, QPT_E_INVALID, "environment pyramid needs a 2:1 map of power-of-two size");
    if (!num_passes) return QPT_OK;
    // the largest Halton index must fit 64 bits
    u128 last = (u128)(first_pass + num_passes) * c->frame.S;
    if (last >> 64) return fail(c, QPT_E_INVALID, "pass range overflows 64-bit sample indices");
    const bool guiding = c->gopts.alpha > 0.0f || c->gopts.train;
    if (guiding && !c->guide_weights)
        return fail(c, QPT_E_STATE, "guide enabled before qpt_guide_set_weights");
    DeviceGuard g(c->device);
    Frame f = c->frame;
    f.max_depth = o->max_depth;
    f.rr = o->rr;
    f.mode = o->mode;
    f.scramble = o->scramble;
    f.light_tree = o->light_tree;
    f.env_pyramid = c->ew ? o->env_sampling : 0;
    f.gauss_filter = o->filter;
    f.tail_depth = o->tail_depth;
    f.compress = o->compress_state;
    f.abort_word = c->abort_dev;
    if (c->abort_host && __atomic_load_n(c->abort_host, __ATOMIC_SEQ_CST))
        return fail(c, QPT_E_ABORTED, "aborted: qpt_readback reports the progress and clears the request");
    Profiler *prof = c->profiling ? &c->prof : nullptr;
    // Two batches in flight: consecutive batches alternate between the
    // caller's stream and the library's second stream, each lane with its own
    // path pool (and, for the guide, its own mixtures and records), so that
    // one batch's deep vertices (few paths, latency-bound traversals) overlap
    // the next batch's first vertices. The framebuffer stays updated in pass
    // order: a batch's accumulation waits for the previous batch's; training
    // samples enter the replay ring one batch after another. Lane 1 starts
    // after the caller's earlier work and the caller's stream waits for lane 1
    // before this call returns.
    // regeneration: whole-frame batches of the plain tracer, one at a time
    const uint32_t npix = c->W * c->H, cap = c->pool_cap;
    const bool regen = o->regen_paths && !guiding && npix <= cap;
    f.regen = regen ? o->regen_paths : 0u;
    const bool two_lanes = !o->single_stream && !regen;
    bool lane_b_used = false;
    // the point lane 1 waits for: the caller's work before this call, which
    // the caller's stream orders after all work of earlier calls (lane 1's
    // included), so no wait on an event of an earlier call is needed
    if (two_lanes) HIP_TRY(c, hipEventRecord(c->ev_lane_in, c->stream));
    c->train_pending[0] = c->train_pending[1] = false;
    c->tdone_pending = false;
    // one batch of passes (or of pixels), then one training step if enabled
    auto batch = [&](uint32_t p0, uint32_t np, uint64_t pass0, uint32_t nb) -> int {
        // pixel chunks of one pass stay on one lane (its first chunk latches the
        // abort decision for the rest); whole-pass batches alternate
        const bool lane_b = two_lanes && (npix > cap ? ((pass0 - first_pass) & 1) != 0 : (c->batches++ & 1) != 0);
        hipStream_t s = lane_b ? c->lstream : c->stream;
        if (lane_b && !lane_b_used) {
            HIP_TRY(c, hipStreamWaitEvent(c->lstream, c->ev_lane_in, 0));
            lane_b_used = true;
        }
        const Pool &P = lane_b ? c->pool_b : c->pool;
        const int lane = lane_b ? 1 : 0;
        f.guide.rec = c->lane_rec[lane];
        f.guide.rec_count = P.counters + 127;
        bool active = c->gopts.alpha > 0.0f && c->guide_steps >= c->gopts.warmup_steps;
        uint64_t thr = active ? (uint64_t)std::llround((double)c->gopts.alpha * 4294967296.0) : 0;
        f.guide.alpha_thr = (uint32_t)std::min<uint64_t>(thr, 0xffffffffull);
        f.guide.alpha = (float)((double)f.guide.alpha_thr / 4294967296.0);
        f.guide.record = c->gopts.train ? 1u : 0u;
        f.guide.max_vertex = c->gopts.max_vertex ? c->gopts.max_vertex : 0xffffffffu;
        // every vertex 1..max_vertex leaves a record, unless a path could
        // leave more than the buffer holds per path: then a uniform hashed subset
        {
            double per_path = (double)std::min<uint32_t>(f.guide.max_vertex, o->max_depth);
            double keep = std::min(1.0, (double)f.guide.rec_cap / (per_path * (double)np * (double)nb));
            f.guide.rec_thr = keep >= 1.0 ? 0xffffffffu : (uint32_t)(keep * 4294967296.0);
        }
        // The renderer's copy of the weights is double-buffered: batch b
        // renders with the weights the step of batch b - 2 published (buffer
        // b mod 2) while the other lane renders batch b - 1 and then takes its
        // step. Any weights give an unbiased estimator; the lag only delays
        // what the guide has learnt. A batch's samples enter the replay ring
        // and its steps run on the lane that rendered it, right after the
        // batch (the lane's next batch overwrites the path radiance the
        // samples are formed from, and renders with the weights these steps
        // publish), behind the previous batch's steps on the other lane (the
        // ring and the Adam state are shared), so steps keep batch order. No
        // third stream: one that shared a hardware queue with a lane would
        // hold that lane's kernels behind its waits.
        const bool train = c->gopts.train > 0;
        const int k = train ? (int)(c->gbatch & 1) : c->last_buf;
        if (guiding) {
            if (c->train_pending[k]) HIP_TRY(c, hipStreamWaitEvent(s, c->ev_train[k], 0));
            f.guide.frag = c->pub_frag[k];
            f.guide.bias = c->pub_bias[k];
        }
        if (regen) HIP_TRY(c, launch_render_regen(f, P, np, pass0, nb, s, prof, c->abort_host + 8, c->ev_regen));
        else HIP_TRY(c, launch_render_paths(f, P, p0, np, pass0, nb, s, prof));
        c->last_batch.valid = true;
        c->last_batch.lane = lane_b ? 1 : 0;
        c->last_batch.p0 = p0;
        c->last_batch.np = np;
        c->last_batch.nb = nb;
        c->last_batch.pass0 = pass0;
        if (two_lanes) HIP_TRY(c, hipStreamWaitEvent(s, c->ev_acc, 0));
        HIP_TRY(c, launch_accumulate(f, P, p0, np, nb, s, prof));
        if (two_lanes) HIP_TRY(c, hipEventRecord(c->ev_acc, s));
        if (train) {
            GuideTrain T = c->gt;
            // finalisation and steps in batch order (see above)
            if (c->tdone_pending) HIP_TRY(c, hipStreamWaitEvent(s, c->ev_tdone, 0));
            if (prof) prof->begin(K_GUIDE_TRAIN, s);
            HIP_TRY(c, launch_guide_finalize(f, P, T, s));
            // `train` Adam steps per pass, taken when a batch completes its passes
            // (a pass split into pixel chunks trains after its last chunk)
            const uint32_t nsteps = (p0 + np >= npix) ? c->gopts.train * nb : 0u;
            if (nsteps) {
                HIP_TRY(c, launch_guide_train_steps(f, T, c->gopts.batch ? c->gopts.batch : (1u << 18),
                                                    c->guide_steps + 1, nsteps, c->gopts.lr, c->gopts.seed,
                                                    s, c->pub_frag[k], c->pub_bias[k]));
                HIP_TRY(c, hipEventRecord(c->ev_train[k], s));
                c->train_pending[k] = true;
                c->last_buf = k;
                c->guide_steps += nsteps;
                ++c->gbatch;
            }
            HIP_TRY(c, hipEventRecord(c->ev_tdone, s));
            c->tdone_pending = true;
            if (prof) prof->end(K_GUIDE_TRAIN, s);
        }
        return QPT_OK;
    };
    auto all_batches = [&]() -> int {
        if (npix <= cap) {
            // as few batches as the pool allows, of nearly equal size (20 passes
            // with room for 16 are two batches of 10), so that both lanes have
            // work of the same length to overlap
            const uint32_t per = std::max(1u, cap / npix);
            const uint32_t nbat = (num_passes + per - 1) / per;
            for (uint32_t b = 0, done = 0; b < nbat; ++b) {
                const uint32_t nb = num_passes / nbat + (b < num_passes % nbat ? 1u : 0u);
                int rc = batch(0, npix, first_pass + done, nb);
                if (rc) return rc;
                done += nb;
            }
        } else {
            for (uint32_t j = 0; j < num_passes; ++j)
                for (uint32_t p0 = 0; p0 < npix; p0 += cap) {
                    int rc = batch(p0, std::min(cap, npix - p0), first_pass + j, 1);
                    if (rc) return rc;
                }
        }
        return QPT_OK;
    };
    const int rc = all_batches();
    // the caller's stream waits for lane 1 also when a launch failed midway
    if (lane_b_used) {
        HIP_TRY(c, hipEventRecord(c->ev_lane_out, c->lstream));
        HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_lane_out, 0));
    }
    return rc;
}

int qpt_readback(qpt_ctx *c, double *sum_rgb, uint32_t *counts, int dst_is_device)
{
    if (!c) return QPT_E_INVALID;
    if (!c->bound) return fail(c, QPT_E_STATE, "readback before bind_workspace");
    DeviceGuard g(c->device);
    size_t npix = (size_t)c->W * c->H;
    hipMemcpyKind k = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (sum_rgb) HIP_TRY(c, hipMemcpyAsync(sum_rgb, c->pool.fb_sum, npix * 3 * 8, k, c->stream));
    if (counts) HIP_TRY(c, hipMemcpyAsync(counts, c->pool.fb_count, npix * 4, k, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    // report (and clear) a stop request; the buffers hold what was rendered
    if (c->abort_host && __atomic_exchange_n(c->abort_host, 0u, __ATOMIC_SEQ_CST))
        return fail(c, QPT_E_ABORTED, "rendering was aborted: the counts show the passes done");
    return QPT_OK;
}

int qpt_abort(qpt_ctx *c)
{
    if (!c) return QPT_E_INVALID;
    if (!c->abort_host) return QPT_E_STATE;
    __atomic_store_n(c->abort_host, 1u, __ATOMIC_SEQ_CST);
    return QPT_OK;
}

int qpt_get_stats(qpt_ctx *c, qpt_stats *out)
{
    if (!c || !out) return QPT_E_INVALID;
    if (!c->bound) return fail(c, QPT_E_STATE, "no workspace bound");
    DeviceGuard g(c->device);
    unsigned long long s[8];
    HIP_TRY(c, hipMemcpyAsync(s, c->pool.stats, sizeof s, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    out->rays_extension = s[0];
    out->rays_shadow = s[1];
    out->paths = s[2];
    out->passes = s[2] / ((uint64_t)c->W * c->H);
    out->nodes_extension = s[4];
    out->tris_extension = s[5];
    out->nodes_shadow = s[6];
    out->tris_shadow = s[7];
    return QPT_OK;
}

int qpt_profile(qpt_ctx *c, int enable)
{
    if (!c) return QPT_E_INVALID;
    if (c->device < 0) return fail(c, QPT_E_STATE, "context has no device");
    DeviceGuard g(c->device);
    if (enable) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        c->prof.clear();
    }
    c->profiling = enable != 0;
    return QPT_OK;
}

int qpt_profile_read(qpt_ctx *c, qpt_kernel_time *out)
{
    if (!c || !out) return QPT_E_INVALID;
    if (c->device < 0) return fail(c, QPT_E_STATE, "context has no device");
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < QPT_K_KINDS; ++k) out[k] = qpt_kernel_time{0, 0, 0.0};
    for (const EventProfiler::Rec &r : c->prof.recs) {
        if (!r.a || !r.b || r.kind < 0 || r.kind >= QPT_K_KINDS) continue;
        float ms = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&ms, r.a, r.b));
        out[r.kind].launches++;
        out[r.kind].total_ms += ms;
    }
    return QPT_OK;
}

int qpt_debug_sample_bits(qpt_ctx *c, const uint64_t *idx, const uint32_t *dim, uint32_t n, int scramble,
                          uint32_t *out)
{
    if (!c || (n && (!idx || !dim || !out))) return QPT_E_INVALID;
    if (!c->bound) return fail(c, QPT_E_STATE, "no workspace bound");
    if (!n) return QPT_OK;
    DeviceGuard g(c->device);
    HIP_TRY(c, launch_debug_sample_bits(c->frame, idx, dim, n, scramble, out, c->stream));
    return QPT_OK;
}

int qpt_debug_wave_sum(qpt_ctx *c, const uint32_t *in, uint32_t n, uint32_t *out)
{
    if (!c || (n && (!in || !out)) || (n & 63u)) return QPT_E_INVALID;
    if (c->device < 0) return fail(c, QPT_E_STATE, "context has no device");
    if (!n) return QPT_OK;
    DeviceGuard g(c->device);
    HIP_TRY(c, launch_debug_wave_sum(in, n, out, c->stream));
    return QPT_OK;
}

int qpt_debug_pixel_index(qpt_ctx *c, uint64_t pass, uint64_t *out)
{
    if (!c || !out) return QPT_E_INVALID;
    if (!c->bound) return fail(c, QPT_E_STATE, "no workspace bound");
    u128 last = (u128)(pass + 1) * c->frame.S;
    if (last >> 64) return fail(c, QPT_E_INVALID, "pass overflows 64-bit sample indices");
    DeviceGuard g(c->device);
    HIP_TRY(c, launch_debug_pixel_index(c->frame, pass, out, c->stream));
    return QPT_OK;
}

int qpt_debug_trace(qpt_ctx *c, const float *rays, uint32_t n, int any_hit, int brute_force, float *t,
                    uint32_t *tri, float *b12, uint32_t *stack_max)
{
    if (!c || (n && (!rays || !tri))) return QPT_E_INVALID;
    if (!any_hit && n && (!t || !b12)) return fail(c, QPT_E_INVALID, "closest hit needs t and b12");
    if (!c->bound) return fail(c, QPT_E_STATE, "no workspace bound");
    if (!n) return QPT_OK;
    DeviceGuard g(c->device);
    HIP_TRY(c, launch_debug_trace(c->frame, c->pool, rays, n, any_hit, brute_force, t, tri, b12,
                                  brute_force ? nullptr : stack_max, c->stream));
    return QPT_OK;
}

int qpt_guide_config(qpt_ctx *c, const qpt_guide_opts *o)
{
    if (!c || !o) return QPT_E_INVALID;
    if (!(o->alpha >= 0.0f && o->alpha < 1.0f) || !(o->lr > 0.0f) || o->batch > (1u << 22) || o->train > 64)
        return fail(c, QPT_E_INVALID,
                    "guide options out of range (alpha in [0, 1), lr > 0, batch <= 2^22, train <= 64)");
    c->gopts = *o;
    return QPT_OK;
}

int qpt_guide_set_weights(qpt_ctx *c, const float *params)
{
    if (!c || !params) return QPT_E_INVALID;
    if (!c->bound) return fail(c, QPT_E_STATE, "guide weights before bind_workspace");
    for (uint32_t p = 0; p < kGuideParams; ++p)
        if (!std::isfinite(params[p])) return fail(c, QPT_E_INVALID, "non-finite guide parameter");
    DeviceGuard g(c->device);
    HIP_TRY(c, hipMemcpyAsync(c->gt.master, params, kGuideParams * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->gt.m, 0, kGuideParams * 4, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->gt.v, 0, kGuideParams * 4, c->stream));
    HIP_TRY(c, launch_guide_frag(c->gt, c->stream, c->pub_frag[0], c->pub_bias[0], c->pub_frag[1], c->pub_bias[1]));
    HIP_TRY(c, launch_guide_ring_clear(c->gt, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->guide_weights = true;
    c->guide_steps = 0;
    return QPT_OK;
}

int qpt_guide_get_state(qpt_ctx *c, float *params, float *m, float *v, uint32_t *steps)
{
    if (!c) return QPT_E_INVALID;
    if (!c->bound || !c->guide_weights) return fail(c, QPT_E_STATE, "no guide weights");
    DeviceGuard g(c->device);
    if (params) HIP_TRY(c, hipMemcpyAsync(params, c->gt.master, kGuideParams * 4, hipMemcpyDeviceToHost, c->stream));
    if (m) HIP_TRY(c, hipMemcpyAsync(m, c->gt.m, kGuideParams * 4, hipMemcpyDeviceToHost, c->stream));
    if (v) HIP_TRY(c, hipMemcpyAsync(v, c->gt.v, kGuideParams * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (steps) *steps = c->guide_steps;
    return QPT_OK;
}

int qpt_guide_set_state(qpt_ctx *c, const float *params, const float *m, const float *v, uint32_t steps)
{
    if (!c || !params || !m || !v) return QPT_E_INVALID;
    if (!c->bound) return fail(c, QPT_E_STATE, "guide state before bind_workspace");
    for (uint32_t p = 0; p < kGuideParams; ++p)
        if (!std::isfinite(params[p]) || !std::isfinite(m[p]) || !(v[p] >= 0.0f) || !std::isfinite(v[p]))
            return fail(c, QPT_E_INVALID, "guide state must be finite (second moments >= 0)");
    int rc = qpt_guide_set_weights(c, params);
    if (rc) return rc;
    DeviceGuard g(c->device);
    HIP_TRY(c, hipMemcpyAsync(c->gt.m, m, kGuideParams * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->gt.v, v, kGuideParams * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->guide_steps = steps;
    return QPT_OK;
}

int qpt_guide_get_weights(qpt_ctx *c, float *params, uint32_t *steps)
{
    if (!c) return QPT_E_INVALID;
    if (!c->bound || !c->guide_weights) return fail(c, QPT_E_STATE, "no guide weights");
    DeviceGuard g(c->device);
    if (params) HIP_TRY(c, hipMemcpyAsync(params, c->gt.master, kGuideParams * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (steps) *steps = c->guide_steps;
    return QPT_OK;
}

int qpt_guide_debug_forward(qpt_ctx *c, const float *x, uint32_t n, float *out)
{
    if (!c || (n && (!x || !out))) return QPT_E_INVALID;
    if (!c->bound || !c->guide_weights) return fail(c, QPT_E_STATE, "no guide weights");
    if (!n) return QPT_OK;
    DeviceGuard g(c->device);
    Frame f = c->frame;
    HIP_TRY(c, launch_guide_debug_forward(f, x, n, out, c->stream));
    return QPT_OK;
}

int qpt_guide_debug_eval(qpt_ctx *c, const float *x, const float *wo, uint32_t n, float *mix)
{
    if (!c || (n && (!x || !wo || !mix))) return QPT_E_INVALID;
    if (!c->bound || !c->guide_weights) return fail(c, QPT_E_STATE, "no guide weights");
    if (!n) return QPT_OK;
    DeviceGuard g(c->device);
    // the renderer's copy of the newest weights (its output order, see k_guide_frag)
    Frame f = c->frame;
    f.guide.frag = c->pub_frag[c->last_buf];
    f.guide.bias = c->pub_bias[c->last_buf];
    HIP_TRY(c, launch_guide_debug_eval(f, c->pool, x, wo, n, mix, c->stream));
    return QPT_OK;
}

int qpt_guide_debug_grad(qpt_ctx *c, const float *x, const float *dirs, const float *w, uint32_t n, float *grad)
{
    if (!c || !n || !x || !dirs || !w || !grad) return QPT_E_INVALID;
    if (!c->bound || !c->guide_weights) return fail(c, QPT_E_STATE, "no guide weights");
    DeviceGuard g(c->device);
    HIP_TRY(c, launch_guide_debug_grad(c->frame, c->gt, x, dirs, w, n, grad, 0, 0u, 0.0f, c->stream, nullptr, nullptr,
                                       nullptr, nullptr));
    return QPT_OK;
}

int qpt_guide_debug_train(qpt_ctx *c, const float *x, const float *dirs, const float *w, uint32_t n, float lr,
                          float *grad)
{
    if (!c || !n || !x || !dirs || !w || !(lr > 0.0f)) return QPT_E_INVALID;
    if (!c->bound || !c->guide_weights) return fail(c, QPT_E_STATE, "no guide weights");
    DeviceGuard g(c->device);
    ++c->guide_steps;
    HIP_TRY(c, launch_guide_debug_grad(c->frame, c->gt, x, dirs, w, n, grad, 1, c->guide_steps, lr, c->stream,
                                       c->pub_frag[0], c->pub_bias[0], c->pub_frag[1], c->pub_bias[1]));
    return QPT_OK;
}

int qpt_guide_loss(qpt_ctx *c, double *loss, double *weight_sum)
{
    if (!c) return QPT_E_INVALID;
    if (!c->bound) return fail(c, QPT_E_STATE, "no workspace bound");
    DeviceGuard g(c->device);
    float sc[2];
    HIP_TRY(c, hipMemcpyAsync(sc, c->gt.scalars, sizeof sc, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (loss) *loss = sc[0] > 0.0f ? (double)sc[1] / (double)sc[0] : 0.0;
    if (weight_sum) *weight_sum = sc[0];
    return QPT_OK;
}

int qpt_guide_debug_records(qpt_ctx *c, uint32_t *ident, float *rec, uint32_t cap, uint32_t *count)
{
    if (!c || !count || (cap && (!ident || !rec))) return QPT_E_INVALID;
    if (!c->bound) return fail(c, QPT_E_STATE, "no workspace bound");
    if (!c->last_batch.valid) return fail(c, QPT_E_STATE, "no batch rendered since the workspace was bound");
    DeviceGuard g(c->device);
    // the caller's stream has waited for lane 1 at the end of qpt_render_pass
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int lane = c->last_batch.lane;
    const Pool &P = lane ? c->pool_b : c->pool;
    uint32_t n = 0;
    HIP_TRY(c, hipMemcpyAsync(&n, P.counters + 127, sizeof n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    n = std::min<uint32_t>(n, c->frame.guide.rec_cap);
    *count = n;
    Frame f = c->frame;
    f.guide.rec = c->lane_rec[lane];
    HIP_TRY(c, launch_debug_records(f, P, c->last_batch.p0, c->last_batch.np, c->last_batch.pass0, c->last_batch.nb,
                                    std::min(n, cap), ident, rec, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return QPT_OK;
}

int qpt_guide_debug_mixture(qpt_ctx *c, const float *out40, const float *dirs, const float *u, uint32_t n,
                            float *pdf, float *sample)
{
    if (!c || (n && (!out40 || !dirs || !u || !pdf || !sample))) return QPT_E_INVALID;
    if (c->device < 0) return fail(c, QPT_E_STATE, "context has no device");
    if (!n) return QPT_OK;
    DeviceGuard g(c->device);
    HIP_TRY(c, launch_guide_debug_mixture(out40, dirs, u, n, pdf, sample, c->stream));
    return QPT_OK;
}

/* host-side table access (no device needed), for cross-checks of the
 * builders against an independent implementation */
int qpt_debug_light_tables(const qpt_ctx *c, uint32_t *emit_tri, double *prob, uint32_t *alias, double *pmf,
                           uint32_t *count)
{
    if (!c || !count) return QPT_E_INVALID;
    if (!c->scene_ok) return QPT_E_STATE;
    size_t ne = c->emit_input_tri.size();
    *count = (uint32_t)ne;
    for (size_t e = 0; e < ne; ++e) {
        if (emit_tri) emit_tri[e] = c->emit_input_tri[e];
        if (prob) prob[e] = c->alias_prob[e];
        if (alias) alias[e] = c->alias_idx[e];
        if (pmf) pmf[e] = c->emit_pmf[e];
    }
    return QPT_OK;
}

int qpt_debug_light_tree(const qpt_ctx *c, float *sphere4, float *flux6, int32_t *left, uint32_t *first,
                         uint32_t *count, uint32_t *emit, uint32_t *weight, uint32_t *num_nodes)
{
    if (!c || !num_nodes) return QPT_E_INVALID;
    if (!c->scene_ok) return QPT_E_STATE;
    const size_t nn = c->lt_nodes.size();
    *num_nodes = (uint32_t)nn;
    for (size_t k = 0; k < nn; ++k) {
        const LtNode &nd = c->lt_nodes[k];
        if (sphere4) {
            sphere4[4 * k + 0] = nd.sphere.x;
            sphere4[4 * k + 1] = nd.sphere.y;
            sphere4[4 * k + 2] = nd.sphere.z;
            sphere4[4 * k + 3] = nd.sphere.w;
        }
        if (flux6)
            for (int r = 0; r < 6; ++r) flux6[6 * k + r] = nd.flux[r];
        if (left) left[k] = nd.left;
        if (first) first[k] = nd.first;
        if (count) count[k] = nd.count;
    }
    if (emit) std::memcpy(emit, c->lt_emit.data(), c->lt_emit.size() * 4);
    if (weight) std::memcpy(weight, c->lt_w.data(), c->lt_w.size() * 4);
    return QPT_OK;
}

int qpt_debug_env_pyramid(const qpt_ctx *c, uint32_t *levels, uint32_t *top, uint32_t *root, uint32_t *q,
                          uint32_t *oq)
{
    if (!c || !levels || !top || !root) return QPT_E_INVALID;
    if (!c->scene_ok) return QPT_E_STATE;
    *levels = c->ep_m;
    *top = c->ep_top;
    *root = c->ep_root;
    if (q) std::memcpy(q, c->ep_q.data(), c->ep_q.size() * 4);
    if (oq) std::memcpy(oq, c->ep_oq.data(), c->ep_oq.size() * 4);
    return QPT_OK;
}

int qpt_debug_env_sample(qpt_ctx *c, const uint32_t *uv, const float *nrm, uint32_t n, uint32_t mode,
                         uint32_t *texel, uint64_t *iv, uint64_t *iv_hit)
{
    if (!c || (n && (!uv || !nrm || !texel || !iv || !iv_hit)) || mode < 1 || mode > 2) return QPT_E_INVALID;
    if (!c->bound) return fail(c, QPT_E_STATE, "no workspace bound");
    if (!c->ep_m) return fail(c, QPT_E_STATE, "no environment pyramid (needs a 2:1 power-of-two map)");
    if (!n) return QPT_OK;
    DeviceGuard g(c->device);
    HIP_TRY(c, launch_debug_env_sample(c->frame, uv, nrm, n, mode, texel, iv, iv_hit, c->stream));
    return QPT_OK;
}

int qpt_debug_light_sample(qpt_ctx *c, const uint64_t *S, const float *x, const float *nrm, uint32_t n,
                           uint32_t *emitter, uint64_t *size, uint64_t *size_hit)
{
    if (!c || (n && (!S || !x || !nrm || !emitter || !size || !size_hit))) return QPT_E_INVALID;
    if (!c->bound) return fail(c, QPT_E_STATE, "no workspace bound");
    if (c->emit_input_tri.empty()) return fail(c, QPT_E_STATE, "the scene has no triangle lights");
    if (!n) return QPT_OK;
    DeviceGuard g(c->device);
    HIP_TRY(c, launch_debug_light_sample(c->frame, S, x, nrm, n, emitter, size, size_hit, c->stream));
    return QPT_OK;
}

int qpt_debug_env_tables(const qpt_ctx *c, uint32_t *row_q, uint32_t *col_q, float *texel_pdf)
{
    if (!c) return QPT_E_INVALID;
    if (!c->scene_ok || !c->ew) return QPT_E_STATE;
    if (row_q) std::memcpy(row_q, c->env_row.data(), c->env_row.size() * 4);
    if (col_q) std::memcpy(col_q, c->env_col.data(), c->env_col.size() * 4);
    if (texel_pdf)
        for (size_t q = 0; q < c->env_texel.size(); ++q) texel_pdf[q] = c->env_texel[q].w;
    return QPT_OK;
}

int qpt_debug_bvh_nodes(const qpt_ctx *c, float *nodes32, uint32_t *tri_order, uint32_t *num_nodes)
{
    if (!c || !num_nodes) return QPT_E_INVALID;
    if (!c->bvh_ok) return QPT_E_STATE;
    *num_nodes = (uint32_t)c->gnodes.size();
    if (nodes32) std::memcpy(nodes32, c->gnodes.data(), c->gnodes.size() * sizeof(Node));
    if (tri_order)
        for (size_t k = 0; k < c->gtris.size(); ++k) std::memcpy(&tri_order[k], &c->gtris[k].v1.w, 4);
    return QPT_OK;
}

}  // extern "C"
