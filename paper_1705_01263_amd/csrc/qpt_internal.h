// Internal layout shared by the host side and the HIP kernels of libqpt.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace qpt {

constexpr uint32_t kMaxDims = 256;       // sample dimensions with a base table
constexpr uint32_t kShortStack = 15;     // traversal stack entries per ray kept in LDS
// the tree's first nodes (its top levels: the host numbers them breadth-first)
// are copied into LDS by every traversal block: 4 KB of quantised nodes, so
// that 8 blocks of 256 threads still fit one CU with their stacks (8 x 19 KB)
constexpr uint32_t kTopNodes = 64;
constexpr uint32_t kMaxTreeDepth = 32;   // depth limit of the binary build tree
constexpr uint32_t kTravBlocksPerCU = 16; // traversal grid: 16 blocks of 4 waves per CU, twice what is resident
constexpr uint32_t kShadeGuidedBlock = 512;     // guided shading: 8 waves share the weights in LDS
constexpr uint32_t kShadeGuidedBlocksPerCU = 2;  // 69 KB of LDS per block (weights, 512 mixtures)
// waves per SIMD of two such blocks on a CU: the register budget the kernel is compiled for (128 VGPRs)
constexpr uint32_t kShadeGuidedWavesPerSIMD = kShadeGuidedBlocksPerCU * kShadeGuidedBlock / 64 / 4;
constexpr uint32_t kShadeGuidedGridPerCU = 8;    // its grid: blocks per CU
constexpr uint32_t kBlock = 256;         // threads per block for the path kernels
constexpr uint32_t kShadeBlock = 256;    // threads per block of the shading kernel (its queue appends are per block)
constexpr uint32_t kNoHit = 0xffffffffu;
// per-lane counter words beyond the queue counts: the abort decision latched
// by a pass's first batch, and whether the current batch renders nothing
constexpr uint32_t kPassLatch = 125, kSkip = 126;
// regeneration (render option regen_paths): the two ping-pong queue counts,
// the shadow-ray count of the current iteration, the terminated slots, the
// next path id to start, and the paths not yet finished (alive + not started),
// in the second half of the lane's 256 counter words; the three that every
// wave of the shading kernel appends to sit in cache lines of their own
constexpr uint32_t kCounters = 256;
constexpr uint32_t kRgQ0 = 128, kRgQ1 = 160, kRgSh = 192, kRgDead = 224, kRgNext = 129, kRgLeft = 130;
// the queue count word of iteration t's queue q_ext[t & 1]
__host__ __device__ constexpr uint32_t rg_queue_count(uint32_t t) { return (t & 1u) ? kRgQ1 : kRgQ0; }
static_assert(kRgQ0 != kRgQ1 && kRgQ0 != kRgSh && kRgQ0 != kRgDead && kRgQ0 != kRgNext && kRgQ0 != kRgLeft &&
                  kRgQ1 != kRgSh && kRgQ1 != kRgDead && kRgQ1 != kRgNext && kRgQ1 != kRgLeft && kRgSh != kRgDead &&
                  kRgSh != kRgNext && kRgSh != kRgLeft && kRgDead != kRgNext && kRgDead != kRgLeft &&
                  kRgNext != kRgLeft,
              "regeneration counter words are distinct");
static_assert(kRgQ0 >= 128 && kRgQ1 < kCounters && kRgSh < kCounters && kRgDead < kCounters && kRgNext >= 128 &&
                  kRgLeft >= 128 && kRgLeft < kCounters,
              "regeneration counters lie above the per-depth and shadow counts");

// One base of the Halton sequence with its strength-reduced divisions
// (Appendix A.2: integer evaluation, division by multiplication).
// Digits are processed in chunks of e digits, B = b^e < 2^32.
struct HaltonBase {
    uint32_t b;        // prime base
    uint32_t f;        // scrambling multiplier: digit a -> f*a mod b
    uint32_t e;        // digits per chunk
    uint32_t m32;      // magic for n/b, n < 2^32
    uint32_t sh32;     // post-shift for n/b
    uint32_t shB;      // post-shift for n/B
    uint64_t B;        // b^e
    uint64_t m64;      // magic for n/B, n < 2^64
};

// 4-wide BVH node (128 bytes, one L2 line): the four children's boxes as
// SoA float4 (component c = child c) and their references.
// ref >= 0: inner node index; ref == kEmptyChild: unused slot;
// other ref < 0: leaf, ~ref = first << 3 | (count - 1).
constexpr int32_t kEmptyChild = (int32_t)0x80000000;
struct alignas(16) Node {
    float4 lox, loy, loz;
    float4 hix, hiy, hiz;
    int4 ref;
    int4 pad;
};

// The same node quantised to 64 bytes (half an L2 line, four 16-byte loads):
// the children's boxes as 8-bit steps on a per-axis power-of-two grid from
// the lower corner of their union, rounded outwards (each child box holds
// its full-precision box), so traversal visits a superset of the nodes it
// would with full boxes and finds the same closest hit.
//   w0: lower corner xyz (FP32), biased exponents of the three grid steps
//       (bytes 0-2: 2^(e - 127)) and the number of used slots (byte 3);
//   w1: lo.x, lo.y, lo.z, hi.x steps, byte c = child c;
//   w2: hi.y, hi.z steps, references of children 0 and 1;
//   w3: references of children 2 and 3, two unused words.
struct alignas(16) QNode {
    uint4 w0, w1, w2, w3;
};
static_assert(sizeof(QNode) == 64, "quantised node is 64 bytes");
// node formats of the device tree
constexpr uint32_t kNodeQuant = 0, kNodeFull = 1;

// Triangle in BVH order (48 bytes): v0.w = material, v1.w = input id,
// v2.w = emitter index (or kNoHit).
struct alignas(16) Tri {
    float4 v0, v1, v2;
};

// Light tree node (the many-light hierarchy of Sec. 2.1.1), 64 bytes:
// bounding sphere of the node's triangles, flux towards each emission region
// (the dominant-axis cells +x, -x, +y, -y, +z, -z of the sphere of
// directions), first of its two adjacent children (-1 for a leaf) and its
// range of emitters in leaf order.
struct alignas(16) LtNode {
    float4 sphere;    // centre xyz, radius
    float flux[6];
    int32_t left;
    uint32_t first, count;
    uint32_t pad[3];
};
static_assert(sizeof(LtNode) == 64, "light tree node is one 64-byte line");
constexpr uint32_t kLtLeaf = 8;   // emitters per leaf at most

struct alignas(16) Material {
    float4 albedo_rough;    // rho.rgb, alpha
    float4 emission_flags;  // Le.rgb, flags (bits)
};

// The learned proposal's device state (a 32-64-64-64-40 network).
constexpr uint32_t kGuideParams = 13032;
constexpr uint32_t kGuideFrags = 56;    // forward weight fragments (64 lanes x 4 bf16 each)
constexpr uint32_t kGuideFragsT = 48;   // transposed fragments for the backward pass
constexpr uint32_t kRecF4 = 6;          // float4 per training record
constexpr uint32_t kRingF4 = 3;         // float4 per replay sample: (x, weight), (wo, -), (wi, -)

struct GuideDev {
    const uint2 *frag;       // kGuideFrags * 64: 4 bf16 per lane (MFMA A operands)
    const uint2 *fragT;      // kGuideFragsT * 64
    const float *bias;       // 4 x 64 (BF16-rounded values, layer 3 zero-padded)
    float bmin[3], binv[3];  // scene box for the position encoding: min corner, 1 / extent
    uint32_t alpha_thr;      // guide iff sample bits < alpha_thr (0: BSDF sampling only)
    float alpha;             // alpha_thr / 2^32
    uint32_t record;         // capture training records
    uint32_t max_vertex;     // guide and record at path vertices 1..max_vertex
    uint32_t rec_thr;        // record a vertex iff its hash < rec_thr (0xffffffff: every vertex)
    float4 *rec;             // kRecF4 float4 per record
    uint32_t rec_cap;
    uint32_t *rec_count;
};

struct Camera {
    float eye[3], fwd[3], right[3], up[3];
    float tan_half, aspect;
};

// Everything a kernel needs, by value (device pointers into the workspace).
struct Frame {
    // scene
    const Node *nodes;                    // node_format kNodeFull
    const QNode *qnodes;                  // node_format kNodeQuant
    uint32_t node_format;
    uint32_t top_nodes;                   // nodes [0, top_nodes) staged in LDS (quantised tree; <= kTopNodes)
    const Tri *tris;
    const Material *mats;
    uint32_t num_tris;
    // lights (emitter order = ascending input triangle id)
    uint32_t num_emit;
    const uint32_t *emit_tri;             // BVH-order triangle of emitter e
    const uint32_t *alias_idx;
    const unsigned long long *alias_thr;  // take column iff bits < thr (2^32 scale)
    const float *emit_pmf;                // realised selection probability
    const LtNode *lt_nodes;               // light tree (root = node 0)
    const uint32_t *lt_emit;              // leaf-order position -> emitter
    const uint32_t *lt_pos;               // emitter -> leaf-order position
    const uint32_t *lt_w;                 // leaf-order position -> cumulative 24-bit weight in its leaf
    // environment
    uint32_t env_w, env_h;
    const float4 *env_texel;              // rgb, solid-angle pdf
    const uint32_t *env_row;              // env_h entries, row_q[0] = 0
    const uint32_t *env_col;              // env_h * env_w
    const float *env_cos;                 // env_h + 1 row boundary cosines
    float p_env;                          // probability of choosing the environment
    // environment pyramid (finest level ep_m, 0 = none): split probabilities
    // (column, row | left column, row | right column, -) per node of levels
    // 0..ep_m-1, and per normal bin (stride ep_stride) the left-root
    // probability followed by the nodes of levels 0..ep_top-1
    const uint4 *ep_q;
    const uint4 *ep_oq;
    uint32_t ep_m, ep_top, ep_root, ep_stride;
    // Halton
    const HaltonBase *bases;              // kMaxDims
    uint32_t k2, l3;                      // 2^k >= W, 3^l >= H
    uint64_t S;                           // 2^k 3^l
    uint64_t p3, m_p3;                    // 3^l and its 64-bit magic
    uint32_t sh_p3, inv2k_mod_p3;         // (2^k)^-1 mod 3^l
    // learned proposal
    GuideDev guide;
    // camera and frame
    Camera cam;
    uint32_t W, H;
    // options
    uint32_t max_depth, rr, mode, scramble;
    uint32_t light_tree;                  // select triangle lights through the light tree
    uint32_t env_pyramid;                 // 0: 2D CDF, 1: pyramid, 2: pyramid with normal-weighted top levels
    uint32_t gauss_filter;                // film samples from the Gaussian pixel filter instead of the box
    uint32_t tail_depth;                  // 0, or the depth from which one launch finishes every path
    uint32_t regen;                       // live path slots while regenerating (0: one path per slot)
    uint32_t compress;                    // path state in the compressed layout (qpt_state_dev.h)
    const uint32_t *abort_word;           // host-mapped: non-zero once the caller asked to stop
};

// Path pool (structure of arrays, Sec. 3.1.1) and queues (Sec. 3.1.2).
struct Pool {
    uint32_t cap;
    float4 *ray_o;      // o.xyz, tmax
    float4 *ray_d;      // d.xyz, previous vertex (triangle | back-face bit 31, as bits)
    float4 *hit;        // t, tri (BVH order, bits), b1, b2
    float4 *thr;        // throughput.rgb, pdf of the last BSDF sample
    float4 *rad;        // radiance.rgb, - (indexed by the path's id in the batch; the slot without regeneration)
    unsigned long long *idx;   // Halton index of the path
    uint32_t *q_ext[2]; // extension-ray queues (ping-pong)
    uint32_t *q_dead;   // regeneration: slots whose paths terminated since the last regeneration
    uint2 *pv;          // regeneration: per slot, the id of its path in the batch and its next vertex
    float4 *sh_o;       // shadow ray o.xyz, tmax
    float4 *sh_d;       // shadow ray d.xyz, slot (bits)
    float4 *sh_c;       // pending contribution rgb, -
    uint32_t *counters;     // [0..63] ext counts per depth, [64..127] shadow counts
    int *gstack;            // traversal stack overflow, deep_stack entries per traversal thread
    uint32_t trav_threads;  // threads of the traversal grid (gstack stride)
    // [0] ext rays [1] shadow rays [2] paths [3] - [4] ext node visits
    // [5] ext triangle tests [6] shadow node visits [7] shadow triangle tests
    unsigned long long *stats;
    double *fb_sum;     // W*H*3
    uint32_t *fb_count; // W*H
};

// kernel kinds timed by the optional profiler
enum KernelKind { K_CLEAR = 0, K_GENERATE, K_TRACE, K_SHADE, K_SHADOW, K_ACCUMULATE, K_SHADE_GUIDED, K_GUIDE_TRAIN,
                  K_TAIL, K_KINDS };

// brackets every kernel launch of a batch with stream events when set
struct Profiler {
    // a span of work on s: events recorded before and after it
    virtual void begin(int kind, hipStream_t s) = 0;
    virtual void end(int kind, hipStream_t s) = 0;
    // one kernel: the two events its launch records at the dispatch's start and end
    virtual void kernel_events(int kind, hipEvent_t *start, hipEvent_t *stop) = 0;
    virtual ~Profiler() {}
};

// training state of the learned proposal (all device pointers)
struct GuideTrain {
    float *master, *m, *v;   // kGuideParams each, FP32
    uint2 *frag, *fragT;     // written from master after every step
    float *bias;             // 256
    float4 *ring;            // replay ring of training samples, kRingF4 float4 each
    uint32_t *ring_head;     // samples ever appended (the ring keeps the last ring_cap)
    uint32_t ring_cap;       // a power of two
    float *partial;          // blocks x kGuideParams unnormalised gradient sums
    float *scalars;          // [0] sum of loss weights [1] weighted loss sum; then both per training block
    uint32_t max_blocks;
};

// GPU BVH build (qpt_build.hip): linear BVH over Morton-sorted centroids,
// collapsed into 4-wide nodes on the device. Its temporaries come from the
// device region `scratch` (at least gpu_build_scratch_bytes(nv, nt) bytes,
// hipErrorInvalidValue otherwise); synchronises `s`, returns the nodes (root
// first), the leaf order of the triangles and the 4-wide depth. Needs nt > leaf.
size_t gpu_build_scratch_bytes(uint32_t nv, uint32_t nt);
hipError_t gpu_build_bvh(const float *pos, uint32_t nv, const uint32_t *idx, uint32_t nt, uint32_t leaf, float pad,
                         void *scratch, size_t scratch_bytes, hipStream_t s, std::vector<Node> &nodes,
                         std::vector<uint32_t> &order, uint32_t &depth);
// The library's one allocation-free scratch region: a file-scope device array
// of kStaticScratch bytes per GPU (qpt_build.hip), its device address looked
// up once per device (hipGetSymbolAddress with that device current).
constexpr size_t kStaticScratch = (size_t)64 << 20;
hipError_t static_scratch(int device, void **ptr);

// kernel launchers (qpt_kernels.hip)
hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_f64(double *p, size_t n, hipStream_t s);
hipError_t launch_render_batch(const Frame &f, const Pool &pool, uint32_t pix0, uint32_t npix,
                               uint64_t pass0, uint32_t npass, hipStream_t s, Profiler *prof);
// the same in two parts: the paths of a batch, then its framebuffer update
hipError_t launch_render_paths(const Frame &f, const Pool &pool, uint32_t pix0, uint32_t npix,
                               uint64_t pass0, uint32_t npass, hipStream_t s, Profiler *prof);
// the paths of a whole-frame batch through f.regen live slots with
// regeneration: iterations are launched in chunks; `left` (host-mapped, two
// words) receives the paths not yet finished after each chunk, `ev` (two
// events) marks each chunk's copy. Returns hipErrorUnknown if the paths do
// not finish within the iteration bound.
hipError_t launch_render_regen(const Frame &f, const Pool &pool, uint32_t npix, uint64_t pass0, uint32_t npass,
                               hipStream_t s, Profiler *prof, uint32_t *left, hipEvent_t ev[2]);
// (a batch that starts a pass latches the abort word; its other pixel chunks follow it)
hipError_t launch_accumulate(const Frame &f, const Pool &pool, uint32_t pix0, uint32_t npix, uint32_t npass,
                             hipStream_t s, Profiler *prof);
// guide launchers (qpt_guide.hip)
hipError_t launch_guide_frag(const GuideTrain &T, hipStream_t s, uint2 *pub_a, float *pub_ab, uint2 *pub_b,
                             float *pub_bb);
hipError_t launch_guide_debug_eval(const Frame &f, const Pool &pool, const float *x, const float *wo, uint32_t n,
                                   float *mix, hipStream_t s);
hipError_t launch_guide_finalize(const Frame &f, const Pool &pool, const GuideTrain &T, hipStream_t s);
hipError_t launch_guide_ring_clear(const GuideTrain &T, hipStream_t s);
hipError_t launch_guide_train_steps(const Frame &f, const GuideTrain &T, uint32_t batch, uint32_t step0,
                                    uint32_t nsteps, float lr, uint32_t seed, hipStream_t s, uint2 *pub_frag,
                                    float *pub_bias);
hipError_t launch_guide_debug_forward(const Frame &f, const float *x, uint32_t n, float *out, hipStream_t s);
hipError_t launch_guide_debug_grad(const Frame &f, const GuideTrain &T, const float *x, const float *dirs,
                                   const float *w, uint32_t n, float *grad, int adam, uint32_t step, float lr,
                                   hipStream_t s, uint2 *pub_a, float *pub_ab, uint2 *pub_b, float *pub_bb);
hipError_t launch_guide_debug_mixture(const float *out40, const float *dirs, const float *u, uint32_t n,
                                      float *pdf, float *sample, hipStream_t s);

hipError_t launch_debug_wave_sum(const uint32_t *in, uint32_t n, uint32_t *out, hipStream_t s);
hipError_t launch_debug_sample_bits(const Frame &f, const uint64_t *idx, const uint32_t *dim,
                                    uint32_t n, int scramble, uint32_t *out, hipStream_t s);
hipError_t launch_debug_pixel_index(const Frame &f, uint64_t pass, uint64_t *out, hipStream_t s);
hipError_t launch_debug_env_sample(const Frame &f, const uint32_t *uv, const float *nrm, uint32_t n, uint32_t mode,
                                   uint32_t *texel, uint64_t *iv, uint64_t *iv_hit, hipStream_t s);
hipError_t launch_debug_light_sample(const Frame &f, const uint64_t *S, const float *x, const float *nrm,
                                     uint32_t n, uint32_t *emitter, uint64_t *size, uint64_t *size_hit,
                                     hipStream_t s);
hipError_t launch_debug_records(const Frame &f, const Pool &pool, uint32_t pix0, uint32_t npix, uint64_t pass0,
                                uint32_t npass, uint32_t n, uint32_t *ident, float *out, hipStream_t s);
hipError_t launch_debug_trace(const Frame &f, const Pool &pool, const float *rays, uint32_t n, int any_hit,
                              int brute, float *t, uint32_t *tri, float *b12, uint32_t *depth, hipStream_t s);

}  // namespace qpt
