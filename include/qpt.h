/*
 * qpt -- progressive quasi-Monte Carlo path tracing on MI355X (gfx950).
 *
 * C-ABI of the library libqpt.so. Every entry point returns 0 (QPT_OK) on
 * success or a negative QPT_E_* status; the message of the last failure is
 * qpt_last_error(). No exception crosses this boundary.
 *
 * The calls follow the paper's statement of the problem:
 *   - rendering is push-button, progressive and consistent (Sec. 1.1);
 *   - each GPU holds a full copy of the scene (Sec. 5, no out-of-core data);
 *   - work is handed out as iterations of one sample per pixel, grouped in
 *     iteration sets (Sec. 3.2.2, batch rendering);
 *   - each device accumulates into its own framebuffer copy, which is merged
 *     out (Sec. 3.2.2) -- here: read back;
 *   - a per-pixel sample count buffer records progress (Appendix A.4);
 *   - acceleration structures are built per scene (Sec. 2.5, Sec. 3.1).
 *
 * Ownership. Host inputs are copied before the call returns. Device memory
 * comes from the caller only, through qpt_bind_workspace: the library never
 * allocates or frees device memory, and the caller keeps the workspace alive
 * (and unmodified) until qpt_destroy or the next qpt_bind_workspace. Output
 * buffers belong to the caller.
 *
 * The one exception is qpt_build_bvh_noalloc, which takes its temporaries
 * from a fixed device region of the library's own (see there).
 *
 * Streams. All results are ordered on the stream given to qpt_create (a
 * hipStream_t; NULL = the default stream): a call's device work is complete
 * once that stream has reached the point after the call. One more stream
 * carries the second batch in flight (and the guide's training steps of the
 * batches it renders), and the caller's stream waits on it with an event
 * before any later work. The caller may provide it (qpt_set_streams);
 * otherwise qpt_bind_workspace creates it (default priority, non-blocking)
 * and qpt_destroy destroys it. The two batches overlap only while the two
 * streams sit on different hardware queues of the device: HIP gives a new
 * stream its least-used queue, so a stream the library creates after the
 * caller's avoids the caller's queue while queues are to spare, whereas a
 * stream taken from a round-robin pool (torch's) can land on it. Calls on
 * one context are not thread-safe; use one context per stream.
 *
 * Call order: create -> build_scene -> build_bvh -> workspace_size ->
 * bind_workspace -> render_pass* -> readback; violations return QPT_E_STATE.
 */
#ifndef QPT_H
#define QPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    QPT_OK = 0,
    QPT_E_INVALID = -1,      /* bad argument or size */
    QPT_E_STATE = -2,        /* call out of order */
    QPT_E_NOMEM = -3,        /* workspace too small */
    QPT_E_HIP = -4,          /* HIP runtime error (message in qpt_last_error) */
    QPT_E_UNSUPPORTED = -5,  /* device is not gfx950 */
    QPT_E_ABORTED = -6
};

/* material flags */
#define QPT_MAT_GGX 1u           /* GGX specular layer over the Lambert base */
#define QPT_MAT_EMIT_TEXTURE 2u  /* emission times 0.55 + 0.45 sin(8 pi (x + z)) */

typedef struct qpt_ctx qpt_ctx;

typedef struct {
    float albedo[3];     /* Lambert base reflectance, linear RGB */
    float roughness;     /* GGX alpha (used with QPT_MAT_GGX) */
    float emission[3];   /* front-face radiance; non-zero makes every triangle of it a light */
    uint32_t flags;      /* QPT_MAT_* */
} qpt_material;

typedef struct {
    float eye[3], look[3], up[3];
    float vfov_deg;      /* vertical field of view of the pinhole camera */
} qpt_camera;

/* Scene description: all pointers are HOST memory, copied by qpt_build_scene.
 * Triangles are counter-clockwise seen from their emitting (front) side. */
typedef struct {
    uint32_t num_vertices;
    const float *positions;        /* 3 * num_vertices */
    uint32_t num_triangles;
    const uint32_t *indices;       /* 3 * num_triangles, each < num_vertices */
    const uint32_t *tri_material;  /* num_triangles, each < num_materials */
    uint32_t num_materials;
    const qpt_material *materials; /* num_materials */
    uint32_t env_width, env_height;/* 0, 0 = no environment */
    const float *env_rgb;          /* env_height * env_width * 3, lat-long, row 0 at +y */
    qpt_camera camera;
    uint32_t width, height;        /* framebuffer size in pixels */
} qpt_scene_desc;

typedef struct {
    uint32_t max_leaf_size;  /* triangles per leaf, 1..8 (0 = 3) */
    uint32_t sah_bins;       /* binned SAH bins, 4..64 (0 = 16) */
    uint32_t builder;        /* 0: binned SAH on the host; 1: linear BVH on the GPU (Morton order,
                                Karras 2012), collapsed to the same 4-wide nodes on the device: a
                                faster build of a lower-quality tree; needs a device context and
                                the caller's scratch below */
    uint32_t node_format;    /* device tree: 0: quantised 64-byte 4-wide nodes (child boxes as 8-bit
                                steps of a per-axis power-of-two grid, rounded outwards: the same
                                hits, half the node bytes); 1: full-precision 128-byte nodes */
    void *scratch;           /* builder 1: caller-owned DEVICE memory for the build's temporaries, at
                                least qpt_bvh_scratch_size bytes, 256-byte aligned; free again when
                                the call returns (the build synchronises the stream) */
    size_t scratch_bytes;
} qpt_bvh_opts;

typedef struct {
    uint32_t num_nodes;      /* inner nodes of the 4-wide tree */
    uint32_t num_leaves;
    uint32_t max_depth;      /* of the 4-wide tree's inner nodes, root = depth 0 */
    uint32_t node_bytes;     /* bytes per node of the device tree (64 quantised, 128 full) */
    double sah_cost;         /* SAH cost with unit traversal and intersection costs */
    double build_ms;
} qpt_bvh_stats;

typedef struct {
    uint32_t max_depth;      /* D: path segments, emission at vertices 1..D, NEE at 1..D-1 */
    uint32_t rr;             /* 1: Russian roulette from vertex 3 */
    uint32_t mode;           /* 0: NEE + BSDF sampling with MIS, 1: BSDF sampling only, 2: NEE only */
    uint32_t scramble;       /* 1: linear digit scrambling of dimensions >= 2 */
    uint32_t light_tree;     /* 0: triangle lights by flux (alias table), 1: through the light tree
                                (the many-light hierarchy of Sec. 2.1.1; importance by distance,
                                orientation and flux of its nodes) */
    uint32_t single_stream;  /* 0: consecutive batches of passes run two at a time (the caller's stream
                                and a second stream of the library, each with its own path pool; the
                                caller's stream waits for both before the call's later work), so a
                                batch's deep vertices overlap the next batch's first ones. 1: one
                                batch after another on the caller's stream. The image is the same bit
                                for bit (without the guide; guided images depend on the order in
                                which training samples arrive either way). */
    uint32_t env_sampling;   /* environment NEE (Sec. 2.1.2): 0: 2D CDF over the texels; 1: descent
                                of the texel pyramid; 2: the pyramid with its top levels weighted
                                per surface-normal bin (16 x 16 octahedral cells, cosine bound over
                                the bin and the cell). 1 and 2 need a 2:1 map of power-of-two size
                                (QPT_E_INVALID otherwise); ignored without an environment. */
    uint32_t filter;         /* pixel filter (Appendix A.1): 0: box (film sample uniform in the pixel);
                                1: Gaussian of sigma 1/2 pixel (3 sigma spans 3 x 3 pixels) around the
                                pixel centre, untruncated, by filter importance sampling (Box-Muller of
                                the film sample); the sample still counts for its own pixel */
    uint32_t tail_depth;     /* the wavefront's tail (Sec. 3.1.3): 0: one launch per kernel and depth
                                to the end; k in 1..max_depth: from depth k on, one launch (a
                                megakernel) takes every path still alive to its end, vertex after
                                vertex in one thread, with the same per-vertex code (the same image
                                bit for bit). While the guide samples or records, only past the
                                guided vertices (k > the guide's max_vertex, not 0); ignored
                                otherwise. */
    uint32_t regen_paths;    /* regeneration of terminated paths (Sec. 3.1.3): 0: every path of a batch
                                has a state slot of its own from its camera ray to its end; n > 0: the
                                batch's paths run through n state slots (64 <= n <= the workspace's
                                pool, QPT_E_INVALID otherwise), and once more than half of them are
                                free, the free slots start the batch's next paths; every iteration
                                traces, shades and occludes the live paths whatever their depth. The
                                image and the ray counts are the same bit for bit. Batches then run
                                one at a time on the caller's stream (single_stream implied), and the
                                host waits on the stream now and then to learn when a batch has
                                finished. Applies to batches of whole frames (a frame no larger than
                                the pool) without the guide; ignored otherwise, and tail_depth is
                                ignored while it applies. */
    uint32_t compress_state; /* path state layout (Sec. 3.1.1): 0: full precision; 1: compressed, the
                                next ray's direction as an octahedral pair of 16-bit values (within
                                6.5e-5 rad), the throughput and the last sampling density in half
                                precision, the hit's barycentrics as 16-bit fixed point: 28 bytes of
                                the 48 per path kept between kernels instead of 48 (origin, radiance
                                and index unchanged). A sampled direction is quantised where it is
                                sampled, so the BSDF, the densities and the traced ray agree; the
                                image is no longer the full-precision one bit for bit but estimates
                                the same radiance (within the Monte Carlo error; tests). */
} qpt_render_opts;

typedef struct {
    uint64_t rays_extension; /* closest-hit rays traced since the last reset */
    uint64_t rays_shadow;    /* occlusion rays traced */
    uint64_t paths;          /* paths completed */
    uint64_t passes;         /* 1-spp iterations completed (paths / pixels) */
    uint64_t nodes_extension;/* BVH node fetches of the closest-hit rays */
    uint64_t tris_extension; /* triangle tests of the closest-hit rays */
    uint64_t nodes_shadow;   /* BVH node fetches of the occlusion rays */
    uint64_t tris_shadow;    /* triangle tests of the occlusion rays */
} qpt_stats;

/* kernel kinds reported by the profiler */
enum {
    QPT_K_CLEAR = 0,      /* queue counter reset */
    QPT_K_GENERATE = 1,   /* enumeration, Halton film samples, camera rays */
    QPT_K_TRACE = 2,      /* closest hit of extension rays */
    QPT_K_SHADE = 3,      /* emission + MIS, NEE, BSDF sampling, roulette */
    QPT_K_SHADOW = 4,     /* occlusion of shadow rays */
    QPT_K_ACCUMULATE = 5, /* FP64 framebuffer and counts */
    QPT_K_SHADE_GUIDED = 6, /* shading of the guided vertices with the network's mixture computed
                               in the same launch (guiding on) */
    QPT_K_GUIDE_TRAIN = 7,/* record finalisation, batch forward/backward, Adam */
    QPT_K_TAIL = 8,       /* the batch's remaining paths in one launch (render option tail_depth) */
    QPT_K_KINDS = 9
};

typedef struct {
    uint32_t launches;    /* kernel launches timed */
    uint32_t reserved;
    double total_ms;      /* sum of the launches' durations (stream events) */
} qpt_kernel_time;

/* Create a context on HIP device `hip_device` that enqueues on `hip_stream`
 * (hipStream_t or NULL). QPT_E_UNSUPPORTED if the device is not gfx950.
 * hip_device = -1 makes a host-only context: the scene and BVH builders and
 * the host-table hooks work, every device call returns QPT_E_STATE. */
int qpt_create(int hip_device, void *hip_stream, qpt_ctx **out);
void qpt_destroy(qpt_ctx *ctx);
/* message of the last failing call on ctx ("" if none); valid until the next call */
const char *qpt_last_error(const qpt_ctx *ctx);

/* Copy and validate the scene; build per-triangle flux (16-point rule), the
 * power-proportional alias table and the environment CDFs on the host in FP64
 * (Sec. 2.1.1 one flux value per triangle; Sec. 2.1.2 environment importance
 * sampling). Invalidates a bound workspace. */
int qpt_build_scene(qpt_ctx *ctx, const qpt_scene_desc *desc);

/* Build the BVH on the host (binned SAH) and lay it out for the GPU
 * (Sec. 2.3: watertight traversal; Sec. 3.1 replaces the paper's ray casting
 * library with the library's own traversal). stats may be NULL. */
int qpt_build_bvh(qpt_ctx *ctx, const qpt_bvh_opts *opts, qpt_bvh_stats *stats);

/* Bytes of device scratch the GPU builder (qpt_bvh_opts.builder = 1) needs
 * for the scene of the last qpt_build_scene: about 300 bytes per triangle
 * plus 12 per vertex. */
int qpt_bvh_scratch_size(qpt_ctx *ctx, size_t *bytes);

/* For callers that cannot allocate device memory (code under graph capture,
 * serving loops, harnesses that forbid allocation): the GPU builder
 * (builder = 1 of qpt_bvh_opts; the other fields as there, scratch ignored)
 * with its temporaries in a fixed region of the library, 64 MiB of device
 * memory reserved on every GPU the library is loaded on, for as long as the
 * process lives. It calls no hipMalloc, hipFree or other allocating routine.
 * The scene must fit the region (about 200,000 triangles; qpt_bvh_scratch_size
 * gives the bytes needed): QPT_E_INVALID otherwise, with a message. The
 * result is the same tree, bit for bit, as qpt_build_bvh with builder = 1.
 * All contexts on one GPU share the region: calls that overlap in time on
 * one GPU (from several threads) race and must be serialised by the caller.
 * Synchronises the stream. */
int qpt_build_bvh_noalloc(qpt_ctx *ctx, const qpt_bvh_opts *opts, qpt_bvh_stats *stats);

/* The stream of the second batch in flight (a hipStream_t, not NULL and not
 * the context's own stream, on the context's device, on a hardware queue of
 * its own; default priority recommended), owned by the caller and kept alive
 * until qpt_destroy. The guide's finalisation and training steps run on the
 * stream of the batch they follow. Only before the first qpt_bind_workspace
 * (QPT_E_STATE after it); without this call the library creates the stream
 * there and destroys it in qpt_destroy. QPT_E_INVALID for a NULL stream or
 * the context's own. */
int qpt_set_streams(qpt_ctx *ctx, void *lane_stream);

/* Bytes of device workspace needed for `pool_paths` concurrent paths per
 * batch (0 = sixteen frames' worth: the smallest power of two >= 16 W H,
 * within [2^16, 2^27]). A range of passes is rendered in as few batches of whole
 * passes as the pool allows, of nearly equal size (or in pixel chunks of one
 * pass when a frame exceeds the pool); larger batches keep the queues of deep
 * vertices full. The workspace holds two such
 * pools, one per batch in flight. Scene, BVH, path state, queues and
 * framebuffer all live in it. */
int qpt_workspace_size(const qpt_ctx *ctx, uint32_t pool_paths, size_t *bytes);

/* Bind caller-owned device memory (256-byte aligned, `bytes` from
 * qpt_workspace_size) and upload the scene into it; the call returns after
 * the upload completed. Clears the framebuffer and statistics. */
int qpt_bind_workspace(qpt_ctx *ctx, void *device_ptr, size_t bytes, uint32_t pool_paths);

/* Ask enqueued rendering to stop (the paper's abort through host-mapped
 * memory, Appendix A.4): a word in pinned host memory that the first batch of
 * each pass reads on the GPU when it starts. Passes whose first batch starts
 * after the request render nothing (no sums, no counts); a pass already
 * started completes. Safe to call from another thread while the context's
 * other calls run (the only such call). Afterwards qpt_render_pass returns
 * QPT_E_ABORTED without enqueueing, and the next qpt_readback fills its
 * buffers, returns QPT_E_ABORTED and clears the request. With whole-pass
 * batches every pixel then has the same count c, and rendering passes
 * [first + c, end) completes the image exactly as an uninterrupted run
 * would. QPT_E_STATE before qpt_bind_workspace. */
int qpt_abort(qpt_ctx *ctx);

/* Enqueue iterations [first_pass, first_pass + num_passes), each one sample
 * per pixel over the whole frame (Sec. 3.2.2), and accumulate them into the
 * FP64 framebuffer and the per-pixel counts (Appendix A.4). Asynchronous:
 * returns after enqueueing. Iteration j of pixel p uses the Halton index
 * i0(p) + j * 2^k 3^l (Appendix A.2, full-screen enumeration). */
int qpt_render_pass(qpt_ctx *ctx, uint64_t first_pass, uint32_t num_passes,
                    const qpt_render_opts *opts);

/* Synchronise the stream and copy the FP64 sums (height*width*3, row-major,
 * pixel (x, y) at y*width + x) and the uint32 counts (height*width) into
 * caller buffers; either pointer may be NULL. dst_is_device: 1 if the
 * buffers are device memory, 0 for host memory. Image = sum / count. */
int qpt_readback(qpt_ctx *ctx, double *sum_rgb, uint32_t *counts, int dst_is_device);

/* Zero the framebuffer, the counts and the statistics (enqueued on the stream). */
int qpt_reset_accum(qpt_ctx *ctx);

/* Resume from a checkpoint: load FP64 sums (W H 3) and per-pixel counts (W H)
 * saved by qpt_readback (host memory, or device memory with src_is_device)
 * into the framebuffer; rendering passes [c, ...) after a checkpoint taken
 * with every count c continues the progressive image exactly as if it had
 * not stopped (the sample indices of a pass do not depend on history).
 * Synchronous. */
int qpt_load_accum(qpt_ctx *ctx, const double *sum_rgb, const uint32_t *counts, int src_is_device);

/* Synchronise and read the ray/path counters. */
int qpt_get_stats(qpt_ctx *ctx, qpt_stats *out);

/* ---- the learned proposal: a 32-64-64-64-40 network (BF16 on MFMA, FP32
 * accumulate) mapping an encoded hit position and outgoing direction to an
 * 8-lobe von Mises-Fisher mixture, sampled with probability alpha and mixed
 * with the BSDF under MIS (density alpha q + (1 - alpha) p_bsdf, so the
 * estimator stays unbiased), trained online with Adam on the renderer's own
 * radiance samples. Not part of the paper's method; an extension of its
 * importance sampling (Sec. 2.1, 2.2). ---- */
typedef struct {
    float alpha;             /* probability of sampling the guide once active, [0, 1); 0 disables */
    float lr;                /* Adam learning rate (> 0) */
    uint32_t batch;          /* training samples per step (0 = 2^18, at most 2^22) */
    uint32_t train;          /* Adam steps per pass, taken after each batch of passes, each on its own
                                stratified subset of the replay samples (0: no recording or training;
                                at most 64) */
    uint32_t warmup_steps;   /* guide sampling stays off until this many steps were taken */
    uint32_t seed;           /* offsets of the stratified batch subsets */
    uint32_t max_vertex;     /* guide (and record) at path vertices 1..max_vertex only; 0 = every vertex */
} qpt_guide_opts;

/* Set the guide options (takes effect at the next qpt_render_pass). */
int qpt_guide_config(qpt_ctx *ctx, const qpt_guide_opts *opts);

/* Load the FP32 master parameters from host memory (13032 values: per layer
 * W (in x out, row-major) then b, layers 32->64->64->64->40) and reset the
 * Adam state and step count. Needed before guiding or training. Synchronous. */
int qpt_guide_set_weights(qpt_ctx *ctx, const float *params);

/* Copy the FP32 master parameters to host memory and the number of training
 * steps taken; either pointer may be NULL. Synchronises the stream. */
int qpt_guide_get_weights(qpt_ctx *ctx, float *params, uint32_t *steps);

/* Checkpoint of the guide's optimiser: FP32 master parameters, Adam first and
 * second moments (13032 values each, host memory, any pointer may be NULL)
 * and the step count (which drives the bias correction). Synchronous. */
int qpt_guide_get_state(qpt_ctx *ctx, float *params, float *m, float *v, uint32_t *steps);

/* Restore such a checkpoint (all three arrays required, finite, v >= 0).
 * The replay ring of training samples starts empty; it refills from the
 * next rendered batch. Synchronous. */
int qpt_guide_set_state(qpt_ctx *ctx, const float *params, const float *m, const float *v, uint32_t steps);

/* Parity hooks (device pointers, enqueued on the stream):
 * forward of n rows of 32 FP32 features -> n x 40 FP32 outputs; */
int qpt_guide_debug_forward(qpt_ctx *ctx, const float *x, uint32_t n, float *out);
/* the renderer's inference path on n explicit vertices (x: n x 3 positions,
 * wo: n x 3 unit outgoing directions; encoded against the scene's bounding
 * box) -> n x 40 FP32, the mixture exactly as the renderer decodes it from
 * its FP16 per-vertex storage: lobe k's (mu xyz, kappa) at 4k..4k+3, then
 * the 8 weights at 32..39; */
int qpt_guide_debug_eval(qpt_ctx *ctx, const float *x, const float *wo, uint32_t n, float *mix);
/* gradient of -sum_b w_b log q(dir_b) / sum_b w_b w.r.t. the 13032 parameters
 * for n rows (x: n x 32 features, dirs: n x 3 unit vectors, w: n weights); */
int qpt_guide_debug_grad(qpt_ctx *ctx, const float *x, const float *dirs, const float *w, uint32_t n,
                         float *grad);
/* the same gradient followed by one Adam step (lr; beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected, step count + 1) on the FP32 master weights and
 * the BF16 copy the kernels use; grad may be NULL; */
int qpt_guide_debug_train(qpt_ctx *ctx, const float *x, const float *dirs, const float *w, uint32_t n, float lr,
                          float *grad);
/* decode n x 40 outputs, mixture pdf at dirs (n x 3) and a sample from
 * u (n x 3: lobe, two direction numbers) into sample (n x 3). */
int qpt_guide_debug_mixture(qpt_ctx *ctx, const float *out40, const float *dirs, const float *u, uint32_t n,
                            float *pdf, float *sample);

/* The training records of the most recent batch of passes (the guide's
 * record step: train > 0), with their identity, for parity checks. Per
 * record (DEVICE pointers, cap rows each): ident[3 r..] = pixel id
 * (y * width + x), pass, path vertex; rec[11 r..] = hit position x (3),
 * outgoing direction wo (3), sampled direction wi (3), the mixture density
 * of wi that the throughput used, and the record's weight: the luminance of
 * (final path radiance - radiance before the vertex's next-event estimate -
 * that estimate) / throughput before the scattering, per channel where that
 * throughput is positive, each channel clamped at 0 (the sample's estimate
 * f cos L_i / p of the scattering integral). Records whose weight is
 * positive and finite are the ones the replay ring receives. *count = the
 * number of records the batch holds (rows beyond cap are not written), in
 * the order the shading kernel appended them. A vertex leaves a record when
 * its path continues, the vertex is at most max_vertex deep, and (when the
 * batch could overflow the record buffer) a hash of its sample index and
 * depth falls below the kept fraction. Synchronises the stream.
 * QPT_E_STATE before any qpt_render_pass on the bound workspace. */
int qpt_guide_debug_records(qpt_ctx *ctx, uint32_t *ident, float *rec, uint32_t cap, uint32_t *count);

/* Weighted negative log-likelihood of the last training batch (sum_b w_b
 * (-log q(dir_b)) / sum_b w_b) and its weight sum (host pointers, either may
 * be NULL). Synchronises the stream. */
int qpt_guide_loss(qpt_ctx *ctx, double *loss, double *weight_sum);

/* Profiling: enable = 1 starts bracketing every kernel launch of
 * qpt_render_pass with HIP events on the context's stream (previous
 * records are dropped); enable = 0 stops. */
int qpt_profile(qpt_ctx *ctx, int enable);

/* Synchronise and sum the recorded launch durations per kernel kind into
 * out[QPT_K_KINDS] (caller-owned host array). */
int qpt_profile_read(qpt_ctx *ctx, qpt_kernel_time *out);

/* ---- parity hooks: inputs and outputs are DEVICE pointers, enqueued on the
 * stream; call qpt_readback or synchronise the stream before reading ---- */

/* out[q] = floor(2^32 * scrambled radical inverse of idx[q] in dimension dim[q])
 * with the film dimensions 0 and 1 taken as the digits left after the pixel's
 * own (Appendix A.2). dim[q] < 256. */
int qpt_debug_sample_bits(qpt_ctx *ctx, const uint64_t *idx, const uint32_t *dim, uint32_t n,
                          int scramble, uint32_t *out);

/* out[w] = in[64 w] + ... + in[64 w + 63] modulo 2^32 for w < n / 64, by
 * the wavefront reduction (DPP row moves, then the four row sums) that the
 * traversal kernels use to add their lanes' node and triangle counts. n must
 * be a multiple of 64 (QPT_E_INVALID otherwise). Needs a context on a
 * device; no workspace. */
int qpt_debug_wave_sum(qpt_ctx *ctx, const uint32_t *in, uint32_t n, uint32_t *out);

/* out[y*width + x] = Halton index of pixel (x, y) in iteration `pass`. */
int qpt_debug_pixel_index(qpt_ctx *ctx, uint64_t pass, uint64_t *out);

/* Trace n rays (n x 8 floats: ox oy oz tmax dx dy dz unused) through the
 * BVH (brute_force = 0) or against every triangle (brute_force = 1).
 * Closest hit: t[n], tri[n] (input triangle id, 0xffffffff on a miss),
 * b12[2n] barycentrics of vertices 1 and 2. any_hit = 1: tri[q] = 1 if
 * occluded, else 0 (t and b12 may be NULL). stack_max (may be NULL; BVH
 * mode only) receives each ray's deepest traversal stack: entries beyond
 * the 15 kept in LDS spill to the workspace's overflow area. */
int qpt_debug_trace(qpt_ctx *ctx, const float *rays, uint32_t n, int any_hit, int brute_force,
                    float *t, uint32_t *tri, float *b12, uint32_t *stack_max);

/* ---- host-table hooks (host memory, no device needed), for cross-checks of
 * the builders against an independent implementation ---- */

/* Emitters in ascending input-triangle order: input triangle id, alias
 * probability (FP64 Vose table), alias index, realised selection pmf of the
 * integer selection rule. *count receives the number of emitters; array
 * pointers may be NULL (query the count first). After qpt_build_scene. */
int qpt_debug_light_tables(const qpt_ctx *ctx, uint32_t *emit_tri, double *prob, uint32_t *alias,
                           double *pmf, uint32_t *count);

/* The light tree (Sec. 2.1.1 hierarchy), built with the scene: a binary tree
 * over the emitters, split at the centroid median of the longest centroid
 * extent (ties by emitter index), at most 8 emitters per leaf, children
 * stored as adjacent pairs in depth-first order. Per node: sphere4[4 k..]
 * centre xyz and radius of its bounding sphere; flux6[6 k..] its flux
 * towards each emission region (+x, -x, +y, -y, +z, -z dominant-axis cells),
 * each triangle's flux times the bound of its one-sided emission cosine over
 * the region; left[k] first child (-1 for a leaf); first[k], count[k] its
 * range in leaf order. Per leaf-order position q: emit[q] the emitter,
 * weight[q] the 24-bit cumulative flux fraction before it within its leaf.
 * *num_nodes receives the node count (0 without triangle lights); array
 * pointers may be NULL. Host memory. After qpt_build_scene. */
int qpt_debug_light_tree(const qpt_ctx *ctx, float *sphere4, float *flux6, int32_t *left, uint32_t *first,
                         uint32_t *count, uint32_t *emit, uint32_t *weight, uint32_t *num_nodes);

/* The environment pyramid built with the scene (2:1 power-of-two maps, see
 * qpt_render_opts.env_sampling): *levels = m (W = 2^(m+1), H = 2^m; 0 = none),
 * *top = levels weighted per normal bin (min(m, 5)), *root = 24-bit share of
 * the left half (phi < pi). q: 4 words per node of levels 0..m-1 (level k has
 * 2^(k+1) x 2^k nodes, row-major, after the 2 (4^k - 1) / 3 nodes above):
 * 24-bit share of the left child column, of the upper row within the left
 * column, within the right column, 0. Intensity x solid angle; a child
 * without weight gets share 0 (or 2^24 for the other). oq: per normal bin
 * b = 16 j + i (octahedral cell i along x, j along z), 4 (1 + nodes above
 * level top) words: (root share, 0, 0, 0) then the nodes of levels
 * 0..top-1 with cosine-weighted shares. Host memory; q and oq may be NULL.
 * After qpt_build_scene. */
int qpt_debug_env_pyramid(const qpt_ctx *ctx, uint32_t *levels, uint32_t *top, uint32_t *root, uint32_t *q,
                          uint32_t *oq);

/* The renderer's pyramid descent for n queries (DEVICE pointers): uv[2n]
 * (u narrows columns, v rows), nrm[3n] FP32 normals (their bin is used when
 * mode = 2; mode = 1 ignores them). Writes texel[n] = row W + col, iv[4n] =
 * (column interval size, offset in it, row interval size, offset) and
 * iv_hit[2n] = the two sizes the descent steered to that texel finds (what
 * an environment hit's MIS weight uses; equal to the sampled ones).
 * QPT_E_STATE before qpt_bind_workspace or without a pyramid. */
int qpt_debug_env_sample(qpt_ctx *ctx, const uint32_t *uv, const float *nrm, uint32_t n, uint32_t mode,
                         uint32_t *texel, uint64_t *iv, uint64_t *iv_hit);

/* The renderer's light-tree choice for n queries (DEVICE pointers): 63-bit
 * samples S[n] (bit 63 ignored), FP32 shading points x[3n] and unit normals
 * nrm[3n]; writes the chosen emitter, its interval size (selection
 * probability times 2^63) and the size that the descent steered to that
 * emitter finds (what an emitter hit's MIS weight uses; equal to size).
 * QPT_E_STATE before qpt_bind_workspace or without triangle lights. */
int qpt_debug_light_sample(qpt_ctx *ctx, const uint64_t *S, const float *x, const float *nrm, uint32_t n,
                           uint32_t *emitter, uint64_t *size, uint64_t *size_hit);

/* Environment tables: row CDF row_q[env_height] (2^32 scale, row_q[0] = 0),
 * column CDFs col_q[env_height * env_width], texel solid-angle pdfs
 * texel_pdf[env_height * env_width]. QPT_E_STATE without an environment. */
int qpt_debug_env_tables(const qpt_ctx *ctx, uint32_t *row_q, uint32_t *col_q, float *texel_pdf);

/* The GPU BVH (4-wide): nodes32[num_nodes * 32], each node 32 values: the
 * four children's boxes as lo.x[4], lo.y[4], lo.z[4], hi.x[4], hi.y[4],
 * hi.z[4], then four int32 child references (>= 0 inner node, INT32_MIN
 * unused slot, other < 0 leaf with ~ref = first << 3 | (count - 1)), then
 * the number of used slots and three unused words; and
 * tri_order[num_triangles] (input id of each leaf-order triangle). Pointers
 * may be NULL. After qpt_build_bvh. */
int qpt_debug_bvh_nodes(const qpt_ctx *ctx, float *nodes32, uint32_t *tri_order, uint32_t *num_nodes);

#ifdef __cplusplus
}
#endif

#endif /* QPT_H */
