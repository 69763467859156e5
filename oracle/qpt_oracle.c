/*
 * CPU oracle for the progressive QMC path tracer -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load or run this code. It shares no code with the GPU library: it reads
 * the same seeded scene arrays and nothing else.
 *
 * What it computes, in plain slow C:
 *   - exact scrambled radical inverses, floor(RI(i) * 2^32), with 128-bit
 *     integers (Appendix A.2: integer evaluation, indices up to 64 bit);
 *   - full-screen sample enumeration (Appendix A.2): the unique index in
 *     [0, 2^k 3^l) whose first base-2 / base-3 digits select a pixel, found
 *     by brute-force search;
 *   - FP32 watertight ray/triangle intersection by brute force over every
 *     triangle (Sec. 2.3: watertight intersection "everywhere"), so that hit
 *     ids can be compared bit-exactly with a kernel deciding in FP32;
 *   - an FP64 path tracer: camera rays with box-filtered film samples,
 *     closest hit, next-event estimation of triangle lights and a lat-long
 *     environment, multiple importance sampling, Lambert and GGX-over-Lambert
 *     BSDFs, Russian roulette, FP64 per-pixel sums and sample counts
 *     (Sec. 2, Sec. 2.1, Sec. 3.2.2, Appendix A.1, A.2, A.4).
 *
 * Every discrete decision that a floating-point value drives is taken either
 * in integers on the exact 32-bit sample value (light and texel selection),
 * or in FP32 precision on the FP32 rounding of this oracle's FP64 value
 * (Russian roulette, lobe choice), which is the precision the GPU kernels
 * decide in.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -ffp-contract=off -pthread -lm
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ primes */

#define OR_MAX_PRIMES 1024
static uint32_t g_primes[OR_MAX_PRIMES];
static int g_primes_ready = 0;

static void init_primes(void)
{
    if (g_primes_ready) return;
    int n = 0;
    for (uint32_t c = 2; n < OR_MAX_PRIMES; ++c) {
        int is_p = 1;
        for (uint32_t d = 2; d * d <= c; ++d)
            if (c % d == 0) { is_p = 0; break; }
        if (is_p) g_primes[n++] = c;
    }
    g_primes_ready = 1;
}

/* base of sample dimension d: the (d+1)-th prime */
uint32_t or_dim_base(uint32_t d)
{
    init_primes();
    return d < OR_MAX_PRIMES ? g_primes[d] : 0;
}

/* Linear digit scrambling pi_b(a) = f_b * a mod b (a Faure-Lemieux style
 * permutation). f_b is round(b * 0.618034) taken in [1, b-1]. pi_b(0) = 0,
 * so the infinite tail of zero digits stays zero. */
uint32_t or_scramble_mult(uint32_t b)
{
    uint64_t f = ((uint64_t)b * 618034u + 500000u) / 1000000u;
    if (f < 1) f = 1;
    if (f > b - 1) f = b - 1;
    return (uint32_t)f;
}

/* floor(2^32 * sum_m pi(d_m) b^-(m+1)) for the base-b digits d_m of i */
uint32_t or_ri_bits(uint64_t i, uint32_t b, uint32_t f)
{
    u128 num = 0, den = 1;
    while (i) {
        uint64_t d = i % b;
        i /= b;
        num = num * b + (u128)((f * d) % b);
        den *= b;
    }
    return (uint32_t)((num << 32) / den);
}

/* ------------------------------------------------------- enumeration */

void or_enum_params(uint32_t W, uint32_t H, uint32_t *k, uint32_t *l, uint64_t *S)
{
    uint32_t kk = 0, ll = 0;
    uint64_t p2 = 1, p3 = 1;
    while (p2 < W) { p2 *= 2; ++kk; }
    while (p3 < H) { p3 *= 3; ++ll; }
    *k = kk; *l = ll; *S = p2 * p3;
}

static uint64_t digit_reverse(uint64_t v, uint32_t base, uint32_t ndig)
{
    uint64_t r = 0;
    for (uint32_t m = 0; m < ndig; ++m) { r = r * base + v % base; v /= base; }
    return r;
}

/* index of pass j for pixel (px, py): i0 + j*S, i0 found by search */
uint64_t or_pixel_index(uint32_t W, uint32_t H, uint32_t px, uint32_t py, uint64_t j)
{
    uint32_t k, l;
    uint64_t S;
    or_enum_params(W, H, &k, &l, &S);
    uint64_t p2 = 1ull << k, p3 = S >> k;
    uint64_t a = digit_reverse(px, 2, k);   /* i mod 2^k */
    uint64_t c = digit_reverse(py, 3, l);   /* i mod 3^l */
    for (uint64_t t = 0; t < p3; ++t) {
        uint64_t i = a + p2 * t;
        if (i % p3 == c) return i + j * S;
    }
    return ~0ull; /* unreachable: 2^k and 3^l are coprime */
}

/* 32-bit sample value of dimension d for index i. Dimensions 0 and 1 are the
 * film offsets inside the pixel: the digits of i left after the pixel's own
 * base-2 (resp. base-3) digits, unscrambled. */
uint32_t or_sample_bits(uint64_t i, uint32_t d, uint32_t W, uint32_t H, int scramble)
{
    uint32_t k, l;
    uint64_t S;
    or_enum_params(W, H, &k, &l, &S);
    if (d == 0) return or_ri_bits(i >> k, 2, 1);
    if (d == 1) return or_ri_bits(i / (S >> k), 3, 1);
    uint32_t b = or_dim_base(d);
    return or_ri_bits(i, b, scramble ? or_scramble_mult(b) : 1);
}

void or_sample_bits_batch(const uint64_t *idx, const uint32_t *dim, uint32_t n, uint32_t W,
                          uint32_t H, int scramble, uint32_t *out)
{
    for (uint32_t q = 0; q < n; ++q) out[q] = or_sample_bits(idx[q], dim[q], W, H, scramble);
}

static double u24(uint32_t bits) { return (double)(bits >> 8) * (1.0 / 16777216.0); }

/* ------------------------------------------- FP32 watertight, brute force */

/* Watertight ray/triangle test in FP32 (Woop, Benthin, Wald 2013): shear the
 * triangle into ray space, edge functions with an exact-zero fallback in
 * FP64, t = T / det. Hit iff 0 < t < tmax. */
static int tri_hit_f32(const float o[3], const float d[3], float tmax, const float *v0,
                       const float *v1, const float *v2, float *t_out, float *b1_out,
                       float *b2_out)
{
    int kz = 0;
    if (fabsf(d[1]) > fabsf(d[kz])) kz = 1;
    if (fabsf(d[2]) > fabsf(d[kz])) kz = 2;
    int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
    if (d[kz] < 0.0f) { int s = kx; kx = ky; ky = s; }
    float Sx = d[kx] / d[kz], Sy = d[ky] / d[kz], Sz = 1.0f / d[kz];

    float A[3], B[3], C[3];
    for (int c = 0; c < 3; ++c) { A[c] = v0[c] - o[c]; B[c] = v1[c] - o[c]; C[c] = v2[c] - o[c]; }
    float Ax = fmaf(-Sx, A[kz], A[kx]), Ay = fmaf(-Sy, A[kz], A[ky]);
    float Bx = fmaf(-Sx, B[kz], B[kx]), By = fmaf(-Sy, B[kz], B[ky]);
    float Cx = fmaf(-Sx, C[kz], C[kx]), Cy = fmaf(-Sy, C[kz], C[ky]);
    /* separately rounded products keep each edge function antisymmetric in its
     * two vertices, so a shared edge evaluates to exactly opposite values in
     * the two triangles that own it (no fused multiply-add here) */
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return 0;
    float det = (U + V) + W;
    if (det == 0.0f) return 0;
    float Az = Sz * A[kz], Bz = Sz * B[kz], Cz = Sz * C[kz];
    float T = fmaf(U, Az, fmaf(V, Bz, W * Cz));
    float t = T / det;
    if (!(t > 0.0f && t < tmax)) return 0;
    *t_out = t;
    *b1_out = V / det;
    *b2_out = W / det;
    return 1;
}

/* rays: n x 8 floats (ox, oy, oz, tmax, dx, dy, dz, unused).
 * Closest hit: smallest t, equal t -> smaller triangle id; miss -> id ~0u.
 * any_hit: out_tri = 0 (visible) or 1 (occluded). */
void or_trace_f32(const float *pos, const uint32_t *idx, uint32_t nt, const float *rays,
                  uint32_t n, int any_hit, float *out_t, uint32_t *out_tri, float *out_b)
{
    for (uint32_t r = 0; r < n; ++r) {
        const float *ry = rays + 8 * (size_t)r;
        float o[3] = {ry[0], ry[1], ry[2]}, d[3] = {ry[4], ry[5], ry[6]};
        float tmax = ry[3];
        float bt = INFINITY, bb1 = 0, bb2 = 0;
        uint32_t bid = 0xffffffffu;
        for (uint32_t q = 0; q < nt; ++q) {
            float t, b1, b2;
            if (!tri_hit_f32(o, d, tmax, pos + 3 * idx[3 * q], pos + 3 * idx[3 * q + 1],
                             pos + 3 * idx[3 * q + 2], &t, &b1, &b2))
                continue;
            if (any_hit) { bid = 1; break; }
            if (t < bt || (t == bt && q < bid)) { bt = t; bid = q; bb1 = b1; bb2 = b2; }
        }
        if (any_hit) {
            out_tri[r] = bid == 1 ? 1u : 0u;
            if (out_t) out_t[r] = 0.0f;
            continue;
        }
        out_tri[r] = bid;
        if (out_t) out_t[r] = bid == 0xffffffffu ? INFINITY : bt;
        if (out_b) { out_b[2 * r] = bb1; out_b[2 * r + 1] = bb2; }
    }
}

/* ------------------------------------------------------------ FP64 math */

typedef struct { double x, y, z; } v3;
static inline v3 V3(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static inline v3 add(v3 a, v3 b) { return V3(a.x + b.x, a.y + b.y, a.z + b.z); }
static inline v3 sub(v3 a, v3 b) { return V3(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline v3 mul(v3 a, double s) { return V3(a.x * s, a.y * s, a.z * s); }
static inline v3 vmul(v3 a, v3 b) { return V3(a.x * b.x, a.y * b.y, a.z * b.z); }
static inline double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline v3 cross(v3 a, v3 b)
{
    return V3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static inline double len(v3 a) { return sqrt(dot(a, a)); }
static inline v3 normalize(v3 a) { return mul(a, 1.0 / len(a)); }
static inline double comp(v3 a, int c) { return c == 0 ? a.x : (c == 1 ? a.y : a.z); }
static inline double maxc(v3 a) { return fmax(a.x, fmax(a.y, a.z)); }
static inline double lum(v3 c) { return 0.2126 * c.x + 0.7152 * c.y + 0.0722 * c.z; }

/* ------------------------------------------------------------ the scene */

typedef struct {
    v3 lo, hi;
    int32_t left, right; /* inner: child nodes; leaf: left = -1 - first, right = count */
} bnode;

typedef struct {
    uint32_t nt;
    v3 *p0, *p1, *p2;       /* triangle corners, FP32 inputs widened exactly */
    uint32_t *mat;
    uint32_t nm;
    v3 *albedo, *emission;
    double *rough;
    uint32_t *flags;
    /* emitters: triangles with a non-zero emission colour */
    uint32_t ne;
    uint32_t *emit_tri;
    double *emit_flux, *alias_prob;
    uint32_t *alias_idx;
    uint64_t *alias_thr;    /* take column c iff sample bits < thr[c] (2^32 scale) */
    double *emit_pmf;       /* realised selection probability of each emitter */
    int32_t *tri_emit;      /* triangle -> emitter index or -1 */
    /* light tree (Sec. 2.1.1): nodes, leaf order of the emitters, cumulative
     * 24-bit flux weights within each leaf */
    uint32_t lt_nn;
    float *lt_c;            /* 4 per node: centre xyz, radius */
    float *lt_f;            /* 6 per node: flux per emission region */
    int32_t *lt_left;       /* inner: first of the two children; leaf: -1 */
    uint32_t *lt_first, *lt_count;
    uint32_t *lt_emit;      /* leaf-order position -> emitter */
    uint32_t *lt_pos;       /* emitter -> leaf-order position */
    uint32_t *lt_w;         /* leaf-order position -> cumulative weight before it in its leaf */
    /* environment */
    uint32_t ew, eh;
    v3 *env;
    uint64_t *row_q;        /* eh + 1 integer CDF (2^32 scale) */
    uint64_t *col_q;        /* eh * (ew + 1) */
    double *env_texel_pdf;  /* solid-angle pdf of each texel under the integer CDFs */
    double p_env;
    /* environment pyramid (Sec. 2.1.2): finest level m (W = 2^(m+1), H = 2^m;
     * 0 = no pyramid), split probabilities of every node above the texels,
     * and per normal bin those of the top levels */
    uint32_t ep_m, ep_top;
    uint32_t ep_root;       /* 24-bit probability of the left root (x < W/2) */
    uint32_t *ep_q;         /* 4 per node of levels 0..m-1: column, row | left column, row | right column, 0 */
    uint32_t *ep_oq;        /* per normal bin: root, 0, 0, 0, then 4 per node of levels 0..top-1 */
    /* camera */
    v3 eye, fwd, right, up;
    double tan_half, aspect;
    uint32_t W, H;
    /* BVH over triangle ids */
    bnode *nodes;
    uint32_t nnodes;
    uint32_t *order;
    /* bounding box of every input position (the guide's position encoding) */
    double bmin[3], bext[3];
    /* the learned proposal, frozen (or_guide_set): BF16-rounded parameters,
     * the integer threshold of the guide choice, guided vertices 1..g_maxv,
     * and the record subset threshold of the training-record hash */
    double *g_par;
    uint32_t g_alpha_thr, g_maxv, g_rec_thr;
} or_scene;

#define MAT_GGX 1u
#define MAT_EMIT_TEXTURE 2u

/* emission at a point of a triangle with material m (front face only) */
static v3 emission_at(const or_scene *s, uint32_t m, v3 x)
{
    v3 E = s->emission[m];
    if (s->flags[m] & MAT_EMIT_TEXTURE) {
        double k = 0.55 + 0.45 * sin(2.0 * M_PI * 4.0 * (x.x + x.z));
        E = mul(E, k);
    }
    return E;
}

/* flux of one emitting triangle: pi * area * lum(mean emission), the mean by
 * the 16-point midpoint rule over the 4x4 split of the triangle */
static double tri_flux(const or_scene *s, uint32_t t)
{
    v3 a = s->p0[t], b = s->p1[t], c = s->p2[t];
    double area = 0.5 * len(cross(sub(b, a), sub(c, a)));
    const int n = 4;
    double acc = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; i + j < n; ++j) {
            /* upright cell centroid */
            double u = (i + 1.0 / 3.0) / n, v = (j + 1.0 / 3.0) / n;
            acc += lum(emission_at(s, s->mat[t], add(a, add(mul(sub(b, a), u), mul(sub(c, a), v)))));
            if (i + j < n - 1) { /* inverted cell centroid */
                u = (i + 2.0 / 3.0) / n; v = (j + 2.0 / 3.0) / n;
                acc += lum(emission_at(s, s->mat[t], add(a, add(mul(sub(b, a), u), mul(sub(c, a), v)))));
            }
        }
    return M_PI * area * acc / (double)(n * n);
}

/* Vose's alias method, deterministic: q_i = P_i N / sum P; two index-ordered
 * FIFO lists; the large entry stays at the head until it drops below one. */
void or_alias_build(uint32_t n, const double *w, double *prob, uint32_t *alias)
{
    double sum = 0.0;
    for (uint32_t i = 0; i < n; ++i) sum += w[i];
    double *q = (double *)malloc(sizeof(double) * n);
    uint32_t *small = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *large = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t sh = 0, st = 0, lh = 0, lt = 0;
    for (uint32_t i = 0; i < n; ++i) {
        q[i] = (w[i] * (double)n) / sum;
        if (q[i] < 1.0) small[st++] = i; else large[lt++] = i;
    }
    while (sh < st && lh < lt) {
        uint32_t sm = small[sh++], lg = large[lh];
        prob[sm] = q[sm];
        alias[sm] = lg;
        q[lg] = (q[lg] + q[sm]) - 1.0;
        if (q[lg] < 1.0) { lh++; small[st++] = lg; }
    }
    while (sh < st) { uint32_t i = small[sh++]; prob[i] = 1.0; alias[i] = i; }
    while (lh < lt) { uint32_t i = large[lh++]; prob[i] = 1.0; alias[i] = i; }
    free(q); free(small); free(large);
}

/* number of r in [0, R) with floor(r * N / R) == c, R a power of two */
static uint64_t col_count(uint64_t c, uint64_t N, uint64_t R)
{
    /* smallest r with r*N >= c*R is ceil(c*R/N) */
    u128 hi = ((u128)(c + 1) * R + N - 1) / N, lo = ((u128)c * R + N - 1) / N;
    return (uint64_t)(hi - lo);
}

static void build_lights(or_scene *s)
{
    s->ne = 0;
    s->tri_emit = (int32_t *)malloc(sizeof(int32_t) * s->nt);
    for (uint32_t t = 0; t < s->nt; ++t) {
        v3 e = s->emission[s->mat[t]];
        s->tri_emit[t] = -1;
        if (e.x > 0 || e.y > 0 || e.z > 0) s->ne++;
    }
    if (!s->ne) return;
    s->emit_tri = (uint32_t *)malloc(sizeof(uint32_t) * s->ne);
    s->emit_flux = (double *)malloc(sizeof(double) * s->ne);
    s->alias_prob = (double *)malloc(sizeof(double) * s->ne);
    s->alias_idx = (uint32_t *)malloc(sizeof(uint32_t) * s->ne);
    s->alias_thr = (uint64_t *)malloc(sizeof(uint64_t) * s->ne);
    s->emit_pmf = (double *)calloc(s->ne, sizeof(double));
    uint32_t k = 0;
    for (uint32_t t = 0; t < s->nt; ++t) {
        v3 e = s->emission[s->mat[t]];
        if (e.x > 0 || e.y > 0 || e.z > 0) { s->tri_emit[t] = (int32_t)k; s->emit_tri[k++] = t; }
    }
    for (uint32_t e = 0; e < s->ne; ++e) s->emit_flux[e] = tri_flux(s, s->emit_tri[e]);
    or_alias_build(s->ne, s->emit_flux, s->alias_prob, s->alias_idx);
    for (uint32_t e = 0; e < s->ne; ++e) {
        double thr = ceil(s->alias_prob[e] * 4294967296.0);
        s->alias_thr[e] = (uint64_t)thr;
    }
}

/* after p_env is known: realised pmf of the integer selection rule */
static void build_light_pmf(or_scene *s)
{
    if (!s->ne) return;
    uint64_t R = s->env ? (1ull << 31) : (1ull << 32);
    double p_tri = 1.0 - s->p_env;
    for (uint32_t c = 0; c < s->ne; ++c) {
        double pc = (double)col_count(c, s->ne, R) / (double)R;
        double take = (double)s->alias_thr[c] / 4294967296.0;
        s->emit_pmf[c] += p_tri * pc * take;
        s->emit_pmf[s->alias_idx[c]] += p_tri * pc * (1.0 - take);
    }
}

/* ---------------------------------------------------------- light tree
 *
 * The paper's hierarchy for many triangle lights (Sec. 2.1.1), made definite:
 * a binary tree over the emitters, split at the median of the longest axis
 * of the centroids (ties by emitter index), leaves of at most 8 emitters.
 * Each node keeps the bounding sphere of its triangles (centre and radius of
 * the box) and, for each of six emission regions of the unit sphere (the
 * dominant-axis cells +x, -x, +y, -y, +z, -z), the sum over its triangles of
 * flux times an upper bound of the one-sided emission cosine within the
 * region (the region lies in the cone of half-angle acos(1/sqrt 3) around its
 * axis). Built in FP64, stored in FP32. */
#define LT_LEAF 8

static double lt_region_bound(v3 n, int region)
{
    int k = region / 2;
    double sgn = (region & 1) ? -1.0 : 1.0;
    double ca = fmax(-1.0, fmin(1.0, sgn * comp(n, k)));
    double a = acos(ca), tc = acos(1.0 / sqrt(3.0));
    return a <= tc ? 1.0 : fmax(0.0, cos(a - tc));
}

typedef struct {
    or_scene *s;
    uint32_t *items;  /* emitters, reordered into leaf order */
    v3 *cen, *nrm;
    uint32_t next;    /* nodes allocated */
} lt_build;

static int lt_axis_k;
static const v3 *lt_cen_k;
static int lt_cmp(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    double kx = comp(lt_cen_k[x], lt_axis_k), ky = comp(lt_cen_k[y], lt_axis_k);
    if (kx != ky) return kx < ky ? -1 : 1;
    return x < y ? -1 : (x > y);
}

static void lt_node(lt_build *b, uint32_t node, uint32_t first, uint32_t count)
{
    or_scene *s = b->s;
    v3 lo = V3(INFINITY, INFINITY, INFINITY), hi = V3(-INFINITY, -INFINITY, -INFINITY);
    v3 clo = lo, chi = hi;
    double fl[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t q = first; q < first + count; ++q) {
        uint32_t e = b->items[q], t = s->emit_tri[e];
        v3 ps[3] = {s->p0[t], s->p1[t], s->p2[t]};
        for (int j = 0; j < 3; ++j) {
            lo = V3(fmin(lo.x, ps[j].x), fmin(lo.y, ps[j].y), fmin(lo.z, ps[j].z));
            hi = V3(fmax(hi.x, ps[j].x), fmax(hi.y, ps[j].y), fmax(hi.z, ps[j].z));
        }
        v3 c = b->cen[e];
        clo = V3(fmin(clo.x, c.x), fmin(clo.y, c.y), fmin(clo.z, c.z));
        chi = V3(fmax(chi.x, c.x), fmax(chi.y, c.y), fmax(chi.z, c.z));
        for (int r = 0; r < 6; ++r) fl[r] += s->emit_flux[e] * lt_region_bound(b->nrm[e], r);
    }
    v3 ctr = mul(add(lo, hi), 0.5);
    double rad = 0.5 * len(sub(hi, lo));
    s->lt_c[4 * node + 0] = (float)ctr.x;
    s->lt_c[4 * node + 1] = (float)ctr.y;
    s->lt_c[4 * node + 2] = (float)ctr.z;
    s->lt_c[4 * node + 3] = (float)rad;
    for (int r = 0; r < 6; ++r) s->lt_f[6 * node + r] = (float)fl[r];
    s->lt_first[node] = first;
    s->lt_count[node] = count;
    if (count <= LT_LEAF) {
        s->lt_left[node] = -1;
        double tot = 0.0;
        for (uint32_t q = first; q < first + count; ++q) tot += s->emit_flux[b->items[q]];
        double acc = 0.0;
        for (uint32_t q = first; q < first + count; ++q) {
            double frac = tot > 0.0 ? acc / tot : (double)(q - first) / (double)count;
            s->lt_w[q] = (uint32_t)nearbyint(frac * 16777216.0);
            acc += s->emit_flux[b->items[q]];
        }
        return;
    }
    v3 ext = sub(chi, clo);
    int axis = (ext.y > ext.x) ? 1 : 0;
    if (ext.z > comp(ext, axis)) axis = 2;
    lt_axis_k = axis;
    lt_cen_k = b->cen;
    qsort(b->items + first, count, sizeof(uint32_t), lt_cmp);
    uint32_t half = count / 2;
    uint32_t left = b->next;
    b->next += 2;
    s->lt_left[node] = (int32_t)left;
    lt_node(b, left, first, half);
    lt_node(b, left + 1, first + half, count - half);
}

static void build_light_tree(or_scene *s)
{
    if (!s->ne) return;
    uint32_t cap = 2 * s->ne;
    s->lt_c = (float *)malloc(sizeof(float) * 4 * cap);
    s->lt_f = (float *)malloc(sizeof(float) * 6 * cap);
    s->lt_left = (int32_t *)malloc(sizeof(int32_t) * cap);
    s->lt_first = (uint32_t *)malloc(sizeof(uint32_t) * cap);
    s->lt_count = (uint32_t *)malloc(sizeof(uint32_t) * cap);
    s->lt_emit = (uint32_t *)malloc(sizeof(uint32_t) * s->ne);
    s->lt_pos = (uint32_t *)malloc(sizeof(uint32_t) * s->ne);
    s->lt_w = (uint32_t *)malloc(sizeof(uint32_t) * s->ne);
    lt_build b = {s, s->lt_emit, (v3 *)malloc(sizeof(v3) * s->ne), (v3 *)malloc(sizeof(v3) * s->ne), 1};
    for (uint32_t e = 0; e < s->ne; ++e) {
        uint32_t t = s->emit_tri[e];
        b.items[e] = e;
        b.cen[e] = mul(add(add(s->p0[t], s->p1[t]), s->p2[t]), 1.0 / 3.0);
        v3 n = cross(sub(s->p1[t], s->p0[t]), sub(s->p2[t], s->p0[t]));
        double l = len(n);
        b.nrm[e] = l > 0.0 ? mul(n, 1.0 / l) : V3(0, 0, 1);
    }
    lt_node(&b, 0, 0, s->ne);
    s->lt_nn = b.next;
    for (uint32_t q = 0; q < s->ne; ++q) s->lt_pos[s->lt_emit[q]] = q;
    free(b.cen);
    free(b.nrm);
}

/* Estimated contribution of a node at shading point x with normal n (both
 * FP32, in FP32): emission-region flux towards x times a conservative bound
 * of the cosine at x over the node's bounding sphere, over max(d^2, r^2). */
static float lt_estimate(const or_scene *s, uint32_t node, const float *x, const float *n)
{
    const float *c = s->lt_c + 4 * node;
    float dx = c[0] - x[0], dy = c[1] - x[1], dz = c[2] - x[2];
    float d2 = (dx * dx + dy * dy) + dz * dz;
    float r = c[3], r2 = r * r;
    /* emission direction x - c: dominant axis, ties to the lower axis */
    float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    int k = 0;
    float m = ax, ek = -dx;
    if (ay > m) { k = 1; m = ay; ek = -dy; }
    if (az > m) { k = 2; m = az; ek = -dz; }
    float F = s->lt_f[6 * node + 2 * k + (ek < 0.0f ? 1 : 0)];
    float cosx = 1.0f;
    if (d2 > r2) {
        float d = sqrtf(d2);
        float sinb = r / d;
        float cosb = sqrtf(1.0f - sinb * sinb);
        float cosa = ((n[0] * dx + n[1] * dy) + n[2] * dz) / d;
        if (cosa < cosb) {
            float sina = sqrtf(fmaxf(0.0f, 1.0f - cosa * cosa));
            cosx = fmaxf(0.0f, cosa * cosb + sina * sinb);
        }
    }
    return F * cosx / fmaxf(d2, r2);
}

/* 24-bit probability of the left child, clamped to [1/16, 15/16] */
static uint32_t lt_left_q(const or_scene *s, uint32_t node, const float *x, const float *n)
{
    int32_t l = s->lt_left[node];
    float el = lt_estimate(s, (uint32_t)l, x, n), er = lt_estimate(s, (uint32_t)l + 1, x, n);
    float sum = el + er;
    float p = (sum > 0.0f && isfinite(sum)) ? el / sum : 0.5f;
    p = fminf(fmaxf(p, 0.0625f), 0.9375f);
    return (uint32_t)(p * 16777216.0f + 0.5f);
}

/* floor(R q / 2^24) exactly, R < 2^63, q <= 2^24 */
static uint64_t lt_split(uint64_t R, uint32_t q)
{
    return (R >> 24) * q + (((R & 0xFFFFFFull) * q) >> 24);
}

/* Descend with the 63-bit sample S; returns the emitter and the size of its
 * interval of [0, 2^63) (its realised selection probability times 2^63). */
static uint32_t lt_sample(const or_scene *s, uint64_t S, const float *x, const float *n, uint64_t *size)
{
    uint64_t R = 1ull << 63;
    uint32_t node = 0;
    while (s->lt_left[node] >= 0) {
        uint64_t T = lt_split(R, lt_left_q(s, node, x, n));
        if (T < 1) T = 1;
        if (T > R - 1) T = R - 1;
        if (S < T) { R = T; node = (uint32_t)s->lt_left[node]; }
        else { S -= T; R -= T; node = (uint32_t)s->lt_left[node] + 1; }
    }
    uint32_t f = s->lt_first[node], c = s->lt_count[node];
    uint32_t j = c - 1;
    for (uint32_t q = 1; q < c; ++q)
        if (S < lt_split(R, s->lt_w[f + q])) { j = q - 1; break; }
    uint64_t a = lt_split(R, s->lt_w[f + j]);
    uint64_t z = j + 1 < c ? lt_split(R, s->lt_w[f + j + 1]) : R;
    *size = z - a;
    return s->lt_emit[f + j];
}

/* the same interval size for a given emitter, by the deterministic descent
 * towards its leaf (for the MIS weight of an emitter hit) */
static uint64_t lt_size_of(const or_scene *s, uint32_t e, const float *x, const float *n)
{
    uint32_t pos = s->lt_pos[e];
    uint64_t R = 1ull << 63;
    uint32_t node = 0;
    while (s->lt_left[node] >= 0) {
        uint32_t l = (uint32_t)s->lt_left[node];
        uint64_t T = lt_split(R, lt_left_q(s, node, x, n));
        if (T < 1) T = 1;
        if (T > R - 1) T = R - 1;
        if (pos < s->lt_first[l + 1]) { R = T; node = l; }
        else { R -= T; node = l + 1; }
    }
    uint32_t f = s->lt_first[node], c = s->lt_count[node], j = pos - f;
    uint64_t a = lt_split(R, s->lt_w[f + j]);
    uint64_t z = j + 1 < c ? lt_split(R, s->lt_w[f + j + 1]) : R;
    return z - a;
}

static void build_env(or_scene *s)
{
    uint32_t W = s->ew, H = s->eh;
    s->row_q = (uint64_t *)malloc(sizeof(uint64_t) * (H + 1));
    s->col_q = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)H * (W + 1));
    s->env_texel_pdf = (double *)malloc(sizeof(double) * (size_t)W * H);
    double *rowsum = (double *)malloc(sizeof(double) * H);
    double *cdf = (double *)malloc(sizeof(double) * (W + 1));
    for (uint32_t r = 0; r < H; ++r) {
        double om = (2.0 * M_PI / W) * (cos(M_PI * r / H) - cos(M_PI * (r + 1) / H));
        cdf[0] = 0.0;
        for (uint32_t c = 0; c < W; ++c) cdf[c + 1] = cdf[c] + lum(s->env[(size_t)r * W + c]) * om;
        rowsum[r] = cdf[W];
        uint64_t *q = s->col_q + (size_t)r * (W + 1);
        for (uint32_t c = 0; c < W; ++c)
            q[c] = cdf[W] > 0.0 ? (uint64_t)floor(cdf[c] / cdf[W] * 4294967296.0)
                                : (uint64_t)(((u128)c << 32) / W);
        q[W] = 1ull << 32;
    }
    double tot = 0.0;
    cdf = (double *)realloc(cdf, sizeof(double) * (H + 1));
    cdf[0] = 0.0;
    for (uint32_t r = 0; r < H; ++r) cdf[r + 1] = cdf[r] + rowsum[r];
    tot = cdf[H];
    for (uint32_t r = 0; r < H; ++r) s->row_q[r] = (uint64_t)floor(cdf[r] / tot * 4294967296.0);
    s->row_q[H] = 1ull << 32;
    for (uint32_t r = 0; r < H; ++r) {
        double om = (2.0 * M_PI / W) * (cos(M_PI * r / H) - cos(M_PI * (r + 1) / H));
        double pr = (double)(s->row_q[r + 1] - s->row_q[r]) / 4294967296.0;
        const uint64_t *q = s->col_q + (size_t)r * (W + 1);
        for (uint32_t c = 0; c < W; ++c) {
            double pc = (double)(q[c + 1] - q[c]) / 4294967296.0;
            s->env_texel_pdf[(size_t)r * W + c] = pr * pc / om;
        }
    }
    free(rowsum);
    free(cdf);
}

/* ------------------------------------------------ environment pyramid
 *
 * Sec. 2.1.2 samples the environment by descending an image pyramid: its
 * finest level is the lat-long map with each texel's intensity times its
 * solid angle, each coarser level sums 2 x 2 nodes, and each step picks one
 * child by its share. Made definite here: a map of W = 2^(m+1) by H = 2^m
 * texels has levels k = 0..m of 2^(k+1) x 2^k nodes (level 0: the two
 * halves of the sphere split at phi = pi). A step first picks the column of
 * the child (left pair against right pair), then the row within it; both as
 * 24-bit probabilities. Two 32-bit samples u (columns) and v (rows) are
 * narrowed as integer intervals, so a texel's probability is exactly the
 * product of its final interval sizes over 2^64, and the remainders place the
 * direction inside the texel uniformly in solid angle.
 *
 * The paper's normal-aware variant weights the first few levels per
 * discretised surface normal, conservatively. Here: 16 x 16 bins of an
 * octahedral map of the normal (+y up), and at levels up to EP_TOP every node
 * below them of level EP_TOP is weighted by a bound of the cosine between any
 * normal of the bin and any direction of the node (the angle between the two
 * bounding cones' axes less both half-angles); deeper levels are shared. */
#define EP_K 16
#define EP_TOP 5

static uint32_t ep_nodes_above(uint32_t k) { return (uint32_t)((2ull * ((1ull << (2 * k)) - 1)) / 3); }

static uint32_t ep_quant(double l, double r)
{
    if (!(l + r > 0.0)) return 1u << 23;
    double q = nearbyint(l / (l + r) * 16777216.0);
    if (l > 0.0 && q < 1.0) q = 1.0;
    if (r > 0.0 && q > 16777215.0) q = 16777215.0;
    return (uint32_t)q;
}

static v3 ep_dir(double th, double ph) { return V3(sin(th) * sin(ph), cos(th), -sin(th) * cos(ph)); }

static double ep_angle(v3 a, v3 b) { return acos(fmax(-1.0, fmin(1.0, dot(a, b)))); }

/* octahedral square (px, pz) in [-1, 1]^2 -> unit normal, +y up */
static v3 ep_oct_decode(double px, double pz)
{
    double y = 1.0 - fabs(px) - fabs(pz);
    if (y < 0.0) {
        double fx = (1.0 - fabs(pz)) * (px >= 0.0 ? 1.0 : -1.0);
        double fz = (1.0 - fabs(px)) * (pz >= 0.0 ? 1.0 : -1.0);
        px = fx;
        pz = fz;
    }
    return normalize(V3(px, y, pz));
}

/* normal bin of an FP32 normal, in FP32 */
static uint32_t ep_bin(const float *n)
{
    float a = (fabsf(n[0]) + fabsf(n[1])) + fabsf(n[2]);
    float px = n[0] / a, pz = n[2] / a;
    if (n[1] < 0.0f) {
        float fx = (1.0f - fabsf(pz)) * (px >= 0.0f ? 1.0f : -1.0f);
        float fz = (1.0f - fabsf(px)) * (pz >= 0.0f ? 1.0f : -1.0f);
        px = fx;
        pz = fz;
    }
    int i = (int)floorf((px + 1.0f) * (0.5f * EP_K)), j = (int)floorf((pz + 1.0f) * (0.5f * EP_K));
    i = i < 0 ? 0 : (i > EP_K - 1 ? EP_K - 1 : i);
    j = j < 0 ? 0 : (j > EP_K - 1 ? EP_K - 1 : j);
    return (uint32_t)(j * EP_K + i);
}

/* split probabilities of levels 0..levels-1 from level-`levels` weights wl
 * (row-major, 2^(levels+1) x 2^levels); out: root q, then 4 per node */
static void ep_splits(const double *wl, uint32_t levels, uint32_t *root, uint32_t *q)
{
    const double *cur = wl;
    double *own = NULL;
    for (int k = (int)levels - 1; k >= 0; --k) {
        uint32_t cw = 2u << k, ch = 1u << k, fw = 2 * cw;
        double *up = (double *)malloc(sizeof(double) * cw * ch);
        for (uint32_t y = 0; y < ch; ++y)
            for (uint32_t x = 0; x < cw; ++x) {
                double a = cur[(size_t)(2 * y) * fw + 2 * x], b = cur[(size_t)(2 * y) * fw + 2 * x + 1];
                double c = cur[(size_t)(2 * y + 1) * fw + 2 * x], d = cur[(size_t)(2 * y + 1) * fw + 2 * x + 1];
                uint32_t *o = q + 4 * ((size_t)ep_nodes_above((uint32_t)k) + (size_t)y * cw + x);
                o[0] = ep_quant(a + c, b + d);
                o[1] = ep_quant(a, c);
                o[2] = ep_quant(b, d);
                o[3] = 0;
                up[(size_t)y * cw + x] = ((a + b) + c) + d;
            }
        free(own);
        own = up;
        cur = up;
    }
    *root = ep_quant(cur[0], cur[1]);
    free(own);
}

static void build_env_pyramid(or_scene *s)
{
    uint32_t W = s->ew, H = s->eh, m = 0;
    while ((1u << m) < H) ++m;
    if (H != (1u << m) || W != 2 * H || m < 1) return;  /* lat-long 2:1 powers of two only */
    s->ep_m = m;
    s->ep_top = m < EP_TOP ? m : EP_TOP;
    double *w = (double *)malloc(sizeof(double) * (size_t)W * H);
    for (uint32_t r = 0; r < H; ++r) {
        double om = (2.0 * M_PI / W) * (cos(M_PI * r / H) - cos(M_PI * (r + 1) / H));
        for (uint32_t c = 0; c < W; ++c) w[(size_t)r * W + c] = lum(s->env[(size_t)r * W + c]) * om;
    }
    s->ep_q = (uint32_t *)calloc(4 * (size_t)ep_nodes_above(m), sizeof(uint32_t));
    ep_splits(w, m, &s->ep_root, s->ep_q);
    /* level-top weights (sums of the texels below each node, same order) */
    uint32_t t = s->ep_top, tw = 2u << t, th = 1u << t, sh = m - t;
    double *wt = (double *)malloc(sizeof(double) * tw * th);
    {
        double *cur = w, *own = NULL;
        for (uint32_t k = m; k > t; --k) {
            uint32_t cw = 1u << k, ch = 1u << (k - 1), fw = 2 * cw;
            double *up = (double *)malloc(sizeof(double) * cw * ch);
            for (uint32_t y = 0; y < ch; ++y)
                for (uint32_t x = 0; x < cw; ++x) {
                    double a = cur[(size_t)(2 * y) * fw + 2 * x], b = cur[(size_t)(2 * y) * fw + 2 * x + 1];
                    double c = cur[(size_t)(2 * y + 1) * fw + 2 * x], d = cur[(size_t)(2 * y + 1) * fw + 2 * x + 1];
                    up[(size_t)y * cw + x] = ((a + b) + c) + d;
                }
            free(own);
            own = up;
            cur = up;
        }
        memcpy(wt, cur, sizeof(double) * tw * th);
        free(own);
    }
    (void)sh;
    /* bounding cones of the level-top cells and of the normal bins */
    v3 *rc = (v3 *)malloc(sizeof(v3) * tw * th);
    double *rd = (double *)malloc(sizeof(double) * tw * th);
    for (uint32_t y = 0; y < th; ++y)
        for (uint32_t x = 0; x < tw; ++x) {
            double t0 = M_PI * y / th, t1 = M_PI * (y + 1) / th;
            double p0 = 2.0 * M_PI * x / tw, p1 = 2.0 * M_PI * (x + 1) / tw;
            v3 c = ep_dir(0.5 * (t0 + t1), 0.5 * (p0 + p1));
            double d = fmax(fmax(ep_angle(c, ep_dir(t0, p0)), ep_angle(c, ep_dir(t0, p1))),
                            fmax(ep_angle(c, ep_dir(t1, p0)), ep_angle(c, ep_dir(t1, p1))));
            rc[(size_t)y * tw + x] = c;
            rd[(size_t)y * tw + x] = d + 0.01;
        }
    uint32_t per = 4 * (1 + ep_nodes_above(t));
    s->ep_oq = (uint32_t *)calloc((size_t)EP_K * EP_K * per, sizeof(uint32_t));
    double *sw = (double *)malloc(sizeof(double) * tw * th);
    const double cell = 2.0 / EP_K;
    for (uint32_t b = 0; b < EP_K * EP_K; ++b) {
        uint32_t i = b % EP_K, j = b / EP_K;
        double x0 = -1.0 + cell * i, z0 = -1.0 + cell * j;
        v3 bc = ep_oct_decode(x0 + 0.5 * cell, z0 + 0.5 * cell);
        double g = 0.0;
        for (int e = 0; e <= 16; ++e) {
            double f = e / 16.0;
            g = fmax(g, ep_angle(bc, ep_oct_decode(x0 + f * cell, z0)));
            g = fmax(g, ep_angle(bc, ep_oct_decode(x0 + f * cell, z0 + cell)));
            g = fmax(g, ep_angle(bc, ep_oct_decode(x0, z0 + f * cell)));
            g = fmax(g, ep_angle(bc, ep_oct_decode(x0 + cell, z0 + f * cell)));
        }
        g += 0.02;
        for (uint32_t q = 0; q < tw * th; ++q) {
            double ang = ep_angle(bc, rc[q]) - g - rd[q];
            double f = ang <= 0.0 ? 1.0 : (ang >= 0.5 * M_PI ? 0.0 : cos(ang));
            sw[q] = wt[q] * f;
        }
        uint32_t *o = s->ep_oq + (size_t)b * per;
        ep_splits(sw, t, &o[0], o + 4);
    }
    free(sw);
    free(rc);
    free(rd);
    free(wt);
    free(w);
}

static uint64_t ep_split(uint64_t R, uint32_t q)
{
    if (q == 0) return 0;
    if (q >= (1u << 24)) return R;
    uint64_t T = (R >> 24) * q + (((R & 0xFFFFFFull) * q) >> 24);
    if (R >= 2) {
        if (T < 1) T = 1;
        if (T > R - 1) T = R - 1;
    }
    return T;
}

/* the split probabilities used at a node of level k for normal bin `bin`
 * (-1: the shared, unoriented ones) */
static const uint32_t *ep_node_q(const or_scene *s, int bin, uint32_t k, uint32_t y, uint32_t x)
{
    size_t at = (size_t)ep_nodes_above(k) + (size_t)y * (2u << k) + x;
    if (bin >= 0 && k < s->ep_top) return s->ep_oq + (size_t)bin * 4 * (1 + ep_nodes_above(s->ep_top)) + 4 + 4 * at;
    return s->ep_q + 4 * at;
}

static uint32_t ep_root_q(const or_scene *s, int bin)
{
    return bin >= 0 ? s->ep_oq[(size_t)bin * 4 * (1 + ep_nodes_above(s->ep_top))] : s->ep_root;
}

/* Descend with samples (u, v): texel (row, col) and the final intervals.
 * With `steer`, follow the given texel instead (u, v ignored). */
static void ep_descend(const or_scene *s, int bin, uint32_t u, uint32_t v, int steer, uint32_t *row,
                       uint32_t *col, uint64_t *Ru, uint64_t *Su, uint64_t *Rv, uint64_t *Sv)
{
    uint32_t m = s->ep_m;
    uint64_t ru = 1ull << 32, su = u, rv = 1ull << 32, sv = v;
    uint32_t x, y = 0;
    uint64_t T = ep_split(ru, ep_root_q(s, bin));
    int right = steer ? (int)((*col >> m) & 1u) : (su >= T);
    if (right) { su -= T; ru -= T; } else ru = T;
    x = (uint32_t)right;
    for (uint32_t k = 0; k < m; ++k) {
        const uint32_t *q = ep_node_q(s, bin, k, y, x);
        T = ep_split(ru, q[0]);
        int cx = steer ? (int)((*col >> (m - 1 - k)) & 1u) : (su >= T);
        if (cx) { su -= T; ru -= T; } else ru = T;
        T = ep_split(rv, cx ? q[2] : q[1]);
        int cy = steer ? (int)((*row >> (m - 1 - k)) & 1u) : (sv >= T);
        if (cy) { sv -= T; rv -= T; } else rv = T;
        x = 2 * x + (uint32_t)cx;
        y = 2 * y + (uint32_t)cy;
    }
    *row = y;
    *col = x;
    *Ru = ru;
    *Su = su;
    *Rv = rv;
    *Sv = sv;
}

/* ----------------------------------------------------------- FP64 BVH */

static void tri_bounds(const or_scene *s, uint32_t t, v3 *lo, v3 *hi)
{
    v3 a = s->p0[t], b = s->p1[t], c = s->p2[t];
    *lo = V3(fmin(a.x, fmin(b.x, c.x)), fmin(a.y, fmin(b.y, c.y)), fmin(a.z, fmin(b.z, c.z)));
    *hi = V3(fmax(a.x, fmax(b.x, c.x)), fmax(a.y, fmax(b.y, c.y)), fmax(a.z, fmax(b.z, c.z)));
}

static double *g_sort_key;
static int cmp_key(const void *a, const void *b)
{
    double x = g_sort_key[*(const uint32_t *)a], y = g_sort_key[*(const uint32_t *)b];
    if (x < y) return -1;
    if (x > y) return 1;
    return (*(const uint32_t *)a < *(const uint32_t *)b) ? -1 : 1;
}

/* median split on the longest centroid axis; leaves of at most 4 triangles */
static int32_t bvh_build(or_scene *s, uint32_t first, uint32_t count, double *key)
{
    int32_t me = (int32_t)s->nnodes++;
    bnode *nd = &s->nodes[me];
    v3 lo = V3(INFINITY, INFINITY, INFINITY), hi = V3(-INFINITY, -INFINITY, -INFINITY);
    v3 clo = lo, chi = hi;
    for (uint32_t q = first; q < first + count; ++q) {
        v3 a, b;
        tri_bounds(s, s->order[q], &a, &b);
        lo = V3(fmin(lo.x, a.x), fmin(lo.y, a.y), fmin(lo.z, a.z));
        hi = V3(fmax(hi.x, b.x), fmax(hi.y, b.y), fmax(hi.z, b.z));
        v3 cc = mul(add(a, b), 0.5);
        clo = V3(fmin(clo.x, cc.x), fmin(clo.y, cc.y), fmin(clo.z, cc.z));
        chi = V3(fmax(chi.x, cc.x), fmax(chi.y, cc.y), fmax(chi.z, cc.z));
    }
    /* pad so that rounding in the slab test never culls a touching triangle */
    double pad = 1e-9 * (1.0 + fmax(maxc(V3(fabs(lo.x), fabs(lo.y), fabs(lo.z))),
                                    maxc(V3(fabs(hi.x), fabs(hi.y), fabs(hi.z)))));
    s->nodes[me].lo = sub(lo, V3(pad, pad, pad));
    s->nodes[me].hi = add(hi, V3(pad, pad, pad));
    if (count <= 4) {
        nd = &s->nodes[me];
        nd->left = -1 - (int32_t)first;
        nd->right = (int32_t)count;
        return me;
    }
    v3 ext = sub(chi, clo);
    int ax = 0;
    if (ext.y > comp(ext, ax)) ax = 1;
    if (ext.z > comp(ext, ax)) ax = 2;
    for (uint32_t q = first; q < first + count; ++q) {
        v3 a, b;
        tri_bounds(s, s->order[q], &a, &b);
        key[s->order[q]] = comp(add(a, b), ax);
    }
    g_sort_key = key;
    qsort(s->order + first, count, sizeof(uint32_t), cmp_key);
    uint32_t half = count / 2;
    int32_t l = bvh_build(s, first, half, key);
    int32_t r = bvh_build(s, first + half, count - half, key);
    s->nodes[me].left = l;
    s->nodes[me].right = r;
    return me;
}

/* FP64 watertight test, same structure as the FP32 one */
static int tri_hit_f64(v3 o, int kx, int ky, int kz, double Sx, double Sy, double Sz,
                       v3 a, v3 b, v3 c, double tmax, double *t_out, double *b1, double *b2)
{
    v3 A = sub(a, o), B = sub(b, o), C = sub(c, o);
    double Ax = comp(A, kx) - Sx * comp(A, kz), Ay = comp(A, ky) - Sy * comp(A, kz);
    double Bx = comp(B, kx) - Sx * comp(B, kz), By = comp(B, ky) - Sy * comp(B, kz);
    double Cx = comp(C, kx) - Sx * comp(C, kz), Cy = comp(C, ky) - Sy * comp(C, kz);
    double U = Cx * By - Cy * Bx, V = Ax * Cy - Ay * Cx, W = Bx * Ay - By * Ax;
    if ((U < 0 || V < 0 || W < 0) && (U > 0 || V > 0 || W > 0)) return 0;
    double det = U + V + W;
    if (det == 0.0) return 0;
    double T = U * (Sz * comp(A, kz)) + V * (Sz * comp(B, kz)) + W * (Sz * comp(C, kz));
    double t = T / det;
    if (!(t > 0.0 && t < tmax)) return 0;
    *t_out = t;
    *b1 = V / det;
    *b2 = W / det;
    return 1;
}

typedef struct { double t, b1, b2; int64_t tri; } hit64;

static int box_hit(const bnode *nd, v3 o, v3 d, double tmax, double *tnear)
{
    double t0 = 0.0, t1 = tmax;
    for (int c = 0; c < 3; ++c) {
        double oc = comp(o, c), dc = comp(d, c), lo = comp(nd->lo, c), hi = comp(nd->hi, c);
        if (dc == 0.0) {
            if (oc < lo || oc > hi) return 0;
            continue;
        }
        double a = (lo - oc) / dc, b = (hi - oc) / dc;
        if (a > b) { double x = a; a = b; b = x; }
        if (a > t0) t0 = a;
        if (b < t1) t1 = b;
        if (t0 > t1) return 0;
    }
    *tnear = t0;
    return 1;
}

/* closest hit (any_hit = 0) or occlusion test (any_hit = 1) over [0, tmax) */
static int trace64(const or_scene *s, v3 o, v3 d, double tmax, int any_hit, int brute, hit64 *h)
{
    int kz = 0;
    if (fabs(d.y) > fabs(comp(d, kz))) kz = 1;
    if (fabs(d.z) > fabs(comp(d, kz))) kz = 2;
    int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
    if (comp(d, kz) < 0.0) { int q = kx; kx = ky; ky = q; }
    double Sx = comp(d, kx) / comp(d, kz), Sy = comp(d, ky) / comp(d, kz), Sz = 1.0 / comp(d, kz);
    h->t = tmax;
    h->tri = -1;
    if (brute || !s->nodes) {
        for (uint32_t t = 0; t < s->nt; ++t) {
            double tt, b1, b2;
            if (!tri_hit_f64(o, kx, ky, kz, Sx, Sy, Sz, s->p0[t], s->p1[t], s->p2[t], tmax,
                             &tt, &b1, &b2))
                continue;
            if (any_hit) return 1;
            if (h->tri < 0 || tt < h->t || (tt == h->t && (int64_t)t < h->tri)) {
                h->t = tt; h->b1 = b1; h->b2 = b2; h->tri = t;
            }
        }
        return h->tri >= 0;
    }
    int32_t stack[128];
    int sp = 0;
    stack[sp++] = 0;
    while (sp) {
        const bnode *nd = &s->nodes[stack[--sp]];
        double tn;
        if (!box_hit(nd, o, d, h->tri >= 0 ? h->t : tmax, &tn)) continue;
        if (nd->left < 0) {
            uint32_t first = (uint32_t)(-1 - nd->left);
            for (uint32_t q = first; q < first + (uint32_t)nd->right; ++q) {
                uint32_t t = s->order[q];
                double tt, b1, b2;
                if (!tri_hit_f64(o, kx, ky, kz, Sx, Sy, Sz, s->p0[t], s->p1[t], s->p2[t], tmax,
                                 &tt, &b1, &b2))
                    continue;
                if (any_hit) return 1;
                if (h->tri < 0 || tt < h->t || (tt == h->t && (int64_t)t < h->tri)) {
                    h->t = tt; h->b1 = b1; h->b2 = b2; h->tri = t;
                }
            }
        } else {
            stack[sp++] = nd->right;
            stack[sp++] = nd->left;
        }
    }
    return h->tri >= 0;
}

/* ------------------------------------------------------------- creation */

or_scene *or_scene_create(uint32_t nv, const float *pos, uint32_t nt, const uint32_t *idx,
                          const uint32_t *tri_mat, uint32_t nm, const float *albedo,
                          const float *rough, const float *emission, const uint32_t *flags,
                          uint32_t ew, uint32_t eh, const float *env, const double *cam,
                          uint32_t W, uint32_t H, int build_bvh)
{
    or_scene *s = (or_scene *)calloc(1, sizeof(or_scene));
    s->nt = nt;
    s->p0 = (v3 *)malloc(sizeof(v3) * nt);
    s->p1 = (v3 *)malloc(sizeof(v3) * nt);
    s->p2 = (v3 *)malloc(sizeof(v3) * nt);
    s->mat = (uint32_t *)malloc(sizeof(uint32_t) * nt);
    for (uint32_t t = 0; t < nt; ++t) {
        const float *a = pos + 3 * idx[3 * t], *b = pos + 3 * idx[3 * t + 1],
                    *c = pos + 3 * idx[3 * t + 2];
        s->p0[t] = V3(a[0], a[1], a[2]);
        s->p1[t] = V3(b[0], b[1], b[2]);
        s->p2[t] = V3(c[0], c[1], c[2]);
        s->mat[t] = tri_mat[t];
    }
    s->nm = nm;
    s->albedo = (v3 *)malloc(sizeof(v3) * nm);
    s->emission = (v3 *)malloc(sizeof(v3) * nm);
    s->rough = (double *)malloc(sizeof(double) * nm);
    s->flags = (uint32_t *)malloc(sizeof(uint32_t) * nm);
    for (uint32_t m = 0; m < nm; ++m) {
        s->albedo[m] = V3(albedo[3 * m], albedo[3 * m + 1], albedo[3 * m + 2]);
        s->emission[m] = V3(emission[3 * m], emission[3 * m + 1], emission[3 * m + 2]);
        s->rough[m] = rough[m];
        s->flags[m] = flags[m];
    }
    build_lights(s);
    build_light_tree(s);
    if (env && ew && eh) {
        s->ew = ew; s->eh = eh;
        s->env = (v3 *)malloc(sizeof(v3) * (size_t)ew * eh);
        for (size_t q = 0; q < (size_t)ew * eh; ++q)
            s->env[q] = V3(env[3 * q], env[3 * q + 1], env[3 * q + 2]);
        build_env(s);
        build_env_pyramid(s);
    }
    s->p_env = s->env ? (s->ne ? 0.5 : 1.0) : 0.0;
    build_light_pmf(s);
    /* camera: cam = eye[3], look[3], up[3], vfov_deg */
    s->eye = V3(cam[0], cam[1], cam[2]);
    s->fwd = normalize(sub(V3(cam[3], cam[4], cam[5]), s->eye));
    s->right = normalize(cross(s->fwd, V3(cam[6], cam[7], cam[8])));
    s->up = cross(s->right, s->fwd);
    s->tan_half = tan(0.5 * cam[9] * M_PI / 180.0);
    s->W = W; s->H = H;
    s->aspect = (double)W / (double)H;
    for (int a = 0; a < 3; ++a) {
        double lo = INFINITY, hi = -INFINITY;
        for (uint32_t q = 0; q < nv; ++q) {
            lo = fmin(lo, (double)pos[3 * q + a]);
            hi = fmax(hi, (double)pos[3 * q + a]);
        }
        s->bmin[a] = nv ? lo : 0.0;
        s->bext[a] = nv ? fmax(hi - lo, 1e-6) : 1.0;
    }
    if (build_bvh && nt) {
        s->nodes = (bnode *)malloc(sizeof(bnode) * 2 * nt);
        s->order = (uint32_t *)malloc(sizeof(uint32_t) * nt);
        for (uint32_t t = 0; t < nt; ++t) s->order[t] = t;
        double *key = (double *)malloc(sizeof(double) * nt);
        bvh_build(s, 0, nt, key);
        free(key);
    }
    return s;
}

void or_scene_destroy(or_scene *s)
{
    if (!s) return;
    free(s->p0); free(s->p1); free(s->p2); free(s->mat);
    free(s->albedo); free(s->emission); free(s->rough); free(s->flags);
    free(s->emit_tri); free(s->emit_flux); free(s->alias_prob); free(s->alias_idx);
    free(s->alias_thr); free(s->emit_pmf); free(s->tri_emit);
    free(s->lt_c); free(s->lt_f); free(s->lt_left); free(s->lt_first); free(s->lt_count);
    free(s->lt_emit); free(s->lt_pos); free(s->lt_w);
    free(s->env); free(s->row_q); free(s->col_q); free(s->env_texel_pdf);
    free(s->ep_q); free(s->ep_oq);
    free(s->nodes); free(s->order);
    free(s->g_par);
    free(s);
}

/* table access for host-builder cross-checks */
uint32_t or_scene_num_emitters(const or_scene *s) { return s->ne; }
void or_scene_lights(const or_scene *s, uint32_t *emit_tri, double *flux, double *prob,
                     uint32_t *alias, double *pmf)
{
    for (uint32_t e = 0; e < s->ne; ++e) {
        if (emit_tri) emit_tri[e] = s->emit_tri[e];
        if (flux) flux[e] = s->emit_flux[e];
        if (prob) prob[e] = s->alias_prob[e];
        if (alias) alias[e] = s->alias_idx[e];
        if (pmf) pmf[e] = s->emit_pmf[e];
    }
}
void or_scene_env_tables(const or_scene *s, uint64_t *row_q, uint64_t *col_q, double *texel_pdf)
{
    if (!s->env) return;
    if (row_q) memcpy(row_q, s->row_q, sizeof(uint64_t) * (s->eh + 1));
    if (col_q) memcpy(col_q, s->col_q, sizeof(uint64_t) * (size_t)s->eh * (s->ew + 1));
    if (texel_pdf) memcpy(texel_pdf, s->env_texel_pdf, sizeof(double) * (size_t)s->ew * s->eh);
}

/* FP64 closest hit / occlusion for a batch of rays (n x 8 doubles) */
void or_trace64(const or_scene *s, const double *rays, uint32_t n, int any_hit, int brute,
                double *out_t, int64_t *out_tri)
{
    for (uint32_t r = 0; r < n; ++r) {
        const double *q = rays + 8 * (size_t)r;
        hit64 h;
        int hit = trace64(s, V3(q[0], q[1], q[2]), V3(q[4], q[5], q[6]), q[3], any_hit, brute, &h);
        out_tri[r] = any_hit ? hit : (hit ? h.tri : -1);
        if (out_t) out_t[r] = hit && !any_hit ? h.t : INFINITY;
    }
}

/* ------------------------------------------------------------ sampling */

/* orthonormal basis around unit n (Duff et al. 2017) */
static void onb(v3 n, v3 *b1, v3 *b2)
{
    double sign = copysign(1.0, n.z);
    double a = -1.0 / (sign + n.z);
    double b = n.x * n.y * a;
    *b1 = V3(1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x);
    *b2 = V3(b, sign + n.y * n.y * a, -n.y);
}

static double fresnel(double c)
{
    double m = 1.0 - c;
    if (m < 0.0) m = 0.0;
    double m2 = m * m;
    return 0.04 + 0.96 * m2 * m2 * m;
}

static double ggx_D(double cos_h, double a2)
{
    double k = cos_h * cos_h * (a2 - 1.0) + 1.0;
    return a2 / (M_PI * k * k);
}

static double ggx_lambda(double cos_t, double a2)
{
    double c2 = cos_t * cos_t;
    double tan2 = (1.0 - c2) / c2;
    return 0.5 * (-1.0 + sqrt(1.0 + a2 * tan2));
}

/* probability of picking the specular lobe, as realised by u < p on the
 * 24-bit sample grid: ceil(p * 2^24) / 2^24 with p first rounded to FP32 */
static double spec_choice(const or_scene *s, uint32_t m, double cos_o)
{
    double F = fresnel(cos_o);
    double p = F / (F + (1.0 - F) * lum(s->albedo[m]));
    if (p < 0.1) p = 0.1;
    if (p > 0.9) p = 0.9;
    float pf = (float)p;
    return ceil((double)pf * 16777216.0) / 16777216.0;
}

/* BSDF value f (without the cosine) and sampling pdf (solid angle) for a
 * reflection on the side of n (n faces wo); wi below the surface -> 0 */
static void bsdf_eval(const or_scene *s, uint32_t m, v3 n, v3 wo, v3 wi, v3 *f, double *pdf)
{
    double co = dot(n, wo), ci = dot(n, wi);
    *f = V3(0, 0, 0);
    *pdf = 0.0;
    if (co <= 0.0 || ci <= 0.0) return;
    v3 rho = s->albedo[m];
    if (!(s->flags[m] & MAT_GGX)) {
        *f = mul(rho, 1.0 / M_PI);
        *pdf = ci / M_PI;
        return;
    }
    double a = s->rough[m], a2 = a * a;
    v3 h = normalize(add(wo, wi));
    double ch = dot(n, h), oh = dot(wo, h);
    double D = ggx_D(ch, a2);
    double G2 = 1.0 / (1.0 + ggx_lambda(co, a2) + ggx_lambda(ci, a2));
    double G1o = 1.0 / (1.0 + ggx_lambda(co, a2));
    double spec = D * G2 * fresnel(oh) / (4.0 * co * ci);
    double kd = (1.0 - fresnel(co)) * (1.0 - fresnel(ci)) / M_PI;
    *f = add(V3(spec, spec, spec), mul(rho, kd));
    double ps = spec_choice(s, m, co);
    *pdf = ps * G1o * D / (4.0 * co) + (1.0 - ps) * ci / M_PI;
}

/* sample wi; returns 0 when the sample leaves the upper hemisphere */
static int bsdf_sample(const or_scene *s, uint32_t m, v3 n, v3 wo, double u3, double u4,
                       double u5, v3 *wi)
{
    v3 b1, b2;
    onb(n, &b1, &b2);
    double co = dot(n, wo);
    int spec = 0;
    if (s->flags[m] & MAT_GGX) spec = u3 < spec_choice(s, m, co);
    if (!spec) {
        double r = sqrt(u4), ph = 2.0 * M_PI * u5;
        double z = sqrt(fmax(0.0, 1.0 - u4));
        *wi = add(add(mul(b1, r * cos(ph)), mul(b2, r * sin(ph))), mul(n, z));
        return 1;
    }
    /* visible-normal sampling (Heitz 2018) in the local frame */
    double a = s->rough[m];
    v3 wl = V3(dot(wo, b1), dot(wo, b2), co);
    v3 vh = normalize(V3(a * wl.x, a * wl.y, wl.z));
    double l2 = vh.x * vh.x + vh.y * vh.y;
    v3 T1 = l2 > 0.0 ? mul(V3(-vh.y, vh.x, 0.0), 1.0 / sqrt(l2)) : V3(1.0, 0.0, 0.0);
    v3 T2 = cross(vh, T1);
    double r = sqrt(u4), ph = 2.0 * M_PI * u5;
    double t1 = r * cos(ph), t2 = r * sin(ph);
    double sh = 0.5 * (1.0 + vh.z);
    t2 = (1.0 - sh) * sqrt(fmax(0.0, 1.0 - t1 * t1)) + sh * t2;
    v3 nh = add(add(mul(T1, t1), mul(T2, t2)), mul(vh, sqrt(fmax(0.0, 1.0 - t1 * t1 - t2 * t2))));
    v3 ne = normalize(V3(a * nh.x, a * nh.y, fmax(0.0, nh.z)));
    v3 hw = add(add(mul(b1, ne.x), mul(b2, ne.y)), mul(n, ne.z));
    *wi = sub(mul(hw, 2.0 * dot(wo, hw)), wo);
    return dot(n, *wi) > 0.0;
}

/* environment radiance and texel pdf for a direction (and its texel) */
static v3 env_lookup_texel(const or_scene *s, v3 w, double *pdf, uint32_t *row, uint32_t *col)
{
    double th = acos(fmax(-1.0, fmin(1.0, w.y)));
    double ph = atan2(w.x, -w.z);
    if (ph < 0.0) ph += 2.0 * M_PI;
    int64_t r = (int64_t)floor(th / M_PI * s->eh), c = (int64_t)floor(ph / (2.0 * M_PI) * s->ew);
    if (r < 0) r = 0;
    if (r >= s->eh) r = s->eh - 1;
    if (c < 0) c = 0;
    if (c >= s->ew) c = s->ew - 1;
    size_t q = (size_t)r * s->ew + c;
    if (pdf) *pdf = s->env_texel_pdf[q];
    if (row) *row = (uint32_t)r;
    if (col) *col = (uint32_t)c;
    return s->env[q];
}
static v3 env_lookup(const or_scene *s, v3 w, double *pdf) { return env_lookup_texel(s, w, pdf, NULL, NULL); }

/* solid angle of a texel of row r */
static double env_texel_omega(const or_scene *s, uint32_t r)
{
    return (2.0 * M_PI / s->ew) * (cos(M_PI * r / s->eh) - cos(M_PI * (r + 1) / s->eh));
}

/* Wachter-Binder origin offset (reading of Sec. 2.2's front/back-side
 * points): each coordinate moves by trunc(256 n_c) steps of the FP32 grid,
 * counted on the bit pattern of its FP32 value (so a step across a power of
 * two uses the finer spacing below it), or by n_c / 65536 within 1/32 of
 * the origin. The oracle adds to its FP64 point exactly the displacement
 * this rule gives to the FP32 rounding of that point. */
static double offset1(double p, double n)
{
    if (fabs(p) < 1.0 / 32.0) return p + n / 65536.0;
    float pf = (float)p;
    int32_t k = (int32_t)(float)(256.0f * (float)n);
    int32_t bits;
    memcpy(&bits, &pf, 4);
    bits += pf < 0.0f ? -k : k;
    float qf;
    memcpy(&qf, &bits, 4);
    return p + ((double)qf - (double)pf);
}
static v3 offset_ray(v3 p, v3 n) { return V3(offset1(p.x, n.x), offset1(p.y, n.y), offset1(p.z, n.z)); }

/* ------------------------------------------- the learned proposal (frozen)
 *
 * Not in the paper: the workload extends its importance sampling (Sec. 2.1,
 * 2.2) by a directional proposal learned from the renderer's own samples and
 * mixed one-sided with BSDF sampling under multiple importance sampling. The
 * oracle evaluates a FROZEN network (parameters given by the caller) step by
 * step as the design readings define it:
 *   - features: the hit position normalised to the scene's box, and the
 *     outgoing direction's polar angle (from +y, over pi) and azimuth
 *     (atan2(x, -z) over 2 pi, in [0, 1)); sin and cos of 2^o pi x_a for
 *     o = 0..3 per axis, then of pi th, 2 pi th, 2 pi ph, 4 pi ph;
 *   - network 32 -> 64 -> 64 -> 64 -> 40, ReLU on the hidden layers, weights,
 *     biases, inputs and hidden activations rounded to BF16 (ties to even),
 *     sums in FP64 (the kernels sum in FP32);
 *   - decode per lobe k (outputs 5k..5k+4: logit, mean xyz, concentration):
 *     softmax weights, unit means, kappa = min(softplus + 1e-3, 1e4);
 *   - the proposal is the mixture these parameters define after rounding
 *     them to FP16 (ties to even), with the rounded means and weights
 *     renormalised: any density gives an unbiased estimator, and this is the
 *     one the renderer stores per path vertex;
 *   - vMF lobe density kappa / (2 pi (1 - e^-2kappa)) e^(kappa (mu.w - 1));
 *     sampling: the lobe is the first k whose cumulative weight exceeds u,
 *     the cosine to the mean w = 1 + log(u1 + (1 - u1) e^-2kappa) / kappa
 *     (Jakob 2012), the azimuth 2 pi u2 in a Duff et al. 2017 frame;
 *   - one-sample mixture: the guide is taken iff the 32-bit sample of slot 3
 *     is below alpha 2^32 (an integer threshold), the rest of that sample,
 *     rescaled to [0, 2^32), picks the lobe (or the BSDF's own lobe); the
 *     density is alpha q + (1 - alpha) p_bsdf, used in the throughput and in
 *     both power-heuristic weights against next-event estimation. */

#define G_LOBES 8
static const int g_sizes[5] = {32, 64, 64, 64, 40};

/* round to the binary format with `bits` significand bits (hidden bit
 * included) whose smallest subnormal step is 2^sub, ties to even */
static double round_fmt(double x, int bits, int sub)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);                       /* |x| in [2^(e-1), 2^e) */
    int q = e - bits;                   /* exponent of the last kept bit */
    if (q < sub) q = sub;
    return ldexp(nearbyint(ldexp(x, -q)), q);   /* default rounding: to nearest, ties to even */
}
double or_round_bf16(double x) { return round_fmt(x, 8, -133); }
double or_round_fp16(double x) { return round_fmt(x, 11, -24); }

/* Load a frozen guide: FP32 parameters (13032: per layer W (in x out,
 * row-major) then b), alpha as its integer threshold (guide iff slot-3 bits
 * < alpha_thr; 0 = off), guided vertices 1..max_vertex (0 = all) and the
 * record-hash threshold (records of vertices whose hash is below it;
 * 0xffffffff = all). */
void or_guide_set(or_scene *s, const float *par, uint32_t alpha_thr, uint32_t max_vertex, uint32_t rec_thr)
{
    size_t n = 0;
    for (int l = 0; l < 4; ++l) n += (size_t)g_sizes[l] * g_sizes[l + 1] + g_sizes[l + 1];
    free(s->g_par);
    s->g_par = (double *)malloc(sizeof(double) * n);
    for (size_t k = 0; k < n; ++k) s->g_par[k] = or_round_bf16((double)par[k]);
    s->g_alpha_thr = alpha_thr;
    s->g_maxv = max_vertex ? max_vertex : 0xffffffffu;
    s->g_rec_thr = rec_thr;
}

static void guide_features(const or_scene *s, v3 x, v3 wo, double f[32])
{
    double xh[3] = {(x.x - s->bmin[0]) / s->bext[0], (x.y - s->bmin[1]) / s->bext[1],
                    (x.z - s->bmin[2]) / s->bext[2]};
    for (int a = 0; a < 3; ++a)
        for (int o = 0; o < 4; ++o) {
            double ang = ldexp(M_PI, o) * xh[a];
            f[8 * a + 2 * o] = sin(ang);
            f[8 * a + 2 * o + 1] = cos(ang);
        }
    double th = acos(fmax(-1.0, fmin(1.0, wo.y))) / M_PI;
    double ph = atan2(wo.x, -wo.z);
    if (ph < 0.0) ph += 2.0 * M_PI;
    ph /= 2.0 * M_PI;
    double ang[4] = {M_PI * th, 2.0 * M_PI * th, 2.0 * M_PI * ph, 4.0 * M_PI * ph};
    for (int j = 0; j < 4; ++j) {
        f[24 + 2 * j] = sin(ang[j]);
        f[25 + 2 * j] = cos(ang[j]);
    }
}

/* network outputs for 32 features (BF16 rounding points as stated above) */
static void guide_forward(const or_scene *s, const double feat[32], double out[40])
{
    double a[64], z[64];
    for (int i = 0; i < 32; ++i) a[i] = or_round_bf16(feat[i]);
    const double *p = s->g_par;
    for (int l = 0; l < 4; ++l) {
        const int fi = g_sizes[l], fo = g_sizes[l + 1];
        const double *Wl = p, *bl = p + (size_t)fi * fo;
        for (int o = 0; o < fo; ++o) {
            double acc = bl[o];
            for (int i = 0; i < fi; ++i) acc += a[i] * Wl[(size_t)i * fo + o];
            z[o] = acc;
        }
        p = bl + fo;
        if (l < 3)
            for (int o = 0; o < fo; ++o) a[o] = or_round_bf16(z[o] > 0.0 ? z[o] : 0.0);
        else
            for (int o = 0; o < fo; ++o) out[o] = z[o];
    }
}

typedef struct {
    double w[G_LOBES];      /* lobe weights, sum 1 */
    v3 mu[G_LOBES];         /* unit means */
    double kappa[G_LOBES];
} gmix;

/* decode, then the FP16 storage of the proposal's parameters */
static void guide_decode(const double out[40], gmix *m)
{
    double mx = out[0];
    for (int k = 1; k < G_LOBES; ++k) mx = fmax(mx, out[5 * k]);
    double e[G_LOBES], se = 0.0;
    for (int k = 0; k < G_LOBES; ++k) {
        e[k] = exp(out[5 * k] - mx);
        se += e[k];
    }
    double wsum = 0.0;
    for (int k = 0; k < G_LOBES; ++k) {
        const double *o = out + 5 * k;
        double n = fmax(sqrt(o[1] * o[1] + o[2] * o[2] + o[3] * o[3]), 1e-12);
        double sp = o[4] > 30.0 ? o[4] : log1p(exp(o[4]));
        double kap = fmin(sp + 1e-3, 1e4);
        v3 mu = V3(or_round_fp16(o[1] / n), or_round_fp16(o[2] / n), or_round_fp16(o[3] / n));
        double mn = fmax(len(mu), 1e-12);
        m->mu[k] = mul(mu, 1.0 / mn);
        m->kappa[k] = or_round_fp16(kap);
        m->w[k] = or_round_fp16(e[k] / se);
        wsum += m->w[k];
    }
    for (int k = 0; k < G_LOBES; ++k) m->w[k] /= wsum;
}

static double vmf_pdf(v3 mu, double kappa, v3 w)
{
    return kappa / (2.0 * M_PI * -expm1(-2.0 * kappa)) * exp(kappa * (dot(mu, w) - 1.0));
}

/* A deliberately planted mistake, for tests that show the pins catch it
 * (0 = none; 1: the mixture density reported twice too large; 2: record
 * weights not divided by the throughput before the vertex; 3: record weights
 * that keep the vertex's own next-event estimate). Not thread-safe
 * to change while rendering. */
static int g_plant = 0;
void or_plant(int which) { g_plant = which; }

static double gmix_pdf(const gmix *m, v3 w)
{
    double q = 0.0;
    for (int k = 0; k < G_LOBES; ++k) q += m->w[k] * vmf_pdf(m->mu[k], m->kappa[k], w);
    return g_plant == 1 ? 2.0 * q : q;
}

static v3 gmix_sample(const gmix *m, double u, double u1, double u2)
{
    int k = G_LOBES - 1;
    double c = 0.0;
    for (int j = 0; j < G_LOBES - 1; ++j) {
        c += m->w[j];
        if (u < c) {
            k = j;
            break;
        }
    }
    double kap = m->kappa[k];
    double w = 1.0 + log(u1 + (1.0 - u1) * exp(-2.0 * kap)) / kap;
    w = fmax(-1.0, fmin(1.0, w));
    v3 t1, t2;
    onb(m->mu[k], &t1, &t2);
    double r = sqrt(fmax(0.0, 1.0 - w * w)), ph = 2.0 * M_PI * u2;
    return add(mul(m->mu[k], w), add(mul(t1, r * cos(ph)), mul(t2, r * sin(ph))));
}

static void guide_mixture(const or_scene *s, v3 x, v3 wo, gmix *m)
{
    double f[32], out[40];
    guide_features(s, x, wo, f);
    guide_forward(s, f, out);
    guide_decode(out, m);
}

/* which vertices leave a training record: the splitmix64 finaliser of the
 * path's sample index and the depth, top 32 bits */
static uint32_t rec_hash(uint64_t idx, uint32_t v)
{
    uint64_t z = idx * 0x9E3779B97F4A7C15ull + (uint64_t)v * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return (uint32_t)((z ^ (z >> 31)) >> 32);
}

/* Training record of a guided-depth vertex whose path continues: position,
 * directions, the mixture density of the sampled direction, and the parts
 * its weight is formed from at the path's end (radiance before the vertex's
 * next-event estimate, that estimate, throughput before the scattering with
 * roulette folded in). Weight = sum_c lum_c max(0, (L_end - (L_before + NEE))_c
 * / T_c) over the channels with T_c > 0: the sample's own estimate
 * f cos L_i / p of the scattering integral. */
typedef struct {
    uint32_t v;
    v3 x, wo, wi;
    double pdf;
    v3 Lb, nee, Tb;
} grec;

#define G_MAX_REC 256

typedef struct {
    uint32_t max_depth;
    uint32_t rr;        /* Russian roulette from vertex 3 */
    uint32_t mode;      /* 0 MIS, 1 BSDF sampling only, 2 NEE only */
    uint32_t scramble;
    uint32_t light_tree; /* select triangle lights through the light tree */
    uint32_t env_pyramid; /* 0: 2D CDF, 1: pyramid, 2: pyramid with normal-weighted top levels */
    uint32_t gauss;       /* film samples from a Gaussian around the pixel centre instead of the box */
    uint32_t guide;       /* the frozen guide of or_guide_set mixes in (when its alpha is not 0) */
    uint32_t record;      /* collect training records (guide vertices whose path continues) */
} or_opts;

/* the caller's mode word: MIS mode in the low byte, light tree in bit 8,
 * environment sampling in bits 9-10, Gaussian pixel filter in bit 11, the
 * frozen guide in bit 12, training records in bit 13 */
static or_opts make_opts(uint32_t max_depth, uint32_t rr, uint32_t mode, uint32_t scramble)
{
    or_opts op = {max_depth, rr, mode & 0xffu, scramble, (mode >> 8) & 1u, (mode >> 9) & 3u, (mode >> 11) & 1u,
                  (mode >> 12) & 1u, (mode >> 13) & 1u};
    return op;
}

static inline double mis2(double a, double b) { return a * a / (a * a + b * b); }

/* optional per-vertex log for single-path debugging (not thread-safe) */
static double *g_log = NULL;
static uint32_t g_log_n = 0, g_log_cap = 0;
static void logv(double a, double b, double c, double d, double e, double f, double g, double h)
{
    if (!g_log || g_log_n + 8 > g_log_cap) return;
    double *q = g_log + g_log_n;
    q[0] = a; q[1] = b; q[2] = c; q[3] = d; q[4] = e; q[5] = f; q[6] = g; q[7] = h;
    g_log_n += 8;
}

/* radiance estimate of one path for sample index i through film point (fx, fy) */
static v3 trace_path(const or_scene *s, const or_opts *op, uint64_t i, uint32_t px, uint32_t py,
                     uint32_t *nrays, grec *recs, uint32_t *nrec)
{
    if (nrec) *nrec = 0;
    const uint32_t W = s->W, H = s->H;
    double u0 = u24(or_sample_bits(i, 0, W, H, 0)), u1 = u24(or_sample_bits(i, 1, W, H, 0));
    double fx = px + u0, fy = py + u1;
    if (op->gauss) {
        /* filter importance sampling (Appendix A.1): a Gaussian whose 3 sigma
         * range spans a 3 x 3 pixel block (sigma = 1/2 pixel) around the
         * centre, untruncated, by the Box-Muller transform of the film sample */
        double r = 0.5 * sqrt(-2.0 * log(1.0 - u0)), ph = 2.0 * M_PI * u1;
        fx = px + 0.5 + r * cos(ph);
        fy = py + 0.5 + r * sin(ph);
    }
    double sx = (2.0 * fx / W - 1.0) * s->tan_half * s->aspect;
    double sy = (1.0 - 2.0 * fy / H) * s->tan_half;
    v3 d = normalize(add(s->fwd, add(mul(s->right, sx), mul(s->up, sy))));
    v3 o = s->eye;
    v3 L = V3(0, 0, 0), T = V3(1, 1, 1);
    double prev_pdf = 0.0;
    v3 prev_n = V3(0, 0, 0);
    const int tree = op->light_tree && s->ne;
    const int pyr = op->env_pyramid && s->ep_m;
    const double p_tri = 1.0 - s->p_env;
    const int gon = op->guide && s->g_par && s->g_alpha_thr;
    const double alpha = gon ? (double)s->g_alpha_thr * 0x1p-32 : 0.0;
    for (uint32_t v = 1; v <= op->max_depth; ++v) {
        hit64 h;
        (*nrays)++;
        if (!trace64(s, o, d, INFINITY, 0, 0, &h)) {
            if (s->env && (v == 1 || op->mode != 2)) {
                double pe;
                uint32_t er, ec;
                v3 Le = env_lookup_texel(s, d, &pe, &er, &ec);
                double w = 1.0;
                if (v > 1 && op->mode == 0 && pyr) {
                    /* the pyramid's probability of this texel from the previous vertex */
                    float nf[3] = {(float)prev_n.x, (float)prev_n.y, (float)prev_n.z};
                    int bin = op->env_pyramid == 2 ? (int)ep_bin(nf) : -1;
                    uint64_t ru, su, rv, sv;
                    ep_descend(s, bin, 0, 0, 1, &er, &ec, &ru, &su, &rv, &sv);
                    pe = (double)ru * (double)rv * 0x1p-64 / env_texel_omega(s, er);
                    logv(5, v, er, ec, pe, 0, 0, 0);
                }
                if (v > 1 && op->mode == 0) w = mis2(prev_pdf, s->p_env * pe);
                L = add(L, mul(vmul(T, Le), w));
            }
            break;
        }
        uint32_t t = (uint32_t)h.tri, m = s->mat[t];
        v3 a = s->p0[t], b = s->p1[t], c = s->p2[t];
        v3 x = add(a, add(mul(sub(b, a), h.b1), mul(sub(c, a), h.b2)));
        logv(1, v, t, h.t, x.x, x.y, x.z, 0);
        logv(2, o.x, o.y, o.z, d.x, d.y, d.z, 0);
        v3 ng = cross(sub(b, a), sub(c, a));
        double area2 = len(ng);
        ng = mul(ng, 1.0 / area2);
        double dn = dot(d, ng);
        int front = dn < 0.0;
        if (front && s->tri_emit[t] >= 0 && !(v > 1 && op->mode == 2)) {
            v3 Le = emission_at(s, m, x);
            double w = 1.0;
            if (v > 1 && op->mode == 0) {
                double pe = s->emit_pmf[s->tri_emit[t]];
                if (tree) {
                    /* the tree's pdf seen from the previous vertex: its ray
                     * origin and normal in FP32, as the sampling used them */
                    float xf[3] = {(float)o.x, (float)o.y, (float)o.z};
                    float nf[3] = {(float)prev_n.x, (float)prev_n.y, (float)prev_n.z};
                    pe = p_tri * (double)lt_size_of(s, (uint32_t)s->tri_emit[t], xf, nf) * 0x1p-63;
                }
                double pl = pe / (0.5 * area2) * h.t * h.t / (-dn);
                w = mis2(prev_pdf, pl);
                logv(4, v, t, pe, pl, w, 0, 0);
            }
            L = add(L, mul(vmul(T, Le), w));
        }
        if (v == op->max_depth) break;
        if (!(maxc(s->albedo[m]) > 0.0 || (s->flags[m] & MAT_GGX))) break;
        v3 n = front ? ng : mul(ng, -1.0);
        v3 wo = mul(d, -1.0);
        v3 xo = offset_ray(x, n);
        uint32_t base = 2 + 8 * (v - 1);
        /* the guide's mixture at this vertex */
        const int guided = gon && v <= s->g_maxv;
        gmix mix;
        if (guided) guide_mixture(s, x, wo, &mix);
        const v3 L_before = L;
        v3 nee = V3(0, 0, 0);
        /* next-event estimation */
        if (op->mode != 1 && (s->ne || s->env)) {
            uint32_t s0 = or_sample_bits(i, base + 0, W, H, op->scramble);
            int use_env = 0;
            uint64_t r = s0, R = 1ull << 32;
            if (s->env && s->ne) {
                use_env = s0 < (1u << 31);
                r = s0 - (1u << 31);
                R = 1ull << 31;
            } else if (s->env) {
                use_env = 1;
            }
            v3 wi, Le;
            double pl = 0.0, dist = INFINITY;
            int ok = 0;
            if (use_env) {
                uint32_t s1 = or_sample_bits(i, base + 1, W, H, op->scramble);
                uint32_t s2 = or_sample_bits(i, base + 2, W, H, op->scramble);
                uint32_t row = 0, col = 0;
                double fyr, fxc, pt;
                if (pyr) {
                    /* pyramid: slot 2 narrows columns, slot 1 rows */
                    float nf[3] = {(float)n.x, (float)n.y, (float)n.z};
                    int bin = op->env_pyramid == 2 ? (int)ep_bin(nf) : -1;
                    uint64_t ru, su, rv, sv;
                    ep_descend(s, bin, s2, s1, 0, &row, &col, &ru, &su, &rv, &sv);
                    fxc = (double)su / (double)ru;
                    fyr = (double)sv / (double)rv;
                    pt = (double)ru * (double)rv * 0x1p-64 / env_texel_omega(s, row);
                } else {
                    while (row + 1 < s->eh && s->row_q[row + 1] <= s1) ++row;
                    const uint64_t *cq = s->col_q + (size_t)row * (s->ew + 1);
                    while (col + 1 < s->ew && cq[col + 1] <= s2) ++col;
                    fyr = (double)(s1 - s->row_q[row]) / (double)(s->row_q[row + 1] - s->row_q[row]);
                    fxc = (double)(s2 - cq[col]) / (double)(cq[col + 1] - cq[col]);
                    pt = s->env_texel_pdf[(size_t)row * s->ew + col];
                }
                double ct = cos(M_PI * row / s->eh), cb = cos(M_PI * (row + 1) / s->eh);
                double cth = ct + fyr * (cb - ct);
                double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
                double ph = 2.0 * M_PI * (col + fxc) / s->ew;
                wi = V3(sth * sin(ph), cth, -sth * cos(ph));
                size_t q = (size_t)row * s->ew + col;
                Le = s->env[q];
                pl = s->p_env * pt;
                ok = pl > 0.0;
            } else {
                uint32_t s7 = or_sample_bits(i, base + 7, W, H, op->scramble);
                uint32_t e;
                double pe;
                if (tree) {
                    /* 63-bit sample: the 31 bits left of slot 0 (its top 31
                     * bits without an environment), then slot 7 */
                    uint64_t hi = s->env ? r : (uint64_t)(s0 >> 1);
                    uint64_t S = (hi << 32) | s7, size;
                    float xf[3] = {(float)xo.x, (float)xo.y, (float)xo.z};
                    float nf[3] = {(float)n.x, (float)n.y, (float)n.z};
                    e = lt_sample(s, S, xf, nf, &size);
                    pe = p_tri * (double)size * 0x1p-63;
                } else {
                    uint32_t col = (uint32_t)(((u128)r * s->ne) / R);
                    e = (uint64_t)s7 < s->alias_thr[col] ? col : s->alias_idx[col];
                    pe = s->emit_pmf[e];
                }
                uint32_t lt = s->emit_tri[e];
                double q1 = u24(or_sample_bits(i, base + 1, W, H, op->scramble));
                double q2 = u24(or_sample_bits(i, base + 2, W, H, op->scramble));
                double su = sqrt(q1);
                double b0 = 1.0 - su, bb1 = q2 * su, bb2 = su * (1.0 - q2);
                v3 la = s->p0[lt], lb = s->p1[lt], lc = s->p2[lt];
                v3 y = add(add(mul(la, b0), mul(lb, bb1)), mul(lc, bb2));
                v3 nl = cross(sub(lb, la), sub(lc, la));
                double la2 = len(nl);
                nl = mul(nl, 1.0 / la2);
                v3 dv = sub(y, xo);
                double d2 = dot(dv, dv);
                dist = sqrt(d2);
                wi = mul(dv, 1.0 / dist);
                double cl = -dot(nl, wi);
                if (cl > 0.0) {
                    Le = emission_at(s, s->mat[lt], y);
                    pl = pe / (0.5 * la2) * d2 / cl;
                    ok = pl > 0.0;
                }
            }
            if (ok) {
                double ci = dot(n, wi);
                if (ci > 0.0) {
                    v3 f;
                    double pb;
                    bsdf_eval(s, m, n, wo, wi, &f, &pb);
                    if (guided) pb = alpha * gmix_pdf(&mix, wi) + (1.0 - alpha) * pb;
                    double w = op->mode == 2 ? 1.0 : mis2(pl, pb);
                    v3 contrib = mul(vmul(vmul(T, f), Le), ci * w / pl);
                    if (maxc(contrib) > 0.0) {
                        hit64 sh;
                        (*nrays)++;
                        double tm = isinf(dist) ? INFINITY : dist * (1.0 - 1e-4);
                        int occ = trace64(s, xo, wi, tm, 1, 0, &sh);
                        logv(3, occ, contrib.x, contrib.y, contrib.z, pl, w, 0);
                        if (!occ) {
                            L = add(L, contrib);
                            nee = contrib;
                        }
                    }
                }
            }
        }
        /* continue the path: slot 3 chooses guide or BSDF (guide iff its bits
         * are below alpha 2^32) and, its remainder rescaled to [0, 2^32), the
         * lobe; slots 4-5 the direction */
        uint32_t s3 = or_sample_bits(i, base + 3, W, H, op->scramble);
        int use_guide = guided && s3 < s->g_alpha_thr;
        uint32_t r3 = s3;
        if (guided) {
            uint64_t lo = use_guide ? 0 : s->g_alpha_thr;
            uint64_t range = use_guide ? s->g_alpha_thr : (1ull << 32) - s->g_alpha_thr;
            r3 = (uint32_t)((((uint64_t)s3 - lo) << 32) / range);
        }
        double u3 = u24(r3);
        double u4 = u24(or_sample_bits(i, base + 4, W, H, op->scramble));
        double u5 = u24(or_sample_bits(i, base + 5, W, H, op->scramble));
        v3 wi;
        if (use_guide) {
            wi = gmix_sample(&mix, u3, u4, u5);
            if (!(dot(n, wi) > 0.0)) break;
        } else if (!bsdf_sample(s, m, n, wo, u3, u4, u5, &wi)) {
            break;
        }
        v3 f;
        double pb;
        bsdf_eval(s, m, n, wo, wi, &f, &pb);
        if (guided) pb = alpha * gmix_pdf(&mix, wi) + (1.0 - alpha) * pb;
        if (!(pb > 0.0)) break;
        v3 Tb = T;
        T = vmul(T, mul(f, dot(n, wi) / pb));
        if (!(maxc(T) > 0.0)) break;
        prev_pdf = pb;
        prev_n = n;
        if (op->rr && v >= 3) {
            double q = fmin(0.95, maxc(T));
            float qf = (float)q;
            double qq = ceil((double)qf * 16777216.0) / 16777216.0;
            double u6 = u24(or_sample_bits(i, base + 6, W, H, op->scramble));
            if (!(u6 < qq)) break;
            T = mul(T, 1.0 / qq);
            Tb = mul(Tb, 1.0 / qq);
        }
        if (op->record && recs && v <= s->g_maxv && *nrec < G_MAX_REC &&
            (s->g_rec_thr == 0xffffffffu || rec_hash(i, v) < s->g_rec_thr)) {
            grec *r = &recs[(*nrec)++];
            r->v = v;
            r->x = x;
            r->wo = wo;
            r->wi = wi;
            r->pdf = pb;
            r->Lb = L_before;
            r->nee = nee;
            r->Tb = Tb;
        }
        o = xo;
        d = wi;
    }
    return L;
}

/* the weight of a record once its path has ended with radiance L (and, in
 * *nee_w, the same luminance-weighted quotient of the vertex's own next-event
 * estimate, which the weight leaves out) */
static double rec_weight(const grec *r, v3 L, double *nee_w)
{
    const double wl[3] = {0.2126, 0.7152, 0.0722};
    const double Lc[3] = {L.x, L.y, L.z}, bc[3] = {r->Lb.x, r->Lb.y, r->Lb.z};
    const double nc[3] = {r->nee.x, r->nee.y, r->nee.z}, tc[3] = {r->Tb.x, r->Tb.y, r->Tb.z};
    double w = 0.0, wn = 0.0;
    for (int c = 0; c < 3; ++c)
        if (tc[c] > 0.0) {
            double own = g_plant == 3 ? 0.0 : nc[c];
            /* the radiance after the vertex's own NEE is L_before + NEE, the
             * same addition the path made, so nothing gained afterwards is
             * an exact zero */
            w += wl[c] * fmax(0.0, (Lc[c] - (bc[c] + own)) / (g_plant == 2 ? 1.0 : tc[c]));
            wn += wl[c] * nc[c] / tc[c];
        }
    if (nee_w) *nee_w = wn;
    return w;
}

typedef struct {
    const or_scene *s;
    const or_opts *op;
    const uint32_t *pix;
    uint32_t npix;
    uint64_t pass0;
    uint32_t npasses;
    double *sum, *sumsq;
    uint32_t *count;
    uint64_t rays;
    volatile uint32_t *next;
    pthread_mutex_t *mu;
    double *rec_out;        /* training records (or_records), OR_REC_COLS doubles each */
    uint32_t rec_cap, *rec_n;
} job;

/* columns of a record row: pixel id, pass, vertex, x (3), wo (3), wi (3),
 * mixture density of wi, weight, the vertex's own NEE term */
#define OR_REC_COLS 15

static void *worker(void *arg)
{
    job *jb = (job *)arg;
    const or_scene *s = jb->s;
    uint64_t rays = 0;
    for (;;) {
        pthread_mutex_lock(jb->mu);
        uint32_t start = *jb->next;
        *jb->next = start + 64;
        pthread_mutex_unlock(jb->mu);
        if (start >= jb->npix) break;
        uint32_t end = start + 64 < jb->npix ? start + 64 : jb->npix;
        for (uint32_t q = start; q < end; ++q) {
            uint32_t p = jb->pix ? jb->pix[q] : q;
            uint32_t px = p % s->W, py = p / s->W;
            for (uint32_t j = 0; j < jb->npasses; ++j) {
                uint64_t i = or_pixel_index(s->W, s->H, px, py, jb->pass0 + j);
                uint32_t nr = 0, nrec = 0;
                grec recs[G_MAX_REC];
                v3 L = trace_path(s, jb->op, i, px, py, &nr, jb->rec_out ? recs : NULL, &nrec);
                rays += nr;
                if (jb->rec_out && nrec) {
                    pthread_mutex_lock(jb->mu);
                    for (uint32_t k = 0; k < nrec && *jb->rec_n < jb->rec_cap; ++k) {
                        double *o = jb->rec_out + (size_t)(*jb->rec_n)++ * OR_REC_COLS;
                        const grec *r = &recs[k];
                        double wn;
                        double w = rec_weight(r, L, &wn);
                        double row[OR_REC_COLS] = {p, (double)(jb->pass0 + j), r->v, r->x.x, r->x.y, r->x.z,
                                                   r->wo.x, r->wo.y, r->wo.z, r->wi.x, r->wi.y, r->wi.z, r->pdf,
                                                   w, wn};
                        memcpy(o, row, sizeof row);
                    }
                    pthread_mutex_unlock(jb->mu);
                }
                jb->sum[3 * q] += L.x; jb->sum[3 * q + 1] += L.y; jb->sum[3 * q + 2] += L.z;
                if (jb->sumsq) {
                    jb->sumsq[3 * q] += L.x * L.x;
                    jb->sumsq[3 * q + 1] += L.y * L.y;
                    jb->sumsq[3 * q + 2] += L.z * L.z;
                }
                jb->count[q] += 1;
            }
        }
    }
    jb->rays = rays;
    return NULL;
}

/* Render passes [pass0, pass0 + npasses) for npix pixels (ids p = y*W + x,
 * or all pixels when pix is NULL). Adds into caller-zeroed sum/sumsq/count,
 * one entry per listed pixel. Returns the number of rays traced. */
static uint64_t render_jobs(const or_scene *s, uint32_t max_depth, uint32_t rr, uint32_t mode,
                            uint32_t scramble, const uint32_t *pix, uint32_t npix, uint64_t pass0,
                            uint32_t npasses, double *sum, double *sumsq, uint32_t *count,
                            uint32_t nthreads, double *rec_out, uint32_t rec_cap, uint32_t *rec_n)
{
    or_opts op = make_opts(max_depth, rr, mode, scramble);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    job jobs[256];
    volatile uint32_t next = 0;
    pthread_mutex_t mu;
    pthread_mutex_init(&mu, NULL);
    for (uint32_t k = 0; k < nthreads; ++k) {
        jobs[k] = (job){s, &op, pix, npix, pass0, npasses, sum, sumsq, count, 0, &next, &mu, rec_out, rec_cap,
                        rec_n};
        pthread_create(&th[k], NULL, worker, &jobs[k]);
    }
    uint64_t rays = 0;
    for (uint32_t k = 0; k < nthreads; ++k) {
        pthread_join(th[k], NULL);
        rays += jobs[k].rays;
    }
    pthread_mutex_destroy(&mu);
    return rays;
}

uint64_t or_render(const or_scene *s, uint32_t max_depth, uint32_t rr, uint32_t mode,
                   uint32_t scramble, const uint32_t *pix, uint32_t npix, uint64_t pass0,
                   uint32_t npasses, double *sum, double *sumsq, uint32_t *count,
                   uint32_t nthreads)
{
    return render_jobs(s, max_depth, rr, mode & ~(1u << 13), scramble, pix, npix, pass0, npasses, sum, sumsq,
                       count, nthreads, NULL, 0, NULL);
}

/* The same rendering, also returning the training records of every path
 * (in no particular order): rows of OR_REC_COLS doubles (pixel id, pass,
 * vertex, x, wo, wi, mixture density, weight, NEE term), at most rec_cap of them;
 * returns how many were produced (rows beyond rec_cap are dropped). */
uint32_t or_records(const or_scene *s, uint32_t max_depth, uint32_t rr, uint32_t mode, uint32_t scramble,
                    const uint32_t *pix, uint32_t npix, uint64_t pass0, uint32_t npasses, double *sum,
                    uint32_t *count, uint32_t nthreads, double *rec_out, uint32_t rec_cap)
{
    uint32_t n = 0;
    render_jobs(s, max_depth, rr, mode | (1u << 13), scramble, pix, npix, pass0, npasses, sum, NULL, count,
                nthreads, rec_out, rec_cap, &n);
    return n;
}

/* one path with a per-vertex log: records of 8 doubles,
 * (1, v, tri, t, x) (2, ray o, ray d) (3, occluded, contrib, pl, w)
 * (4, v, tri, selection probability, pl, w) at an emitter hit under MIS
 * (5, v, row, col, texel pdf) at an environment hit under MIS with the pyramid */
uint32_t or_debug_path(const or_scene *s, uint32_t max_depth, uint32_t rr, uint32_t mode, uint32_t scramble,
                       uint32_t px, uint32_t py, uint64_t pass, double *L_out, double *log, uint32_t cap)
{
    or_opts op = make_opts(max_depth, rr, mode, scramble);
    g_log = log; g_log_n = 0; g_log_cap = cap;
    uint32_t nr = 0;
    uint64_t i = or_pixel_index(s->W, s->H, px, py, pass);
    v3 L = trace_path(s, &op, i, px, py, &nr, NULL, NULL);
    g_log = NULL;
    L_out[0] = L.x; L_out[1] = L.y; L_out[2] = L.z;
    return g_log_n;
}

/* ---------------------------------------------- pieces exposed for pins */

/* the guide's mixture (after the FP16 storage step) at n vertices: x, wo
 * (3 n each); out: 8 weights, 8 x (mu xyz, kappa) per row (40 values) */
void or_guide_mix(const or_scene *s, const double *x, const double *wo, uint32_t n, double *out)
{
    for (uint32_t r = 0; r < n; ++r) {
        gmix m;
        guide_mixture(s, V3(x[3 * r], x[3 * r + 1], x[3 * r + 2]), V3(wo[3 * r], wo[3 * r + 1], wo[3 * r + 2]),
                      &m);
        double *o = out + 40 * (size_t)r;
        for (int k = 0; k < G_LOBES; ++k) {
            o[k] = m.w[k];
            o[8 + 4 * k] = m.mu[k].x;
            o[9 + 4 * k] = m.mu[k].y;
            o[10 + 4 * k] = m.mu[k].z;
            o[11 + 4 * k] = m.kappa[k];
        }
    }
}

/* the guide's features and network outputs at n vertices (32 and 40 per row) */
void or_guide_forward(const or_scene *s, const double *x, const double *wo, uint32_t n, double *feat, double *out)
{
    for (uint32_t r = 0; r < n; ++r) {
        double f[32], o[40];
        guide_features(s, V3(x[3 * r], x[3 * r + 1], x[3 * r + 2]), V3(wo[3 * r], wo[3 * r + 1], wo[3 * r + 2]), f);
        guide_forward(s, f, o);
        if (feat) memcpy(feat + 32 * (size_t)r, f, sizeof f);
        if (out) memcpy(out + 40 * (size_t)r, o, sizeof o);
    }
}

/* density and samples of n explicit mixtures (rows of 40 as or_guide_mix
 * writes them): pdf[r] at dirs[3r..], sample[3r..] from u[3r..] (lobe,
 * cosine, azimuth numbers) */
void or_guide_mix_eval(const double *mix, const double *dirs, const double *u, uint32_t n, double *pdf,
                       double *sample)
{
    for (uint32_t r = 0; r < n; ++r) {
        const double *o = mix + 40 * (size_t)r;
        gmix m;
        for (int k = 0; k < G_LOBES; ++k) {
            m.w[k] = o[k];
            m.mu[k] = V3(o[8 + 4 * k], o[9 + 4 * k], o[10 + 4 * k]);
            m.kappa[k] = o[11 + 4 * k];
        }
        if (pdf) pdf[r] = gmix_pdf(&m, V3(dirs[3 * r], dirs[3 * r + 1], dirs[3 * r + 2]));
        if (sample) {
            v3 w = gmix_sample(&m, u[3 * r], u[3 * r + 1], u[3 * r + 2]);
            sample[3 * r] = w.x;
            sample[3 * r + 1] = w.y;
            sample[3 * r + 2] = w.z;
        }
    }
}

uint32_t or_rec_hash(uint64_t idx, uint32_t v) { return rec_hash(idx, v); }

/* The light tree's tables: node count; with non-NULL arrays, per node the
 * centre and radius (c4), region fluxes (f6), first child (-1 leaf), first
 * and count of its emitters in leaf order; per leaf-order position the
 * emitter and its cumulative 24-bit weight within its leaf. */
uint32_t or_light_tree(const or_scene *s, float *c4, float *f6, int32_t *left, uint32_t *first,
                       uint32_t *count, uint32_t *emit, uint32_t *w)
{
    if (!s->ne) return 0;
    uint32_t nn = s->lt_nn;
    if (c4) memcpy(c4, s->lt_c, sizeof(float) * 4 * nn);
    if (f6) memcpy(f6, s->lt_f, sizeof(float) * 6 * nn);
    if (left) memcpy(left, s->lt_left, sizeof(int32_t) * nn);
    if (first) memcpy(first, s->lt_first, sizeof(uint32_t) * nn);
    if (count) memcpy(count, s->lt_count, sizeof(uint32_t) * nn);
    if (emit) memcpy(emit, s->lt_emit, sizeof(uint32_t) * s->ne);
    if (w) memcpy(w, s->lt_w, sizeof(uint32_t) * s->ne);
    return nn;
}

/* n queries at FP32 points x[3n] and normals nrm[3n] with 63-bit samples
 * S[n]: chosen emitter and its interval size (probability times 2^63) */
void or_light_tree_sample(const or_scene *s, const uint64_t *S, const float *x, const float *nrm, uint32_t n,
                          uint32_t *e_out, uint64_t *size_out)
{
    for (uint32_t k = 0; k < n; ++k) e_out[k] = lt_sample(s, S[k], x + 3 * k, nrm + 3 * k, size_out + k);
}

/* interval size of every emitter (ne values) seen from one point */
void or_light_tree_sizes(const or_scene *s, const float *x, const float *nrm, uint64_t *size_out)
{
    for (uint32_t e = 0; e < s->ne; ++e) size_out[e] = lt_size_of(s, e, x, nrm);
}

/* The environment pyramid's tables: *m finest level (0: none), *top levels
 * weighted per normal bin, *root; q (4 per node of levels 0..m-1) and oq
 * (per bin: root, 0, 0, 0, then 4 per node of levels 0..top-1) if not NULL. */
void or_env_pyramid(const or_scene *s, uint32_t *m, uint32_t *top, uint32_t *root, uint32_t *q, uint32_t *oq)
{
    *m = s->ep_m;
    *top = s->ep_top;
    *root = s->ep_root;
    if (!s->ep_m) return;
    if (q) memcpy(q, s->ep_q, sizeof(uint32_t) * 4 * ep_nodes_above(s->ep_m));
    if (oq) memcpy(oq, s->ep_oq, sizeof(uint32_t) * (size_t)EP_K * EP_K * 4 * (1 + ep_nodes_above(s->ep_top)));
}

/* n descents: bin[k] (-1 unoriented), samples u[k] (columns), v[k] (rows);
 * steer != 0 follows texel (row[k], col[k]) instead. Out: row, col and the
 * final intervals ru, su, rv, sv (4 per query). */
void or_env_descend(const or_scene *s, const int32_t *bin, const uint32_t *u, const uint32_t *v, int steer,
                    uint32_t n, uint32_t *row, uint32_t *col, uint64_t *iv)
{
    for (uint32_t k = 0; k < n; ++k)
        ep_descend(s, bin[k], u[k], v[k], steer, row + k, col + k, iv + 4 * k, iv + 4 * k + 1, iv + 4 * k + 2,
                   iv + 4 * k + 3);
}

uint32_t or_env_bin(const float *n) { return ep_bin(n); }

/* the node estimate and the left-child probability, for pins */
float or_light_tree_estimate(const or_scene *s, uint32_t node, const float *x, const float *nrm)
{
    return lt_estimate(s, node, x, nrm);
}
uint32_t or_light_tree_left_q(const or_scene *s, uint32_t node, const float *x, const float *nrm)
{
    return s->lt_left[node] >= 0 ? lt_left_q(s, node, x, nrm) : 0;
}

void or_camera_ray(const or_scene *s, double fx, double fy, double *o, double *d)
{
    double sx = (2.0 * fx / s->W - 1.0) * s->tan_half * s->aspect;
    double sy = (1.0 - 2.0 * fy / s->H) * s->tan_half;
    v3 dd = normalize(add(s->fwd, add(mul(s->right, sx), mul(s->up, sy))));
    o[0] = s->eye.x; o[1] = s->eye.y; o[2] = s->eye.z;
    d[0] = dd.x; d[1] = dd.y; d[2] = dd.z;
}

/* f (rgb) and pdf of material m for unit n, wo, wi */
void or_bsdf(const or_scene *s, uint32_t m, const double *n, const double *wo, const double *wi,
             double *f, double *pdf)
{
    v3 ff;
    bsdf_eval(s, m, V3(n[0], n[1], n[2]), V3(wo[0], wo[1], wo[2]), V3(wi[0], wi[1], wi[2]), &ff, pdf);
    f[0] = ff.x; f[1] = ff.y; f[2] = ff.z;
}

int or_bsdf_sample(const or_scene *s, uint32_t m, const double *n, const double *wo, double u3,
                   double u4, double u5, double *wi)
{
    v3 w;
    int ok = bsdf_sample(s, m, V3(n[0], n[1], n[2]), V3(wo[0], wo[1], wo[2]), u3, u4, u5, &w);
    wi[0] = w.x; wi[1] = w.y; wi[2] = w.z;
    return ok;
}

double or_env_lookup(const or_scene *s, const double *w, double *rgb)
{
    double pdf;
    v3 L = env_lookup(s, V3(w[0], w[1], w[2]), &pdf);
    rgb[0] = L.x; rgb[1] = L.y; rgb[2] = L.z;
    return pdf;
}

double or_ggx_D(double cos_h, double alpha) { return ggx_D(cos_h, alpha * alpha); }

void or_bsdf_batch(const or_scene *s, uint32_t m, const double *n, const double *wo,
                   const double *wi, uint32_t cnt, double *f, double *pdf)
{
    for (uint32_t q = 0; q < cnt; ++q) or_bsdf(s, m, n, wo, wi + 3 * (size_t)q, f + 3 * (size_t)q, pdf + q);
}

void or_bsdf_sample_batch(const or_scene *s, uint32_t m, const double *n, const double *wo,
                          const double *u, uint32_t cnt, double *wi, int32_t *ok)
{
    for (uint32_t q = 0; q < cnt; ++q)
        ok[q] = or_bsdf_sample(s, m, n, wo, u[3 * (size_t)q], u[3 * (size_t)q + 1],
                               u[3 * (size_t)q + 2], wi + 3 * (size_t)q);
}
