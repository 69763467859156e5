/* Runs the CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (host code only): reads a scene written by the test, builds it, renders a
 * few passes in every estimator option and frees it. Exit code 0 when all
 * calls return and the sums are finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct or_scene or_scene;
or_scene *or_scene_create(uint32_t nv, const float *pos, uint32_t nt, const uint32_t *idx, const uint32_t *tri_mat,
                          uint32_t nm, const float *albedo, const float *rough, const float *emission,
                          const uint32_t *flags, uint32_t ew, uint32_t eh, const float *env, const double *cam,
                          uint32_t W, uint32_t H, int build_bvh);
void or_scene_destroy(or_scene *s);
uint64_t or_render(const or_scene *s, uint32_t max_depth, uint32_t rr, uint32_t mode, uint32_t scramble,
                   const uint32_t *pix, uint32_t npix, uint64_t pass0, uint32_t npasses, double *sum, double *sumsq,
                   uint32_t *count, uint32_t nthreads);

static void *slurp(FILE *f, size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p || (bytes && fread(p, 1, bytes, f) != bytes)) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv)
{
    if (argc != 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    uint32_t h[8];  /* nv nt nm ew eh W H max_depth */
    if (fread(h, 4, 8, f) != 8) return 2;
    float *pos = slurp(f, 12ull * h[0]);
    uint32_t *idx = slurp(f, 12ull * h[1]);
    uint32_t *tm = slurp(f, 4ull * h[1]);
    float *alb = slurp(f, 12ull * h[2]);
    float *rough = slurp(f, 4ull * h[2]);
    float *emis = slurp(f, 12ull * h[2]);
    uint32_t *flags = slurp(f, 4ull * h[2]);
    float *env = h[3] ? slurp(f, 12ull * h[3] * h[4]) : NULL;
    double *cam = slurp(f, 8 * 10);
    fclose(f);
    or_scene *s = or_scene_create(h[0], pos, h[1], idx, tm, h[2], alb, rough, emis, flags, h[3], h[4], env, cam,
                                  h[5], h[6], 1);
    if (!s) return 3;
    const uint32_t npix = h[5] * h[6];
    double *sum = calloc(3ull * npix, 8), *sq = calloc(3ull * npix, 8);
    uint32_t *cnt = calloc(npix, 4);
    /* MIS / BSDF only / NEE only; light tree; pyramid (both); Gaussian filter */
    const uint32_t modes[] = {0, 1, 2, 0x100, 0x102, 0x200, 0x400, 0x402, 0x800, 0xd00};
    for (size_t k = 0; k < sizeof modes / sizeof modes[0]; ++k)
        or_render(s, h[7], 1, modes[k], 1, NULL, npix, 3 * k, 3, sum, sq, cnt, 4);
    int bad = 0;
    for (size_t q = 0; q < 3ull * npix; ++q) bad |= !isfinite(sum[q]);
    or_scene_destroy(s);
    free(sum);
    free(sq);
    free(cnt);
    free(pos);
    free(idx);
    free(tm);
    free(alb);
    free(rough);
    free(emis);
    free(flags);
    free(env);
    free(cam);
    return bad ? 4 : 0;
}
