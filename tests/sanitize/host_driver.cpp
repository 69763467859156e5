// Runs the library's host side (scene ingest, light tables, light tree,
// environment CDFs and pyramid, binned-SAH BVH and its 4-wide collapse,
// workspace sizing, the host-table hooks, argument and call-order checks)
// under AddressSanitizer and UndefinedBehaviorSanitizer on a host-only
// context (device -1). Reads scenes written by the test (same format as the
// oracle's driver). Exit code 0 when every call behaves as documented.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "qpt.h"

#define CHECK(x)                                                            \
    do {                                                                    \
        if (!(x)) {                                                         \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__); \
            std::exit(3);                                                   \
        }                                                                   \
    } while (0)

template <class T> static std::vector<T> slurp(FILE *f, size_t n)
{
    std::vector<T> v(n);
    if (n && std::fread(v.data(), sizeof(T), n, f) != n) {
        std::fprintf(stderr, "short read\n");
        std::exit(2);
    }
    return v;
}

static void run_scene(const char *path)
{
    FILE *f = std::fopen(path, "rb");
    CHECK(f);
    auto hdr = slurp<uint32_t>(f, 8);
    const uint32_t nv = hdr[0], nt = hdr[1], nm = hdr[2], ew = hdr[3], eh = hdr[4], W = hdr[5], H = hdr[6];
    auto pos = slurp<float>(f, 3 * (size_t)nv);
    auto idx = slurp<uint32_t>(f, 3 * (size_t)nt);
    auto tm = slurp<uint32_t>(f, nt);
    auto alb = slurp<float>(f, 3 * (size_t)nm);
    auto rough = slurp<float>(f, nm);
    auto emis = slurp<float>(f, 3 * (size_t)nm);
    auto flags = slurp<uint32_t>(f, nm);
    auto env = slurp<float>(f, 3 * (size_t)ew * eh);
    auto cam = slurp<double>(f, 10);
    std::fclose(f);
    std::vector<qpt_material> mats(nm);
    for (uint32_t m = 0; m < nm; ++m) {
        for (int c = 0; c < 3; ++c) {
            mats[m].albedo[c] = alb[3 * m + c];
            mats[m].emission[c] = emis[3 * m + c];
        }
        mats[m].roughness = rough[m];
        mats[m].flags = flags[m];
    }
    qpt_scene_desc d{};
    d.num_vertices = nv;
    d.positions = pos.data();
    d.num_triangles = nt;
    d.indices = idx.data();
    d.tri_material = tm.data();
    d.num_materials = nm;
    d.materials = mats.data();
    d.env_width = ew;
    d.env_height = eh;
    d.env_rgb = ew ? env.data() : nullptr;
    for (int c = 0; c < 3; ++c) {
        d.camera.eye[c] = (float)cam[c];
        d.camera.look[c] = (float)cam[3 + c];
        d.camera.up[c] = (float)cam[6 + c];
    }
    d.camera.vfov_deg = (float)cam[9];
    d.width = W;
    d.height = H;

    qpt_ctx *c = nullptr;
    CHECK(qpt_create(-1, nullptr, &c) == QPT_OK && c);
    // call order and argument checks
    CHECK(qpt_build_bvh(c, nullptr, nullptr) == QPT_E_STATE);
    size_t bytes = 0;
    CHECK(qpt_workspace_size(c, 0, &bytes) == QPT_E_STATE);
    qpt_scene_desc bad = d;
    bad.width = 0;
    CHECK(qpt_build_scene(c, &bad) == QPT_E_INVALID);
    std::vector<uint32_t> badidx(idx);
    badidx[0] = nv;  // out of range
    bad = d;
    bad.indices = badidx.data();
    CHECK(qpt_build_scene(c, &bad) == QPT_E_INVALID);
    CHECK(qpt_build_scene(c, &d) == QPT_OK);
    CHECK(qpt_bvh_scratch_size(c, &bytes) == QPT_OK);  // (sized by the device file: stubbed here)
    // the host tables
    uint32_t ne = 0;
    CHECK(qpt_debug_light_tables(c, nullptr, nullptr, nullptr, nullptr, &ne) == QPT_OK);
    std::vector<uint32_t> et(ne), al(ne);
    std::vector<double> prob(ne), pmf(ne);
    CHECK(qpt_debug_light_tables(c, et.data(), prob.data(), al.data(), pmf.data(), &ne) == QPT_OK);
    double psum = 0.0;
    for (double p : pmf) psum += p;
    // the realised pmf includes the choice against the environment (1/2 when both exist)
    CHECK(ne == 0 || std::fabs(psum - (ew ? 0.5 : 1.0)) < 1e-9);
    uint32_t nn = 0;
    CHECK(qpt_debug_light_tree(c, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, &nn) == QPT_OK);
    std::vector<float> sph(4 * (size_t)nn), fl(6 * (size_t)nn);
    std::vector<int32_t> left(nn);
    std::vector<uint32_t> first(nn), count(nn), emit(ne), weight(ne);
    CHECK(qpt_debug_light_tree(c, sph.data(), fl.data(), left.data(), first.data(), count.data(), emit.data(),
                               weight.data(), &nn) == QPT_OK);
    if (ew) {
        std::vector<uint32_t> rq(eh), cq((size_t)eh * ew);
        std::vector<float> tp((size_t)eh * ew);
        CHECK(qpt_debug_env_tables(c, rq.data(), cq.data(), tp.data()) == QPT_OK);
        uint32_t levels = 0, top = 0, root = 0;
        CHECK(qpt_debug_env_pyramid(c, &levels, &top, &root, nullptr, nullptr) == QPT_OK);
        if (levels) {
            size_t nodes = 0;
            for (uint32_t k = 0; k < levels; ++k) nodes += ((size_t)2 << k) << k;
            size_t tnodes = 0;
            for (uint32_t k = 0; k < top; ++k) tnodes += ((size_t)2 << k) << k;
            std::vector<uint32_t> q(4 * nodes), oq(256 * 4 * (1 + tnodes));
            CHECK(qpt_debug_env_pyramid(c, &levels, &top, &root, q.data(), oq.data()) == QPT_OK);
        }
    }
    // BVH: the GPU builder needs a device; the host builder at several leaf sizes
    qpt_bvh_opts o{};
    o.builder = 1;
    CHECK(qpt_build_bvh(c, &o, nullptr) == QPT_E_STATE);
    CHECK(qpt_build_bvh_noalloc(c, &o, nullptr) == QPT_E_STATE);
    o.builder = 7;
    CHECK(qpt_build_bvh(c, &o, nullptr) == QPT_E_INVALID);
    for (uint32_t leaf : {1u, 3u, 8u}) {
        o = qpt_bvh_opts{};
        o.max_leaf_size = leaf;
        o.sah_bins = leaf == 8 ? 64 : 0;
        qpt_bvh_stats st{};
        CHECK(qpt_build_bvh(c, &o, &st) == QPT_OK);
        CHECK(st.num_nodes >= 1 && std::isfinite(st.sah_cost));
        uint32_t nnodes = 0;
        CHECK(qpt_debug_bvh_nodes(c, nullptr, nullptr, &nnodes) == QPT_OK && nnodes == st.num_nodes);
        std::vector<float> nodes(32 * (size_t)nnodes);
        std::vector<uint32_t> order(nt);
        CHECK(qpt_debug_bvh_nodes(c, nodes.data(), order.data(), &nnodes) == QPT_OK);
        std::vector<char> seen(nt, 0);
        for (uint32_t t : order) {
            CHECK(t < nt && !seen[t]);
            seen[t] = 1;
        }
        CHECK(qpt_workspace_size(c, 0, &bytes) == QPT_OK && bytes > 0);
        CHECK(qpt_workspace_size(c, 1u << 16, &bytes) == QPT_OK && bytes > 0);
    }
    // device calls on a host-only context are refused
    CHECK(qpt_bind_workspace(c, nullptr, 0, 0) != QPT_OK);
    qpt_render_opts ro{};
    ro.max_depth = 4;
    CHECK(qpt_render_pass(c, 0, 1, &ro) == QPT_E_STATE);
    CHECK(qpt_set_streams(c, nullptr) == QPT_E_INVALID);
    std::printf("%s: %u triangles, %u emitters, %u light-tree nodes: ok\n", path, nt, ne, nn);
    qpt_destroy(c);
}

int main(int argc, char **argv)
{
    for (int k = 1; k < argc; ++k) run_scene(argv[k]);
    return 0;
}
