// Host-only checks of the graph build (problem images, union plans, workspace
// layout) and of the serving arena's range allocator, built with a plain C++
// compiler under AddressSanitizer / UndefinedBehaviorSanitizer by
// tests/test_host_sanitized.py.  No GPU is touched: the kernel launchers the
// host driver references are stubs that abort if called.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "gba_host.hip"
#include "gba_range.h"

namespace gba {
#define GBA_STUB(name, ...)                                        \
    hipError_t name(__VA_ARGS__) {                                 \
        std::fprintf(stderr, "unexpected launch: %s\n", #name);    \
        std::abort();                                              \
    }
GBA_STUB(launch_linearize, const DeviceGraph&, hipStream_t, const RawOut*, bool)
GBA_STUB(launch_assemble, const DeviceGraph&, hipStream_t)
GBA_STUB(launch_cost, const DeviceGraph&, hipStream_t, const double*, const double*)
GBA_STUB(launch_cost_finish, const DeviceGraph&, hipStream_t)
GBA_STUB(launch_damp, const DeviceGraph&, hipStream_t, double, double)
GBA_STUB(launch_precond, const DeviceGraph&, hipStream_t, double, double, int, int)
GBA_STUB(launch_rhs, const DeviceGraph&, hipStream_t)
GBA_STUB(launch_pcg_init, const DeviceGraph&, hipStream_t, double, int)
GBA_STUB(launch_pcg_iter, const DeviceGraph&, hipStream_t, double, double, int, double, hipEvent_t,
         hipEvent_t)
GBA_STUB(launch_matvec, const DeviceGraph&, hipStream_t, int, double)
GBA_STUB(launch_backsub, const DeviceGraph&, hipStream_t)
GBA_STUB(launch_finish, const DeviceGraph&, hipStream_t)
GBA_STUB(launch_commit, const DeviceGraph&, hipStream_t)
bool precond_forms_rhs(const DeviceGraph&, int) { return false; }
}  // namespace gba

using namespace gba;

static int g_fail = 0;
#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++g_fail;                                                              \
        }                                                                          \
    } while (0)

// ------------------------------------------------------------ range allocator
// Reference model: a byte map of the arena.
struct ByteMap {
    std::vector<char> used;
    explicit ByteMap(size_t n) : used(n, 0) {}
    bool first_fit(size_t n, size_t& off) const {
        size_t run = 0;
        for (size_t k = 0; k < used.size(); ++k) {
            run = used[k] ? 0 : run + 1;
            if (run == n) {
                off = k + 1 - n;
                return true;
            }
        }
        return n == 0 ? (off = 0, true) : false;
    }
    bool last_fit(size_t n, size_t& off) const {
        size_t run = 0;
        for (size_t k = used.size(); k-- > 0;) {
            run = used[k] ? 0 : run + 1;
            // the end of the highest free range that holds n bytes
            if (run >= n && (k == 0 || used[k - 1])) {
                off = k + run - n;
                return true;
            }
        }
        return false;
    }
    void set(size_t off, size_t n, char v) {
        for (size_t k = off; k < off + n; ++k) used[k] = v;
    }
};

static void check_range_alloc_against_byte_map() {
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 200; ++trial) {
        const size_t N = 64 + rng() % 512;
        RangeAlloc ra;
        ra.reset(N);
        ByteMap bm(N);
        std::vector<std::pair<size_t, size_t>> live;
        for (int op = 0; op < 200; ++op) {
            const int kind = (int)(rng() % 3);
            if (kind < 2) {
                const size_t n = 1 + rng() % 40;
                size_t o1 = 0, o2 = 0;
                const bool a = kind == 0 ? ra.alloc_low(n, o1) : ra.alloc_high(n, o1);
                const bool b = kind == 0 ? bm.first_fit(n, o2) : bm.last_fit(n, o2);
                CHECK(a == b);
                if (a && b) {
                    CHECK(o1 == o2);
                    bm.set(o1, n, 1);
                    live.push_back({o1, n});
                }
            } else if (!live.empty()) {
                const size_t k = rng() % live.size();
                ra.release(live[k].first, live[k].second);
                bm.set(live[k].first, live[k].second, 0);
                live.erase(live.begin() + (long)k);
            }
            size_t fb = 0;
            for (char c : bm.used) fb += c ? 0 : 1;
            CHECK(ra.free_bytes() == fb);
        }
    }
}

// The admission check must find the offset the real sequence then gets: the
// image first-fit while the batch workspace is still held, the workspace
// released and the grown one placed from the top only afterwards.
static void check_admission_order() {
    // the case that once diverged: a gap below the workspace too small for the
    // image; releasing the workspace first would have placed the image inside
    // the old workspace range, which the real allocation cannot use yet
    {
        RangeAlloc ra;
        ra.reset(1000);
        size_t img0 = 0, gap = 0, un = 0;
        CHECK(ra.alloc_low(600, img0));      // a resident image [0, 600)
        CHECK(ra.alloc_high(300, un));       // the workspace [700, 1000)
        CHECK(un == 700);
        size_t off = 0;
        // a 150-byte image does not fit in the 100-byte gap [600, 700)
        CHECK(!simulate_admission(ra, true, un, 300, 150, 200, off));
        // a 80-byte image fits the gap, and a grown workspace of 300 still fits
        // above it once the old workspace is released
        CHECK(simulate_admission(ra, true, un, 300, 80, 300, off));
        size_t real = 0;
        CHECK(ra.alloc_low(80, real));
        CHECK(real == off);
        ra.release(un, 300);
        CHECK(ra.alloc_high(300, gap));
        (void)gap;
    }
    // random arenas: whenever the check admits, the real sequence succeeds at
    // the same image offset
    std::mt19937_64 rng(11);
    for (int trial = 0; trial < 2000; ++trial) {
        RangeAlloc ra;
        const size_t N = 256 + rng() % 4096;
        ra.reset(N);
        std::vector<std::pair<size_t, size_t>> imgs;
        for (int k = 0; k < (int)(rng() % 12); ++k) {
            size_t o = 0, n = 1 + rng() % (N / 8);
            if (ra.alloc_low(n, o)) imgs.push_back({o, n});
        }
        for (size_t k = 0; k < imgs.size(); ++k)
            if (rng() % 3 == 0) ra.release(imgs[k].first, imgs[k].second);
        bool have_union = rng() % 4 != 0;
        size_t un = 0, ub = 1 + rng() % (N / 3);
        if (have_union && !ra.alloc_high(ub, un)) have_union = false;
        const size_t img = 1 + rng() % (N / 6), grown = 1 + rng() % (N / 2);
        size_t off = 0;
        if (simulate_admission(ra, have_union, un, ub, img, grown, off)) {
            RangeAlloc real = ra;
            size_t o = 0, u2 = 0;
            CHECK(real.alloc_low(img, o));
            CHECK(o == off);
            if (have_union) real.release(un, ub);
            CHECK(real.alloc_high(grown, u2));
            CHECK(u2 >= o + img || u2 + grown <= o);   // disjoint
        }
    }
}

// ------------------------------------------------------- images and plans
static HostProblem random_problem(std::mt19937_64& rng, int nc, int np, bool info, bool long_tracks) {
    HostProblem h;
    h.cam_fixed.assign(nc, 0);
    h.pt_fixed.assign(np, 0);
    h.cam_params.assign(9 * (size_t)nc, 0.5);
    h.pt_params.assign(3 * (size_t)np, -1.0);
    h.cam_init = h.cam_params;
    h.pt_init = h.pt_params;
    for (int j = 0; j < np; ++j) {
        int L = 2 + (int)(rng() % 5);
        if (long_tracks && rng() % 20 == 0) L = 65 + (int)(rng() % 80);
        L = std::min(L, nc);
        std::set<int> cams;
        while ((int)cams.size() < L) cams.insert((int)(rng() % nc));
        for (int i : cams) {
            h.e_cam.push_back(i);
            h.e_pt.push_back(j);
            h.e_uv.push_back(1.0);
            h.e_uv.push_back(-2.0);
            h.e_active.push_back(rng() % 17 ? 1 : 0);
            if (info) {
                h.e_info.push_back(2.0);
                h.e_info.push_back(0.3);
                h.e_info.push_back(1.5);
            }
        }
    }
    // shuffle the edges (the build sorts them)
    const size_t ne = h.e_cam.size();
    std::vector<size_t> perm(ne);
    for (size_t k = 0; k < ne; ++k) perm[k] = k;
    std::shuffle(perm.begin(), perm.end(), rng);
    HostProblem s = h;
    for (size_t k = 0; k < ne; ++k) {
        const size_t e = perm[k];
        s.e_cam[k] = h.e_cam[e];
        s.e_pt[k] = h.e_pt[e];
        s.e_uv[2 * k] = h.e_uv[2 * e];
        s.e_uv[2 * k + 1] = h.e_uv[2 * e + 1];
        s.e_active[k] = h.e_active[e];
        if (info)
            for (int c = 0; c < 3; ++c) s.e_info[3 * k + c] = h.e_info[3 * e + c];
    }
    return s;
}

static void check_image(const HostProblem& h, const HostImage& im) {
    const int ne = im.n.ne;
    int active = 0;
    for (unsigned char a : h.e_active) active += a ? 1 : 0;
    CHECK(ne == active);
    // point-major order, pm_edge a permutation of the active edges
    std::vector<char> seen(h.n_edges(), 0);
    for (int q = 0; q < ne; ++q) {
        const int e = im.pm_edge[q];
        CHECK(e >= 0 && e < h.n_edges() && h.e_active[e] && !seen[e]);
        seen[e] = 1;
        CHECK(im.e_cam[q] == h.e_cam[e] && im.e_pt[q] == h.e_pt[e]);
        if (q > 0)
            CHECK(im.e_pt[q - 1] < im.e_pt[q] ||
                  (im.e_pt[q - 1] == im.e_pt[q] && im.e_cam[q - 1] <= im.e_cam[q]));
    }
    // tiles: contiguous, whole points, <= 64 edges unless one long point
    CHECK(im.tile_off.front() == 0 && im.tile_off.back() == ne);
    for (int t = 0; t < im.n.n_tiles; ++t) {
        const int a = im.tile_off[t], b = im.tile_off[t + 1];
        CHECK(b > a);
        if (b - a > kTileEdges) CHECK(im.e_pt[a] == im.e_pt[b - 1]);
        if (a > 0) CHECK(im.e_pt[a - 1] != im.e_pt[a]);
    }
    // camera-major runs and chunks
    CHECK(im.cm_run_off.back() == ne);
    for (int c = 0; c < im.n.n_chunks; ++c) {
        const int r0 = im.chunk_run_off[c], r1 = im.chunk_run_off[c + 1];
        CHECK(r1 > r0 && r1 - r0 <= kChunkRuns);
    }
    for (int i = 0; i < im.n.nc; ++i) CHECK(im.cam_chunk_off[i] <= im.cam_chunk_off[i + 1]);
    long long cm_sum = 0;
    for (int q = 0; q < ne; ++q) cm_sum += im.cm_pt[q];
    long long pm_sum = 0;
    for (int q = 0; q < ne; ++q) pm_sum += im.e_pt[q];
    CHECK(cm_sum == pm_sum);
    if (h.e_info.empty()) CHECK(im.sinfo.empty());
}

static void check_decomp(const HostDecomp& d, const std::vector<int>& off, bool aligned, int per) {
    const int P = (int)off.size() - 1;
    CHECK((int)d.prob_blk.size() == P + 1);
    for (int p = 0; p < P; ++p) {
        int expect = off[p];
        for (int b = d.prob_blk[p]; b < d.prob_blk[p + 1]; ++b) {
            CHECK(d.blk[3 * b + 2] == p);
            CHECK(d.blk[3 * b] == expect);
            CHECK(d.blk[3 * b + 1] > d.blk[3 * b] && d.blk[3 * b + 1] - d.blk[3 * b] <= per);
            if (aligned) CHECK((d.blk[3 * b] - off[p]) % per == 0);
            expect = d.blk[3 * b + 1];
        }
        CHECK(expect == off[p + 1] || (d.prob_blk[p] == d.prob_blk[p + 1] && off[p] == off[p + 1]));
    }
}

static void check_plans() {
    std::mt19937_64 rng(3);
    for (int trial = 0; trial < 30; ++trial) {
        const int P = 1 + (int)(rng() % 6);
        std::vector<HostProblem> probs;
        std::vector<HostImage> imgs(P);
        std::vector<const ImageCounts*> counts;
        for (int p = 0; p < P; ++p) {
            const int nc = 2 + (int)(rng() % 40), np = 1 + (int)(rng() % 400);
            probs.push_back(random_problem(rng, nc, np, rng() % 2 == 0, rng() % 3 == 0));
        }
        for (int p = 0; p < P; ++p) {
            std::string msg;
            CHECK(make_image(probs[p], imgs[p], msg) == GBA_OK);
            check_image(probs[p], imgs[p]);
            counts.push_back(&imgs[p].n);
        }
        for (int det = 0; det < 2; ++det) {
            Tuning tune;
            tune.tiles_per_block = 1 + (int)(rng() % 20);
            tune.edges_per_block = 64 + (int)(rng() % 300);
            tune.pts_per_block = 32 + (int)(rng() % 300);
            tune.deterministic = det;
            DeviceInfo dev;
            dev.max_lds = 160 * 1024;
            UnionPlan u;
            std::string msg;
            CHECK(plan_union(counts, tune, dev, GBA_FP64, u, msg) == GBA_OK);
            CHECK(u.cam_pass == (det == 1));
            check_decomp(u.pp, u.tile_off, false, tune.tiles_per_block);
            std::vector<int> comp(P + 1);
            for (int p = 0; p <= P; ++p) comp[p] = 9 * u.cam_off[p];
            check_decomp(u.red, comp, true, kRedComps);
            check_decomp(u.cam, u.cam_off, false, kCamsPerBlock);
            check_decomp(u.edges, u.edge_off, false, tune.edges_per_block);
            check_decomp(u.pts, u.pt_off, false, tune.pts_per_block);
            // workspace arrays: 256-byte aligned, inside the arena, disjoint
            for (int prec = 0; prec < 3; ++prec) {
                const size_t bytes = layout_union(u, prec, nullptr, nullptr);
                char* base = (char*)(uintptr_t)0x10000000;   // addresses only, never dereferenced
                DeviceGraph d{};
                CHECK(layout_union(u, prec, base, &d) == bytes);
                const void* arr[] = {d.tile_off, d.e_cam, d.e_pt, d.obs, d.cm_run_off, d.cm_pt,
                                     d.cm_obs, d.jst, d.jst_cm, d.hpp, d.hpp_inv, d.minv,
                                     d.v_x, d.v_z, d.cam_partial, d.chunk_partial};
                std::set<uintptr_t> addrs;
                for (const void* a : arr) {
                    const uintptr_t v = (uintptr_t)a;
                    CHECK(v >= (uintptr_t)base && v < (uintptr_t)base + bytes);
                    CHECK(v % 256 == 0);
                    CHECK(addrs.insert(v).second);
                }
            }
        }
        // an LDS-only plan with the fixed-order flag is refused
        Tuning bad;
        bad.accumulation = GBA_ACC_LDS;
        bad.deterministic = 1;
        UnionPlan u;
        std::string msg;
        DeviceInfo dev;
        dev.max_lds = 160 * 1024;
        CHECK(plan_union(counts, bad, dev, GBA_FP64, u, msg) == GBA_ERR_INVALID_ARG);
    }
    // a non positive-definite information matrix is refused by the build
    std::mt19937_64 r2(5);
    HostProblem h = random_problem(r2, 4, 10, true, false);
    h.e_info[0] = -1.0;
    HostImage im;
    std::string msg;
    CHECK(make_image(h, im, msg) == GBA_ERR_INVALID_ARG);
}

int main() {
    check_range_alloc_against_byte_map();
    check_admission_order();
    check_plans();
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
