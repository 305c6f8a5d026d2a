// Problem images, union planning, batch build and the per-problem
// Levenberg-Marquardt driver.
#include "gba_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace gba {

#define HIP_OR(msgv, call)                                                        \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            msgv = std::string(#call) + ": " + hipGetErrorString(e_);             \
            return GBA_ERR_HIP;                                                   \
        }                                                                         \
    } while (0)

bool HostProblem::any_free() const {
    for (unsigned char f : cam_fixed)
        if (!f) return true;
    for (unsigned char f : pt_fixed)
        if (!f) return true;
    return false;
}

void* Allocator::allocate(size_t bytes) const {
    if (alloc) return alloc(bytes, ctx);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void Allocator::release(void* p) const {
    if (!p) return;
    if (free_fn)
        free_fn(p, ctx);
    else
        (void)hipFree(p);
}

void Batch::drop_graphs() {
    for (auto& row : pcg_graph)
        for (auto& pg : row) {
            if (pg.exec) (void)hipGraphExecDestroy(pg.exec);
            pg = PcgGraph{};
        }
    pcg_warm = false;
}

void Batch::release() {
    drop_graphs();
    if (arena && owns_arena) {
        (void)hipStreamSynchronize(stream);
        allocator.release(arena);
    }
    arena = nullptr;
    arena_bytes = 0;
    P = 0;
}

gba_status Batch::ensure_mirrors(int n, std::string& msg) {
    if (n <= h_cap) return GBA_OK;
    if (h_scal) (void)hipHostFree(h_scal);
    if (h_pcg) (void)hipHostFree(h_pcg);
    if (h_lam) (void)hipHostFree(h_lam);
    if (h_accept) (void)hipHostFree(h_accept);
    h_scal = nullptr;
    h_pcg = nullptr;
    h_lam = nullptr;
    h_accept = nullptr;
    h_cap = 0;
    d_scal_host = nullptr;
    d_pcg_host = nullptr;
    // the per-trial and per-chunk results come back through mapped, coherent
    // pinned memory that the finishing kernels write (no copy per readback)
    const unsigned mapped = hipHostMallocMapped | hipHostMallocCoherent;
    if (hipHostMalloc((void**)&h_scal, sizeof(TrialScalars) * n, mapped) != hipSuccess ||
        hipHostMalloc((void**)&h_pcg, sizeof(PcgState) * n, mapped) != hipSuccess ||
        hipHostMalloc((void**)&h_lam, sizeof(double) * n, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h_accept, sizeof(int) * n, hipHostMallocDefault) != hipSuccess ||
        hipHostGetDevicePointer((void**)&d_scal_host, h_scal, 0) != hipSuccess ||
        hipHostGetDevicePointer((void**)&d_pcg_host, h_pcg, 0) != hipSuccess) {
        msg = "pinned host allocation failed";
        return GBA_ERR_HIP;
    }
    std::memset(h_scal, 0, sizeof(TrialScalars) * n);
    std::memset(h_pcg, 0, sizeof(PcgState) * n);
    h_cap = n;
    return GBA_OK;
}

Batch::~Batch() {
    release();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (h_scal) (void)hipHostFree(h_scal);
    if (h_pcg) (void)hipHostFree(h_pcg);
    if (h_lam) (void)hipHostFree(h_lam);
    if (h_accept) (void)hipHostFree(h_accept);
}

hipError_t Timers::init() {
    ev.resize(4 + 2 * 64);
    for (auto& e : ev) {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

Timers::~Timers() {
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------- images
gba_status make_image(const HostProblem& h, HostImage& img, std::string& msg) {
    img = HostImage{};
    const int nc = h.nc(), np = h.np();
    std::vector<int> act;
    act.reserve(h.n_edges());
    for (int e = 0; e < h.n_edges(); ++e)
        if (h.e_active[e]) act.push_back(e);
    const int ne = (int)act.size();
    const bool info = !h.e_info.empty();

    // point-major order: counting sort by point, camera order inside a point,
    // insertion order for ties
    std::vector<int> cnt(np + 1, 0);
    for (int e : act) cnt[h.e_pt[e] + 1]++;
    for (int j = 0; j < np; ++j) cnt[j + 1] += cnt[j];
    std::vector<int> pm(ne);
    {
        std::vector<int> pos(cnt.begin(), cnt.end() - 1);
        for (int e : act) pm[pos[h.e_pt[e]]++] = e;
        for (int j = 0; j < np; ++j)
            std::stable_sort(pm.begin() + cnt[j], pm.begin() + cnt[j + 1],
                             [&](int a, int c) { return h.e_cam[a] < h.e_cam[c]; });
    }
    img.e_cam.resize(ne);
    img.e_pt.resize(ne);
    img.obs.resize(2 * (size_t)ne);
    for (int q = 0; q < ne; ++q) {
        const int e = pm[q];
        img.e_cam[q] = h.e_cam[e];
        img.e_pt[q] = h.e_pt[e];
        img.obs[q] = h.e_uv[2 * (size_t)e];
        img.obs[(size_t)ne + q] = h.e_uv[2 * (size_t)e + 1];
    }
    // tiles of whole points (<= 64 edges) or one long point
    img.tile_off.push_back(0);
    {
        int cur = 0;
        for (int j = 0; j < np; ++j) {
            const int c = cnt[j + 1] - cnt[j];
            if (c == 0) continue;
            if (c > kTileEdges) {
                if (cur > 0) {
                    img.tile_off.push_back(img.tile_off.back() + cur);
                    cur = 0;
                }
                img.tile_off.push_back(img.tile_off.back() + c);
            } else {
                if (cur + c > kTileEdges) {
                    img.tile_off.push_back(img.tile_off.back() + cur);
                    cur = 0;
                }
                cur += c;
            }
        }
        if (cur > 0) img.tile_off.push_back(img.tile_off.back() + cur);
    }
    // camera-major order (point order inside a camera), runs of equal
    // (camera, point), chunks of at most kChunkRuns runs of one camera
    std::vector<int> ccount(nc + 1, 0);
    for (int q = 0; q < ne; ++q) ccount[img.e_cam[q] + 1]++;
    for (int i = 0; i < nc; ++i) ccount[i + 1] += ccount[i];
    std::vector<int> cm(ne);  // camera-major position -> point-major position
    {
        std::vector<int> pos(ccount.begin(), ccount.end() - 1);
        for (int q = 0; q < ne; ++q) cm[pos[img.e_cam[q]]++] = q;
    }
    img.cam_chunk_off.assign(nc + 1, 0);
    for (int i = 0; i < nc; ++i) {
        img.cam_chunk_off[i] = (int)img.chunk_cam.size();
        int runs_in_chunk = 0;
        for (int c = ccount[i]; c < ccount[i + 1]; ++c) {
            const bool new_run = c == ccount[i] || img.e_pt[cm[c]] != img.e_pt[cm[c - 1]];
            if (!new_run) continue;
            if (runs_in_chunk == 0) {
                img.chunk_run_off.push_back((int)img.cm_run_off.size());
                img.chunk_cam.push_back(i);
            }
            img.cm_run_off.push_back(c);
            if (++runs_in_chunk == kChunkRuns) runs_in_chunk = 0;
        }
    }
    img.cam_chunk_off[nc] = (int)img.chunk_cam.size();
    const int n_runs = (int)img.cm_run_off.size();
    img.cm_run_off.push_back(ne);
    img.chunk_run_off.push_back(n_runs);
    img.cm_pt.resize(ne);
    img.cm_obs.resize(2 * (size_t)ne);
    for (int c = 0; c < ne; ++c) {
        const int q = cm[c];
        img.cm_pt[c] = img.e_pt[q];
        img.cm_obs[c] = img.obs[q];
        img.cm_obs[(size_t)ne + c] = img.obs[(size_t)ne + q];
    }
    // square-root information factors (Omega = A^T A, A upper triangular)
    if (info) {
        img.sinfo.resize(3 * (size_t)ne);
        img.cm_sinfo.resize(3 * (size_t)ne);
        for (int q = 0; q < ne; ++q) {
            const int e = pm[q];
            const double o00 = h.e_info[3 * (size_t)e], o01 = h.e_info[3 * (size_t)e + 1],
                         o11 = h.e_info[3 * (size_t)e + 2];
            if (!(o00 > 0.0)) {
                msg = "information matrix not positive definite";
                return GBA_ERR_INVALID_ARG;
            }
            const double a00 = std::sqrt(o00), a01 = o01 / a00, d = o11 - a01 * a01;
            if (!(d > 0.0)) {
                msg = "information matrix not positive definite";
                return GBA_ERR_INVALID_ARG;
            }
            img.sinfo[q] = a00;
            img.sinfo[(size_t)ne + q] = a01;
            img.sinfo[2 * (size_t)ne + q] = std::sqrt(d);
        }
        for (int c = 0; c < ne; ++c)
            for (int k = 0; k < 3; ++k)
                img.cm_sinfo[(size_t)k * ne + c] = img.sinfo[(size_t)k * ne + cm[c]];
    }
    img.pm_edge = std::move(pm);
    img.n.nc = nc;
    img.n.np = np;
    img.n.ne = ne;
    img.n.n_tiles = (int)img.tile_off.size() - 1;
    img.n.n_runs = n_runs;
    img.n.n_chunks = (int)img.chunk_cam.size();
    img.n.info = info;
    return GBA_OK;
}

// ---------------------------------------------------------------- planning
namespace {

// Problem-aligned decomposition of item ranges [off[p], off[p+1]) into
// workgroups of at most `per_block` items, split evenly inside a problem.
HostDecomp make_decomp(const std::vector<int>& off, long long per_block, bool aligned = false) {
    HostDecomp d;
    const int P = (int)off.size() - 1;
    d.prob_blk.resize(P + 1);
    per_block = std::max<long long>(1, per_block);
    for (int p = 0; p < P; ++p) {
        d.prob_blk[p] = d.nblk();
        const long long n = (long long)off[p + 1] - off[p];
        if (n <= 0) continue;
        const long long nb = (n + per_block - 1) / per_block;
        for (long long q = 0; q < nb; ++q) {
            // even split, or full blocks from the problem's start (aligned)
            const long long b = aligned ? per_block * q : n * q / nb;
            const long long e = aligned ? std::min(n, per_block * (q + 1)) : n * (q + 1) / nb;
            d.blk.push_back((int)(off[p] + b));
            d.blk.push_back((int)(off[p] + e));
            d.blk.push_back(p);
        }
    }
    d.prob_blk[P] = d.nblk();
    return d;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Sequential layout of 256-byte aligned arrays; with a null base it only
// counts bytes.
struct Planner {
    char* base;
    size_t off = 0;
    explicit Planner(void* b) : base((char*)b) {}
    template <typename T>
    void add(T*& slot, size_t bytes) {
        if (base) slot = (T*)(base + off);
        off += align_up(bytes ? bytes : 1);
    }
};

}  // namespace

gba_status plan_union(const std::vector<const ImageCounts*>& probs, const Tuning& tune,
                      const DeviceInfo& dev, int precision, UnionPlan& u, std::string& msg) {
    u = UnionPlan{};
    const int P = (int)probs.size();
    if (P < 1 || P > kMaxProblems) {
        msg = "a batch holds 1.." + std::to_string(kMaxProblems) + " problems";
        return GBA_ERR_INVALID_ARG;
    }
    u.P = P;
    u.cam_off.assign(P + 1, 0);
    u.pt_off.assign(P + 1, 0);
    u.edge_off.assign(P + 1, 0);
    u.tile_off.assign(P + 1, 0);
    u.run_off.assign(P + 1, 0);
    u.chunk_off.assign(P + 1, 0);
    long long sc = 0, sp = 0, se = 0, st = 0, sr = 0, sk = 0;
    for (int p = 0; p < P; ++p) {
        const ImageCounts& n = *probs[p];
        sc += n.nc;
        sp += n.np;
        se += n.ne;
        st += n.n_tiles;
        sr += n.n_runs;
        sk += n.n_chunks;
        if (se > std::numeric_limits<int>::max() / 32 || sp > std::numeric_limits<int>::max() / 16 ||
            sc > std::numeric_limits<int>::max() / 64) {
            msg = "batch too large for 32-bit indexing";
            return GBA_ERR_UNSUPPORTED;
        }
        u.cam_off[p + 1] = (int)sc;
        u.pt_off[p + 1] = (int)sp;
        u.edge_off[p + 1] = (int)se;
        u.tile_off[p + 1] = (int)st;
        u.run_off[p + 1] = (int)sr;
        u.chunk_off[p + 1] = (int)sk;
        u.tot.info = u.tot.info || n.info;
        u.max_cams = std::max(u.max_cams, n.nc);
    }
    u.tot.nc = (int)sc;
    u.tot.np = (int)sp;
    u.tot.ne = (int)se;
    u.tot.n_tiles = (int)st;
    u.tot.n_runs = (int)sr;
    u.tot.n_chunks = (int)sk;
    // the LDS camera sums of the point passes are FP64 in every mode
    (void)precision;
    const size_t lds = 9 * (size_t)u.max_cams * sizeof(double);
    const bool fits = lds + 1024 <= dev.max_lds;
    if (tune.accumulation == GBA_ACC_LDS && tune.deterministic) {
        msg = "fixed-order sums need the camera-major pass, not LDS partials";
        return GBA_ERR_INVALID_ARG;
    }
    if (tune.accumulation == GBA_ACC_LDS && !fits) {
        msg = "the camera vector of one problem does not fit in LDS (" +
              std::to_string(u.max_cams) + " cameras)";
        return GBA_ERR_UNSUPPORTED;
    }
    // the LDS partials are combined by atomics in a varying order; the
    // camera-major pass sums every camera in a fixed order
    u.deterministic = tune.deterministic != 0;
    u.full = tune.solver == GBA_SOLVER_FULL;
    u.dynamic = u.full && tune.dynamic != 0;
    if (u.full && (u.deterministic || tune.accumulation == GBA_ACC_CAMERA_PASS || !fits)) {
        msg = "the full-Hessian PCG sums the camera side in LDS (at most " +
              std::to_string((dev.max_lds - 1024) / 72) + " cameras per problem, no fixed-order mode)";
        return GBA_ERR_UNSUPPORTED;
    }
    u.cam_pass = tune.accumulation == GBA_ACC_CAMERA_PASS || tune.accumulation == GBA_ACC_CAMERA_BLOCKS ||
                 !fits || u.deterministic;
    u.lds_pp = u.cam_pass ? 0 : (int)lds;
    // the camera-blocked product pass: one problem, stored Jacobians, sums
    // by LDS atomics (so not in the fixed-order mode)
    u.cam_blocks = u.cam_pass && P == 1 && !u.deterministic && !u.full && u.tot.ne > 0 &&
                   (tune.accumulation == GBA_ACC_CAMERA_BLOCKS ||
                    (tune.accumulation == GBA_ACC_AUTO && u.tot.nc > kCamBlock));
    if (u.cam_blocks) {
        u.bo_nblk = (u.tot.nc + kCamBlock - 1) / kCamBlock;
        u.bo_target = std::max(4096, (u.tot.ne + dev.n_cu - 1) / std::max(1, dev.n_cu));
        u.bo_chunk_cap = u.bo_nblk + u.tot.ne / u.bo_target + 1;
    }
    // automatic: one point-pass workgroup per CU (each flushes one LDS camera
    // partial; the flush grows with the workgroup count, and smaller
    // workgroups measured slower in both schemes)
    const long long tpb = tune.tiles_per_block > 0
                              ? tune.tiles_per_block
                              : std::max<long long>(16, (st + dev.n_cu - 1) / std::max(1, dev.n_cu));
    const long long epb = tune.edges_per_block > 0 ? tune.edges_per_block
                                                   : std::max<long long>(256, (se + 2047) / 2048);
    const long long ppb = tune.pts_per_block > 0 ? tune.pts_per_block
                                                 : std::max<long long>(256, (sp + 2047) / 2048);
    std::vector<int> comp(P + 1);
    for (int p = 0; p <= P; ++p) comp[p] = 9 * u.cam_off[p];
    u.pp = make_decomp(u.tile_off, tpb);
    u.red = make_decomp(comp, kRedComps, true);   // 16-byte aligned partial reads
    u.cam = make_decomp(u.cam_off, kCamsPerBlock);
    u.edges = make_decomp(u.edge_off, epb);
    u.pts = make_decomp(u.pt_off, ppb);
    u.part_off.assign(std::max(1, u.pp.nblk()), 0);
    long long part = 0;
    for (int p = 0; p < P && !u.cam_pass; ++p) {
        const int ncp = u.cam_off[p + 1] - u.cam_off[p];
        for (int q = u.pp.prob_blk[p]; q < u.pp.prob_blk[p + 1]; ++q) {
            // one partial vector per workgroup, a problem's consecutive and
            // each padded to 4 entries (k_reduce computes the addresses
            // from this layout and reads 16 bytes per lane)
            u.part_off[q] = (int)part;
            part += (9LL * ncp + 3) / 4 * 4;
        }
    }
    if (part > std::numeric_limits<int>::max()) {
        msg = "camera partial buffer too large";
        return GBA_ERR_UNSUPPORTED;
    }
    u.part_total = part;
    u.cam_prob.resize(sc);
    u.pt_prob.resize(sp);
    for (int p = 0; p < P; ++p) {
        for (int i = u.cam_off[p]; i < u.cam_off[p + 1]; ++i) u.cam_prob[i] = p;
        for (int j = u.pt_off[p]; j < u.pt_off[p + 1]; ++j) u.pt_prob[j] = p;
    }
    return GBA_OK;
}

size_t layout_union(const UnionPlan& u, int precision, void* base, DeviceGraph* dptr) {
    DeviceGraph tmp{};
    DeviceGraph& d = dptr ? *dptr : tmp;
    Planner L(dptr ? base : nullptr);
    const size_t NE = (size_t)u.tot.ne, NP = (size_t)u.tot.np, NC = (size_t)u.tot.nc;
    const int P = u.P;
    const size_t tsz = precision == GBA_FP64 ? 8 : 4;
    const size_t jsz = precision == GBA_FP64 ? 8 : (precision == GBA_MIXED_FP32 ? 4 : 2);
    auto decomp = [&](Decomp& dc, const HostDecomp& h) {
        L.add(dc.blk, sizeof(int) * std::max<size_t>(3, h.blk.size()));
        L.add(dc.prob_blk, sizeof(int) * h.prob_blk.size());
    };
    L.add(d.tile_off, sizeof(int) * (u.tot.n_tiles + 1));
    L.add(d.e_cam, sizeof(int) * NE);
    L.add(d.e_pt, sizeof(int) * NE);
    L.add(d.obs, sizeof(double) * 2 * NE);
    if (u.tot.info) L.add(d.sinfo, sizeof(double) * 3 * NE);
    L.add(d.cm_run_off, sizeof(int) * (u.tot.n_runs + 1));
    L.add(d.cm_pt, sizeof(int) * NE);
    L.add(d.cm_obs, sizeof(double) * 2 * NE);
    if (u.tot.info) L.add(d.cm_sinfo, sizeof(double) * 3 * NE);
    L.add(d.chunk_run_off, sizeof(int) * (u.tot.n_chunks + 1));
    L.add(d.chunk_cam, sizeof(int) * u.tot.n_chunks);
    L.add(d.cam_chunk_off, sizeof(int) * (NC + 1));
    L.add(d.cam_fixed, NC);
    L.add(d.pt_fixed, NP);
    L.add(d.cam_prob, sizeof(int) * NC);
    L.add(d.pt_prob, sizeof(int) * NP);
    L.add(d.prob_cam_off, sizeof(int) * (P + 1));
    L.add(d.lam, sizeof(double) * P);
    L.add(d.accept, sizeof(int) * P);
    L.add(d.pcg, sizeof(PcgState) * P);
    L.add(d.pcg_dec, sizeof(PcgState) * P);
    L.add(d.scal, sizeof(TrialScalars) * P);
    L.add(d.cam, sizeof(double) * 9 * NC);
    L.add(d.cam_c, sizeof(double) * 9 * NC);
    L.add(d.cam_init, sizeof(double) * 9 * NC);
    L.add(d.pt, sizeof(double) * 3 * NP);
    L.add(d.pt_c, sizeof(double) * 3 * NP);
    L.add(d.pt_init, sizeof(double) * 3 * NP);
    L.add(d.dpt, sizeof(double) * 3 * NP);
    const size_t NE64 = (NE + 63) / 64 * 64;   // the stored Jacobian pads to whole 64-edge groups
    if (!u.dynamic) L.add(d.jst, jsz * 24 * NE64);
    else if (dptr) d.jst = nullptr;
    L.add(d.rw, tsz * 2 * NE);
    L.add(d.hpp, tsz * 6 * NP);
    L.add(d.bp, tsz * 3 * NP);
    L.add(d.hcc, tsz * 45 * NC);
    L.add(d.bc, tsz * 9 * NC);
    L.add(d.hpp_inv, tsz * kHinvStride * NP);
    if (!u.dynamic) L.add(d.jst_cm, jsz * 24 * NE64);   // camera-major copy (preconditioner, two-pass products)
    else if (dptr) d.jst_cm = nullptr;
    if (u.cam_pass) L.add(d.zbuf, tsz * 4 * NP);
    if (u.cam_blocks) {
        const size_t cap = (size_t)u.bo_chunk_cap;
        L.add(d.bo_off, sizeof(int) * (cap + 1));
        L.add(d.bo_blk, sizeof(int) * cap);
        L.add(d.bo_blk_chunk, sizeof(int) * (u.bo_nblk + 1));
        L.add(d.bo_perm, sizeof(int) * NE);
        L.add(d.bo_pt, sizeof(int) * NE);
        L.add(d.bo_cam, sizeof(int) * NE);
        L.add(d.jst_bo, jsz * 24 * NE64);
        L.add(d.bo_partial, tsz * cap * kCamBlock * 9);
    } else if (dptr) {
        d.bo_off = d.bo_blk = d.bo_blk_chunk = d.bo_perm = d.bo_pt = d.bo_cam = nullptr;
        d.jst_bo = d.bo_partial = nullptr;
    }
    L.add(d.minv, tsz * 45 * NC);
    L.add(d.v_x, tsz * 9 * NC + 64);   // slack: 16-byte gathers (gather9); back-substitution
    L.add(d.v_r, tsz * 9 * NC);
    L.add(d.v_z, tsz * 9 * NC + 64);   // the product gathers z
    L.add(d.v_p, tsz * 9 * NC);
    L.add(d.v_q, tsz * 9 * NC);
    L.add(d.v_best, tsz * 9 * NC);
    decomp(d.dc_pp, u.pp);
    decomp(d.dc_red, u.red);
    decomp(d.dc_cam, u.cam);
    decomp(d.dc_edges, u.edges);
    decomp(d.dc_pts, u.pts);
    L.add(d.pp_part_off, sizeof(int) * u.part_off.size());
    L.add(d.cam_partial, sizeof(double) * std::max<long long>(1, u.part_total));
    L.add(d.pq_partial, sizeof(double) * std::max(1, u.red.nblk()));
    L.add(d.dot_partial, sizeof(double) * 2 * std::max(1, u.cam.nblk()));
    L.add(d.camupd_partial, sizeof(double) * 3 * std::max(1, u.cam.nblk()));
    L.add(d.chunk_partial, sizeof(double) * 54 * std::max(1, u.tot.n_chunks));
    L.add(d.red_partial, sizeof(double) * 4 * std::max(1, u.pp.nblk()));
    L.add(d.cost_partial, sizeof(double) * std::max(1, u.edges.nblk()));
    L.add(d.damp_partial, sizeof(double) * std::max(1, u.pts.nblk()));
    L.add(d.gbar, sizeof(unsigned int) * kGbarWords);
    L.add(d.red_count, sizeof(unsigned int) * u.P);
    if (u.full) {
        for (void** v : {&d.w_x, &d.w_r, &d.w_z, &d.w_p, &d.w_q, &d.w_best})
            L.add(*v, tsz * 3 * NP + 64);
        L.add(d.pdot_partial, sizeof(double) * 2 * std::max(1, u.pts.nblk()));
        L.add(d.ppq_partial, sizeof(double) * std::max(1, u.pp.nblk()));
    } else if (dptr) {
        d.w_x = d.w_r = d.w_z = d.w_p = d.w_q = d.w_best = nullptr;
        d.pdot_partial = d.ppq_partial = nullptr;
    }
    return L.off;
}

void set_union_scalars(Batch& b, int precision, int loss, double delta) {
    const UnionPlan& u = b.plan;
    DeviceGraph& d = b.dg;
    d.nc = u.tot.nc;
    d.np = u.tot.np;
    d.ne = u.tot.ne;
    d.n_tiles = u.tot.n_tiles;
    d.n_runs = u.tot.n_runs;
    d.n_chunks = u.tot.n_chunks;
    d.n_probs = u.P;
    d.has_info = u.tot.info ? 1 : 0;
    d.loss = loss;
    d.delta = delta;
    d.mode = precision;
    d.pcg_host = b.d_pcg_host;
    d.scal_host = b.d_scal_host;
    d.jac_bytes = precision == GBA_FP64 ? 8 : (precision == GBA_MIXED_FP32 ? 4 : 2);
    d.block_pp = kPointPassBlock;
    d.cam_pass = u.cam_pass ? 1 : 0;
    d.deterministic = u.deterministic ? 1 : 0;
    d.full = u.full ? 1 : 0;
    d.dynamic = u.dynamic ? 1 : 0;
    d.lds_pp = u.lds_pp;
    d.fuse_apply = !u.full && u.max_cams <= kFuseApplyCams ? 1 : 0;
    d.dc_pp.nblk = u.pp.nblk();
    d.dc_red.nblk = u.red.nblk();
    d.dc_cam.nblk = u.cam.nblk();
    d.dc_edges.nblk = u.edges.nblk();
    d.dc_pts.nblk = u.pts.nblk();
    b.P = u.P;
    b.precision = precision;
}

gba_status upload_plan(Batch& b, std::string& msg) {
    const UnionPlan& u = b.plan;
    const DeviceGraph& d = b.dg;
    hipStream_t s = b.stream;
    auto up = [&](const void* dst, const void* src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync((void*)dst, src, bytes, hipMemcpyHostToDevice, s);
    };
    auto up_decomp = [&](const Decomp& dc, const HostDecomp& h) -> hipError_t {
        hipError_t r = up(dc.blk, h.blk.data(), sizeof(int) * h.blk.size());
        if (r != hipSuccess) return r;
        return up(dc.prob_blk, h.prob_blk.data(), sizeof(int) * h.prob_blk.size());
    };
    HIP_OR(msg, up_decomp(d.dc_pp, u.pp));
    HIP_OR(msg, up_decomp(d.dc_red, u.red));
    HIP_OR(msg, up_decomp(d.dc_cam, u.cam));
    HIP_OR(msg, up_decomp(d.dc_edges, u.edges));
    HIP_OR(msg, up_decomp(d.dc_pts, u.pts));
    HIP_OR(msg, up(d.pp_part_off, u.part_off.data(), sizeof(int) * u.part_off.size()));
    HIP_OR(msg, up(d.cam_prob, u.cam_prob.data(), sizeof(int) * u.cam_prob.size()));
    HIP_OR(msg, up(d.pt_prob, u.pt_prob.data(), sizeof(int) * u.pt_prob.size()));
    HIP_OR(msg, up(d.prob_cam_off, u.cam_off.data(), sizeof(int) * u.cam_off.size()));
    return GBA_OK;
}

gba_status build_batch(const std::vector<const HostProblem*>& probs, int precision, int loss,
                       double delta, const DeviceInfo& dev, const Tuning& tune,
                       const Allocator& alloc, hipStream_t stream, Batch& b, std::string& msg) {
    b.release();
    b.stream = stream;
    b.allocator = alloc;
    b.owns_arena = true;
    const int P = (int)probs.size();
    std::vector<HostImage> imgs(P);
    std::vector<const ImageCounts*> counts(P);
    for (int p = 0; p < P; ++p) {
        gba_status st = make_image(*probs[p], imgs[p], msg);
        if (st != GBA_OK) return st;
        counts[p] = &imgs[p].n;
    }
    gba_status st = plan_union(counts, tune, dev, precision, b.plan, msg);
    if (st != GBA_OK) return st;
    if ((st = b.ensure_mirrors(P, msg)) != GBA_OK) return st;
    const UnionPlan& u = b.plan;
    const size_t bytes = layout_union(u, precision, nullptr, nullptr);
    void* arena = alloc.allocate(bytes);
    if (!arena) {
        msg = "device allocation of " + std::to_string(bytes) + " bytes failed";
        return GBA_ERR_OOM;
    }
    b.arena = arena;
    b.arena_bytes = bytes;
    b.dg = DeviceGraph{};
    b.blocks_zeroed = false;
    b.persistent_ok = -1;
    layout_union(u, precision, arena, &b.dg);
    set_union_scalars(b, precision, loss, delta);
    DeviceGraph& d = b.dg;

    // concatenate the images with offsets (host), then upload
    const size_t NE = u.tot.ne, NP = u.tot.np, NC = u.tot.nc;
    std::vector<int> e_cam(NE), e_pt(NE), cm_pt(NE), tile_off(u.tot.n_tiles + 1),
        run_off(u.tot.n_runs + 1), chunk_run_off(u.tot.n_chunks + 1), chunk_cam(u.tot.n_chunks),
        cam_chunk_off(NC + 1);
    std::vector<double> obs(2 * NE), cm_obs(2 * NE), sinfo, cm_sinfo;
    if (u.tot.info) {
        sinfo.resize(3 * NE);
        cm_sinfo.resize(3 * NE);
    }
    std::vector<unsigned char> cfix(NC), pfix(NP);
    std::vector<double> cams(9 * NC), cams0(9 * NC), pts(3 * NP), pts0(3 * NP);
    b.pm_edge.assign(P, {});
    for (int p = 0; p < P; ++p) {
        const HostImage& im = imgs[p];
        const HostProblem& h = *probs[p];
        const int eo = u.edge_off[p], co = u.cam_off[p], po = u.pt_off[p];
        const int ne = im.n.ne;
        for (int q = 0; q < ne; ++q) {
            e_cam[eo + q] = im.e_cam[q] + co;
            e_pt[eo + q] = im.e_pt[q] + po;
            cm_pt[eo + q] = im.cm_pt[q] + po;
            for (int k = 0; k < 2; ++k) {
                obs[k * NE + eo + q] = im.obs[(size_t)k * ne + q];
                cm_obs[k * NE + eo + q] = im.cm_obs[(size_t)k * ne + q];
            }
            if (u.tot.info)
                for (int k = 0; k < 3; ++k) {
                    const double id = k == 1 ? 0.0 : 1.0;
                    sinfo[k * NE + eo + q] = im.n.info ? im.sinfo[(size_t)k * ne + q] : id;
                    cm_sinfo[k * NE + eo + q] = im.n.info ? im.cm_sinfo[(size_t)k * ne + q] : id;
                }
        }
        for (int t = 0; t < im.n.n_tiles; ++t) tile_off[u.tile_off[p] + t] = im.tile_off[t] + eo;
        for (int r = 0; r < im.n.n_runs; ++r) run_off[u.run_off[p] + r] = im.cm_run_off[r] + eo;
        for (int c = 0; c < im.n.n_chunks; ++c) {
            chunk_run_off[u.chunk_off[p] + c] = im.chunk_run_off[c] + u.run_off[p];
            chunk_cam[u.chunk_off[p] + c] = im.chunk_cam[c] + co;
        }
        for (int i = 0; i < im.n.nc; ++i) cam_chunk_off[co + i] = im.cam_chunk_off[i] + u.chunk_off[p];
        std::copy(h.cam_fixed.begin(), h.cam_fixed.end(), cfix.begin() + co);
        std::copy(h.pt_fixed.begin(), h.pt_fixed.end(), pfix.begin() + po);
        std::copy(h.cam_params.begin(), h.cam_params.end(), cams.begin() + 9 * (size_t)co);
        std::copy(h.cam_init.begin(), h.cam_init.end(), cams0.begin() + 9 * (size_t)co);
        std::copy(h.pt_params.begin(), h.pt_params.end(), pts.begin() + 3 * (size_t)po);
        std::copy(h.pt_init.begin(), h.pt_init.end(), pts0.begin() + 3 * (size_t)po);
        b.pm_edge[p] = std::move(imgs[p].pm_edge);
    }
    tile_off[u.tot.n_tiles] = (int)NE;
    run_off[u.tot.n_runs] = (int)NE;
    chunk_run_off[u.tot.n_chunks] = u.tot.n_runs;
    cam_chunk_off[NC] = u.tot.n_chunks;
    std::vector<int> accept0(P, 0);
    auto up = [&](const void* dst, const void* src, size_t n) -> hipError_t {
        if (!n) return hipSuccess;
        return hipMemcpyAsync((void*)dst, src, n, hipMemcpyHostToDevice, stream);
    };
    HIP_OR(msg, up(d.tile_off, tile_off.data(), sizeof(int) * tile_off.size()));
    HIP_OR(msg, up(d.e_cam, e_cam.data(), sizeof(int) * NE));
    HIP_OR(msg, up(d.e_pt, e_pt.data(), sizeof(int) * NE));
    // the camera-blocked order: the point-major edges bucketed by camera
    // block (so point order inside a block), each block cut into chunks of
    // about bo_target edges
    std::vector<int> bo_off, bo_blk, bo_blk_chunk, bo_perm, bo_pt, bo_cam;
    d.bo_chunks = 0;
    d.bo_nblk = 0;
    if (u.cam_blocks) {
        const int nb = u.bo_nblk;
        std::vector<int> bstart(nb + 1, 0);
        for (size_t e = 0; e < NE; ++e) ++bstart[e_cam[e] / kCamBlock + 1];
        for (int b = 0; b < nb; ++b) bstart[b + 1] += bstart[b];
        bo_perm.resize(NE);
        bo_pt.resize(NE);
        bo_cam.resize(NE);
        {
            std::vector<int> at(bstart.begin(), bstart.end() - 1);
            for (size_t e = 0; e < NE; ++e) {
                const int q = at[e_cam[e] / kCamBlock]++;
                bo_perm[q] = (int)e;
                bo_pt[q] = e_pt[e];
                bo_cam[q] = e_cam[e];
            }
        }
        bo_blk_chunk.assign(nb + 1, 0);
        for (int b = 0; b < nb; ++b) {
            bo_blk_chunk[b] = (int)bo_blk.size();
            const long long n_b = bstart[b + 1] - bstart[b];
            const long long k = std::max(1LL, (n_b + u.bo_target - 1) / u.bo_target);
            for (long long c = 0; c < k && n_b > 0; ++c) {
                bo_off.push_back(bstart[b] + (int)(n_b * c / k));
                bo_blk.push_back(b);
            }
        }
        bo_blk_chunk[nb] = (int)bo_blk.size();
        bo_off.push_back((int)NE);
        if ((int)bo_blk.size() > u.bo_chunk_cap) {
            msg = "camera-blocked chunk count above its bound";
            return GBA_ERR_STATE;
        }
        d.bo_chunks = (int)bo_blk.size();
        d.bo_nblk = nb;
        HIP_OR(msg, up(d.bo_off, bo_off.data(), sizeof(int) * bo_off.size()));
        HIP_OR(msg, up(d.bo_blk, bo_blk.data(), sizeof(int) * bo_blk.size()));
        HIP_OR(msg, up(d.bo_blk_chunk, bo_blk_chunk.data(), sizeof(int) * bo_blk_chunk.size()));
        HIP_OR(msg, up(d.bo_perm, bo_perm.data(), sizeof(int) * NE));
        HIP_OR(msg, up(d.bo_pt, bo_pt.data(), sizeof(int) * NE));
        HIP_OR(msg, up(d.bo_cam, bo_cam.data(), sizeof(int) * NE));
    }
    HIP_OR(msg, up(d.obs, obs.data(), sizeof(double) * 2 * NE));
    if (u.tot.info) {
        HIP_OR(msg, up(d.sinfo, sinfo.data(), sizeof(double) * 3 * NE));
        HIP_OR(msg, up(d.cm_sinfo, cm_sinfo.data(), sizeof(double) * 3 * NE));
    }
    HIP_OR(msg, up(d.cm_run_off, run_off.data(), sizeof(int) * run_off.size()));
    HIP_OR(msg, up(d.cm_pt, cm_pt.data(), sizeof(int) * NE));
    HIP_OR(msg, up(d.cm_obs, cm_obs.data(), sizeof(double) * 2 * NE));
    HIP_OR(msg, up(d.chunk_run_off, chunk_run_off.data(), sizeof(int) * chunk_run_off.size()));
    HIP_OR(msg, up(d.chunk_cam, chunk_cam.data(), sizeof(int) * chunk_cam.size()));
    HIP_OR(msg, up(d.cam_chunk_off, cam_chunk_off.data(), sizeof(int) * cam_chunk_off.size()));
    HIP_OR(msg, up(d.cam_fixed, cfix.data(), NC));
    HIP_OR(msg, up(d.pt_fixed, pfix.data(), NP));
    HIP_OR(msg, up(d.accept, accept0.data(), sizeof(int) * P));
    HIP_OR(msg, up(d.cam, cams.data(), sizeof(double) * 9 * NC));
    HIP_OR(msg, up(d.cam_init, cams0.data(), sizeof(double) * 9 * NC));
    HIP_OR(msg, up(d.pt, pts.data(), sizeof(double) * 3 * NP));
    HIP_OR(msg, up(d.pt_init, pts0.data(), sizeof(double) * 3 * NP));
    if ((st = upload_plan(b, msg)) != GBA_OK) return st;
    HIP_OR(msg, hipStreamSynchronize(stream));
    return GBA_OK;
}

// ---------------------------------------------------------------- LM driver
namespace {

// h_scal is written by k_finish / k_cost_finish through its mapping
gba_status read_scal(Batch& b, std::string& msg) {
    HIP_OR(msg, hipStreamSynchronize(b.stream));
    return GBA_OK;
}

}  // namespace

gba_status batch_linearize(Batch& b, const RawOut* raw, Timers* tm, std::string& msg) {
    const bool timing = tm && tm->on;
    b.dg.jacobian = b.jacobian;
    if (timing) HIP_OR(msg, hipEventRecord(tm->ev[0], b.stream));
    HIP_OR(msg, launch_linearize(b.dg, b.stream, raw, !b.blocks_zeroed));
    b.blocks_zeroed = true;
    if (!raw) HIP_OR(msg, launch_assemble(b.dg, b.stream));
    if (timing) {
        HIP_OR(msg, hipEventRecord(tm->ev[1], b.stream));
        HIP_OR(msg, hipEventSynchronize(tm->ev[1]));
        float ms = 0.f;
        HIP_OR(msg, hipEventElapsedTime(&ms, tm->ev[0], tm->ev[1]));
        tm->ms_phase[0] += ms;
    }
    return GBA_OK;
}

gba_status batch_damped_step(Batch& b, const gba_options& o, const Tuning& tune, Timers* tm,
                             std::string& msg) {
    b.dg.min_diag = o.min_diag;   // the full system's products damp the point rows
    b.dg.max_diag = o.max_diag;
    const DeviceGraph& d = b.dg;
    hipStream_t s = b.stream;
    const bool timing = tm && tm->on;
    HIP_OR(msg, hipMemcpyAsync(d.lam, b.h_lam, sizeof(double) * b.P, hipMemcpyHostToDevice, s));
    if (timing) HIP_OR(msg, hipEventRecord(tm->ev[0], s));
    HIP_OR(msg, launch_damp(d, s, o.min_diag, o.max_diag));
    // the block-Jacobi pass forms the reduced RHS on its way (one-pass scheme)
    const int block_jacobi = o.precond == GBA_PRECOND_BLOCK_JACOBI ? 1 : 0;
    // the full system needs no reduced RHS (its PCG starts from -b)
    if (!d.full && !precond_forms_rhs(d, block_jacobi)) HIP_OR(msg, launch_rhs(d, s));
    HIP_OR(msg, launch_precond(d, s, o.min_diag, o.max_diag, block_jacobi, o.jacobi_scaling));
    if (timing) HIP_OR(msg, hipEventRecord(tm->ev[1], s));
    HIP_OR(msg, launch_pcg_init(d, s, o.pcg_tol, o.pcg_tol_relative));
    // one cooperative launch for every PCG iteration (the trial then runs to
    // its end without a host check), or chunks of launched iterations
    bool persistent = false;
    if (!timing && o.pcg_schedule == GBA_PCG_PERSISTENT) {
        if (b.persistent_ok < 0) b.persistent_ok = pcg_persistent_ok(d) ? 1 : 0;
        if (!b.persistent_ok) {
            msg = "the persistent PCG needs cooperative launches and a co-resident grid";
            return GBA_ERR_UNSUPPORTED;
        }
        persistent = true;
    }
    if (persistent) {
        HIP_OR(msg, launch_pcg_persistent(d, s, o.min_diag, o.max_diag, o.pcg_max_iters,
                                          o.pcg_rejection_ratio));
        if (timing) HIP_OR(msg, hipEventRecord(tm->ev[2], s));
        HIP_OR(msg, launch_backsub(d, s));
        HIP_OR(msg, launch_cost(d, s, d.cam_c, d.pt_c));
        HIP_OR(msg, launch_finish(d, s));
        gba_status st = read_scal(b, msg);
        if (st != GBA_OK) return st;
        int iters = 0;
        for (int p = 0; p < b.P; ++p) {
            if (b.h_scal[p].barrier_err) {
                msg = "persistent PCG: a grid barrier wait exceeded its bound";
                return GBA_ERR_HIP;
            }
            iters = std::max(iters, b.h_scal[p].pcg_iters);
        }
        b.last_pcg_iters = iters;
        return GBA_OK;
    }
    const int chunk = std::max(1, std::min(kMaxPcgChunk, tune.pcg_sync_every));
    // A PCG of k steps takes k + 1 launched iterations: an iteration decides
    // at its start whether the previous step ended the PCG.  The first chunk
    // is the previous step's launch count (successive LM trials need similar
    // counts; an idle iteration costs a few microseconds, a further host
    // check about thirty), replayed as a graph or launched directly, and the
    // rest are chunks of two.  Without a previous count: chunks of
    // pcg_sync_every.
    int first = chunk, rest = chunk;
    if (b.last_pcg_iters > 0) {
        first = std::min(kMaxPcgChunk, b.last_pcg_iters + 1);
        rest = std::min(chunk, 2);
    }
    const int max_launch = o.pcg_max_iters + 1;
    int launched = 0;
    int last_iters = 0;
    int products = 0;   // timing: launches that ran a product
    while (launched < max_launch) {
        const int c = std::min(launched == 0 ? first : rest, max_launch - launched);
        if (b.use_graphs && !timing && b.pcg_warm) {
            // replay the chunk as one graph (captured on first use, cached by length)
            // the dynamic product reads the parameters: one graph per
            // orientation of the current/candidate buffers
            const int orient = d.dynamic && d.cam > d.cam_c ? 1 : 0;
            Batch::PcgGraph& pg = b.pcg_graph[c][orient];
            const bool moved = d.dynamic && (pg.cam != d.cam || pg.pt != d.pt);
            if (pg.exec && (pg.iters != c || pg.max_iters != o.pcg_max_iters ||
                            pg.min_diag != o.min_diag || pg.max_diag != o.max_diag ||
                            pg.ratio != o.pcg_rejection_ratio || moved)) {
                (void)hipGraphExecDestroy(pg.exec);
                pg = Batch::PcgGraph{};
            }
            if (!pg.exec) {
                // captured on a private stream, replayed on the batch stream
                if (!b.cap_stream)
                    HIP_OR(msg, hipStreamCreateWithFlags(&b.cap_stream, hipStreamNonBlocking));
                hipStream_t cs = b.cap_stream;
                hipGraph_t graph = nullptr;
                HIP_OR(msg, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                hipError_t r = hipSuccess;
                for (int k = 0; k < c && r == hipSuccess; ++k)
                    r = launch_pcg_iter(d, cs, o.min_diag, o.max_diag, o.pcg_max_iters,
                                        o.pcg_rejection_ratio, nullptr, nullptr);
                hipError_t r2 = hipStreamEndCapture(cs, &graph);
                HIP_OR(msg, r);
                HIP_OR(msg, r2);
                r = hipGraphInstantiate(&pg.exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                HIP_OR(msg, r);
                pg.iters = c;
                pg.max_iters = o.pcg_max_iters;
                pg.min_diag = o.min_diag;
                pg.max_diag = o.max_diag;
                pg.ratio = o.pcg_rejection_ratio;
                pg.cam = d.cam;
                pg.pt = d.pt;
            }
            HIP_OR(msg, hipGraphLaunch(pg.exec, s));
        } else {
            for (int k = 0; k < c; ++k) {
                hipEvent_t e0 = timing ? tm->ev[4 + 2 * k] : nullptr;
                hipEvent_t e1 = timing ? tm->ev[5 + 2 * k] : nullptr;
                HIP_OR(msg, launch_pcg_iter(d, s, o.min_diag, o.max_diag, o.pcg_max_iters,
                                            o.pcg_rejection_ratio, e0, e1));
            }
            b.pcg_warm = true;
        }
        launched += c;
        // h_pcg is written by the apply kernels through its mapping
        HIP_OR(msg, hipStreamSynchronize(s));
        int max_iters_now = 0;
        bool all_done = true;
        for (int p = 0; p < b.P; ++p) {
            max_iters_now = std::max(max_iters_now, b.h_pcg[p].iters);
            all_done = all_done && b.h_pcg[p].done != 0;
        }
        if (timing) {
            // only launches in which some problem still stepped time a
            // product: every launch until all PCGs have stopped, then as many
            // as the longest one took steps
            const int ran = std::min(c, std::max(0, (all_done ? max_iters_now : launched) - products));
            products += ran;
            for (int k = 0; k < ran; ++k) {
                float ms = 0.f;
                HIP_OR(msg, hipEventElapsedTime(&ms, tm->ev[4 + 2 * k], tm->ev[5 + 2 * k]));
                tm->ms_mv += ms;
                tm->n_mv += 1;
            }
        }
        last_iters = max_iters_now;
        if (all_done) break;
    }
    b.last_pcg_iters = last_iters;
    if (timing) HIP_OR(msg, hipEventRecord(tm->ev[2], s));
    HIP_OR(msg, launch_backsub(d, s));
    HIP_OR(msg, launch_cost(d, s, d.cam_c, d.pt_c));
    HIP_OR(msg, launch_finish(d, s));
    if (timing) HIP_OR(msg, hipEventRecord(tm->ev[3], s));
    gba_status st = read_scal(b, msg);
    if (st != GBA_OK) return st;
    if (timing) {
        float a = 0.f, c = 0.f, e = 0.f;
        HIP_OR(msg, hipEventElapsedTime(&a, tm->ev[0], tm->ev[1]));
        HIP_OR(msg, hipEventElapsedTime(&c, tm->ev[1], tm->ev[2]));
        HIP_OR(msg, hipEventElapsedTime(&e, tm->ev[2], tm->ev[3]));
        tm->ms_phase[1] += a;
        tm->ms_phase[2] += c;
        tm->ms_phase[3] += e;
    }
    return GBA_OK;
}

gba_status batch_time_matvec(Batch& b, const gba_options& o, int launches, double* ms,
                             std::string& msg) {
    b.dg.min_diag = o.min_diag;
    b.dg.max_diag = o.max_diag;
    const DeviceGraph& d = b.dg;
    hipStream_t s = b.stream;
    HIP_OR(msg, hipMemcpyAsync(d.lam, b.h_lam, sizeof(double) * b.P, hipMemcpyHostToDevice, s));
    HIP_OR(msg, launch_damp(d, s, o.min_diag, o.max_diag));
    // the block-Jacobi pass forms the reduced RHS on its way (one-pass scheme)
    const int block_jacobi = o.precond == GBA_PRECOND_BLOCK_JACOBI ? 1 : 0;
    // the full system needs no reduced RHS (its PCG starts from -b)
    if (!d.full && !precond_forms_rhs(d, block_jacobi)) HIP_OR(msg, launch_rhs(d, s));
    HIP_OR(msg, launch_precond(d, s, o.min_diag, o.max_diag, block_jacobi, o.jacobi_scaling));
    // tolerance 0 and no iteration limit: the products below run for every
    // problem with work.  One iteration first, so that they take the decision
    // of a later iteration, as in the PCG loop.
    constexpr int kNoLimit = 1 << 30;
    HIP_OR(msg, launch_pcg_init(d, s, 0.0, 0));
    HIP_OR(msg, launch_pcg_iter(d, s, o.min_diag, o.max_diag, kNoLimit, 0.0, nullptr, nullptr));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OR(msg, hipEventCreate(&e0));
    hipError_t r = hipEventCreate(&e1);
    if (r == hipSuccess) r = hipEventRecord(e0, s);
    for (int k = 0; k < launches && r == hipSuccess; ++k) r = launch_matvec(d, s, kNoLimit, 0.0);
    if (r == hipSuccess) r = hipEventRecord(e1, s);
    if (r == hipSuccess) r = hipEventSynchronize(e1);
    float t = 0.f;
    if (r == hipSuccess) r = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    HIP_OR(msg, r);
    *ms = launches > 0 ? (double)t / launches : 0.0;
    return GBA_OK;
}

gba_status batch_cost(Batch& b, std::string& msg) {
    HIP_OR(msg, launch_cost(b.dg, b.stream, b.dg.cam, b.dg.pt));
    HIP_OR(msg, launch_cost_finish(b.dg, b.stream));
    return read_scal(b, msg);
}

gba_status batch_begin(Batch& b, const std::vector<const HostProblem*>& probs,
                       std::vector<ProblemLM>& lm, const std::vector<char>& fresh,
                       const gba_options& o, Timers* tm, std::string& msg) {
    gba_status st = batch_cost(b, msg);
    if (st != GBA_OK) return st;
    bool any = false;
    for (int p = 0; p < b.P; ++p) {
        ProblemLM& s = lm[p];
        if (!fresh[p]) {
            any = any || s.running;
            continue;
        }
        const bool edges = b.plan.edge_off[p + 1] > b.plan.edge_off[p];
        s.F = edges ? b.h_scal[p].cost : 0.0;
        s.F0 = s.F;
        s.lam = o.initial_lambda;
        s.nu = 2.0;
        s.trials = s.accepted = s.pcg_total = 0;
        s.log.clear();
        s.running = false;
        if (!edges || !probs[p]->any_free()) {
            s.term = GBA_TERM_NO_WORK;
        } else if (s.max_iters <= 0) {
            s.term = GBA_TERM_MAX_ITERS;
        } else if (!std::isfinite(s.F)) {
            s.term = GBA_TERM_NUMERICAL_FAILURE;
        } else {
            s.term = GBA_TERM_NONE;
            s.running = true;
            any = true;
        }
    }
    if (any) return batch_linearize(b, nullptr, tm, msg);
    return GBA_OK;
}

gba_status batch_trial(Batch& b, std::vector<ProblemLM>& lm, const gba_options& o,
                       const Tuning& tune, Timers* tm, std::string& msg) {
    // idle problems (terminated or without work) carry a negative damping: the
    // device skips their PCG
    for (int p = 0; p < b.P; ++p) b.h_lam[p] = lm[p].running ? lm[p].lam : -o.initial_lambda;
    gba_status st = batch_damped_step(b, o, tune, tm, msg);
    if (st != GBA_OK) return st;
    bool any_accept = false, any_running = false;
    for (int p = 0; p < b.P; ++p) {
        b.h_accept[p] = 0;
        ProblemLM& s = lm[p];
        if (!s.running) continue;
        const TrialScalars& sc = b.h_scal[p];
        const double Fn = sc.cost;
        const double L = -(sc.b_dot_dx + 0.5 * sc.quad);
        const double dnorm = std::sqrt(sc.step2), xnorm = std::sqrt(sc.x2);
        const bool accepted = (L > 0.0) && (Fn < s.F);
        const double gain = L != 0.0 ? (s.F - Fn) / L : std::numeric_limits<double>::quiet_NaN();
        gba_trial tr;
        tr.cost = s.F;
        tr.candidate_cost = Fn;
        tr.lambda = s.lam;
        tr.model_decrease = L;
        tr.step_norm = dnorm;
        tr.accepted = accepted ? 1 : 0;
        tr.pcg_iters = sc.pcg_iters;
        s.log.push_back(tr);
        s.trials += 1;
        s.pcg_total += sc.pcg_iters;
        int stop = 0;
        if (accepted) {
            const double rel = (s.F - Fn) / s.F;
            s.F = Fn;
            const double t3 = 2.0 * gain - 1.0;
            s.lam *= std::max(1.0 / 3.0, 1.0 - t3 * t3 * t3);
            s.nu = 2.0;
            s.accepted += 1;
            b.h_accept[p] = 1;
            any_accept = true;
            if (rel < s.tol) stop = GBA_TERM_COST_TOL;
        } else {
            s.lam *= s.nu;
            s.nu *= 2.0;
        }
        if (!stop && dnorm <= s.tol * (xnorm + s.tol)) stop = GBA_TERM_STEP_TOL;
        if (!stop && s.lam > 1e32) stop = GBA_TERM_LAMBDA_OVERFLOW;
        if (!stop && s.trials >= s.max_iters) stop = GBA_TERM_MAX_ITERS;
        if (stop) {
            s.term = stop;
            s.running = false;
        }
        any_running = any_running || s.running;
    }
    if (any_accept) {
        if (b.P == 1) {
            // one problem: the candidate buffers become the current ones
            std::swap(b.dg.cam, b.dg.cam_c);
            std::swap(b.dg.pt, b.dg.pt_c);
        } else {
            HIP_OR(msg, hipMemcpyAsync(b.dg.accept, b.h_accept, sizeof(int) * b.P,
                                       hipMemcpyHostToDevice, b.stream));
            HIP_OR(msg, launch_commit(b.dg, b.stream));
        }
        if (any_running) return batch_linearize(b, nullptr, tm, msg);
        HIP_OR(msg, hipStreamSynchronize(b.stream));
    }
    return GBA_OK;
}

gba_status batch_download(Batch& b, int p, double* cams, double* pts, std::string& msg) {
    const int c0 = b.plan.cam_off[p], c1 = b.plan.cam_off[p + 1];
    const int p0 = b.plan.pt_off[p], p1 = b.plan.pt_off[p + 1];
    if (cams && c1 > c0)
        HIP_OR(msg, hipMemcpyAsync(cams, b.dg.cam + 9 * (size_t)c0, sizeof(double) * 9 * (c1 - c0),
                                   hipMemcpyDeviceToHost, b.stream));
    if (pts && p1 > p0)
        HIP_OR(msg, hipMemcpyAsync(pts, b.dg.pt + 3 * (size_t)p0, sizeof(double) * 3 * (p1 - p0),
                                   hipMemcpyDeviceToHost, b.stream));
    HIP_OR(msg, hipStreamSynchronize(b.stream));
    return GBA_OK;
}

}  // namespace gba
