// C ABI, graph build and Levenberg-Marquardt driver of the gfx950
// bundle-adjustment solver.  The per-iteration arithmetic runs in the
// kernels of gba_kernels.hip; this file plans memory, orders the edges and
// takes the scalar LM decisions (accept / reject / damping update) from FP64
// values computed on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <unordered_map>
#include <vector>

#include "gba.h"
#include "gba_internal.h"

namespace gba {
hipError_t launch_cost_finish(const DeviceGraph& g, hipStream_t s);
}

using gba::DeviceGraph;

struct gba_graph {
    int precision = 0;
    int device = 0;
    gba_alloc_fn alloc = nullptr;
    gba_free_fn free_fn = nullptr;
    void* ctx = nullptr;
    hipStream_t stream = nullptr;
    gba_options opts{};
    int loss = GBA_LOSS_SQUARED;
    double delta = 1.0;

    // host staging, insertion order
    std::vector<int64_t> cam_ids, pt_ids;
    std::unordered_map<int64_t, int> cam_map, pt_map;
    std::vector<double> cam_params, pt_params;      // current values
    std::vector<double> cam_init, pt_init;          // values at insertion
    std::vector<unsigned char> cam_fixed, pt_fixed;
    std::vector<int> e_cam, e_pt;
    std::vector<double> e_uv, e_info;
    std::vector<unsigned char> e_active;
    bool any_info = false;

    // device state
    bool dirty = true;
    bool built = false;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    DeviceGraph dg{};
    std::vector<int> pm_edge;  // point-major position -> insertion index
    gba::TrialScalars* h_scal = nullptr;
    gba::PcgState* h_pcg = nullptr;
    int n_cu = 256;
    size_t max_lds = 65536;

    std::vector<gba_trial> trials;
    std::string err;
};

namespace {

gba_status fail(gba_graph* g, gba_status code, const std::string& msg) {
    if (g) g->err = msg;
    return code;
}

#define HIP_TRY(g, call)                                                               \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail((g), GBA_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool finite_all(const double* p, size_t n) {
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(p[k])) return false;
    return true;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct Planner {
    size_t off = 0;
    std::vector<std::pair<void**, size_t>> items;
    void add(void** slot, size_t bytes) {
        items.push_back({slot, off});
        off += align_up(bytes ? bytes : 1);
    }
};

void* dev_alloc(gba_graph* g, size_t bytes) {
    if (g->alloc) return g->alloc(bytes, g->ctx);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void dev_free(gba_graph* g, void* p) {
    if (!p) return;
    if (g->free_fn)
        g->free_fn(p, g->ctx);
    else
        (void)hipFree(p);
}

void release_device(gba_graph* g) {
    if (g->arena) {
        (void)hipStreamSynchronize(g->stream);
        dev_free(g, g->arena);
    }
    g->arena = nullptr;
    g->arena_bytes = 0;
    g->built = false;
}

// Pull the current device parameters back into host staging (so a rebuild
// keeps the optimised values).
gba_status sync_params_to_host(gba_graph* g) {
    if (!g->built) return GBA_OK;
    HIP_TRY(g, hipMemcpyAsync(g->cam_params.data(), g->dg.cam, sizeof(double) * 9 * g->dg.nc,
                              hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(g, hipMemcpyAsync(g->pt_params.data(), g->dg.pt, sizeof(double) * 3 * g->dg.np,
                              hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(g, hipStreamSynchronize(g->stream));
    return GBA_OK;
}

gba_status build(gba_graph* g) {
    HIP_TRY(g, hipSetDevice(g->device));
    gba_status st = sync_params_to_host(g);
    if (st != GBA_OK) return st;
    release_device(g);

    const int nc = (int)g->cam_ids.size();
    const int np = (int)g->pt_ids.size();
    const size_t n_all = g->e_cam.size();
    if (n_all > (size_t)std::numeric_limits<int>::max() / 32)
        return fail(g, GBA_ERR_UNSUPPORTED, "too many edges for 32-bit indexing");

    // active edges in point-major order (counting sort by point, then by
    // camera inside each point; insertion order breaks ties)
    std::vector<int> act;
    act.reserve(n_all);
    for (size_t e = 0; e < n_all; ++e)
        if (g->e_active[e]) act.push_back((int)e);
    const int ne = (int)act.size();
    std::vector<int> pcount(np + 1, 0);
    for (int e : act) pcount[g->e_pt[e] + 1]++;
    for (int j = 0; j < np; ++j) pcount[j + 1] += pcount[j];
    std::vector<int> pm(ne);
    {
        std::vector<int> pos(pcount.begin(), pcount.end() - 1);
        for (int e : act) pm[pos[g->e_pt[e]]++] = e;
        for (int j = 0; j < np; ++j) {
            auto b = pm.begin() + pcount[j], en = pm.begin() + pcount[j + 1];
            std::stable_sort(b, en, [&](int a, int c) { return g->e_cam[a] < g->e_cam[c]; });
        }
    }
    // tiles of whole points (<= 64 edges) or one long point
    std::vector<int> tile_off;
    tile_off.push_back(0);
    {
        int cur = 0;
        for (int j = 0; j < np; ++j) {
            const int c = pcount[j + 1] - pcount[j];
            if (c == 0) continue;
            if (c > gba::kTileEdges) {
                if (cur > 0) {
                    tile_off.push_back(tile_off.back() + cur);
                    cur = 0;
                }
                tile_off.push_back(tile_off.back() + c);
            } else {
                if (cur + c > gba::kTileEdges) {
                    tile_off.push_back(tile_off.back() + cur);
                    cur = 0;
                }
                cur += c;
            }
        }
        if (cur > 0) tile_off.push_back(tile_off.back() + cur);
    }
    const int n_tiles = (int)tile_off.size() - 1;

    // camera-major order, runs of equal (camera, point), chunks per camera
    std::vector<int> ccount(nc + 1, 0);
    for (int e : act) ccount[g->e_cam[e] + 1]++;
    for (int i = 0; i < nc; ++i) ccount[i + 1] += ccount[i];
    std::vector<int> cm(ne);
    {
        std::vector<int> pos(ccount.begin(), ccount.end() - 1);
        for (int e : pm) cm[pos[g->e_cam[e]]++] = e;  // point order inside a camera
    }
    std::vector<int> run_off, chunk_run_off, chunk_cam, cam_chunk_off(nc + 1, 0);
    for (int i = 0; i < nc; ++i) {
        cam_chunk_off[i] = (int)chunk_cam.size();
        int runs_in_chunk = 0;
        for (int q = ccount[i]; q < ccount[i + 1]; ++q) {
            const bool new_run = q == ccount[i] || g->e_pt[cm[q]] != g->e_pt[cm[q - 1]];
            if (!new_run) continue;
            if (runs_in_chunk == 0) {
                chunk_run_off.push_back((int)run_off.size());
                chunk_cam.push_back(i);
            }
            run_off.push_back(q);
            if (++runs_in_chunk == gba::kChunkRuns) runs_in_chunk = 0;
        }
    }
    cam_chunk_off[nc] = (int)chunk_cam.size();
    const int n_runs = (int)run_off.size();
    run_off.push_back(ne);
    const int n_chunks = (int)chunk_cam.size();
    chunk_run_off.push_back(n_runs);

    // square-root information factors (Omega = A^T A, A upper triangular)
    std::vector<double> sinfo, cm_sinfo;
    if (g->any_info) {
        sinfo.resize(3 * (size_t)ne);
        cm_sinfo.resize(3 * (size_t)ne);
        for (int pass = 0; pass < 2; ++pass) {
            const std::vector<int>& ord = pass == 0 ? pm : cm;
            std::vector<double>& dst = pass == 0 ? sinfo : cm_sinfo;
            for (int q = 0; q < ne; ++q) {
                const int e = ord[q];
                const double o00 = g->e_info[3 * e], o01 = g->e_info[3 * e + 1],
                             o11 = g->e_info[3 * e + 2];
                if (!(o00 > 0.0)) return fail(g, GBA_ERR_INVALID_ARG, "information matrix not positive definite");
                const double a00 = std::sqrt(o00), a01 = o01 / a00, d = o11 - a01 * a01;
                if (!(d > 0.0)) return fail(g, GBA_ERR_INVALID_ARG, "information matrix not positive definite");
                dst[q] = a00;
                dst[(size_t)ne + q] = a01;
                dst[2 * (size_t)ne + q] = std::sqrt(d);
            }
        }
    }

    // launch geometry
    DeviceGraph& d = g->dg;
    d = DeviceGraph{};
    d.nc = nc;
    d.np = np;
    d.ne = ne;
    d.n_tiles = n_tiles;
    d.n_runs = n_runs;
    d.n_chunks = n_chunks;
    d.has_info = g->any_info ? 1 : 0;
    d.loss = g->loss;
    d.delta = g->delta;
    d.mode = g->precision;
    const size_t tsz = g->precision == GBA_FP64 ? 8 : 4;
    d.block_pp = 1024;
    const int waves_pp = d.block_pp / 64;
    int gpp = (n_tiles + waves_pp - 1) / waves_pp;
    d.grid_pp = std::max(1, std::min(g->n_cu, gpp));
    // camera partial sums are FP64 in every mode: the Schur product subtracts
    // the point-elimination term from Hcc p, so summation noise is amplified
    d.lds_pp = (int)(9 * (size_t)nc * sizeof(double));
    if ((size_t)d.lds_pp + 1024 > g->max_lds)
        return fail(g, GBA_ERR_UNSUPPORTED,
                    "camera vector does not fit in LDS (" + std::to_string(nc) + " cameras)");
    d.grid_red = std::max(1, (9 * nc + 63) / 64);
    d.grid_edges = std::max(1, std::min((ne + 255) / 256, 2048));
    d.grid_pts = std::max(1, std::min((np + 255) / 256, 2048));

    // memory plan: one arena
    Planner P;
    const size_t NE = (size_t)ne, NP = (size_t)np, NC = (size_t)nc;
    P.add((void**)&d.tile_off, sizeof(int) * (n_tiles + 1));
    P.add((void**)&d.e_cam, sizeof(int) * NE);
    P.add((void**)&d.e_pt, sizeof(int) * NE);
    P.add((void**)&d.obs, sizeof(double) * 2 * NE);
    if (g->any_info) P.add((void**)&d.sinfo, sizeof(double) * 3 * NE);
    P.add((void**)&d.cm_run_off, sizeof(int) * (n_runs + 1));
    P.add((void**)&d.cm_pt, sizeof(int) * NE);
    P.add((void**)&d.cm_obs, sizeof(double) * 2 * NE);
    if (g->any_info) P.add((void**)&d.cm_sinfo, sizeof(double) * 3 * NE);
    P.add((void**)&d.chunk_run_off, sizeof(int) * (n_chunks + 1));
    P.add((void**)&d.chunk_cam, sizeof(int) * n_chunks);
    P.add((void**)&d.cam_chunk_off, sizeof(int) * (nc + 1));
    P.add((void**)&d.cam_fixed, NC);
    P.add((void**)&d.pt_fixed, NP);
    P.add((void**)&d.cam, sizeof(double) * 9 * NC);
    P.add((void**)&d.cam_c, sizeof(double) * 9 * NC);
    P.add((void**)&d.cam_init, sizeof(double) * 9 * NC);
    P.add((void**)&d.pt, sizeof(double) * 3 * NP);
    P.add((void**)&d.pt_c, sizeof(double) * 3 * NP);
    P.add((void**)&d.pt_init, sizeof(double) * 3 * NP);
    P.add((void**)&d.dpt, sizeof(double) * 3 * NP);
    const size_t jsz = g->precision == GBA_FP64 ? 8 : (g->precision == GBA_MIXED_FP32 ? 4 : 2);
    d.jac_bytes = (int)jsz;
    P.add(&d.jc, jsz * 18 * NE);
    P.add(&d.jp, jsz * 6 * NE);
    P.add(&d.rw, tsz * 2 * NE);
    P.add(&d.hpp, tsz * 6 * NP);
    P.add(&d.bp, tsz * 3 * NP);
    P.add(&d.hcc, tsz * 45 * NC);
    P.add(&d.wrun, tsz * 27 * (size_t)std::max(1, n_runs));
    P.add(&d.bc, tsz * 9 * NC);
    P.add((void**)&d.hpp_inv, sizeof(double) * gba::kHinvStride * NP);
    P.add(&d.minv, tsz * 45 * NC);
    P.add(&d.v_x, tsz * 9 * NC);
    P.add(&d.v_r, tsz * 9 * NC);
    P.add(&d.v_z, tsz * 9 * NC);
    P.add(&d.v_p, tsz * 9 * NC);
    P.add(&d.v_q, tsz * 9 * NC);
    P.add(&d.v_best, tsz * 9 * NC);
    P.add(&d.cam_partial, sizeof(double) * 9 * NC * (size_t)d.grid_pp);
    P.add((void**)&d.pq_partial, sizeof(double) * d.grid_red);
    P.add((void**)&d.dot_partial, sizeof(double) * 2 * ((nc + 27) / 28 + 1));
    P.add((void**)&d.chunk_partial, sizeof(double) * 54 * std::max(1, n_chunks));
    P.add((void**)&d.red_partial, sizeof(double) * 4 * d.grid_pp);
    P.add((void**)&d.cost_partial, sizeof(double) * d.grid_edges);
    P.add((void**)&d.damp_partial, sizeof(double) * d.grid_pts);
    P.add((void**)&d.pcg, sizeof(gba::PcgState));
    P.add((void**)&d.scal, sizeof(gba::TrialScalars));

    void* arena = dev_alloc(g, P.off);
    if (!arena) return fail(g, GBA_ERR_OOM, "device allocation of " + std::to_string(P.off) + " bytes failed");
    g->arena = arena;
    g->arena_bytes = P.off;
    for (auto& it : P.items) *it.first = (char*)arena + it.second;

    // upload
    std::vector<int> h_ecam(ne), h_ept(ne), h_cmpt(ne);
    std::vector<double> h_obs(2 * NE), h_cmobs(2 * NE);
    for (int q = 0; q < ne; ++q) {
        const int e = pm[q];
        h_ecam[q] = g->e_cam[e];
        h_ept[q] = g->e_pt[e];
        h_obs[q] = g->e_uv[2 * (size_t)e];
        h_obs[NE + q] = g->e_uv[2 * (size_t)e + 1];
        const int c = cm[q];
        h_cmpt[q] = g->e_pt[c];
        h_cmobs[q] = g->e_uv[2 * (size_t)c];
        h_cmobs[NE + q] = g->e_uv[2 * (size_t)c + 1];
    }
    hipStream_t s = g->stream;
    auto up = [&](const void* dst, const void* src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync((void*)dst, src, bytes, hipMemcpyHostToDevice, s);
    };
    HIP_TRY(g, up(d.tile_off, tile_off.data(), sizeof(int) * tile_off.size()));
    HIP_TRY(g, up(d.e_cam, h_ecam.data(), sizeof(int) * NE));
    HIP_TRY(g, up(d.e_pt, h_ept.data(), sizeof(int) * NE));
    HIP_TRY(g, up(d.obs, h_obs.data(), sizeof(double) * 2 * NE));
    if (g->any_info) {
        HIP_TRY(g, up(d.sinfo, sinfo.data(), sizeof(double) * 3 * NE));
        HIP_TRY(g, up(d.cm_sinfo, cm_sinfo.data(), sizeof(double) * 3 * NE));
    }
    HIP_TRY(g, up(d.cm_run_off, run_off.data(), sizeof(int) * run_off.size()));
    HIP_TRY(g, up(d.cm_pt, h_cmpt.data(), sizeof(int) * NE));
    HIP_TRY(g, up(d.cm_obs, h_cmobs.data(), sizeof(double) * 2 * NE));
    HIP_TRY(g, up(d.chunk_run_off, chunk_run_off.data(), sizeof(int) * chunk_run_off.size()));
    HIP_TRY(g, up(d.chunk_cam, chunk_cam.data(), sizeof(int) * chunk_cam.size()));
    HIP_TRY(g, up(d.cam_chunk_off, cam_chunk_off.data(), sizeof(int) * cam_chunk_off.size()));
    HIP_TRY(g, up(d.cam_fixed, g->cam_fixed.data(), NC));
    HIP_TRY(g, up(d.pt_fixed, g->pt_fixed.data(), NP));
    HIP_TRY(g, up(d.cam, g->cam_params.data(), sizeof(double) * 9 * NC));
    HIP_TRY(g, up(d.cam_init, g->cam_init.data(), sizeof(double) * 9 * NC));
    HIP_TRY(g, up(d.pt, g->pt_params.data(), sizeof(double) * 3 * NP));
    HIP_TRY(g, up(d.pt_init, g->pt_init.data(), sizeof(double) * 3 * NP));
    HIP_TRY(g, hipStreamSynchronize(s));
    g->pm_edge = std::move(pm);
    g->built = true;
    g->dirty = false;
    return GBA_OK;
}

gba_status ensure_built(gba_graph* g) {
    if (!g->dirty && g->built) return GBA_OK;
    return build(g);
}

gba_status read_scalars(gba_graph* g) {
    HIP_TRY(g, hipMemcpyAsync(g->h_scal, g->dg.scal, sizeof(gba::TrialScalars), hipMemcpyDeviceToHost,
                              g->stream));
    HIP_TRY(g, hipStreamSynchronize(g->stream));
    return GBA_OK;
}

gba_status eval_cost(gba_graph* g, const double* cam, const double* pt, double* out) {
    HIP_TRY(g, gba::launch_cost(g->dg, g->stream, cam, pt));
    HIP_TRY(g, gba::launch_cost_finish(g->dg, g->stream));
    gba_status st = read_scalars(g);
    if (st != GBA_OK) return st;
    *out = g->h_scal->cost;
    return GBA_OK;
}

gba_status linearize(gba_graph* g, const gba::RawOut* raw) {
    HIP_TRY(g, gba::launch_linearize(g->dg, g->stream, raw));
    HIP_TRY(g, gba::launch_assemble(g->dg, g->stream));
    return GBA_OK;
}

struct Timers {
    bool on = false;
    std::vector<hipEvent_t> ev;
    double ms_mv = 0.0;
    int n_mv = 0;
};

// One damped solve at the current linearisation: point damping, reduced RHS,
// preconditioner, PCG, back-substitution and candidate evaluation.  Leaves
// the trial scalars in g->h_scal.
gba_status damped_step(gba_graph* g, double lambda, Timers* tm, double* ms_phase) {
    const gba_options& o = g->opts;
    const DeviceGraph& d = g->dg;
    hipStream_t s = g->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
    if (tm && tm->on) {
        e0 = tm->ev[0];
        e1 = tm->ev[1];
        e2 = tm->ev[2];
        e3 = tm->ev[3];
        HIP_TRY(g, hipEventRecord(e0, s));
    }
    HIP_TRY(g, gba::launch_damp(d, s, lambda, o.min_diag, o.max_diag));
    HIP_TRY(g, gba::launch_rhs(d, s));
    HIP_TRY(g, gba::launch_precond(d, s, lambda, o.min_diag, o.max_diag,
                                   o.precond == GBA_PRECOND_BLOCK_JACOBI ? 1 : 0));
    if (e1) HIP_TRY(g, hipEventRecord(e1, s));
    HIP_TRY(g, gba::launch_pcg_init(d, s, o.pcg_tol, o.pcg_tol_relative));
    const int chunk = 8;
    int launched = 0;
    int last_iters = 0;
    while (launched < o.pcg_max_iters) {
        const int c = std::min(chunk, o.pcg_max_iters - launched);
        for (int k = 0; k < c; ++k) {
            hipEvent_t a = nullptr, b = nullptr;
            if (tm && tm->on) {
                a = tm->ev[4 + 2 * k];
                b = tm->ev[5 + 2 * k];
            }
            HIP_TRY(g, gba::launch_pcg_iter(d, s, lambda, o.min_diag, o.max_diag, o.pcg_max_iters,
                                            o.pcg_rejection_ratio, a, b));
        }
        launched += c;
        HIP_TRY(g, hipMemcpyAsync(g->h_pcg, d.pcg, sizeof(gba::PcgState), hipMemcpyDeviceToHost, s));
        HIP_TRY(g, hipStreamSynchronize(s));
        if (tm && tm->on) {
            const int ran = std::min(c, g->h_pcg->iters - last_iters);
            for (int k = 0; k < ran; ++k) {
                float ms = 0.f;
                HIP_TRY(g, hipEventElapsedTime(&ms, tm->ev[4 + 2 * k], tm->ev[5 + 2 * k]));
                tm->ms_mv += ms;
                tm->n_mv += 1;
            }
        }
        last_iters = g->h_pcg->iters;
        if (g->h_pcg->done) break;
    }
    if (e2) HIP_TRY(g, hipEventRecord(e2, s));
    HIP_TRY(g, gba::launch_backsub(d, s));
    HIP_TRY(g, gba::launch_cost(d, s, d.cam_c, d.pt_c));
    HIP_TRY(g, gba::launch_finish(d, s));
    if (e3) HIP_TRY(g, hipEventRecord(e3, s));
    gba_status st = read_scalars(g);
    if (st != GBA_OK) return st;
    if (tm && tm->on && ms_phase) {
        float a = 0.f, b = 0.f, c = 0.f;
        HIP_TRY(g, hipEventElapsedTime(&a, e0, e1));
        HIP_TRY(g, hipEventElapsedTime(&b, e1, e2));
        HIP_TRY(g, hipEventElapsedTime(&c, e2, e3));
        ms_phase[0] += a;
        ms_phase[1] += b;
        ms_phase[2] += c;
    }
    return GBA_OK;
}

bool has_free_vertex(const gba_graph* g) {
    for (unsigned char f : g->cam_fixed)
        if (!f) return true;
    for (unsigned char f : g->pt_fixed)
        if (!f) return true;
    return false;
}

template <typename T>
void to_double(const std::vector<unsigned char>& raw, double* dst, size_t n) {
    const T* s = (const T*)raw.data();
    for (size_t k = 0; k < n; ++k) dst[k] = (double)s[k];
}

gba_status download_typed(gba_graph* g, const void* src, size_t n, std::vector<double>& dst) {
    const size_t tsz = g->precision == GBA_FP64 ? 8 : 4;
    std::vector<unsigned char> raw(n * tsz);
    dst.resize(n);
    if (n) {
        HIP_TRY(g, hipMemcpyAsync(raw.data(), src, n * tsz, hipMemcpyDeviceToHost, g->stream));
        HIP_TRY(g, hipStreamSynchronize(g->stream));
    }
    if (tsz == 8)
        to_double<double>(raw, dst.data(), n);
    else
        to_double<float>(raw, dst.data(), n);
    return GBA_OK;
}

}  // namespace

// ============================================================== C ABI
extern "C" {

void gba_default_options(gba_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->initial_lambda = 1e-4;
    o->min_diag = 1e-6;
    o->max_diag = 1e32;
    o->pcg_max_iters = 100;
    o->pcg_tol = 1e-6;
    o->pcg_tol_relative = 1;
    o->pcg_rejection_ratio = 0.0;
    o->precond = GBA_PRECOND_BLOCK_JACOBI;
    o->timing = 0;
}

gba_status gba_create(gba_precision precision, int device, gba_alloc_fn alloc, gba_free_fn free_fn,
                      void* ctx, gba_graph** out) {
    if (!out) return GBA_ERR_INVALID_ARG;
    *out = nullptr;
    if (precision != GBA_FP64 && precision != GBA_MIXED_FP32 && precision != GBA_MIXED_BF16)
        return GBA_ERR_INVALID_ARG;
    if ((alloc == nullptr) != (free_fn == nullptr)) return GBA_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GBA_ERR_HIP;
    gba_graph* g = new gba_graph();
    g->precision = precision;
    g->device = device;
    g->alloc = alloc;
    g->free_fn = free_fn;
    g->ctx = ctx;
    gba_default_options(&g->opts);
    if (hipSetDevice(device) != hipSuccess) {
        delete g;
        return GBA_ERR_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        g->n_cu = prop.multiProcessorCount;
        g->max_lds = prop.sharedMemPerBlock;
    }
    if (hipHostMalloc((void**)&g->h_scal, sizeof(gba::TrialScalars), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&g->h_pcg, sizeof(gba::PcgState), hipHostMallocDefault) != hipSuccess) {
        delete g;
        return GBA_ERR_HIP;
    }
    *out = g;
    return GBA_OK;
}

gba_status gba_set_stream(gba_graph* g, void* hip_stream) {
    if (!g) return GBA_ERR_INVALID_ARG;
    g->stream = (hipStream_t)hip_stream;
    return GBA_OK;
}

gba_status gba_reserve(gba_graph* g, int64_t n_cams, int64_t n_pts, int64_t n_edges) {
    if (!g || n_cams < 0 || n_pts < 0 || n_edges < 0) return fail(g, GBA_ERR_INVALID_ARG, "negative size");
    g->cam_ids.reserve(n_cams);
    g->cam_params.reserve(9 * n_cams);
    g->cam_init.reserve(9 * n_cams);
    g->cam_fixed.reserve(n_cams);
    g->cam_map.reserve(n_cams);
    g->pt_ids.reserve(n_pts);
    g->pt_params.reserve(3 * n_pts);
    g->pt_init.reserve(3 * n_pts);
    g->pt_fixed.reserve(n_pts);
    g->pt_map.reserve(n_pts);
    g->e_cam.reserve(n_edges);
    g->e_pt.reserve(n_edges);
    g->e_uv.reserve(2 * n_edges);
    g->e_active.reserve(n_edges);
    return GBA_OK;
}

gba_status add_vertices(gba_graph* g, int64_t n, const int64_t* ids, const double* v, int dim,
                               std::vector<int64_t>& idv, std::unordered_map<int64_t, int>& map,
                               std::vector<double>& par, std::vector<double>& init,
                               std::vector<unsigned char>& fixed) {
    if (!g || n < 0 || (n > 0 && (!ids || !v))) return fail(g, GBA_ERR_INVALID_ARG, "bad vertex arrays");
    if (!finite_all(v, (size_t)n * dim)) return fail(g, GBA_ERR_NONFINITE, "non-finite vertex parameters");
    if ((int64_t)idv.size() + n > std::numeric_limits<int>::max() / 16)
        return fail(g, GBA_ERR_UNSUPPORTED, "too many vertices");
    for (int64_t k = 0; k < n; ++k) {
        if (map.count(ids[k])) return fail(g, GBA_ERR_DUPLICATE_ID, "duplicate vertex id " + std::to_string(ids[k]));
        for (int64_t q = 0; q < k; ++q)
            if (ids[q] == ids[k] && n < 64)
                return fail(g, GBA_ERR_DUPLICATE_ID, "duplicate vertex id " + std::to_string(ids[k]));
    }
    // duplicates inside a large batch
    if (n >= 64) {
        std::vector<int64_t> s(ids, ids + n);
        std::sort(s.begin(), s.end());
        for (int64_t k = 1; k < n; ++k)
            if (s[k] == s[k - 1]) return fail(g, GBA_ERR_DUPLICATE_ID, "duplicate vertex id " + std::to_string(s[k]));
    }
    gba_status st = sync_params_to_host(g);
    if (st != GBA_OK) return st;
    for (int64_t k = 0; k < n; ++k) {
        map[ids[k]] = (int)idv.size();
        idv.push_back(ids[k]);
        fixed.push_back(0);
    }
    par.insert(par.end(), v, v + n * dim);
    init.insert(init.end(), v, v + n * dim);
    g->dirty = true;
    return GBA_OK;
}

gba_status gba_add_cameras(gba_graph* g, int64_t n, const int64_t* ids, const double* params) {
    if (!g) return GBA_ERR_INVALID_ARG;
    return add_vertices(g, n, ids, params, 9, g->cam_ids, g->cam_map, g->cam_params, g->cam_init,
                        g->cam_fixed);
}

gba_status gba_add_points(gba_graph* g, int64_t n, const int64_t* ids, const double* xyz) {
    if (!g) return GBA_ERR_INVALID_ARG;
    return add_vertices(g, n, ids, xyz, 3, g->pt_ids, g->pt_map, g->pt_params, g->pt_init, g->pt_fixed);
}

gba_status gba_add_edges(gba_graph* g, int64_t n, const int64_t* cam_ids, const int64_t* pt_ids,
                         const double* uv, const double* info) {
    if (!g) return GBA_ERR_INVALID_ARG;
    if (n < 0 || (n > 0 && (!cam_ids || !pt_ids || !uv))) return fail(g, GBA_ERR_INVALID_ARG, "bad edge arrays");
    if (!finite_all(uv, 2 * (size_t)n)) return fail(g, GBA_ERR_NONFINITE, "non-finite observation");
    if (info && !finite_all(info, 3 * (size_t)n)) return fail(g, GBA_ERR_NONFINITE, "non-finite information");
    if (info) {
        for (int64_t k = 0; k < n; ++k) {
            const double o00 = info[3 * k], o01 = info[3 * k + 1], o11 = info[3 * k + 2];
            if (!(o00 > 0.0) || !(o00 * o11 - o01 * o01 > 0.0))
                return fail(g, GBA_ERR_INVALID_ARG, "information matrix not positive definite at edge " +
                                                        std::to_string(g->e_cam.size() + k));
        }
    }
    if ((int64_t)g->e_cam.size() + n > std::numeric_limits<int>::max() / 32)
        return fail(g, GBA_ERR_UNSUPPORTED, "too many edges");
    std::vector<int> ci(n), pi(n);
    for (int64_t k = 0; k < n; ++k) {
        auto a = g->cam_map.find(cam_ids[k]);
        if (a == g->cam_map.end()) return fail(g, GBA_ERR_UNKNOWN_ID, "unknown camera id " + std::to_string(cam_ids[k]));
        auto b = g->pt_map.find(pt_ids[k]);
        if (b == g->pt_map.end()) return fail(g, GBA_ERR_UNKNOWN_ID, "unknown point id " + std::to_string(pt_ids[k]));
        ci[k] = a->second;
        pi[k] = b->second;
    }
    if (info && !g->any_info) {
        // earlier edges had the identity
        g->e_info.assign(3 * g->e_cam.size(), 0.0);
        for (size_t e = 0; e < g->e_cam.size(); ++e) {
            g->e_info[3 * e] = 1.0;
            g->e_info[3 * e + 2] = 1.0;
        }
        g->any_info = true;
    }
    g->e_cam.insert(g->e_cam.end(), ci.begin(), ci.end());
    g->e_pt.insert(g->e_pt.end(), pi.begin(), pi.end());
    g->e_uv.insert(g->e_uv.end(), uv, uv + 2 * n);
    g->e_active.insert(g->e_active.end(), (size_t)n, 1);
    if (g->any_info) {
        if (info)
            g->e_info.insert(g->e_info.end(), info, info + 3 * n);
        else
            for (int64_t k = 0; k < n; ++k) {
                g->e_info.push_back(1.0);
                g->e_info.push_back(0.0);
                g->e_info.push_back(1.0);
            }
    }
    g->dirty = true;
    return GBA_OK;
}

gba_status gba_set_fixed(gba_graph* g, int kind, int64_t id, int fixed) {
    if (!g || (kind != 0 && kind != 1)) return fail(g, GBA_ERR_INVALID_ARG, "kind must be 0 or 1");
    auto& map = kind == 0 ? g->cam_map : g->pt_map;
    auto it = map.find(id);
    if (it == map.end()) return fail(g, GBA_ERR_UNKNOWN_ID, "unknown vertex id " + std::to_string(id));
    auto& f = kind == 0 ? g->cam_fixed : g->pt_fixed;
    const unsigned char v = fixed ? 1 : 0;
    if (f[it->second] != v) {
        gba_status st = sync_params_to_host(g);
        if (st != GBA_OK) return st;
        f[it->second] = v;
        g->dirty = true;
    }
    return GBA_OK;
}

gba_status gba_set_edge_active(gba_graph* g, int64_t edge_index, int active) {
    if (!g || edge_index < 0 || edge_index >= (int64_t)g->e_cam.size())
        return fail(g, GBA_ERR_INVALID_ARG, "edge index out of range");
    const unsigned char v = active ? 1 : 0;
    if (g->e_active[edge_index] != v) {
        gba_status st = sync_params_to_host(g);
        if (st != GBA_OK) return st;
        g->e_active[edge_index] = v;
        g->dirty = true;
    }
    return GBA_OK;
}

gba_status gba_set_robust_kernel(gba_graph* g, gba_loss loss, double delta) {
    if (!g || (loss != GBA_LOSS_SQUARED && loss != GBA_LOSS_HUBER))
        return fail(g, GBA_ERR_INVALID_ARG, "unknown loss");
    if (loss == GBA_LOSS_HUBER && !(delta > 0.0 && std::isfinite(delta)))
        return fail(g, GBA_ERR_INVALID_ARG, "Huber delta must be positive and finite");
    g->loss = loss;
    g->delta = loss == GBA_LOSS_HUBER ? delta : 1.0;
    g->dg.loss = g->loss;
    g->dg.delta = g->delta;
    return GBA_OK;
}

gba_status gba_set_options(gba_graph* g, const gba_options* o) {
    if (!g || !o) return fail(g, GBA_ERR_INVALID_ARG, "null options");
    if (!(o->initial_lambda > 0.0) || !(o->min_diag > 0.0) || !(o->max_diag >= o->min_diag) ||
        o->pcg_max_iters < 1 || !(o->pcg_tol >= 0.0) ||
        (o->precond != GBA_PRECOND_IDENTITY && o->precond != GBA_PRECOND_BLOCK_JACOBI))
        return fail(g, GBA_ERR_INVALID_ARG, "invalid option value");
    g->opts = *o;
    return GBA_OK;
}

gba_status gba_prepare(gba_graph* g) {
    if (!g) return GBA_ERR_INVALID_ARG;
    return ensure_built(g);
}

gba_status gba_solve(gba_graph* g, int max_iters, double tol, gba_report* report) {
    if (!g || max_iters < 0 || !(tol >= 0.0)) return fail(g, GBA_ERR_INVALID_ARG, "bad solve arguments");
    auto t_start = std::chrono::steady_clock::now();
    HIP_TRY(g, hipSetDevice(g->device));
    gba_status st = ensure_built(g);
    if (st != GBA_OK) return st;
    gba_report rep;
    std::memset(&rep, 0, sizeof(rep));
    rep.workspace_bytes = g->arena_bytes;
    g->trials.clear();
    DeviceGraph& d = g->dg;
    const gba_options& o = g->opts;

    Timers tm;
    tm.on = o.timing != 0;
    if (tm.on) {
        tm.ev.resize(4 + 2 * 8);
        for (auto& e : tm.ev) HIP_TRY(g, hipEventCreate(&e));
    }
    struct EvGuard {
        Timers* t;
        ~EvGuard() {
            for (auto& e : t->ev) (void)hipEventDestroy(e);
        }
    } guard{&tm};

    double F = 0.0;
    if (d.ne > 0) {
        st = eval_cost(g, d.cam, d.pt, &F);
        if (st != GBA_OK) return st;
    }
    rep.initial_cost = F;
    rep.final_cost = F;
    rep.final_lambda = o.initial_lambda;
    if (d.ne == 0 || !has_free_vertex(g) || max_iters == 0) {
        rep.termination = (d.ne == 0 || !has_free_vertex(g)) ? GBA_TERM_NO_WORK : GBA_TERM_MAX_ITERS;
    } else if (!std::isfinite(F)) {
        rep.termination = GBA_TERM_NUMERICAL_FAILURE;
    } else {
        double ms_phase[3] = {0, 0, 0};
        double ms_lin = 0.0;
        auto timed_linearize = [&]() -> gba_status {
            hipEvent_t a = nullptr, b = nullptr;
            if (tm.on) {
                a = tm.ev[0];
                b = tm.ev[1];
                HIP_TRY(g, hipEventRecord(a, g->stream));
            }
            gba_status s2 = linearize(g, nullptr);
            if (s2 != GBA_OK) return s2;
            if (tm.on) {
                HIP_TRY(g, hipEventRecord(b, g->stream));
                HIP_TRY(g, hipEventSynchronize(b));
                float ms = 0.f;
                HIP_TRY(g, hipEventElapsedTime(&ms, a, b));
                ms_lin += ms;
            }
            return GBA_OK;
        };
        st = timed_linearize();
        if (st != GBA_OK) return st;
        double lam = o.initial_lambda, nu = 2.0;
        int term = GBA_TERM_MAX_ITERS;
        for (int trial = 0; trial < max_iters; ++trial) {
            st = damped_step(g, lam, &tm, ms_phase);
            if (st != GBA_OK) return st;
            const gba::TrialScalars& sc = *g->h_scal;
            const double Fn = sc.cost;
            const double L = -(sc.b_dot_dx + 0.5 * sc.quad);
            const double dnorm = std::sqrt(sc.step2), xnorm = std::sqrt(sc.x2);
            const bool accepted = (L > 0.0) && (Fn < F);
            const double gain = L != 0.0 ? (F - Fn) / L : std::numeric_limits<double>::quiet_NaN();
            gba_trial tr;
            tr.cost = F;
            tr.candidate_cost = Fn;
            tr.lambda = lam;
            tr.model_decrease = L;
            tr.step_norm = dnorm;
            tr.accepted = accepted ? 1 : 0;
            tr.pcg_iters = sc.pcg_iters;
            g->trials.push_back(tr);
            rep.pcg_iters_total += sc.pcg_iters;
            int stop = 0;
            if (accepted) {
                const double rel = (F - Fn) / F;
                std::swap(d.cam, d.cam_c);
                std::swap(d.pt, d.pt_c);
                F = Fn;
                const double t3 = 2.0 * gain - 1.0;
                lam *= std::max(1.0 / 3.0, 1.0 - t3 * t3 * t3);
                nu = 2.0;
                rep.accepted += 1;
                if (rel < tol) stop = GBA_TERM_COST_TOL;
            } else {
                lam *= nu;
                nu *= 2.0;
            }
            if (!stop && dnorm <= tol * (xnorm + tol)) stop = GBA_TERM_STEP_TOL;
            if (!stop && lam > 1e32) stop = GBA_TERM_LAMBDA_OVERFLOW;
            if (stop) {
                term = stop;
                break;
            }
            if (accepted) {
                st = timed_linearize();
                if (st != GBA_OK) return st;
            }
        }
        rep.trials = (int)g->trials.size();
        rep.termination = term;
        rep.final_cost = F;
        rep.final_lambda = lam;
        rep.ms_linearize = ms_lin;
        rep.ms_precond = ms_phase[0];
        rep.ms_pcg = ms_phase[1];
        rep.ms_other = ms_phase[2];
        rep.ms_matvec = tm.ms_mv;
        rep.matvec_count = tm.n_mv;
    }
    HIP_TRY(g, hipStreamSynchronize(g->stream));
    rep.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (report) *report = rep;
    return GBA_OK;
}

gba_status gba_reset(gba_graph* g) {
    if (!g) return GBA_ERR_INVALID_ARG;
    HIP_TRY(g, hipSetDevice(g->device));
    if (!g->built || g->dirty) {
        g->cam_params = g->cam_init;
        g->pt_params = g->pt_init;
        if (g->built) {
            // rebuild picks up the host values; do not pull device values back
            g->built = false;
            release_device(g);
            g->dirty = true;
        }
        return GBA_OK;
    }
    const DeviceGraph& d = g->dg;
    HIP_TRY(g, hipMemcpyAsync(d.cam, d.cam_init, sizeof(double) * 9 * d.nc, hipMemcpyDeviceToDevice, g->stream));
    HIP_TRY(g, hipMemcpyAsync(d.pt, d.pt_init, sizeof(double) * 3 * d.np, hipMemcpyDeviceToDevice, g->stream));
    HIP_TRY(g, hipStreamSynchronize(g->stream));
    return GBA_OK;
}

gba_status gba_get_cost(gba_graph* g, double* cost) {
    if (!g || !cost) return fail(g, GBA_ERR_INVALID_ARG, "null output");
    HIP_TRY(g, hipSetDevice(g->device));
    gba_status st = ensure_built(g);
    if (st != GBA_OK) return st;
    if (g->dg.ne == 0) {
        *cost = 0.0;
        return GBA_OK;
    }
    return eval_cost(g, g->dg.cam, g->dg.pt, cost);
}

gba_status gba_get_cameras(gba_graph* g, double* out) {
    if (!g || (!out && !g->cam_ids.empty())) return fail(g, GBA_ERR_INVALID_ARG, "null output");
    if (!g->built) {
        std::memcpy(out, g->cam_params.data(), sizeof(double) * g->cam_params.size());
        return GBA_OK;
    }
    HIP_TRY(g, hipSetDevice(g->device));
    HIP_TRY(g, hipMemcpyAsync(out, g->dg.cam, sizeof(double) * 9 * g->dg.nc, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(g, hipStreamSynchronize(g->stream));
    return GBA_OK;
}

gba_status gba_get_points(gba_graph* g, double* out) {
    if (!g || (!out && !g->pt_ids.empty())) return fail(g, GBA_ERR_INVALID_ARG, "null output");
    if (!g->built) {
        std::memcpy(out, g->pt_params.data(), sizeof(double) * g->pt_params.size());
        return GBA_OK;
    }
    HIP_TRY(g, hipSetDevice(g->device));
    HIP_TRY(g, hipMemcpyAsync(out, g->dg.pt, sizeof(double) * 3 * g->dg.np, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(g, hipStreamSynchronize(g->stream));
    return GBA_OK;
}

gba_status gba_get_trials(gba_graph* g, int max_entries, gba_trial* out, int* n_out) {
    if (!g || max_entries < 0 || (max_entries > 0 && !out)) return fail(g, GBA_ERR_INVALID_ARG, "bad arguments");
    const int n = std::min(max_entries, (int)g->trials.size());
    for (int k = 0; k < n; ++k) out[k] = g->trials[k];
    if (n_out) *n_out = (int)g->trials.size();
    return GBA_OK;
}

// ---- step-level entry points -------------------------------------------
gba_status gba_eval_edges(gba_graph* g, double* r, double* jc, double* jp, double* w) {
    if (!g) return GBA_ERR_INVALID_ARG;
    HIP_TRY(g, hipSetDevice(g->device));
    gba_status st = ensure_built(g);
    if (st != GBA_OK) return st;
    const DeviceGraph& d = g->dg;
    const size_t ne = d.ne, nall = g->e_cam.size();
    if (r) std::memset(r, 0, sizeof(double) * 2 * nall);
    if (jc) std::memset(jc, 0, sizeof(double) * 18 * nall);
    if (jp) std::memset(jp, 0, sizeof(double) * 6 * nall);
    if (w) std::memset(w, 0, sizeof(double) * nall);
    if (ne == 0) return GBA_OK;
    double* buf = (double*)dev_alloc(g, sizeof(double) * 27 * ne);
    if (!buf) return fail(g, GBA_ERR_OOM, "scratch allocation failed");
    gba::RawOut raw{buf, buf + 2 * ne, buf + 20 * ne, buf + 26 * ne};
    std::vector<double> h(27 * ne);
    hipError_t e1 = gba::launch_linearize(d, g->stream, &raw);
    hipError_t e2 = e1 == hipSuccess ? hipMemcpyAsync(h.data(), buf, sizeof(double) * 27 * ne,
                                                        hipMemcpyDeviceToHost, g->stream)
                                     : e1;
    hipError_t e3 = hipStreamSynchronize(g->stream);
    dev_free(g, buf);
    if (e2 != hipSuccess || e3 != hipSuccess)
        return fail(g, GBA_ERR_HIP, std::string("eval_edges: ") + hipGetErrorString(e2 != hipSuccess ? e2 : e3));
    for (size_t q = 0; q < ne; ++q) {
        const size_t e = (size_t)g->pm_edge[q];
        if (r) {
            r[2 * e] = h[q];
            r[2 * e + 1] = h[ne + q];
        }
        if (jc)
            for (int k = 0; k < 18; ++k) jc[18 * e + k] = h[(2 + k) * ne + q];
        if (jp)
            for (int k = 0; k < 6; ++k) jp[6 * e + k] = h[(20 + k) * ne + q];
        if (w) w[e] = h[26 * ne + q];
    }
    return GBA_OK;
}

gba_status gba_eval_normal_equations(gba_graph* g, double* hcc, double* bc, double* hpp, double* bp) {
    if (!g) return GBA_ERR_INVALID_ARG;
    HIP_TRY(g, hipSetDevice(g->device));
    gba_status st = ensure_built(g);
    if (st != GBA_OK) return st;
    const DeviceGraph& d = g->dg;
    if (d.ne > 0) {
        st = linearize(g, nullptr);
        if (st != GBA_OK) return st;
    }
    std::vector<double> H, B, HP, BP;
    if (d.ne > 0) {
        if ((st = download_typed(g, d.hcc, 45 * (size_t)d.nc, H)) != GBA_OK) return st;
        if ((st = download_typed(g, d.bc, 9 * (size_t)d.nc, B)) != GBA_OK) return st;
        if ((st = download_typed(g, d.hpp, 6 * (size_t)d.np, HP)) != GBA_OK) return st;
        if ((st = download_typed(g, d.bp, 3 * (size_t)d.np, BP)) != GBA_OK) return st;
    } else {
        H.assign(45 * (size_t)d.nc, 0.0);
        B.assign(9 * (size_t)d.nc, 0.0);
        HP.assign(6 * (size_t)d.np, 0.0);
        BP.assign(3 * (size_t)d.np, 0.0);
    }
    for (int i = 0; i < d.nc; ++i) {
        if (hcc)
            for (int a = 0; a < 9; ++a)
                for (int b = 0; b < 9; ++b) hcc[81 * (size_t)i + 9 * a + b] = H[45 * (size_t)i + gba::sym9(a, b)];
        if (bc)
            for (int a = 0; a < 9; ++a) bc[9 * (size_t)i + a] = B[9 * (size_t)i + a];
    }
    for (int j = 0; j < d.np; ++j) {
        if (hpp)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) hpp[9 * (size_t)j + 3 * a + b] = HP[gba::sym3(a, b) * (size_t)d.np + j];
        if (bp)
            for (int a = 0; a < 3; ++a) bp[3 * (size_t)j + a] = BP[a * (size_t)d.np + j];
    }
    return GBA_OK;
}

gba_status gba_eval_step(gba_graph* g, double lambda, double* dcam, double* dpt, int* pcg_iters) {
    if (!g || !(lambda > 0.0)) return fail(g, GBA_ERR_INVALID_ARG, "lambda must be positive");
    HIP_TRY(g, hipSetDevice(g->device));
    gba_status st = ensure_built(g);
    if (st != GBA_OK) return st;
    const DeviceGraph& d = g->dg;
    if (d.ne == 0) {
        if (dcam) std::memset(dcam, 0, sizeof(double) * 9 * d.nc);
        if (dpt) std::memset(dpt, 0, sizeof(double) * 3 * d.np);
        if (pcg_iters) *pcg_iters = 0;
        return GBA_OK;
    }
    if ((st = linearize(g, nullptr)) != GBA_OK) return st;
    if ((st = damped_step(g, lambda, nullptr, nullptr)) != GBA_OK) return st;
    std::vector<double> x;
    if ((st = download_typed(g, d.v_x, 9 * (size_t)d.nc, x)) != GBA_OK) return st;
    if (dpt) {
        HIP_TRY(g, hipMemcpyAsync(dpt, d.dpt, sizeof(double) * 3 * d.np, hipMemcpyDeviceToHost, g->stream));
        HIP_TRY(g, hipStreamSynchronize(g->stream));
    }
    if (dcam)
        for (int i = 0; i < d.nc; ++i)
            for (int a = 0; a < 9; ++a) dcam[9 * (size_t)i + a] = g->cam_fixed[i] ? 0.0 : x[9 * (size_t)i + a];
    if (pcg_iters) *pcg_iters = g->h_scal->pcg_iters;
    return GBA_OK;
}

const char* gba_last_error(const gba_graph* g) {
    if (!g) return "null graph handle";
    return g->err.c_str();
}

void gba_destroy(gba_graph* g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    release_device(g);
    if (g->h_scal) (void)hipHostFree(g->h_scal);
    if (g->h_pcg) (void)hipHostFree(g->h_pcg);
    delete g;
}

}  // extern "C"
