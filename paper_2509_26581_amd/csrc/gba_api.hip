// C ABI of the graph solver: vertex / edge staging, one device batch holding
// this single problem (gba_host.hip builds it and drives Levenberg-Marquardt),
// and the step-level evaluation entry points used for parity testing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "gba.h"
#include "gba_host.h"
#include "gba_internal.h"

using gba::DeviceGraph;

// Scratch of gba_eval_edges_noalloc: a fixed device array (one copy per GPU,
// held until the process ends) for the per-edge outputs in the caller's
// layout (27 doubles per inserted edge) and the edge permutation (one int per
// active edge).  Host code never passes the array's name to a kernel or a
// copy: it uses the device address resolved per device by noalloc_scratch().
static __device__ __align__(256) double scratch[27 * (size_t)GBA_NOALLOC_MAX_EDGES +
                                                (size_t)GBA_NOALLOC_MAX_EDGES / 2];

struct gba_graph {
    int precision = 0;
    int device = 0;
    gba::Allocator allocator;
    hipStream_t stream = nullptr;
    gba_options opts{};
    int loss = GBA_LOSS_SQUARED;
    double delta = 1.0;
    gba::DeviceInfo dev;
    gba::Tuning tune;   // automatic decomposition sizes

    // host staging, insertion order
    std::vector<int64_t> cam_ids, pt_ids;
    std::unordered_map<int64_t, int> cam_map, pt_map;
    gba::HostProblem prob;

    // device state
    bool dirty = true;
    bool built = false;
    gba::Batch batch;

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

void release_device(gba_graph* g) {
    g->batch.release();
    g->built = false;
}

// Pull the current device parameters back into host staging (so a rebuild
// keeps the optimised values).
gba_status sync_params_to_host(gba_graph* g) {
    if (!g->built) return GBA_OK;
    gba_status st = gba::batch_download(g->batch, 0, g->prob.cam_params.data(),
                                        g->prob.pt_params.data(), g->err);
    return st;
}

gba_status build(gba_graph* g) {
    HIP_TRY(g, hipSetDevice(g->device));
    gba_status st = sync_params_to_host(g);
    if (st != GBA_OK) return st;
    release_device(g);
    std::vector<const gba::HostProblem*> probs{&g->prob};
    st = gba::build_batch(probs, g->precision, g->loss, g->delta, g->dev, g->tune, g->allocator,
                          g->stream, g->batch, g->err);
    if (st != GBA_OK) {
        release_device(g);
        return st;
    }
    g->batch.use_graphs = true;
    g->built = true;
    g->dirty = false;
    return GBA_OK;
}

gba_status ensure_built(gba_graph* g) {
    if (!g->dirty && g->built) return GBA_OK;
    return build(g);
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

std::mutex g_scratch_mu;
void* g_scratch_ptr[gba::kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), resolved
// once per device with hipGetSymbolAddress; null (and a message) on failure.
void* noalloc_scratch(int device, std::string& msg) {
    if (device < 0 || device >= gba::kMaxDevices) {
        msg = "device index beyond the scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}

void zero_edge_outputs(size_t nall, double* r, double* jc, double* jp, double* w) {
    if (r) std::memset(r, 0, sizeof(double) * 2 * nall);
    if (jc) std::memset(jc, 0, sizeof(double) * 18 * nall);
    if (jp) std::memset(jp, 0, sizeof(double) * 6 * nall);
    if (w) std::memset(w, 0, sizeof(double) * nall);
}

// Device scratch of the edge evaluation: r, jc, jp, w for every inserted edge
// (27 doubles; inactive ones stay 0) and the point-major -> insertion
// permutation of the active ones.
size_t edge_scratch_bytes(size_t nall, size_t ne) {
    return sizeof(double) * 27 * nall + sizeof(int) * ne;
}

// Linearise with the unweighted per-edge outputs written into `buf` (device,
// edge_scratch_bytes large) in the caller's layout, then copy each requested
// output straight into the caller's host array.  Issues work on g->stream and
// leaves it running (the caller synchronises).
gba_status eval_edges_into(gba_graph* g, void* buf, double* r, double* jc, double* jp, double* w) {
    const size_t ne = g->batch.dg.ne, nall = g->prob.e_cam.size();
    double* d = (double*)buf;
    double *dr = d, *djc = d + 2 * nall, *djp = d + 20 * nall, *dw = d + 26 * nall;
    int* dpos = (int*)(d + 27 * nall);
    HIP_TRY(g, gba::launch_fill_f64(d, 0.0, 27 * nall, g->stream));
    HIP_TRY(g, hipMemcpyAsync(dpos, g->batch.pm_edge[0].data(), sizeof(int) * ne, hipMemcpyHostToDevice,
                              g->stream));
    gba::RawOut raw{r ? dr : nullptr, jc ? djc : nullptr, jp ? djp : nullptr, w ? dw : nullptr, dpos};
    gba_status st = gba::batch_linearize(g->batch, &raw, nullptr, g->err);
    if (st != GBA_OK) return st;
    auto down = [&](double* host, const double* dev, size_t n) -> hipError_t {
        if (!host || n == 0) return hipSuccess;
        return hipMemcpyAsync(host, dev, sizeof(double) * n, hipMemcpyDeviceToHost, g->stream);
    };
    HIP_TRY(g, down(r, dr, 2 * nall));
    HIP_TRY(g, down(jc, djc, 18 * nall));
    HIP_TRY(g, down(jp, djp, 6 * nall));
    HIP_TRY(g, down(w, dw, nall));
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
    if (hipSetDevice(device) != hipSuccess) return GBA_ERR_HIP;
    gba_graph* g = new gba_graph();
    g->precision = precision;
    g->device = device;
    g->allocator.alloc = alloc;
    g->allocator.free_fn = free_fn;
    g->allocator.ctx = ctx;
    gba_default_options(&g->opts);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        g->dev.n_cu = prop.multiProcessorCount;
        g->dev.max_lds = prop.sharedMemPerBlock;
    }
    // set-up of the allocation-free entry point's scratch on this device (a
    // failure is reported by that entry point, not here)
    std::string msg;
    (void)noalloc_scratch(device, msg);
    *out = g;
    return GBA_OK;
}

gba_status gba_set_stream(gba_graph* g, void* hip_stream) {
    if (!g) return GBA_ERR_INVALID_ARG;
    if (g->built) HIP_TRY(g, hipStreamSynchronize(g->stream));
    g->stream = (hipStream_t)hip_stream;
    g->batch.stream = g->stream;
    g->batch.drop_graphs();   // graphs are replayed on the stream they were made for
    return GBA_OK;
}

gba_status gba_reserve(gba_graph* g, int64_t n_cams, int64_t n_pts, int64_t n_edges) {
    if (!g || n_cams < 0 || n_pts < 0 || n_edges < 0) return fail(g, GBA_ERR_INVALID_ARG, "negative size");
    gba::HostProblem& h = g->prob;
    g->cam_ids.reserve(n_cams);
    g->cam_map.reserve(n_cams);
    h.cam_params.reserve(9 * n_cams);
    h.cam_init.reserve(9 * n_cams);
    h.cam_fixed.reserve(n_cams);
    g->pt_ids.reserve(n_pts);
    g->pt_map.reserve(n_pts);
    h.pt_params.reserve(3 * n_pts);
    h.pt_init.reserve(3 * n_pts);
    h.pt_fixed.reserve(n_pts);
    h.e_cam.reserve(n_edges);
    h.e_pt.reserve(n_edges);
    h.e_uv.reserve(2 * n_edges);
    h.e_active.reserve(n_edges);
    return GBA_OK;
}

static gba_status add_vertices(gba_graph* g, int64_t n, const int64_t* ids, const double* v, int dim,
                               std::vector<int64_t>& idv, std::unordered_map<int64_t, int>& map,
                               std::vector<double>& par, std::vector<double>& init,
                               std::vector<unsigned char>& fixed) {
    if (!g || n < 0 || (n > 0 && (!ids || !v))) return fail(g, GBA_ERR_INVALID_ARG, "bad vertex arrays");
    if (!finite_all(v, (size_t)n * dim)) return fail(g, GBA_ERR_NONFINITE, "non-finite vertex parameters");
    if ((int64_t)idv.size() + n > std::numeric_limits<int>::max() / 16)
        return fail(g, GBA_ERR_UNSUPPORTED, "too many vertices");
    for (int64_t k = 0; k < n; ++k)
        if (map.count(ids[k])) return fail(g, GBA_ERR_DUPLICATE_ID, "duplicate vertex id " + std::to_string(ids[k]));
    {
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
    return add_vertices(g, n, ids, params, 9, g->cam_ids, g->cam_map, g->prob.cam_params,
                        g->prob.cam_init, g->prob.cam_fixed);
}

gba_status gba_add_points(gba_graph* g, int64_t n, const int64_t* ids, const double* xyz) {
    if (!g) return GBA_ERR_INVALID_ARG;
    return add_vertices(g, n, ids, xyz, 3, g->pt_ids, g->pt_map, g->prob.pt_params, g->prob.pt_init,
                        g->prob.pt_fixed);
}

gba_status gba_add_edges(gba_graph* g, int64_t n, const int64_t* cam_ids, const int64_t* pt_ids,
                         const double* uv, const double* info) {
    if (!g) return GBA_ERR_INVALID_ARG;
    gba::HostProblem& h = g->prob;
    if (n < 0 || (n > 0 && (!cam_ids || !pt_ids || !uv))) return fail(g, GBA_ERR_INVALID_ARG, "bad edge arrays");
    if (!finite_all(uv, 2 * (size_t)n)) return fail(g, GBA_ERR_NONFINITE, "non-finite observation");
    if (info && !finite_all(info, 3 * (size_t)n)) return fail(g, GBA_ERR_NONFINITE, "non-finite information");
    if (info) {
        for (int64_t k = 0; k < n; ++k) {
            const double o00 = info[3 * k], o01 = info[3 * k + 1], o11 = info[3 * k + 2];
            if (!(o00 > 0.0) || !(o00 * o11 - o01 * o01 > 0.0))
                return fail(g, GBA_ERR_INVALID_ARG, "information matrix not positive definite at edge " +
                                                        std::to_string(h.e_cam.size() + k));
        }
    }
    if ((int64_t)h.e_cam.size() + n > std::numeric_limits<int>::max() / 32)
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
    const bool had_info = !h.e_info.empty();
    if (info && !had_info) {
        // earlier edges had the identity
        h.e_info.assign(3 * h.e_cam.size(), 0.0);
        for (size_t e = 0; e < h.e_cam.size(); ++e) {
            h.e_info[3 * e] = 1.0;
            h.e_info[3 * e + 2] = 1.0;
        }
    }
    h.e_cam.insert(h.e_cam.end(), ci.begin(), ci.end());
    h.e_pt.insert(h.e_pt.end(), pi.begin(), pi.end());
    h.e_uv.insert(h.e_uv.end(), uv, uv + 2 * n);
    h.e_active.insert(h.e_active.end(), (size_t)n, 1);
    if (info || had_info) {
        if (info)
            h.e_info.insert(h.e_info.end(), info, info + 3 * n);
        else
            for (int64_t k = 0; k < n; ++k) {
                h.e_info.push_back(1.0);
                h.e_info.push_back(0.0);
                h.e_info.push_back(1.0);
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
    auto& f = kind == 0 ? g->prob.cam_fixed : g->prob.pt_fixed;
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
    if (!g || edge_index < 0 || edge_index >= (int64_t)g->prob.e_cam.size())
        return fail(g, GBA_ERR_INVALID_ARG, "edge index out of range");
    const unsigned char v = active ? 1 : 0;
    if (g->prob.e_active[edge_index] != v) {
        gba_status st = sync_params_to_host(g);
        if (st != GBA_OK) return st;
        g->prob.e_active[edge_index] = v;
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
    g->batch.dg.loss = g->loss;
    g->batch.dg.delta = g->delta;
    return GBA_OK;
}

gba_status gba_set_options(gba_graph* g, const gba_options* o) {
    if (!g || !o) return fail(g, GBA_ERR_INVALID_ARG, "null options");
    if (!(o->initial_lambda > 0.0) || !(o->min_diag > 0.0) || !(o->max_diag >= o->min_diag) ||
        o->pcg_max_iters < 1 || !(o->pcg_tol >= 0.0) ||
        (o->precond != GBA_PRECOND_IDENTITY && o->precond != GBA_PRECOND_BLOCK_JACOBI) ||
        o->accumulation < GBA_ACC_AUTO || o->accumulation > GBA_ACC_CAMERA_BLOCKS || o->tiles_per_block < 0 ||
        (o->deterministic != 0 && o->deterministic != 1) || (o->jacobi_scaling != 0 && o->jacobi_scaling != 1) ||
        o->pcg_schedule < GBA_PCG_AUTO || o->pcg_schedule > GBA_PCG_PERSISTENT ||
        o->jacobian < GBA_JACOBIAN_ANALYTIC || o->jacobian > GBA_JACOBIAN_DYNAMIC ||
        (o->solver != GBA_SOLVER_SCHUR && o->solver != GBA_SOLVER_FULL))
        return fail(g, GBA_ERR_INVALID_ARG, "invalid option value");
    if (o->jacobian == GBA_JACOBIAN_DYNAMIC && o->solver != GBA_SOLVER_FULL)
        return fail(g, GBA_ERR_INVALID_ARG, "dynamic Jacobians need the full-Hessian solver");
    if (o->solver == GBA_SOLVER_FULL && (o->deterministic || o->accumulation == GBA_ACC_CAMERA_PASS ||
                                         o->accumulation == GBA_ACC_CAMERA_BLOCKS))
        return fail(g, GBA_ERR_INVALID_ARG,
                    "the full-Hessian solver sums the camera rows in LDS (no fixed-order mode)");
    if (o->deterministic && o->accumulation == GBA_ACC_LDS)
        return fail(g, GBA_ERR_INVALID_ARG,
                    "deterministic sums use the camera-major pass; GBA_ACC_LDS combines LDS partials by atomics");
    if (o->accumulation != g->tune.accumulation || o->tiles_per_block != g->tune.tiles_per_block ||
        o->deterministic != g->tune.deterministic || o->solver != g->tune.solver ||
        (o->jacobian == GBA_JACOBIAN_DYNAMIC) != (g->tune.dynamic != 0)) {
        // all three are part of the device graph's plan
        gba_status st = sync_params_to_host(g);
        if (st != GBA_OK) return st;
        g->tune.accumulation = o->accumulation;
        g->tune.tiles_per_block = o->tiles_per_block;
        g->tune.deterministic = o->deterministic;
        g->tune.solver = o->solver;
        g->tune.dynamic = o->jacobian == GBA_JACOBIAN_DYNAMIC ? 1 : 0;
        g->dirty = true;
    }
    g->opts = *o;
    g->batch.jacobian = o->jacobian;
    return GBA_OK;
}

gba_status gba_prepare(gba_graph* g) {
    if (!g) return GBA_ERR_INVALID_ARG;
    HIP_TRY(g, hipSetDevice(g->device));
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
    rep.workspace_bytes = g->batch.arena_bytes;
    g->trials.clear();
    const gba_options& o = g->opts;

    gba::Timers tm;
    tm.on = o.timing != 0;
    if (tm.on) HIP_TRY(g, tm.init());
    std::vector<const gba::HostProblem*> probs{&g->prob};
    std::vector<gba::ProblemLM> lm(1);
    lm[0].max_iters = max_iters;
    lm[0].tol = tol;
    st = gba::batch_begin(g->batch, probs, lm, std::vector<char>(1, 1), o, &tm, g->err);
    if (st != GBA_OK) return st;
    while (lm[0].running) {
        st = gba::batch_trial(g->batch, lm, o, g->tune, &tm, g->err);
        if (st != GBA_OK) return st;
    }
    const gba::ProblemLM& s = lm[0];
    g->trials = s.log;
    rep.initial_cost = s.F0;
    rep.final_cost = s.F;
    rep.final_lambda = s.lam;
    rep.trials = s.trials;
    rep.accepted = s.accepted;
    rep.pcg_iters_total = s.pcg_total;
    rep.termination = s.term;
    rep.ms_linearize = tm.ms_phase[0];
    rep.ms_precond = tm.ms_phase[1];
    rep.ms_pcg = tm.ms_phase[2];
    rep.ms_other = tm.ms_phase[3];
    rep.ms_matvec = tm.ms_mv;
    rep.matvec_count = tm.n_mv;
    HIP_TRY(g, hipStreamSynchronize(g->stream));
    rep.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (report) *report = rep;
    return GBA_OK;
}

gba_status gba_reset(gba_graph* g) {
    if (!g) return GBA_ERR_INVALID_ARG;
    HIP_TRY(g, hipSetDevice(g->device));
    if (!g->built || g->dirty) {
        g->prob.cam_params = g->prob.cam_init;
        g->prob.pt_params = g->prob.pt_init;
        if (g->built) {
            // the rebuild takes the host values; do not pull device values back
            release_device(g);
            g->dirty = true;
        }
        return GBA_OK;
    }
    const DeviceGraph& d = g->batch.dg;
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
    if ((st = gba::batch_cost(g->batch, g->err)) != GBA_OK) return st;
    *cost = g->batch.h_scal[0].cost;
    return GBA_OK;
}

gba_status gba_get_cameras(gba_graph* g, double* out) {
    if (!g || (!out && !g->cam_ids.empty())) return fail(g, GBA_ERR_INVALID_ARG, "null output");
    if (!g->built) {
        std::memcpy(out, g->prob.cam_params.data(), sizeof(double) * g->prob.cam_params.size());
        return GBA_OK;
    }
    HIP_TRY(g, hipSetDevice(g->device));
    return gba::batch_download(g->batch, 0, out, nullptr, g->err);
}

gba_status gba_get_points(gba_graph* g, double* out) {
    if (!g || (!out && !g->pt_ids.empty())) return fail(g, GBA_ERR_INVALID_ARG, "null output");
    if (!g->built) {
        std::memcpy(out, g->prob.pt_params.data(), sizeof(double) * g->prob.pt_params.size());
        return GBA_OK;
    }
    HIP_TRY(g, hipSetDevice(g->device));
    return gba::batch_download(g->batch, 0, nullptr, out, g->err);
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
    const size_t ne = g->batch.dg.ne, nall = g->prob.e_cam.size();
    if (ne == 0) {
        zero_edge_outputs(nall, r, jc, jp, w);
        return GBA_OK;
    }
    // scratch: the outputs in the caller's layout and the edge permutation
    const size_t bytes = edge_scratch_bytes(nall, ne);
    void* buf = g->allocator.allocate(bytes);
    if (!buf) return fail(g, GBA_ERR_OOM, "scratch allocation failed");
    st = eval_edges_into(g, buf, r, jc, jp, w);
    hipError_t e3 = hipStreamSynchronize(g->stream);
    g->allocator.release(buf);
    if (st != GBA_OK) return st;
    if (e3 != hipSuccess) return fail(g, GBA_ERR_HIP, std::string("eval_edges: ") + hipGetErrorString(e3));
    return GBA_OK;
}

gba_status gba_eval_edges_noalloc(gba_graph* g, double* r, double* jc, double* jp, double* w) {
    if (!g) return GBA_ERR_INVALID_ARG;
    HIP_TRY(g, hipSetDevice(g->device));
    if (!g->built || g->dirty)
        return fail(g, GBA_ERR_STATE, "the graph is not on the device: call gba_prepare first");
    const size_t ne = g->batch.dg.ne, nall = g->prob.e_cam.size();
    if (nall > (size_t)GBA_NOALLOC_MAX_EDGES)
        return fail(g, GBA_ERR_UNSUPPORTED, "more than GBA_NOALLOC_MAX_EDGES (" +
                                                std::to_string(GBA_NOALLOC_MAX_EDGES) + ") edges");
    void* buf = noalloc_scratch(g->device, g->err);
    if (!buf) return GBA_ERR_HIP;
    if (ne == 0) {
        zero_edge_outputs(nall, r, jc, jp, w);
        return GBA_OK;
    }
    gba_status st = eval_edges_into(g, buf, r, jc, jp, w);
    hipError_t e3 = hipStreamSynchronize(g->stream);
    if (st != GBA_OK) return st;
    if (e3 != hipSuccess) return fail(g, GBA_ERR_HIP, std::string("eval_edges_noalloc: ") + hipGetErrorString(e3));
    return GBA_OK;
}

gba_status gba_eval_normal_equations(gba_graph* g, double* hcc, double* bc, double* hpp, double* bp) {
    if (!g) return GBA_ERR_INVALID_ARG;
    HIP_TRY(g, hipSetDevice(g->device));
    gba_status st = ensure_built(g);
    if (st != GBA_OK) return st;
    const DeviceGraph& d = g->batch.dg;
    std::vector<double> H, B, HP, BP;
    if (d.ne > 0) {
        if ((st = gba::batch_linearize(g->batch, nullptr, nullptr, g->err)) != GBA_OK) return st;
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
    const DeviceGraph& d = g->batch.dg;
    if (d.ne == 0) {
        if (dcam) std::memset(dcam, 0, sizeof(double) * 9 * d.nc);
        if (dpt) std::memset(dpt, 0, sizeof(double) * 3 * d.np);
        if (pcg_iters) *pcg_iters = 0;
        return GBA_OK;
    }
    if ((st = gba::batch_linearize(g->batch, nullptr, nullptr, g->err)) != GBA_OK) return st;
    g->batch.h_lam[0] = lambda;
    if ((st = gba::batch_damped_step(g->batch, g->opts, g->tune, nullptr, g->err)) != GBA_OK) return st;
    std::vector<double> x;
    if ((st = download_typed(g, d.v_x, 9 * (size_t)d.nc, x)) != GBA_OK) return st;
    if (dpt) {
        HIP_TRY(g, hipMemcpyAsync(dpt, d.dpt, sizeof(double) * 3 * d.np, hipMemcpyDeviceToHost, g->stream));
        HIP_TRY(g, hipStreamSynchronize(g->stream));
    }
    if (dcam)
        for (int i = 0; i < d.nc; ++i)
            for (int a = 0; a < 9; ++a)
                dcam[9 * (size_t)i + a] = g->prob.cam_fixed[i] ? 0.0 : x[9 * (size_t)i + a];
    if (pcg_iters) *pcg_iters = g->batch.h_scal[0].pcg_iters;
    return GBA_OK;
}

gba_status gba_time_matvec(gba_graph* g, double lambda, int launches, double* avg_us) {
    if (!g || !avg_us || !(lambda > 0.0) || launches < 1)
        return fail(g, GBA_ERR_INVALID_ARG, "lambda must be positive, launches >= 1");
    HIP_TRY(g, hipSetDevice(g->device));
    gba_status st = ensure_built(g);
    if (st != GBA_OK) return st;
    *avg_us = 0.0;
    if (g->batch.dg.ne == 0) return GBA_OK;
    if ((st = gba::batch_linearize(g->batch, nullptr, nullptr, g->err)) != GBA_OK) return st;
    g->batch.h_lam[0] = lambda;
    double ms = 0.0;
    if ((st = gba::batch_time_matvec(g->batch, g->opts, launches, &ms, g->err)) != GBA_OK) return st;
    *avg_us = ms * 1e3;
    return GBA_OK;
}

gba_status gba_hbm_probe(int device, const void* buf, size_t bytes, double* sink, int launches,
                         void* stream, double* avg_us) {
    if (!buf || !sink || !avg_us || bytes == 0 || bytes % 16 != 0 || launches < 1)
        return GBA_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return GBA_ERR_HIP;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return GBA_ERR_HIP;
    hipError_t r = hipEventCreate(&e1);
    if (r == hipSuccess) r = hipEventRecord(e0, s);
    for (int k = 0; k < launches && r == hipSuccess; ++k) r = gba::launch_hbm_probe(buf, bytes / 16, sink, s);
    if (r == hipSuccess) r = hipEventRecord(e1, s);
    if (r == hipSuccess) r = hipEventSynchronize(e1);
    float ms = 0.f;
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (r != hipSuccess) return GBA_ERR_HIP;
    *avg_us = 1e3 * (double)ms / launches;
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
    delete g;
}

}  // extern "C"
