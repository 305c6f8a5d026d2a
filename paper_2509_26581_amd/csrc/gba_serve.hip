// Serving loop: requests are validated and sorted on the caller's thread,
// admitted by slot count and device-memory budget, uploaded asynchronously
// into a resident device image, packed (device-side copy with index
// rebasing) into one batch, and solved by batched LM trials.  Finished
// problems leave the batch at the next trial boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gba.h"
#include "gba_host.h"
#include "gba_internal.h"
#include "gba_range.h"

namespace gba {
namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Byte offsets of the arrays of one problem's device image (the same layout
// is used for the pinned host copy that is uploaded).
struct ImageLayout {
    size_t e_cam, e_pt, obs, sinfo, tile_off, cm_run_off, cm_pt, cm_obs, cm_sinfo, chunk_run_off,
        chunk_cam, cam_chunk_off, cam_fixed, pt_fixed, cam_init, pt_init, cam_cur, pt_cur;
    size_t bytes;
};

ImageLayout image_layout(const ImageCounts& n) {
    ImageLayout L{};
    size_t off = 0;
    auto add = [&](size_t& slot, size_t b) {
        slot = off;
        off += align256(b ? b : 1);
    };
    const size_t ne = n.ne;
    add(L.e_cam, 4 * ne);
    add(L.e_pt, 4 * ne);
    add(L.obs, 16 * ne);
    add(L.sinfo, n.info ? 24 * ne : 0);
    add(L.tile_off, 4 * (size_t)(n.n_tiles + 1));
    add(L.cm_run_off, 4 * (size_t)(n.n_runs + 1));
    add(L.cm_pt, 4 * ne);
    add(L.cm_obs, 16 * ne);
    add(L.cm_sinfo, n.info ? 24 * ne : 0);
    add(L.chunk_run_off, 4 * (size_t)(n.n_chunks + 1));
    add(L.chunk_cam, 4 * (size_t)n.n_chunks);
    add(L.cam_chunk_off, 4 * (size_t)(n.nc + 1));
    add(L.cam_fixed, (size_t)n.nc);
    add(L.pt_fixed, (size_t)n.np);
    add(L.cam_init, 72 * (size_t)n.nc);
    add(L.pt_init, 24 * (size_t)n.np);
    add(L.cam_cur, 72 * (size_t)n.nc);
    add(L.pt_cur, 24 * (size_t)n.np);
    L.bytes = off;
    return L;
}

enum ReqState { kQueued = 0, kStaged = 1, kResident = 2, kDone = 3 };

struct Request {
    uint64_t ticket = 0;
    HostProblem prob;          // fixed masks only after the image is made
    ImageCounts counts;
    ImageLayout lay{};
    void* h_blob = nullptr;    // pinned host image
    size_t dev_off = 0;        // device image inside the arena
    hipEvent_t uploaded = nullptr;
    long long staged_step = -1;
    int max_iters = 0;
    double tol = 0.0;
    Clock::time_point t_submit, t_admit, t_done;
    ProblemLM lm;
    int state = kQueued;
    int batch_peak = 0;
    std::vector<double> cams_out, pts_out;
    gba_report rep{};
};

void read_tune_db(const char* path, int precision, Tuning& t, bool& ok) {
    ok = true;
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) {
        ok = false;
        return;
    }
    const char* pname = precision == GBA_FP64 ? "fp64" : (precision == GBA_MIXED_FP32 ? "fp32" : "bf16");
    const std::string pre = std::string(pname) + ".";
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        char key[128];
        long v = 0;
        if (std::sscanf(line, "%127s %ld", key, &v) != 2) continue;
        const std::string k(key);
        if (k.compare(0, pre.size(), pre) != 0 || v <= 0 || v > (1L << 24)) continue;
        const std::string name = k.substr(pre.size());
        if (name == "tiles_per_block") t.tiles_per_block = (int)v;
        else if (name == "edges_per_block") t.edges_per_block = (int)v;
        else if (name == "pts_per_block") t.pts_per_block = (int)v;
        else if (name == "pcg_sync_every") t.pcg_sync_every = (int)v;
    }
    std::fclose(f);
}

}  // namespace
}  // namespace gba

using namespace gba;

struct gba_server {
    gba_server_config cfg{};
    Allocator allocator;
    DeviceInfo dev;
    Tuning tune;
    hipStream_t stream = nullptr;  // batch work
    hipStream_t copy = nullptr;    // image uploads
    hipEvent_t ev_admit = nullptr;
    void* arena = nullptr;
    RangeAlloc ra;
    bool have_union = false;
    size_t union_off = 0, union_bytes = 0;
    size_t image_bytes_in_use = 0;
    Batch batch;
    std::vector<Request*> resident;   // batch order
    std::vector<ProblemLM> lm;        // batch order (live LM states)
    // descriptor staging for the pack kernel
    PackDesc* h_desc = nullptr;
    PackChunk* h_chunk = nullptr;
    PackDesc* d_desc = nullptr;
    PackChunk* d_chunk = nullptr;
    size_t desc_cap = 0, chunk_cap = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::vector<Request*> staged;
    std::unordered_map<uint64_t, Request*> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool failed = false;
    std::string thread_err;
    std::string err;
    std::thread worker;
    long long step = 0;

    // statistics (under mu)
    long long submitted = 0, admitted = 0, rejected = 0, completed = 0, collected = 0;
    long long trials_run = 0, repacks = 0, batch_sum = 0;
    std::vector<double> lat_ms, svc_ms;
    bool any_submit = false;
    Clock::time_point t_first_submit, t_last_done;
    size_t bytes_peak = 0;

    void run();
    gba_status admit_locked(std::vector<Request*>& newly);
    bool fits_locked(const Request* r, size_t& img_off);
    gba_status upload(Request* r);
    gba_status repack();
    gba_status collect_finished();
    gba_status ensure_desc(size_t nd, size_t nch);
    gba_status launch_descs(const std::vector<PackDesc>& descs);
    size_t union_bytes_for(const std::vector<const ImageCounts*>& c);
    size_t bytes_in_use() const { return image_bytes_in_use + (have_union ? union_bytes : 0); }
};

namespace {

gba_status fail_s(gba_server* s, gba_status code, const std::string& msg) {
    if (s) s->err = msg;
    return code;
}

#define HIP_S(s, call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            (s)->err = std::string(#call) + ": " + hipGetErrorString(e_);                \
            return GBA_ERR_HIP;                                                           \
        }                                                                                 \
    } while (0)

}  // namespace

size_t gba_server::union_bytes_for(const std::vector<const ImageCounts*>& c) {
    UnionPlan u;
    std::string m;
    if (c.empty()) return 0;
    if (plan_union(c, tune, dev, cfg.precision, u, m) != GBA_OK) return std::numeric_limits<size_t>::max();
    return align256(layout_union(u, cfg.precision, nullptr, nullptr));
}

// Can r join now?  Simulates the image allocation and the grown batch
// workspace on a copy of the range allocator.
bool gba_server::fits_locked(const Request* r, size_t& img_off) {
    if ((int)(resident.size() + staged.size()) >= cfg.max_slots) return false;
    std::vector<const ImageCounts*> c;
    for (Request* q : resident)
        if (q && q->state == kResident) c.push_back(&q->counts);
    for (Request* q : staged) c.push_back(&q->counts);
    c.push_back(&r->counts);
    const size_t ub = union_bytes_for(c);
    if (ub == std::numeric_limits<size_t>::max()) return false;
    return simulate_admission(ra, have_union, union_off, union_bytes, r->lay.bytes, ub, img_off);
}

gba_status gba_server::admit_locked(std::vector<Request*>& newly) {
    while (!queue.empty()) {
        Request* r = queue.front();
        size_t off = 0;
        if (!fits_locked(r, off)) break;
        size_t got = 0;
        if (!ra.alloc_low(r->lay.bytes, got) || got != off) {
            err = "internal: image allocation mismatch";
            return GBA_ERR_STATE;
        }
        queue.pop_front();
        r->dev_off = got;
        r->state = kStaged;
        r->staged_step = step;
        r->t_admit = Clock::now();
        image_bytes_in_use += r->lay.bytes;
        staged.push_back(r);
        newly.push_back(r);
        admitted += 1;
    }
    return GBA_OK;
}

gba_status gba_server::upload(Request* r) {
    // the image range may have been read by earlier batch work: order the
    // copy after everything issued so far on the batch stream
    HIP_S(this, hipEventRecord(ev_admit, stream));
    HIP_S(this, hipStreamWaitEvent(copy, ev_admit, 0));
    HIP_S(this, hipMemcpyAsync((char*)arena + r->dev_off, r->h_blob, r->lay.bytes,
                               hipMemcpyHostToDevice, copy));
    HIP_S(this, hipEventRecord(r->uploaded, copy));
    return GBA_OK;
}

gba_status gba_server::ensure_desc(size_t nd, size_t nch) {
    if (nd <= desc_cap && nch <= chunk_cap) return GBA_OK;
    HIP_S(this, hipStreamSynchronize(stream));
    const size_t dc = std::max(nd, 2 * desc_cap), cc = std::max(nch, 2 * chunk_cap);
    if (h_desc) (void)hipHostFree(h_desc);
    if (h_chunk) (void)hipHostFree(h_chunk);
    if (d_desc) (void)hipFree(d_desc);
    if (d_chunk) (void)hipFree(d_chunk);
    h_desc = nullptr;
    h_chunk = nullptr;
    d_desc = nullptr;
    d_chunk = nullptr;
    desc_cap = chunk_cap = 0;
    HIP_S(this, hipHostMalloc((void**)&h_desc, sizeof(PackDesc) * dc, hipHostMallocDefault));
    HIP_S(this, hipHostMalloc((void**)&h_chunk, sizeof(PackChunk) * cc, hipHostMallocDefault));
    HIP_S(this, hipMalloc((void**)&d_desc, sizeof(PackDesc) * dc));
    HIP_S(this, hipMalloc((void**)&d_chunk, sizeof(PackChunk) * cc));
    desc_cap = dc;
    chunk_cap = cc;
    return GBA_OK;
}

// Upload descriptors and launch the pack kernel on the batch stream, then
// wait for it (the pinned staging is reused by the next call).
gba_status gba_server::launch_descs(const std::vector<PackDesc>& descs) {
    size_t nch = 0;
    for (const PackDesc& d : descs) nch += (size_t)((d.n + kPackChunk - 1) / kPackChunk);
    if (nch == 0) return GBA_OK;
    if (nch > (size_t)std::numeric_limits<int>::max()) return fail_s(this, GBA_ERR_UNSUPPORTED, "pack too large");
    gba_status st = ensure_desc(descs.size(), nch);
    if (st != GBA_OK) return st;
    size_t c = 0;
    for (size_t k = 0; k < descs.size(); ++k) {
        h_desc[k] = descs[k];
        for (long long b = 0; b < descs[k].n; b += kPackChunk) h_chunk[c++] = PackChunk{(int)k, (int)b};
    }
    HIP_S(this, hipMemcpyAsync(d_desc, h_desc, sizeof(PackDesc) * descs.size(), hipMemcpyHostToDevice, stream));
    HIP_S(this, hipMemcpyAsync(d_chunk, h_chunk, sizeof(PackChunk) * nch, hipMemcpyHostToDevice, stream));
    HIP_S(this, launch_pack(d_desc, d_chunk, (int)nch, stream));
    HIP_S(this, hipStreamSynchronize(stream));
    return GBA_OK;
}

// Rebuild the batch: continuing problems keep their current parameters
// (saved into their images first), staged problems whose upload was issued
// before this step join, finished problems are gone.
gba_status gba_server::repack() {
    const DeviceGraph old = batch.dg;
    const UnionPlan old_plan = batch.plan;
    std::vector<Request*> keep;
    std::vector<PackDesc> descs;
    for (size_t p = 0; p < resident.size(); ++p) {
        Request* r = resident[p];
        if (!r || r->state != kResident) continue;   // finished (collected or not)
        r->lm = lm[p];
        char* base = (char*)arena + r->dev_off;
        const int co = old_plan.cam_off[p], po = old_plan.pt_off[p];
        if (r->counts.nc)
            descs.push_back(PackDesc{old.cam + 9 * (size_t)co, base + r->lay.cam_cur,
                                     9LL * r->counts.nc, 0, kPackF64, 0.0});
        if (r->counts.np)
            descs.push_back(PackDesc{old.pt + 3 * (size_t)po, base + r->lay.pt_cur,
                                     3LL * r->counts.np, 0, kPackF64, 0.0});
        keep.push_back(r);
    }
    gba_status st = launch_descs(descs);
    if (st != GBA_OK) return st;
    // joiners: uploads issued at an earlier step, or any when nothing else runs
    std::vector<Request*> join, wait_more;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (Request* r : staged) {
            if (r->staged_step < step || keep.empty())
                join.push_back(r);
            else
                wait_more.push_back(r);
        }
        staged = wait_more;
    }
    std::vector<Request*> order = keep;
    order.insert(order.end(), join.begin(), join.end());
    {
        std::lock_guard<std::mutex> lk(mu);
        if (have_union) {
            ra.release(union_off, union_bytes);
            have_union = false;
            union_bytes = 0;
        }
    }
    resident = order;
    lm.assign(order.size(), ProblemLM{});
    batch.P = 0;
    if (order.empty()) return GBA_OK;
    std::vector<const ImageCounts*> counts;
    for (Request* r : order) counts.push_back(&r->counts);
    st = plan_union(counts, tune, dev, cfg.precision, batch.plan, err);
    if (st != GBA_OK) return st;
    const UnionPlan& u = batch.plan;
    const size_t ub = align256(layout_union(u, cfg.precision, nullptr, nullptr));
    size_t uo = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!ra.alloc_high(ub, uo))
            return fail_s(this, GBA_ERR_STATE, "internal: batch workspace does not fit");
        have_union = true;
        union_off = uo;
        union_bytes = ub;
        bytes_peak = std::max(bytes_peak, bytes_in_use());
    }
    if ((st = batch.ensure_mirrors(std::max<int>(cfg.max_slots, (int)order.size()), err)) != GBA_OK) return st;
    batch.dg = DeviceGraph{};
    batch.blocks_zeroed = false;
    batch.persistent_ok = -1;
    batch.jacobian = cfg.options.jacobian;
    layout_union(u, cfg.precision, (char*)arena + uo, &batch.dg);
    batch.dg.bo_chunks = 0;   // the packed batch takes the camera-major pass
    batch.dg.bo_nblk = 0;
    set_union_scalars(batch, cfg.precision, cfg.loss, cfg.delta);
    batch.arena = (char*)arena + uo;
    batch.arena_bytes = ub;
    const DeviceGraph& d = batch.dg;
    const size_t NE = u.tot.ne, NC = u.tot.nc;
    descs.clear();
    auto i32 = [&](const void* src, void* dst, long long n, int add) {
        if (n > 0) descs.push_back(PackDesc{src, dst, n, add, kPackI32, 0.0});
    };
    auto f64 = [&](const void* src, void* dst, long long n) {
        if (n > 0) descs.push_back(PackDesc{src, dst, n, 0, kPackF64, 0.0});
    };
    auto u8 = [&](const void* src, void* dst, long long n) {
        if (n > 0) descs.push_back(PackDesc{src, dst, n, 0, kPackU8, 0.0});
    };
    auto filli = [&](void* dst, long long n, int v) {
        if (n > 0) descs.push_back(PackDesc{nullptr, dst, n, v, kPackFillI32, 0.0});
    };
    auto filld = [&](void* dst, long long n, double v) {
        if (n > 0) descs.push_back(PackDesc{nullptr, dst, n, 0, kPackFillF64, v});
    };
    for (size_t p = 0; p < order.size(); ++p) {
        const Request* r = order[p];
        const ImageCounts& n = r->counts;
        const ImageLayout& L = r->lay;
        const char* base = (const char*)arena + r->dev_off;
        const int eo = u.edge_off[p], co = u.cam_off[p], po = u.pt_off[p];
        const int to = u.tile_off[p], ro = u.run_off[p], ko = u.chunk_off[p];
        const long long ne = n.ne;
        i32(base + L.e_cam, (int*)d.e_cam + eo, ne, co);
        i32(base + L.e_pt, (int*)d.e_pt + eo, ne, po);
        i32(base + L.cm_pt, (int*)d.cm_pt + eo, ne, po);
        for (int k = 0; k < 2; ++k) {
            f64(base + L.obs + 8 * k * ne, (double*)d.obs + k * NE + eo, ne);
            f64(base + L.cm_obs + 8 * k * ne, (double*)d.cm_obs + k * NE + eo, ne);
        }
        if (u.tot.info)
            for (int k = 0; k < 3; ++k) {
                if (n.info) {
                    f64(base + L.sinfo + 8 * k * ne, (double*)d.sinfo + k * NE + eo, ne);
                    f64(base + L.cm_sinfo + 8 * k * ne, (double*)d.cm_sinfo + k * NE + eo, ne);
                } else {
                    filld((double*)d.sinfo + k * NE + eo, ne, k == 1 ? 0.0 : 1.0);
                    filld((double*)d.cm_sinfo + k * NE + eo, ne, k == 1 ? 0.0 : 1.0);
                }
            }
        i32(base + L.tile_off, (int*)d.tile_off + to, n.n_tiles, eo);
        i32(base + L.cm_run_off, (int*)d.cm_run_off + ro, n.n_runs, eo);
        i32(base + L.chunk_run_off, (int*)d.chunk_run_off + ko, n.n_chunks, ro);
        i32(base + L.chunk_cam, (int*)d.chunk_cam + ko, n.n_chunks, co);
        i32(base + L.cam_chunk_off, (int*)d.cam_chunk_off + co, n.nc, ko);
        u8(base + L.cam_fixed, (unsigned char*)d.cam_fixed + co, n.nc);
        u8(base + L.pt_fixed, (unsigned char*)d.pt_fixed + po, n.np);
        f64(base + L.cam_init, d.cam_init + 9 * (size_t)co, 9LL * n.nc);
        f64(base + L.pt_init, d.pt_init + 3 * (size_t)po, 3LL * n.np);
        f64(base + L.cam_cur, d.cam + 9 * (size_t)co, 9LL * n.nc);
        f64(base + L.pt_cur, d.pt + 3 * (size_t)po, 3LL * n.np);
    }
    filli((int*)d.tile_off + u.tot.n_tiles, 1, (int)NE);
    filli((int*)d.cm_run_off + u.tot.n_runs, 1, (int)NE);
    filli((int*)d.chunk_run_off + u.tot.n_chunks, 1, u.tot.n_runs);
    filli((int*)d.cam_chunk_off + NC, 1, u.tot.n_chunks);
    filli(d.accept, u.P, 0);
    for (Request* r : join) HIP_S(this, hipStreamWaitEvent(stream, r->uploaded, 0));
    if ((st = upload_plan(batch, err)) != GBA_OK) return st;
    if ((st = launch_descs(descs)) != GBA_OK) return st;
    // LM states: continuing problems resume, joiners start
    std::vector<const HostProblem*> probs;
    std::vector<char> fresh;
    for (size_t p = 0; p < order.size(); ++p) {
        Request* r = order[p];
        probs.push_back(&r->prob);
        const bool is_new = r->state == kStaged;
        fresh.push_back(is_new ? 1 : 0);
        if (is_new) {
            r->state = kResident;
            lm[p].max_iters = r->max_iters;
            lm[p].tol = r->tol;
        } else {
            lm[p] = r->lm;
        }
    }
    if ((st = batch_begin(batch, probs, lm, fresh, cfg.options, nullptr, err)) != GBA_OK) return st;
    // the pinned host images of joiners are no longer needed
    for (Request* r : join) {
        if (r->h_blob) (void)hipHostFree(r->h_blob);
        r->h_blob = nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    repacks += 1;
    return GBA_OK;
}

// Download finished problems, record their results and free their images.
gba_status gba_server::collect_finished() {
    bool any = false;
    for (size_t p = 0; p < resident.size(); ++p) {
        Request* r = resident[p];
        if (!r || r->state != kResident || lm[p].running) continue;
        r->cams_out.resize(9 * (size_t)r->counts.nc);
        r->pts_out.resize(3 * (size_t)r->counts.np);
        gba_status st = batch_download(batch, (int)p, r->cams_out.data(), r->pts_out.data(), err);
        if (st != GBA_OK) return st;
        const ProblemLM& s = lm[p];
        r->lm = s;
        std::memset(&r->rep, 0, sizeof(r->rep));
        r->rep.initial_cost = s.F0;
        r->rep.final_cost = s.F;
        r->rep.final_lambda = s.lam;
        r->rep.trials = s.trials;
        r->rep.accepted = s.accepted;
        r->rep.pcg_iters_total = s.pcg_total;
        r->rep.termination = s.term;
        r->rep.workspace_bytes = r->lay.bytes;
        r->t_done = Clock::now();
        r->rep.ms_total = ms_between(r->t_admit, r->t_done);
        {
            std::lock_guard<std::mutex> lk(mu);
            r->state = kDone;
            ra.release(r->dev_off, r->lay.bytes);
            image_bytes_in_use -= r->lay.bytes;
            completed += 1;
            lat_ms.push_back(ms_between(r->t_submit, r->t_done));
            svc_ms.push_back(r->rep.ms_total);
            t_last_done = r->t_done;
            if (r->uploaded) {
                (void)hipEventDestroy(r->uploaded);
                r->uploaded = nullptr;
            }
            // a collected request is deleted by gba_server_poll: the batch
            // keeps only an empty slot until the next repack
            resident[p] = nullptr;
        }
        any = true;
    }
    if (any) cv_done.notify_all();
    return GBA_OK;
}

void gba_server::run() {
    (void)hipSetDevice(cfg.device);
    auto die = [&](const std::string& m) {
        std::lock_guard<std::mutex> lk(mu);
        failed = true;
        thread_err = m;
        cv_done.notify_all();
    };
    bool changed = false;
    while (true) {
        std::vector<Request*> newly;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] {
                return stop || !queue.empty() || !staged.empty() || !resident.empty();
            });
            if (stop) break;
            if (admit_locked(newly) != GBA_OK) {
                lk.unlock();
                die(err);
                return;
            }
        }
        for (Request* r : newly)
            if (upload(r) != GBA_OK) {
                die(err);
                return;
            }
        bool running = false;
        for (const ProblemLM& s : lm) running = running || s.running;
        bool can_join = false;   // a staged request whose upload overlapped the last trial
        {
            std::lock_guard<std::mutex> lk(mu);
            for (const Request* r : staged) can_join = can_join || r->staged_step < step || !running;
        }
        if (changed || can_join) {
            if (repack() != GBA_OK) {
                die(err);
                return;
            }
            changed = false;
        }
        running = false;
        for (const ProblemLM& s : lm) running = running || s.running;
        if (running) {
            if (batch_trial(batch, lm, cfg.options, tune, nullptr, err) != GBA_OK) {
                die(err);
                return;
            }
            std::lock_guard<std::mutex> lk(mu);
            trials_run += 1;
            batch_sum += batch.P;
            for (Request* r : resident)
                if (r) r->batch_peak = std::max(r->batch_peak, batch.P);
        }
        const long long before = completed;
        if (collect_finished() != GBA_OK) {
            die(err);
            return;
        }
        if (completed != before) changed = true;
        // problems that all finished without a trial (no work) leave too
        if (!running && !resident.empty()) changed = true;
        step += 1;
    }
}

// ============================================================== C ABI
extern "C" {

void gba_server_default_config(gba_server_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->precision = GBA_MIXED_FP32;
    c->device = 0;
    c->hbm_budget_bytes = (size_t)4 << 30;
    c->max_slots = 64;
    c->loss = GBA_LOSS_HUBER;
    c->delta = 1.0;
    gba_default_options(&c->options);
    c->tune_db = nullptr;
}

gba_status gba_server_create(const gba_server_config* cfg, gba_alloc_fn alloc, gba_free_fn free_fn,
                             void* ctx, gba_server** out) {
    if (!cfg || !out) return GBA_ERR_INVALID_ARG;
    *out = nullptr;
    if (cfg->precision != GBA_FP64 && cfg->precision != GBA_MIXED_FP32 && cfg->precision != GBA_MIXED_BF16)
        return GBA_ERR_INVALID_ARG;
    if ((alloc == nullptr) != (free_fn == nullptr)) return GBA_ERR_INVALID_ARG;
    if (cfg->max_slots < 1 || cfg->max_slots > kMaxProblems || cfg->hbm_budget_bytes < ((size_t)1 << 20))
        return GBA_ERR_INVALID_ARG;
    if (cfg->loss != GBA_LOSS_SQUARED && cfg->loss != GBA_LOSS_HUBER) return GBA_ERR_INVALID_ARG;
    if (cfg->loss == GBA_LOSS_HUBER && !(cfg->delta > 0.0 && std::isfinite(cfg->delta)))
        return GBA_ERR_INVALID_ARG;
    const gba_options& o = cfg->options;
    if (!(o.initial_lambda > 0.0) || !(o.min_diag > 0.0) || !(o.max_diag >= o.min_diag) ||
        o.pcg_max_iters < 1 || !(o.pcg_tol >= 0.0) ||
        (o.precond != GBA_PRECOND_IDENTITY && o.precond != GBA_PRECOND_BLOCK_JACOBI) ||
        o.accumulation < GBA_ACC_AUTO || o.accumulation > GBA_ACC_CAMERA_PASS ||
        (o.deterministic != 0 && o.deterministic != 1) || (o.jacobi_scaling != 0 && o.jacobi_scaling != 1) ||
        (o.deterministic && o.accumulation == GBA_ACC_LDS) ||
        o.pcg_schedule < GBA_PCG_AUTO || o.pcg_schedule > GBA_PCG_PERSISTENT ||
        o.jacobian < GBA_JACOBIAN_ANALYTIC || o.jacobian > GBA_JACOBIAN_DYNAMIC ||
        (o.solver != GBA_SOLVER_SCHUR && o.solver != GBA_SOLVER_FULL) ||
        (o.jacobian == GBA_JACOBIAN_DYNAMIC && o.solver != GBA_SOLVER_FULL) ||
        (o.solver == GBA_SOLVER_FULL && (o.deterministic || o.accumulation == GBA_ACC_CAMERA_PASS)))
        return GBA_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) return GBA_ERR_HIP;
    if (hipSetDevice(cfg->device) != hipSuccess) return GBA_ERR_HIP;
    gba_server* s = new gba_server();
    s->cfg = *cfg;
    s->cfg.tune_db = nullptr;
    s->allocator.alloc = alloc;
    s->allocator.free_fn = free_fn;
    s->allocator.ctx = ctx;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, cfg->device) == hipSuccess) {
        s->dev.n_cu = prop.multiProcessorCount;
        s->dev.max_lds = prop.sharedMemPerBlock;
    }
    // fixed decomposition sizes: built-in, then the database, then overrides
    s->tune.tiles_per_block = 16;
    s->tune.edges_per_block = 1024;
    s->tune.pts_per_block = 512;
    s->tune.pcg_sync_every = 8;
    bool db_ok = true;
    read_tune_db(cfg->tune_db, cfg->precision, s->tune, db_ok);
    if (!db_ok) {
        delete s;
        return GBA_ERR_INVALID_ARG;
    }
    if (cfg->tiles_per_block > 0) s->tune.tiles_per_block = cfg->tiles_per_block;
    if (cfg->edges_per_block > 0) s->tune.edges_per_block = cfg->edges_per_block;
    if (cfg->pts_per_block > 0) s->tune.pts_per_block = cfg->pts_per_block;
    if (cfg->pcg_sync_every > 0) s->tune.pcg_sync_every = cfg->pcg_sync_every;
    s->tune.accumulation = o.accumulation;
    s->tune.deterministic = o.deterministic;
    s->tune.solver = o.solver;
    s->tune.dynamic = o.jacobian == GBA_JACOBIAN_DYNAMIC ? 1 : 0;
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->ev_admit, hipEventDisableTiming) != hipSuccess) {
        gba_server_destroy(s);
        return GBA_ERR_HIP;
    }
    s->arena = s->allocator.allocate(cfg->hbm_budget_bytes);
    if (!s->arena) {
        gba_server_destroy(s);
        return GBA_ERR_OOM;
    }
    s->ra.reset(cfg->hbm_budget_bytes);
    s->batch.stream = s->stream;
    s->batch.owns_arena = false;
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return GBA_OK;
}

gba_status gba_server_submit(gba_server* s, const gba_problem* q, uint64_t* ticket) {
    if (!s || !q || !ticket) return GBA_ERR_INVALID_ARG;
    *ticket = 0;
    const auto t_submit = Clock::now();
    if (q->n_cams < 0 || q->n_pts < 0 || q->n_edges < 0 || q->max_iters < 0 || !(q->tol >= 0.0))
        return fail_s(s, GBA_ERR_INVALID_ARG, "negative size, iteration count or tolerance");
    if ((q->n_cams > 0 && !q->cams) || (q->n_pts > 0 && !q->pts) ||
        (q->n_edges > 0 && (!q->cam_idx || !q->pt_idx || !q->uv)))
        return fail_s(s, GBA_ERR_INVALID_ARG, "missing request array");
    if (q->n_edges > std::numeric_limits<int>::max() / 32 || q->n_pts > std::numeric_limits<int>::max() / 16)
        return fail_s(s, GBA_ERR_UNSUPPORTED, "request too large for 32-bit indexing");
    Request* r = new Request();
    HostProblem& h = r->prob;
    const size_t nc = q->n_cams, np = q->n_pts, ne = (size_t)q->n_edges;
    h.cam_params.assign(q->cams, q->cams + 9 * nc);
    h.pt_params.assign(q->pts, q->pts + 3 * np);
    h.cam_fixed.assign(nc, 0);
    h.pt_fixed.assign(np, 0);
    if (q->cam_fixed)
        for (size_t i = 0; i < nc; ++i) h.cam_fixed[i] = q->cam_fixed[i] ? 1 : 0;
    if (q->pt_fixed)
        for (size_t j = 0; j < np; ++j) h.pt_fixed[j] = q->pt_fixed[j] ? 1 : 0;
    h.e_cam.resize(ne);
    h.e_pt.resize(ne);
    h.e_uv.assign(q->uv, q->uv + 2 * ne);
    h.e_active.assign(ne, 1);
    auto finite = [](const std::vector<double>& v) {
        for (double x : v)
            if (!std::isfinite(x)) return false;
        return true;
    };
    gba_status bad = GBA_OK;
    std::string why;
    for (size_t e = 0; e < ne && bad == GBA_OK; ++e) {
        const int ci = q->cam_idx[e], pj = q->pt_idx[e];
        if (ci < 0 || (size_t)ci >= nc || pj < 0 || (size_t)pj >= np) {
            bad = GBA_ERR_UNKNOWN_ID;
            why = "edge " + std::to_string(e) + " names a vertex outside the request";
        }
        h.e_cam[e] = ci;
        h.e_pt[e] = pj;
    }
    if (bad == GBA_OK && (!finite(h.cam_params) || !finite(h.pt_params) || !finite(h.e_uv))) {
        bad = GBA_ERR_NONFINITE;
        why = "non-finite request value";
    }
    if (bad == GBA_OK && q->info) {
        h.e_info.assign(q->info, q->info + 3 * ne);
        if (!finite(h.e_info)) {
            bad = GBA_ERR_NONFINITE;
            why = "non-finite information matrix";
        }
        for (size_t e = 0; e < ne && bad == GBA_OK; ++e) {
            const double o00 = h.e_info[3 * e], o01 = h.e_info[3 * e + 1], o11 = h.e_info[3 * e + 2];
            if (!(o00 > 0.0) || !(o00 * o11 - o01 * o01 > 0.0)) {
                bad = GBA_ERR_INVALID_ARG;
                why = "information matrix not positive definite at edge " + std::to_string(e);
            }
        }
    }
    HostImage img;
    if (bad == GBA_OK) bad = make_image(h, img, why);
    size_t need = 0;
    if (bad == GBA_OK) {
        r->counts = img.n;
        r->lay = image_layout(img.n);
        std::vector<const ImageCounts*> one{&r->counts};
        need = r->lay.bytes + s->union_bytes_for(one);
        if (need > s->cfg.hbm_budget_bytes) {
            bad = GBA_ERR_BUDGET;
            why = "request needs " + std::to_string(need) + " device bytes, budget " +
                  std::to_string(s->cfg.hbm_budget_bytes);
        }
    }
    if (bad == GBA_OK) {
        (void)hipSetDevice(s->cfg.device);
        if (hipHostMalloc(&r->h_blob, r->lay.bytes, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&r->uploaded, hipEventDisableTiming) != hipSuccess) {
            bad = GBA_ERR_HIP;
            why = "pinned host allocation failed";
        }
    }
    if (bad != GBA_OK) {
        if (r->h_blob) (void)hipHostFree(r->h_blob);
        if (r->uploaded) (void)hipEventDestroy(r->uploaded);
        delete r;
        std::lock_guard<std::mutex> lk(s->mu);
        s->rejected += 1;
        s->err = why;
        return bad;
    }
    // pinned host image in the device layout
    char* b = (char*)r->h_blob;
    const ImageLayout& L = r->lay;
    auto put = [&](size_t off, const void* src, size_t bytes) {
        if (bytes) std::memcpy(b + off, src, bytes);
    };
    const size_t ien = img.n.ne;
    put(L.e_cam, img.e_cam.data(), 4 * ien);
    put(L.e_pt, img.e_pt.data(), 4 * ien);
    put(L.obs, img.obs.data(), 16 * ien);
    if (img.n.info) {
        put(L.sinfo, img.sinfo.data(), 24 * ien);
        put(L.cm_sinfo, img.cm_sinfo.data(), 24 * ien);
    }
    put(L.tile_off, img.tile_off.data(), 4 * img.tile_off.size());
    put(L.cm_run_off, img.cm_run_off.data(), 4 * img.cm_run_off.size());
    put(L.cm_pt, img.cm_pt.data(), 4 * ien);
    put(L.cm_obs, img.cm_obs.data(), 16 * ien);
    put(L.chunk_run_off, img.chunk_run_off.data(), 4 * img.chunk_run_off.size());
    put(L.chunk_cam, img.chunk_cam.data(), 4 * img.chunk_cam.size());
    put(L.cam_chunk_off, img.cam_chunk_off.data(), 4 * img.cam_chunk_off.size());
    put(L.cam_fixed, h.cam_fixed.data(), nc);
    put(L.pt_fixed, h.pt_fixed.data(), np);
    put(L.cam_init, h.cam_params.data(), 72 * nc);
    put(L.pt_init, h.pt_params.data(), 24 * np);
    put(L.cam_cur, h.cam_params.data(), 72 * nc);
    put(L.pt_cur, h.pt_params.data(), 24 * np);
    // keep only what the LM driver reads (the fixed masks)
    std::vector<double>().swap(h.cam_params);
    std::vector<double>().swap(h.pt_params);
    std::vector<int>().swap(h.e_cam);
    std::vector<int>().swap(h.e_pt);
    std::vector<double>().swap(h.e_uv);
    std::vector<double>().swap(h.e_info);
    std::vector<unsigned char>().swap(h.e_active);
    r->max_iters = q->max_iters;
    r->tol = q->tol;
    r->t_submit = t_submit;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->failed) {
            (void)hipHostFree(r->h_blob);
            (void)hipEventDestroy(r->uploaded);
            delete r;
            s->err = s->thread_err;
            return GBA_ERR_HIP;
        }
        r->ticket = s->next_ticket++;
        s->all[r->ticket] = r;
        s->queue.push_back(r);
        s->submitted += 1;
        if (!s->any_submit) {
            s->any_submit = true;
            s->t_first_submit = t_submit;
        }
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return GBA_OK;
}

gba_status gba_server_poll(gba_server* s, uint64_t ticket, int wait, gba_result* out) {
    if (!s) return GBA_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) {
        s->err = "unknown or already collected ticket " + std::to_string(ticket);
        return GBA_ERR_UNKNOWN_ID;
    }
    Request* r = it->second;
    while (r->state != kDone) {
        if (s->failed) {
            s->err = s->thread_err;
            return GBA_ERR_HIP;
        }
        if (!wait) return GBA_PENDING;
        s->cv_done.wait(lk);
    }
    if (out) {
        if (out->cams && !r->cams_out.empty())
            std::memcpy(out->cams, r->cams_out.data(), sizeof(double) * r->cams_out.size());
        if (out->pts && !r->pts_out.empty())
            std::memcpy(out->pts, r->pts_out.data(), sizeof(double) * r->pts_out.size());
        out->report = r->rep;
        out->latency_ms = ms_between(r->t_submit, r->t_done);
        out->queue_ms = ms_between(r->t_submit, r->t_admit);
        out->batch_peak = r->batch_peak;
    }
    s->all.erase(it);
    s->collected += 1;
    delete r;
    return GBA_OK;
}

static double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t lo = (size_t)std::floor(pos), hi = (size_t)std::ceil(pos);
    return v[lo] + (v[hi] - v[lo]) * (pos - (double)lo);
}

gba_status gba_server_stats(gba_server* s, gba_serving_stats* out) {
    if (!s || !out) return GBA_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->admitted = s->admitted;
    out->rejected = s->rejected;
    out->completed = s->completed;
    out->collected = s->collected;
    out->queued = (int64_t)s->queue.size();
    out->in_flight = s->admitted - s->completed;
    out->trials_run = s->trials_run;
    out->repacks = s->repacks;
    out->mean_batch = s->trials_run ? (double)s->batch_sum / (double)s->trials_run : 0.0;
    out->p50_latency_ms = percentile(s->lat_ms, 0.50);
    out->p99_latency_ms = percentile(s->lat_ms, 0.99);
    out->p50_service_ms = percentile(s->svc_ms, 0.50);
    out->p99_service_ms = percentile(s->svc_ms, 0.99);
    if (s->completed > 0) {
        const double span = ms_between(s->t_first_submit, s->t_last_done) / 1e3;
        out->solves_per_s = span > 0 ? (double)s->completed / span : 0.0;
    }
    out->bytes_in_use = s->bytes_in_use();
    out->bytes_peak = s->bytes_peak;
    out->budget = s->cfg.hbm_budget_bytes;
    out->tiles_per_block = s->tune.tiles_per_block;
    out->edges_per_block = s->tune.edges_per_block;
    out->pts_per_block = s->tune.pts_per_block;
    out->pcg_sync_every = s->tune.pcg_sync_every;
    return GBA_OK;
}

const char* gba_server_last_error(gba_server* s) {
    if (!s) return "null server handle";
    return s->err.c_str();
}

void gba_server_destroy(gba_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->cfg.device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->copy) (void)hipStreamSynchronize(s->copy);
    for (auto& kv : s->all) {
        Request* r = kv.second;
        if (r->h_blob) (void)hipHostFree(r->h_blob);
        if (r->uploaded) (void)hipEventDestroy(r->uploaded);
        delete r;
    }
    s->all.clear();
    s->batch.arena = nullptr;
    if (s->arena) s->allocator.release(s->arena);
    if (s->h_desc) (void)hipHostFree(s->h_desc);
    if (s->h_chunk) (void)hipHostFree(s->h_chunk);
    if (s->d_desc) (void)hipFree(s->d_desc);
    if (s->d_chunk) (void)hipFree(s->d_chunk);
    if (s->ev_admit) (void)hipEventDestroy(s->ev_admit);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
