// Serving runtime: many tracks, per-track FIFOs, a native worker thread that
// runs rounds of fused batched cycles and single ops (see the serving section of
// include/pmf.h for the contract).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "api_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr int SINGLE_STREAMS = 4;

struct SrvOp {
    long long tag;
    int op;
    double T;
    double z[3];
    Clock::time_point t0;
};

struct Track {
    pmf_filter* f = nullptr;
    std::deque<SrvOp> q;
    bool busy = false;      // ops of this track are in the running round
    bool fusable = false;
    size_t bytes = 0;
    int nz = 1;
};

// one op taken into a round
struct Taken {
    int track;
    SrvOp op;
    bool fused;
    int slot;               // fused: row in its batch; single: pinned loglik slot
};

}  // namespace

struct pmf_server {
    pmf_ctx* ctx = nullptr;
    size_t budget = 0, used = 0;
    int max_tracks = 0;
    std::vector<Track> tracks;          // index = track id; f == nullptr: free slot
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<pmf_completion> done;
    long long submitted = 0, completed = 0, rounds = 0, fused_ops = 0, single_ops = 0;
    bool stop = false;
    std::thread worker;
    hipStream_t fused_stream = nullptr;
    hipStream_t streams[SINGLE_STREAMS] = {};
    DynBatch* db = nullptr;
    double* h_ll = nullptr;             // pinned, one slot per track
};

namespace pmf {

static bool has_ready(const pmf_server* s) {
    for (const Track& t : s->tracks)
        if (t.f && !t.busy && !t.q.empty()) return true;
    return false;
}

// Post the completions of taken[i] for the listed i.
static void post(pmf_server* s, const std::vector<Taken>& taken, const std::vector<int>& which,
                 const std::vector<int>& status, const std::vector<double>& ll) {
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    for (int i : which) {
        pmf_completion c;
        c.tag = taken[i].op.tag;
        c.track = taken[i].track;
        c.op = taken[i].op.op;
        c.status = status[i];
        c.fused = taken[i].fused ? 1 : 0;
        c.loglik = taken[i].op.op == PMF_OP_UPDATE ? ll[i] : 0.0;
        c.latency_us = std::chrono::duration<double, std::micro>(now - taken[i].op.t0).count();
        s->done.push_back(c);
        s->tracks[taken[i].track].busy = false;
        if (taken[i].fused) s->fused_ops++;
        else s->single_ops++;
    }
    s->completed += (long long)which.size();
    s->cv_done.notify_all();
    s->cv_work.notify_one();
}

// One round: the fused batches are enqueued first, then the single ops on their
// streams; the fused ops complete (and their tracks become idle) as soon as the
// fused stream is done, without waiting for the single ops.
static void run_round(pmf_server* s, std::vector<Taken>& taken) {
    std::map<double, std::vector<int>> fused;   // T -> indexes of the predict ops in `taken`
    std::vector<int> singles;
    for (int i = 0; i < (int)taken.size(); ++i) {
        if (!taken[i].fused) singles.push_back(i);
        else if (taken[i].op.op == PMF_OP_PREDICT) fused[taken[i].op.T].push_back(i);
    }
    std::vector<int> status(taken.size(), PMF_OK);
    std::vector<double> ll(taken.size(), 0.0);
    std::vector<int> fused_done;
    // fused cycles: predict at taken[i], its update at taken[i + 1]; the staging
    // of the batch buffers is reused, so a second interval waits for the first
    int ngroup = 0;
    std::vector<std::pair<const std::vector<int>*, pmf_status>> launched;
    auto finish_fused = [&]() {
        hipError_t e = hipStreamSynchronize(s->fused_stream);
        const double* out = dyn_loglik(s->db);
        for (auto& g : launched) {
            pmf_status st = g.second;
            if (st == PMF_OK && e != hipSuccess) st = PMF_E_DEVICE;
            const std::vector<int>& idx = *g.first;
            for (size_t j = 0; j < idx.size(); ++j) {
                const int p = idx[j], u = idx[j] + 1;
                status[p] = st;
                ll[u] = st == PMF_OK ? out[j] : NAN;
                status[u] = st != PMF_OK ? st : (std::isnan(out[j]) ? PMF_E_DEGENERATE : PMF_OK);
                fused_done.push_back(p);
                fused_done.push_back(u);
            }
        }
        launched.clear();
    };
    for (auto& kv : fused) {
        if (ngroup++ > 0) finish_fused();
        const std::vector<int>& idx = kv.second;
        std::vector<pmf_filter*> fs(idx.size());
        std::vector<double> z(3 * idx.size(), 0.0);
        for (size_t j = 0; j < idx.size(); ++j) {
            fs[j] = s->tracks[taken[idx[j]].track].f;
            std::memcpy(&z[3 * j], taken[idx[j] + 1].op.z, 3 * sizeof(double));
        }
        launched.push_back({&idx, dyn_run(s->ctx, s->db, fs.data(), (int)fs.size(), kv.first, z.data(),
                                          s->fused_stream)});
    }
    // single ops, spread over the streams
    int k = 0;
    for (int i : singles) {
        Track& t = s->tracks[taken[i].track];
        hipStream_t st = s->streams[k++ % SINGLE_STREAMS];
        if (taken[i].op.op == PMF_OP_PREDICT) {
            status[i] = pmf_predict(t.f, taken[i].op.T, st);
        } else {
            s->h_ll[taken[i].track] = NAN;
            status[i] = pmf_update(t.f, taken[i].op.z, &s->h_ll[taken[i].track], st);
        }
    }
    if (!launched.empty()) finish_fused();
    if (!fused_done.empty()) post(s, taken, fused_done, status, ll);
    if (!singles.empty()) {
        for (int q = 0; q < SINGLE_STREAMS; ++q) {
            hipError_t e = hipStreamSynchronize(s->streams[q]);
            if (e != hipSuccess)
                for (int i : singles)
                    if (status[i] == PMF_OK) status[i] = PMF_E_DEVICE;
        }
        for (int i : singles) {
            if (taken[i].op.op != PMF_OP_UPDATE || status[i] != PMF_OK) continue;
            ll[i] = s->h_ll[taken[i].track];
            if (std::isnan(ll[i])) status[i] = PMF_E_DEGENERATE;
        }
        post(s, taken, singles, status, ll);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->rounds++;
}

static void worker_main(pmf_server* s) {
    (void)hipSetDevice(s->ctx->device);
    std::vector<Taken> taken;
    for (;;) {
        taken.clear();
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || has_ready(s); });
            if (s->stop && !has_ready(s)) return;
            for (int id = 0; id < (int)s->tracks.size(); ++id) {
                Track& t = s->tracks[id];
                if (!t.f || t.busy || t.q.empty()) continue;
                if (t.fusable && t.q.size() >= 2 && t.q[0].op == PMF_OP_PREDICT && t.q[0].T > 0.0 &&
                    t.q[1].op == PMF_OP_UPDATE) {
                    taken.push_back({id, t.q[0], true, 0});
                    taken.push_back({id, t.q[1], true, 0});
                    t.q.pop_front();
                    t.q.pop_front();
                } else {
                    taken.push_back({id, t.q[0], false, 0});
                    t.q.pop_front();
                }
                t.busy = true;
            }
        }
        run_round(s, taken);
    }
}

}  // namespace pmf

using namespace pmf;

extern "C" pmf_status pmf_server_create(pmf_ctx* ctx, size_t budget_bytes, int max_tracks, pmf_server** out) {
    if (!ctx || !out || max_tracks < 1) return fail(PMF_E_INVALID, "NULL argument or max_tracks < 1");
    *out = nullptr;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    pmf_server* s = new pmf_server();
    s->ctx = ctx;
    s->budget = budget_bytes;
    s->max_tracks = max_tracks;
    e = hipStreamCreateWithFlags(&s->fused_stream, hipStreamNonBlocking);
    for (int q = 0; q < SINGLE_STREAMS && e == hipSuccess; ++q)
        e = hipStreamCreateWithFlags(&s->streams[q], hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s->h_ll), sizeof(double) * max_tracks, hipHostMallocDefault);
    if (e != hipSuccess) {
        pmf_status r = hip_fail(e, "server set-up");
        if (s->fused_stream) (void)hipStreamDestroy(s->fused_stream);
        for (int q = 0; q < SINGLE_STREAMS; ++q)
            if (s->streams[q]) (void)hipStreamDestroy(s->streams[q]);
        if (s->h_ll) (void)hipHostFree(s->h_ll);
        delete s;
        return r;
    }
    s->db = dyn_create(ctx);
    s->tracks.reserve(max_tracks);
    s->worker = std::thread(worker_main, s);
    *out = s;
    return PMF_OK;
}

extern "C" pmf_status pmf_server_drain(pmf_server* s) {
    if (!s) return fail(PMF_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->completed == s->submitted; });
    return PMF_OK;
}

extern "C" void pmf_server_destroy(pmf_server* s) {
    if (!s) return;
    pmf_server_drain(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->worker.join();
    for (Track& t : s->tracks)
        if (t.f) pmf_destroy(t.f);
    dyn_destroy(s->ctx, s->db);
    (void)hipStreamDestroy(s->fused_stream);
    for (int q = 0; q < SINGLE_STREAMS; ++q) (void)hipStreamDestroy(s->streams[q]);
    (void)hipHostFree(s->h_ll);
    delete s;
}

extern "C" pmf_status pmf_server_add_track(pmf_server* s, const pmf_model* model, const pmf_prior* prior,
                                           int* track) {
    if (!s || !model || !prior || !track) return fail(PMF_E_INVALID, "NULL argument");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        int live = 0;
        for (const Track& t : s->tracks) live += t.f != nullptr;
        if (live >= s->max_tracks) return fail(PMF_E_NOMEM, "max_tracks tracks are live");
    }
    pmf_filter* f = nullptr;
    pmf_status r = pmf_create(s->ctx, model, prior, &f);
    if (r != PMF_OK) return r;
    std::string why;
    const bool fusable = batch_fusable(f, &why);
    // (a fusable filter's fused-step constants are allocated at create)
    const size_t bytes = f->bytes;
    std::lock_guard<std::mutex> lk(s->mu);
    int live = 0, slot = -1;
    for (int i = 0; i < (int)s->tracks.size(); ++i) {
        live += s->tracks[i].f != nullptr;
        if (!s->tracks[i].f && slot < 0) slot = i;
    }
    if (live >= s->max_tracks || s->used + bytes > s->budget) {
        pmf_destroy(f);
        return fail(PMF_E_NOMEM, "device-memory budget of the server exceeded");
    }
    if (slot < 0) {
        slot = (int)s->tracks.size();
        s->tracks.emplace_back();
    }
    Track& t = s->tracks[slot];
    t.f = f;
    t.q.clear();
    t.busy = false;
    t.fusable = fusable;
    t.bytes = bytes;
    t.nz = model->nz;
    s->used += bytes;
    *track = slot;
    return PMF_OK;
}

extern "C" pmf_status pmf_server_remove_track(pmf_server* s, int track) {
    if (!s) return fail(PMF_E_INVALID, "server is NULL");
    pmf_filter* f = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (track < 0 || track >= (int)s->tracks.size() || !s->tracks[track].f)
            return fail(PMF_E_INVALID, "no such track");
        Track& t = s->tracks[track];
        if (t.busy || !t.q.empty()) return fail(PMF_E_BUSY, "track has queued or running ops");
        f = t.f;
        t.f = nullptr;
        s->used -= t.bytes;
        t.bytes = 0;
    }
    pmf_destroy(f);
    return PMF_OK;
}

// validated op of a submission; the caller holds s->mu
static pmf_status make_op(pmf_server* s, int track, int op, double T, const double* z, long long tag, SrvOp* o) {
    if (track < 0 || track >= (int)s->tracks.size() || !s->tracks[track].f)
        return fail(PMF_E_INVALID, "no such track");
    const Track& t = s->tracks[track];
    o->tag = tag;
    o->op = op;
    o->T = 0.0;
    o->z[0] = o->z[1] = o->z[2] = 0.0;
    if (op == PMF_OP_PREDICT) {
        if (!std::isfinite(T) || T < 0.0) return fail(PMF_E_INVALID, "T must be finite and >= 0");
        o->T = T;
    } else if (op == PMF_OP_UPDATE) {
        if (!z) return fail(PMF_E_INVALID, "z is NULL");
        for (int i = 0; i < t.nz; ++i) {
            if (!std::isfinite(z[i])) return fail(PMF_E_INVALID, "non-finite measurement");
            o->z[i] = z[i];
        }
    } else {
        return fail(PMF_E_INVALID, "unknown op");
    }
    o->t0 = Clock::now();
    return PMF_OK;
}

extern "C" pmf_status pmf_server_submit(pmf_server* s, int track, int op, double T, const double* z, long long tag) {
    if (!s) return fail(PMF_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    SrvOp o;
    pmf_status r = make_op(s, track, op, T, z, tag, &o);
    if (r != PMF_OK) return r;
    s->tracks[track].q.push_back(o);
    s->submitted++;
    s->cv_work.notify_one();
    return PMF_OK;
}

extern "C" pmf_status pmf_server_submit_cycle(pmf_server* s, int track, double T, const double* z, long long tag) {
    if (!s) return fail(PMF_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    SrvOp p, u;
    pmf_status r = make_op(s, track, PMF_OP_PREDICT, T, nullptr, tag, &p);
    if (r == PMF_OK) r = make_op(s, track, PMF_OP_UPDATE, 0.0, z, tag + 1, &u);
    if (r != PMF_OK) return r;
    s->tracks[track].q.push_back(p);
    s->tracks[track].q.push_back(u);
    s->submitted += 2;
    s->cv_work.notify_one();
    return PMF_OK;
}

extern "C" pmf_status pmf_server_poll(pmf_server* s, pmf_completion* out, int cap, int* n) {
    if (!s || !n || (cap > 0 && !out)) return fail(PMF_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    int k = 0;
    while (k < cap && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n = k;
    return PMF_OK;
}

extern "C" pmf_status pmf_server_stats_get(pmf_server* s, pmf_server_stats* out) {
    if (!s || !out) return fail(PMF_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->budget_bytes = s->budget;
    out->used_bytes = s->used;
    int live = 0;
    for (const Track& t : s->tracks) live += t.f != nullptr;
    out->tracks = live;
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->rounds = s->rounds;
    out->fused_ops = s->fused_ops;
    out->single_ops = s->single_ops;
    return PMF_OK;
}

extern "C" pmf_filter* pmf_server_filter(pmf_server* s, int track) {
    if (!s) return nullptr;
    std::lock_guard<std::mutex> lk(s->mu);
    if (track < 0 || track >= (int)s->tracks.size()) return nullptr;
    return s->tracks[track].f;
}
