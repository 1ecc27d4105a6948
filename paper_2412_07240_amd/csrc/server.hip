// Serving runtime: many tracks, per-track FIFOs, admission by device memory (a
// track that does not fit waits until memory frees), and a native worker thread
// that keeps the device busy with fused batched cycles and single ops as tracks
// become ready (see the serving section of include/pmf.h for the contract).
#include <hip/hip_runtime.h>

#include <atomic>
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
constexpr int FUSED_IN_FLIGHT = 4;     // fused batches on the device at once (staging sets)

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
    bool live = false;      // slot in use (admitted or waiting for admission)
    bool busy = false;      // an op of this track is on the device
    bool in_ready = false;  // listed in the server's ready queue
    bool fusable = false;
    size_t bytes = 0;       // device bytes (reserved from the budget once admitted)
    int nz = 1;
    long long ticket = 0;   // admission order of a waiting track (0: admitted)
    pmf_model model{};      // kept until admission
    pmf_prior prior{};
};

// one op taken onto the device
struct Taken {
    int track;
    SrvOp op;
    pmf_filter* f = nullptr;
};

// work on the device whose completion the worker waits for: a fused batch
// (predict/update pairs, ops = p0 u0 p1 u1 ...), or the single ops of one track
// (one op, or a predict and the update after it) launched back to back
struct Flight {
    hipEvent_t ev = nullptr;
    std::vector<Taken> ops;
    int dyn = -1;                       // fused: staging set holding the log-likelihoods
    pmf_status launch = PMF_OK;         // fused: the batch's launch status
    std::vector<pmf_status> launches;   // single ops: each op's launch status
};

}  // namespace

// a thread that launches single ops on its own stream and retires them
struct Launcher {
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::vector<Taken>> q;   // runs of one track's ops
    std::atomic<int> load{0};           // ops handed to it and not yet retired
    hipStream_t st = nullptr;
};

struct pmf_server {
    pmf_ctx* ctx = nullptr;
    size_t budget = 0, used = 0;
    int max_tracks = 0;
    std::vector<Track> tracks;          // index = track id
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<pmf_completion> done;
    long long submitted = 0, completed = 0, rounds = 0, fused_ops = 0, single_ops = 0, admitted_late = 0;
    long long next_ticket = 1;
    std::atomic<bool> stop{false};      // read by the launchers without the lock
    std::deque<int> ready;              // tracks that may have an op to run (no duplicates)
    std::thread worker;
    hipStream_t fused_stream = nullptr;
    Launcher launchers[SINGLE_STREAMS];
    DynBatch* db[FUSED_IN_FLIGHT] = {};
    double* h_ll = nullptr;             // pinned, one slot per track
};

namespace pmf {

static bool has_ready(const pmf_server* s) { return !s->ready.empty(); }

// List track id as possibly ready (the caller holds s->mu): an admitted, idle
// track with queued ops.
static void mark_ready(pmf_server* s, int id) {
    Track& t = s->tracks[id];
    if (t.f && !t.busy && !t.q.empty() && !t.in_ready) {
        t.in_ready = true;
        s->ready.push_back(id);
    }
}

static int waiting_tracks(const pmf_server* s) {
    int n = 0;
    for (const Track& t : s->tracks) n += t.live && !t.f;
    return n;
}

// Completions of a flight's ops, with their statuses and log-likelihoods.
static void post(pmf_server* s, const Flight& fl, const std::vector<int>& status, const std::vector<double>& ll) {
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    const bool fused = fl.dyn >= 0;
    for (size_t i = 0; i < fl.ops.size(); ++i) {
        pmf_completion c;
        c.tag = fl.ops[i].op.tag;
        c.track = fl.ops[i].track;
        c.op = fl.ops[i].op.op;
        c.status = status[i];
        c.fused = fused ? 1 : 0;
        c.loglik = fl.ops[i].op.op == PMF_OP_UPDATE ? ll[i] : 0.0;
        c.latency_us = std::chrono::duration<double, std::micro>(now - fl.ops[i].op.t0).count();
        s->done.push_back(c);
        s->tracks[fl.ops[i].track].busy = false;
        if (fused) s->fused_ops++;
        else s->single_ops++;
    }
    for (size_t i = 0; i < fl.ops.size(); ++i) mark_ready(s, fl.ops[i].track);
    s->completed += (long long)fl.ops.size();
    s->cv_done.notify_all();
    s->cv_work.notify_one();
}

// A finished flight: statuses and log-likelihoods of its ops, then its completions.
static void retire(pmf_server* s, Flight& fl, hipError_t ev_state) {
    const size_t n = fl.ops.size();
    std::vector<int> status(n, PMF_OK);
    std::vector<double> ll(n, 0.0);
    const bool dev_ok = ev_state == hipSuccess;
    if (fl.dyn >= 0) {
        const double* out = dyn_loglik(s->db[fl.dyn]);
        for (size_t j = 0; 2 * j + 1 < n; ++j) {
            pmf_status st = fl.launch;
            if (st == PMF_OK && !dev_ok) st = PMF_E_DEVICE;
            status[2 * j] = st;
            ll[2 * j + 1] = st == PMF_OK ? out[j] : NAN;
            status[2 * j + 1] = st != PMF_OK ? st : (std::isnan(out[j]) ? PMF_E_DEGENERATE : PMF_OK);
        }
    } else {
        // at most one update per run: its log-likelihood is in the track's slot
        for (size_t i = 0; i < n; ++i) {
            pmf_status st = fl.launches[i];
            if (st == PMF_OK && !dev_ok) st = PMF_E_DEVICE;
            status[i] = st;
            if (fl.ops[i].op.op == PMF_OP_UPDATE && st == PMF_OK) {
                ll[i] = s->h_ll[fl.ops[i].track];
                if (std::isnan(ll[i])) status[i] = PMF_E_DEGENERATE;
            }
        }
    }
    post(s, fl, status, ll);
}

// The worker: a loop that retires finished device work (event queries, no
// waiting) and, whenever tracks are idle with queued ops, puts their next ops on
// the device at once, so that requests arriving while others run are admitted
// as soon as their track (and, for fused batches, a staging set) is free.  A
// track whose FIFO starts with predict(T) + update(z) and that the fused kernel
// accepts runs that pair as one fused cycle, batched with the other such tracks
// taken in the same pass that have the same T; every other op runs through the
// generic path on the least loaded of the single-op streams, a predict followed
// by an update of the same track as one run (back to back on one stream, no
// round trip through the worker in between).  One op, fused pair or run of a
// track is on the device at a time, so each track's ops run in submission order.
static void worker_main(pmf_server* s) {
    (void)hipSetDevice(s->ctx->device);
    std::vector<Flight> flights;
    std::vector<hipEvent_t> ev_free;
    bool dyn_busy[FUSED_IN_FLIGHT] = {};
    int rr = 0;
    auto get_event = [&]() {
        hipEvent_t e = nullptr;
        if (!ev_free.empty()) {
            e = ev_free.back();
            ev_free.pop_back();
        } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            e = nullptr;
        }
        return e;
    };
    bool stalled = false;   // the last pass found only fused work and no free staging set
    for (;;) {
        // 1. retire whatever finished
        bool retired = false;
        for (size_t i = 0; i < flights.size();) {
            const hipError_t q = flights[i].ev ? hipEventQuery(flights[i].ev) : hipSuccess;
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            retire(s, flights[i], q);
            retired = true;
            if (flights[i].dyn >= 0) dyn_busy[flights[i].dyn] = false;
            if (flights[i].ev) ev_free.push_back(flights[i].ev);
            flights[i] = std::move(flights.back());
            flights.pop_back();
        }
        if (stalled && !retired && !flights.empty()) {
            // nothing can start until a staging set frees: poll without the lock
            std::this_thread::yield();
            continue;
        }
        // 2. take the next op of every idle track with queued ops
        std::map<double, std::vector<Taken>> fused;   // T -> predict/update pairs
        std::vector<std::vector<Taken>> singles;      // runs of one track's ops
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->ready.empty()) {
                if (flights.empty()) {
                    s->cv_work.wait(lk, [&] { return s->stop || !s->ready.empty(); });
                    if (s->stop && !has_ready(s)) return;
                } else {
                    // device work in flight: poll again soon (events are not waited on,
                    // so that new requests are taken while it runs)
                    lk.unlock();
                    std::this_thread::yield();
                    continue;
                }
            }
            int free_sets = 0;
            for (int d = 0; d < FUSED_IN_FLIGHT; ++d) free_sets += !dyn_busy[d];
            std::deque<int> cand;
            cand.swap(s->ready);
            for (int id : cand) {
                Track& t = s->tracks[id];
                t.in_ready = false;
                if (!t.f || t.busy || t.q.empty()) continue;
                if (t.fusable && t.q.size() >= 2 && t.q[0].op == PMF_OP_PREDICT && t.q[0].T > 0.0 &&
                    t.q[1].op == PMF_OP_UPDATE) {
                    auto it = fused.find(t.q[0].T);
                    if (it == fused.end()) {
                        if ((int)fused.size() >= free_sets) {
                            mark_ready(s, id);      // no staging set free: take it next pass
                            continue;
                        }
                        it = fused.emplace(t.q[0].T, std::vector<Taken>()).first;
                    }
                    it->second.push_back({id, t.q[0], t.f});
                    it->second.push_back({id, t.q[1], t.f});
                    t.q.pop_front();
                    t.q.pop_front();
                } else {
                    std::vector<Taken> run{{id, t.q[0], t.f}};
                    t.q.pop_front();
                    if (run[0].op.op == PMF_OP_PREDICT && !t.q.empty() && t.q[0].op == PMF_OP_UPDATE) {
                        run.push_back({id, t.q[0], t.f});
                        t.q.pop_front();
                    }
                    singles.push_back(std::move(run));
                }
                t.busy = true;
            }
            stalled = fused.empty() && singles.empty();
            if (!stalled) s->rounds++;
        }
        // 3. put them on the device
        for (auto& kv : fused) {
            int d = 0;
            while (dyn_busy[d]) ++d;
            Flight fl;
            fl.ops = std::move(kv.second);
            fl.dyn = d;
            const int n = (int)fl.ops.size() / 2;
            std::vector<pmf_filter*> fs(n);
            std::vector<double> z(3 * (size_t)n, 0.0);
            for (int j = 0; j < n; ++j) {
                fs[j] = fl.ops[2 * j].f;
                std::memcpy(&z[3 * (size_t)j], fl.ops[2 * j + 1].op.z, 3 * sizeof(double));
            }
            fl.launch = dyn_run(s->ctx, s->db[d], fs.data(), n, kv.first, z.data(), s->fused_stream);
            fl.ev = get_event();
            if (fl.ev) (void)hipEventRecord(fl.ev, s->fused_stream);
            dyn_busy[d] = true;
            flights.push_back(std::move(fl));
        }
        for (std::vector<Taken>& run : singles) {
            // the launcher with the fewest ops outstanding (ties: round robin)
            int best = rr++ % SINGLE_STREAMS;
            for (int q = 0; q < SINGLE_STREAMS; ++q)
                if (s->launchers[q].load.load() < s->launchers[best].load.load()) best = q;
            Launcher& L = s->launchers[best];
            L.load += (int)run.size();
            {
                std::lock_guard<std::mutex> lk(L.mu);
                L.q.push_back(std::move(run));
            }
            L.cv.notify_one();
        }
    }
}

// A single-op launcher: puts the runs handed to it on its stream (each run's ops
// back to back, then an event) and retires them as their events complete, so
// that the host cost of the generic path's many launches is spread over several
// threads.
static void launcher_main(pmf_server* s, Launcher* L) {
    (void)hipSetDevice(s->ctx->device);
    std::vector<Flight> flights;
    std::vector<hipEvent_t> ev_free;
    std::vector<std::vector<Taken>> take;
    for (;;) {
        for (size_t i = 0; i < flights.size();) {
            const hipError_t q = flights[i].ev ? hipEventQuery(flights[i].ev) : hipSuccess;
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            L->load -= (int)flights[i].ops.size();
            retire(s, flights[i], q);
            if (flights[i].ev) ev_free.push_back(flights[i].ev);
            flights[i] = std::move(flights.back());
            flights.pop_back();
        }
        take.clear();
        {
            std::unique_lock<std::mutex> lk(L->mu);
            if (L->q.empty()) {
                if (flights.empty()) {
                    L->cv.wait(lk, [&] { return !L->q.empty() || s->stop; });
                    if (L->q.empty() && s->stop) return;
                } else {
                    lk.unlock();
                    std::this_thread::yield();
                    continue;
                }
            }
            while (!L->q.empty()) {
                take.push_back(std::move(L->q.front()));
                L->q.pop_front();
            }
        }
        for (std::vector<Taken>& run : take) {
            Flight fl;
            fl.ops = std::move(run);
            for (const Taken& tk : fl.ops) {
                if (tk.op.op == PMF_OP_PREDICT) {
                    fl.launches.push_back(pmf_predict(tk.f, tk.op.T, L->st));
                } else {
                    s->h_ll[tk.track] = NAN;
                    fl.launches.push_back(pmf_update(tk.f, tk.op.z, &s->h_ll[tk.track], L->st));
                }
            }
            hipEvent_t e = nullptr;
            if (!ev_free.empty()) {
                e = ev_free.back();
                ev_free.pop_back();
            } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                e = nullptr;
            }
            fl.ev = e;
            if (fl.ev) (void)hipEventRecord(fl.ev, L->st);
            flights.push_back(std::move(fl));
        }
    }
}

// Admit waiting tracks in the order they were added while the budget and the
// live-track limit allow (their filters are created here, outside the lock).
static void admit_waiting(pmf_server* s) {
    for (;;) {
        int id = -1;
        pmf_model model;
        pmf_prior prior;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            long long best = 0;
            for (int i = 0; i < (int)s->tracks.size(); ++i) {
                const Track& t = s->tracks[i];
                if (t.live && !t.f && t.ticket > 0 && (best == 0 || t.ticket < best)) {
                    best = t.ticket;
                    id = i;
                }
            }
            if (id < 0) return;
            Track& t = s->tracks[id];
            if (s->used + t.bytes > s->budget) return;   // the oldest waits; none jumps it
            s->used += t.bytes;                          // reserved while it is created
            t.ticket = -1;                               // being created
            model = t.model;
            prior = t.prior;
        }
        pmf_filter* f = nullptr;
        const pmf_status r = pmf_create(s->ctx, &model, &prior, &f);
        std::lock_guard<std::mutex> lk(s->mu);
        Track& t = s->tracks[id];
        if (r != PMF_OK) {
            // the track cannot be created: its queued ops fail, its slot is freed
            s->used -= t.bytes;
            const Clock::time_point now = Clock::now();
            for (const SrvOp& o : t.q) {
                pmf_completion c{};
                c.tag = o.tag;
                c.track = id;
                c.op = o.op;
                c.status = r;
                c.loglik = NAN;
                c.latency_us = std::chrono::duration<double, std::micro>(now - o.t0).count();
                s->done.push_back(c);
                s->completed++;
            }
            t = Track();
            s->cv_done.notify_all();
            continue;
        }
        t.f = f;
        t.ticket = 0;
        s->admitted_late++;
        mark_ready(s, id);
        s->cv_work.notify_one();
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
        e = hipStreamCreateWithFlags(&s->launchers[q].st, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s->h_ll), sizeof(double) * max_tracks, hipHostMallocDefault);
    if (e != hipSuccess) {
        pmf_status r = hip_fail(e, "server set-up");
        if (s->fused_stream) (void)hipStreamDestroy(s->fused_stream);
        for (int q = 0; q < SINGLE_STREAMS; ++q)
            if (s->launchers[q].st) (void)hipStreamDestroy(s->launchers[q].st);
        if (s->h_ll) (void)hipHostFree(s->h_ll);
        delete s;
        return r;
    }
    for (int d = 0; d < FUSED_IN_FLIGHT; ++d) s->db[d] = dyn_create(ctx);
    s->tracks.reserve(max_tracks);
    for (int q = 0; q < SINGLE_STREAMS; ++q) s->launchers[q].th = std::thread(launcher_main, s, &s->launchers[q]);
    s->worker = std::thread(worker_main, s);
    *out = s;
    return PMF_OK;
}

extern "C" pmf_status pmf_server_drain(pmf_server* s) {
    if (!s) return fail(PMF_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    // ops of tracks still waiting for admission cannot complete until memory frees
    s->cv_done.wait(lk, [&] {
        long long waiting_ops = 0;
        for (const Track& t : s->tracks)
            if (t.live && !t.f && t.ticket > 0) waiting_ops += (long long)t.q.size();
        return s->completed + waiting_ops == s->submitted;
    });
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
    for (int q = 0; q < SINGLE_STREAMS; ++q) {
        {
            std::lock_guard<std::mutex> lk(s->launchers[q].mu);
        }
        s->launchers[q].cv.notify_all();
        s->launchers[q].th.join();
    }
    for (Track& t : s->tracks)
        if (t.f) pmf_destroy(t.f);
    for (int d = 0; d < FUSED_IN_FLIGHT; ++d) dyn_destroy(s->ctx, s->db[d]);
    (void)hipStreamDestroy(s->fused_stream);
    for (int q = 0; q < SINGLE_STREAMS; ++q) (void)hipStreamDestroy(s->launchers[q].st);
    (void)hipHostFree(s->h_ll);
    delete s;
}

extern "C" pmf_status pmf_server_add_track(pmf_server* s, const pmf_model* model, const pmf_prior* prior,
                                           int* track) {
    if (!s || !model || !prior || !track) return fail(PMF_E_INVALID, "NULL argument");
    pmf_status r = check_model(model);
    if (r != PMF_OK) return r;
    std::string why;
    const bool fusable = model_fusable(*model, &why);
    const size_t bytes = filter_device_bytes(*model) + (fusable ? fused_const_bytes() : 0);
    if (bytes > s->budget) return fail(PMF_E_NOMEM, "the track needs more device memory than the server's budget");
    int slot = -1;
    bool now = false;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        int live = 0;
        for (int i = 0; i < (int)s->tracks.size(); ++i) {
            live += s->tracks[i].live;
            if (!s->tracks[i].live && slot < 0) slot = i;
        }
        if (live >= s->max_tracks) return fail(PMF_E_NOMEM, "max_tracks tracks are live");
        if (slot < 0) {
            slot = (int)s->tracks.size();
            s->tracks.emplace_back();
        }
        Track& t = s->tracks[slot];
        t = Track();
        t.live = true;
        t.fusable = fusable;
        t.bytes = bytes;
        t.nz = model->nz;
        t.model = *model;
        t.prior = *prior;
        // admitted at once if it fits and no earlier track is waiting; else it waits
        // (its ops are queued) until memory frees
        int earlier = 0;
        for (const Track& w : s->tracks) earlier += w.live && !w.f && w.ticket > 0;
        now = earlier == 0 && s->used + bytes <= s->budget;
        if (now) {
            s->used += bytes;
            t.ticket = -1;
        } else {
            t.ticket = s->next_ticket++;
        }
    }
    if (now) {
        pmf_filter* f = nullptr;
        r = pmf_create(s->ctx, model, prior, &f);
        std::lock_guard<std::mutex> lk(s->mu);
        Track& t = s->tracks[slot];
        if (r != PMF_OK) {
            s->used -= t.bytes;
            t = Track();
            return r;
        }
        t.f = f;
        t.ticket = 0;
        mark_ready(s, slot);
        s->cv_work.notify_one();
    }
    *track = slot;
    return PMF_OK;
}

extern "C" pmf_status pmf_server_remove_track(pmf_server* s, int track) {
    if (!s) return fail(PMF_E_INVALID, "server is NULL");
    pmf_filter* f = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (track < 0 || track >= (int)s->tracks.size() || !s->tracks[track].live)
            return fail(PMF_E_INVALID, "no such track");
        Track& t = s->tracks[track];
        if (t.busy || !t.q.empty() || t.ticket < 0) return fail(PMF_E_BUSY, "track has queued or running ops");
        f = t.f;
        if (f) s->used -= t.bytes;
        t = Track();
    }
    if (f) pmf_destroy(f);
    admit_waiting(s);
    return PMF_OK;
}

// validated op of a submission; the caller holds s->mu
static pmf_status make_op(pmf_server* s, int track, int op, double T, const double* z, long long tag, SrvOp* o) {
    if (track < 0 || track >= (int)s->tracks.size() || !s->tracks[track].live)
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
    mark_ready(s, track);
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
    mark_ready(s, track);
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
    out->waiting_tracks = waiting_tracks(s);
    out->admitted_late = s->admitted_late;
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
