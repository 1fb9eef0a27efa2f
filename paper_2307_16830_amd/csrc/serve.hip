// Continuous-batching solve server (declared in opf.h).
//
// Worker slots, each a host thread with its own non-blocking HIP stream at the default priority, pull
// requests in arrival order.  A slot first does the request's host work on its own (model structure,
// symbolic analysis of the condensed pattern), so the host work of different requests runs in parallel;
// submission only checks and copies the grid.  One
// device allocation (the pool) is carved into per-request regions: at admission a slot takes the largest
// free block as a provisional region, creates the request's device buffers and IPM state inside it (every
// DBuf of the calling thread is bump-allocated there), keeps exactly what was used (the request's
// footprint) and returns the rest.  Admission is one slot at a time, so the provisional block is never
// contended; the solves themselves run concurrently and overlap on the device.  A request that does not fit
// waits (no further admissions) until a running request returns its region; one that does not fit an empty
// pool is answered with OPF_E_BUDGET.  Nothing is hipMalloc'ed, hipFree'd or host-pinned while serving (each
// slot keeps one pinned scalar buffer and its events for all its requests), so no request's creation or
// completion synchronizes the device under the others.  With ipm_options.graphs each solve's factorization
// and triangular solves are captured once on the slot's stream and replayed.
#include <algorithm>
#include <cstdio>
#include <array>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "common.h"

using namespace opf;

int ipm_prepare_device(ipm_state* S);  // ipm.hip: perform every pending device upload of a state now
namespace opf {
int validate_grid(const opf_grid* g);  // model.hip: the grid checks of opf_create
}
// ipm.hip: ipm_create with a prebuilt analysis (ownership passes) and a lent pinned buffer and events
int ipm_create_ex(opf_model* M, const ipm_options* opts, const chol_options* copts, void* stream, chol_sym* prebuilt,
                  double* host, const hipEvent_t* events, ipm_state** out);

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) & ~(ALIGN - 1); }

// Free blocks of the pool, [offset, offset + length), first-fit; neighbours coalesce on release.
class Regions {
  public:
    void init(size_t cap) {
        free_.clear();
        if (cap) free_[0] = cap;
    }
    std::pair<size_t, size_t> largest() const {
        std::pair<size_t, size_t> b{0, 0};
        for (const auto& kv : free_)
            if (kv.second > b.second) b = kv;
        return b;
    }
    void take(size_t off) { free_.erase(off); }  // a whole free block, as returned by largest()
    void give(size_t off, size_t len) {
        if (!len) return;
        auto it = free_.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<size_t, size_t> free_;
};

// Host copy of a submitted grid (the caller's arrays may go away after submission).
struct GridCopy {
    opf_grid g{};
    std::vector<double> d[20];
    std::vector<int32_t> i[3];
    explicit GridCopy(const opf_grid& src) : g(src) {
        const int N = src.nbus, E = src.nbranch, G = src.ngen;
        int k = 0;
        auto dv = [&](const double*& p, int len) {
            d[k].assign(p, p + (p ? len : 0));
            p = p ? d[k].data() : nullptr;
            k++;
        };
        auto iv = [&](const int32_t*& p, int len, int q) {
            i[q].assign(p, p + (p ? len : 0));
            p = p ? i[q].data() : nullptr;
        };
        dv(g.pd, N), dv(g.qd, N), dv(g.gs, N), dv(g.bs, N), dv(g.vmin, N), dv(g.vmax, N);
        dv(g.r, E), dv(g.x, E), dv(g.b, E), dv(g.rate, E), dv(g.angmin, E), dv(g.angmax, E);
        dv(g.c2, G), dv(g.c1, G), dv(g.c0, G), dv(g.pmin, G), dv(g.pmax, G), dv(g.qmin, G), dv(g.qmax, G);
        iv(g.f, E, 0), iv(g.t, E, 1), iv(g.gbus, G, 2);
    }
};

struct Request {
    int64_t tag = 0;
    double t_submit = 0;
    std::shared_ptr<GridCopy> grid;
    opf_model* model = nullptr;  // built by the worker that takes the request (again after a failed admission)
};

struct Done {
    serve_result r{};
    std::vector<double> x;
};

}  // namespace

struct opf_server {
    serve_options o{};
    int device = 0;
    char* pool = nullptr;
    size_t cap = 0;
    Regions regions;
    size_t in_use = 0, peak = 0;
    std::mutex mu;
    std::condition_variable cv_work;  // queue grew, memory returned, a creation ended, or stop
    std::condition_variable cv_done;  // a result is ready or the server went idle
    std::deque<Request> queue;
    std::deque<int64_t> ready;
    std::unordered_map<int64_t, Done> done;
    std::unordered_set<int64_t> active;  // tags submitted and not finished
    int running = 0;        // admitted, solve not finished
    int preparing = 0;      // taken from the queue, host phase or waiting for admission
    bool creating = false;  // a slot holds the provisional block
    bool blocked = false;   // the queue head did not fit: admit nothing until memory comes back
    bool stop = false;
    std::vector<hipStream_t> streams;
    // per slot: a pinned buffer of 16 doubles and 10 events lent to every state the slot creates, so no
    // request allocates or frees pinned memory or events while others run
    std::vector<double*> pinned;
    std::vector<std::array<hipEvent_t, 10>> events;
    std::vector<std::thread> workers;
};

namespace {

void finish(opf_server* S, Done&& d) {
    const int64_t tag = d.r.tag;
    // a failed request carries the message its failure left on this worker thread
    if (d.r.status < 0) snprintf(d.r.message, sizeof d.r.message, "%s", opf_last_error());
    S->active.erase(tag);
    S->done[tag] = std::move(d);
    S->ready.push_back(tag);
    S->cv_done.notify_all();
}

void worker(opf_server* S, int slot) {
    (void)hipSetDevice(S->device);
    hipStream_t st = S->streams[slot];
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        S->cv_work.wait(lk, [&] { return (S->stop && S->queue.empty()) || (!S->queue.empty() && !S->blocked); });
        if (S->queue.empty()) break;
        Request rq = std::move(S->queue.front());
        S->queue.pop_front();
        S->preparing++;
        lk.unlock();

        // host phase, outside admission: model structure (if rebuilt) and the symbolic analysis; device
        // buffers of both are deferred, so they are carved from the pool block at admission
        Done d;
        d.r.tag = rq.tag;
        d.r.t_submit = rq.t_submit;
        int rc = OPF_OK;
        if (!rq.model) rc = opf_create(&rq.grid->g, nullptr, st, &rq.model);
        if (rc == OPF_OK) {
            int64_t a, b, c;
            rc = opf_dims(rq.model, &d.r.n, &d.r.m, &a, &b, &c);
        }
        chol_sym* sym = nullptr;
        if (rc == OPF_OK) {
            std::vector<int32_t> cp(d.r.n + 1), ri;
            int64_t nj, nh, nk;
            int32_t n2, m2;
            rc = opf_dims(rq.model, &n2, &m2, &nj, &nh, &nk);
            if (rc == OPF_OK) {
                ri.resize(nk);
                rc = kkt_pattern(rq.model, cp.data(), ri.data());
            }
            if (rc == OPF_OK) rc = chol_analyze(d.r.n, cp.data(), ri.data(), &S->o.chol, &sym);
        }

        // admission: one slot at a time takes the largest free block, creates the state inside it and keeps
        // only what it used
        lk.lock();
        S->cv_work.wait(lk, [&] { return !S->creating; });
        const auto blk = S->regions.largest();
        if (blk.second) S->regions.take(blk.first);
        S->creating = true;
        S->preparing--;
        const bool alone = S->running == 0;  // then the block is the whole pool
        lk.unlock();

        ipm_state* state = nullptr;
        DeviceRegion reg{S->pool + blk.first, blk.second, 0};
        if (rc == OPF_OK) {
            thread_region() = &reg;
            rc = ipm_create_ex(rq.model, &S->o.ipm, &S->o.chol, st, sym, S->pinned[slot], S->events[slot].data(),
                               &state);
            sym = nullptr;  // owned by the state (or freed by the failed creation)
            if (rc == OPF_OK) rc = ipm_prepare_device(state);
            thread_region() = nullptr;
        }
        if (sym) chol_destroy(sym);
        const size_t used = align_up(reg.used);
        if (rc != OPF_OK) {
            // nothing of this request may touch the block once it is returned
            (void)hipStreamSynchronize(st);
            ipm_destroy(state);
            opf_destroy(rq.model);
            rq.model = nullptr;
            lk.lock();
            S->regions.give(blk.first, blk.second);
            S->creating = false;
            if (rc == OPF_E_NOMEM && !alone) {
                // retried when a running request returns memory (at once if one already did meanwhile)
                S->queue.push_front(std::move(rq));
                S->blocked = S->running > 0;
            } else {
                d.r.status = rc == OPF_E_NOMEM ? OPF_E_BUDGET : rc;
                d.r.t_admit = d.r.t_done = now_s();
                finish(S, std::move(d));
            }
            S->cv_work.notify_all();
            continue;
        }
        lk.lock();
        S->regions.give(blk.first + used, blk.second - used);
        S->in_use += used;
        S->peak = std::max(S->peak, S->in_use);
        S->creating = false;
        S->running++;
        S->cv_work.notify_all();
        lk.unlock();

        d.r.footprint = (int64_t)used;
        d.r.t_admit = now_s();
        ipm_result res{};
        rc = ipm_solve(state, &res);
        d.r.status = rc == OPF_OK ? 1 : rc;
        d.r.iterations = res.iterations;
        d.r.objective = res.objective;
        d.x.assign(d.r.n, 0.0);
        if (ipm_get_iterate(state, d.x.data(), nullptr, nullptr) != OPF_OK && d.r.status == 1) d.r.status = OPF_E_DEVICE;
        (void)hipStreamSynchronize(st);
        ipm_destroy(state);
        opf_destroy(rq.model);
        d.r.t_done = now_s();

        lk.lock();
        S->regions.give(blk.first, used);
        S->in_use -= used;
        S->running--;
        S->blocked = false;
        finish(S, std::move(d));
        S->cv_work.notify_all();
    }
    S->cv_done.notify_all();
}

}  // namespace

extern "C" void serve_default_options(serve_options* o) {
    o->slots = 8;
    o->hbm_budget = int64_t(8) << 30;
    ipm_default_options(&o->ipm);
    chol_default_options(&o->chol);
}

extern "C" double opf_serve_now(void) { return now_s(); }

extern "C" int opf_serve_create(const serve_options* o, opf_server** out) {
    return guarded([&] {
        OPF_CHECK(out, OPF_E_INVALID, "opf_serve_create: null argument");
        *out = nullptr;
        auto S = std::make_unique<opf_server>();
        serve_default_options(&S->o);
        if (o) S->o = *o;
        OPF_CHECK(S->o.slots >= 1 && S->o.slots <= 64 && S->o.hbm_budget > 0, OPF_E_INVALID,
                  "opf_serve_create: need 1 <= slots <= 64 and hbm_budget > 0");
        OPF_HIP(hipGetDevice(&S->device));
        S->cap = (size_t)S->o.hbm_budget & ~(ALIGN - 1);
        if (hipMalloc((void**)&S->pool, S->cap) != hipSuccess) {
            S->pool = nullptr;
            set_error("opf_serve_create: pool of %zu bytes not available", S->cap);
            throw Error{OPF_E_NOMEM};
        }
        S->regions.init(S->cap);
        auto cleanup = [&] {
            for (hipStream_t q : S->streams) (void)hipStreamDestroy(q);
            for (double* p : S->pinned) (void)hipHostFree(p);
            for (auto& ev : S->events)
                for (hipEvent_t e : ev)
                    if (e) (void)hipEventDestroy(e);
            (void)hipFree(S->pool);
        };
        for (int k = 0; k < S->o.slots; k++) {
            hipStream_t s = nullptr;
            double* pin = nullptr;
            std::array<hipEvent_t, 10> ev{};
            bool ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
            if (ok) S->streams.push_back(s);
            ok = ok && hipHostMalloc((void**)&pin, 16 * sizeof(double)) == hipSuccess;
            if (ok) S->pinned.push_back(pin);
            for (auto& e : ev) ok = ok && hipEventCreate(&e) == hipSuccess;
            S->events.push_back(ev);
            if (!ok) {
                cleanup();
                set_error("opf_serve_create: stream, pinned buffer or event creation failed");
                throw Error{OPF_E_DEVICE};
            }
        }
        opf_server* raw = S.release();
        for (int k = 0; k < raw->o.slots; k++) raw->workers.emplace_back(worker, raw, k);
        *out = raw;
    });
}

extern "C" int opf_serve_submit(opf_server* S, const opf_grid* grid, int64_t tag) {
    return guarded([&] {
        OPF_CHECK(S && grid, OPF_E_INVALID, "opf_serve_submit: null argument");
        Request rq;
        rq.tag = tag;
        rq.t_submit = now_s();
        rq.grid = std::make_shared<GridCopy>(*grid);
        // only the grid's checks here: its model is built by the worker that takes it, in parallel with the
        // other workers (building it here made every submission wait for the ones before it)
        const int rc = validate_grid(&rq.grid->g);
        if (rc != OPF_OK) throw Error{rc};
        std::lock_guard<std::mutex> lk(S->mu);
        OPF_CHECK(!S->done.count(tag) && !S->active.count(tag), OPF_E_INVALID,
                  "opf_serve_submit: tag %lld is already in use", (long long)tag);
        S->active.insert(tag);
        S->queue.push_back(std::move(rq));
        S->cv_work.notify_one();
    });
}

extern "C" int opf_serve_poll(opf_server* S, serve_result* out, int32_t max, int32_t* count, int32_t wait) {
    return guarded([&] {
        OPF_CHECK(S && count && (out || max == 0) && max >= 0, OPF_E_INVALID, "opf_serve_poll: bad argument");
        std::unique_lock<std::mutex> lk(S->mu);
        if (wait)
            S->cv_done.wait(lk, [&] {
                return !S->ready.empty() ||
                       (S->queue.empty() && S->running == 0 && !S->creating && S->preparing == 0);
            });
        int k = 0;
        while (k < max && !S->ready.empty()) {
            out[k++] = S->done[S->ready.front()].r;
            S->ready.pop_front();
        }
        *count = k;
    });
}

extern "C" int opf_serve_get_x(opf_server* S, int64_t tag, double* x, int32_t n) {
    return guarded([&] {
        OPF_CHECK(S && x, OPF_E_INVALID, "opf_serve_get_x: null argument");
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->done.find(tag);
        OPF_CHECK(it != S->done.end(), OPF_E_INVALID, "opf_serve_get_x: no result for tag %lld", (long long)tag);
        OPF_CHECK((size_t)n == it->second.x.size() && n > 0, OPF_E_INVALID, "opf_serve_get_x: n is %d, the result has %zu",
                  n, it->second.x.size());
        std::copy(it->second.x.begin(), it->second.x.end(), x);
    });
}

extern "C" int opf_serve_stats(const opf_server* S, int64_t* in_use, int64_t* peak_in_use, int32_t* running,
                               int32_t* queued) {
    return guarded([&] {
        OPF_CHECK(S, OPF_E_INVALID, "opf_serve_stats: null server");
        auto* M = const_cast<opf_server*>(S);
        std::lock_guard<std::mutex> lk(M->mu);
        if (in_use) *in_use = (int64_t)M->in_use;
        if (peak_in_use) *peak_in_use = (int64_t)M->peak;
        if (running) *running = M->running + (M->creating ? 1 : 0);
        if (queued) *queued = (int32_t)M->queue.size() + M->preparing;
    });
}

extern "C" int opf_serve_destroy(opf_server* S) {
    if (!S) return OPF_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
    }
    for (auto& t : S->workers) t.join();
    for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
    for (double* p : S->pinned) (void)hipHostFree(p);
    for (auto& ev : S->events)
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    if (S->pool) (void)hipFree(S->pool);
    delete S;
    return OPF_OK;
}
