// Serving form (qsim_server_*): continuous batching of circuit requests.
//
// Requests are copied at submit and compiled (lowering, fusion, pass plan)
// by host worker threads.  A scheduler thread admits compiled requests in
// arrival order as soon as a slot (one HIP stream with its own operator
// tables and reduction buffers) and pool memory for the 2^n-element state
// are free, enqueues the request's passes and FP64 reductions on the slot's
// stream, and retires it when the stream's completion event fires.  Admitted
// requests overlap on the device.  A request whose compile is still running
// may be passed by later compiled requests; a request waiting for memory is
// never passed, so wide states cannot starve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "host.h"
#include "launch.h"
#include "runtime.h"

using namespace qs;

namespace {

double clock_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) in 256-byte units.
class PoolAlloc {
  public:
    explicit PoolAlloc(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
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
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t size() const { return size_; }

  private:
    size_t size_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Request {
    int64_t id = 0;
    int n = 0;
    std::vector<qsim_gate> g;
    std::vector<double> mats;
    std::vector<qsim_pauli> terms;
    void *host_state_out = nullptr;
    Compiled c;
    bool compiled = false;
    int status = QSIM_OK;
    size_t bytes = 0, off = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    DeviceTables dt;
    Request *req = nullptr;
    double *d_red = nullptr;      // partials + outputs
    size_t cap_red = 0;
    uint64_t *d_masks = nullptr;
    size_t cap_masks = 0;
    double *h_out = nullptr;      // pinned: [norm][2 * nterms]
    size_t cap_out = 0;
};

int grow_dev(void **p, size_t *cap, size_t need) {
    if (need <= *cap) return QSIM_OK;
    if (alloc_fault()) return QSIM_E_NOMEM;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    size_t sz = std::max<size_t>(need + need / 4, 4096);
    hipError_t e = hipMalloc(p, sz);
    if (e != hipSuccess) { qk::note_hip(e, "hipMalloc (server)"); *p = nullptr; return QSIM_E_NOMEM; }
    *cap = sz;
    return QSIM_OK;
}

int grow_pinned(void **p, size_t *cap, size_t need) {
    if (need <= *cap) return QSIM_OK;
    if (alloc_fault()) return QSIM_E_NOMEM;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    size_t sz = std::max<size_t>(need + need / 4, 4096);
    hipError_t e = hipHostMalloc(p, sz, hipHostMallocDefault);
    if (e != hipSuccess) { qk::note_hip(e, "hipHostMalloc (server)"); *p = nullptr; return QSIM_E_NOMEM; }
    *cap = sz;
    return QSIM_OK;
}

}  // namespace

struct qsim_server {
    qsim_server_opts opt{};
    int device = 0;
    void *pool = nullptr;
    std::unique_ptr<PoolAlloc> alloc;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work;      // compile workers
    std::condition_variable cv_sched;     // scheduler
    std::condition_variable cv_done;      // pollers
    std::deque<Request *> to_compile;
    std::deque<Request *> waiting;        // arrival order, not yet admitted
    std::deque<qsim_result> done;
    std::vector<std::thread> workers;
    std::thread scheduler;
    bool stop = false;
    int64_t next_id = 0;
    qsim_server_stats st{};
};

namespace {

void finish(qsim_server *s, Request *r, int status, double norm, double expval) {
    qsim_result res{};
    res.id = r->id;
    res.status = status;
    res.n = r->n;
    res.norm = norm;
    res.expval = expval;
    res.t_submit = r->t_submit;
    res.t_admit = r->t_admit;
    res.t_done = clock_s();
    res.passes = r->c.stats.passes;
    std::lock_guard<std::mutex> lk(s->mu);
    s->done.push_back(res);
    s->st.completed++;
    s->cv_done.notify_all();
    delete r;
}

void worker_loop(qsim_server *s) {
    (void)hipSetDevice(s->device);
    const qsim_fuse_opts *fo = s->opt.fuse.level > 0 ? &s->opt.fuse : nullptr;
    for (;;) {
        Request *r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->to_compile.empty(); });
            if (s->to_compile.empty()) return;
            r = s->to_compile.front();
            s->to_compile.pop_front();
        }
        int rc;
        try {
            rc = compile_circuit(r->n, s->opt.dtype, r->g.data(), r->g.size(),
                                 GateInputs{r->mats.empty() ? nullptr : r->mats.data(),
                                            r->mats.size() / 2, nullptr, 0},
                                 fo, &r->c);
        } catch (const std::bad_alloc &) {
            rc = QSIM_E_NOMEM;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        r->status = rc;
        r->compiled = true;
        s->cv_sched.notify_all();
    }
}

// Enqueue a request on a slot's stream.  Called by the scheduler thread only.
int launch_request(qsim_server *s, Slot &sl, Request *r) {
    const int dtype = s->opt.dtype;
    void *state = (char *)s->pool + r->off;
    int rc;
    const Compiled &c = r->c;
    if (!c.plan.ops.empty()) {
        if ((rc = upload_plan(&sl.dt, dtype, c.plan, sl.st))) return rc;
    }
    const bool first_tile = !c.passes.empty() && c.passes[0].kind == Pass::TILE;
    if (!first_tile && (rc = qk::launch_init_zero(dtype, state, 0, 1, r->n, sl.st))) return rc;
    if (!c.passes.empty() && (rc = enqueue_passes(c, sl.dt, dtype, state, sl.st, first_tile))) return rc;
    const size_t nt = r->terms.size();
    const uint32_t nch = qk::marginal_chunks(r->n, 0);
    const uint32_t pch = qk::pauli_chunks(r->n);
    const size_t part = std::max<size_t>(nch, size_t(pch) * 2 * nt);
    if ((rc = grow_dev((void **)&sl.d_red, &sl.cap_red, (part + 1 + 2 * nt + 64) * 8))) return rc;
    double *d_part = sl.d_red, *d_out = sl.d_red + part + 32;
    if ((rc = grow_pinned((void **)&sl.h_out, &sl.cap_out, (1 + 2 * nt) * 8))) return rc;
    if ((rc = qk::launch_marginal(dtype, state, 0, 1, r->n, nullptr, 0, d_part, d_out, sl.st))) return rc;
    if (nt) {
        std::vector<uint64_t> m;
        const qk::PauliRows nrows = qk::pauli_rows(r->terms.data(), nt, &m);
        if ((rc = grow_dev((void **)&sl.d_masks, &sl.cap_masks, 8 * m.size()))) return rc;
        // synchronous copy: the slot's previous request has completed
        if ((rc = qk::note_hip(hipMemcpy(sl.d_masks, m.data(), 8 * m.size(), hipMemcpyHostToDevice), "masks")))
            return rc;
        if ((rc = qk::launch_pauli(dtype, state, 0, 1, r->n, sl.d_masks, int(nt), nrows, d_part, d_out + 1, sl.st)))
            return rc;
    }
    if ((rc = qk::note_hip(hipMemcpyAsync(sl.h_out, d_out, (1 + 2 * nt) * 8, hipMemcpyDeviceToHost, sl.st),
                           "results")))
        return rc;
    if (r->host_state_out &&
        (rc = qk::note_hip(hipMemcpyAsync(r->host_state_out, state, (size_t(1) << r->n) * elem_bytes(dtype),
                                          hipMemcpyDeviceToHost, sl.st),
                           "state out")))
        return rc;
    return qk::note_hip(hipEventRecord(sl.done, sl.st), "event");
}

void retire(qsim_server *s, Slot &sl) {
    Request *r = sl.req;
    sl.req = nullptr;
    const size_t nt = r->terms.size();
    const double norm = sl.h_out[0];
    double total = 0;
    for (size_t k = 0; k < nt; k++) {
        const double re = sl.h_out[1 + 2 * k], im = sl.h_out[2 + 2 * k];
        double v;
        switch (__builtin_popcountll(r->terms[k].xmask & r->terms[k].zmask) & 3) {
        case 0: v = re; break;
        case 1: v = -im; break;
        case 2: v = -re; break;
        default: v = im; break;
        }
        total += r->terms[k].coeff * v;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->alloc->release(r->off, r->bytes);
        s->st.in_flight--;
    }
    finish(s, r, QSIM_OK, norm, nt ? total / norm : 0.0);
}

void scheduler_loop(qsim_server *s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        bool progressed = false;
        // retire finished slots
        for (Slot &sl : s->slots) {
            if (sl.req && hipEventQuery(sl.done) == hipSuccess) {
                retire(s, sl);
                progressed = true;
            }
        }
        // admit in arrival order
        for (;;) {
            Request *r = nullptr;
            Slot *free_slot = nullptr;
            for (Slot &sl : s->slots)
                if (!sl.req) { free_slot = &sl; break; }
            {
                std::lock_guard<std::mutex> lk(s->mu);
                // first compiled request; stop at the first compiled one that does not fit
                for (auto it = s->waiting.begin(); it != s->waiting.end(); ++it) {
                    Request *q = *it;
                    if (!q->compiled) continue;
                    if (q->status != QSIM_OK) {   // compile error: report, do not admit
                        s->waiting.erase(it);
                        r = q;
                        break;
                    }
                    if (!free_slot) break;
                    if (!s->alloc->alloc(q->bytes, &q->off)) break;
                    s->waiting.erase(it);
                    s->st.in_flight++;
                    s->st.peak_in_flight = std::max(s->st.peak_in_flight, s->st.in_flight);
                    r = q;
                    break;
                }
            }
            if (!r) break;
            progressed = true;
            if (r->status != QSIM_OK) {
                finish(s, r, r->status, 0.0, 0.0);
                continue;
            }
            r->t_admit = clock_s();
            free_slot->req = r;
            const int rc = launch_request(s, *free_slot, r);
            if (rc) {
                (void)hipStreamSynchronize(free_slot->st);
                free_slot->req = nullptr;
                {
                    std::lock_guard<std::mutex> lk(s->mu);
                    s->alloc->release(r->off, r->bytes);
                    s->st.in_flight--;
                }
                finish(s, r, rc, 0.0, 0.0);
            }
        }
        bool busy = false;
        for (Slot &sl : s->slots) busy |= sl.req != nullptr;
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && !busy && s->waiting.empty() && s->to_compile.empty()) return;
        if (!progressed) {
            if (busy)
                s->cv_sched.wait_for(lk, std::chrono::microseconds(50));
            else
                s->cv_sched.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

}  // namespace

extern "C" {

double qsim_server_clock(void) { return clock_s(); }

int qsim_server_create(const qsim_server_opts *opt, qsim_server_h *out) {
    if (!opt || !out) return QSIM_E_ARG;
    if ((opt->dtype != QSIM_C64 && opt->dtype != QSIM_C128) || opt->slots < 1 || opt->slots > 64 ||
        opt->compile_threads < 1 || opt->compile_threads > 64 || opt->pool_bytes < 4096)
        return QSIM_E_ARG;
    int rc = qk::init_kernels();
    if (rc) return rc;
    qsim_server *s = new (std::nothrow) qsim_server;
    if (!s) return QSIM_E_NOMEM;
    s->opt = *opt;
    (void)hipGetDevice(&s->device);
    hipError_t e = hipMalloc(&s->pool, opt->pool_bytes);
    if (e != hipSuccess) {
        qk::note_hip(e, "hipMalloc (server pool)");
        delete s;
        return QSIM_E_NOMEM;
    }
    s->alloc.reset(new PoolAlloc(opt->pool_bytes));
    s->st.pool_bytes = opt->pool_bytes;
    s->slots.resize(size_t(opt->slots));
    for (Slot &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            s->stop = true;
            qsim_server_destroy(s);
            return QSIM_E_HIP;
        }
    }
    for (int i = 0; i < opt->compile_threads; i++) s->workers.emplace_back(worker_loop, s);
    s->scheduler = std::thread(scheduler_loop, s);
    *out = s;
    return QSIM_OK;
}

int qsim_server_submit(qsim_server_h s, const qsim_request *r, int64_t *id) {
    if (!s || !r || !id || r->n < 1 || r->n > kMaxQubits || (r->ng && !r->g) || (r->n_terms && !r->terms))
        return QSIM_E_ARG;
    const size_t bytes = (size_t(1) << r->n) * elem_bytes(s->opt.dtype);
    if (bytes > s->opt.pool_bytes) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->st.rejected++;
        return QSIM_E_CAPACITY;
    }
    Request *q = new (std::nothrow) Request;
    if (!q) return QSIM_E_NOMEM;
    try {
        q->n = r->n;
        q->g.assign(r->g, r->g + r->ng);
        if (r->mats && r->n_mats) q->mats.assign(r->mats, r->mats + 2 * r->n_mats);
        if (r->terms) q->terms.assign(r->terms, r->terms + r->n_terms);
    } catch (const std::bad_alloc &) {
        delete q;
        return QSIM_E_NOMEM;
    }
    const uint64_t lim = (uint64_t(1) << r->n) - 1;
    for (const qsim_pauli &t : q->terms)
        if ((t.xmask & ~lim) || (t.zmask & ~lim)) { delete q; return QSIM_E_ARG; }
    q->host_state_out = r->host_state_out;
    q->bytes = bytes;
    q->t_submit = clock_s();
    std::lock_guard<std::mutex> lk(s->mu);
    q->id = s->next_id++;
    *id = q->id;
    s->to_compile.push_back(q);
    s->waiting.push_back(q);
    s->st.submitted++;
    s->cv_work.notify_one();
    return QSIM_OK;
}

int qsim_server_poll(qsim_server_h s, qsim_result *out, int max, int *n_out, int wait_ms) {
    if (!s || !n_out || (max > 0 && !out)) return QSIM_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (wait_ms > 0 && s->done.empty())
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
    int k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = k;
    return QSIM_OK;
}

int qsim_server_get_stats(qsim_server_h s, qsim_server_stats *out) {
    if (!s || !out) return QSIM_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->waiting = int64_t(s->waiting.size());
    out->pool_in_use = s->alloc->used();
    out->pool_peak = s->alloc->peak();
    return QSIM_OK;
}

int qsim_server_destroy(qsim_server_h s) {
    if (!s) return QSIM_E_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
        s->cv_sched.notify_all();
    }
    for (std::thread &t : s->workers)
        if (t.joinable()) t.join();
    if (s->scheduler.joinable()) s->scheduler.join();
    for (Slot &sl : s->slots) {
        if (sl.st) (void)hipStreamSynchronize(sl.st);
        free_tables(&sl.dt);
        if (sl.d_red) (void)hipFree(sl.d_red);
        if (sl.d_masks) (void)hipFree(sl.d_masks);
        if (sl.h_out) (void)hipHostFree(sl.h_out);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.st) (void)hipStreamDestroy(sl.st);
    }
    for (Request *r : s->waiting) delete r;
    if (s->pool) (void)hipFree(s->pool);
    delete s;
    return QSIM_OK;
}

}  // extern "C"
