// Serving loop: continuous batching of t-SVT and completion requests.
//
// A host thread owns the device state of every admitted request.  Requests
// are admitted in arrival order (first in, first out, so none starves) while
// their device-memory footprint fits the budget and fewer than max_active are
// running.  Each tick advances every admitted request by one step in a single
// batched call: a t-SVT request finishes in one tick; a completion request
// runs one iteration of Algorithm 1 per tick with its iterates X, M (and, for
// FP32 data, the right singular vectors that warm-start its next Jacobi SVDs)
// kept on the device between ticks.  A request that arrives while a tick runs
// joins at the next tick; a finished one releases its memory at once.
//
// Every request carries its own device status word through the batched step,
// so a failure (a non-finite input, a Jacobi SVD that hit its sweep limit)
// marks only that request.  Device buffers come from a pool owned by the
// server: steady-state ticks make no device allocation.  Admission, ordering,
// cancellation and deadlines are decided by the host-only scheduler in
// sched.h, which the tests drive without a GPU.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/tsvdmi.h"
#include "internal.h"
#include "sched.h"

namespace {

struct Req {
    int64_t id = 0;
    int kind = TSVD_REQ_TSVT;
    int64_t n1 = 0, n2 = 0, n3 = 0, N = 0;
    double tau = 0.0, tau0 = 0.0, tau1 = 0.0;
    int iters = 1, done_iters = 0;
    std::vector<unsigned char> input;  // Z (t-SVT) or B (completion), element type of the server
    std::vector<uint8_t> mask;
    double t_submit = 0.0, t_admit = -1.0, t_done = -1.0;
    int status = TSVD_OK;
    void *dIn = nullptr, *dOut = nullptr, *dM = nullptr, *dV = nullptr;
    uint8_t* dMask = nullptr;
    std::vector<unsigned char> result;
};

double tau_at(const Req& r, int l) {
    if (r.iters <= 1) return r.tau0;
    return r.tau0 * pow(r.tau1 / r.tau0, (double)l / (double)(r.iters - 1));
}

// Device buffers kept for reuse: a freed buffer goes back to a free list keyed
// by size and serves any later request of up to its size (and at least half
// of it).  Only a miss allocates.  Cached bytes beyond `cap` are released.
struct DevPool {
    std::multimap<size_t, void*> free_;
    size_t cached = 0, cap = 0;
    static size_t round(size_t b) { return (b + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1); }
    void* get(size_t bytes, size_t* got) {
        const size_t want = round(bytes);
        auto it = free_.lower_bound(want);
        if (it != free_.end() && it->first <= 2 * want) {
            void* p = it->second;
            *got = it->first;
            cached -= it->first;
            free_.erase(it);
            return p;
        }
        void* p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            trim(0);  // give cached buffers back and retry once
            if (hipMalloc(&p, want) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
        }
        *got = want;
        return p;
    }
    void put(void* p, size_t bytes) {
        if (!p) return;
        free_.emplace(bytes, p);
        cached += bytes;
        trim(cap);
    }
    void trim(size_t keep) {
        while (cached > keep && !free_.empty()) {
            auto it = std::prev(free_.end());
            (void)hipFree(it->second);
            cached -= it->first;
            free_.erase(it);
        }
    }
};

}  // namespace

struct tsvd_server {
    tsvd_ctx* ctx = nullptr;
    int prec = TSVD_FP32;
    size_t es = 4;
    int warm_period = 0;  // completion requests: Jacobi warm start, V reset every warm_period iterations (0: off)
    std::mutex mu;
    std::condition_variable cv;
    tsvd::Scheduler sched;                                 // admission, order, cancel, deadlines (under mu)
    std::unordered_map<int64_t, std::shared_ptr<Req>> all;  // submitted and not yet polled
    std::vector<std::shared_ptr<Req>> active;               // server thread only
    int64_t n_ticks = 0;
    bool stop = false;
    std::thread th;
    hipStream_t stream = nullptr;
    DevPool pool;
    std::unordered_map<void*, size_t> pool_sizes;  // server thread only
    std::chrono::steady_clock::time_point t0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    void* dev(size_t bytes) {
        size_t got = 0;
        void* p = pool.get(bytes, &got);
        if (p) pool_sizes[p] = got;
        return p;
    }
    void release(void* p) {
        if (!p) return;
        auto it = pool_sizes.find(p);
        pool.put(p, it->second);
        pool_sizes.erase(it);
    }
    void free_dev(Req& r) {
        release(r.dIn);
        release(r.dOut);
        release(r.dM);
        release(r.dV);
        release(r.dMask);
        r.dIn = r.dOut = r.dM = r.dV = nullptr;
        r.dMask = nullptr;
    }

    size_t vbytes(int64_t n1, int64_t n2, int64_t n3) const {
        const int64_t p = n1 < n2 ? n1 : n2;
        return (size_t)p * p * n3 * es;
    }

    // Device state of an admitted request: inputs copied in, the completion's
    // initial iterate X = B on the observed set (Algorithm 1), M = 0.
    int stage(Req& r) {
        const size_t bytes = (size_t)r.N * es;
        const int dp = prec == TSVD_FP64 ? 0 : 1;
        if (!(r.dIn = dev(bytes)) || !(r.dOut = dev(bytes))) return TSVD_ENOMEM;
        if (hipMemcpyAsync(r.dIn, r.input.data(), bytes, hipMemcpyHostToDevice, stream) != hipSuccess) return TSVD_EHIP;
        if (r.kind == TSVD_REQ_COMPLETE) {
            if (!(r.dM = dev(bytes)) || !(r.dMask = (uint8_t*)dev((size_t)r.N))) return TSVD_ENOMEM;
            if (hipMemcpyAsync(r.dMask, r.mask.data(), (size_t)r.N, hipMemcpyHostToDevice, stream) != hipSuccess)
                return TSVD_EHIP;
            if (tsvd::launch_observed_init(dp, r.dOut, r.dIn, r.dMask, r.N, stream) != hipSuccess ||
                tsvd::launch_fill_zero(r.dM, (int64_t)bytes, stream) != hipSuccess)
                return TSVD_EHIP;
            // the request's right singular vectors, kept across its iterations (the first
            // step starts them from the identity)
            if (warm_period > 0 && !(r.dV = dev(vbytes(r.n1, r.n2, r.n3)))) return TSVD_ENOMEM;
        }
        return TSVD_OK;
    }

    void finish(Req& r, int status) {
        if (status >= 0) {
            r.result.resize((size_t)r.N * es);
            if (hipMemcpy(r.result.data(), r.dOut, r.result.size(), hipMemcpyDeviceToHost) != hipSuccess)
                status = TSVD_EHIP;
        }
        free_dev(r);
        std::lock_guard<std::mutex> lk(mu);
        r.status = status;
        r.t_done = now();
        sched.finish(r.id, status);
    }

    void loop() {
        (void)hipSetDevice(tsvd_ctx_device(ctx));
        for (;;) {
            std::vector<std::shared_ptr<Req>> fresh;
            std::vector<std::pair<int64_t, int>> ended;  // active requests cancelled or past their deadline
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    const double t = now();
                    sched.expire(t);  // pending requests past their deadline end here
                    for (int64_t id : sched.admit(t)) {
                        auto r = all.at(id);
                        r->t_admit = t;
                        fresh.push_back(r);
                    }
                    ended = sched.take_stopped(t);
                    if (stop) return;
                    if (!fresh.empty() || !ended.empty() || !active.empty()) break;
                    cv.wait_for(lk, std::chrono::milliseconds(20));
                }
            }
            for (auto& r : fresh) {
                const int rc = stage(*r);
                if (rc != TSVD_OK) r->status = rc;
                active.push_back(r);
            }
            // one batched step over every admitted request still running
            std::vector<tsvd::BatchJobSpec> jb;
            std::vector<std::shared_ptr<Req>> in_step;
            for (auto& r : active) {
                bool stopped = false;
                for (auto& e : ended)
                    if (e.first == r->id) {
                        r->status = e.second;
                        stopped = true;
                    }
                if (stopped || r->status < 0) continue;
                tsvd::BatchJobSpec s{};
                s.n1 = r->n1;
                s.n2 = r->n2;
                s.n3 = r->n3;
                if (r->kind == TSVD_REQ_TSVT) {
                    s.Z = r->dIn;
                    s.Y = r->dOut;
                    s.tau = r->tau;
                    s.beta = 1.0;
                } else {
                    const double t = tau_at(*r, r->done_iters);
                    s.X = r->dOut;
                    s.M = r->dM;
                    s.B = r->dIn;
                    s.mask = r->dMask;
                    s.tau = t;
                    s.beta = 1.0 / t;
                    if (r->dV) {
                        s.V = r->dV;
                        s.vinit = (r->done_iters % warm_period) != 0;
                    }
                }
                jb.push_back(s);
                in_step.push_back(r);
            }
            std::vector<int> js(jb.size(), TSVD_OK);
            int rc = TSVD_OK;
            if (!jb.empty()) rc = tsvd_batched_step_sync(ctx, prec, (int)jb.size(), jb.data(), js.data(), stream);
            {
                std::lock_guard<std::mutex> lk(mu);
                ++n_ticks;
            }
            for (size_t j = 0; j < in_step.size(); ++j) {
                Req& r = *in_step[j];
                if (rc < 0) {
                    r.status = rc;  // the step itself failed: none of its jobs has a result
                    continue;
                }
                if (js[j] < 0) {
                    r.status = js[j];  // this request alone failed
                    continue;
                }
                if (js[j] > 0 && r.status == TSVD_OK) r.status = js[j];  // a warning: outputs written
                r.done_iters += 1;
            }
            std::vector<std::shared_ptr<Req>> still;
            for (auto& r : active) {
                const bool fin = r->status < 0 || r->kind == TSVD_REQ_TSVT || r->done_iters >= r->iters;
                if (fin) finish(*r, r->status);
                else still.push_back(r);
            }
            active.swap(still);
        }
    }
};

extern "C" {

int tsvd_server_create(tsvd_server** out, tsvd_ctx* ctx, int prec, int64_t budget_bytes, int max_active) {
    if (!out) return TSVD_EINVAL;
    *out = nullptr;
    if (!ctx || budget_bytes <= 0 || max_active <= 0) return TSVD_EINVAL;
    if (prec != TSVD_FP64 && prec != TSVD_FP32 && prec != TSVD_MIXED) return TSVD_EINVAL;
    auto* s = new tsvd_server();
    s->ctx = ctx;
    s->prec = prec;
    s->es = prec == TSVD_FP64 ? 8 : 4;
    s->sched.configure(budget_bytes, max_active);
    s->pool.cap = (size_t)budget_bytes;
    // the context's warm-start setting (FP32 data only: the batched kernel's one-workgroup
    // blocks of FP64 columns with V do not fit in LDS for the largest slices)
    const int ws = (int)tsvd_get_option(ctx, TSVD_OPT_WARM_START);
    s->warm_period = prec == TSVD_FP64 ? 0 : (ws < 0 ? 64 : ws);
    s->t0 = std::chrono::steady_clock::now();
    (void)hipSetDevice(tsvd_ctx_device(ctx));
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return TSVD_EHIP;
    }
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return TSVD_OK;
}

int64_t tsvd_server_submit(tsvd_server* s, const tsvd_request* q) {
    if (!s || !q) return TSVD_EINVAL;
    if (q->n1 <= 0 || q->n2 <= 0 || q->n3 <= 0 || !q->input) return TSVD_EINVAL;
    if (q->kind != TSVD_REQ_TSVT && q->kind != TSVD_REQ_COMPLETE) return TSVD_EINVAL;
    if (q->kind == TSVD_REQ_TSVT && (!(q->tau >= 0.0) || !isfinite(q->tau))) return TSVD_EINVAL;
    if (q->kind == TSVD_REQ_COMPLETE &&
        (!q->mask || q->iters <= 0 || !(q->tau0 > 0.0) || !(q->tau1 > 0.0) || !isfinite(q->tau0) ||
         !isfinite(q->tau1)))
        return TSVD_EINVAL;
    if (!(q->deadline_s >= 0.0) && !(q->deadline_s < 0.0)) return TSVD_EINVAL;  // NaN
    const int with_v = q->kind == TSVD_REQ_COMPLETE && s->warm_period > 0;
    // the shapes a batched step can hold (slices of at most 512 rows, Jacobi block in LDS)
    if (tsvd_batched_shape_check(s->prec, q->n1, q->n2, with_v) != TSVD_OK) return TSVD_EINVAL;
    auto r = std::make_shared<Req>();
    r->kind = q->kind;
    r->n1 = q->n1;
    r->n2 = q->n2;
    r->n3 = q->n3;
    r->N = q->n1 * q->n2 * q->n3;
    const size_t N = (size_t)r->N;
    if (q->kind == TSVD_REQ_TSVT) {
        r->tau = q->tau;
        r->iters = 1;
    } else {
        r->iters = q->iters;
        r->tau0 = q->tau0;
        r->tau1 = q->tau1;
        r->mask.assign(q->mask, q->mask + N);
    }
    r->input.resize(N * s->es);
    if (s->es == 8) {
        double* d = (double*)r->input.data();
        for (size_t e = 0; e < N; ++e) d[e] = (double)q->input[e];
    } else {
        memcpy(r->input.data(), q->input, N * 4);
    }
    const size_t tensors = q->kind == TSVD_REQ_TSVT ? 2 : 3;
    const size_t footprint = tensors * N * s->es + (q->kind == TSVD_REQ_COMPLETE ? N : 0) +
                             (with_v ? s->vbytes(q->n1, q->n2, q->n3) : 0) +
                             tsvd_batched_workspace_bytes(s->prec, q->n1, q->n2, q->n3);
    std::lock_guard<std::mutex> lk(s->mu);
    const double t = s->now();
    const int64_t id = s->sched.submit((int64_t)footprint, t, q->deadline_s > 0.0 ? t + q->deadline_s : 0.0);
    if (id < 0) return id;  // TSVD_EBUSY: can never fit the budget
    r->id = id;
    r->t_submit = t;
    s->all[id] = r;
    s->cv.notify_one();
    return id;
}

int tsvd_server_cancel(tsvd_server* s, int64_t id) {
    if (!s) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return TSVD_EINVAL;
    const int rc = s->sched.cancel(id, s->now());
    if (rc == 0 && s->sched.state(id) == tsvd::Scheduler::kDone) {
        // it was still queued: it ends now, with no device state
        it->second->status = TSVD_ECANCELED;
        it->second->t_done = s->now();
    }
    s->cv.notify_one();
    return rc;
}

int tsvd_server_poll(tsvd_server* s, int64_t id, float* out, double* t_submit, double* t_admit, double* t_done) {
    if (!s) return TSVD_EINVAL;
    std::shared_ptr<Req> r;
    int st = TSVD_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(id);
        if (it == s->all.end()) return TSVD_EINVAL;
        r = it->second;
        if (s->sched.state(id) != tsvd::Scheduler::kDone) return 0;
        st = s->sched.status(id);
        if (r->t_done < 0.0) r->t_done = s->now();  // ended in the queue (deadline)
        s->sched.forget(id);
        s->all.erase(it);
    }
    if (t_submit) *t_submit = r->t_submit;
    if (t_admit) *t_admit = r->t_admit;
    if (t_done) *t_done = r->t_done;
    if (st < 0) return st;
    if (out) {
        const size_t N = (size_t)r->N;
        if (s->es == 8)
            for (size_t e = 0; e < N; ++e) out[e] = (float)((const double*)r->result.data())[e];
        else
            memcpy(out, r->result.data(), N * 4);
    }
    return st == TSVD_WARN_NOCONV ? 2 : 1;
}

double tsvd_server_now(tsvd_server* s) { return s ? s->now() : -1.0; }

int tsvd_server_stats(tsvd_server* s, int64_t* admitted, int64_t* completed, int64_t* ticks, int64_t* peak_bytes) {
    if (!s) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (admitted) *admitted = s->sched.admitted();
    if (completed) *completed = s->sched.completed();
    if (ticks) *ticks = s->n_ticks;
    if (peak_bytes) *peak_bytes = s->sched.peak();
    return TSVD_OK;
}

void tsvd_server_destroy(tsvd_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    (void)hipStreamSynchronize(s->stream);
    for (auto& r : s->active) s->free_dev(*r);
    s->pool.trim(0);
    (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
