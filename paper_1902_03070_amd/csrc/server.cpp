// Serving loop: continuous batching of t-SVT and completion requests.
//
// A host thread owns the device state of every admitted request.  Requests
// are admitted in arrival order (first in, first out, so none starves) while
// their device-memory footprint fits the budget and fewer than max_active are
// running.  Each tick advances every admitted request by one step in a single
// batched call: a t-SVT request finishes in one tick; a completion request
// runs one iteration of Algorithm 1 per tick with its iterates X, M (and, for
// FP32 data, the right singular vectors that warm-start its next Jacobi SVDs)
// kept on the device between ticks.  A request that arrives while a tick runs joins
// at the next tick; a finished one releases its memory at once.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/tsvdmi.h"
#include "internal.h"

namespace {

struct Req {
    int64_t id = 0;
    int kind = TSVD_REQ_TSVT;
    int64_t n1 = 0, n2 = 0, n3 = 0, N = 0;
    double tau = 0.0, tau0 = 0.0, tau1 = 0.0;
    int iters = 1, done_iters = 0;
    std::vector<unsigned char> input;  // Z (t-SVT) or B (completion), element type of the server
    std::vector<unsigned char> x0;     // completion: initial X (B on the observed set)
    std::vector<uint8_t> mask;
    size_t footprint = 0;
    double t_submit = 0.0, t_admit = -1.0, t_done = -1.0;
    bool admitted = false, done = false;
    int status = TSVD_OK;
    void *dIn = nullptr, *dOut = nullptr, *dM = nullptr, *dV = nullptr;
    uint8_t* dMask = nullptr;
    std::vector<unsigned char> result;
};

double tau_at(const Req& r, int l) {
    if (r.iters <= 1) return r.tau0;
    return r.tau0 * pow(r.tau1 / r.tau0, (double)l / (double)(r.iters - 1));
}

}  // namespace

struct tsvd_server {
    tsvd_ctx* ctx = nullptr;
    int prec = TSVD_FP32;
    size_t es = 4;
    int64_t budget = 0;
    int max_active = 1;
    int warm_period = 0;  // completion requests: Jacobi warm start, V reset every warm_period iterations (0: off)
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Req>> pending;
    std::vector<std::shared_ptr<Req>> active;
    std::unordered_map<int64_t, std::shared_ptr<Req>> all;
    int64_t next_id = 1, held = 0, peak = 0, n_admitted = 0, n_completed = 0, n_ticks = 0;
    bool stop = false;
    std::thread th;
    hipStream_t stream = nullptr;
    std::chrono::steady_clock::time_point t0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    void free_dev(Req& r) {
        if (r.dIn) (void)hipFree(r.dIn);
        if (r.dOut) (void)hipFree(r.dOut);
        if (r.dM) (void)hipFree(r.dM);
        if (r.dV) (void)hipFree(r.dV);
        if (r.dMask) (void)hipFree(r.dMask);
        r.dIn = r.dOut = r.dM = r.dV = nullptr;
        r.dMask = nullptr;
    }

    size_t vbytes(const Req& r) const {
        const int64_t p = r.n1 < r.n2 ? r.n1 : r.n2;
        return (size_t)p * p * r.n3 * es;
    }

    // Allocate and fill the request's device state (server thread, no lock held).
    int stage(Req& r) {
        const size_t bytes = (size_t)r.N * es;
        if (hipMalloc(&r.dIn, bytes) != hipSuccess || hipMalloc(&r.dOut, bytes) != hipSuccess) return TSVD_ENOMEM;
        if (hipMemcpyAsync(r.dIn, r.input.data(), bytes, hipMemcpyHostToDevice, stream) != hipSuccess) return TSVD_EHIP;
        if (r.kind == TSVD_REQ_COMPLETE) {
            if (hipMalloc(&r.dM, bytes) != hipSuccess || hipMalloc((void**)&r.dMask, (size_t)r.N) != hipSuccess)
                return TSVD_ENOMEM;
            if (hipMemcpyAsync(r.dOut, r.x0.data(), bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
                hipMemsetAsync(r.dM, 0, bytes, stream) != hipSuccess ||
                hipMemcpyAsync(r.dMask, r.mask.data(), (size_t)r.N, hipMemcpyHostToDevice, stream) != hipSuccess)
                return TSVD_EHIP;
            // the request's right singular vectors, kept across its iterations (the first
            // step starts them from the identity)
            if (warm_period > 0 && hipMalloc(&r.dV, vbytes(r)) != hipSuccess) return TSVD_ENOMEM;
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
        r.status = status;
        std::lock_guard<std::mutex> lk(mu);
        r.t_done = now();
        r.done = true;
        held -= (int64_t)r.footprint;
        ++n_completed;
    }

    void loop() {
        (void)hipSetDevice(tsvd_ctx_device(ctx));
        for (;;) {
            std::vector<std::shared_ptr<Req>> fresh;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    while (!pending.empty() && (int)active.size() < max_active &&
                           held + (int64_t)pending.front()->footprint <= budget) {
                        auto r = pending.front();
                        pending.pop_front();
                        held += (int64_t)r->footprint;
                        peak = held > peak ? held : peak;
                        r->admitted = true;
                        r->t_admit = now();
                        ++n_admitted;
                        active.push_back(r);
                        fresh.push_back(r);
                    }
                    if (stop) return;
                    if (!active.empty()) break;
                    cv.wait_for(lk, std::chrono::milliseconds(50));
                }
            }
            for (auto& r : fresh) {
                const int rc = stage(*r);
                if (rc != TSVD_OK) r->status = rc;
            }
            // one batched step over every admitted request
            std::vector<tsvd::BatchJobSpec> jb;
            std::vector<std::shared_ptr<Req>> in_step;
            for (auto& r : active) {
                if (r->status < 0) continue;
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
            int rc = TSVD_OK;
            if (!jb.empty()) rc = tsvd_batched_step_sync(ctx, prec, (int)jb.size(), jb.data(), stream);
            {
                std::lock_guard<std::mutex> lk(mu);
                ++n_ticks;
            }
            std::vector<std::shared_ptr<Req>> still;
            for (auto& r : active) {
                bool fin = false;
                int st = r->status;
                if (st < 0) {
                    fin = true;
                } else if (rc < 0) {
                    fin = true;
                    st = rc;
                } else {
                    if (rc > 0 && st == TSVD_OK) st = rc;
                    r->status = st;
                    r->done_iters += 1;
                    fin = (r->kind == TSVD_REQ_TSVT) || r->done_iters >= r->iters;
                }
                if (fin) finish(*r, st);
                else still.push_back(r);
            }
            std::lock_guard<std::mutex> lk(mu);
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
    s->budget = budget_bytes;
    s->max_active = max_active;
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
    auto r = std::make_shared<Req>();
    r->kind = q->kind;
    r->n1 = q->n1;
    r->n2 = q->n2;
    r->n3 = q->n3;
    r->N = q->n1 * q->n2 * q->n3;
    const size_t N = (size_t)r->N;
    if (q->kind == TSVD_REQ_TSVT) {
        if (!(q->tau >= 0.0) || !isfinite(q->tau)) return TSVD_EINVAL;
        r->tau = q->tau;
        r->iters = 1;
    } else {
        if (!q->mask || q->iters <= 0 || !(q->tau0 > 0.0) || !(q->tau1 > 0.0)) return TSVD_EINVAL;
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
    if (q->kind == TSVD_REQ_COMPLETE) {
        r->x0.resize(N * s->es);
        for (size_t e = 0; e < N; ++e) {
            const bool o = r->mask[e] != 0;
            if (s->es == 8) ((double*)r->x0.data())[e] = o ? ((double*)r->input.data())[e] : 0.0;
            else ((float*)r->x0.data())[e] = o ? q->input[e] : 0.0f;
        }
    }
    const size_t tensors = q->kind == TSVD_REQ_TSVT ? 2 : 3;
    r->footprint = tensors * N * s->es + (q->kind == TSVD_REQ_COMPLETE ? N : 0) +
                   (q->kind == TSVD_REQ_COMPLETE && s->warm_period > 0 ? s->vbytes(*r) : 0) +
                   tsvd_batched_workspace_bytes(s->prec, q->n1, q->n2, q->n3);
    std::lock_guard<std::mutex> lk(s->mu);
    if ((int64_t)r->footprint > s->budget) return TSVD_EBUSY;
    r->id = s->next_id++;
    r->t_submit = s->now();
    s->all[r->id] = r;
    s->pending.push_back(r);
    s->cv.notify_one();
    return r->id;
}

int tsvd_server_poll(tsvd_server* s, int64_t id, float* out, double* t_submit, double* t_admit, double* t_done) {
    if (!s) return TSVD_EINVAL;
    std::shared_ptr<Req> r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(id);
        if (it == s->all.end()) return TSVD_EINVAL;
        r = it->second;
        if (!r->done) return 0;
        s->all.erase(it);
    }
    if (t_submit) *t_submit = r->t_submit;
    if (t_admit) *t_admit = r->t_admit;
    if (t_done) *t_done = r->t_done;
    if (r->status < 0) return r->status;
    if (out) {
        const size_t N = (size_t)r->N;
        if (s->es == 8)
            for (size_t e = 0; e < N; ++e) out[e] = (float)((const double*)r->result.data())[e];
        else
            memcpy(out, r->result.data(), N * 4);
    }
    return 1;
}

double tsvd_server_now(tsvd_server* s) { return s ? s->now() : -1.0; }

int tsvd_server_stats(tsvd_server* s, int64_t* admitted, int64_t* completed, int64_t* ticks, int64_t* peak_bytes) {
    if (!s) return TSVD_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (admitted) *admitted = s->n_admitted;
    if (completed) *completed = s->n_completed;
    if (ticks) *ticks = s->n_ticks;
    if (peak_bytes) *peak_bytes = s->peak;
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
    (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
