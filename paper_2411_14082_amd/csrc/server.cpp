// Request loop: circuits of different sizes, each a sequence of Newton-Raphson
// refactorization + solve steps, served with continuous admission.  A fixed
// number of slots (host worker threads, each with its own HIP stream of default
// priority) take requests in arrival order; a request is analysed and factored
// on the host, then admitted when its resident device footprint fits the HBM
// budget next to the requests already on the device, runs its steps on its
// slot's stream (so the kernels of different requests overlap on the GPU), and
// releases its memory.  The numerical work of a request is the same calls as a
// single context would make, so its results do not depend on the mix.
#include <hip/hip_runtime_api.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "cktlu.h"

struct cktlu_server {
    cktlu_server_options opt;
    std::chrono::steady_clock::time_point t0;
    struct Req {
        cktlu_request r;
        std::vector<int32_t> colptr, rowind;
    };
    std::mutex mu;
    std::condition_variable cv_work, cv_mem, cv_done;
    std::deque<Req> pending;
    std::deque<cktlu_request_done> done;
    double used = 0.0;             // footprint of the admitted requests
    int resident = 0;
    bool stopping = false;
    std::vector<std::thread> workers;
    int device = 0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void worker(int slot);
};

namespace {

// One request on one slot; fills everything in d except tag and the arrival time.
int serve_one(cktlu_server *srv, cktlu_server::Req &q, hipStream_t st, cktlu_request_done &d) {
    const cktlu_request &r = q.r;
    const int64_t nnz = q.colptr.empty() ? 0 : q.colptr.back();
    cktlu_options o = srv->opt.lu;
    o.stream = st;
    o.timing = 0;
    // no slot map: a request's few steps do not repay building it on the host, and the
    // slots' requests would each size it against the same free memory
    o.sweep_slot_map = -1;
    cktlu_ctx *ctx = nullptr;
    int rc = cktlu_create(&ctx, &o);
    if (rc) return rc;
    struct Guard {
        cktlu_ctx *c;
        ~Guard() { cktlu_destroy(c); }
    } guard{ctx};
    if ((rc = cktlu_analyze(ctx, r.n, q.colptr.data(), q.rowind.data()))) return rc;
    // host factorization with the first step's values; nothing is on the device yet
    std::vector<double> v0((size_t)nnz);
    if (nnz && hipMemcpyAsync(v0.data(), r.values_dev, (size_t)nnz * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
        return CKTLU_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return CKTLU_E_HIP;
    if ((rc = cktlu_factorize_host(ctx, v0.data()))) return rc;
    d.footprint = cktlu_footprint_bytes(ctx, 1);
    {
        // admission: wait until the footprint fits next to the resident requests
        // (a request larger than the whole budget runs alone)
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->cv_mem.wait(lk, [&] {
            return srv->resident == 0 || srv->used + (double)d.footprint <= srv->opt.hbm_budget_bytes;
        });
        srv->used += (double)d.footprint;
        srv->resident++;
    }
    d.admit_s = srv->now();
    int first_err = 0;
    for (int t = 0; t < r.nsteps; t++) {
        cktlu_refactor_info ri;
        cktlu_solve_info si;
        int a = cktlu_refactorize(ctx, r.values_dev + (size_t)t * nnz, &ri);
        if (a < 0) { first_err = a; break; }
        if (a == CKTLU_W_REPIVOTED) d.repivots++;
        int b = cktlu_solve(ctx, 1, r.b_dev, r.n, r.x_dev + (size_t)t * r.n, r.n, &si);
        if (b < 0) { first_err = b; break; }
        if (b == CKTLU_W_IR_FALLBACK) d.fp64_fallbacks++;
        d.backward_err = si.backward_err;
        if (a > 0 && !d.status) d.status = a;
        if (b > 0 && !d.status) d.status = b;
    }
    if (hipStreamSynchronize(st) != hipSuccess && !first_err) first_err = CKTLU_E_HIP;
    d.end_s = srv->now();
    return first_err ? first_err : d.status;
}

}  // namespace

void cktlu_server::worker(int slot) {
    (void)slot;
    if (hipSetDevice(device) != hipSuccess) return;
    hipStream_t st = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
        Req q;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stopping || !pending.empty(); });
            if (pending.empty()) break;              // stopping, nothing left
            q = std::move(pending.front());
            pending.pop_front();
        }
        cktlu_request_done d;
        std::memset(&d, 0, sizeof(d));
        d.tag = q.r.tag;
        d.arrival_s = q.r.arrival_s;
        d.start_s = now();
        d.backward_err = -1.0;
        d.status = have_stream ? serve_one(this, q, st, d) : CKTLU_E_HIP;
        if (!d.end_s) d.end_s = now();
        {
            std::lock_guard<std::mutex> lk(mu);
            if (d.admit_s > 0) {
                used -= (double)d.footprint;
                resident--;
            }
            done.push_back(d);
        }
        cv_mem.notify_all();
        cv_done.notify_all();
    }
    if (st) (void)hipStreamDestroy(st);
}

extern "C" {

void cktlu_server_default_options(cktlu_server_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->slots = 4;
    o->hbm_budget_bytes = 0.0;
    cktlu_default_options(&o->lu);
}

int cktlu_server_create(cktlu_server **out, const cktlu_server_options *opt) {
    if (!out) return CKTLU_E_ARG;
    *out = nullptr;
    cktlu_server *s = new (std::nothrow) cktlu_server();
    if (!s) return CKTLU_E_NOMEM;
    if (opt) s->opt = *opt; else cktlu_server_default_options(&s->opt);
    if (s->opt.slots < 1 || s->opt.slots > 64) { delete s; return CKTLU_E_ARG; }
    if (hipGetDevice(&s->device) != hipSuccess) { delete s; return CKTLU_E_HIP; }
    if (s->opt.hbm_budget_bytes <= 0.0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) { delete s; return CKTLU_E_HIP; }
        s->opt.hbm_budget_bytes = 0.8 * (double)fr;
    }
    s->t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < s->opt.slots; i++) s->workers.emplace_back(&cktlu_server::worker, s, i);
    *out = s;
    return CKTLU_OK;
}

double cktlu_server_now(const cktlu_server *s) { return s ? s->now() : 0.0; }

int cktlu_server_submit(cktlu_server *s, const cktlu_request *r) {
    if (!s || !r || r->n < 0 || r->nsteps < 0 || !r->colptr || (r->nsteps > 0 && (!r->values_dev || !r->b_dev || !r->x_dev)))
        return CKTLU_E_ARG;
    cktlu_server::Req q;
    q.r = *r;
    q.colptr.assign(r->colptr, r->colptr + r->n + 1);
    q.rowind.assign(r->rowind, r->rowind + q.colptr.back());
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return CKTLU_E_STATE;
        s->pending.push_back(std::move(q));
    }
    s->cv_work.notify_one();
    return CKTLU_OK;
}

int cktlu_server_poll(cktlu_server *s, cktlu_request_done *out, int32_t max, int32_t wait_ms) {
    if (!s || (!out && max > 0) || max < 0) return CKTLU_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
    int k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    return k;
}

void cktlu_server_destroy(cktlu_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    delete s;
}

}  // extern "C"
