// C ABI of the cktlu library: context, device memory, and the control flow of
// factorize / refactorize (with the pivot-check fallback) / solve.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "internal.h"

using namespace cktlu;
using namespace cktlu_dev;

struct cktlu_ctx {
    cktlu_options opt;
    int state = 0;                 // 0 created, 1 analyzed, 2 factored
    Analysis an;
    Factor f;                      // pattern, pivots and (host) values of the current factors
    Schedule s;
    Device dev;
    cktlu_stats stats;
    bool dev_values_newer = false; // device factors hold values newer than f.Fx
    bool fp64_sticky = false;      // FP32_IR: refinement fell back; FP64 until the next factorize
    int force_fail_pending = -1;
    int last_batch = 0;            // batch of the last batched refactorization
    // the last pivot-check fallback: columns the device had not finished, and the restart set
    std::vector<char> last_unfinished, last_restart;
    // cktlu_factorize_host: the values, uploaded with the factors (FP32_IR residuals read them)
    std::vector<double> host_values;
    // options.timing: event pairs recorded around device phases, read by cktlu_get_timing
    struct Pending { int phase; hipEvent_t a, b; int launches; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    cktlu_timing timing_acc;
    // captured batched step (cktlu_step_batched_graph): replayed while its key holds
    struct GraphKey {
        int batch = 0, nrhs = 0, ir_steps = 0;
        const void *values = nullptr, *b = nullptr;
        void *status = nullptr, *x = nullptr, *eta = nullptr;
        uint64_t gen = 0;
        bool operator==(const GraphKey &o) const {
            return batch == o.batch && nrhs == o.nrhs && ir_steps == o.ir_steps && values == o.values &&
                   b == o.b && status == o.status && x == o.x && eta == o.eta && gen == o.gen;
        }
    } graph_key;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t capture_stream = nullptr;
    uint64_t buffers_gen = 1;      // bumped whenever device buffers may have moved
    // dense-block look-ahead: a second stream (default priority) and its ordering events
    hipStream_t side_stream = nullptr;
    std::vector<hipEvent_t> la_events;
};

namespace {

// CKTLU_DEBUG=1 in the environment prints the site of every HIP failure.
bool debug_on() {
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("CKTLU_DEBUG");
        v = (e && *e && *e != '0') ? 1 : 0;
    }
    return v == 1;
}
void debug_hip(int e, const char *what, int line) {
    if (debug_on())
        fprintf(stderr, "[cktlu] %s failed at cktlu.cpp:%d: %s (%d)\n", what, line,
                hipGetErrorString((hipError_t)e), e);
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) { debug_hip((int)e_, #expr, __LINE__); return CKTLU_E_HIP; }   \
    } while (0)
#define LCHK(expr)                                                                            \
    do {                                                                                      \
        int e_ = (expr);                                                                      \
        if (e_ != 0) { debug_hip(e_, #expr, __LINE__); return CKTLU_E_HIP; }                 \
    } while (0)

inline hipStream_t stream_of(const cktlu_ctx *c) { return (hipStream_t)c->opt.stream; }

// ---- phase timing (options.timing)
enum { PH_INIT, PH_SWEEP, PH_DENSE, PH_SOLVE_SPARSE, PH_SOLVE_DENSE, PH_SCHUR };

hipEvent_t take_event(cktlu_ctx *c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records the start event of a phase (nullptr when timing is off or no event).
hipEvent_t phase_begin(cktlu_ctx *c) {
    if (!c->opt.timing) return nullptr;
    hipEvent_t e = take_event(c);
    if (e && hipEventRecord(e, stream_of(c)) != hipSuccess) {
        c->event_pool.push_back(e);
        return nullptr;
    }
    return e;
}

void phase_end(cktlu_ctx *c, hipEvent_t start, int phase, int launches) {
    if (!start) return;
    hipEvent_t e = take_event(c);
    if (!e || hipEventRecord(e, stream_of(c)) != hipSuccess) {
        c->event_pool.push_back(start);
        if (e) c->event_pool.push_back(e);
        return;
    }
    c->pending.push_back({phase, start, e, launches});
}

int collect_timing(cktlu_ctx *c) {
    for (const auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess)
            return CKTLU_E_HIP;
        cktlu_timing &t = c->timing_acc;
        switch (p.phase) {
            case PH_INIT: t.init_ms += ms; break;
            case PH_SWEEP: t.sweep_ms += ms; t.sweep_launches += p.launches; break;
            case PH_DENSE: t.dense_ms += ms; t.dense_launches += p.launches; break;
            case PH_SCHUR: t.schur_ms += ms; break;
            case PH_SOLVE_SPARSE: t.solve_sparse_ms += ms; t.solve_sparse_launches += p.launches; break;
            case PH_SOLVE_DENSE: t.solve_dense_ms += ms; t.solve_dense_launches += p.launches; break;
        }
        c->event_pool.push_back(p.a);
        c->event_pool.push_back(p.b);
    }
    c->pending.clear();
    return CKTLU_OK;
}

void dfree(DevBuf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

int dalloc(DevBuf &b, size_t bytes) {
    if (b.p && b.bytes >= bytes) return CKTLU_OK;
    dfree(b);
    if (bytes == 0) bytes = 8;
    if (hipMalloc(&b.p, bytes) != hipSuccess) { b.p = nullptr; return CKTLU_E_NOMEM; }
    b.bytes = bytes;
    return CKTLU_OK;
}

template <typename V>
int upload(DevBuf &b, const std::vector<V> &v, hipStream_t st) {
    int rc = dalloc(b, v.size() * sizeof(V));
    if (rc) return rc;
    if (!v.empty()) HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, st));
    return CKTLU_OK;
}

DevBuf *all_buffers(Device &d, int i) {
    DevBuf *all[] = {&d.seq, &d.Dp, &d.Dlen, &d.Fi, &d.nU, &d.Ap, &d.colperm, &d.amap, &d.colrec, &d.task8,
                     &d.item4, &d.smap, &d.tmoff, &d.tail_nb, &d.schur_parts, &d.schur_add, &d.schur_scr,
                     &d.l21, &d.lrec, &d.urec,
                     &d.Lrjs, &d.Urjs, &d.lsptr, &d.usptr, &d.rowperm,
                     &d.colperm_sol, &d.Acp, &d.Acj, &d.Acsrc, &d.Fx64, &d.Fx32, &d.Aval, &d.done,
                     &d.ctrl, &d.vec, &d.S, &d.Dg, &d.Dinv, &d.sn_rec, &d.sn_cb, &d.sn_seq, &d.sn_task,
                     &d.sn_item, &d.sn_moff, &d.sn_item2, &d.sn_map, &d.snl_seq, &d.snu_seq, &d.Lrp, &d.Urp,
                     &d.ascale, &d.gscale, &d.sscale, &d.schur_sn_items,
                     &d.snl_unit, &d.snu_unit, &d.snl_urange, &d.snl_runs, &d.snu_urange, &d.snu_runs,
                     &d.sn_part, &d.sn_cnt, &d.sn_punit, &d.sn_sunit, &d.sn_pu2, &d.sn_su2, &d.sn_grp, &d.sn_gsrc, &d.sn_gent};
    const int cnt = (int)(sizeof(all) / sizeof(all[0]));
    return i < cnt ? all[i] : nullptr;
}

void free_device(Device &d) {
    for (int i = 0; DevBuf *b = all_buffers(d, i); i++) dfree(*b);
    d.uploaded = false;
    d.batch_cap = 0;
    d.vec_cap = 0;
    d.S_prec = -1;
}

// entries of one instance of the (padded) device factor storage
int64_t nnzF(const cktlu_ctx *c) { return c->s.nnz_dev; }

// host factor values (compact) -> device layout (columns on cache-line boundaries)
std::vector<double> pad_values(const cktlu_ctx *c, const double *compact) {
    std::vector<double> out(c->s.nnz_dev, 0.0);
    for (int k = 0; k < c->an.n; k++)
        std::copy(compact + c->f.Fp[k], compact + c->f.Fp[k + 1], out.begin() + c->s.Dp[k]);
    return out;
}

// device layout -> compact host order
void unpad_values(const cktlu_ctx *c, const double *padded, double *compact) {
    for (int k = 0; k < c->an.n; k++)
        std::copy(padded + c->s.Dp[k], padded + c->s.Dp[k] + c->s.Dlen[k], compact + c->f.Fp[k]);
}

// Status words (int32, B = batch capacity): [1, 1+B) interrupt flags,
// [1+B, 1+2B) smallest failing column per instance.
int ensure_batch(cktlu_ctx *c, int batch) {
    Device &d = c->dev;
    if (d.batch_cap >= batch) return CKTLU_OK;
    c->buffers_gen++;                 // captured graphs hold the old pointers
    const int n = c->an.n;
    const int64_t F = nnzF(c);
    hipStream_t st = stream_of(c);
    // keep instance 0 of the FP64 factors
    DevBuf old = d.Fx64;
    d.Fx64 = DevBuf();
    int rc = dalloc(d.Fx64, (size_t)F * batch * sizeof(double));
    if (rc) { d.Fx64 = old; return rc; }
    if (old.p) {
        HIPCHK(hipMemcpyAsync(d.Fx64.p, old.p, (size_t)F * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        dfree(old);
    }
    if (c->opt.precision == CKTLU_FP32_IR) {
        dfree(d.Fx32);
        if ((rc = dalloc(d.Fx32, (size_t)F * batch * sizeof(float)))) return rc;
    }
    if ((rc = dalloc(d.Aval, (size_t)c->an.nnz * batch * sizeof(double)))) return rc;
    dfree(d.done);
    if ((rc = dalloc(d.done, (size_t)n * batch * sizeof(int)))) return rc;
    HIPCHK(hipMemsetAsync(d.done.p, 0, (size_t)n * batch * sizeof(int), st));
    dfree(d.ctrl);
    if ((rc = dalloc(d.ctrl, (size_t)(8 + 2 * batch) * sizeof(int)))) return rc;
    HIPCHK(hipMemsetAsync(d.ctrl.p, 0, (size_t)(8 + 2 * batch) * sizeof(int), st));
    const size_t D = (size_t)(n - c->s.tail0);
    if (D > 0) {
        dfree(d.S);
        if ((rc = dalloc(d.S, D * D * sizeof(double) * batch))) return rc;
        dfree(d.Dg);
        if ((rc = dalloc(d.Dg, (size_t)kDenseBlock * kDenseBlock * sizeof(double) * batch))) return rc;
        dfree(d.Dinv);
        const size_t nblk = (D + kDenseBlock - 1) / kDenseBlock;
        if ((rc = dalloc(d.Dinv, nblk * 2 * kDenseBlock * kDenseBlock * sizeof(double) * batch))) return rc;
        dfree(d.schur_scr);
        if (c->s.schur_nscr > 0 &&
            (rc = dalloc(d.schur_scr, (size_t)c->s.schur_nscr * D * sizeof(double) * batch)))
            return rc;
    }
    // split supernodal solves: partial sums (512 doubles per scratch block and instance) and one
    // arrival counter per supernode, direction and instance (zero between launches)
    dfree(d.sn_part);
    dfree(d.sn_cnt);
    // (also the column maxima of split wide panels in the sweep, 64 doubles per block, and their
    // counters after the solves' two segments)
    const size_t part = std::max((size_t)std::max(c->s.snl_nscr, c->s.snu_nscr) * 512, (size_t)c->s.sn_pnscr * 64);
    if (part > 0) {
        if ((rc = dalloc(d.sn_part, part * batch * sizeof(double)))) return rc;
        const size_t cb = (size_t)3 * c->s.sn_count * batch * sizeof(int);
        if ((rc = dalloc(d.sn_cnt, cb))) return rc;
        HIPCHK(hipMemsetAsync(d.sn_cnt.p, 0, cb, st));
    }
    d.S_prec = -1;
    d.batch_cap = batch;
    return CKTLU_OK;
}

// Upload pattern, schedule and the host factor values (instance 0).
int upload_all(cktlu_ctx *c) {
    Device &d = c->dev;
    c->buffers_gen++;
    const Schedule &s = c->s;
    hipStream_t st = stream_of(c);
    int rc;
    if ((rc = upload(d.seq, s.seq, st))) return rc;
    if ((rc = upload(d.Dp, s.Dp, st))) return rc;
    if ((rc = upload(d.Dlen, s.Dlen, st))) return rc;
    if ((rc = upload(d.Fi, s.Fi_dev, st))) return rc;
    if ((rc = upload(d.nU, c->f.nU, st))) return rc;
    if ((rc = upload(d.Ap, c->an.Ap, st))) return rc;
    if ((rc = upload(d.colperm, c->an.colperm, st))) return rc;
    if ((rc = upload(d.amap, s.amap, st))) return rc;
    if ((rc = upload(d.colrec, s.colrec, st))) return rc;
    if ((rc = upload(d.task8, s.task8, st))) return rc;
    if ((rc = upload(d.tail_nb, s.tail_nb, st))) return rc;
    if ((rc = upload(d.schur_parts, s.schur_parts, st))) return rc;
    if ((rc = upload(d.schur_add, s.schur_add, st))) return rc;
    if ((rc = upload(d.l21, s.l21, st))) return rc;
    if ((rc = upload(d.item4, s.item4, st))) return rc;
    {
        // the sweep's slot map, when it takes at most a quarter of the free HBM
        dfree(d.smap);
        dfree(d.tmoff);
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = 0;
        const double mb = (double)s.smap.size() * sizeof(int);
        if (!s.smap.empty() && mb <= 0.25 * (double)fr) {
            if ((rc = upload(d.smap, s.smap, st))) return rc;
            if ((rc = upload(d.tmoff, s.tmoff, st))) return rc;
        }
        c->stats.slot_map_entries = d.smap.p ? (int64_t)s.smap.size() : 0;
    }
    if ((rc = upload(d.sn_rec, s.sn_rec, st))) return rc;
    if ((rc = upload(d.sn_cb, s.sn_cb, st))) return rc;
    if ((rc = upload(d.sn_seq, s.sn_seq, st))) return rc;
    if ((rc = upload(d.sn_task, s.sn_task, st))) return rc;
    if ((rc = upload(d.sn_item, s.sn_item, st))) return rc;
    if ((rc = upload(d.sn_moff, s.sn_moff, st))) return rc;
    if ((rc = upload(d.sn_item2, s.sn_item2, st))) return rc;
    if ((rc = upload(d.sn_map, s.sn_map, st))) return rc;
    if ((rc = upload(d.schur_sn_items, s.schur_sn_items, st))) return rc;
    if (!c->an.rscale.empty()) {
        // static scaling A' = S_r P A S_c: per nonzero of A, per solve row and per solve column
        const Analysis &an = c->an;
        std::vector<double> as(an.nnz), gs(an.n), ss(an.n);
        for (int j = 0; j < an.n; j++)
            for (int p = an.Ap[j]; p < an.Ap[j + 1]; p++) as[p] = an.rscale[an.Ai[p]] * an.cscale[j];
        for (int k = 0; k < an.n; k++) {
            gs[k] = an.rscale[s.rowperm_final[k]];
            ss[k] = an.cscale[an.colperm[k]];
        }
        if ((rc = upload(d.ascale, as, st))) return rc;
        if ((rc = upload(d.gscale, gs, st))) return rc;
        if ((rc = upload(d.sscale, ss, st))) return rc;
        HIPCHK(hipStreamSynchronize(st));
    } else {
        dfree(d.ascale);
        dfree(d.gscale);
        dfree(d.sscale);
    }
    if ((rc = upload(d.snl_seq, s.snl_sw, st))) return rc;
    if ((rc = upload(d.snu_seq, s.snu_sw, st))) return rc;
    if ((rc = upload(d.snl_unit, s.snl_unit, st))) return rc;
    if ((rc = upload(d.snl_urange, s.snl_urange, st))) return rc;
    if ((rc = upload(d.snl_runs, s.snl_runs, st))) return rc;
    if ((rc = upload(d.sn_punit, s.sn_punit, st))) return rc;
    if ((rc = upload(d.sn_sunit, s.sn_sunit, st))) return rc;
    if ((rc = upload(d.sn_pu2, s.sn_pu2, st))) return rc;
    if ((rc = upload(d.sn_su2, s.sn_su2, st))) return rc;
    if ((rc = upload(d.sn_grp, s.sn_grp, st))) return rc;
    if ((rc = upload(d.sn_gsrc, s.sn_gsrc, st))) return rc;
    if ((rc = upload(d.sn_gent, s.sn_gent, st))) return rc;
    if ((rc = upload(d.snu_unit, s.snu_unit, st))) return rc;
    if ((rc = upload(d.snu_urange, s.snu_urange, st))) return rc;
    if ((rc = upload(d.snu_runs, s.snu_runs, st))) return rc;
    if ((rc = upload(d.Lrp, s.Lrp, st))) return rc;
    if ((rc = upload(d.Urp, s.Urp, st))) return rc;
    if ((rc = upload(d.lrec, s.lrec, st))) return rc;
    if ((rc = upload(d.urec, s.urec, st))) return rc;
    if ((rc = upload(d.Lrjs, s.Lrjs, st))) return rc;
    if ((rc = upload(d.Urjs, s.Urjs, st))) return rc;
    if ((rc = upload(d.lsptr, s.lsptr, st))) return rc;
    if ((rc = upload(d.usptr, s.usptr, st))) return rc;
    if ((rc = upload(d.rowperm, s.rowperm_final, st))) return rc;
    {
        // the solution scatter takes, per user index, its solve position
        std::vector<int> inv(c->an.colperm.size());
        for (size_t k = 0; k < inv.size(); k++) inv[c->an.colperm[k]] = (int)k;
        if ((rc = upload(d.colperm_sol, inv, st))) return rc;
    }
    if ((rc = upload(d.Acp, s.Acp, st))) return rc;
    if ((rc = upload(d.Acj, s.Acj, st))) return rc;
    if ((rc = upload(d.Acsrc, s.Acsrc, st))) return rc;
    // value buffers sized for the current batch capacity (at least one instance)
    const int batch = std::max(1, d.batch_cap);
    d.batch_cap = 0;
    dfree(d.Fx64);
    dfree(d.Fx32);
    if ((rc = ensure_batch(c, batch))) return rc;
    {
        const std::vector<double> padded = pad_values(c, c->f.Fx.data());
        HIPCHK(hipMemcpyAsync(d.Fx64.p, padded.data(), padded.size() * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    if (c->opt.precision == CKTLU_FP32_IR)
        LCHK(launch_f64_to_f32((const double *)d.Fx64.p, (float *)d.Fx32.p, nnzF(c), st));
    if (!c->host_values.empty()) {
        // values of cktlu_factorize_host: the matrix of these factors, for residuals
        HIPCHK(hipMemcpyAsync(d.Aval.p, c->host_values.data(), c->host_values.size() * sizeof(double),
                              hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        c->host_values.clear();
    }
    d.uploaded = true;
    c->dev_values_newer = false;
    return CKTLU_OK;
}

// Launches of supernodal sweep level l: singletons, small panels, panels, update tasks.
int sn_level_launches(const Schedule &s, int l) {
    return (s.sn_lvl_single[l] > s.sn_lvl[l]) + (s.sn_lvl_small[l] > s.sn_lvl_single[l]) +
           (s.sn_pulvl[l + 1] > s.sn_pulvl[l]) + (s.sn_task_lvl[l + 1] > s.sn_task_lvl[l]);
}


void fill_stats_pattern(cktlu_ctx *c) {
    cktlu_stats &t = c->stats;
    t.n = c->an.n;
    t.nnz_a = c->an.nnz;
    t.nnz_u = c->f.nnz_u();
    t.nnz_l = c->f.nnz_l();
    t.macs = c->s.macs;
    t.flops = c->s.flops;
    t.levels = c->s.nlevels;
    t.max_width = c->s.max_width;
    t.etree_height = c->an.etree_height;
    t.ordering_used = c->an.ordering_used;
    t.fill_amd = c->an.fill_amd;
    t.fill_amf = c->an.fill_amf;
    t.fill_nd = c->an.fill_nd;
    t.fill_ndc = c->an.fill_ndc;
    t.schur_parts = (int64_t)(c->s.schur_parts.size() / 4);
    t.schur_scratch_cols = c->s.schur_nscr;
    t.dense_tail = c->an.n - c->s.tail0;
    const double fb = c->opt.precision == CKTLU_FP32_IR ? 4.0 : 8.0;
    const double nF = (double)(t.nnz_l + t.nnz_u);
    // values + value map of A read once; factor indices read and values written once
    t.bytes_refactor = 12.0 * (double)t.nnz_a + (4.0 + fb) * nF;
    // factor values + indices read once, plus the solution vectors
    t.bytes_solve = (4.0 + fb) * nF + 24.0 * (double)t.n;
    const Schedule &s = c->s;
    t.macs_sweep = s.macs_sweep;
    t.macs_schur = s.macs_schur;
    // traffic models: column sweep 28 B per multiply-add (L value and slot gathered, target read and
    // written) + 24 B per L entry; supernodal sweep 8 B per multiply-add (the panel's L entry) + 20 B
    // per row of R applied to a target (slot, target read and written) + 24 B per L entry (panel)
    t.bytes_sweep = s.sn_count ? 8.0 * s.sn_macs + 20.0 * (double)(s.sn_moff.empty() ? 0 : s.sn_moff.back()) +
                                     24.0 * s.lnz_front
                               : 28.0 * s.macs_sweep + 24.0 * s.lnz_front;
    t.entries_sweep = s.entries_sweep;
    t.entries_dense = s.entries_dense;
    t.macs_dense = s.macs_dense;
    t.alg_bytes_refactor_sweep = (4.0 + fb) * s.entries_sweep;
    const double D = (double)(c->an.n - s.tail0);
    t.flops_dense = 2.0 / 3.0 * D * D * D + D * D / 2.0;
    t.sweep_launches = 0;
    for (int l = 0; l <= s.n_rlevels; l++) {
        const int64_t w = (l < s.n_rlevels ? (s.lvl_ptr[l + 1] - s.lvl_ptr[l]) + (s.task_ptr[l + 1] - s.task_ptr[l]) : 0) +
                          (l > 0 ? s.lvl_ptr[l] - s.lvl_ptr[l - 1] : 0);
        if (w > 0) t.sweep_launches++;
    }
    for (int l = 0; l < s.sn_levels; l++) t.sweep_launches += sn_level_launches(s, l);
    t.sweep_supernodes = s.sn_count;
    t.sweep_levels = s.sn_count ? s.sn_levels : s.n_rlevels;
    const int64_t panels = (int64_t)((D + kDenseBlock - 1) / kDenseBlock);
    t.dense_launches = D > 0 ? 2 * panels - 1 + 2 : 0;        // panels, updates, pivot test, scatter
    t.solve_launches = s.sn_count ? (int64_t)s.snl_levels + s.snu_levels + (D > 0 ? 1 + 2 * panels : 0)
                                  : (int64_t)(s.lseg.size() / 3) + (int64_t)(s.useg.size() / 3) + (D > 0 ? 2 * panels : 0);
}

// Host factorization with pivoting (keep == nullptr: every column), then
// schedule and upload.
int factor_and_setup(cktlu_ctx *c, const double *values_host, const std::vector<char> *keep, bool device,
                     const DenseSource *dsrc = nullptr) {
    std::vector<int> init = c->f.pivrow;
    if ((int)init.size() != c->an.n) {
        init.resize(c->an.n);
        for (int k = 0; k < c->an.n; k++) init[k] = k;
    }
    Factor nf;
    int fail = -1, nswaps = 0;
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<double> scaled;
    if (!c->an.rscale.empty()) {          // the factored matrix is S_r P A S_c
        const Analysis &an = c->an;
        scaled.resize(an.nnz);
        for (int j = 0; j < an.n; j++)
            for (int p = an.Ap[j]; p < an.Ap[j + 1]; p++)
                scaled[p] = values_host[p] * an.rscale[an.Ai[p]] * an.cscale[j];
        values_host = scaled.data();
    }
    int rc = host_gp_factor(c->an, values_host, c->opt.pivot_eps, init, keep ? &c->f : nullptr, keep, nf,
                            fail, nswaps, dsrc);
    if (rc != CKTLU_OK) return rc;
    // same pattern and pivot sequence: the device schedule stays valid, only values change
    const bool same = !c->f.Fi.empty() && nf.Fi == c->f.Fi && nf.Fp == c->f.Fp && nf.pivrow == c->f.pivrow;
    c->f = std::move(nf);
    const auto t1 = std::chrono::steady_clock::now();
    if (!same || c->s.n != c->an.n) build_schedule(c->an, c->f, c->opt, c->s);
    if (debug_on())
        fprintf(stderr, "[cktlu] host factorization %.3f s, schedule %.3f s\n",
                std::chrono::duration<double>(t1 - t0).count(),
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count());
    fill_stats_pattern(c);
    c->state = 2;
    if (device) {
        if (same && c->dev.uploaded) {
            hipStream_t st = stream_of(c);
            const std::vector<double> padded = pad_values(c, c->f.Fx.data());
            HIPCHK(hipMemcpyAsync(c->dev.Fx64.p, padded.data(), padded.size() * sizeof(double),
                                  hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
            if (c->opt.precision == CKTLU_FP32_IR)
                LCHK(launch_f64_to_f32((const double *)c->dev.Fx64.p, (float *)c->dev.Fx32.p, nnzF(c), st));
            c->dev_values_newer = false;
            c->dev.S_prec = -1;
        } else {
            rc = upload_all(c);
            if (rc) return rc;
        }
        HIPCHK(hipStreamSynchronize(stream_of(c)));
    } else {
        c->dev.uploaded = false;
    }
    return CKTLU_OK;
}

int ensure_device(cktlu_ctx *c) {
    if (!c->dev.uploaded) return upload_all(c);
    return CKTLU_OK;
}

// Arguments of the dense trailing-block kernels for `batch` instances.
DenseArgs dense_args(cktlu_ctx *c, int batch, bool fp32) {
    Device &d = c->dev;
    DenseArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = c->an.n;
    a.T = c->s.tail0;
    a.D = c->an.n - c->s.tail0;
    a.batch = batch;
    a.Dp = (const int *)d.Dp.p;
    a.Dlen = (const int *)d.Dlen.p;
    a.Fi = (const int *)d.Fi.p;
    a.Fx = fp32 ? d.Fx32.p : d.Fx64.p;
    a.nnzF = nnzF(c);
    a.S = d.S.p;
    a.Dg = d.Dg.p;
    a.Dinv = (double *)d.Dinv.p;
    a.ctrl = (int *)d.ctrl.p;
    a.done = (int *)d.done.p;
    a.force_fail_col = -1;
    a.fp32 = fp32 ? 1 : 0;
    a.W = c->opt.dense_panel_width ? c->opt.dense_panel_width : 256;
    a.scr = d.schur_scr.p;
    a.nscr = c->s.schur_nscr;
    return a;
}

// The side stream and events of the dense-block look-ahead (created before any capture).
int ensure_lookahead(cktlu_ctx *c, const DenseArgs &da) {
    const int nev = dense_lookahead_events(da);
    if (c->opt.dense_lookahead != 1 || nev == 0) return CKTLU_OK;
    if (!c->side_stream) HIPCHK(hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking));
    while ((int)c->la_events.size() < nev) {
        hipEvent_t e = nullptr;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->la_events.push_back(e);
    }
    return CKTLU_OK;
}

// Make S hold the dense block of the current factors of the given precision.
int ensure_S(cktlu_ctx *c, bool fp32, int batch) {
    if (c->s.tail0 >= c->an.n || c->dev.S_prec == (fp32 ? 1 : 0)) return CKTLU_OK;
    LCHK(launch_dense_gather(dense_args(c, batch, fp32), stream_of(c)));
    LCHK(launch_dense_inverses(dense_args(c, batch, fp32), stream_of(c)));
    c->dev.S_prec = fp32 ? 1 : 0;
    return CKTLU_OK;
}

// S -= L21 U12: by supernodes when the sweep is supernodal, by bridge columns otherwise
// (the schedule builds the parts of the matching kind).  Returns the launch's error code.
int schur_update(cktlu_ctx *c, const DenseArgs &da, hipStream_t st) {
    const Device &d = c->dev;
    const Schedule &s = c->s;
    const int np = (int)(s.schur_parts.size() / 4), na = (int)(s.schur_add.size() / 4);
    if (s.sn_count > 0)
        return launch_schur_sn(da, (const int *)d.schur_parts.p, np, (const int *)d.schur_add.p, na,
                               (const int *)d.schur_sn_items.p, (const int *)d.sn_rec.p, (const int *)d.sn_cb.p, st);
    return launch_schur(da, (const int *)d.schur_parts.p, np, (const int *)d.schur_add.p, na, (const int *)d.l21.p, st);
}

// The level-by-level refactorization of `batch` instances (cluster mode):
// one launch per dependency level of the sparse columns, then the dense block.
int run_refactor(cktlu_ctx *c, int batch, const double *values_dev, bool fp32, bool check, int force_col) {
    Device &d = c->dev;
    hipStream_t st = stream_of(c);
    d.epoch++;
    if (d.epoch == 0 || d.epoch > 0x7ffffff0u) {   // keep completion epochs distinct after wrap
        LCHK(launch_fill_i32((int *)d.done.p, (int64_t)c->an.n * d.batch_cap, 0, st));
        d.epoch = 1;
    }
    LCHK(launch_reset_ctrl((int *)d.ctrl.p, 1 + 2 * batch, INT_MAX, st));
    const Schedule &s = c->s;
    RefactorArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = c->an.n;
    a.batch = batch;
    a.seq = (const int *)d.seq.p;
    a.Dp = (const int *)d.Dp.p;
    a.Dlen = (const int *)d.Dlen.p;
    a.Fi = (const int *)d.Fi.p;
    a.nU = (const int *)d.nU.p;
    a.Ap = (const int *)d.Ap.p;
    a.colperm = (const int *)d.colperm.p;
    a.amap = (const int *)d.amap.p;
    a.Aval = values_dev;
    a.nnzA = c->an.nnz;
    a.nnzF = nnzF(c);
    a.Fx = fp32 ? d.Fx32.p : d.Fx64.p;
    a.done = (int *)d.done.p;
    a.ctrl = (int *)d.ctrl.p;
    a.eps = c->opt.pivot_eps;
    a.epoch = d.epoch;
    a.force_fail_col = force_col;
    a.ascale = (const double *)d.ascale.p;
    a.colrec = (const int *)d.colrec.p;
    a.task8 = (const int *)d.task8.p;
    a.item4 = (const int *)d.item4.p;
    a.smap = d.smap.p ? (const int *)d.smap.p : nullptr;
    a.tmoff = d.smap.p ? (const int64_t *)d.tmoff.p : nullptr;
    a.T = s.tail0;
    a.D = c->an.n - s.tail0;
    a.S = d.S.p;
    a.fp32 = fp32 ? 1 : 0;
    a.check = check ? 1 : 0;
    hipEvent_t t0 = phase_begin(c);
    LCHK(launch_refactor_init(a, st));
    phase_end(c, t0, PH_INIT, 1);
    t0 = phase_begin(c);
    int launches = 0;
    a.sn_rec = (const int *)d.sn_rec.p;
    a.sn_cb = (const int *)d.sn_cb.p;
    a.sn_seq = (const int *)d.sn_seq.p;
    a.sn_task = (const int *)d.sn_task.p;
    a.sn_item = (const int *)d.sn_item.p;
    a.sn_map = (const int *)d.sn_map.p;
    a.sn_moff = (const int64_t *)d.sn_moff.p;
    a.sn_item2 = (const int *)d.sn_item2.p;
    a.sn_punit = (const int *)d.sn_punit.p;
    a.sn_sunit = (const int *)d.sn_sunit.p;
    a.sn_pu2 = (const int *)d.sn_pu2.p;
    a.sn_su2 = (const int *)d.sn_su2.p;
    a.sn_grp = (const int *)d.sn_grp.p;
    a.sn_gsrc = (const int *)d.sn_gsrc.p;
    a.sn_gent = (const int *)d.sn_gent.p;
    a.sn_pmax = (double *)d.sn_part.p;
    a.sn_pcnt = d.sn_cnt.p ? (int *)d.sn_cnt.p + (size_t)2 * s.sn_count * batch : nullptr;
    // supernodal sweep: per level, the supernodes' panels, then the updates they apply
    for (int l = 0; l < s.sn_levels; l++) {
        LCHK(launch_sn_panels(a, l, s.sn_lvl[l], s.sn_lvl_single[l], s.sn_sulvl[l], s.sn_sulvl[l + 1], s.sn_pulvl[l],
                              s.sn_pulvl[l + 1], st));
        LCHK(launch_sn_updates(a, l, s.sn_grp_lvl[l], s.sn_grp_lvl[l + 1], s.sn_task_heavy[l], s.sn_task_tiny[l],
                               s.sn_task_lvl[l + 1], st));
        launches += sn_level_launches(s, l);
    }
    // column sweep: level l checks level l, normalises level l-1, runs the update tasks of
    // level l; then the last level is normalised
    for (int l = 0; l <= s.n_rlevels && s.n_rlevels > 0; l++) {
        const int cb = l < s.n_rlevels ? s.lvl_ptr[l] : 0, ce = l < s.n_rlevels ? s.lvl_ptr[l + 1] : 0;
        const int pb = l > 0 ? s.lvl_ptr[l - 1] : 0, pe = l > 0 ? s.lvl_ptr[l] : 0;
        const int tb = l < s.n_rlevels ? s.task_ptr[l] : 0, te = l < s.n_rlevels ? s.task_ptr[l + 1] : 0;
        LCHK(launch_refactor_level(a, cb, ce, pb, pe, tb, te, l, st));
        launches += (ce - cb) + (pe - pb) + (te - tb) > 0;
    }
    phase_end(c, t0, PH_SWEEP, launches);
    if (c->opt.timing) c->timing_acc.refactors++;
    if (s.tail0 < c->an.n) {
        DenseArgs da = dense_args(c, batch, fp32);
        da.ctrl = a.ctrl;
        da.done = a.done;
        da.eps = a.eps;
        da.epoch = a.epoch;
        da.force_fail_col = force_col;
        da.check = a.check;
        DenseStreams la{nullptr, nullptr, 0};
        int rc = ensure_lookahead(c, da);
        if (rc) return rc;
        if (c->side_stream && !c->la_events.empty()) {
            la.side = c->side_stream;
            la.ev = reinterpret_cast<void *const *>(c->la_events.data());
            la.nev = (int)c->la_events.size();
        }
        t0 = phase_begin(c);
        LCHK(schur_update(c, da, st));
        phase_end(c, t0, PH_SCHUR, c->s.schur_add.empty() ? 1 : 2);
        t0 = phase_begin(c);
        LCHK(launch_dense_refactor(da, false, &la, st));
        phase_end(c, t0, PH_DENSE, (int)c->stats.dense_launches);
        d.S_prec = fp32 ? 1 : 0;
    }
    return CKTLU_OK;
}

// Pivot-check fallback (Sections IV-C, IV-D): restart set from the unfinished
// columns, host re-factorization of that set with pivoting, re-setup.
// Device re-factorization of the dense block with pivoting (instead of the host
// fallback when every column to restart lies in the block): S = A22 - L21 U12 again, the
// pivoted dense LU, then the host takes its pivots and values and computes only the
// new pattern.  Returns 1 when the block had no usable pivot somewhere (the caller
// then takes the host path), CKTLU_OK when done, or an error.
int dense_pivot_refactor(cktlu_ctx *c, const std::vector<double> &vals, cktlu_refactor_info *info) {
    const int n = c->an.n, T = c->s.tail0, D = n - T;
    Device &d = c->dev;
    hipStream_t st = stream_of(c);
    RefactorArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.n = n; ra.batch = 1; ra.T = T; ra.D = D;
    ra.Dp = (const int *)d.Dp.p; ra.Fi = (const int *)d.Fi.p; ra.Ap = (const int *)d.Ap.p;
    ra.colperm = (const int *)d.colperm.p; ra.amap = (const int *)d.amap.p;
    ra.Aval = (const double *)d.Aval.p; ra.S = d.S.p;
    ra.ascale = (const double *)d.ascale.p;
    DenseArgs da = dense_args(c, 1, false);
    da.ctrl = (int *)d.ctrl.p;
    da.done = (int *)d.done.p;
    da.eps = c->opt.pivot_eps;
    DevBuf tmp;
    int rc = dalloc(tmp, (size_t)(D + 1) * sizeof(int));
    if (rc) return rc;
    struct Free { DevBuf &b; ~Free() { dfree(b); } } guard{tmp};
    int *swp = (int *)tmp.p, *dinfo = swp + D;
    const auto t0 = std::chrono::steady_clock::now();
    LCHK(launch_dense_reinit(ra, st));
    LCHK(schur_update(c, da, st));
    LCHK(launch_dense_pivoted_lu(da, swp, dinfo, st));
    std::vector<double> Sh((size_t)D * D);
    std::vector<int> sw(D + 1);
    HIPCHK(hipMemcpyAsync(Sh.data(), d.S.p, Sh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(sw.data(), swp, (size_t)(D + 1) * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    d.S_prec = -1;
    if (sw[D] != 0) {
        if (debug_on()) fprintf(stderr, "[cktlu] dense re-pivot: no usable pivot at block column %d\n", sw[D] - 1);
        return 1;
    }
    std::vector<char> keep(n, 0);
    for (int k = 0; k < T; k++) keep[k] = 1;
    DenseSource ds;
    ds.T = T; ds.D = D; ds.swap = sw.data(); ds.S = Sh.data();
    std::vector<int> oldFi = c->f.Fi;
    const auto t1 = std::chrono::steady_clock::now();
    rc = factor_and_setup(c, vals.data(), &keep, true, &ds);
    if (debug_on())
        fprintf(stderr, "[cktlu] dense re-pivot: device LU and copy %.3f s, pattern and set-up %.3f s\n",
                std::chrono::duration<double>(t1 - t0).count(),
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count());
    if (rc == CKTLU_E_STATE) {                              // the block disagreed with the pattern: host path
        if (debug_on()) fprintf(stderr, "[cktlu] dense re-pivot: pattern disagreement, host fallback\n");
        return 1;
    }
    if (rc != CKTLU_OK) return rc;
    c->stats.n_repivot++;
    c->stats.n_restart_cols += D;
    c->stats.n_device_repivot++;
    if (info) {
        info->repivoted = 1;
        info->restart_size = D;
        info->pattern_changed = oldFi != c->f.Fi;
    }
    return CKTLU_OK;
}

int fallback(cktlu_ctx *c, const double *values_dev, cktlu_refactor_info *info) {
    const int n = c->an.n;
    hipStream_t st = stream_of(c);
    std::vector<int> done(n);
    std::vector<double> vals(c->an.nnz);
    std::vector<double> padded(nnzF(c));
    HIPCHK(hipMemcpyAsync(done.data(), c->dev.done.p, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(padded.data(), c->dev.Fx64.p, padded.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(vals.data(), values_dev, vals.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    unpad_values(c, padded.data(), c->f.Fx.data());
    std::vector<char> unfinished(n), in_set, keep(n);
    for (int k = 0; k < n; k++) unfinished[k] = done[k] != (int)c->dev.epoch;
    restart_closure(c->an.parent, unfinished, in_set);
    c->last_unfinished = unfinished;
    c->last_restart = in_set;
    int rsize = 0, first = n;
    for (int k = 0; k < n; k++) {
        keep[k] = !in_set[k];
        rsize += in_set[k];
        if (in_set[k] && k < first) first = k;
    }
    if (debug_on())
        fprintf(stderr, "[cktlu] fallback: restart set %d columns from %d (dense block from %d)\n", rsize, first,
                c->s.tail0);
    // every column to restart inside the dense block: pivot it on the device
    if (c->s.tail0 < n && first >= c->s.tail0 && c->opt.dense_device_repivot >= 0) {
        int rc = dense_pivot_refactor(c, vals, info);
        if (rc <= 0) return rc;
    }
    std::vector<int> oldFi = c->f.Fi;
    const auto t0 = std::chrono::steady_clock::now();
    int rc = factor_and_setup(c, vals.data(), &keep, true);
    if (debug_on())
        fprintf(stderr, "[cktlu] host fallback: factorization and set-up %.3f s\n",
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    if (rc != CKTLU_OK) return rc;
    c->stats.n_repivot++;
    c->stats.n_restart_cols += rsize;
    if (info) {
        info->repivoted = 1;
        info->restart_size = rsize;
        info->pattern_changed = oldFi != c->f.Fi;
    }
    return CKTLU_OK;
}

int read_status(cktlu_ctx *c, int *h) {
    hipStream_t st = stream_of(c);
    HIPCHK(hipMemcpyAsync(h, c->dev.ctrl.p, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return CKTLU_OK;
}

int refactor_single(cktlu_ctx *c, const double *values_dev, cktlu_refactor_info *info, bool check) {
    if (!c || (!values_dev && c->an.nnz > 0)) return CKTLU_E_ARG;
    if (c->state < 2) return CKTLU_E_STATE;
    if (info) { info->repivoted = 0; info->first_fail_col = -1; info->restart_size = 0; info->pattern_changed = 0; }
    if (c->an.n == 0) return CKTLU_OK;
    int rc = ensure_device(c);
    if (rc) return rc;
    if ((rc = ensure_batch(c, 1))) return rc;
    Device &d = c->dev;
    hipStream_t st = stream_of(c);
    const bool fp32 = c->opt.precision == CKTLU_FP32_IR && !c->fp64_sticky;
    const int force = check ? c->force_fail_pending : -1;
    c->force_fail_pending = -1;
    // keep a copy of the values for residuals of iterative refinement
    LCHK(launch_copy_f64(values_dev, (double *)d.Aval.p, c->an.nnz, st));
    if ((rc = run_refactor(c, 1, values_dev, fp32, check, force))) return rc;
    c->stats.n_refactorize++;
    c->last_batch = 0;
    c->dev_values_newer = true;
    if (!check) return CKTLU_OK;
    int h[3];
    if ((rc = read_status(c, h))) return rc;
    if (!h[1]) return CKTLU_OK;
    int first = h[2];
    if (fp32) {
        // pivot decisions come from FP64: retry the check with FP64 arithmetic.  When it passes,
        // the FP32 values sit too close to the threshold for this circuit: like a stalled
        // refinement, the context keeps FP64 factors until its next full factorization (each
        // later step would otherwise pay both refactorizations)
        if ((rc = run_refactor(c, 1, values_dev, false, true, force))) return rc;
        if ((rc = read_status(c, h))) return rc;
        if (!h[1]) {
            c->stats.n_fp32_check_retries++;
            c->fp64_sticky = true;
            d.S_prec = -1;
            return CKTLU_OK;
        }
        first = h[2];
    }
    if ((rc = fallback(c, values_dev, info))) return rc;
    if (info) info->first_fail_col = first;
    return CKTLU_W_REPIVOTED;
}

int ensure_vec(cktlu_ctx *c, size_t doubles) {
    if (c->dev.vec_cap >= doubles) return CKTLU_OK;
    c->buffers_gen++;
    int rc = dalloc(c->dev.vec, doubles * sizeof(double));
    if (rc) return rc;
    c->dev.vec_cap = doubles;
    return CKTLU_OK;
}

// z (n rows of solve_slots(nrhs) doubles per instance) <- (LU)^{-1} z, in place; level by level.
int tri_solves(cktlu_ctx *c, int nrhs, int batch, double *z, bool fp32, const int *skip) {
    Device &d = c->dev;
    hipStream_t st = stream_of(c);
    nrhs = solve_slots(nrhs);     // the rows carry the padded slot count (zeros past the user's nrhs)
    SolveArgs a;
    a.n = c->an.n;
    a.nrhs = nrhs;
    a.batch = batch;
    a.lrec = (const int *)d.lrec.p;
    a.urec = (const int *)d.urec.p;
    a.Lrjs = (const int *)d.Lrjs.p;
    a.Urjs = (const int *)d.Urjs.p;
    a.Fx = fp32 ? d.Fx32.p : d.Fx64.p;
    a.nnzF = nnzF(c);
    a.fp32 = fp32 ? 1 : 0;
    a.y = z;
    a.skip = skip;
    a.sn_rec = (const int *)d.sn_rec.p;
    a.sn_cb = (const int *)d.sn_cb.p;
    a.Lrp = (const int *)d.Lrp.p;
    a.Urp = (const int *)d.Urp.p;
    a.sn_part = (double *)d.sn_part.p;
    const Schedule &s = c->s;
    const bool snodal = s.sn_count > 0;
    // sparse L levels (the last one holds the dense rows: their entries in sparse columns); with
    // supernodes, the rows < T by supernode levels and then only that last level
    hipEvent_t t0 = phase_begin(c);
    int launches = 0;
    for (int l = 0; snodal && l < s.snl_levels; l++, launches++)
        LCHK(launch_sn_lsolve(a, (const int *)d.snl_seq.p, (const int *)d.snl_unit.p, (const int *)d.snl_urange.p,
                              (const int *)d.snl_runs.p, s.snl_first[l], s.snl_tiny[l],
                              s.snl_single[l],
                              s.snl_ulvl[l], s.snl_ulvl[l + 1], (int *)d.sn_cnt.p, st));
    const int ldense = s.tail0 < c->an.n ? (int)s.lsptr.size() - 2 : -1;   // level of the dense rows
    for (size_t g = 0; g < s.lseg.size(); g += 3) {
        const int l0 = s.lseg[g], l1 = s.lseg[g + 1];
        if (snodal && !(l0 <= ldense && ldense < l1)) continue;
        const int a0 = snodal ? ldense : l0, a1 = snodal ? ldense + 1 : l1;
        if (s.lseg[g + 2] == 1 && !snodal) LCHK(launch_lsolve_chain(a, (const int *)d.lsptr.p, l0, l1, st));
        else if (s.lseg[g + 2] == 2) LCHK(launch_lsolve_level_wg(a, s.lsptr[a0], s.lsptr[a1], st));
        else LCHK(launch_lsolve_level(a, s.lsptr[a0], s.lsptr[a1], st));
        launches++;
    }
    phase_end(c, t0, PH_SOLVE_SPARSE, launches);
    if (s.tail0 < c->an.n) {
        int rc = ensure_S(c, fp32, batch);
        if (rc) return rc;
        const DenseArgs da = dense_args(c, batch, fp32);
        const int nblk = (da.D + kDenseBlock - 1) / kDenseBlock;
        t0 = phase_begin(c);
        LCHK(launch_dense_solve(da, z, nrhs, skip, false, st));
        LCHK(launch_dense_solve(da, z, nrhs, skip, true, st));
        phase_end(c, t0, PH_SOLVE_DENSE, 2 * nblk);
    }
    t0 = phase_begin(c);
    launches = 0;
    for (int l = 0; snodal && l < s.snu_levels; l++, launches++)
        LCHK(launch_sn_usolve(a, (const int *)d.snu_seq.p, (const int *)d.snu_unit.p, (const int *)d.snu_urange.p,
                              (const int *)d.snu_runs.p, s.snu_first[l], s.snu_tiny[l],
                              s.snu_single[l],
                              s.snu_ulvl[l], s.snu_ulvl[l + 1],
                              d.sn_cnt.p ? (int *)d.sn_cnt.p + (size_t)s.sn_count * batch : nullptr, st));
    for (size_t g = 0; !snodal && g < s.useg.size(); g += 3, launches++) {
        const int l0 = s.useg[g], l1 = s.useg[g + 1];
        if (s.useg[g + 2] == 1) LCHK(launch_usolve_chain(a, (const int *)d.usptr.p, l0, l1, st));
        else if (s.useg[g + 2] == 2) LCHK(launch_usolve_level_wg(a, s.usptr[l0], s.usptr[l1], st));
        else LCHK(launch_usolve_level(a, s.usptr[l0], s.usptr[l1], st));
    }
    phase_end(c, t0, PH_SOLVE_SPARSE, launches);
    if (c->opt.timing) c->timing_acc.solve_passes++;
    return CKTLU_OK;
}

// Device work vectors: z = room for n rows of YS doubles, then r = n x nrhs doubles, then
// 3 x nrhs norms and one more word.
size_t vec_need(const cktlu_ctx *c, int nrhs) {
    return (size_t)c->an.n * YS + 64 + (size_t)c->an.n * nrhs + 3 * (size_t)nrhs + 8;
}

// zbuf: work rows (room for n x YS doubles) supplied by the caller, or nullptr for the context's own
// skip: a device status word (-1 = solve), or null
int solve_chunk(cktlu_ctx *c, int nrhs, const double *b, int64_t ldb, double *x, int64_t ldx, bool fp32,
                bool accumulate, double *zbuf = nullptr, const int *skip = nullptr) {
    const int n = c->an.n;
    int rc;
    double *z = zbuf;
    if (!z) {
        if ((rc = ensure_vec(c, vec_need(c, nrhs)))) return rc;
        z = (double *)c->dev.vec.p;
    }
    hipStream_t st = stream_of(c);
    LCHK(launch_gather_rhs(n, nrhs, 1, b, ldb, (const int *)c->dev.rowperm.p, z, st, (const double *)c->dev.gscale.p));
    if ((rc = tri_solves(c, nrhs, 1, z, fp32, skip))) return rc;
    LCHK(launch_scatter_sol(n, nrhs, 1, z, (const int *)c->dev.colperm_sol.p, x, ldx, accumulate ? 1 : 0,
                            skip, st, (const double *)c->dev.sscale.p));
    return CKTLU_OK;
}

int solve_plain(cktlu_ctx *c, int nrhs, const double *b, int64_t ldb, double *x, int64_t ldx, bool fp32,
                bool accumulate, double *zbuf = nullptr, const int *skip = nullptr) {
    for (int r0 = 0; r0 < nrhs;) {
        int chunk = nrhs - r0 >= 8 ? 8 : nrhs - r0 >= 4 ? 4 : nrhs - r0 >= 2 ? 2 : 1;
        int rc = solve_chunk(c, chunk, b + r0 * ldb, ldb, x + r0 * ldx, ldx, fp32, accumulate, zbuf, skip);
        if (rc) return rc;
        r0 += chunk;
    }
    return CKTLU_OK;
}

// Iterative refinement with FP32 factors: x = 0, r = b; repeat d = (LU)^{-1} r
// (FP32 factors, FP64 accumulation), x += d, r = b - A x (FP64) until the
// backward error of every right-hand side is at most ir_tol.  The first two steps are
// queued together and decide convergence on the device (a converged step leaves the status
// word, and the second step's kernels then return at once); the host reads the outcome once
// after them and takes any further step, with the stall test, one at a time.
int solve_ir(cktlu_ctx *c, int nrhs, const double *b, int64_t ldb, double *x, int64_t ldx,
             cktlu_solve_info *info, bool *converged) {
    const int n = c->an.n;
    hipStream_t st = stream_of(c);
    int rc = ensure_vec(c, vec_need(c, nrhs));
    if (rc) return rc;
    double *vec = (double *)c->dev.vec.p;
    double *r = vec + (size_t)n * YS + 64;
    double *norms = r + (size_t)n * nrhs;
    double *anorm = vec + vec_need(c, nrhs) - 1;      // written by cktlu_solve
    double *eta_d = anorm - 1;
    int *skip = (int *)(anorm - 2);
    for (int q = 0; q < nrhs; q++) LCHK(launch_fill_f64(x + q * ldx, n, 0.0, st));
    LCHK(launch_fill_i32(skip, 1, -1, st));
    LCHK(launch_fill_f64(eta_d, 1, INFINITY, st));
    const int *Acp = (const int *)c->dev.Acp.p, *Acj = (const int *)c->dev.Acj.p;
    const int *Acsrc = (const int *)c->dev.Acsrc.p;
    const double *Aval = (const double *)c->dev.Aval.p;
    auto step = [&](int it) -> int {
        int e = solve_plain(c, nrhs, it == 1 ? b : r, it == 1 ? ldb : n, x, ldx, true, true, nullptr, skip);
        if (e) return e;
        LCHK(launch_fill_f64(norms, 3 * (int64_t)nrhs, 0.0, st));
        LCHK(launch_residual(n, nrhs, Acp, Acj, Acsrc, Aval, x, ldx, b, ldb, r, n, norms, st, skip));
        LCHK(launch_ir_check(1, nrhs, norms, anorm, c->opt.ir_tol, skip, eta_d, st));
        return CKTLU_OK;
    };
    const int queued = std::min(2, c->opt.ir_max_iter);
    int it = 0, hskip = -1;
    double eta = INFINITY, prev_eta = INFINITY;
    auto outcome = [&]() -> int {
        HIPCHK(hipMemcpyAsync(&eta, eta_d, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(&hskip, skip, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return CKTLU_OK;
    };
    *converged = false;
    for (it = 1; it <= queued; it++)
        if ((rc = step(it))) return rc;
    if ((rc = outcome())) return rc;
    it = queued;
    while (hskip == -1 && it < c->opt.ir_max_iter) {
        if (it >= 3 && eta > 0.5 * prev_eta) break;     // stalled
        prev_eta = eta;
        if ((rc = step(++it))) return rc;
        if ((rc = outcome())) return rc;
    }
    *converged = hskip != -1;
    if (info) {
        info->backward_err = eta;
        info->ir_iters = it;
    }
    return CKTLU_OK;
}

}  // namespace

extern "C" {

void cktlu_default_options(cktlu_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->pivot_eps = 1e-3;
    o->precision = CKTLU_FP64;
    o->ir_tol = 1e-10;
    o->ir_max_iter = 10;
    o->ordering = CKTLU_ORDER_AUTO;
    o->transversal = 1;
    o->stream = nullptr;
    o->force_fail_col = -1;
    o->dense_tail_size = 0;
    o->dense_tail_density = 0.3;
}

int cktlu_create(cktlu_ctx **out, const cktlu_options *opt) {
    if (!out) return CKTLU_E_ARG;
    *out = nullptr;
    cktlu_ctx *c = new (std::nothrow) cktlu_ctx();
    if (!c) return CKTLU_E_NOMEM;
    if (opt) c->opt = *opt; else cktlu_default_options(&c->opt);
    if (!(c->opt.pivot_eps > 0.0 && c->opt.pivot_eps <= 1.0) ||
        (c->opt.precision != CKTLU_FP64 && c->opt.precision != CKTLU_FP32_IR) || c->opt.ir_max_iter < 1 ||
        c->opt.solve_chain_width < -1 || (c->opt.dense_lookahead != 0 && c->opt.dense_lookahead != 1) ||
        c->opt.ordering < CKTLU_ORDER_AMD || c->opt.ordering > CKTLU_ORDER_ND_CAMD ||
        (c->opt.dense_device_repivot != 0 && c->opt.dense_device_repivot != -1) ||
        (c->opt.sweep_slot_map != 0 && c->opt.sweep_slot_map != -1) ||
        c->opt.sweep_supernodes < -1 || c->opt.sweep_supernodes > 64 ||
        c->opt.static_pivoting < 0 || c->opt.static_pivoting > 2 ||
        (c->opt.sweep_panel_rows != 0 && (c->opt.sweep_panel_rows < 16 || c->opt.sweep_panel_rows > 65536)) ||
        (c->opt.solve_split_entries != 0 && (c->opt.solve_split_entries < 64 || c->opt.solve_split_entries > (1 << 30))) ||
        (c->opt.dense_panel_width != 0 && c->opt.dense_panel_width != 64 && c->opt.dense_panel_width != 128 &&
         c->opt.dense_panel_width != 256)) {
        delete c;
        return CKTLU_E_ARG;
    }
    std::memset(&c->stats, 0, sizeof(c->stats));
    std::memset(&c->timing_acc, 0, sizeof(c->timing_acc));
    c->force_fail_pending = c->opt.force_fail_col;
    *out = c;
    return CKTLU_OK;
}

void cktlu_destroy(cktlu_ctx *c) {
    if (!c) return;
    if (!c->pending.empty()) (void)hipStreamSynchronize(stream_of(c));
    for (auto &p : c->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->side_stream) {
        (void)hipStreamSynchronize(c->side_stream);
        (void)hipStreamDestroy(c->side_stream);
    }
    for (hipEvent_t e : c->la_events) (void)hipEventDestroy(e);
    free_device(c->dev);
    delete c;
}

const char *cktlu_strerror(int s) {
    switch (s) {
        case CKTLU_OK: return "ok";
        case CKTLU_W_REPIVOTED: return "warning: pivot check failed, re-pivoted";
        case CKTLU_W_IR_FALLBACK: return "warning: refinement fell back to FP64";
        case CKTLU_E_ARG: return "invalid argument";
        case CKTLU_E_STATE: return "call out of order";
        case CKTLU_E_STRUCT_SINGULAR: return "structurally singular matrix";
        case CKTLU_E_NUM_SINGULAR: return "numerically singular matrix";
        case CKTLU_E_NOMEM: return "out of memory";
        case CKTLU_E_HIP: return "HIP runtime error";
        case CKTLU_E_LIMIT: return "size limit exceeded";
        default: return "unknown status";
    }
}

int cktlu_set_stream(cktlu_ctx *c, void *stream) {
    if (!c) return CKTLU_E_ARG;
    c->opt.stream = stream;
    return CKTLU_OK;
}

int cktlu_analyze_values(cktlu_ctx *c, int32_t n, const int32_t *colptr, const int32_t *rowind,
                         const double *values) {
    if (!c || (n > 0 && !values && c->opt.static_pivoting > 0)) return CKTLU_E_ARG;
    if (n > (1 << 28)) return CKTLU_E_LIMIT;
    free_device(c->dev);
    c->f = Factor();
    c->s = Schedule();
    c->last_unfinished.clear();
    c->last_restart.clear();
    c->host_values.clear();
    int rc = run_analysis(c->an, n, colptr, rowind, c->opt.ordering, c->opt.transversal, values,
                          c->opt.static_pivoting);
    if (rc != CKTLU_OK) { c->state = 0; return rc; }
    c->state = 1;
    return CKTLU_OK;
}

int cktlu_get_scaling(const cktlu_ctx *c, double *rscale, double *cscale) {
    if (!c) return CKTLU_E_ARG;
    if (c->state < 1) return CKTLU_E_STATE;
    const bool sc = !c->an.rscale.empty();
    for (int i = 0; i < c->an.n; i++) {
        if (rscale) rscale[i] = sc ? c->an.rscale[i] : 1.0;
        if (cscale) cscale[i] = sc ? c->an.cscale[i] : 1.0;
    }
    return CKTLU_OK;
}

int cktlu_analyze(cktlu_ctx *c, int32_t n, const int32_t *colptr, const int32_t *rowind) {
    if (!c) return CKTLU_E_ARG;
    if (n > (1 << 28)) return CKTLU_E_LIMIT;
    free_device(c->dev);
    c->f = Factor();
    c->s = Schedule();
    c->last_unfinished.clear();
    c->last_restart.clear();
    c->host_values.clear();
    int rc = run_analysis(c->an, n, colptr, rowind, c->opt.ordering, c->opt.transversal);
    if (rc != CKTLU_OK) { c->state = 0; return rc; }
    c->state = 1;
    return CKTLU_OK;
}

int cktlu_factorize_host(cktlu_ctx *c, const double *values_host) {
    if (!c || (!values_host && c->an.nnz > 0)) return CKTLU_E_ARG;
    if (c->state < 1) return CKTLU_E_STATE;
    c->f.pivrow.clear();
    c->fp64_sticky = false;
    int rc = factor_and_setup(c, values_host, nullptr, false);
    if (rc == CKTLU_OK) {
        c->stats.n_factorize++;
        c->host_values.assign(values_host, values_host + c->an.nnz);
    }
    return rc;
}

int cktlu_factorize(cktlu_ctx *c, const double *values_dev) {
    if (!c || (!values_dev && c->an.nnz > 0)) return CKTLU_E_ARG;
    if (c->state < 1) return CKTLU_E_STATE;
    std::vector<double> v(c->an.nnz);
    hipStream_t st = stream_of(c);
    if (!v.empty()) {
        HIPCHK(hipMemcpyAsync(v.data(), values_dev, v.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    c->f.pivrow.clear();
    c->fp64_sticky = false;
    c->host_values.clear();
    int rc = factor_and_setup(c, v.data(), nullptr, true);
    if (rc != CKTLU_OK) return rc;
    c->stats.n_factorize++;
    if (c->an.nnz > 0) {
        if ((rc = ensure_batch(c, 1))) return rc;
        LCHK(launch_copy_f64(values_dev, (double *)c->dev.Aval.p, c->an.nnz, st));
    }
    return CKTLU_OK;
}

int cktlu_refactorize(cktlu_ctx *c, const double *values_dev, cktlu_refactor_info *info) {
    return refactor_single(c, values_dev, info, true);
}

int cktlu_refactorize_nocheck(cktlu_ctx *c, const double *values_dev) {
    return refactor_single(c, values_dev, nullptr, false);
}

int cktlu_solve(cktlu_ctx *c, int32_t nrhs, const double *b, int32_t ldb, double *x, int32_t ldx,
                cktlu_solve_info *info) {
    if (!c || nrhs < 0 || (nrhs > 0 && (!b || !x))) return CKTLU_E_ARG;
    if (c->state < 2) return CKTLU_E_STATE;
    if (ldb < c->an.n || ldx < c->an.n) return CKTLU_E_ARG;
    if (info) { info->ir_iters = 0; info->backward_err = -1.0; info->used_fp64 = 0; }
    if (nrhs == 0 || c->an.n == 0) return CKTLU_OK;
    int rc = ensure_device(c);
    if (rc) return rc;
    if (c->opt.precision == CKTLU_FP64) return solve_plain(c, nrhs, b, ldb, x, ldx, false, false);
    if (c->fp64_sticky) {                  // refinement failed on this circuit before: FP64 factors
        if (info) info->used_fp64 = 1;
        return solve_plain(c, nrhs, b, ldb, x, ldx, false, false);
    }
    // FP32 factors + FP64 refinement
    hipStream_t st = stream_of(c);
    if ((rc = ensure_vec(c, vec_need(c, nrhs)))) return rc;
    {
        double *an = (double *)c->dev.vec.p + vec_need(c, nrhs) - 1;   // |A|_inf, read by solve_ir on the device
        LCHK(launch_fill_f64(an, 1, 0.0, st));
        LCHK(launch_anorm(c->an.n, (const int *)c->dev.Acp.p, (const int *)c->dev.Acsrc.p,
                          (const double *)c->dev.Aval.p, an, st));
    }
    bool conv = false;
    if ((rc = solve_ir(c, nrhs, b, ldb, x, ldx, info, &conv))) return rc;
    if (conv) return CKTLU_OK;
    // refinement stalled: FP64 refactorization of the same values and an FP64 solve
    if ((rc = run_refactor(c, 1, (const double *)c->dev.Aval.p, false, false, -1))) return rc;
    if ((rc = solve_plain(c, nrhs, b, ldb, x, ldx, false, false))) return rc;
    c->stats.n_fp64_fallback_solves++;
    c->fp64_sticky = true;
    if (info) info->used_fp64 = 1;
    return CKTLU_W_IR_FALLBACK;
}

int cktlu_solve_noalloc(cktlu_ctx *c, int32_t nrhs, const double *b, int32_t ldb, double *x, int32_t ldx) {
    if (!c || nrhs < 0 || (nrhs > 0 && (!b || !x))) return CKTLU_E_ARG;
    if (c->state < 2 || !c->dev.uploaded) return CKTLU_E_STATE;      // nothing may be uploaded here
    if (c->opt.precision != CKTLU_FP64 && !c->fp64_sticky) return CKTLU_E_STATE;
    if (ldb < c->an.n || ldx < c->an.n) return CKTLU_E_ARG;
    if (c->an.n > kNoAllocRows) return CKTLU_E_LIMIT;
    if (nrhs == 0 || c->an.n == 0) return CKTLU_OK;
    double *z = nullptr;
    LCHK(noalloc_scratch(&z));
    const int saved_timing = c->opt.timing;        // phase timing would create events
    c->opt.timing = 0;
    const int rc = solve_plain(c, nrhs, b, ldb, x, ldx, false, false, z);
    c->opt.timing = saved_timing;
    return rc;
}

int cktlu_step_batched_graph(cktlu_ctx *c, int32_t batch, const double *values_dev, int32_t *status_dev,
                             int32_t nrhs, const double *b, double *x, double *eta_dev, int32_t ir_steps) {
    if (!c || batch < 1 || !values_dev || !status_dev || nrhs < 1 || nrhs > 8 || !b || !x) return CKTLU_E_ARG;
    const bool fp32 = c->opt.precision == CKTLU_FP32_IR;
    if (fp32 && ir_steps < 1) return CKTLU_E_ARG;
    if (c->state < 2) return CKTLU_E_STATE;
    if ((int64_t)batch * c->an.n >= INT_MAX) return CKTLU_E_LIMIT;
    int rc = ensure_device(c);
    if (rc) return rc;
    if ((rc = ensure_batch(c, batch))) return rc;
    const int n = c->an.n;
    const int64_t nnzA = c->an.nnz;
    const size_t nv = (size_t)n * nrhs * batch;
    const size_t zd = (size_t)n * YS * batch + 64;
    if ((rc = ensure_vec(c, zd + nv + 3 * (size_t)nrhs * batch + 3 * (size_t)batch + 64))) return rc;
    // the dense block must hold factors of the precision the solve reads (set by the refactorization)
    cktlu_ctx::GraphKey key;
    key.batch = batch; key.nrhs = nrhs; key.ir_steps = fp32 ? ir_steps : 0;
    key.values = values_dev; key.b = b; key.status = status_dev; key.x = x; key.eta = eta_dev;
    key.gen = c->buffers_gen;
    hipStream_t user = stream_of(c);
    if (!c->graph_exec || !(key == c->graph_key)) {
        if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
        if (!c->capture_stream) HIPCHK(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
        if (c->s.tail0 < c->an.n && (rc = ensure_lookahead(c, dense_args(c, batch, fp32)))) return rc;
        // everything below is enqueued on the capture stream and recorded, not run
        HIPCHK(hipStreamSynchronize(user));
        void *saved_stream = c->opt.stream;
        const int saved_timing = c->opt.timing;
        c->opt.stream = c->capture_stream;
        c->opt.timing = 0;
        hipStream_t st = c->capture_stream;
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        auto body = [&]() -> int {
            double *z = (double *)c->dev.vec.p;
            double *r = z + zd;
            double *norms = r + nv;
            double *anorm = norms + 3 * (size_t)nrhs * batch;
            double *eta = anorm + batch;
            int *skip = (int *)(eta + batch);
            const int *rowperm = (const int *)c->dev.rowperm.p, *colperm = (const int *)c->dev.colperm_sol.p;
            LCHK(launch_copy_f64(values_dev, (double *)c->dev.Aval.p, nnzA * (int64_t)batch, st));
            int e = run_refactor(c, batch, values_dev, fp32, true, -1);
            if (e) return e;
            LCHK(launch_status_out((const int *)c->dev.ctrl.p + 1 + batch, status_dev, batch, st));
            if (!fp32) {
                LCHK(launch_gather_rhs(n, nrhs, batch, b, n, rowperm, z, st, (const double *)c->dev.gscale.p));
                if ((e = tri_solves(c, nrhs, batch, z, false, status_dev))) return e;
                LCHK(launch_scatter_sol(n, nrhs, batch, z, colperm, x, n, 0, status_dev, st, (const double *)c->dev.sscale.p));
                if (eta_dev) LCHK(launch_fill_f64(eta_dev, batch, -1.0, st));
                return CKTLU_OK;
            }
            // FP32 factors, ir_steps FP64 refinement steps decided on the device
            const int *Acp = (const int *)c->dev.Acp.p, *Acj = (const int *)c->dev.Acj.p;
            const int *Acsrc = (const int *)c->dev.Acsrc.p;
            const double *Aval = (const double *)c->dev.Aval.p;
            LCHK(launch_fill_f64(anorm, batch, 0.0, st));
            LCHK(launch_fill_f64(eta, batch, -1.0, st));
            LCHK(launch_anorm_batched(n, batch, nnzA, Acp, Acsrc, Aval, anorm, st));
            LCHK(launch_copy_i32(status_dev, skip, batch, st));
            for (int it = 1; it <= ir_steps; it++) {
                LCHK(launch_gather_rhs(n, nrhs, batch, it == 1 ? b : r, n, rowperm, z, st, (const double *)c->dev.gscale.p));
                if ((e = tri_solves(c, nrhs, batch, z, true, skip))) return e;
                // x = d on the first step (x of skipped instances is never written), then x += d
                LCHK(launch_scatter_sol(n, nrhs, batch, z, colperm, x, n, it > 1 ? 1 : 0, skip, st, (const double *)c->dev.sscale.p));
                LCHK(launch_fill_f64(norms, 3 * (int64_t)nrhs * batch, 0.0, st));
                LCHK(launch_residual_batched(n, nrhs, batch, nnzA, Acp, Acj, Acsrc, Aval, x, b, r, norms, skip, st));
                LCHK(launch_ir_check(batch, nrhs, norms, anorm, c->opt.ir_tol, skip, eta, st));
            }
            if (eta_dev) LCHK(launch_copy_f64(eta, eta_dev, batch, st));
            return CKTLU_OK;
        };
        const int brc = body();
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &graph);
        c->opt.stream = saved_stream;
        c->opt.timing = saved_timing;
        if (brc) { if (graph) (void)hipGraphDestroy(graph); return brc; }
        if (ec != hipSuccess || !graph) { debug_hip((int)ec, "hipStreamEndCapture", __LINE__); return CKTLU_E_HIP; }
        const hipError_t ei = hipGraphInstantiate(&c->graph_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) { c->graph_exec = nullptr; debug_hip((int)ei, "hipGraphInstantiate", __LINE__); return CKTLU_E_HIP; }
        c->graph_key = key;
    }
    HIPCHK(hipGraphLaunch(c->graph_exec, user));
    c->last_batch = batch;
    c->stats.n_refactorize += batch;
    c->dev_values_newer = true;
    return CKTLU_OK;
}

int cktlu_autotune(cktlu_ctx *c, int32_t batch, const double *values_dev, int32_t reps, cktlu_tune_result *out) {
    if (!c || !out || batch < 1 || reps < 1 || !values_dev) return CKTLU_E_ARG;
    if (c->state < 2) return CKTLU_E_STATE;
    std::memset(out, 0, sizeof(*out));
    const int n = c->an.n;
    struct Cand { int size; double density; };
    std::vector<Cand> cands = {{-1, 0.3}, {0, 0.5}, {0, 0.3}, {0, 0.2}};
    for (int d = 512; d <= 8192 && d <= n; d *= 2) cands.push_back({d, 0.3});
    // larger blocks (fewer, longer levels traded for dense work) while they fit a quarter of free HBM
    size_t hbm_free = 0, hbm_total = 0;
    if (hipMemGetInfo(&hbm_free, &hbm_total) != hipSuccess) hbm_free = 0;
    for (int d : {10240, 12288, 16384})
        if (d <= n && (double)d * d * 8.0 * batch <= 0.25 * (double)hbm_free) cands.push_back({d, 0.3});
    const cktlu_options saved = c->opt;
    c->opt.timing = 0;
    hipStream_t st = stream_of(c);
    // work buffers: one right-hand side of ones per instance, solutions, status
    DevBuf rhs, sol, status;
    auto release = [&]() { dfree(rhs); dfree(sol); dfree(status); };
    if (dalloc(rhs, (size_t)n * batch * sizeof(double)) || dalloc(sol, (size_t)n * batch * sizeof(double)) ||
        dalloc(status, (size_t)batch * sizeof(int))) {
        release();
        return CKTLU_E_NOMEM;
    }
    if (launch_fill_f64((double *)rhs.p, (int64_t)n * batch, 1.0, st)) { release(); return CKTLU_E_HIP; }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        release();
        return CKTLU_E_HIP;
    }
    auto step = [&]() -> int {
        int rc;
        if (batch == 1) {
            rc = refactor_single(c, values_dev, nullptr, true);
            if (rc < 0) return rc;
            rc = cktlu_solve(c, 1, (const double *)rhs.p, n, (double *)sol.p, n, nullptr);
            return rc < 0 ? rc : CKTLU_OK;
        }
        if ((rc = cktlu_refactorize_batched(c, batch, values_dev, (int *)status.p))) return rc;
        rc = cktlu_solve_batched(c, batch, 1, (const double *)rhs.p, (double *)sol.p, (const int *)status.p, nullptr);
        return rc < 0 ? rc : CKTLU_OK;
    };
    int rc = CKTLU_OK;
    std::vector<int> seen;
    double best_ms = INFINITY;
    int best_size = saved.dense_tail_size;
    double best_density = saved.dense_tail_density;
    for (const Cand &cd : cands) {
        if (out->n_tried >= 16) break;
        c->opt.dense_tail_size = cd.size;
        c->opt.dense_tail_density = cd.density;
        Schedule trial;
        // trials build a slot map of at most 2^30 entries (a few seconds); the kept schedule
        // gets the full one
        size_t fr = 0, tot = 0;
        const int64_t cap = hipMemGetInfo(&fr, &tot) == hipSuccess ? (int64_t)(0.25 * (double)fr / sizeof(int)) : 0;
        build_schedule(c->an, c->f, c->opt, trial, std::min<int64_t>(cap, (int64_t)1 << 30));
        const int D = n - trial.tail0;
        if (std::find(seen.begin(), seen.end(), D) != seen.end()) continue;
        seen.push_back(D);
        c->s = std::move(trial);
        fill_stats_pattern(c);
        if ((rc = upload_all(c))) break;
        if ((rc = step())) break;                          // warm-up
        HIPCHK(hipEventRecord(e0, st));
        for (int r = 0; r < reps && !rc; r++) rc = step();
        if (rc) break;
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        const int k = out->n_tried++;
        out->dense_tail[k] = D;
        out->ms_per_step[k] = ms / reps;
        if (ms / reps < best_ms) {
            best_ms = ms / reps;
            out->best = k;
            best_size = D > 0 ? D : -1;
            best_density = cd.density;
        }
    }
    // second stage: with the best D, each knob left at 0 by the caller, one value at a time
    cktlu_options tuned = saved;
    tuned.dense_tail_size = best_size;
    tuned.dense_tail_density = best_density;
    struct Knob { int id; int cktlu_options::*field; std::vector<int> values; };
    const std::vector<Knob> knobs = {
        {CKTLU_KNOB_SUPERNODE_WIDTH, &cktlu_options::sweep_supernodes, {32}},
        {CKTLU_KNOB_PANEL_ROWS, &cktlu_options::sweep_panel_rows, {128, 512}},
        {CKTLU_KNOB_SOLVE_SPLIT, &cktlu_options::solve_split_entries, {4096, 16384}},
        {CKTLU_KNOB_DENSE_PANEL, &cktlu_options::dense_panel_width, {128}},
    };
    for (const Knob &kb : knobs) {
        if (rc || saved.*kb.field != 0) continue;
        if (kb.id == CKTLU_KNOB_DENSE_PANEL && best_size <= 0) continue;
        for (int v : kb.values) {
            if (out->n_knob_tried >= 16) break;
            c->opt = tuned;
            c->opt.timing = 0;
            c->opt.*kb.field = v;
            Schedule trial;
            size_t fr = 0, tot = 0;
            const int64_t cap = hipMemGetInfo(&fr, &tot) == hipSuccess ? (int64_t)(0.25 * (double)fr / sizeof(int)) : 0;
            build_schedule(c->an, c->f, c->opt, trial, std::min<int64_t>(cap, (int64_t)1 << 30));
            c->s = std::move(trial);
            fill_stats_pattern(c);
            if ((rc = upload_all(c))) break;
            if ((rc = step())) break;
            if (hipEventRecord(e0, st) != hipSuccess) { rc = CKTLU_E_HIP; break; }
            for (int r = 0; r < reps && !rc; r++) rc = step();
            if (rc) break;
            float ms = 0.f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = CKTLU_E_HIP; break; }
            const int k = out->n_knob_tried++;
            out->knob[k] = kb.id;
            out->knob_value[k] = v;
            out->knob_ms_per_step[k] = ms / reps;
            if (ms / reps < 0.98 * best_ms) {
                best_ms = ms / reps;
                tuned.*kb.field = v;
            }
        }
    }
    out->sweep_supernodes = tuned.sweep_supernodes;
    out->sweep_panel_rows = tuned.sweep_panel_rows;
    out->solve_split_entries = tuned.solve_split_entries;
    out->dense_panel_width = tuned.dense_panel_width;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    release();
    c->opt = saved;
    if (rc) return rc;
    // keep the fastest schedule
    c->opt.dense_tail_size = tuned.dense_tail_size;
    c->opt.dense_tail_density = tuned.dense_tail_density;
    c->opt.sweep_supernodes = tuned.sweep_supernodes;
    c->opt.sweep_panel_rows = tuned.sweep_panel_rows;
    c->opt.solve_split_entries = tuned.solve_split_entries;
    c->opt.dense_panel_width = tuned.dense_panel_width;
    build_schedule(c->an, c->f, c->opt, c->s);
    fill_stats_pattern(c);
    return upload_all(c);
}

int cktlu_refactorize_batched(cktlu_ctx *c, int32_t batch, const double *values_dev, int32_t *status_dev) {
    if (!c || batch < 1 || !values_dev || !status_dev) return CKTLU_E_ARG;
    if (c->state < 2) return CKTLU_E_STATE;
    if ((int64_t)batch * c->an.n >= INT_MAX) return CKTLU_E_LIMIT;
    int rc = ensure_device(c);
    if (rc) return rc;
    if ((rc = ensure_batch(c, batch))) return rc;
    const bool fp32 = c->opt.precision == CKTLU_FP32_IR;
    hipStream_t st = stream_of(c);
    LCHK(launch_copy_f64(values_dev, (double *)c->dev.Aval.p, c->an.nnz * (int64_t)batch, st));
    if ((rc = run_refactor(c, batch, values_dev, fp32, true, -1))) return rc;
    LCHK(launch_status_out((const int *)c->dev.ctrl.p + 1 + batch, status_dev, batch, st));
    c->last_batch = batch;
    c->stats.n_refactorize += batch;
    c->dev_values_newer = true;
    return CKTLU_OK;
}

int cktlu_solve_batched(cktlu_ctx *c, int32_t batch, int32_t nrhs, const double *b, double *x,
                        const int32_t *status_dev, double *eta_dev) {
    if (!c || batch < 1 || nrhs < 1 || nrhs > 8 || !b || !x || !status_dev) return CKTLU_E_ARG;
    if (c->state < 2 || c->last_batch < batch) return CKTLU_E_STATE;
    const int n = c->an.n;
    const int64_t nnzA = c->an.nnz;
    const size_t nv = (size_t)n * nrhs * batch;
    // work vectors: z (batch x n rows of YS), r (nv), norms (3 nrhs per instance),
    // |A| and eta per instance, then two int arrays of batch (refinement skip, FP64 skip)
    const size_t zd = (size_t)n * YS * batch + 64;
    const size_t need = zd + nv + 3 * (size_t)nrhs * batch + 2 * (size_t)batch + (size_t)batch + 64;
    int rc = ensure_vec(c, need);
    if (rc) return rc;
    hipStream_t st = stream_of(c);
    double *z = (double *)c->dev.vec.p;
    double *r = z + zd;
    double *norms = r + nv;
    double *anorm = norms + 3 * (size_t)nrhs * batch;
    double *eta = anorm + batch;
    int *skip = (int *)(eta + batch);
    int *skip64 = skip + batch;
    const int *rowperm = (const int *)c->dev.rowperm.p, *colperm = (const int *)c->dev.colperm_sol.p;
    if (eta_dev) LCHK(launch_fill_f64(eta_dev, batch, -1.0, st));
    if (c->opt.precision == CKTLU_FP64) {
        LCHK(launch_gather_rhs(n, nrhs, batch, b, n, rowperm, z, st, (const double *)c->dev.gscale.p));
        if ((rc = tri_solves(c, nrhs, batch, z, false, status_dev))) return rc;
        LCHK(launch_scatter_sol(n, nrhs, batch, z, colperm, x, n, 0, status_dev, st, (const double *)c->dev.sscale.p));
        return CKTLU_OK;
    }
    // FP32 factors with FP64 refinement per instance: x = 0; repeat d = (LU)^-1 r, x += d,
    // r = b - A x, until eta <= ir_tol (instances leave as they converge) or the limit
    const int *Acp = (const int *)c->dev.Acp.p, *Acj = (const int *)c->dev.Acj.p;
    const int *Acsrc = (const int *)c->dev.Acsrc.p;
    const double *Aval = (const double *)c->dev.Aval.p;
    LCHK(launch_fill_f64(anorm, batch, 0.0, st));
    LCHK(launch_anorm_batched(n, batch, nnzA, Acp, Acsrc, Aval, anorm, st));
    LCHK(launch_copy_i32(status_dev, skip, batch, st));
    std::vector<int> hskip(batch), hstatus(batch);
    std::vector<double> heta(batch), prev(batch, INFINITY);
    std::vector<char> stalled(batch, 0);
    HIPCHK(hipMemcpyAsync(hstatus.data(), status_dev, batch * sizeof(int), hipMemcpyDeviceToHost, st));
    for (int it = 1; it <= c->opt.ir_max_iter; it++) {
        LCHK(launch_gather_rhs(n, nrhs, batch, it == 1 ? b : r, n, rowperm, z, st, (const double *)c->dev.gscale.p));
        if ((rc = tri_solves(c, nrhs, batch, z, true, skip))) return rc;
        // x = d on the first step (x of skipped instances is never written), then x += d
        LCHK(launch_scatter_sol(n, nrhs, batch, z, colperm, x, n, it > 1 ? 1 : 0, skip, st, (const double *)c->dev.sscale.p));
        LCHK(launch_fill_f64(norms, 3 * (int64_t)nrhs * batch, 0.0, st));
        LCHK(launch_residual_batched(n, nrhs, batch, nnzA, Acp, Acj, Acsrc, Aval, x, b, r, norms, skip, st));
        LCHK(launch_ir_check(batch, nrhs, norms, anorm, c->opt.ir_tol, skip, eta, st));
        // the first step's outcome stays on the device (converged instances skip the second
        // step's kernels); the host reads it after the second
        if (it == 1 && c->opt.ir_max_iter >= 2) continue;
        HIPCHK(hipMemcpyAsync(hskip.data(), skip, batch * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(heta.data(), eta, batch * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        int active = 0;
        for (int i = 0; i < batch; i++) {
            if (hskip[i] != -1) continue;
            if (it >= 3 && heta[i] > 0.5 * prev[i]) { stalled[i] = 1; hskip[i] = 2; continue; }   // no progress
            prev[i] = heta[i];
            active++;
        }
        if (!active) break;
        HIPCHK(hipMemcpyAsync(skip, hskip.data(), batch * sizeof(int), hipMemcpyHostToDevice, st));
    }
    if (eta_dev) LCHK(launch_copy_f64(eta, eta_dev, batch, st));
    // instances that did not reach ir_tol: FP64 factors and an FP64 solve for them
    std::vector<int> h64(batch, 1);
    int nfb = 0;
    for (int i = 0; i < batch; i++)
        if (hstatus[i] == -1 && (hskip[i] == -1 || stalled[i])) { h64[i] = -1; nfb++; }
    if (!nfb) return CKTLU_OK;
    if ((rc = run_refactor(c, batch, Aval, false, false, -1))) return rc;
    HIPCHK(hipMemcpyAsync(skip64, h64.data(), batch * sizeof(int), hipMemcpyHostToDevice, st));
    LCHK(launch_gather_rhs(n, nrhs, batch, b, n, rowperm, z, st, (const double *)c->dev.gscale.p));
    if ((rc = tri_solves(c, nrhs, batch, z, false, skip64))) return rc;
    LCHK(launch_scatter_sol(n, nrhs, batch, z, colperm, x, n, 0, skip64, st, (const double *)c->dev.sscale.p));
    if (eta_dev) {
        LCHK(launch_fill_f64(norms, 3 * (int64_t)nrhs * batch, 0.0, st));
        LCHK(launch_residual_batched(n, nrhs, batch, nnzA, Acp, Acj, Acsrc, Aval, x, b, r, norms, skip64, st));
        LCHK(launch_ir_check(batch, nrhs, norms, anorm, 0.0, skip64, eta, st));
        LCHK(launch_copy_f64(eta, eta_dev, batch, st));   // instances solved in FP64 get their eta
    }
    HIPCHK(hipStreamSynchronize(st));
    c->stats.n_fp64_fallback_solves += nfb;
    return CKTLU_W_IR_FALLBACK;
}

int cktlu_restart_closure(int32_t n, const int32_t *parent, const int32_t *unfinished, int32_t *in_set) {
    if (n < 0 || (n > 0 && (!parent || !unfinished || !in_set))) return CKTLU_E_ARG;
    std::vector<int> par(parent, parent + n);
    std::vector<char> unf(n), set;
    for (int k = 0; k < n; k++) {
        if (par[k] != -1 && (par[k] <= k || par[k] >= n)) return CKTLU_E_ARG;
        unf[k] = unfinished[k] != 0;
    }
    restart_closure(par, unf, set);
    for (int k = 0; k < n; k++) in_set[k] = set[k];
    return CKTLU_OK;
}

int cktlu_get_last_restart(const cktlu_ctx *c, int32_t *unfinished, int32_t *in_set) {
    if (!c) return CKTLU_E_ARG;
    if (c->last_restart.empty() || (int)c->last_restart.size() != c->an.n) return CKTLU_E_STATE;
    for (int k = 0; k < c->an.n; k++) {
        if (unfinished) unfinished[k] = c->last_unfinished[k];
        if (in_set) in_set[k] = c->last_restart[k];
    }
    return CKTLU_OK;
}

int cktlu_get_perm(const cktlu_ctx *c, int32_t *rowperm, int32_t *colperm) {
    if (!c) return CKTLU_E_ARG;
    if (c->state < 2) return CKTLU_E_STATE;
    for (int k = 0; k < c->an.n; k++) {
        if (rowperm) rowperm[k] = c->an.rowperm_pre[c->f.pivrow[k]];
        if (colperm) colperm[k] = c->an.colperm[k];
    }
    return CKTLU_OK;
}

int cktlu_get_analysis(const cktlu_ctx *c, int32_t *rowperm_pre, int32_t *colperm, int32_t *pivrow,
                       int32_t *parent) {
    if (!c) return CKTLU_E_ARG;
    if (c->state < 1) return CKTLU_E_STATE;
    if (pivrow && c->state < 2) return CKTLU_E_STATE;
    const int n = c->an.n;
    if (rowperm_pre) std::copy(c->an.rowperm_pre.begin(), c->an.rowperm_pre.end(), rowperm_pre);
    if (colperm) std::copy(c->an.colperm.begin(), c->an.colperm.end(), colperm);
    if (pivrow) std::copy(c->f.pivrow.begin(), c->f.pivrow.begin() + n, pivrow);
    if (parent) std::copy(c->an.parent.begin(), c->an.parent.end(), parent);
    return CKTLU_OK;
}

int cktlu_get_factor_nnz(const cktlu_ctx *c, int64_t *nnz_l, int64_t *nnz_u) {
    if (!c) return CKTLU_E_ARG;
    if (c->state < 2) return CKTLU_E_STATE;
    if (nnz_l) *nnz_l = c->f.nnz_l();
    if (nnz_u) *nnz_u = c->f.nnz_u();
    return CKTLU_OK;
}

int cktlu_get_factors(cktlu_ctx *c, int32_t instance, int32_t *Lp, int32_t *Li, double *Lx, int32_t *Up,
                      int32_t *Ui, double *Ux) {
    if (!c) return CKTLU_E_ARG;
    if (c->state < 2) return CKTLU_E_STATE;
    const int n = c->an.n;
    const int64_t F = nnzF(c);
    std::vector<double> compact;
    const double *src = c->f.Fx.data();
    if (c->dev.uploaded && (c->dev_values_newer || instance > 0)) {
        if (instance < 0 || instance >= std::max(1, c->dev.batch_cap)) return CKTLU_E_ARG;
        std::vector<double> padded(F);
        hipStream_t st = stream_of(c);
        if (c->opt.precision == CKTLU_FP32_IR) {
            std::vector<float> v32(F);
            HIPCHK(hipMemcpyAsync(v32.data(), (float *)c->dev.Fx32.p + (size_t)instance * F, F * sizeof(float),
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int64_t q = 0; q < F; q++) padded[q] = v32[q];
        } else {
            HIPCHK(hipMemcpyAsync(padded.data(), (double *)c->dev.Fx64.p + (size_t)instance * F,
                                  F * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        compact.resize(c->f.Fx.size());
        unpad_values(c, padded.data(), compact.data());
        src = compact.data();
    } else if (instance != 0) {
        return CKTLU_E_ARG;
    }
    int64_t lo = 0, uo = 0;
    if (Lp) Lp[0] = 0;
    if (Up) Up[0] = 0;
    for (int k = 0; k < n; k++) {
        const int64_t b = c->f.Fp[k], d = b + c->f.nU[k], e = c->f.Fp[k + 1];
        for (int64_t q = b; q < d; q++, uo++) {
            if (Ui) Ui[uo] = c->f.Fi[q];
            if (Ux) Ux[uo] = src[q];
        }
        for (int64_t q = d; q < e; q++, lo++) {
            if (Li) Li[lo] = c->f.Fi[q];
            if (Lx) Lx[lo] = src[q];
        }
        if (Lp) Lp[k + 1] = (int32_t)lo;
        if (Up) Up[k + 1] = (int32_t)uo;
    }
    return CKTLU_OK;
}

int cktlu_get_levels(const cktlu_ctx *c, int32_t *level) {
    if (!c || !level) return CKTLU_E_ARG;
    if (c->state < 2) return CKTLU_E_STATE;
    std::copy(c->s.level.begin(), c->s.level.end(), level);
    return CKTLU_OK;
}

int cktlu_get_stats(const cktlu_ctx *c, cktlu_stats *out) {
    if (!c || !out) return CKTLU_E_ARG;
    *out = c->stats;
    if (c->state >= 1) {                  // the ordering is known from analyze on
        out->ordering_used = c->an.ordering_used;
        out->fill_amd = c->an.fill_amd;
        out->fill_amf = c->an.fill_amf;
        out->fill_nd = c->an.fill_nd;
        out->fill_ndc = c->an.fill_ndc;
    }
    return CKTLU_OK;
}

int cktlu_get_timing(cktlu_ctx *c, cktlu_timing *out, int reset) {
    if (!c || !out) return CKTLU_E_ARG;
    int rc = collect_timing(c);
    if (rc) return rc;
    *out = c->timing_acc;
    if (reset) std::memset(&c->timing_acc, 0, sizeof(c->timing_acc));
    return CKTLU_OK;
}

size_t cktlu_footprint_bytes(const cktlu_ctx *c, int32_t batch) {
    if (!c) return 0;
    Device &d = const_cast<Device &>(c->dev);
    size_t s = 0;
    for (int i = 0; DevBuf *b = all_buffers(d, i); i++) s += b->bytes;
    const int64_t F = c->s.nnz_dev;
    const size_t Dt = (size_t)(c->an.n - c->s.tail0);
    const size_t nblk = (Dt + kDenseBlock - 1) / kDenseBlock;
    const size_t per = (size_t)F * (c->opt.precision == CKTLU_FP32_IR ? 12 : 8) + (size_t)c->an.nnz * 8 +
                       (size_t)c->an.n * (4 + 8 * YS) + Dt * Dt * 8 +
                       nblk * 2 * kDenseBlock * kDenseBlock * 8 + (size_t)c->s.schur_nscr * Dt * 8;
    if (!c->dev.uploaded)
        s += (size_t)F * 12 + (size_t)c->an.nnz * 12 + (size_t)c->an.n * 64 + c->s.smap.size() * sizeof(int) +
             c->s.tmoff.size() * sizeof(int64_t);
    return s + (batch > 0 ? per * (size_t)batch : 0);
}

}  // extern "C"
