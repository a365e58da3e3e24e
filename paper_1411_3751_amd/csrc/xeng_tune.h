// Autotuner and whole-step graph capture. Part of the libxeng.so translation
// unit (included by xeng.hip after the context API).
//
// The autotuner times, on the caller's own sample buffers, every kernel
// family that can run each subarray (the persistent 128 x 128 tile kernel,
// and the register-staging kernel with 32, 64 or 128-input tiles), keeps the
// fastest per subarray, then times the schedule options of the batched
// persistent launch (workgroups per CU, tile order) with all subarrays
// together, and finally whole steps with every subarray the persistent kernel
// can run moved into that one launch (then handed back one at a time while
// that helps). Choices go to a process-wide cache
// keyed by the subarray shapes (per shape for a subarray alone, per set of
// shapes for a batch), which xeng_create consults.
#pragma once

namespace {

struct EvPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EvPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Milliseconds per run of fn: after one untimed run, untimed batches of
// `reps` runs until about settle_ms of work has run, then the median of
// three timed batches of `reps` runs. Under sustained MFMA load the chip is
// power-limited: its clock falls within milliseconds and again over a few
// hundred, so a candidate timed on a cooler chip, or one whose extra memory
// traffic costs clock only once the limit holds, would be favoured. Every
// run starts from a logically zero accumulator, like a step after a dump.
constexpr float TUNE_SETTLE_MS = 30.f;        // kernel family of one subarray
constexpr float TUNE_SETTLE_STEP_MS = 60.f;   // schedules of whole steps
template <class Fn>
int time_runs(xeng_ctx *ctx, int reps, Fn fn, float &ms, float settle_ms = TUNE_SETTLE_MS)
{
    EvPair e;
    HIP_TRY(hipEventCreate(&e.a));
    HIP_TRY(hipEventCreate(&e.b));
    auto zero_state = [&]() {
        for (Sub &s : ctx->subs) s.acc_zero = true;
    };
    auto batch = [&](float &t) -> int {
        HIP_TRY(hipEventRecord(e.a, ctx->stream));
        for (int r = 0; r < reps; ++r) {
            zero_state();
            const int rc = fn();
            if (rc) return rc;
        }
        HIP_TRY(hipEventRecord(e.b, ctx->stream));
        HIP_TRY(hipEventSynchronize(e.b));
        HIP_TRY(hipEventElapsedTime(&t, e.a, e.b));
        return XENG_OK;
    };
    zero_state();
    int rc = fn();
    if (rc) return rc;
    float t[3] = {0.f, 0.f, 0.f};
    rc = batch(t[0]);
    if (rc) return rc;
    const int settle = t[0] > 0.f ? std::min(1000, (int)(settle_ms / t[0])) : 0;
    for (int q = 0; q < settle; ++q) {
        rc = batch(t[1]);
        if (rc) return rc;
    }
    for (int q = 0; q < 3; ++q) {
        rc = batch(t[q]);
        if (rc) return rc;
    }
    std::sort(t, t + 3);
    ms = t[1] / (float)reps;
    return XENG_OK;
}

// Append one JSON object to the context's record of the last autotune.
void tune_note(xeng_ctx *ctx, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void tune_note(xeng_ctx *ctx, const char *fmt, ...)
{
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (!ctx->tune_log.empty()) ctx->tune_log += ", ";
    ctx->tune_log += buf;
}

// Milliseconds of one subarray's work alone under its current choice.
int time_one(xeng_ctx *ctx, int k, const void *const *d_samples, int reps, float &ms)
{
    Sub &s = ctx->subs[k];
    if (!s.wave)
        return time_runs(ctx, reps, [&]() { return launch_regs(s, d_samples[k], ctx->stream); }, ms);
    WavePlan p;
    p.engine = s.cfg.engine;
    p.in_bits = s.cfg.in_bits;
    p.w1 = s.w1;
    p.wv = s.wv;
    p.subs = {k};
    build_schedule(p, ctx->subs, ctx->n_cu, ctx->wg_per_cu, ctx->order);
    int rc = upload_plan(p);
    if (!rc) rc = time_runs(ctx, reps, [&]() { return launch_wave(ctx, p, d_samples); }, ms);
    (void)hipStreamSynchronize(ctx->stream);
    return rc;
}

int launch_all(xeng_ctx *ctx, const void *const *d_samples)
{
    for (WavePlan &p : ctx->plans) {
        int rc = launch_wave(ctx, p, d_samples);
        if (rc) return rc;
    }
    for (size_t k = 0; k < ctx->subs.size(); ++k)
        if (!ctx->subs[k].wave) {
            int rc = launch_regs(ctx->subs[k], d_samples[k], ctx->stream);
            if (rc) return rc;
        }
    return XENG_OK;
}

// The launches of a correlate-and-dump into out (the persistent kernels
// write their last segment straight to out, the others are dumped)
int launch_fused(xeng_ctx *ctx, const void *const *d_samples, void *const *out)
{
    for (WavePlan &p : ctx->plans) {
        int rc = launch_wave(ctx, p, d_samples, out);
        if (rc) return rc;
    }
    for (size_t k = 0; k < ctx->subs.size(); ++k) {
        const Sub &s = ctx->subs[k];
        if (s.wave) continue;
        int rc = launch_regs(ctx->subs[k], d_samples[k], ctx->stream);
        if (!rc) rc = dump_device(s, (uint32_t *)out[k], ctx->stream);
        if (rc) return rc;
    }
    return XENG_OK;
}

} // namespace

struct xeng_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<DevBuf> keep; // tile lists the captured launches read
};

extern "C" {

int xeng_autotune(xeng_ctx *ctx, const void *const *d_samples, int reps)
{
    if (!ctx || !d_samples) return fail(XENG_EINVAL, "NULL argument");
    for (size_t k = 0; k < ctx->subs.size(); ++k) {
        if (!d_samples[k]) return fail(XENG_EINVAL, "d_samples[%zu] is NULL", k);
        if (((uintptr_t)d_samples[k] & 15) != 0)
            return fail(XENG_EINVAL, "d_samples[%zu] is not 16-byte aligned", k);
    }
    if (reps < 1) reps = 1;
    if (reps > 100) reps = 100;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->tune_log.clear();
    // (1) kernel family per subarray, each timed alone
    for (size_t k = 0; k < ctx->subs.size(); ++k) {
        Sub &s = ctx->subs[k];
        if (s.cfg.engine == XENG_ENGINE_FP8) continue; // one kernel family only
        std::vector<SubChoice> cands;
        if (w1_path(s.cfg)) {
            cands.push_back({FAM_W2, 4});
            cands.push_back({FAM_W1, 4});
        }
        if (sn_path(s.cfg)) cands.push_back({FAM_SN, 4});
        if (wave_path(s.cfg)) cands.push_back({FAM_WG, 4});
        const int N = s.cfg.n_inputs;
        if (N <= 128) cands.push_back({FAM_REG, 1});
        if (N <= 1024) cands.push_back({FAM_REG, 2});
        cands.push_back({FAM_REG, 4});
        float best = 0.f;
        SubChoice pick = cands[0];
        for (size_t q = 0; q < cands.size(); ++q) {
            set_choice(s, cands[q].fam, cands[q].wt);
            float ms = 0.f;
            int rc = time_one(ctx, (int)k, d_samples, reps, ms);
            if (rc) return rc;
            tune_note(ctx, "{\"step\": \"alone\", \"sub\": %zu, \"kernel\": \"%s\", \"tile\": %d, "
                           "\"ms\": %.4f}",
                      k, fam_name(cands[q].fam),
                      cands[q].fam == FAM_REG ? 32 * cands[q].wt
                                              : (cands[q].fam == FAM_W2 || cands[q].fam == FAM_SN ? 64 : 128),
                      ms);
            if (q == 0 || ms < best) {
                best = ms;
                pick = cands[q];
            }
        }
        set_choice(s, pick.fam, pick.wt);
    }
    // the picks of each subarray timed alone (kept for contexts of that shape)
    std::vector<SubChoice> alone;
    for (const Sub &s : ctx->subs) alone.push_back(SubChoice{fam_of(s), s.wt});
    // (2) schedule of the batched persistent launch, all subarrays together:
    // whole steps under each schedule option. A step is timed both as a
    // correlate (the launches that integrate) and as a correlate-and-dump
    // into scratch outputs (the last launch writes the exact output, and
    // its flush differs), and an option's time is the sum: the two kinds
    // of step can favour different schedules.
    std::vector<DevBuf> scratch_out;
    std::vector<void *> outs;
    for (const Sub &s : ctx->subs) {
        void *p = nullptr;
        const size_t bytes = (size_t)s.tri * (size_t)s.cfg.n_chans * 8;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            scratch_out.clear();
            outs.clear();
            break;
        }
        scratch_out.push_back(DevBuf(p, DevFree()));
        outs.push_back(p);
    }
    auto time_step = [&](float &ms) -> int {
        int rc = time_runs(ctx, reps, [&]() { return launch_all(ctx, d_samples); }, ms,
                           TUNE_SETTLE_STEP_MS);
        if (rc || outs.empty()) return rc;
        float ms_fused = 0.f;
        rc = time_runs(ctx, reps, [&]() { return launch_fused(ctx, d_samples, outs.data()); },
                       ms_fused, TUNE_SETTLE_STEP_MS);
        ms += ms_fused;
        return rc;
    };
    // (each option timed in a forward and a reverse pass over the options,
    // its time the mean of the two, so a drift of the clock over the passes
    // favours none of them)
    auto tune_schedule = [&](float &best, int &bw, int &bo) -> int {
        const int opts[4][2] = {{2, 0}, {2, 1}, {1, 0}, {1, 1}};
        bool any_wave = false;
        for (const Sub &s : ctx->subs) any_wave |= s.wave;
        const int n_opt = any_wave ? 4 : 1;
        float sum[4] = {0.f, 0.f, 0.f, 0.f};
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < n_opt; ++i) {
                const int q = pass == 0 ? i : n_opt - 1 - i;
                ctx->wg_per_cu = opts[q][0];
                ctx->order = opts[q][1];
                int rc = replan(ctx);
                if (rc) return rc;
                float ms = 0.f;
                rc = time_step(ms);
                if (rc) return rc;
                sum[q] += ms;
            }
        for (int q = 0; q < n_opt; ++q) {
            const float ms = sum[q] / 2.f;
            tune_note(ctx, "{\"step\": \"schedule\", \"workgroups_per_cu\": %d, \"order\": %d, "
                           "\"ms\": %.4f, \"timed\": \"%s\"}",
                      opts[q][0], opts[q][1], ms,
                      outs.empty() ? "correlate" : "correlate + correlate_dump");
            if (q == 0 || ms < best) {
                best = ms;
                bw = opts[q][0];
                bo = opts[q][1];
            }
        }
        return XENG_OK;
    };
    float best = 0.f;
    int bw = 2, bo = 0;
    int rc = tune_schedule(best, bw, bo);
    if (rc) return rc;
    // (3) the batch as a whole. Step (1) times each subarray alone, but one
    // persistent launch over several subarrays balances its workgroups far
    // better than any of them alone (more tiles per workgroup), so also time
    // whole steps with every subarray the persistent kernel can take on it,
    // and keep whichever assignment is faster.
    bool can_move = false;
    for (const Sub &s : ctx->subs) can_move |= wave_path(s.cfg) && !s.wave;
    if (ctx->subs.size() > 1 && can_move) {
        for (Sub &s : ctx->subs)
            if (wave_path(s.cfg)) set_choice(s, FAM_WG, s.wt);
        float best_all = 0.f;
        int bw_all = 2, bo_all = 0;
        rc = tune_schedule(best_all, bw_all, bo_all);
        if (rc) return rc;
        if (best_all < best) {
            best = best_all;
            bw = bw_all;
            bo = bo_all;
            // then hand back, smallest N first, each subarray whose own pick
            // was the register kernel, while whole steps get faster
            std::vector<size_t> order_n(ctx->subs.size());
            std::iota(order_n.begin(), order_n.end(), (size_t)0);
            std::stable_sort(order_n.begin(), order_n.end(), [&](size_t a, size_t b) {
                return ctx->subs[a].cfg.n_inputs < ctx->subs[b].cfg.n_inputs;
            });
            ctx->wg_per_cu = bw;
            ctx->order = bo;
            for (size_t k : order_n) {
                Sub &s = ctx->subs[k];
                if (alone[k].fam != FAM_REG || !s.wave || s.cfg.engine == XENG_ENGINE_FP8) continue;
                const int wt_now = s.wt, fam_now = fam_of(s);
                set_choice(s, FAM_REG, alone[k].wt);
                rc = replan(ctx);
                if (rc) return rc;
                float ms = 0.f;
                rc = time_step(ms);
                if (rc) return rc;
                if (ms < best) best = ms;
                else set_choice(s, fam_now, wt_now);
            }
        } else {
            for (size_t k = 0; k < ctx->subs.size(); ++k)
                set_choice(ctx->subs[k], alone[k].fam, alone[k].wt);
        }
    }
    ctx->wg_per_cu = bw;
    ctx->order = bo;
    rc = replan(ctx);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (Sub &s : ctx->subs) {
        s.acc_zero = true;
        s.since_dump = 0;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (size_t k = 0; k < ctx->subs.size(); ++k)
            g_tune_sub[ArchKey{ctx->arch, key_of(ctx->subs[k].cfg)}] = alone[k];
        std::vector<SubChoice> chosen;
        for (const Sub &s : ctx->subs) chosen.push_back(SubChoice{fam_of(s), s.wt});
        g_tune_set[ArchSet{ctx->arch, keys_of(ctx)}] = chosen;
        g_tune_sched[ArchSet{ctx->arch, keys_of(ctx)}] = SchedChoice{bw, bo};
    }
    ctx->tuned = true;
    tuning_file_autosave();
    return XENG_OK;
}

int xeng_graph_create(xeng_ctx *ctx, const void *const *d_samples, void *const *out,
                      xeng_graph **out_graph)
{
    if (!out_graph) return fail(XENG_EINVAL, "out_graph is NULL");
    *out_graph = nullptr;
    if (!ctx || !d_samples || !out) return fail(XENG_EINVAL, "NULL argument");
    for (const Sub &s : ctx->subs)
        if (s.since_dump != 0)
            return fail(XENG_EINVAL, "graph capture needs a context with nothing accumulated");
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    hipStream_t cap = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t saved = ctx->stream;
    ctx->stream = cap;
    hipGraph_t g = nullptr;
    int rc = XENG_OK;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        rc = fail(XENG_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    } else {
        rc = xeng_correlate_dump(ctx, d_samples, out, 1, 1);
        e = hipStreamEndCapture(cap, &g);
        if (!rc && e != hipSuccess) rc = fail(XENG_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    ctx->stream = saved;
    for (Sub &s : ctx->subs) {
        s.acc_zero = true;
        s.since_dump = 0;
    }
    (void)hipStreamDestroy(cap);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    xeng_graph *xg = new (std::nothrow) xeng_graph;
    if (!xg) {
        (void)hipGraphDestroy(g);
        return fail(XENG_ENOMEM, "host allocation failed");
    }
    xg->graph = g;
    for (const WavePlan &p : ctx->plans) xg->keep.push_back(p.d_mem);
    e = hipGraphInstantiate(&xg->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete xg;
        return fail(XENG_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    *out_graph = xg;
    return XENG_OK;
}

int xeng_graph_launch(xeng_graph *g, void *hip_stream)
{
    if (!g) return fail(XENG_EINVAL, "graph is NULL");
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)hip_stream));
    return XENG_OK;
}

int xeng_graph_destroy(xeng_graph *g)
{
    if (!g) return XENG_OK;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return XENG_OK;
}

} // extern "C"
