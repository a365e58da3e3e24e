// Streaming integration: a device ring of gulp slots feeding one context.
// Part of the libxeng.so translation unit (included by xeng.hip after the
// context API); uses only that API and the HIP runtime.
//
// Gulps are numbered in arrival order; a gulp is either pushed (filled and
// correlated) or dropped (counted, adds nothing). Per pushed gulp g (slot
// g % n_slots):
//   clock stream  : record arrive[g] when the caller asks for the slot (this
//                   stream never waits, so the event marks the host's request)
//   ingest stream : wait slot_free[slot] (the slot's previous gulp
//                   correlated), caller's fill work, record ready[g]
//   compute stream: wait ready[g]; the correlation; record slot_free[slot]
// and for every gulp g, pushed or dropped, on the compute stream:
//   - if g ends a fast period: the selected autocorrelations are copied to
//     fast buffer k % 2 and cleared, record fast_dumped[k % 2]; the output
//     stream copies them to the caller's host buffer and records
//     fast_out_done[k % 2];
//   - if g ends a dump period d: wait out_done[d % 2] (dump d - 2 copied
//     out), dump into buffer d % 2 with reset (fused into the correlation
//     when g was pushed and ends no fast period), record dumped[d % 2]; the
//     output stream copies it to host_dumps[d % n_host] and records
//     out_done[d % 2];
//   - record done[g].
// In non-blocking mode a gulp whose slot is still in use (its previous gulp
// not yet correlated: the engine is behind) is dropped at next_slot instead
// of waited for, which is how an overrun shows: the drop count grows.
#pragma once

namespace {

constexpr int STREAM_HIST = 1024; // gulps whose events are kept

struct GulpEv {
    hipEvent_t arrive = nullptr, ready = nullptr, done = nullptr;
};

} // namespace

struct xeng_stream {
    xeng_subarray cfg{};
    xeng_ctx *ctx = nullptr;
    hipStream_t s_in = nullptr, s_comp = nullptr, s_out = nullptr;
    hipStream_t s_clk = nullptr;         // arrival stamps only: never waits
    int n_slots = 0, dump_every = 0;
    size_t gulp_bytes = 0, dump_bytes = 0;
    uint8_t *ring = nullptr;
    std::vector<hipEvent_t> slot_free;   // per slot, recorded after its correlation
    std::vector<bool> slot_used;
    std::vector<GulpEv> ev;              // per gulp, ring of STREAM_HIST
    std::vector<uint8_t> was_dropped;    // per gulp, ring of STREAM_HIST
    uint32_t *d_dump[2] = {nullptr, nullptr};
    hipEvent_t dumped[2] = {nullptr, nullptr}, out_done[2] = {nullptr, nullptr};
    bool out_pending[2] = {false, false};
    std::vector<void *> host;            // caller's host dump buffers
    bool nonblocking = false;
    int64_t n_gulps = 0;                 // gulps so far (pushed + dropped)
    int64_t n_dropped = 0;
    int64_t n_dumps = 0;                 // dumps enqueued
    bool have_slot = false;              // next_slot called, push pending
    // fast-cadence autocorrelations of selected inputs
    int fast_every = 0, n_sel = 0;
    size_t fast_bytes = 0;
    int32_t *d_fast[2] = {nullptr, nullptr};
    hipEvent_t fast_dumped[2] = {nullptr, nullptr}, fast_out_done[2] = {nullptr, nullptr};
    bool fast_pending[2] = {false, false};
    std::vector<void *> fast_host;
    int64_t n_fast = 0;                  // fast dumps enqueued
};

namespace {

void stream_free(xeng_stream *s)
{
    if (!s) return;
    if (s->s_in) (void)hipStreamSynchronize(s->s_in);
    if (s->s_comp) (void)hipStreamSynchronize(s->s_comp);
    if (s->s_out) (void)hipStreamSynchronize(s->s_out);
    if (s->s_clk) (void)hipStreamSynchronize(s->s_clk);
    if (s->ctx) xeng_destroy(s->ctx);
    for (hipEvent_t e : s->slot_free)
        if (e) (void)hipEventDestroy(e);
    for (GulpEv &g : s->ev) {
        if (g.arrive) (void)hipEventDestroy(g.arrive);
        if (g.ready) (void)hipEventDestroy(g.ready);
        if (g.done) (void)hipEventDestroy(g.done);
    }
    for (int k = 0; k < 2; ++k) {
        if (s->dumped[k]) (void)hipEventDestroy(s->dumped[k]);
        if (s->out_done[k]) (void)hipEventDestroy(s->out_done[k]);
        if (s->d_dump[k]) (void)hipFree(s->d_dump[k]);
        if (s->fast_dumped[k]) (void)hipEventDestroy(s->fast_dumped[k]);
        if (s->fast_out_done[k]) (void)hipEventDestroy(s->fast_out_done[k]);
        if (s->d_fast[k]) (void)hipFree(s->d_fast[k]);
    }
    if (s->ring) (void)hipFree(s->ring);
    if (s->s_in) (void)hipStreamDestroy(s->s_in);
    if (s->s_comp) (void)hipStreamDestroy(s->s_comp);
    if (s->s_out) (void)hipStreamDestroy(s->s_out);
    if (s->s_clk) (void)hipStreamDestroy(s->s_clk);
    delete s;
}

int stream_init(xeng_stream *s)
{
    HIP_TRY(hipStreamCreateWithFlags(&s->s_in, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&s->s_comp, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&s->s_out, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&s->s_clk, hipStreamNonBlocking));
    int rc = xeng_create(&s->cfg, 1, s->s_comp, &s->ctx);
    if (rc) return rc;
    hipError_t e = hipMalloc((void **)&s->ring, s->gulp_bytes * (size_t)s->n_slots);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(XENG_ENOMEM, "hipMalloc(%zu) for the gulp ring: %s",
                    s->gulp_bytes * (size_t)s->n_slots, hipGetErrorString(e));
    }
    for (int k = 0; k < 2; ++k) {
        e = hipMalloc((void **)&s->d_dump[k], s->dump_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(XENG_ENOMEM, "hipMalloc(%zu) for a dump buffer: %s", s->dump_bytes,
                        hipGetErrorString(e));
        }
        HIP_TRY(hipEventCreateWithFlags(&s->dumped[k], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&s->out_done[k], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&s->fast_dumped[k], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&s->fast_out_done[k], hipEventDisableTiming));
    }
    s->slot_free.assign(s->n_slots, nullptr);
    s->slot_used.assign(s->n_slots, false);
    for (int k = 0; k < s->n_slots; ++k)
        HIP_TRY(hipEventCreateWithFlags(&s->slot_free[k], hipEventDisableTiming));
    s->ev.resize(STREAM_HIST);
    s->was_dropped.assign(STREAM_HIST, 0);
    for (GulpEv &g : s->ev) {
        HIP_TRY(hipEventCreate(&g.arrive));
        HIP_TRY(hipEventCreate(&g.ready));
        HIP_TRY(hipEventCreate(&g.done));
    }
    return XENG_OK;
}

// The cadence work of gulp g on the compute stream, after its correlation
// (pushed) or in its place (dropped). `slot` is the slot of a pushed gulp
// (its correlation is fused into the dump when it ends a dump period and no
// fast period), else -1.
int stream_cadence(xeng_stream *s, int64_t g, int slot)
{
    const bool fast = s->fast_every > 0 && (g + 1) % s->fast_every == 0;
    const bool dump = (g + 1) % s->dump_every == 0;
    const void *p = slot >= 0 ? (const void *)(s->ring + (size_t)slot * s->gulp_bytes) : nullptr;
    const bool fused = p && dump && !fast;
    int rc;
    const int b = (int)(s->n_dumps % 2);
    // the dump buffer's previous dump (d - 2) must be copied out first
    if (dump && s->out_pending[b]) HIP_TRY(hipStreamWaitEvent(s->s_comp, s->out_done[b], 0));
    if (fused) {
        void *outp = s->d_dump[b];
        rc = xeng_correlate_dump(s->ctx, &p, &outp, 1, 1);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(s->slot_free[slot], s->s_comp));
    } else if (p) {
        rc = xeng_correlate(s->ctx, &p);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(s->slot_free[slot], s->s_comp));
    }
    if (fast) {
        const int f = (int)(s->n_fast % 2);
        if (s->fast_pending[f]) HIP_TRY(hipStreamWaitEvent(s->s_comp, s->fast_out_done[f], 0));
        void *fo = s->d_fast[f];
        rc = xeng_dump_fast_autos(s->ctx, &fo, 1, 1);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(s->fast_dumped[f], s->s_comp));
        HIP_TRY(hipStreamWaitEvent(s->s_out, s->fast_dumped[f], 0));
        if (!s->fast_host.empty())
            HIP_TRY(hipMemcpyAsync(s->fast_host[s->n_fast % s->fast_host.size()], s->d_fast[f],
                                   s->fast_bytes, hipMemcpyDeviceToHost, s->s_out));
        HIP_TRY(hipEventRecord(s->fast_out_done[f], s->s_out));
        s->fast_pending[f] = true;
        ++s->n_fast;
    }
    if (dump) {
        if (!fused) {
            // the sums of the period so far (zeros if nothing was correlated)
            void *outp = s->d_dump[b];
            rc = xeng_dump(s->ctx, &outp, 1, 1);
            if (rc) return rc;
        }
        HIP_TRY(hipEventRecord(s->dumped[b], s->s_comp));
        HIP_TRY(hipStreamWaitEvent(s->s_out, s->dumped[b], 0));
        if (!s->host.empty())
            HIP_TRY(hipMemcpyAsync(s->host[s->n_dumps % s->host.size()], s->d_dump[b], s->dump_bytes,
                                   hipMemcpyDeviceToHost, s->s_out));
        HIP_TRY(hipEventRecord(s->out_done[b], s->s_out));
        s->out_pending[b] = true;
        ++s->n_dumps;
    }
    HIP_TRY(hipEventRecord(s->ev[g % STREAM_HIST].done, s->s_comp));
    return XENG_OK;
}

// Gulp n_gulps is lost: counted, its cadence work done, nothing correlated.
int stream_drop(xeng_stream *s)
{
    const int64_t g = s->n_gulps;
    s->was_dropped[g % STREAM_HIST] = 1;
    int rc = stream_cadence(s, g, -1);
    if (rc) return rc;
    ++s->n_dropped;
    ++s->n_gulps;
    s->have_slot = false;
    return XENG_OK;
}

} // namespace

extern "C" {

int xeng_stream_create(const xeng_subarray *sub, int n_slots, int dump_every,
                       void *const *host_dumps, int n_host_dumps, xeng_stream **out)
{
    if (!out) return fail(XENG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!sub) return fail(XENG_EINVAL, "sub is NULL");
    if (n_slots < 2) return fail(XENG_EINVAL, "n_slots %d < 2", n_slots);
    if (dump_every < 1) return fail(XENG_EINVAL, "dump_every %d < 1", dump_every);
    if (host_dumps && n_host_dumps < 1)
        return fail(XENG_EINVAL, "n_host_dumps %d < 1 with host buffers", n_host_dumps);
    int rc = validate(*sub, 0);
    if (rc) return rc;
    const int64_t bound =
        sub->in_bits == 4 ? XENG_MAX_DUMP_SAMPLES_4BIT : XENG_MAX_DUMP_SAMPLES_8BIT;
    if ((int64_t)dump_every * sub->n_time > bound)
        return fail(XENG_ERANGE, "dump period %d x %d samples exceeds the dump limit %lld",
                    dump_every, sub->n_time, (long long)bound);
    if (host_dumps)
        for (int k = 0; k < n_host_dumps; ++k)
            if (!host_dumps[k]) return fail(XENG_EINVAL, "host_dumps[%d] is NULL", k);
    xeng_stream *s = new (std::nothrow) xeng_stream;
    if (!s) return fail(XENG_ENOMEM, "host allocation failed");
    s->cfg = *sub;
    s->n_slots = n_slots;
    s->dump_every = dump_every;
    s->gulp_bytes = (size_t)sub->n_time * (size_t)sub->n_chans * (size_t)sub->n_inputs *
                    (size_t)(sub->in_bits / 4);
    s->dump_bytes = (size_t)sub->n_chans * (size_t)sub->n_inputs * (size_t)(sub->n_inputs + 1) / 2 * 8;
    if (host_dumps) s->host.assign(host_dumps, host_dumps + n_host_dumps);
    rc = stream_init(s);
    if (rc) {
        stream_free(s);
        return rc;
    }
    *out = s;
    return XENG_OK;
}

int xeng_stream_set_nonblocking(xeng_stream *s, int on)
{
    if (!s) return fail(XENG_EINVAL, "s is NULL");
    s->nonblocking = on != 0;
    return XENG_OK;
}

int xeng_stream_set_fast_autos(xeng_stream *s, const int32_t *inputs, int n, int every,
                               void *const *host_out, int n_host)
{
    if (!s) return fail(XENG_EINVAL, "s is NULL");
    if (s->n_gulps != 0)
        return fail(XENG_EINVAL, "fast-cadence autocorrelations are set before the first gulp");
    if (n < 1 || every < 1) return fail(XENG_EINVAL, "n %d and every %d must be >= 1", n, every);
    if (host_out && n_host < 1) return fail(XENG_EINVAL, "n_host %d < 1 with host buffers", n_host);
    if (host_out)
        for (int k = 0; k < n_host; ++k)
            if (!host_out[k]) return fail(XENG_EINVAL, "host_out[%d] is NULL", k);
    int rc = xeng_set_fast_autos(s->ctx, 0, inputs, n);
    if (rc) return rc;
    for (int k = 0; k < 2; ++k) {
        if (s->d_fast[k]) (void)hipFree(s->d_fast[k]);
        s->d_fast[k] = nullptr;
    }
    s->fast_bytes = (size_t)s->cfg.n_chans * (size_t)n * 4;
    for (int k = 0; k < 2; ++k) {
        hipError_t e = hipMalloc((void **)&s->d_fast[k], s->fast_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(XENG_ENOMEM, "hipMalloc(%zu) for a fast-cadence buffer: %s", s->fast_bytes,
                        hipGetErrorString(e));
        }
    }
    s->fast_host.clear();
    if (host_out) s->fast_host.assign(host_out, host_out + n_host);
    s->n_sel = n;
    s->fast_every = every;
    return XENG_OK;
}

int xeng_stream_next_slot(xeng_stream *s, void **d_slot, void **ingest_stream)
{
    if (!s || !d_slot) return fail(XENG_EINVAL, "NULL argument");
    const int64_t g = s->n_gulps;
    const int slot = (int)(g % s->n_slots);
    if (!s->have_slot) {
        if (s->nonblocking && s->slot_used[slot]) {
            const hipError_t q = hipEventQuery(s->slot_free[slot]);
            if (q == hipErrorNotReady) {
                int rc = stream_drop(s);
                if (rc) return rc;
                *d_slot = nullptr;
                if (ingest_stream) *ingest_stream = nullptr;
                return fail(XENG_EBUSY, "gulp %lld dropped: slot %d still in use", (long long)g, slot);
            }
            if (q != hipSuccess) return fail(XENG_EHIP, "hipEventQuery: %s", hipGetErrorString(q));
        }
        // arrival first, on the idle clock stream: the latency then includes
        // any wait for the slot's previous gulp
        HIP_TRY(hipEventRecord(s->ev[g % STREAM_HIST].arrive, s->s_clk));
        if (s->slot_used[slot]) HIP_TRY(hipStreamWaitEvent(s->s_in, s->slot_free[slot], 0));
        s->have_slot = true;
    }
    *d_slot = s->ring + (size_t)slot * s->gulp_bytes;
    if (ingest_stream) *ingest_stream = (void *)s->s_in;
    return XENG_OK;
}

int xeng_stream_push(xeng_stream *s, int64_t *gulp)
{
    if (!s) return fail(XENG_EINVAL, "s is NULL");
    if (!s->have_slot) return fail(XENG_EINVAL, "push without next_slot");
    const int64_t g = s->n_gulps;
    const int slot = (int)(g % s->n_slots);
    GulpEv &e = s->ev[g % STREAM_HIST];
    HIP_TRY(hipEventRecord(e.ready, s->s_in));
    HIP_TRY(hipStreamWaitEvent(s->s_comp, e.ready, 0));
    s->was_dropped[g % STREAM_HIST] = 0;
    int rc = stream_cadence(s, g, slot);
    if (rc) return rc;
    s->slot_used[slot] = true;
    s->have_slot = false;
    ++s->n_gulps;
    if (gulp) *gulp = g;
    return XENG_OK;
}

int xeng_stream_drop(xeng_stream *s, int64_t *gulp)
{
    if (!s) return fail(XENG_EINVAL, "s is NULL");
    const int64_t g = s->n_gulps;
    int rc = stream_drop(s);
    if (rc) return rc;
    if (gulp) *gulp = g;
    return XENG_OK;
}

int xeng_stream_dump_wait(xeng_stream *s, int64_t d, void **d_dump)
{
    if (!s) return fail(XENG_EINVAL, "s is NULL");
    if (d < 0 || d >= s->n_dumps || d < s->n_dumps - 2)
        return fail(XENG_EINVAL, "dump %lld is not one of the last two enqueued (%lld so far)",
                    (long long)d, (long long)s->n_dumps);
    const int b = (int)(d % 2);
    HIP_TRY(hipEventSynchronize(s->out_done[b]));
    if (d_dump) *d_dump = s->d_dump[b];
    return XENG_OK;
}

int xeng_stream_fast_wait(xeng_stream *s, int64_t k, void **d_out)
{
    if (!s) return fail(XENG_EINVAL, "s is NULL");
    if (k < 0 || k >= s->n_fast || k < s->n_fast - 2)
        return fail(XENG_EINVAL, "fast dump %lld is not one of the last two enqueued (%lld so far)",
                    (long long)k, (long long)s->n_fast);
    const int f = (int)(k % 2);
    HIP_TRY(hipEventSynchronize(s->fast_out_done[f]));
    if (d_out) *d_out = s->d_fast[f];
    return XENG_OK;
}

int xeng_stream_gulp_times(xeng_stream *s, int64_t g, float *arrive_ms, float *ready_ms)
{
    if (!s) return fail(XENG_EINVAL, "s is NULL");
    if (g < 0 || g >= s->n_gulps || g < s->n_gulps - STREAM_HIST)
        return fail(XENG_EINVAL, "gulp %lld is not among the last %d", (long long)g, STREAM_HIST);
    if (s->was_dropped[g % STREAM_HIST]) return fail(XENG_EINVAL, "gulp %lld was dropped", (long long)g);
    GulpEv &e = s->ev[g % STREAM_HIST];
    HIP_TRY(hipEventSynchronize(e.done));
    HIP_TRY(hipEventSynchronize(e.arrive));
    if (arrive_ms) HIP_TRY(hipEventElapsedTime(arrive_ms, e.arrive, e.done));
    if (ready_ms) HIP_TRY(hipEventElapsedTime(ready_ms, e.ready, e.done));
    return XENG_OK;
}

int xeng_stream_gulps(const xeng_stream *s, int64_t *out)
{
    if (!s || !out) return fail(XENG_EINVAL, "NULL argument");
    *out = s->n_gulps;
    return XENG_OK;
}

int xeng_stream_backlog(xeng_stream *s, int64_t *out)
{
    if (!s || !out) return fail(XENG_EINVAL, "NULL argument");
    // gulps whose work on the compute stream has not finished: done events
    // complete in gulp order there, so count back from the newest until one
    // has completed
    int64_t n = 0;
    const int64_t lo = std::max<int64_t>(0, s->n_gulps - STREAM_HIST);
    for (int64_t g = s->n_gulps - 1; g >= lo; --g) {
        const hipError_t q = hipEventQuery(s->ev[g % STREAM_HIST].done);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) return fail(XENG_EHIP, "hipEventQuery: %s", hipGetErrorString(q));
        ++n;
    }
    *out = n;
    return XENG_OK;
}

int xeng_stream_stats(xeng_stream *s, xeng_stream_counts *out)
{
    if (!s || !out) return fail(XENG_EINVAL, "NULL argument");
    int64_t backlog = 0;
    int rc = xeng_stream_backlog(s, &backlog);
    if (rc) return rc;
    out->gulps = s->n_gulps;
    out->correlated = s->n_gulps - s->n_dropped;
    out->dropped = s->n_dropped;
    out->dumps = s->n_dumps;
    out->fast_dumps = s->n_fast;
    out->backlog = backlog;
    return XENG_OK;
}

int xeng_stream_destroy(xeng_stream *s)
{
    if (!s) return XENG_OK;
    stream_free(s);
    return XENG_OK;
}

} // extern "C"
