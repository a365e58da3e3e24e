// Streaming integration: a device ring of gulp slots feeding one context.
// Part of the libxeng.so translation unit (included by xeng.hip after the
// context API); uses only that API and the HIP runtime.
//
// Per gulp g (slot g % n_slots):
//   clock stream  : record arrive[g] when the caller asks for the slot (this
//                   stream never waits, so the event marks the host's request)
//   ingest stream : wait slot_free[slot] (gulp g - n_slots correlated),
//                   caller's fill work, record ready[g]
//   compute stream: wait ready[g]; xeng_correlate, or, if g completes dump
//                   d: wait out_done[d % 2] (dump d - 2 copied out), then
//                   xeng_correlate_dump into dump buffer d % 2 with reset and
//                   record dumped[d % 2]; record slot_free[slot] and done[g]
//   output stream : wait dumped[d % 2], copy to host_dumps[d % n_host],
//                   record out_done[d % 2]
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
    uint32_t *d_dump[2] = {nullptr, nullptr};
    hipEvent_t dumped[2] = {nullptr, nullptr}, out_done[2] = {nullptr, nullptr};
    bool out_pending[2] = {false, false};
    std::vector<void *> host;            // caller's host dump buffers
    int64_t n_pushed = 0;                // gulps pushed
    int64_t n_dumps = 0;                 // dumps enqueued
    bool have_slot = false;              // next_slot called, push pending
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
    }
    s->slot_free.assign(s->n_slots, nullptr);
    s->slot_used.assign(s->n_slots, false);
    for (int k = 0; k < s->n_slots; ++k)
        HIP_TRY(hipEventCreateWithFlags(&s->slot_free[k], hipEventDisableTiming));
    s->ev.resize(STREAM_HIST);
    for (GulpEv &g : s->ev) {
        HIP_TRY(hipEventCreate(&g.arrive));
        HIP_TRY(hipEventCreate(&g.ready));
        HIP_TRY(hipEventCreate(&g.done));
    }
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

int xeng_stream_next_slot(xeng_stream *s, void **d_slot, void **ingest_stream)
{
    if (!s || !d_slot) return fail(XENG_EINVAL, "NULL argument");
    const int64_t g = s->n_pushed;
    const int slot = (int)(g % s->n_slots);
    if (!s->have_slot) {
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
    const int64_t g = s->n_pushed;
    const int slot = (int)(g % s->n_slots);
    GulpEv &e = s->ev[g % STREAM_HIST];
    HIP_TRY(hipEventRecord(e.ready, s->s_in));
    HIP_TRY(hipStreamWaitEvent(s->s_comp, e.ready, 0));
    const void *p = s->ring + (size_t)slot * s->gulp_bytes;
    int rc;
    if ((g + 1) % s->dump_every == 0) {
        // the gulp that completes a dump period is correlated and dumped in
        // one call (fused where the kernel allows it)
        const int64_t d = s->n_dumps;
        const int b = (int)(d % 2);
        // the buffer's previous dump (d - 2) must be copied out first
        if (s->out_pending[b]) HIP_TRY(hipStreamWaitEvent(s->s_comp, s->out_done[b], 0));
        void *outp = s->d_dump[b];
        rc = xeng_correlate_dump(s->ctx, &p, &outp, 1, 1);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(s->slot_free[slot], s->s_comp));
        HIP_TRY(hipEventRecord(s->dumped[b], s->s_comp));
        HIP_TRY(hipStreamWaitEvent(s->s_out, s->dumped[b], 0));
        if (!s->host.empty())
            HIP_TRY(hipMemcpyAsync(s->host[d % s->host.size()], s->d_dump[b], s->dump_bytes,
                                   hipMemcpyDeviceToHost, s->s_out));
        HIP_TRY(hipEventRecord(s->out_done[b], s->s_out));
        s->out_pending[b] = true;
        ++s->n_dumps;
    } else {
        rc = xeng_correlate(s->ctx, &p);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(s->slot_free[slot], s->s_comp));
    }
    s->slot_used[slot] = true;
    HIP_TRY(hipEventRecord(e.done, s->s_comp));
    s->have_slot = false;
    ++s->n_pushed;
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

int xeng_stream_gulp_times(xeng_stream *s, int64_t g, float *arrive_ms, float *ready_ms)
{
    if (!s) return fail(XENG_EINVAL, "s is NULL");
    if (g < 0 || g >= s->n_pushed || g < s->n_pushed - STREAM_HIST)
        return fail(XENG_EINVAL, "gulp %lld is not among the last %d pushed", (long long)g,
                    STREAM_HIST);
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
    *out = s->n_pushed;
    return XENG_OK;
}

int xeng_stream_backlog(xeng_stream *s, int64_t *out)
{
    if (!s || !out) return fail(XENG_EINVAL, "NULL argument");
    // gulps whose correlation (and dump) has not finished: done events
    // complete in push order on the compute stream, so count back from the
    // newest until one has completed
    int64_t n = 0;
    const int64_t lo = std::max<int64_t>(0, s->n_pushed - STREAM_HIST);
    for (int64_t g = s->n_pushed - 1; g >= lo; --g) {
        const hipError_t q = hipEventQuery(s->ev[g % STREAM_HIST].done);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) return fail(XENG_EHIP, "hipEventQuery: %s", hipGetErrorString(q));
        ++n;
    }
    *out = n;
    return XENG_OK;
}

int xeng_stream_destroy(xeng_stream *s)
{
    if (!s) return XENG_OK;
    stream_free(s);
    return XENG_OK;
}

} // extern "C"
