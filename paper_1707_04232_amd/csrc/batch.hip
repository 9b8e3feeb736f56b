// Batched replicas: many independent boxes (each its own context and
// stream) advanced together by HIP graphs holding fd_every consecutive steps
// of every box, captured once from the same launch sequence the eager
// sdpd_step issues.  Two layouts:
//   * one graph per stream (the boxes of that stream, replayed on it), when
//     the process has a hardware queue for every stream (GPU_MAX_HW_QUEUES,
//     4 unless set): the streams then run side by side;
//   * otherwise one graph for all boxes, the boxes' streams forked from and
//     joined back into the batch's origin stream with events.
// Either way each box keeps its own launch order, and the F/D sweep is
// captured as one launch per group: boxes that share the GPU would otherwise
// hold workgroup slots while waiting on ranges of their own sweep that are
// descheduled behind the other boxes' work.  The step index of the
// random draws lives on the device: set once per run, advanced by every
// replayed step, so one capture serves every step block.
#include <stdlib.h>

#include <algorithm>
#include <new>
#include <vector>

#include "sdpd_internal.hpp"

struct sdpd_batch {
    std::vector<sdpd_ctx *> ctx;
    std::vector<sdpd_state> st;
    std::vector<int> gen;               // the contexts' tuning at capture
    std::vector<hipStream_t> streams;   // distinct streams of the boxes
    std::vector<hipEvent_t> join, ready;
    hipStream_t origin = nullptr;
    hipEvent_t fork = nullptr, done = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraph_t> sgraph;   // per-stream layout
    std::vector<hipGraphExec_t> sexec;
    int theta = 1;
};

// hardware queues HIP gives the process (its default is 4)
static int hw_queues()
{
    const char *v = getenv("GPU_MAX_HW_QUEUES");
    const int q = v ? atoi(v) : 0;
    return q > 0 ? q : 4;
}

using namespace sdpd;

static void batch_free(sdpd_batch *b)
{
    if (b->origin) (void)hipStreamSynchronize(b->origin);
    for (hipStream_t st : b->streams) (void)hipStreamSynchronize(st);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipGraphExec_t e : b->sexec)
        if (e) (void)hipGraphExecDestroy(e);
    for (hipGraph_t g : b->sgraph)
        if (g) (void)hipGraphDestroy(g);
    for (hipEvent_t e : b->join)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->ready)
        if (e) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->origin) (void)hipStreamDestroy(b->origin);
    delete b;
}

extern "C" {

int sdpd_batch_create(sdpd_ctx *const *ctxs, const sdpd_state *states, int nbox,
                      sdpd_batch **out)
{
    if (!out || !ctxs || !states || nbox < 1) return SDPD_EINVAL;
    *out = nullptr;
    const int theta = ctxs[0] ? ctxs[0]->prm.fd_every : 0;
    for (int k = 0; k < nbox; ++k) {
        const sdpd_ctx *c = ctxs[k];
        if (!c || !c->cells_valid || c->timing || c->prm.fd_every != theta ||
            c->device != ctxs[0]->device || c->stream == nullptr)
            return SDPD_EINVAL;   // the null stream cannot join a capture
        const sdpd_state &s = states[k];
        if (c->n > 0 && (!s.q || !s.p || !s.eps || !s.rho || !s.f || !s.id)) return SDPD_EINVAL;
        for (int j = 0; j < k; ++j)
            if (ctxs[j] == c) return SDPD_EINVAL;   // a box appears once
    }
    sdpd_batch *b = new (std::nothrow) sdpd_batch();
    if (!b) return SDPD_ENOMEM;
    b->ctx.assign(ctxs, ctxs + nbox);
    b->st.assign(states, states + nbox);
    for (sdpd_ctx *c : b->ctx) b->gen.push_back(c->tune_gen);
    b->theta = theta;
    for (sdpd_ctx *c : b->ctx)
        if (std::find(b->streams.begin(), b->streams.end(), c->stream) == b->streams.end())
            b->streams.push_back(c->stream);
    int rc = SDPD_OK;
    if (hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess)
        rc = SDPD_EHIP;
    for (size_t i = 0; !rc && i < b->streams.size(); ++i) {
        hipEvent_t e1 = nullptr, e2 = nullptr;
        if (hipEventCreateWithFlags(&e1, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&e2, hipEventDisableTiming) != hipSuccess)
            rc = SDPD_EHIP;
        b->join.push_back(e1);
        b->ready.push_back(e2);
    }
    // the boxes' pending work finishes before the capture starts
    for (hipStream_t s : b->streams)
        if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = SDPD_EHIP;
    if (rc) {
        batch_free(b);
        return rc;
    }
    if (b->streams.size() > 1 && (int)b->streams.size() <= hw_queues()) {
        // per-stream graphs: each stream captures theta steps of its boxes
        for (size_t i = 0; !rc && i < b->streams.size(); ++i) {
            hipStream_t st = b->streams[i];
            if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                rc = SDPD_EHIP;
                break;
            }
            for (int k = 0; !rc && k < theta; ++k)
                for (int j = 0; !rc && j < nbox; ++j)
                    if (b->ctx[j]->stream == st) {
                        b->ctx[j]->fd_per_group = 1;
                        rc = enqueue_step(b->ctx[j], &b->st[j], (uint64_t)k, false);
                        b->ctx[j]->fd_per_group = 0;
                    }
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(st, &g);
            b->sgraph.push_back(g);
            if (!rc && ec != hipSuccess) rc = SDPD_EHIP;
            hipGraphExec_t e = nullptr;
            if (!rc && hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess)
                rc = SDPD_EHIP;
            b->sexec.push_back(e);
        }
        if (rc) {
            (void)hipGetLastError();
            batch_free(b);
            return rc;
        }
        *out = b;
        return SDPD_OK;
    }
    // one graph: capture theta steps of every box
    if (hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        batch_free(b);
        return SDPD_EHIP;
    }
    rc = check_hip(hipEventRecord(b->fork, b->origin));
    for (hipStream_t s : b->streams)
        if (!rc) rc = check_hip(hipStreamWaitEvent(s, b->fork, 0));
    for (int k = 0; !rc && k < theta; ++k)
        for (int i = 0; !rc && i < nbox; ++i) {
            b->ctx[i]->fd_per_group = 1;
            rc = enqueue_step(b->ctx[i], &b->st[i], (uint64_t)k, false);
            b->ctx[i]->fd_per_group = 0;
        }
    for (size_t i = 0; !rc && i < b->streams.size(); ++i) {
        rc = check_hip(hipEventRecord(b->join[i], b->streams[i]));
        if (!rc) rc = check_hip(hipStreamWaitEvent(b->origin, b->join[i], 0));
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->origin, &g);
    b->graph = g;
    if (!rc && ec != hipSuccess) rc = SDPD_EHIP;
    if (!rc && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
        rc = SDPD_EHIP;
    if (rc) {
        (void)hipGetLastError();
        batch_free(b);
        return rc;
    }
    *out = b;
    return SDPD_OK;
}

int sdpd_batch_run(sdpd_batch *b, uint64_t step0, int nsteps)
{
    if (!b || nsteps < 0 || step0 % (uint64_t)b->theta != 0 || nsteps % b->theta != 0)
        return SDPD_EINVAL;
    for (size_t k = 0; k < b->ctx.size(); ++k)
        if (b->ctx[k]->tune_gen != b->gen[k]) return SDPD_EINVAL;   // retuned since the capture
    if (nsteps == 0) return SDPD_OK;
    int rc;
    for (sdpd_ctx *c : b->ctx)
        if ((rc = launch_fill_u64(c, (unsigned long long *)c->dstep, step0, 1))) return rc;
    if (!b->sexec.empty()) {
        for (int r = 0; r < nsteps / b->theta; ++r)
            for (size_t i = 0; i < b->streams.size(); ++i)
                if ((rc = check_hip(hipGraphLaunch(b->sexec[i], b->streams[i])))) return rc;
        return SDPD_OK;
    }
    for (size_t i = 0; i < b->streams.size(); ++i) {
        if ((rc = check_hip(hipEventRecord(b->ready[i], b->streams[i])))) return rc;
        if ((rc = check_hip(hipStreamWaitEvent(b->origin, b->ready[i], 0)))) return rc;
    }
    for (int r = 0; r < nsteps / b->theta; ++r)
        if ((rc = check_hip(hipGraphLaunch(b->exec, b->origin)))) return rc;
    if ((rc = check_hip(hipEventRecord(b->done, b->origin)))) return rc;
    for (hipStream_t s : b->streams)
        if ((rc = check_hip(hipStreamWaitEvent(s, b->done, 0)))) return rc;
    return SDPD_OK;
}

int sdpd_batch_destroy(sdpd_batch *b)
{
    if (!b) return SDPD_EINVAL;
    batch_free(b);
    return SDPD_OK;
}

}  // extern "C"
