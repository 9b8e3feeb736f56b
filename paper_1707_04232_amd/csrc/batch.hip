// Batched replicas: many independent boxes (each its own context and
// stream) advanced together by HIP graphs holding fd_every consecutive steps
// of every box.
//
// Fused layout (the default): every stage of the step runs for all boxes in
// one launch.  Each box's contexts records the launches its eager step would
// issue (kernel, grid, LDS, argument struct); position k of every box's
// sequence becomes one multi-box launch per distinct kernel at that position,
// whose workgroups are the boxes' workgroups, each reading its box's
// argument struct from a device table.  A box's launches stay in their order
// and keep their grids, so each box computes exactly what its eager step
// computes, bit for bit; a step of 256 boxes is ~50 launches instead of
// ~13,000.  The boxes are dealt into a few parts of about equal particle
// count (largest first); each part's launch sequence for fd_every steps is
// captured in a graph of its own on a stream of its own, so that one part's
// launches fill the GPU while another's drain (the launch of a sweep group
// ends with its slowest task range).
//
// Graph layouts (the previous one, selectable): the launch sequence of
// each box captured as it is:
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

namespace {

// one multi-box launch of the fused layout
struct FusedLaunch {
    sdpd::MultiKernel multi = nullptr;
    unsigned block = 0, nblocks = 0;
    size_t lds = 0;
    void *tab = nullptr;   // device: argument structs of the participating boxes
    uint2 *wg = nullptr;   // device: (slot in tab, workgroup of that box)
    bool is_flow = false;  // instead: the one-launch F/D sweep of the boxes
    sdpd::FlowSweep flow;
};

// boxes advanced by one sequence of multi-box launches on one stream
struct FusedPart {
    std::vector<int> boxes;
    std::vector<FusedLaunch> launches;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
};

}  // namespace

struct sdpd_batch {
    int layout = SDPD_BATCH_GRAPHS;
    bool flow = false;   // fused layout with one sweep launch for all boxes of a part
    std::vector<FusedPart> parts;
    unsigned long long **dsteps = nullptr;   // device: each box's step-index word
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
    for (FusedPart &p : b->parts) {
        if (p.stream) (void)hipStreamSynchronize(p.stream);
        for (FusedLaunch &f : p.launches) {
            if (f.tab) (void)hipFree(f.tab);
            if (f.wg) (void)hipFree(f.wg);
            fd_flow_free(f.flow);
        }
        if (p.exec) (void)hipGraphExecDestroy(p.exec);
        if (p.graph) (void)hipGraphDestroy(p.graph);
        if (p.done) (void)hipEventDestroy(p.done);
        if (p.stream) (void)hipStreamDestroy(p.stream);
    }
    if (b->dsteps) (void)hipFree(b->dsteps);
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

// every box's step-index word set to v (one launch)
__global__ void k_set_steps(unsigned long long *const *dsteps, int nbox, unsigned long long v)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < nbox) *dsteps[i] = v;
}

// Record theta steps of every box, deal the boxes into parts and merge each
// part's records into multi-box launches (see the header of this file).
static int build_fused(sdpd_batch *b, int nparts)
{
    const int nbox = (int)b->ctx.size();
    std::vector<LaunchRecord> recs(nbox);
    int rc = SDPD_OK;
    for (int i = 0; i < nbox && !rc; ++i) {
        sdpd_ctx *c = b->ctx[i];
        c->rec = &recs[i];
        c->fd_per_group = 1;
        c->fd_record_flow = b->flow ? 1 : 0;
        for (int k = 0; k < b->theta && !rc; ++k) rc = enqueue_step(c, &b->st[i], (uint64_t)k, false);
        c->fd_per_group = 0;
        c->fd_record_flow = 0;
        c->rec = nullptr;
    }
    if (rc) return rc;
    // parts of about equal particle count: largest box first to the lightest part
    nparts = std::max(1, std::min(nparts, nbox));
    std::vector<int> order(nbox);
    for (int i = 0; i < nbox; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->ctx[x]->n > b->ctx[y]->n; });
    b->parts.resize(nparts);
    std::vector<int64_t> load(nparts, 0);
    for (int i : order) {
        const int p = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        b->parts[p].boxes.push_back(i);
        load[p] += std::max<int64_t>(b->ctx[i]->n, 1);
    }
    for (FusedPart &part : b->parts) {
        std::sort(part.boxes.begin(), part.boxes.end());
        size_t maxlen = 0;
        for (int i : part.boxes) maxlen = std::max(maxlen, recs[i].size());
        for (size_t pos = 0; pos < maxlen; ++pos) {
            // boxes with the same kernel at this position share one launch
            using Key = std::pair<MultiKernel, int>;   // (kernel, kind of a flow sweep)
            std::vector<Key> kinds;
            for (int i : part.boxes)
                if (pos < recs[i].size()) {
                    const Key k(recs[i][pos].multi, recs[i][pos].flow_kind);
                    if (std::find(kinds.begin(), kinds.end(), k) == kinds.end()) kinds.push_back(k);
                }
            for (const Key &key : kinds) {
                const MultiKernel kind = key.first;
                if (key.second >= 0) {   // the boxes' F/D sweeps as one launch
                    std::vector<sdpd_ctx *> cs;
                    std::vector<const RecordedLaunch *> rs;
                    for (int i : part.boxes)
                        if (pos < recs[i].size() && recs[i][pos].flow_kind == key.second) {
                            cs.push_back(b->ctx[i]);
                            rs.push_back(&recs[i][pos]);
                        }
                    part.launches.push_back(FusedLaunch());   // freed with the batch from here on
                    FusedLaunch &g = part.launches.back();
                    g.is_flow = true;
                    if ((rc = fd_flow_build(cs, rs, g.flow))) return rc;
                    continue;
                }
                FusedLaunch f;
                f.multi = kind;
                std::vector<unsigned char> tab;
                std::vector<uint2> wg;
                unsigned slot = 0;
                for (int i : part.boxes) {
                    if (pos >= recs[i].size() || recs[i][pos].multi != kind ||
                        recs[i][pos].flow_kind >= 0)
                        continue;
                    const RecordedLaunch &r = recs[i][pos];
                    if (f.block && r.block != f.block) return SDPD_EINVAL;
                    f.block = r.block;
                    f.lds = std::max(f.lds, r.lds);
                    tab.insert(tab.end(), r.args.begin(), r.args.end());
                    for (unsigned blk = 0; blk < r.grid; ++blk) wg.push_back(make_uint2(slot, blk));
                    ++slot;
                }
                if (wg.empty()) continue;
                if (wg.size() > 0x7fffffffull) return SDPD_EINVAL;
                f.nblocks = (unsigned)wg.size();
                part.launches.push_back(f);   // freed with the batch from here on
                FusedLaunch &g = part.launches.back();
                if (hipMalloc(&g.tab, tab.size()) != hipSuccess) return SDPD_ENOMEM;
                if (hipMalloc((void **)&g.wg, sizeof(uint2) * wg.size()) != hipSuccess)
                    return SDPD_ENOMEM;
                if ((rc = check_hip(hipMemcpy(g.tab, tab.data(), tab.size(),
                                              hipMemcpyHostToDevice))) ||
                    (rc = check_hip(hipMemcpy(g.wg, wg.data(), sizeof(uint2) * wg.size(),
                                              hipMemcpyHostToDevice))))
                    return rc;
            }
        }
    }
    std::vector<unsigned long long *> ds(nbox);
    for (int i = 0; i < nbox; ++i) ds[i] = (unsigned long long *)b->ctx[i]->dstep;
    if (hipMalloc((void **)&b->dsteps, sizeof(void *) * nbox) != hipSuccess) return SDPD_ENOMEM;
    return check_hip(hipMemcpy(b->dsteps, ds.data(), sizeof(void *) * nbox, hipMemcpyHostToDevice));
}

// capture each part's fused launches of theta steps into a graph on its stream
static int capture_fused(sdpd_batch *b)
{
    for (FusedPart &part : b->parts) {
        if (hipStreamCreateWithFlags(&part.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&part.done, hipEventDisableTiming) != hipSuccess)
            return SDPD_EHIP;
        if (hipStreamBeginCapture(part.stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return SDPD_EHIP;
        int rc = SDPD_OK;
        for (const FusedLaunch &f : part.launches) {
            if (f.is_flow) {
                const int r = fd_flow_launch(f.flow, part.stream);
                rc = rc ? rc : r;
                continue;
            }
            hipLaunchKernelGGL(f.multi, dim3(f.nblocks), dim3(f.block), f.lds, part.stream,
                               (const void *)f.tab, (const uint2 *)f.wg);
        }
        const int rl = check_hip(hipGetLastError());
        rc = rc ? rc : rl;
        const hipError_t ec = hipStreamEndCapture(part.stream, &part.graph);
        if (!rc && ec != hipSuccess) rc = SDPD_EHIP;
        if (!rc && hipGraphInstantiate(&part.exec, part.graph, nullptr, nullptr, 0) != hipSuccess)
            rc = SDPD_EHIP;
        if (rc) return rc;
    }
    return SDPD_OK;
}

extern "C" {

int sdpd_batch_create(sdpd_ctx *const *ctxs, const sdpd_state *states, int nbox,
                      sdpd_batch **out)
{
    return sdpd_batch_create_layout(ctxs, states, nbox, SDPD_BATCH_AUTO, 0, out);
}

int sdpd_batch_layout(const sdpd_batch *b)
{
    return b ? b->layout : SDPD_EINVAL;
}

int sdpd_batch_create_layout(sdpd_ctx *const *ctxs, const sdpd_state *states, int nbox,
                             int layout, int parts, sdpd_batch **out)
{
    if (!out || !ctxs || !states || nbox < 1) return SDPD_EINVAL;
    *out = nullptr;
    if (layout < SDPD_BATCH_AUTO || layout > SDPD_BATCH_FUSED_FLOW) return SDPD_EINVAL;
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
    if (layout != SDPD_BATCH_GRAPHS) {
        b->layout = layout == SDPD_BATCH_FUSED_FLOW ? SDPD_BATCH_FUSED_FLOW : SDPD_BATCH_FUSED;
        b->flow = b->layout == SDPD_BATCH_FUSED_FLOW;
        rc = build_fused(b, parts > 0 ? parts : std::min(hw_queues(), 16));
        if (!rc) rc = capture_fused(b);
        if (rc) {
            (void)hipGetLastError();
            batch_free(b);
            return rc;
        }
        *out = b;
        return SDPD_OK;
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
    if (b->layout != SDPD_BATCH_GRAPHS) {
        // the boxes' earlier work first, then everything on the batch's stream
        for (size_t i = 0; i < b->streams.size(); ++i) {
            if ((rc = check_hip(hipEventRecord(b->ready[i], b->streams[i])))) return rc;
            if ((rc = check_hip(hipStreamWaitEvent(b->origin, b->ready[i], 0)))) return rc;
        }
        const int nbox = (int)b->ctx.size();
        hipLaunchKernelGGL(k_set_steps, dim3((unsigned)((nbox + 255) / 256)), dim3(256), 0,
                           b->origin, b->dsteps, nbox, (unsigned long long)step0);
        if ((rc = check_hip(hipGetLastError()))) return rc;
        if ((rc = check_hip(hipEventRecord(b->fork, b->origin)))) return rc;
        for (FusedPart &part : b->parts) {
            if ((rc = check_hip(hipStreamWaitEvent(part.stream, b->fork, 0)))) return rc;
            for (int r = 0; r < nsteps / b->theta; ++r)
                if ((rc = check_hip(hipGraphLaunch(part.exec, part.stream)))) return rc;
            if ((rc = check_hip(hipEventRecord(part.done, part.stream)))) return rc;
            if ((rc = check_hip(hipStreamWaitEvent(b->origin, part.done, 0)))) return rc;
        }
        if ((rc = check_hip(hipEventRecord(b->done, b->origin)))) return rc;
        for (hipStream_t s : b->streams)
            if ((rc = check_hip(hipStreamWaitEvent(s, b->done, 0)))) return rc;
        return SDPD_OK;
    }
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
