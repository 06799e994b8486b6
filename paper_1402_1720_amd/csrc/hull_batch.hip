// Batches of scans: a plan spreads independent per-scan calls over internal
// streams (longest first onto the least loaded stream), gives every stream a
// workspace of its own and, when asked, captures the fork/join of the whole
// batch into a HIP graph on the first launch and replays it afterwards.
// Untuned plans take their launch choices from a per-process cache filled by
// timing a few candidates on the batch itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hull_host.h"
#include "hull_runtime.h"
#include "hullmi.h"

struct hullmi_plan {
    int device = 0;
    std::vector<hullmi_job> jobs;
    hullmi_tuning tuning{};
    std::vector<int> job_stream;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> joins;
    std::vector<void *> ws;
    std::vector<size_t> ws_bytes;
    hipStream_t capture = nullptr;
    hipEvent_t fork = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace hullmi {
namespace {

constexpr int kMaxStreams = 16;

// Relative cost of a job for the stream assignment: walk steps grow with the
// histories times the in-plane extent; the epilogue and FDK backprojection
// with the voxels; the binned SC with its histories (three record passes)
// and its carve lines (one per bin, each about the in-plane extent long).
double job_cost(const hullmi_job &j)
{
    const double n = (double)j.hist.n;
    const double V = (double)j.grid.nx * j.grid.ny * j.grid.nz;
    const double bins = (double)j.fbp.nu * j.fbp.nv * j.fbp.n_angles;
    switch (j.op) {
    case HULL_OP_FBP: return n * 4.0 + V * (double)j.fbp.n_angles / 8.0;
    case HULL_OP_FBP_CUT: return n * 16.0 + V * (double)j.fbp.n_angles / 8.0;
    case HULL_OP_SC_BINNED: return n * 12.0 + bins * 0.5 * (j.grid.nx + j.grid.ny) / 4.0 + V;
    default: return n * 0.5 * (j.grid.nx + j.grid.ny) + V;
    }
}

void free_plan(hullmi_plan *p)
{
    if (!p) return;
    for (hipStream_t s : p->streams) (void)hipStreamSynchronize(s);
    if (p->capture) (void)hipStreamSynchronize(p->capture);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (void *w : p->ws)
        if (w) (void)hipFree(w);
    for (hipEvent_t e : p->joins) (void)hipEventDestroy(e);
    if (p->fork) (void)hipEventDestroy(p->fork);
    for (hipStream_t s : p->streams) (void)hipStreamDestroy(s);
    if (p->capture) (void)hipStreamDestroy(p->capture);
    delete p;
}

int build_plan(const hullmi_job *jobs, int n_jobs, const hullmi_tuning &t, hullmi_plan **out)
{
    auto *p = new hullmi_plan;
    p->jobs.assign(jobs, jobs + n_jobs);
    p->tuning = t;
    p->tuning.streams = std::max(1, std::min({t.streams, kMaxStreams, std::max(1, n_jobs)}));
    if (hipGetDevice(&p->device) != hipSuccess) { free_plan(p); return HULL_EDEVICE; }
    const int S = p->tuning.streams;
    std::vector<double> cost(n_jobs);
    for (int j = 0; j < n_jobs; ++j) cost[j] = job_cost(jobs[j]);
    p->job_stream = assign_streams(cost, S);
    p->ws.assign(S, nullptr);
    p->ws_bytes.assign(S, 0);
    for (int j = 0; j < n_jobs; ++j) {
        const int s = p->job_stream[j];
        p->ws_bytes[s] = std::max(p->ws_bytes[s], job_ws_bytes(jobs[j]));
    }
    for (int s = 0; s < S; ++s) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            free_plan(p);
            return HULL_EDEVICE;
        }
        p->streams.push_back(st);
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            free_plan(p);
            return HULL_EDEVICE;
        }
        p->joins.push_back(ev);
        if (p->ws_bytes[s] > 0 && hipMalloc(&p->ws[s], p->ws_bytes[s]) != hipSuccess) {
            (void)hipGetLastError();
            p->ws[s] = nullptr;
            free_plan(p);
            return HULL_ENOMEM;
        }
    }
    if (hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) != hipSuccess) {
        free_plan(p);
        return HULL_EDEVICE;
    }
    *out = p;
    return HULL_OK;
}

// Fork from `origin` to every internal stream, the jobs, join back.
int enqueue(hullmi_plan *p, hipStream_t origin)
{
    if (hipEventRecord(p->fork, origin) != hipSuccess) return HULL_EDEVICE;
    for (hipStream_t s : p->streams)
        if (hipStreamWaitEvent(s, p->fork, 0) != hipSuccess) return HULL_EDEVICE;
    for (size_t j = 0; j < p->jobs.size(); ++j) {
        const int s = p->job_stream[j];
        CountOpts o;
        o.walk_blocks = p->tuning.walk_blocks;
        o.ranges_per_group = p->tuning.ranges_per_group;
        o.length_classes = p->tuning.length_classes;
        o.run_stride = p->tuning.run_stride;
        const int rc = job_run(p->jobs[j], p->ws[s], p->ws_bytes[s], p->streams[s], o);
        if (rc != HULL_OK) return rc;
    }
    for (size_t s = 0; s < p->streams.size(); ++s) {
        if (hipEventRecord(p->joins[s], p->streams[s]) != hipSuccess) return HULL_EDEVICE;
        if (hipStreamWaitEvent(origin, p->joins[s], 0) != hipSuccess) return HULL_EDEVICE;
    }
    return HULL_OK;
}

int capture(hullmi_plan *p)
{
    if (hipStreamBeginCapture(p->capture, hipStreamCaptureModeRelaxed) != hipSuccess)
        return HULL_EDEVICE;
    const int rc = enqueue(p, p->capture);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->capture, &g);
    if (rc != HULL_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return rc != HULL_OK ? rc : HULL_EDEVICE;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return HULL_EDEVICE;
    }
    p->graph = g;
    p->exec = x;
    return HULL_OK;
}

int launch(hullmi_plan *p, hipStream_t s)
{
    if (!p->tuning.use_graph) return enqueue(p, s);
    if (!p->exec) {
        const int rc = capture(p);
        if (rc != HULL_OK) return rc;
    }
    return hipGraphLaunch(p->exec, s) == hipSuccess ? HULL_OK : HULL_EDEVICE;
}

// ---- autotuning ----

std::mutex g_cache_mu;
std::map<std::string, hullmi_tuning> g_cache;

std::string shape_key(int device, const hullmi_job *jobs, int n)
{
    std::string k = std::to_string(device) + ":";
    char buf[96];
    for (int j = 0; j < n; ++j) {
        const int lg = jobs[j].hist.n > 0 ? (int)std::log2((double)jobs[j].hist.n) : -1;
        std::snprintf(buf, sizeof buf, "%d/%dx%dx%d/%d;", jobs[j].op, jobs[j].grid.nx,
                      jobs[j].grid.ny, jobs[j].grid.nz, lg);
        k += buf;
    }
    return k;
}

hullmi_tuning default_tuning(int n_jobs)
{
    hullmi_tuning t{};
    t.streams = std::max(1, std::min(4, n_jobs));
    t.use_graph = 1;
    return t;
}

bool tuning_ok(const hullmi_tuning &t)
{
    return t.streams >= 1 && t.streams <= kMaxStreams && t.walk_blocks >= 0 &&
           (t.use_graph == 0 || t.use_graph == 1) && t.ranges_per_group >= 0 &&
           t.ranges_per_group <= 64 && t.length_classes >= 0 && t.length_classes <= 16 &&
           t.run_stride >= 0 && t.run_stride <= 256;
}

// The byte ranges a job reads (its histories) and writes (the outputs its op
// fills), for the check that the jobs of a plan do not race.
void job_spans(const hullmi_job &j, int idx, std::vector<Span> &out)
{
    const uintptr_t n4 = 4 * (uintptr_t)j.hist.n;
    const uintptr_t V = (uintptr_t)j.grid.nx * j.grid.ny * j.grid.nz;
    auto add = [&](const void *p, uintptr_t bytes, bool w) {
        if (p && bytes) out.push_back(Span{(uintptr_t)p, (uintptr_t)p + bytes, idx, w});
    };
    const float *in[8] = {j.hist.x_in, j.hist.y_in, j.hist.z_in, j.hist.x_out,
                          j.hist.y_out, j.hist.z_out, j.hist.angle_deg, j.hist.wepl};
    for (const float *p : in) add(p, n4, false);
    const bool counting = j.op == HULL_OP_SC || j.op == HULL_OP_MSC || j.op == HULL_OP_SM ||
                          j.op == HULL_OP_ALL;
    if (j.op == HULL_OP_SC || j.op == HULL_OP_MSC || j.op == HULL_OP_ALL) add(j.N, 4 * V, true);
    if (j.op == HULL_OP_SM || j.op == HULL_OP_ALL) add(j.M, 4 * V, true);
    if (j.op == HULL_OP_SC || j.op == HULL_OP_ALL) add(j.sc_mask, V, true);
    if (j.op == HULL_OP_MSC || j.op == HULL_OP_ALL) add(j.msc_mask, V, true);
    if (j.op == HULL_OP_SM || j.op == HULL_OP_ALL) add(j.sm_mask, V, true);
    if (counting) add(j.stats, sizeof(hullmi_stats), true);
    if (j.op == HULL_OP_FBP || j.op == HULL_OP_FBP_CUT) {
        add(j.image, 4 * V, true);
        add(j.fbp_mask, V, true);
    }
    if (j.op == HULL_OP_SC_BINNED) {
        add(j.bsc_mask, V, true);
        add(j.bsc_stats, sizeof(hullmi_bsc_stats), true);
    }
}

// Median time of five launches after one untimed launch (which also
// captures): the median keeps one slow launch from deciding the choice.
int time_tuning(const hullmi_job *jobs, int n, const hullmi_tuning &t, hipStream_t s, float *ms)
{
    constexpr int kReps = 5;
    hullmi_plan *p = nullptr;
    int rc = build_plan(jobs, n, t, &p);
    if (rc != HULL_OK) return rc;
    hipEvent_t ev[kReps + 1] = {};
    rc = HULL_OK;
    for (int r = 0; r <= kReps && rc == HULL_OK; ++r)
        if (hipEventCreate(&ev[r]) != hipSuccess) rc = HULL_EDEVICE;
    if (rc == HULL_OK) rc = launch(p, s);
    for (int r = 0; r < kReps && rc == HULL_OK; ++r) {
        if (hipEventRecord(ev[r], s) != hipSuccess) rc = HULL_EDEVICE;
        if (rc == HULL_OK) rc = launch(p, s);
    }
    if (rc == HULL_OK && hipEventRecord(ev[kReps], s) != hipSuccess) rc = HULL_EDEVICE;
    if (rc == HULL_OK && hipEventSynchronize(ev[kReps]) != hipSuccess) rc = HULL_EDEVICE;
    float t_ms[kReps] = {};
    for (int r = 0; r < kReps && rc == HULL_OK; ++r)
        if (hipEventElapsedTime(&t_ms[r], ev[r], ev[r + 1]) != hipSuccess) rc = HULL_EDEVICE;
    if (rc == HULL_OK) {
        std::sort(t_ms, t_ms + kReps);
        *ms = t_ms[kReps / 2];
    }
    (void)hipStreamSynchronize(s);
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    free_plan(p);
    return rc;
}

// Coordinate search over the launch choices, timed on the batch itself:
// streams x graph first, then one knob of the counting pass at a time
// (ranges per walk workgroup, the walk grid cap, length classes, run
// stride), each kept only when it beats the best so far by more than 1%.
int autotune(const hullmi_job *jobs, int n, hullmi_tuning *best)
{
    *best = default_tuning(n);
    for (int j = 0; j < n; ++j)
        if (jobs[j].flags & HULL_ACCUMULATE) return HULL_OK;   // timing runs would add up
    bool counting = false;
    for (int j = 0; j < n; ++j)
        counting |= jobs[j].op == HULL_OP_SC || jobs[j].op == HULL_OP_MSC ||
                    jobs[j].op == HULL_OP_SM || jobs[j].op == HULL_OP_ALL;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return HULL_EDEVICE;
    float best_ms = INFINITY;
    int rc = HULL_OK;
    auto consider = [&](const hullmi_tuning &t, float margin) {
        float ms = 0.0f;
        rc = time_tuning(jobs, n, t, s, &ms);
        if (rc == HULL_OK && ms < best_ms * margin) {
            best_ms = ms;
            *best = t;
        }
        return rc == HULL_OK;
    };
    for (int streams : {1, 2, 4, 8}) {
        if (streams > 1 && streams > n) break;
        for (int graph : {0, 1}) {
            hullmi_tuning t{};
            t.streams = streams;
            t.use_graph = graph;
            if (!consider(t, 1.0f)) break;
        }
        if (rc != HULL_OK) break;
    }
    if (rc == HULL_OK && counting) {
        for (int v : {2, 4, 8}) {
            hullmi_tuning t = *best;
            t.ranges_per_group = v;
            if (!consider(t, 0.99f)) break;
        }
        for (int v : {128, 256}) {
            hullmi_tuning t = *best;
            t.walk_blocks = v;
            if (rc != HULL_OK || !consider(t, 0.99f)) break;
        }
        for (int v : {8}) {
            hullmi_tuning t = *best;
            t.length_classes = v;
            if (rc != HULL_OK || !consider(t, 0.99f)) break;
        }
        for (int v : {4, 16, 64}) {
            hullmi_tuning t = *best;
            t.run_stride = v;
            if (rc != HULL_OK || !consider(t, 0.99f)) break;
        }
    }
    (void)hipStreamDestroy(s);
    return rc;
}

}  // namespace
}  // namespace hullmi

using namespace hullmi;

extern "C" {

int hull_batch_plan(const hullmi_job *jobs, int n_jobs, const hullmi_tuning *tuning,
                    hullmi_plan **plan)
{
    if (!plan || n_jobs < 0 || (n_jobs > 0 && !jobs)) return HULL_EINVAL;
    *plan = nullptr;
    for (int j = 0; j < n_jobs; ++j)
        if (job_check(jobs[j]) != HULL_OK) return HULL_EINVAL;
    // jobs may run concurrently on different streams: none may write what
    // another reads or writes
    std::vector<Span> spans;
    for (int j = 0; j < n_jobs; ++j) job_spans(jobs[j], j, spans);
    if (spans_conflict(spans)) return HULL_EINVAL;
    hullmi_tuning t;
    if (tuning) {
        if (!tuning_ok(*tuning)) return HULL_EINVAL;
        t = *tuning;
    } else {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return HULL_EDEVICE;
        const std::string key = shape_key(dev, jobs, n_jobs);
        bool hit = false;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_cache.find(key);
            if (it != g_cache.end()) {
                t = it->second;
                hit = true;
            }
        }
        if (!hit) {
            const int rc = autotune(jobs, n_jobs, &t);
            if (rc != HULL_OK) return rc;
            std::lock_guard<std::mutex> lk(g_cache_mu);
            g_cache[key] = t;
        }
    }
    return build_plan(jobs, n_jobs, t, plan);
}

int hull_batch_launch(hullmi_plan *plan, void *stream)
{
    if (!plan) return HULL_EINVAL;
    return launch(plan, reinterpret_cast<hipStream_t>(stream));
}

int hull_batch_tuning(const hullmi_plan *plan, hullmi_tuning *out)
{
    if (!plan || !out) return HULL_EINVAL;
    *out = plan->tuning;
    return HULL_OK;
}

int hull_batch_destroy(hullmi_plan *plan)
{
    free_plan(plan);
    return HULL_OK;
}

}  // extern "C"
