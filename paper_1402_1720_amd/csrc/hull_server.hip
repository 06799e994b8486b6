// Serving loop: requests carry host histories and take masks back to the
// host. One device arena holds every admitted request; worker threads, each
// with its own stream, admit the request at the head of the arrival queue as
// soon as its footprint fits, run copy-in, the per-scan call and copy-out on
// their stream, and release the space, so requests of any size join and
// leave continuously.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hull_host.h"
#include "hull_runtime.h"
#include "hullmi.h"

namespace hullmi {
namespace {

constexpr int kMaxSlots = 64;
constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Ticket {
    hullmi_request req{};
    size_t footprint = 0;
    bool done = false;
    hullmi_result res{};
};

// Device buffers of one admitted request, carved from its arena block in the
// order hull_footprint_bytes counts them.
struct Carve {
    const float *in[8];
    int32_t *N = nullptr, *M = nullptr;
    uint8_t *sc = nullptr, *msc = nullptr, *sm = nullptr, *fmask = nullptr, *bmask = nullptr;
    float *image = nullptr;
    hullmi_stats *stats = nullptr;
    hullmi_bsc_stats *bstats = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    size_t total = 0;
};

Carve carve(char *base, const hullmi_request &r, size_t ws_bytes)
{
    Carve c;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base + off;
        off += align_up(bytes);
        return p;
    };
    const size_t n = (size_t)r.hist.n, V = (size_t)r.grid.nx * r.grid.ny * r.grid.nz;
    for (int a = 0; a < 8; ++a) c.in[a] = reinterpret_cast<const float *>(take(4 * n));
    switch (r.op) {
    case HULL_OP_SC:
        c.N = reinterpret_cast<int32_t *>(take(4 * V));
        c.sc = reinterpret_cast<uint8_t *>(take(V));
        break;
    case HULL_OP_MSC:
        c.N = reinterpret_cast<int32_t *>(take(4 * V));
        c.msc = reinterpret_cast<uint8_t *>(take(V));
        break;
    case HULL_OP_SM:
        c.M = reinterpret_cast<int32_t *>(take(4 * V));
        c.sm = reinterpret_cast<uint8_t *>(take(V));
        break;
    case HULL_OP_ALL:
        c.N = reinterpret_cast<int32_t *>(take(4 * V));
        c.M = reinterpret_cast<int32_t *>(take(4 * V));
        c.sc = reinterpret_cast<uint8_t *>(take(V));
        c.msc = reinterpret_cast<uint8_t *>(take(V));
        c.sm = reinterpret_cast<uint8_t *>(take(V));
        break;
    case HULL_OP_FBP:
    case HULL_OP_FBP_CUT:
        c.image = reinterpret_cast<float *>(take(4 * V));
        c.fmask = reinterpret_cast<uint8_t *>(take(V));
        break;
    case HULL_OP_SC_BINNED:
        c.bmask = reinterpret_cast<uint8_t *>(take(V));
        break;
    }
    c.stats = reinterpret_cast<hullmi_stats *>(take(sizeof(hullmi_stats)));
    c.bstats = reinterpret_cast<hullmi_bsc_stats *>(take(sizeof(hullmi_bsc_stats)));
    c.ws = take(ws_bytes);
    c.ws_bytes = ws_bytes;
    c.total = off;
    return c;
}

hullmi_job job_of(const hullmi_request &r)
{
    hullmi_job j;
    std::memset(&j, 0, sizeof j);
    j.op = r.op;
    j.flags = 0;
    j.hist = r.hist;
    j.grid = r.grid;
    j.params = r.params;
    j.fbp = r.fbp;
    j.bsc = r.bsc;
    return j;
}

}  // namespace
}  // namespace hullmi

using namespace hullmi;

struct hullmi_server {
    int device = 0;
    char *base = nullptr;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Ticket> tickets;
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::vector<std::thread> workers;
    int64_t submitted = 0, completed = 0, failed = 0, running = 0, histories_done = 0;
    int workers_up = 0, workers_ok = 0;   // workers done with set-up / that succeeded

    void worker();
    int process(const hullmi_request &r, char *mem, hipStream_t s, hipEvent_t ev[4],
                hullmi_result *res);
};

int hullmi_server::process(const hullmi_request &r, char *mem, hipStream_t s, hipEvent_t ev[4],
                           hullmi_result *res)
{
    hullmi_job j = job_of(r);
    const size_t n = (size_t)r.hist.n, V = (size_t)r.grid.nx * r.grid.ny * r.grid.nz;
    Carve c = carve(mem, r, job_ws_bytes(j));
    const float *host_in[8] = {r.hist.x_in, r.hist.y_in, r.hist.z_in, r.hist.x_out,
                               r.hist.y_out, r.hist.z_out, r.hist.angle_deg, r.hist.wepl};
    bool ok = hipEventRecord(ev[0], s) == hipSuccess;
    for (int a = 0; a < 8 && ok && n > 0; ++a)
        ok = hipMemcpyAsync(const_cast<float *>(c.in[a]), host_in[a], 4 * n,
                            hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && hipEventRecord(ev[1], s) == hipSuccess;
    if (!ok) {
        // copies enqueued before the failure may still be writing into the
        // block: wait for them before the block goes back to the arena
        (void)hipStreamSynchronize(s);
        return HULL_EDEVICE;
    }
    j.hist.x_in = c.in[0]; j.hist.y_in = c.in[1]; j.hist.z_in = c.in[2];
    j.hist.x_out = c.in[3]; j.hist.y_out = c.in[4]; j.hist.z_out = c.in[5];
    j.hist.angle_deg = c.in[6]; j.hist.wepl = c.in[7];
    j.N = c.N; j.M = c.M; j.sc_mask = c.sc; j.msc_mask = c.msc; j.sm_mask = c.sm;
    j.image = c.image; j.fbp_mask = c.fmask; j.stats = c.stats;
    j.bsc_mask = c.bmask; j.bsc_stats = c.bstats;
    const int rc = job_run(j, c.ws, c.ws_bytes, s, CountOpts{});
    if (rc != HULL_OK) {
        (void)hipStreamSynchronize(s);
        return rc;
    }
    ok = hipEventRecord(ev[2], s) == hipSuccess;
    auto out = [&](void *host, const void *dev, size_t bytes) {
        if (ok && host && dev && bytes)
            ok = hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s) == hipSuccess;
    };
    out(r.N, c.N, 4 * V);
    out(r.M, c.M, 4 * V);
    out(r.sc_mask, c.sc, V);
    out(r.msc_mask, c.msc, V);
    out(r.sm_mask, c.sm, V);
    out(r.image, c.image, 4 * V);
    out(r.fbp_mask, c.fmask, V);
    out(r.bsc_mask, c.bmask, V);
    // each op fills one counter block, or none (the FDK hulls)
    if (r.op <= HULL_OP_ALL) out(&res->stats, c.stats, sizeof(hullmi_stats));
    if (r.op == HULL_OP_SC_BINNED) out(&res->bsc_stats, c.bstats, sizeof(hullmi_bsc_stats));
    ok = ok && hipEventRecord(ev[3], s) == hipSuccess;
    ok = hipStreamSynchronize(s) == hipSuccess && ok;
    if (!ok) return HULL_EDEVICE;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, ev[0], ev[3]) == hipSuccess) res->device_ms = t;
    if (hipEventElapsedTime(&t, ev[0], ev[1]) == hipSuccess) res->h2d_ms = t;
    if (hipEventElapsedTime(&t, ev[1], ev[2]) == hipSuccess) res->compute_ms = t;
    if (hipEventElapsedTime(&t, ev[2], ev[3]) == hipSuccess) res->d2h_ms = t;
    return HULL_OK;
}

void hullmi_server::worker()
{
    hipStream_t s = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool ready = hipSetDevice(device) == hipSuccess &&
                 hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    for (int e = 0; e < 4 && ready; ++e) ready = hipEventCreate(&ev[e]) == hipSuccess;
    std::unique_lock<std::mutex> lk(mu);
    ++workers_up;
    if (ready) ++workers_ok;
    cv_done.notify_all();
    while (ready) {
        cv_work.wait(lk, [&] {
            return stopping ||
                   (!queue.empty() && arena.fits(tickets.at(queue.front()).footprint));
        });
        if (stopping) break;
        const uint64_t id = queue.front();
        queue.pop_front();
        Ticket &tk = tickets.at(id);
        const size_t off = arena.alloc(tk.footprint);
        tk.res.t_admit_ns = now_ns();
        const hullmi_request req = tk.req;
        ++running;
        cv_work.notify_all();   // the next request may fit as well
        lk.unlock();

        hullmi_result res{};
        const int rc = process(req, base + off, s, ev, &res);

        lk.lock();
        arena.release(off);
        --running;
        Ticket &t2 = tickets.at(id);
        res.status = rc;
        res.t_arrive_ns = t2.res.t_arrive_ns;
        res.t_admit_ns = t2.res.t_admit_ns;
        res.t_done_ns = now_ns();
        t2.res = res;
        t2.done = true;
        if (rc == HULL_OK) {
            ++completed;
            histories_done += req.hist.n;
        } else {
            ++failed;
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }
    lk.unlock();
    if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
}

namespace {

bool request_ok(const hullmi_request &r)
{
    hullmi_job j = job_of(r);
    // the outputs of the call live in the server's arena: stand-ins here
    static int32_t i32;
    static uint8_t u8;
    static float f32;
    j.N = j.M = &i32;
    j.sc_mask = j.msc_mask = j.sm_mask = j.fbp_mask = j.bsc_mask = &u8;
    j.image = &f32;
    return job_check(j) == HULL_OK;
}

}  // namespace

extern "C" {

int hull_server_create(size_t hbm_budget, int max_slots, int device, hullmi_server **srv)
{
    if (!srv || hbm_budget == 0 || max_slots < 1 || max_slots > kMaxSlots || device < 0)
        return HULL_EINVAL;
    *srv = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) return HULL_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return HULL_EDEVICE;
    auto *s = new hullmi_server;
    s->device = device;
    const size_t budget = hbm_budget / kAlign * kAlign;
    if (budget == 0 || hipMalloc(reinterpret_cast<void **>(&s->base), budget) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return HULL_ENOMEM;
    }
    s->arena = Arena(budget, kAlign);
    for (int w = 0; w < max_slots; ++w) s->workers.emplace_back([s] { s->worker(); });
    bool all_ok;
    {
        // every worker reports whether it could set up its stream
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->workers_up == max_slots; });
        all_ok = s->workers_ok == max_slots;
    }
    if (!all_ok) {
        hull_server_destroy(s);
        return HULL_EDEVICE;
    }
    *srv = s;
    return HULL_OK;
}

int hull_server_submit(hullmi_server *srv, const hullmi_request *req, uint64_t *ticket)
{
    if (!srv || !req || !ticket) return HULL_EINVAL;
    if (!request_ok(*req)) return HULL_EINVAL;
    const bool bins = req->op == HULL_OP_FBP || req->op == HULL_OP_FBP_CUT ||
                      req->op == HULL_OP_SC_BINNED;
    const size_t fp = footprint_bytes(req->op, &req->grid, req->hist.n, bins ? &req->fbp : nullptr);
    if (fp == (size_t)-1) return HULL_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return HULL_EBUSY;
    if (srv->arena.round(fp) > srv->arena.size()) return HULL_ENOMEM;
    const uint64_t id = srv->next_ticket++;
    Ticket &t = srv->tickets[id];
    t.req = *req;
    t.footprint = fp;
    t.res.t_arrive_ns = now_ns();
    srv->queue.push_back(id);
    ++srv->submitted;
    *ticket = id;
    srv->cv_work.notify_all();
    return HULL_OK;
}

int hull_server_wait(hullmi_server *srv, uint64_t ticket, hullmi_result *result, int64_t timeout_us)
{
    if (!srv || !result) return HULL_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->tickets.find(ticket) == srv->tickets.end()) return HULL_EINVAL;
    // done, or retired by another waiter meanwhile
    auto settled = [&] {
        auto it = srv->tickets.find(ticket);
        return it == srv->tickets.end() || it->second.done;
    };
    if (timeout_us < 0) {
        srv->cv_done.wait(lk, settled);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), settled)) {
        return HULL_ETIMEDOUT;
    }
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return HULL_EINVAL;
    *result = it->second.res;
    srv->tickets.erase(it);
    return HULL_OK;
}

int hull_server_stats(hullmi_server *srv, hullmi_server_stats *out)
{
    if (!srv || !out) return HULL_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->failed = srv->failed;
    out->queued = (int64_t)srv->queue.size();
    out->running = srv->running;
    out->histories_done = srv->histories_done;
    out->bytes_budget = srv->arena.size();
    out->bytes_in_use = srv->arena.in_use();
    out->bytes_peak = srv->arena.peak();
    return HULL_OK;
}

int hull_server_destroy(hullmi_server *srv)
{
    if (!srv) return HULL_OK;
    {
        // queued requests are dropped: they settle with HULL_EBUSY
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
        for (uint64_t id : srv->queue) {
            Ticket &t = srv->tickets.at(id);
            t.res.status = HULL_EBUSY;
            t.done = true;
        }
        srv->queue.clear();
    }
    srv->cv_work.notify_all();
    srv->cv_done.notify_all();
    for (auto &t : srv->workers) t.join();
    (void)hipSetDevice(srv->device);
    if (srv->base) (void)hipFree(srv->base);
    delete srv;
    return HULL_OK;
}

}  // extern "C"
