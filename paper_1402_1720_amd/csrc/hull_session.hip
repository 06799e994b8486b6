// Sessions: counts kept resident on the device while chunks of histories
// arrive, masks computed on demand (hull_session_* in hullmi.h).
//
// Pushed chunks are appended to one of two device buffers (structure of
// arrays, `cap` histories each) on the session's copy stream; a full buffer
// is counted on the compute stream while the next chunks fill the other one,
// and a read counts what the current buffer holds. A counting pass has a fixed
// cost of a few hundred microseconds whatever its size, so counting buffers
// of millions of histories instead of every chunk keeps the session's rate
// close to that of one call over the whole scan. Events order the two streams:
// a buffer is refilled only after its last count, and counted only after its
// copies have landed. Both streams have the default priority.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "hull_runtime.h"
#include "hullmi.h"

namespace {

// The eight arrays of a chunk as the device reads them.
struct Src8 {
    const float *p[8];
};

// Appends n histories to a buffer of eight arrays `stride` floats apart:
// one launch for the whole chunk, reading device memory or pinned host
// memory mapped into the device's address space.
__global__ void __launch_bounds__(256) k_session_append(Src8 src, int64_t n, float *dst,
                                                        int64_t stride)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
#pragma unroll
        for (int f = 0; f < 8; ++f) dst[(int64_t)f * stride + i] = src.p[f][i];
    }
}

// The device address of p when the device can read it directly (device
// memory, or pinned host memory mapped for the device), else null.
const float *device_view(const float *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();   // pageable host memory is unknown to HIP
        return nullptr;
    }
    if (a.type == hipMemoryTypeDevice) return p;
    if (a.type == hipMemoryTypeHost && a.devicePointer) return static_cast<const float *>(a.devicePointer);
    return nullptr;
}

constexpr size_t kAlign = 256;
constexpr int64_t kSessionBatch = int64_t(1) << 22;   // histories counted at once (at least)
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Makes `dev` current for the lifetime of the guard, then restores the
// caller's device.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct hullmi_session {
    int device = 0;
    hullmi_grid grid{};
    hullmi_params params{};
    int64_t max_chunk = 0, cap = 0, V = 0;
    hipStream_t compute = nullptr, copy = nullptr;
    char *mem = nullptr;                 // one device allocation holds everything below
    int32_t *N = nullptr, *M = nullptr;
    hullmi_stats *stats = nullptr;
    uint8_t *masks = nullptr;            // sc, msc, sm
    void *ws = nullptr;                  // counting workspace for cap histories, then the rules'
    size_t count_ws = 0, ws_bytes = 0;
    float *buf[2] = {nullptr, nullptr};  // 8 arrays of cap floats each
    int64_t fill[2] = {0, 0};
    hipEvent_t counted[2] = {nullptr, nullptr}, copied[2] = {nullptr, nullptr};
    int cur = 0;
    std::mutex mu;                       // calls on one session serialise
};

namespace {

int session_status(hipError_t e) { return e == hipSuccess ? HULL_OK : HULL_EDEVICE; }

float *field(hullmi_session *s, int k, int f) { return s->buf[k] + (int64_t)f * s->cap; }

// Counts buffer k (after its copies) and marks it free again once counted.
int flush(hullmi_session *s, int k)
{
    if (s->fill[k] == 0) return HULL_OK;
    if (hipStreamWaitEvent(s->compute, s->copied[k], 0) != hipSuccess) return HULL_EDEVICE;
    hullmi_histories h{field(s, k, 0), field(s, k, 1), field(s, k, 2), field(s, k, 3),
                       field(s, k, 4), field(s, k, 5), field(s, k, 6), field(s, k, 7), s->fill[k]};
    const int rc = hullmi::counts_accumulate(&h, &s->grid, &s->params, s->N, s->M, s->stats, s->ws,
                                             s->count_ws, s->compute);
    if (rc != HULL_OK) return rc;
    if (hipEventRecord(s->counted[k], s->compute) != hipSuccess) return HULL_EDEVICE;
    s->fill[k] = 0;
    return HULL_OK;
}

void session_free(hullmi_session *s)
{
    if (!s) return;
    if (s->compute) (void)hipStreamSynchronize(s->compute);
    if (s->copy) (void)hipStreamSynchronize(s->copy);
    for (int k = 0; k < 2; ++k) {
        if (s->counted[k]) (void)hipEventDestroy(s->counted[k]);
        if (s->copied[k]) (void)hipEventDestroy(s->copied[k]);
    }
    if (s->mem) (void)hipFree(s->mem);
    if (s->compute) (void)hipStreamDestroy(s->compute);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    delete s;
}

}  // namespace

extern "C" {

int hull_session_create(const hullmi_grid *grid, const hullmi_params *params, int64_t max_chunk,
                        int device, hullmi_session **out)
{
    if (!out) return HULL_EINVAL;
    *out = nullptr;
    if (!hullmi::grid_valid(grid) || !hullmi::params_ok(params) || max_chunk < 1 ||
        max_chunk > INT32_MAX)
        return HULL_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HULL_EINVAL;
    DeviceGuard guard(device);
    if (!guard.ok) return HULL_EDEVICE;
    auto *s = new hullmi_session;
    s->device = device;
    s->grid = *grid;
    s->params = *params;
    s->max_chunk = max_chunk;
    s->cap = std::max<int64_t>(max_chunk, kSessionBatch);
    s->V = (int64_t)grid->nx * grid->ny * grid->nz;
    s->count_ws = align_up(hullmi::counting_ws_bytes(grid, s->cap));
    s->ws_bytes = s->count_ws + align_up(hullmi::rules_ws_bytes(grid));
    const size_t bufb = align_up((size_t)s->cap * 8 * sizeof(float));
    const size_t total = 2 * align_up((size_t)s->V * 4) + align_up(sizeof(hullmi_stats)) +
                         align_up((size_t)s->V * 3) + s->ws_bytes + 2 * bufb;
    int rc = HULL_OK;
    if (hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess)
        rc = HULL_EDEVICE;
    for (int k = 0; k < 2 && rc == HULL_OK; ++k)
        if (hipEventCreateWithFlags(&s->counted[k], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&s->copied[k], hipEventDisableTiming) != hipSuccess)
            rc = HULL_EDEVICE;
    if (rc == HULL_OK && hipMalloc(reinterpret_cast<void **>(&s->mem), total) != hipSuccess) {
        (void)hipGetLastError();
        s->mem = nullptr;
        rc = HULL_ENOMEM;
    }
    if (rc != HULL_OK) {
        session_free(s);
        return rc;
    }
    char *p = s->mem;
    s->N = reinterpret_cast<int32_t *>(p);            p += align_up((size_t)s->V * 4);
    s->M = reinterpret_cast<int32_t *>(p);            p += align_up((size_t)s->V * 4);
    s->stats = reinterpret_cast<hullmi_stats *>(p);   p += align_up(sizeof(hullmi_stats));
    s->masks = reinterpret_cast<uint8_t *>(p);        p += align_up((size_t)s->V * 3);
    s->ws = p;                                        p += s->ws_bytes;
    s->buf[0] = reinterpret_cast<float *>(p);         p += bufb;
    s->buf[1] = reinterpret_cast<float *>(p);
    hullmi::zero_counts(s->N, s->M, s->stats, s->V, s->compute);
    // both buffers start free and with nothing to count
    hipError_t e = hipSuccess;
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = hipEventRecord(s->counted[k], s->compute);
        if (e == hipSuccess) e = hipEventRecord(s->copied[k], s->copy);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->compute);
    if (e != hipSuccess) {
        session_free(s);
        return HULL_EDEVICE;
    }
    *out = s;
    return HULL_OK;
}

int hull_session_push(hullmi_session *s, const hullmi_histories *chunk, int host)
{
    if (!s || !hullmi::hist_valid(chunk) || chunk->n > s->max_chunk) return HULL_EINVAL;
    if (chunk->n == 0) return HULL_OK;
    std::lock_guard<std::mutex> lock(s->mu);
    DeviceGuard guard(s->device);
    if (!guard.ok) return HULL_EDEVICE;
    const int64_t n = chunk->n;
    int k = s->cur;
    if (s->fill[k] + n > s->cap) {
        // count the full buffer; fill the other one once its last count is done
        const int rc = flush(s, k);
        if (rc != HULL_OK) return rc;
        k = s->cur = 1 - k;
        if (hipStreamWaitEvent(s->copy, s->counted[k], 0) != hipSuccess) return HULL_EDEVICE;
    }
    const float *src[8] = {chunk->x_in, chunk->y_in, chunk->z_in, chunk->x_out,
                           chunk->y_out, chunk->z_out, chunk->angle_deg, chunk->wepl};
    // one append kernel when the device can read all eight arrays (device
    // memory, pinned host memory), else one copy per array
    Src8 view;
    bool direct = true;
    for (int f = 0; f < 8 && direct; ++f) direct = (view.p[f] = device_view(src[f])) != nullptr;
    hipError_t e = hipSuccess;
    if (direct) {
        const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
        k_session_append<<<blocks, 256, 0, s->copy>>>(view, n, field(s, k, 0) + s->fill[k], s->cap);
        e = hipGetLastError();
    } else {
        const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        for (int f = 0; f < 8 && e == hipSuccess; ++f)
            e = hipMemcpyAsync(field(s, k, f) + s->fill[k], src[f], (size_t)n * sizeof(float), kind,
                               s->copy);
    }
    if (e == hipSuccess) e = hipEventRecord(s->copied[k], s->copy);
    if (e != hipSuccess) return HULL_EDEVICE;
    s->fill[k] += n;
    // the caller may reuse its arrays once their bytes have been copied
    return session_status(hipEventSynchronize(s->copied[k]));
}

int hull_session_read(hullmi_session *s, int32_t *N, int32_t *M, uint8_t *sc_mask,
                      uint8_t *msc_mask, uint8_t *sm_mask, hullmi_stats *stats, int host)
{
    if (!s) return HULL_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    DeviceGuard guard(s->device);
    if (!guard.ok) return HULL_EDEVICE;
    int rc = flush(s, s->cur);
    if (rc != HULL_OK) return rc;
    uint8_t *m_sc = sc_mask ? s->masks : nullptr;
    uint8_t *m_msc = msc_mask ? s->masks + s->V : nullptr;
    uint8_t *m_sm = sm_mask ? s->masks + 2 * s->V : nullptr;
    rc = hullmi::masks_from_counts(&s->grid, &s->params, s->N, s->M, m_sc, m_msc, m_sm,
                                   reinterpret_cast<char *>(s->ws) + s->count_ws, s->compute);
    if (rc != HULL_OK) return rc;
    const hipMemcpyKind kind = host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    struct Out { void *dst; const void *src; size_t bytes; };
    const Out outs[6] = {{N, s->N, (size_t)s->V * 4},       {M, s->M, (size_t)s->V * 4},
                         {sc_mask, m_sc, (size_t)s->V},      {msc_mask, m_msc, (size_t)s->V},
                         {sm_mask, m_sm, (size_t)s->V},      {stats, s->stats, sizeof(hullmi_stats)}};
    hipError_t e = hipSuccess;
    for (const Out &o : outs)
        if (o.dst && e == hipSuccess) e = hipMemcpyAsync(o.dst, o.src, o.bytes, kind, s->compute);
    if (e == hipSuccess) e = hipStreamSynchronize(s->compute);
    return session_status(e);
}

int hull_session_reset(hullmi_session *s)
{
    if (!s) return HULL_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    DeviceGuard guard(s->device);
    if (!guard.ok) return HULL_EDEVICE;
    // histories waiting in the buffers belong to the old scan: drop them
    for (int k = 0; k < 2; ++k) {
        s->fill[k] = 0;
        if (hipStreamWaitEvent(s->compute, s->copied[k], 0) != hipSuccess) return HULL_EDEVICE;
    }
    hullmi::zero_counts(s->N, s->M, s->stats, s->V, s->compute);
    hipError_t e = hipGetLastError();
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventRecord(s->counted[k], s->compute);
    return session_status(e);
}

int hull_session_destroy(hullmi_session *s)
{
    if (!s) return HULL_EINVAL;
    DeviceGuard guard(s->device);
    session_free(s);
    return HULL_OK;
}

}  // extern "C"
