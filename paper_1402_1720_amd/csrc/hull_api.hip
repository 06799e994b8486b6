// Host side of the C ABI declared in hullmi.h: argument checks, workspace
// layout and kernel launches. Everything here runs on the calling thread and
// only enqueues work on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "hull_binned.h"
#include "hull_bsc.h"
#include "hull_device.h"
#include "hull_kernels.h"
#include "hull_runtime.h"
#include "hullmi.h"

namespace hullmi {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxAxis = 2048;
constexpr int kMaxNu = 2048;     // detector bins per row (the filter keeps a row in LDS)
constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

inline bool finite_pos(float v) { return std::isfinite(v) && v > 0.0f; }

bool grid_ok(const hullmi_grid *g)
{
    if (!g) return false;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return false;
    if (g->nx > kMaxAxis || g->ny > kMaxAxis || g->nz > kMaxAxis) return false;
    const int64_t V = (int64_t)g->nx * g->ny * g->nz;
    if (V > INT32_MAX) return false;
    if (!finite_pos(g->dx) || !finite_pos(g->dy) || !finite_pos(g->dz)) return false;
    if (!std::isfinite(g->x0) || !std::isfinite(g->y0) || !std::isfinite(g->z0)) return false;
    // voxel units must stay finite: 1/dx rounded in FP32 must not overflow
    if (!std::isfinite(1.0f / g->dx) || !std::isfinite(1.0f / g->dy) || !std::isfinite(1.0f / g->dz))
        return false;
    return true;
}

inline int64_t voxels(const hullmi_grid *g) { return (int64_t)g->nx * g->ny * g->nz; }

bool hist_ok(const hullmi_histories *h)
{
    if (!h) return false;
    if (h->n < 0 || h->n > INT32_MAX) return false;
    if (h->n == 0) return true;
    return h->x_in && h->y_in && h->z_in && h->x_out && h->y_out && h->z_out && h->angle_deg &&
           h->wepl;
}

bool fbp_ok(const hullmi_fbp_params *p)
{
    if (!p) return false;
    if (!finite_pos(p->src_dist_mm) || !finite_pos(p->du_mm) || !finite_pos(p->dv_mm) ||
        !finite_pos(p->dangle_deg))
        return false;
    if (!std::isfinite(p->u0_mm) || !std::isfinite(p->v0_mm) || !std::isfinite(p->angle0_deg) ||
        !std::isfinite(p->threshold))
        return false;
    if (p->nu < 1 || p->nv < 1 || p->n_angles < 1 || p->nu > kMaxNu) return false;
    if ((int64_t)p->nu * p->nv * p->n_angles > INT32_MAX) return false;
    if (p->filter != 0) return false;
    return true;
}

DevGrid dev_grid(const hullmi_grid *g)
{
    DevGrid d;
    d.nx = g->nx; d.ny = g->ny; d.nz = g->nz;
    d.rdx = 1.0f / g->dx; d.rdy = 1.0f / g->dy; d.rdz = 1.0f / g->dz;
    d.x0 = g->x0; d.y0 = g->y0; d.z0 = g->z0;
    return d;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

int launch_status()
{
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HULL_OK : HULL_EDEVICE;
}

void fill_u32(void *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (!p || n <= 0) return;
    const unsigned b = (unsigned)std::min<int64_t>(blocks_for(n), 4096);
    k_fill_u32<<<b, kBlock, 0, s>>>(reinterpret_cast<uint32_t *>(p), v, n);
}

void fill_u64(void *p, unsigned long long v, int64_t n, hipStream_t s)
{
    if (!p || n <= 0) return;
    const unsigned b = (unsigned)std::min<int64_t>(blocks_for(n), 4096);
    k_fill_u64<<<b, kBlock, 0, s>>>(reinterpret_cast<unsigned long long *>(p), v, n);
}

// Workspace of the SM rules: one 64-bit slot per z-slice (covers both scopes),
// and for the EDGE rule a threshold per slice, the packed gradient per voxel
// and the overflow space of the edge lists (two ints per voxel).
size_t sm_ws_bytes(const hullmi_grid *g)
{
    const size_t V = (size_t)g->nx * g->ny * g->nz;
    return 2 * align_up((size_t)g->nz * 8) + align_up(V * 8) + align_up(V * 8);
}

// Device properties the launch shapes depend on (queried per call: cheap).
struct DevProps {
    size_t max_lds;
    int cus;
};

DevProps dev_props()
{
    DevProps p{65536, 256};
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return p;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
        p.max_lds = (size_t)v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
        p.cus = v;
    return p;
}

// Raises a kernel's dynamic LDS limit to all that its static LDS leaves free
// and returns that limit (0 when it cannot be set). The value depends only on
// the kernel and the device, so concurrent calls on different grids never
// lower it under each other's launches.
size_t allow_max_lds(const void *fn, size_t max_lds)
{
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, fn) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const size_t lim = max_lds > a.sharedSizeBytes ? max_lds - a.sharedSizeBytes : 0;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return lim;
}

inline int64_t plane_of(const hullmi_grid *g) { return (int64_t)g->nx * g->ny; }

// Counters per tile row: odd (the walk loops rely on an x step and a y step
// both moving to the other half of a 32-bit word), nx or nx + 1; two more
// when a row would be a whole multiple of 64 words plus a half, where the
// rows a walk wave adds into at the same step would share LDS banks; not
// widened by those two when that would cost the second walk workgroup on a
// CU.
// LDS bytes of a walk workgroup for tile rows of `stride` counters: the tile
// rounded up to whole 16-byte quads (the flush and the reduce move four words
// at a time), then the control words.
inline int64_t tile_lds_bytes(int64_t stride, int ny)
{
    return (((stride * ny + 1) / 2 + 3) & ~int64_t(3)) * 4 + 16;
}
inline int tile_stride(const hullmi_grid *g)
{
    const int o = g->nx | 1;
    const int s = (o / 2) % 64 == 0 ? o + 2 : o;
    const int64_t two = 2 * tile_lds_bytes(s, g->ny), two_o = 2 * tile_lds_bytes(o, g->ny);
    return two <= 160 * 1024 || two_o > 160 * 1024 ? s : o;
}
// A slice fits the LDS tile when its 16-bit counters, padded rows included,
// fit the 160 KB of LDS.
inline bool tile_fits(const hullmi_grid *g)
{
    return tile_lds_bytes(tile_stride(g), g->ny) <= 160 * 1024;
}

// Length classes per slice: up to 16, fewer when there are many slices, so
// that the sub-bin histogram of a block fits its LDS. The workspace is laid
// out for this many; a tuning may ask for fewer.
inline int length_classes(const hullmi_grid *g) { return std::max(1, std::min(16, 2048 / g->nz)); }

// Length-class width (voxels of in-plane extent) for nl classes per slice.
// Width of a length class in voxels: the last of the nl classes holds the
// lines that may meet a voxel corner, the other nl - 1 split the lengths up
// to nx + ny (a single class holds every line).
inline int length_width(const hullmi_grid *g, int nl)
{
    const int m = nl > 1 ? nl - 1 : 1;
    return std::max(1, (g->nx + g->ny + m - 1) / m);
}

// Runs of a sub-bin are ordered by classification block modulo a stride r,
// so that neighbouring runs come from blocks r apart. By default r is the
// batch's block count over 128: for scans of 180 to 360 gantry angles that
// puts neighbouring runs about one angle apart. Measured: 8 best on the
// 200x200x32 scan (1221 blocks of 8192 histories), 32 to 64 on the full-scale
// one (8192 blocks per batch; 22.6, 22.0, 21.9 and 22.5 ms per pass with 8,
// 32, 64 and 256).
constexpr int kRunStrideBlocks = 128;
inline int default_run_stride(int nblk) { return std::max(1, std::min(256, nblk / kRunStrideBlocks)); }

// Workgroups of the persistent walk at most, and ranges per workgroup: the
// ranges of equal estimated work are dealt out round-robin, and two per
// workgroup even out the estimate's errors (one per workgroup left the walk
// 18% longer; four cost more in extra tile flushes than they saved).
constexpr int kMaxWalkGroups = 1024;
constexpr int kRangesPerGroup = 2;
// Where one walk workgroup fills a CU (slices of 256 x 256), more and shorter
// ranges even out the work better: 2, 3, 4, 6 and 8 per workgroup took the
// full-scale pass (256x256x64, 2e8 histories) to 31.9, 29.7, 28.6, 28.0 and
// 27.3 ms. The workspace holds kMaxWalkGroups * kRangesPerGroup coarse
// ranges, which caps this at 8 for 256 workgroups.
constexpr int kRangesPerGroupAlone = 8;

// Layout of the slice-binned counting workspace for internal batches of B
// histories. With base == nullptr only the size is computed.
BinWs bin_ws_layout(const hullmi_grid *g, int64_t B, void *base, size_t *bytes)
{
    BinWs w;
    w.B = B;
    w.nz = g->nz;
    w.nl = length_classes(g);
    w.lwidth = length_width(g, w.nl);
    w.ntiles = 2 * g->nz;
    w.nsub = w.ntiles * w.nl + 2;
    w.nblk = (int)((B + kHistPerBlock - 1) / kHistPerBlock);
    w.stride = tile_stride(g);
    w.gnx = g->nx;
    w.gny = g->ny;
    w.run_stride = default_run_stride(w.nblk);
    w.tile_words = tile_fits(g) ? (int)(((int64_t)w.stride * g->ny + 1) / 2) : 1;
    w.slot_words = (w.tile_words + 3) & ~3;
    w.min_ranges = kMaxWalkGroups * kRangesPerGroup;
    // ranges: P0 = max(min_ranges, ceil(I / kItemsPerRange)) coarse ranges,
    // each split into ceil(items / kItemsPerRange) <= 1 + items / kItemsPerRange
    // pieces: P <= P0 + I / kItemsPerRange <= min_ranges + 2 ceil(I / kItemsPerRange)
    const int64_t imax = B * kMaxSlicesPerLine;
    w.max_ranges = (int)(kMaxWalkGroups * kRangesPerGroup +
                         2 * ((imax + kItemsPerRange - 1) / kItemsPerRange));
    w.max_slots = w.max_ranges + w.ntiles;
    char *b = reinterpret_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t nbytes) {
        char *p = b ? b + off : nullptr;
        off += align_up(nbytes);
        return p;
    };
    const size_t Bp = (size_t)w.nblk * kHistPerBlock;   // whole classification blocks
    w.hrec = reinterpret_cast<uint4 *>(take(Bp * 16));
    w.meta = reinterpret_cast<uint32_t *>(take(Bp * 4));
    w.lpack = reinterpret_cast<uint32_t *>(take(Bp * 4));
    w.ngroups = (w.nblk + kScanGroup - 1) / kScanGroup;
    w.blk = reinterpret_cast<uint32_t *>(take((size_t)w.nsub * w.nblk * 4));
    w.boff = reinterpret_cast<uint32_t *>(take((size_t)w.nsub * w.nblk * 4));
    w.gsum = reinterpret_cast<uint32_t *>(take((size_t)w.nsub * w.ngroups * 4));
    w.goff = reinterpret_cast<uint32_t *>(take((size_t)w.nsub * w.ngroups * 4));
    w.sub_total = reinterpret_cast<uint32_t *>(take((size_t)w.nsub * 4));
    w.sub_start = reinterpret_cast<uint32_t *>(take((size_t)(w.nsub + 1) * 4));
    w.tile_start = reinterpret_cast<uint32_t *>(take((size_t)(w.ntiles + 1) * 4));
    w.range_start = reinterpret_cast<uint32_t *>(take((size_t)(w.max_ranges + 1) * 4));
    w.range_coarse = reinterpret_cast<uint32_t *>(take((size_t)(w.max_ranges + 1) * 4));
    w.range_piece = reinterpret_cast<uint32_t *>(take((size_t)(w.max_ranges + 1) * 4));
    w.wprefix = reinterpret_cast<unsigned long long *>(take((size_t)(w.nsub + 1) * 8));
    w.ctl = reinterpret_cast<int32_t *>(take((size_t)kCtlWords * 4));
    w.item = reinterpret_cast<uint4 *>(take((size_t)imax * 16));
    w.partial = reinterpret_cast<uint32_t *>(
        take(tile_fits(g) ? (size_t)w.max_slots * w.slot_words * 4 : 0));
    if (bytes) *bytes = off;
    return w;
}

inline int64_t batch_of(int64_t n, int64_t cap) { return std::max<int64_t>(1, std::min(n, cap)); }

size_t bin_ws_bytes(const hullmi_grid *g, int64_t B)
{
    size_t bytes = 0;
    bin_ws_layout(g, B, nullptr, &bytes);
    return bytes;
}

// Counting workspace for n histories: one batch of all of them up to kBatch;
// above that, two halves, each for a batch of n / k histories (rounded up to
// whole classification blocks), k the smallest even number of batches of at
// most kBatch / 2, which the per-scan calls' two-stream pass alternates
// between its streams. On the 256x256x64 grid with 2e8 histories that is six
// batches of 33.3M in about the 10.2 GB one batch of 2^26 takes; seven
// batches (halves of one 2^26 batch's workspace) took 0.35 ms longer per pass.
size_t counts_ws_bytes(const hullmi_grid *g, int64_t n)
{
    if (n <= kBatch) return bin_ws_bytes(g, batch_of(n, kBatch));
    int64_t k = (n + kBatch / 2 - 1) / (kBatch / 2);
    k += k & 1;
    const int64_t b = ((n + k - 1) / k + kHistPerBlock - 1) / kHistPerBlock * kHistPerBlock;
    return 2 * align_up(bin_ws_bytes(g, b)) + kAlign;
}

// The smallest counting workspace that n histories can run in.
size_t counts_ws_min_bytes(const hullmi_grid *g, int64_t n)
{
    return bin_ws_bytes(g, batch_of(n, kMinBatch));
}

// The largest internal batch for n histories whose workspace fits in avail
// bytes (the size grows with the batch), 0 when not even the smallest fits.
int64_t batch_for(const hullmi_grid *g, int64_t n, size_t avail)
{
    int64_t hi = batch_of(n, kBatch);
    if (bin_ws_bytes(g, hi) <= avail) return hi;
    int64_t lo = batch_of(n, kMinBatch);
    if (bin_ws_bytes(g, lo) > avail) return 0;
    while (hi - lo > 1) {   // bytes(lo) fits, bytes(hi) does not
        const int64_t mid = lo + (hi - lo) / 2;
        if (bin_ws_bytes(g, mid) <= avail) lo = mid; else hi = mid;
    }
    return lo;
}

struct FbpWs {
    unsigned long long *sum;
    unsigned *cnt;
    float *q;
    size_t qn;
    float2 *cs;
    int4 *fp;          // footprint of every (backprojection tile, angle)
    size_t bytes;
};

// Tiles of the tiled backprojection (kBpTile x kBpTile columns x kFbpZ slices).
inline int64_t bp_tiles(const hullmi_grid *g, int &ntx, int &nty, int &ntz)
{
    ntx = (g->nx + kBpTile - 1) / kBpTile;
    nty = (g->ny + kBpTile - 1) / kBpTile;
    ntz = (g->nz + 7) / 8;
    return (int64_t)ntx * nty * ntz;
}

FbpWs fbp_ws_layout(const hullmi_fbp_params *p, const hullmi_grid *g, void *base)
{
    const size_t nb = (size_t)p->nu * p->nv * p->n_angles;
    FbpWs w;
    char *b = reinterpret_cast<char *>(base);
    size_t off = 0;
    w.sum = reinterpret_cast<unsigned long long *>(b + off); off += align_up(nb * 8);
    w.cnt = reinterpret_cast<unsigned *>(b + off);           off += align_up(nb * 4);
    w.q = reinterpret_cast<float *>(b + off);
    w.qn = (size_t)p->n_angles * (p->nv + 4) * (p->nu + 4);   // padded filtered projections
    off += align_up(w.qn * 4);
    w.cs = reinterpret_cast<float2 *>(b + off);              off += align_up((size_t)p->n_angles * 8);
    int ntx, nty, ntz;
    w.fp = reinterpret_cast<int4 *>(b + off);
    off += align_up((size_t)bp_tiles(g, ntx, nty, ntz) * p->n_angles * sizeof(int4));
    w.bytes = off;
    return w;
}

// The second stream of the two-stream counting pass: one per device, created
// on first use (non-blocking, default priority) and kept until the process
// ends. Calls from several host threads may share it: every dependency between
// it and a caller's stream goes through events recorded before they are waited
// on, so the shared stream can only add waits, never a cycle.
constexpr int kMaxDevices = 64;

hipStream_t second_stream()
{
    static std::mutex mu;
    static hipStream_t streams[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        streams[dev] = nullptr;
    }
    return streams[dev];
}

// Whether work enqueued on s is being captured into a graph (then the pass
// stays on s alone); unknown counts as captured.
bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) {
        (void)hipGetLastError();
        return true;
    }
    return st != hipStreamCaptureStatusNone;
}

// Zero (unless accumulating) and count: the shared core of every hull call.
// Histories go through in internal batches, as large as the workspace allows
// (up to kBatch); counts add up across them. With o.two_streams, a pass that
// needs several batches splits the workspace in two halves and runs batches
// of equal size that fit a half, alternately on s and on the second stream:
// one batch's classification, scatter and set-up then run beside the other's
// walk. The reduce and the overflow walk add into N and M, so each batch's
// waits for the previous batch's (an event recorded after them).
int run_counts(const hullmi_histories *h, const hullmi_grid *g, float e_low, float e_high, int32_t *N,
               int32_t *M, uint32_t flags, hullmi_stats *stats, void *ws, size_t ws_bytes,
               hipStream_t s, const CountOpts &o)
{
    const int64_t V = voxels(g);
    const int64_t B = h->n > 0 ? batch_for(g, h->n, ws_bytes) : 1;
    if (B == 0) return HULL_ENOMEM;
    if (!(flags & HULL_ACCUMULATE)) {
        fill_u32(N, 0u, N ? V : 0, s);
        fill_u32(M, 0u, M ? V : 0, s);
        fill_u64(stats, 0ull, stats ? 6 : 0, s);
    }
    if (h->n == 0) return launch_status();
    int64_t Bw = B;
    char *second_half = nullptr;
    hipStream_t s2 = nullptr;
    if (o.two_streams && h->n > B && !stream_capturing(s)) {
        const size_t half = ws_bytes / 2 / kAlign * kAlign;
        const int64_t B2 = batch_for(g, h->n, half);
        if (B2 > 0) {
            const int64_t nbat = (h->n + B2 - 1) / B2;
            const int64_t even = ((h->n + nbat - 1) / nbat + kHistPerBlock - 1) / kHistPerBlock * kHistPerBlock;
            Bw = std::min(B2, even);
            second_half = reinterpret_cast<char *>(ws) + half;
            if (!o.prof) s2 = second_stream();
        }
    }
    hipEvent_t ev_fork = nullptr, ev_acc = nullptr, ev_join = nullptr;
    auto drop_events = [&]() {
        for (hipEvent_t e : {ev_fork, ev_acc, ev_join})
            if (e) (void)hipEventDestroy(e);
        ev_fork = ev_acc = ev_join = nullptr;
    };
    if (s2) {
        // the second stream starts after everything enqueued on s so far
        if (hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ev_acc, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ev_join, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(ev_fork, s) != hipSuccess || hipStreamWaitEvent(s2, ev_fork, 0) != hipSuccess) {
            (void)hipGetLastError();
            drop_events();
            s2 = nullptr;   // the same batches, on s alone
        }
    }
    BinWs w = bin_ws_layout(g, Bw, ws, nullptr);
    BinWs w_second = second_half ? bin_ws_layout(g, Bw, second_half, nullptr) : w;
    const DevProps dp = dev_props();
    const size_t tile_bytes = (size_t)tile_lds_bytes(w.stride, g->ny);   // tile + control words
    const bool tile_ok =
        tile_fits(g) &&
        tile_bytes <= allow_max_lds(reinterpret_cast<const void *>(k_walk_tiles), dp.max_lds);
    int per_cu = 1;
    if (tile_ok) {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_walk_tiles, kTileThreads,
                                                         tile_bytes) == hipSuccess && occ > 0)
            per_cu = occ;
    }
    int walk_grid = std::min(dp.cus * per_cu, kMaxWalkGroups);
    if (o.walk_blocks > 0) walk_grid = std::min(walk_grid, o.walk_blocks);
    const int rpg_want = o.ranges_per_group > 0 ? o.ranges_per_group
                                                : (per_cu >= 2 ? kRangesPerGroup : kRangesPerGroupAlone);
    const int rpg = std::max(1, std::min(rpg_want, kMaxWalkGroups * kRangesPerGroup / walk_grid));
    // measurement: an event pair around every launch when asked for
    auto mark = [&](int k) { if (o.prof) o.prof->begin(k, s); };
    auto done = [&]() { if (o.prof) o.prof->end(s); };
    if (o.length_classes > 0 && o.length_classes < w.nl) {
        // fewer sub-bins than the workspace is laid out for
        for (BinWs *x : {&w, &w_second}) {
            x->nl = o.length_classes;
            x->lwidth = length_width(g, x->nl);
            x->nsub = x->ntiles * x->nl + 2;
        }
    }
    const DevGrid dg = dev_grid(g);
    const int plane = (int)plane_of(g);
    int rc = HULL_OK;
    int64_t bi = 0;
    for (int64_t h0 = 0; h0 < h->n && rc == HULL_OK; h0 += Bw, ++bi) {
        const int64_t nb = std::min<int64_t>(Bw, h->n - h0);
        const bool second = (bi & 1) != 0;
        hipStream_t st = s2 && second ? s2 : s;
        BinWs wb = second ? w_second : w;
        wb.nblk = (int)((nb + kHistPerBlock - 1) / kHistPerBlock);
        wb.ngroups = (wb.nblk + kScanGroup - 1) / kScanGroup;
        wb.min_ranges = rpg * walk_grid;
        wb.run_stride = o.run_stride > 0 ? o.run_stride : default_run_stride(wb.nblk);
        mark(HULL_PROF_CLASSIFY);
        k_bin_classify<<<wb.nblk, kBinThreads, 0, st>>>(*h, h0, nb, dg, e_low, e_high, N != nullptr,
                                                       M != nullptr, tile_ok ? 1 : 0, wb, stats);
        done();
        mark(HULL_PROF_SCAN);
        k_bin_scan_groups<<<wb.ngroups, 256, 0, st>>>(wb);
        k_bin_scan_sums<<<(wb.nsub + 3) / 4, 256, 0, st>>>(wb);
        done();
        mark(HULL_PROF_PLAN);
        k_bin_plan<<<1, 1024, 0, st>>>(wb);
        done();
        mark(HULL_PROF_SCATTER);
        k_bin_scatter<<<wb.nblk, kScatterThreads, 0, st>>>(nb, wb);
        done();
        if (tile_ok) {
            // 16 blocks per CU: 125 us against 131 us with 8 and 153 us with 4
            // (1.1e7 items, 200x200x32)
            mark(HULL_PROF_SETUP);
            k_item_setup<<<dp.cus * 16, 256, (size_t)(wb.ntiles + 1) * 4, st>>>(wb, g->nx, g->ny);
            done();
            mark(HULL_PROF_WALK);
            k_walk_tiles<<<walk_grid, kTileThreads, tile_bytes, st>>>(wb, g->nx, g->ny);
            done();
        }
        // N and M: after the previous batch's reduce and overflow walk
        if (s2 && bi > 0 && hipStreamWaitEvent(st, ev_acc, 0) != hipSuccess) rc = HULL_EDEVICE;
        if (tile_ok) {
            dim3 rg((unsigned)((wb.slot_words / 4 + 255) / 256), (unsigned)wb.ntiles);
            mark(HULL_PROF_REDUCE);
            k_reduce_tiles<<<rg, 256, 0, st>>>(wb, plane, N, M, stats);
            done();
        }
        mark(HULL_PROF_OVERFLOW);
        k_walk_overflow<<<1024, 256, 0, st>>>(*h, h0, dg, wb, N, M, stats);
        done();
        if (s2 && hipEventRecord(ev_acc, st) != hipSuccess) rc = HULL_EDEVICE;
        if (rc == HULL_OK) rc = launch_status();
    }
    if (s2) {
        // the caller's stream covers every batch, also after an error, so that
        // its completion still means the workspace is free
        if (hipEventRecord(ev_join, s2) != hipSuccess || hipStreamWaitEvent(s, ev_join, 0) != hipSuccess) {
            (void)hipGetLastError();
            if (rc == HULL_OK) rc = HULL_EDEVICE;
        }
        drop_events();
    }
    return rc == HULL_OK ? launch_status() : rc;
}

// Launch choices of the per-scan calls: the two-stream pass where it applies.
CountOpts per_scan_opts()
{
    CountOpts o;
    o.two_streams = true;
    return o;
}

int run_msc_mask(const hullmi_grid *g, const int32_t *N, uint8_t *mask, int n_t, int mode, int nbr,
                 hipStream_t s)
{
    if (!mask) return HULL_OK;
    const int64_t V = voxels(g);
    k_msc_mask<<<blocks_for(V), kBlock, 0, s>>>(N, mask, g->nx, g->ny, g->nz, n_t, mode, nbr);
    return launch_status();
}

int run_sm_mask(const hullmi_grid *g, const int32_t *M, uint8_t *mask, int num, int den, int mode,
                int scope, int nbr, void *ws, hipStream_t s)
{
    if (!mask) return HULL_OK;
    const int64_t V = voxels(g);
    if (mode == HULL_SM_EDGE) {
        char *b = reinterpret_cast<char *>(ws);
        auto *seed = reinterpret_cast<unsigned long long *>(b);
        auto *mt = reinterpret_cast<long long *>(b + align_up((size_t)g->nz * 8));
        auto *gp = reinterpret_cast<unsigned long long *>(b + 2 * align_up((size_t)g->nz * 8));
        auto *glist = reinterpret_cast<int *>(b + 2 * align_up((size_t)g->nz * 8) + align_up((size_t)V * 8));
        const int64_t plane = (int64_t)g->nx * g->ny;
        fill_u64(seed, 0ull, g->nz, s);
        k_sm_edge_thin<<<dim3((unsigned)((plane + kBlock - 1) / kBlock), (unsigned)g->nz), kBlock, 0, s>>>(
            M, gp, seed, g->nx, g->ny);
        // edge lists in LDS up to all the LDS there is (two ints per entry)
        const DevProps dp = dev_props();
        const size_t lim = allow_max_lds(reinterpret_cast<const void *>(k_sm_edge_trace), dp.max_lds);
        const int cap = (int)std::min<int64_t>((int64_t)(lim / 8), plane);
        k_sm_edge_trace<<<(unsigned)g->nz, 1024, (size_t)cap * 8, s>>>(M, gp, seed, mt, glist, g->nx,
                                                                       g->ny, num, den, cap);
        k_sm_edge_mask<<<blocks_for(V), kBlock, 0, s>>>(M, mt, mask, V, plane);
        return launch_status();
    }
    const int64_t seg_len = scope == HULL_SCOPE_SLICE ? (int64_t)g->nx * g->ny : V;
    const int64_t nseg = V / seg_len;
    auto *seg = reinterpret_cast<unsigned long long *>(ws);
    fill_u64(seg, 0ull, nseg, s);
    // a few blocks per segment, each striding over it with one atomic at the end
    const unsigned per_seg = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, seg_len / (kBlock * 8)));
    const dim3 rg(per_seg, (unsigned)nseg);
    if (mode == HULL_SM_FRACTION)
        k_seg_max<<<rg, kBlock, 0, s>>>(M, seg, V, seg_len);
    else
        k_seg_slope_argmax<<<rg, kBlock, 0, s>>>(M, seg, g->nx, g->ny, g->nz, nbr, seg_len);
    k_sm_mask<<<blocks_for(V), kBlock, 0, s>>>(M, mask, V, seg_len, mode, num, den, seg);
    return launch_status();
}

bool msc_args_ok(int n_t, int mode, int nbr)
{
    return n_t >= 1 && (mode == HULL_MSC_COUNT || mode == HULL_MSC_NEIGHBOR_DIFF) &&
           (nbr == HULL_NBR_INPLANE4 || nbr == HULL_NBR_SPATIAL6);
}

bool sm_args_ok(int num, int den, int mode, int scope, int nbr)
{
    if (mode == HULL_SM_EDGE && scope != HULL_SCOPE_SLICE) return false;
    return den > 0 && num >= 0 &&
           (mode == HULL_SM_FRACTION || mode == HULL_SM_MAX_SLOPE || mode == HULL_SM_EDGE) &&
           (scope == HULL_SCOPE_VOLUME || scope == HULL_SCOPE_SLICE) &&
           (nbr == HULL_NBR_INPLANE4 || nbr == HULL_NBR_SPATIAL6);
}

int sc_impl(const hullmi_histories *hist, const hullmi_grid *grid, float wepl_low, int32_t *N,
            uint8_t *mask, uint32_t flags, hullmi_stats *stats, void *ws, size_t ws_bytes,
            hipStream_t s, const CountOpts &o)
{
    if (!hist_ok(hist) || !grid_ok(grid) || !N || !std::isfinite(wepl_low)) return HULL_EINVAL;
    if (hist->n > 0 && (!ws || ws_bytes < counts_ws_min_bytes(grid, hist->n))) return HULL_ENOMEM;
    int rc = run_counts(hist, grid, wepl_low, 0.0f, N, nullptr, flags, stats, ws, ws_bytes, s, o);
    if (rc != HULL_OK) return rc;
    if (mask) k_sc_mask<<<blocks_for(voxels(grid)), kBlock, 0, s>>>(N, mask, voxels(grid));
    return launch_status();
}

int msc_impl(const hullmi_histories *hist, const hullmi_grid *grid, float wepl_low, int32_t n_t,
             int mode, int nbr, int32_t *N, uint8_t *mask, uint32_t flags, hullmi_stats *stats,
             void *ws, size_t ws_bytes, hipStream_t s, const CountOpts &o)
{
    if (!hist_ok(hist) || !grid_ok(grid) || !N || !std::isfinite(wepl_low) ||
        !msc_args_ok(n_t, mode, nbr))
        return HULL_EINVAL;
    if (hist->n > 0 && (!ws || ws_bytes < counts_ws_min_bytes(grid, hist->n))) return HULL_ENOMEM;
    int rc = run_counts(hist, grid, wepl_low, 0.0f, N, nullptr, flags, stats, ws, ws_bytes, s, o);
    if (rc != HULL_OK) return rc;
    return run_msc_mask(grid, N, mask, n_t, mode, nbr, s);
}

int sm_impl(const hullmi_histories *hist, const hullmi_grid *grid, float wepl_high, int32_t frac_num,
            int32_t frac_den, int mode, int scope, int nbr, int32_t *M, uint8_t *mask,
            uint32_t flags, hullmi_stats *stats, void *ws, size_t ws_bytes, hipStream_t s,
            const CountOpts &o)
{
    if (!hist_ok(hist) || !grid_ok(grid) || !M || !std::isfinite(wepl_high) ||
        !sm_args_ok(frac_num, frac_den, mode, scope, nbr))
        return HULL_EINVAL;
    // the rule's part of the workspace first, the counting part after it
    const size_t rw = sm_ws_bytes(grid);
    if (!ws || ws_bytes < rw + counts_ws_min_bytes(grid, hist->n)) return HULL_ENOMEM;
    int rc = run_counts(hist, grid, 0.0f, wepl_high, nullptr, M, flags, stats,
                        reinterpret_cast<char *>(ws) + rw, ws_bytes - rw, s, o);
    if (rc != HULL_OK) return rc;
    return run_sm_mask(grid, M, mask, frac_num, frac_den, mode, scope, nbr, ws, s);
}

int all_impl(const hullmi_histories *hist, const hullmi_grid *grid, const hullmi_params *p,
             int32_t *N, int32_t *M, uint8_t *sc_mask, uint8_t *msc_mask, uint8_t *sm_mask,
             uint32_t flags, hullmi_stats *stats, void *ws, size_t ws_bytes, hipStream_t s,
             const CountOpts &o)
{
    if (!hist_ok(hist) || !grid_ok(grid) || !p || !N || !M) return HULL_EINVAL;
    if (!std::isfinite(p->wepl_low) || !std::isfinite(p->wepl_high)) return HULL_EINVAL;
    if (msc_mask && !msc_args_ok(p->msc_n_t, p->msc_mode, p->nbr)) return HULL_EINVAL;
    if (sm_mask && !sm_args_ok(p->sm_frac_num, p->sm_frac_den, p->sm_mode, p->sm_scope, p->nbr))
        return HULL_EINVAL;
    const size_t rw = sm_ws_bytes(grid);   // the rules' part first, the counting part after it
    if (!ws || ws_bytes < rw + counts_ws_min_bytes(grid, hist->n)) return HULL_ENOMEM;
    int rc = run_counts(hist, grid, p->wepl_low, p->wepl_high, N, M, flags, stats,
                        reinterpret_cast<char *>(ws) + rw, ws_bytes - rw, s, o);
    if (rc != HULL_OK) return rc;
    if (sc_mask) k_sc_mask<<<blocks_for(voxels(grid)), kBlock, 0, s>>>(N, sc_mask, voxels(grid));
    rc = launch_status();
    if (rc == HULL_OK) rc = run_msc_mask(grid, N, msc_mask, p->msc_n_t, p->msc_mode, p->nbr, s);
    if (rc == HULL_OK)
        rc = run_sm_mask(grid, M, sm_mask, p->sm_frac_num, p->sm_frac_den, p->sm_mode, p->sm_scope,
                         p->nbr, ws, s);
    return rc;
}

FbpDev fbp_dev(const hullmi_fbp_params *fbp)
{
    FbpDev p;
    p.src_dist = fbp->src_dist_mm; p.du = fbp->du_mm; p.dv = fbp->dv_mm;
    p.u0 = fbp->u0_mm; p.v0 = fbp->v0_mm;
    p.rdu = 1.0f / fbp->du_mm; p.rdv = 1.0f / fbp->dv_mm; p.rda = 1.0f / fbp->dangle_deg;
    p.angle0 = fbp->angle0_deg; p.dangle = fbp->dangle_deg; p.threshold = fbp->threshold;
    p.half_dth = (float)(0.5 * (double)fbp->dangle_deg * 3.14159265358979323846 / 180.0);
    p.nu = fbp->nu; p.nv = fbp->nv; p.n_angles = fbp->n_angles;
    return p;
}

// Weighting, filtering and backprojection of per-bin sums (fixed point of
// `unit` mm) and counts: the FDK steps after the binning.
void fbp_reconstruct(const hullmi_grid *grid, const FbpDev &p, const FbpWs &w,
                     const unsigned long long *sum, const unsigned *cnt, double unit, float *image,
                     uint8_t *mask, hipStream_t s, KernelProf *prof = nullptr)
{
    auto mark = [&](int k) { if (prof) prof->begin(k, s); };
    auto done = [&]() { if (prof) prof->end(s); };
    // the kernel table and one row per wavefront of the block (up to 98 KB
    // for 2048 bins per row, above the default dynamic LDS limit)
    const size_t lds = (size_t)(2 * p.nu + kFbpFilterRows * p.nu) * sizeof(double);
    allow_max_lds(reinterpret_cast<const void *>(k_fbp_filter), dev_props().max_lds);
    mark(HULL_PROF_FBP_FILTER);
    fill_u32(w.q, 0u, (int64_t)w.qn, s);   // zero borders of the padded projections
    const int64_t rows = (int64_t)p.n_angles * p.nv;
    k_fbp_filter<<<(unsigned)((rows + kFbpFilterRows - 1) / kFbpFilterRows), 64 * kFbpFilterRows, lds,
                   s>>>(sum, cnt, w.q, p, unit);
    done();
    mark(HULL_PROF_FBP_GEOMETRY);
    k_fbp_trig<<<(p.n_angles + 63) / 64, 64, 0, s>>>(w.cs, p);
    FbpGridDev gd{grid->nx, grid->ny, grid->nz, grid->dx, grid->dy, grid->dz,
                  grid->x0, grid->y0, grid->z0};
    int ntx, nty, ntz;
    const int64_t ntiles = bp_tiles(grid, ntx, nty, ntz);
    k_fbp_footprint<<<blocks_for(ntiles * p.n_angles), kBlock, 0, s>>>(w.cs, p, gd, w.fp, ntx, nty,
                                                                       ntz);
    done();
    mark(HULL_PROF_FBP_BACKPROJECT);
    k_fbp_backproject_tiles<<<(unsigned)ntiles, kBpTile * kBpTile, 0, s>>>(w.q, w.cs, w.fp, p, gd,
                                                                          image, mask, ntx, nty);
    done();
}

void fbp_bin_stage(const hullmi_histories *hist, const FbpDev &p, const FbpWs &w, hipStream_t s,
                   KernelProf *prof = nullptr);

int fbp_impl(const hullmi_histories *hist, const hullmi_grid *grid, const hullmi_fbp_params *fbp,
             float *image, uint8_t *mask, void *ws, size_t ws_bytes, hipStream_t s,
             KernelProf *prof = nullptr)
{
    if (!hist_ok(hist) || !grid_ok(grid) || !fbp_ok(fbp) || !image) return HULL_EINVAL;
    const size_t need = fbp_ws_layout(fbp, grid, nullptr).bytes;
    if (!ws || ws_bytes < need) return HULL_ENOMEM;
    FbpWs w = fbp_ws_layout(fbp, grid, ws);
    const FbpDev p = fbp_dev(fbp);
    fbp_bin_stage(hist, p, w, s, prof);
    fbp_reconstruct(grid, p, w, w.sum, w.cnt, 1.0 / 65536.0, image, mask, s, prof);
    return launch_status();
}

// Zeroes the FDK bin sums and counts and bins the histories into them (WEPL
// in 2^-16 mm).
void fbp_bin_stage(const hullmi_histories *hist, const FbpDev &p, const FbpWs &w, hipStream_t s,
                   KernelProf *prof)
{
    auto mark = [&](int k) { if (prof) prof->begin(k, s); };
    auto done = [&]() { if (prof) prof->end(s); };
    const int64_t nb = (int64_t)p.nu * p.nv * p.n_angles;
    mark(HULL_PROF_FBP_CLEAR);
    fill_u64(w.sum, 0ull, nb, s);
    fill_u32(w.cnt, 0u, nb, s);
    done();
    mark(HULL_PROF_FBP_BIN);
    if (hist->n > 0) {
        // an LDS copy of one detector plane (12 bytes per bin); chunks so
        // that every resident block gets one
        const size_t plane_lds = (size_t)p.nu * p.nv * 12;
        const DevProps dp = dev_props();
        const size_t lim = allow_max_lds(reinterpret_cast<const void *>(k_fbp_bin_lds), dp.max_lds);
        if (plane_lds <= lim) {
            const size_t lds = plane_lds;
            int occ = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_fbp_bin_lds, kFbpBinThreads,
                                                             lds) != hipSuccess || occ < 1)
                occ = 1;
            const int64_t want = std::min<int64_t>((int64_t)dp.cus * occ,
                                                   (hist->n + kFbpBinThreads - 1) / kFbpBinThreads);
            const int64_t chunk = (hist->n + want - 1) / want;
            k_fbp_bin_lds<<<(unsigned)((hist->n + chunk - 1) / chunk), kFbpBinThreads, lds, s>>>(
                *hist, p, w.sum, w.cnt, chunk);
        } else {
            k_fbp_bin<<<blocks_for(hist->n), kBlock, 0, s>>>(*hist, p, w.sum, w.cnt);
        }
    }
    done();
}

bool bsc_ok(const hullmi_bsc_params *b)
{
    if (!b) return false;
    if (!std::isfinite(b->wepl_low) || !(std::fabs(b->wepl_low) < 65536.0f)) return false;
    if (b->cut_sigmas < 0 || b->cut_sigmas > 64) return false;
    if (b->window < 1 || b->window > 31 || b->window % 2 == 0) return false;
    return b->thr_den > 0 && b->thr_num >= 0;
}

// Workspace of the binned SC: the per-history records, the per-bin sums and
// kept ranges, kept counts and sums, the carved bit volume and the counters
// (the last three used when the caller passes no array of its own).
BscWs bsc_ws_layout(const hullmi_fbp_params *p, const hullmi_grid *g, int64_t n, void *base,
                    size_t *bytes)
{
    BscWs w;
    const size_t nb = (size_t)p->nu * p->nv * p->n_angles;
    char *b = reinterpret_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t nbytes) {
        char *q = b ? b + off : nullptr;
        off += align_up(nbytes);
        return q;
    };
    w.rec = reinterpret_cast<int2 *>(take((size_t)std::max<int64_t>(n, 1) * 8));
    w.cnt = reinterpret_cast<unsigned *>(take(nb * 4));
    w.s1 = reinterpret_cast<unsigned long long *>(take(nb * 8));
    w.s2lo = reinterpret_cast<unsigned long long *>(take(nb * 8));
    w.s2hi = reinterpret_cast<unsigned long long *>(take(nb * 8));
    w.bnd = reinterpret_cast<int2 *>(take(nb * 8));
    w.kept_n = reinterpret_cast<unsigned *>(take(nb * 4));
    w.kept_s = reinterpret_cast<unsigned long long *>(take(nb * 8));
    w.cbits = reinterpret_cast<unsigned *>(take((size_t)(voxels(g) + 31) / 32 * 4));
    w.stats = reinterpret_cast<unsigned long long *>(take(kBscStatWords * 8));
    w.cs = reinterpret_cast<float2 *>(take((size_t)p->n_angles * 8));
    w.list = reinterpret_cast<int *>(take(nb * 4));
    w.nlist = reinterpret_cast<int *>(take(4));
    w.nb = (int64_t)nb;
    if (bytes) *bytes = off;
    return w;
}


// The data-cut stage shared by the binned SC and the FDK hull after cuts:
// zero the per-bin sums, counters, statistics and `vwords` words of the
// carved bit volume, then bin (stats), sum squares, find the kept ranges
// (bounds) and sum the kept histories (cut). Returns the block count of the
// per-bin passes.
unsigned bsc_cut_stage(const hullmi_histories *hist, const FbpDev &p, BscWs &w, int ksig,
                       int64_t vwords, const DevProps &dp, hipStream_t s,
                       unsigned long long *fsum = nullptr, unsigned *fcnt = nullptr)
{
    const int plane = p.nu * p.nv;
    k_bsc_clear<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(
                      blocks_for(std::max<int64_t>(w.nb, vwords)), 2048)),
                  kBlock, 0, s>>>(w, vwords);
    const int64_t n = hist->n;
    // per-bin passes: one block of kBscThreads per CU (or fewer for few bins)
    const unsigned per_bin_blocks = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>(dp.cus, (w.nb + kBscThreads - 1) / kBscThreads));
    if (n > 0) {
        // the three history passes share one shape: LDS copies of one or two
        // detector planes at 8 bytes per bin, chunks so that every resident
        // block gets one (at most kBscMaxChunk histories each)
        const size_t plane_lds = (size_t)plane * 8;
        auto shape = [&](const void *fn, int &np, int64_t &chunk) {
            const size_t lim = allow_max_lds(fn, dp.max_lds);
            np = 2 * plane_lds <= lim ? 2 : (plane_lds <= lim ? 1 : 0);
            int occ = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kBscThreads, np * plane_lds) !=
                    hipSuccess ||
                occ < 1) {
                (void)hipGetLastError();
                occ = 1;
            }
            const int64_t want = std::min<int64_t>((int64_t)dp.cus * occ,
                                                   (n + kBscThreads - 1) / kBscThreads);
            chunk = std::min<int64_t>((n + want - 1) / want, kBscMaxChunk);
        };
        int np;
        int64_t ch;
        shape(reinterpret_cast<const void *>(k_bsc_stats), np, ch);
        k_bsc_stats<<<(unsigned)((n + ch - 1) / ch), kBscThreads, np * plane_lds, s>>>(*hist, p, w,
                                                                                       ch, np);
        shape(reinterpret_cast<const void *>(k_bsc_squares), np, ch);
        k_bsc_squares<<<(unsigned)((n + ch - 1) / ch), kBscThreads, np * plane_lds, s>>>(w, n, plane,
                                                                                         ch, np);
        k_bsc_bounds<<<per_bin_blocks, kBscThreads, 0, s>>>(w, ksig);
        shape(reinterpret_cast<const void *>(k_bsc_cut), np, ch);
        k_bsc_cut<<<(unsigned)((n + ch - 1) / ch), kBscThreads, np * plane_lds, s>>>(
            w, n, plane, ch, np, hist->wepl, fsum, fcnt);
    } else {
        k_bsc_bounds<<<per_bin_blocks, kBscThreads, 0, s>>>(w, ksig);
    }
    return per_bin_blocks;
}

int bsc_impl(const hullmi_histories *hist, const hullmi_grid *grid, const hullmi_fbp_params *fbp,
             const hullmi_bsc_params *bp, uint32_t *kept_n, int64_t *kept_sum, uint8_t *carved,
             uint8_t *mask, hullmi_bsc_stats *stats, void *ws, size_t ws_bytes, hipStream_t s)
{
    if (!hist_ok(hist) || !grid_ok(grid) || !fbp_ok(fbp) || !bsc_ok(bp) || !mask)
        return HULL_EINVAL;
    size_t need = 0;
    bsc_ws_layout(fbp, grid, hist->n, nullptr, &need);
    if (!ws || ws_bytes < need) return HULL_ENOMEM;
    BscWs w = bsc_ws_layout(fbp, grid, hist->n, ws, nullptr);
    if (kept_n) w.kept_n = kept_n;
    if (kept_sum) w.kept_s = reinterpret_cast<unsigned long long *>(kept_sum);
    if (stats) w.stats = reinterpret_cast<unsigned long long *>(stats);
    const FbpDev p = fbp_dev(fbp);
    const int64_t V = voxels(grid);
    const int64_t vwords = (V + 31) / 32;
    const DevProps dp = dev_props();
    const unsigned per_bin_blocks = bsc_cut_stage(hist, p, w, bp->cut_sigmas, vwords, dp, s);
    const long long e_q = std::llrint((double)bp->wepl_low * 1024.0);
    k_bsc_trig<<<(p.n_angles + 63) / 64, 64, 0, s>>>(w, p);
    // carve blocks: one per CU, each with an LDS bit window of all the LDS
    // there is (at most the whole volume); when the volume does not fit, the
    // carve list runs detector rows first so that each block's lines stay in
    // a few slices
    const size_t lim_v = allow_max_lds(reinterpret_cast<const void *>(k_bsc_carve), dp.max_lds);
    const int lwords = (int)std::min<int64_t>((int64_t)(lim_v / 4), vwords);
    k_bsc_select<<<per_bin_blocks, kBscThreads, 0, s>>>(w, p, e_q, lwords < vwords ? 1 : 0);
    k_bsc_carve<<<per_bin_blocks, kCarveThreads, (size_t)lwords * 4, s>>>(w, p, dev_grid(grid),
                                                                          lwords);
    const int r = bp->window / 2;
    const dim3 bgrid((unsigned)((grid->nx + kBlurTx - 1) / kBlurTx),
                     (unsigned)((grid->ny + kBlurTy - 1) / kBlurTy), (unsigned)grid->nz);
    k_bsc_blur<<<bgrid, dim3(kBlurTx, kBlurTy), 0, s>>>(
        w.cbits, carved, mask, grid->nx, grid->ny, r, (long long)bp->thr_num * bp->window * bp->window,
        bp->thr_den);
    return launch_status();
}

// Workspace of the FDK hull after cuts: the cut stage's, then the FDK steps'.
size_t fbp_cut_ws_bytes(const hullmi_fbp_params *fbp, const hullmi_grid *g, int64_t n, size_t *cut)
{
    size_t b = 0;
    bsc_ws_layout(fbp, g, n, nullptr, &b);
    if (cut) *cut = align_up(b);
    return align_up(b) + fbp_ws_layout(fbp, g, nullptr).bytes;
}

int fbp_cut_impl(const hullmi_histories *hist, const hullmi_grid *grid, const hullmi_fbp_params *fbp,
                 int32_t cut_sigmas, float *image, uint8_t *mask, void *ws, size_t ws_bytes,
                 hipStream_t s)
{
    if (!hist_ok(hist) || !grid_ok(grid) || !fbp_ok(fbp) || !image || cut_sigmas < 0 ||
        cut_sigmas > 64)
        return HULL_EINVAL;
    size_t cut = 0;
    const size_t need = fbp_cut_ws_bytes(fbp, grid, hist->n, &cut);
    if (!ws || ws_bytes < need) return HULL_ENOMEM;
    BscWs w = bsc_ws_layout(fbp, grid, hist->n, ws, nullptr);
    const FbpWs f = fbp_ws_layout(fbp, grid, reinterpret_cast<char *>(ws) + cut);
    const FbpDev p = fbp_dev(fbp);
    // the FDK bins of every history (2^-16 mm sums), then the cut stage takes
    // the cut histories out of them
    fbp_bin_stage(hist, p, f, s);
    bsc_cut_stage(hist, p, w, cut_sigmas, 0, dev_props(), s, f.sum, f.cnt);
    fbp_reconstruct(grid, p, f, f.sum, f.cnt, 1.0 / 65536.0, image, mask, s);
    return launch_status();
}

size_t ws_bytes_of(int op, const hullmi_grid *grid, int64_t n, const hullmi_fbp_params *fbp)
{
    if (n < 0) return (size_t)-1;
    switch (op) {
    case HULL_OP_COUNT_LINES:
        if (!grid_ok(grid)) return (size_t)-1;
        return 0;
    case HULL_OP_SC:
    case HULL_OP_MSC:
        if (!grid_ok(grid)) return (size_t)-1;
        return counts_ws_bytes(grid, n);
    case HULL_OP_SM:
    case HULL_OP_ALL:
        if (!grid_ok(grid)) return (size_t)-1;
        return counts_ws_bytes(grid, n) + sm_ws_bytes(grid);
    case HULL_OP_FBP:
        if (!grid_ok(grid) || !fbp_ok(fbp)) return (size_t)-1;
        return fbp_ws_layout(fbp, grid, nullptr).bytes;
    case HULL_OP_FBP_CUT:
        if (!grid_ok(grid) || !fbp_ok(fbp) || n > INT32_MAX) return (size_t)-1;
        return fbp_cut_ws_bytes(fbp, grid, n, nullptr);
    case HULL_OP_SC_BINNED: {
        if (!grid_ok(grid) || !fbp_ok(fbp) || n > INT32_MAX) return (size_t)-1;
        size_t bytes = 0;
        bsc_ws_layout(fbp, grid, n, nullptr, &bytes);
        return bytes;
    }
    default:
        return (size_t)-1;
    }
}

}  // namespace

// ---- shared with the batch, server and session runtime ----

size_t rules_ws_bytes(const hullmi_grid *g) { return sm_ws_bytes(g); }

size_t counting_ws_bytes(const hullmi_grid *g, int64_t n) { return counts_ws_bytes(g, n); }

bool params_ok(const hullmi_params *p)
{
    return p && std::isfinite(p->wepl_low) && std::isfinite(p->wepl_high) &&
           msc_args_ok(p->msc_n_t, p->msc_mode, p->nbr) &&
           sm_args_ok(p->sm_frac_num, p->sm_frac_den, p->sm_mode, p->sm_scope, p->nbr);
}

bool grid_valid(const hullmi_grid *g) { return grid_ok(g); }

bool hist_valid(const hullmi_histories *h) { return hist_ok(h); }

int masks_from_counts(const hullmi_grid *g, const hullmi_params *p, const int32_t *N,
                      const int32_t *M, uint8_t *sc, uint8_t *msc, uint8_t *sm, void *ws,
                      hipStream_t s)
{
    if (sc) k_sc_mask<<<blocks_for(voxels(g)), kBlock, 0, s>>>(N, sc, voxels(g));
    int rc = launch_status();
    if (rc == HULL_OK) rc = run_msc_mask(g, N, msc, p->msc_n_t, p->msc_mode, p->nbr, s);
    if (rc == HULL_OK)
        rc = run_sm_mask(g, M, sm, p->sm_frac_num, p->sm_frac_den, p->sm_mode, p->sm_scope, p->nbr,
                         ws, s);
    return rc;
}

int counts_accumulate(const hullmi_histories *h, const hullmi_grid *g, const hullmi_params *p,
                      int32_t *N, int32_t *M, hullmi_stats *stats, void *ws, size_t ws_bytes,
                      hipStream_t s)
{
    return run_counts(h, g, p->wepl_low, p->wepl_high, N, M, HULL_ACCUMULATE, stats, ws, ws_bytes, s,
                      CountOpts{});
}

void zero_counts(int32_t *N, int32_t *M, hullmi_stats *stats, int64_t V, hipStream_t s)
{
    fill_u32(N, 0u, V, s);
    fill_u32(M, 0u, V, s);
    fill_u64(stats, 0ull, (int64_t)(sizeof(hullmi_stats) / 8), s);
}

namespace {

// The ops whose call takes detector bins (the FDK parameters).
bool bins_op(int op)
{
    return op == HULL_OP_FBP || op == HULL_OP_FBP_CUT || op == HULL_OP_SC_BINNED;
}

}  // namespace

size_t job_ws_bytes(const hullmi_job &j)
{
    return ws_bytes_of(j.op, &j.grid, j.hist.n, bins_op(j.op) ? &j.fbp : nullptr);
}

int job_check(const hullmi_job &j)
{
    if (!hist_ok(&j.hist) || !grid_ok(&j.grid)) return HULL_EINVAL;
    const hullmi_params &p = j.params;
    switch (j.op) {
    case HULL_OP_SC:
        return j.N && std::isfinite(p.wepl_low) ? HULL_OK : HULL_EINVAL;
    case HULL_OP_MSC:
        return j.N && std::isfinite(p.wepl_low) && msc_args_ok(p.msc_n_t, p.msc_mode, p.nbr)
                   ? HULL_OK : HULL_EINVAL;
    case HULL_OP_SM:
        return j.M && std::isfinite(p.wepl_high) &&
                       sm_args_ok(p.sm_frac_num, p.sm_frac_den, p.sm_mode, p.sm_scope, p.nbr)
                   ? HULL_OK : HULL_EINVAL;
    case HULL_OP_ALL:
        if (!j.N || !j.M || !std::isfinite(p.wepl_low) || !std::isfinite(p.wepl_high))
            return HULL_EINVAL;
        if (j.msc_mask && !msc_args_ok(p.msc_n_t, p.msc_mode, p.nbr)) return HULL_EINVAL;
        if (j.sm_mask && !sm_args_ok(p.sm_frac_num, p.sm_frac_den, p.sm_mode, p.sm_scope, p.nbr))
            return HULL_EINVAL;
        return HULL_OK;
    case HULL_OP_FBP:
        return j.image && fbp_ok(&j.fbp) ? HULL_OK : HULL_EINVAL;
    case HULL_OP_FBP_CUT:
        return j.image && fbp_ok(&j.fbp) && j.bsc.cut_sigmas >= 0 && j.bsc.cut_sigmas <= 64 &&
                       j.hist.n <= INT32_MAX
                   ? HULL_OK : HULL_EINVAL;
    case HULL_OP_SC_BINNED:
        return j.bsc_mask && fbp_ok(&j.fbp) && bsc_ok(&j.bsc) && j.hist.n <= INT32_MAX
                   ? HULL_OK : HULL_EINVAL;
    default:
        return HULL_EINVAL;
    }
}

int job_run(const hullmi_job &j, void *ws, size_t ws_bytes, hipStream_t s, const CountOpts &o)
{
    const hullmi_params &p = j.params;
    switch (j.op) {
    case HULL_OP_SC:
        return sc_impl(&j.hist, &j.grid, p.wepl_low, j.N, j.sc_mask, j.flags, j.stats, ws, ws_bytes,
                       s, o);
    case HULL_OP_MSC:
        return msc_impl(&j.hist, &j.grid, p.wepl_low, p.msc_n_t, p.msc_mode, p.nbr, j.N,
                        j.msc_mask, j.flags, j.stats, ws, ws_bytes, s, o);
    case HULL_OP_SM:
        return sm_impl(&j.hist, &j.grid, p.wepl_high, p.sm_frac_num, p.sm_frac_den, p.sm_mode,
                       p.sm_scope, p.nbr, j.M, j.sm_mask, j.flags, j.stats, ws, ws_bytes, s, o);
    case HULL_OP_ALL:
        return all_impl(&j.hist, &j.grid, &p, j.N, j.M, j.sc_mask, j.msc_mask, j.sm_mask, j.flags,
                        j.stats, ws, ws_bytes, s, o);
    case HULL_OP_FBP:
        return fbp_impl(&j.hist, &j.grid, &j.fbp, j.image, j.fbp_mask, ws, ws_bytes, s);
    case HULL_OP_FBP_CUT:
        return fbp_cut_impl(&j.hist, &j.grid, &j.fbp, j.bsc.cut_sigmas, j.image, j.fbp_mask, ws,
                            ws_bytes, s);
    case HULL_OP_SC_BINNED:
        return bsc_impl(&j.hist, &j.grid, &j.fbp, &j.bsc, nullptr, nullptr, nullptr, j.bsc_mask,
                        j.bsc_stats, ws, ws_bytes, s);
    default:
        return HULL_EINVAL;
    }
}

size_t footprint_bytes(int op, const hullmi_grid *grid, int64_t n, const hullmi_fbp_params *fbp)
{
    if (op < HULL_OP_SC || op == HULL_OP_COUNT_LINES || op > HULL_OP_FBP_CUT || n < 0 ||
        n > INT32_MAX)
        return (size_t)-1;
    const size_t ws = ws_bytes_of(op, grid, n, fbp);
    if (ws == (size_t)-1) return ws;
    const size_t V = (size_t)voxels(grid);
    size_t out = 0;
    switch (op) {
    case HULL_OP_SC:
    case HULL_OP_MSC:
    case HULL_OP_SM: out = align_up(4 * V) + align_up(V); break;
    case HULL_OP_ALL: out = 2 * align_up(4 * V) + 3 * align_up(V); break;
    case HULL_OP_FBP:
    case HULL_OP_FBP_CUT: out = align_up(4 * V) + align_up(V); break;
    case HULL_OP_SC_BINNED: out = align_up(V); break;
    }
    return 8 * align_up(4 * (size_t)n) + out + align_up(sizeof(hullmi_stats)) +
           align_up(sizeof(hullmi_bsc_stats)) + align_up(ws);
}

}  // namespace hullmi

using namespace hullmi;

extern "C" {

int hull_abi_version(void) { return HULLMI_ABI_VERSION; }

const char *hull_strerror(int status)
{
    switch (status) {
    case HULL_OK: return "ok";
    case HULL_EINVAL: return "invalid argument";
    case HULL_ENOMEM: return "workspace too small";
    case HULL_EDEVICE: return "device launch failed";
    case HULL_EBUSY: return "busy";
    case HULL_ENOTSUP: return "not supported";
    case HULL_ETIMEDOUT: return "timed out";
    default: return "unknown status";
    }
}

size_t hull_workspace_bytes(int op, const hullmi_grid *grid, int64_t n, const hullmi_fbp_params *fbp)
{
    return ws_bytes_of(op, grid, n, fbp);
}

size_t hull_footprint_bytes(int op, const hullmi_grid *grid, int64_t n, const hullmi_fbp_params *fbp)
{
    return footprint_bytes(op, grid, n, fbp);
}

int hull_sc(const hullmi_histories *hist, const hullmi_grid *grid, float wepl_low, int32_t *N,
            uint8_t *mask, uint32_t flags, hullmi_stats *stats, void *ws, size_t ws_bytes,
            void *stream)
{
    return sc_impl(hist, grid, wepl_low, N, mask, flags, stats, ws, ws_bytes, as_stream(stream),
                   per_scan_opts());
}

int hull_msc(const hullmi_histories *hist, const hullmi_grid *grid, float wepl_low, int32_t n_t,
             int mode, int nbr, int32_t *N, uint8_t *mask, uint32_t flags, hullmi_stats *stats,
             void *ws, size_t ws_bytes, void *stream)
{
    return msc_impl(hist, grid, wepl_low, n_t, mode, nbr, N, mask, flags, stats, ws, ws_bytes,
                    as_stream(stream), per_scan_opts());
}

int hull_sm(const hullmi_histories *hist, const hullmi_grid *grid, float wepl_high, int32_t frac_num,
            int32_t frac_den, int mode, int scope, int nbr, int32_t *M, uint8_t *mask,
            uint32_t flags, hullmi_stats *stats, void *ws, size_t ws_bytes, void *stream)
{
    return sm_impl(hist, grid, wepl_high, frac_num, frac_den, mode, scope, nbr, M, mask, flags,
                   stats, ws, ws_bytes, as_stream(stream), per_scan_opts());
}

int hull_all(const hullmi_histories *hist, const hullmi_grid *grid, const hullmi_params *p,
             int32_t *N, int32_t *M, uint8_t *sc_mask, uint8_t *msc_mask, uint8_t *sm_mask,
             uint32_t flags, hullmi_stats *stats, void *ws, size_t ws_bytes, void *stream)
{
    return all_impl(hist, grid, p, N, M, sc_mask, msc_mask, sm_mask, flags, stats, ws, ws_bytes,
                    as_stream(stream), per_scan_opts());
}

// Sums the recorded event pairs per kernel (after the stream has finished).
static int prof_collect(const KernelProf &prof, float *ms, int32_t *launches)
{
    if (prof.failed) return HULL_EDEVICE;
    for (int k = 0; k < HULL_PROF_KERNELS; ++k) {
        ms[k] = 0.0f;
        if (launches) launches[k] = 0;
    }
    for (const KernelProf::Mark &m : prof.marks) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, m.a, m.b) != hipSuccess) return HULL_EDEVICE;
        ms[m.kernel] += t;
        if (launches) ++launches[m.kernel];
    }
    return HULL_OK;
}

// Waits for the profiled call's work (unless its arguments were refused and
// nothing was enqueued) and sums its event pairs.
static int prof_finish(int rc, hipStream_t s, const KernelProf &prof, float *ms, int32_t *launches)
{
    if (rc == HULL_EINVAL || rc == HULL_ENOMEM) return rc;
    const bool synced = hipStreamSynchronize(s) == hipSuccess;
    if (rc != HULL_OK) return rc;
    if (!synced) return HULL_EDEVICE;
    return prof_collect(prof, ms, launches);
}

int hull_count_profile(const hullmi_histories *hist, const hullmi_grid *grid,
                       const hullmi_params *p, int32_t *N, int32_t *M, uint32_t flags,
                       hullmi_stats *stats, void *ws, size_t ws_bytes, void *stream, float *ms,
                       int32_t *launches)
{
    if (!ms) return HULL_EINVAL;
    KernelProf prof;
    CountOpts o = per_scan_opts();   // the batches of hull_all, one after another
    o.prof = &prof;
    const int rc = all_impl(hist, grid, p, N, M, nullptr, nullptr, nullptr, flags, stats, ws,
                            ws_bytes, as_stream(stream), o);
    return prof_finish(rc, as_stream(stream), prof, ms, launches);
}

int hull_fbp_profile(const hullmi_histories *hist, const hullmi_grid *grid,
                     const hullmi_fbp_params *fbp, float *image, uint8_t *mask, void *ws,
                     size_t ws_bytes, void *stream, float *ms, int32_t *launches)
{
    if (!ms) return HULL_EINVAL;
    KernelProf prof;
    const int rc = fbp_impl(hist, grid, fbp, image, mask, ws, ws_bytes, as_stream(stream), &prof);
    return prof_finish(rc, as_stream(stream), prof, ms, launches);
}

int hull_fbp(const hullmi_histories *hist, const hullmi_grid *grid, const hullmi_fbp_params *fbp,
             float *image, uint8_t *mask, void *ws, size_t ws_bytes, void *stream)
{
    return fbp_impl(hist, grid, fbp, image, mask, ws, ws_bytes, as_stream(stream));
}

int hull_sc_binned(const hullmi_histories *hist, const hullmi_grid *grid,
                   const hullmi_fbp_params *bins, const hullmi_bsc_params *params,
                   uint32_t *kept_n, int64_t *kept_sum, uint8_t *carved, uint8_t *mask,
                   hullmi_bsc_stats *stats, void *ws, size_t ws_bytes, void *stream)
{
    return bsc_impl(hist, grid, bins, params, kept_n, kept_sum, carved, mask, stats, ws, ws_bytes,
                    as_stream(stream));
}

int hull_fbp_cut(const hullmi_histories *hist, const hullmi_grid *grid, const hullmi_fbp_params *fbp,
                 int32_t cut_sigmas, float *image, uint8_t *mask, void *ws, size_t ws_bytes,
                 void *stream)
{
    return fbp_cut_impl(hist, grid, fbp, cut_sigmas, image, mask, ws, ws_bytes, as_stream(stream));
}

int hull_count_lines(const int32_t *q_in, const int32_t *q_out, int64_t n, const hullmi_grid *grid,
                     int32_t *counts, uint32_t flags, hullmi_stats *stats, void *ws,
                     size_t ws_bytes, void *stream)
{
    (void)ws; (void)ws_bytes;
    if (!grid_ok(grid) || !counts || n < 0 || n > INT32_MAX) return HULL_EINVAL;
    if (n > 0 && (!q_in || !q_out)) return HULL_EINVAL;
    hipStream_t s = as_stream(stream);
    if (!(flags & HULL_ACCUMULATE)) {
        fill_u32(counts, 0u, voxels(grid), s);
        fill_u64(stats, 0ull, stats ? 6 : 0, s);
    }
    if (n > 0)
        k_walk_lines<<<blocks_for(n), kBlock, 0, s>>>(q_in, q_out, n, grid->nx, grid->ny, grid->nz,
                                                     counts, stats);
    return launch_status();
}

int hull_quantize(const hullmi_histories *hist, const hullmi_grid *grid, int32_t *status,
                  int32_t *q_in, int32_t *q_out, void *stream)
{
    if (!hist_ok(hist) || !grid_ok(grid)) return HULL_EINVAL;
    if (hist->n > 0 && (!status || !q_in || !q_out)) return HULL_EINVAL;
    if (hist->n > 0)
        k_quantize<<<blocks_for(hist->n), kBlock, 0, as_stream(stream)>>>(*hist, dev_grid(grid),
                                                                         status, q_in, q_out);
    return launch_status();
}

}  // extern "C"
