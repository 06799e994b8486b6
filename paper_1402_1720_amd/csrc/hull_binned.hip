// Slice-binned counting kernels. A batch of histories goes through:
//   classify : class, geometry, whether A_i is empty (exact), a z-slice range
//              that covers A_i, a length class per slice, per-block counts of
//              the sub-bins (class, slice, length)
//   scan     : per sub-bin offsets of every block
//   plan     : sub-bin starts, slice (tile) starts, ranges of equal estimated
//              work over the sorted item list
//   scatter  : (history, slice) items in sub-bin order, each a copy of the
//              history's 16-byte packed endpoint record
//   setup    : each tile item's endpoints replaced by its packed slice-walk
//              state
//   walk     : persistent workgroups; each range is cut at slice boundaries
//              into segments, each accumulated in a 16-bit LDS copy of its
//              slice and written to its own partial slot
//   reduce   : the partial slots of every slice summed into N / M
//   overflow : lines spanning many slices walked with global atomics
// Counts are integers, so the result does not depend on any of this order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hull_binned.h"
#include "hull_device.h"

namespace hullmi {

__device__ __forceinline__ void add_stats(hullmi_stats *st, int idx, unsigned long long v)
{
    if (v) atomicAdd(reinterpret_cast<unsigned long long *>(st) + idx, v);
}

// Block-wide sum (wave64, up to 1024 threads); the result is valid in thread 0.
__device__ __forceinline__ unsigned long long block_sum(unsigned long long v, unsigned long long *sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    unsigned long long s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    return s;
}

// Column of block b in the per-block count rows: blocks ordered by b % r,
// then b / r (r = the run stride, 8 by default). Runs of one sub-bin that lie
// next to each other in the item list then come from blocks r apart (r x 8192
// histories), so the 64 items of a walk wave hold lines of several gantry
// angles instead of one, which made the walk about 10% faster on the
// 200x200x32 scan (strides of 16 to 256 gave the same). The order inside a
// sub-bin changes no count.
__device__ __forceinline__ int blk_col(int b, int nblk, int r)
{
    const int x = b % r;
    int before = 0;
    for (int i = 0; i < x; ++i) before += (nblk - i + r - 1) / r;
    return before + b / r;
}

// Number of entries of the non-decreasing array a[lo..hi) that are <= x.
__device__ __forceinline__ int count_le(const uint32_t *a, int lo, int hi, uint32_t x)
{
    int l = lo, r = hi;
    while (l < r) {
        const int m = (l + r) >> 1;
        if (a[m] <= x) l = m + 1; else r = m;
    }
    return l - lo;
}

// Partial slot of the segment that starts at item x: the number of range and
// slice boundaries at or before x. Distinct non-empty segments get distinct
// slots, at most ranges + slices of them.
__device__ __forceinline__ int slot_of(const BinWs &w, int nranges, uint32_t x)
{
    return count_le(w.range_start, 1, nranges + 1, x) + count_le(w.tile_start, 1, w.ntiles, x);
}

// Endpoints of a tile line, every coordinate in [-kPackLimit, kPackLimit),
// as six 21-bit two's-complement fields, three in each 64-bit half: one
// 16-byte store per item in the scatter instead of three 8-byte ones.
__device__ __forceinline__ uint4 pack_line(const int q[6])
{
    auto f = [](int v) { return (uint64_t)(uint32_t)v & 0x1fffffull; };
    const uint64_t lo = f(q[0]) | f(q[1]) << 21 | f(q[2]) << 42;
    const uint64_t hi = f(q[3]) | f(q[4]) << 21 | f(q[5]) << 42;
    return make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
}

__device__ __forceinline__ void unpack_line(const uint4 r, int q[6])
{
    const uint64_t lo = (uint64_t)r.x | (uint64_t)r.y << 32;
    const uint64_t hi = (uint64_t)r.z | (uint64_t)r.w << 32;
    // the field's top bit to bit 63, then an arithmetic shift back
    auto g = [](uint64_t h, int off) { return (int)((int64_t)(h << (43 - off)) >> 43); };
    q[0] = g(lo, 0); q[1] = g(lo, 21); q[2] = g(lo, 42);
    q[3] = g(hi, 0); q[4] = g(hi, 21); q[5] = g(hi, 42);
}

// Slice-walk state in 16 bytes: d; the tile counters of the first and the
// last voxel of the slice part (17 bits each, a tile has at most 81912
// counters: the low 16 bits in the second word, bit 16 in bits 22 and 23 of
// the third); |Dy| and |Dx| (below 2^19 on a tile line), the signs of the x
// and y steps and a flag for a slice the line does not meet.
// Bit 24 of the third word marks a line whose d is never zero in the slice
// (odd d, or no voxel corner on the projected line): the walk may take the
// corner-free loop for it.
constexpr uint32_t kStateEmpty = 1u << 21;
constexpr uint32_t kStateNoCorner = 1u << 24;

__device__ __forceinline__ uint4 pack_state(const SliceState &s, bool no_corner)
{
    const bool e = s.first < 0;
    const uint4 r = make_uint4((uint32_t)s.d, ((uint32_t)s.first & 0xffffu) | (uint32_t)s.last << 16,
                               (uint32_t)s.ay | (uint32_t)(s.sx < 0) << 19 | (uint32_t)(s.sy < 0) << 20 |
                                   ((uint32_t)s.first >> 16) << 22 | ((uint32_t)s.last >> 16) << 23 |
                                   (no_corner ? kStateNoCorner : 0u),
                               (uint32_t)s.ax);
    return make_uint4(e ? 0u : r.x, e ? 0u : r.y, e ? kStateEmpty : r.z, e ? 0u : r.w);
}

// Approximate number of voxels of the line inside slice k (FP32, only used to
// group lines of similar length), as a class in [0, nl): the in-plane extent
// of the part of the slab that lies in the slice.
__device__ __forceinline__ int length_class(const LineSlab &b, float rdz, int k, int nl, float rlw)
{
    float tlo = b.tlo, thi = b.thi;
    if (b.d[2] != 0.0f) {
        const float t0 = ((float)k - b.p[2]) * rdz, t1 = ((float)(k + 1) - b.p[2]) * rdz;
        tlo = fmaxf(tlo, fminf(t0, t1));
        thi = fminf(thi, fmaxf(t0, t1));
    }
    const float len = (fabsf(b.d[0]) + fabsf(b.d[1])) * fmaxf(thi - tlo, 0.0f) + 1.0f;
    const float c = fminf(len * rlw, (float)(nl - 1));
    return c > 0.0f ? (int)c : 0;
}

// Whether the walk cannot rule out a voxel corner on the line's projection
// (the state flag the set-up writes, from the line alone): d is even, i.e. the
// x and y steps have the same sign, and the corner test cannot clear it.
// Nearly all such lines come from the gantry angles along the grid axes,
// where a line starts on a grid face and spans whole voxels in x or y.
__device__ __forceinline__ bool may_meet_corner(const int q[6])
{
    const int32_t dx = q[3] - q[0], dy = q[4] - q[1];
    return ((dx < 0) == (dy < 0)) && !corner_free(q[0], q[1], dx, dy);
}

// Quantised endpoints of history i (batch-relative index into h, whose
// arrays start at h0): kGeoOk or the reason the history is skipped. c, s and
// bits cache the cosine and sine of the last angle seen (histories come in
// long runs of one gantry angle, and equal angle bits give equal c, s).
__device__ __forceinline__ int history_line(float xi, float yi, float zi, float xo, float yo,
                                            float zo, float a, const DevGrid &g, uint32_t &bits,
                                            float &c, float &s, int q[6])
{
    int st = (isfinite(xi) && isfinite(yi) && isfinite(zi) && isfinite(xo) && isfinite(yo) &&
              isfinite(zo) && isfinite(a))
                 ? kGeoOk
                 : kGeoNonFinite;
    if (st == kGeoOk) {
        if (__float_as_uint(a) != bits) {
            deg_cos_sin(a, c, s);
            bits = __float_as_uint(a);
        }
        st = quantize_point(c, s, xi, yi, zi, g, q[0], q[1], q[2]);
        if (st == kGeoOk) st = quantize_point(c, s, xo, yo, zo, g, q[3], q[4], q[5]);
        if (st == kGeoOk && q[0] == q[3] && q[1] == q[4] && q[2] == q[5]) st = kGeoDegenerate;
    }
    return st;
}

// Every lane loads every field of every history of its block, in range or
// not (an index past the batch is clamped to its last history, and what a
// lane computes there is dropped), and stores its three words for each
// (the per-history arrays are padded to whole blocks): with no memory
// operation under a lane-dependent condition the compiler counts the loads in
// flight exactly, and a history's loads no longer wait for the previous
// history's stores. A wave's 64 consecutive histories share the cache lines
// of every field, so loading the geometry of the histories outside the
// counted classes costs little traffic.
__global__ void __launch_bounds__(kBinThreads)
k_bin_classify(hullmi_histories h, int64_t h0, int64_t nb, DevGrid g, float e_low, float e_high,
               int use_low, int use_high, int tile_ok, BinWs w, hullmi_stats *st)
{
    __shared__ uint32_t lh[kMaxSubBins];
    __shared__ unsigned long long red[16];
    for (int b = threadIdx.x; b < w.nsub; b += blockDim.x) lh[b] = 0;
    __syncthreads();
    unsigned long long nl = 0, nh = 0, nsk = 0, nmi = 0;
    uint32_t trig_bits = 0x7fc00001u;   // a NaN: finite angles never match it
    float tc = 1.0f, ts = 0.0f;
    const int64_t base = (int64_t)blockIdx.x * kHistPerBlock;
    auto hist_at = [&](int r) { return base + (int64_t)r * kBinThreads + threadIdx.x; };
    auto src = [&](int r) { return h0 + min(hist_at(r), nb - 1); };
    struct Geo { float xi, yi, zi, xo, yo, zo, a, wv; };
    auto fetch = [&](int64_t i, Geo &f) {
        f.xi = h.x_in[i]; f.yi = h.y_in[i]; f.zi = h.z_in[i];
        f.xo = h.x_out[i]; f.yo = h.y_out[i]; f.zo = h.z_out[i]; f.a = h.angle_deg[i];
        f.wv = h.wepl[i];
    };
    // the next history's fields are in flight while the current one is classified
    Geo nxt;
    fetch(src(0), nxt);
    for (int r = 0; r < kHistPerThread; ++r) {
        const int64_t j = hist_at(r);
        const bool live = j < nb;
        const Geo cf = nxt;
        fetch(src(r + 1 < kHistPerThread ? r + 1 : r), nxt);
        const float wv = cf.wv;
        uint32_t meta = 0;
        // every history's record and length word is written (zeros when
        // unused), so that the block writes whole cache lines
        uint4 rec = make_uint4(0u, 0u, 0u, 0u);
        uint32_t lp = 0;
        if (!live) {
        } else if (!isfinite(wv)) {
            ++nsk;
        } else {
            const bool low = use_low && wv < e_low;
            const bool high = use_high && wv > e_high;
            if (low || high) {
                int q[6];
                const int stg = history_line(cf.xi, cf.yi, cf.zi, cf.xo, cf.yo, cf.zo, cf.a, g,
                                             trig_bits, tc, ts, q);
                if (stg != kGeoOk) {
                    ++nsk;
                } else {
                    if (low) ++nl; else ++nh;
                    int k0, k1;
                    // whether A_i is empty (from the slab where it is clear, else
                    // exactly), then a slice range that covers A_i (a slice the
                    // line does not meet gives an empty item)
                    LineSlab sb;
                    line_slab(q[0], q[1], q[2], q[3], q[4], q[5], g.nx, g.ny, g.nz, sb);
                    int meets = slab_meets(sb, q[0], q[1], q[2], q[3], q[4], q[5], g.nx, g.ny, g.nz);
                    if (meets < 0)
                        meets = line_meets_grid(q[0], q[1], q[2], q[3], q[4], q[5], g.nx, g.ny, g.nz);
                    if (!meets) {
                        ++nmi;
                    } else {
                        slab_z_cover(sb, g.nz, k0, k1);
                        const int cls = low ? 0 : 1;
                        const int ns = k1 - k0 + 1;
                        meta = kMetaValid | (cls ? kMetaHigh : 0u) | ((uint32_t)ns << 12) | (uint32_t)k0;
                        // the tile walk keeps its decision variable in 32 bits: that
                        // needs |D| < 2^19 on x and y, else the global walk takes the line
                        const int64_t adx = (int64_t)q[3] - q[0], ady = (int64_t)q[4] - q[1];
                        const bool wide = max(adx < 0 ? -adx : adx, ady < 0 ? -ady : ady) >= (int64_t(1) << 19);
                        bool packs = true;
                        for (int c = 0; c < 6; ++c) packs &= q[c] >= -kPackLimit && q[c] < kPackLimit;
                        if (!tile_ok || ns > kMaxSlicesPerLine || wide || !packs) {
                            // the global walk quantises the history again
                            meta |= kMetaOverflow;
                            atomicAdd(&lh[w.nsub - 2 + cls], 1u);
                        } else {
                            rec = pack_line(q);
                            const float rdz = sb.d[2] != 0.0f ? __builtin_amdgcn_rcpf(sb.d[2]) : 0.0f;
                            const float rlw = __builtin_amdgcn_rcpf((float)w.lwidth);
                            // a line that may pass through a voxel corner makes its
                            // whole wave take the longer walk loop: such lines get
                            // the last length class to themselves
                            const int corner_cls = may_meet_corner(q) ? w.nl - 1 : -1;
                            for (int k = k0; k <= k1; ++k) {
                                const int lc = corner_cls >= 0 ? corner_cls
                                                               : length_class(sb, rdz, k, w.nl - 1, rlw);
                                lp |= (uint32_t)lc << (4 * (k - k0));
                                atomicAdd(&lh[(cls * w.nz + k) * w.nl + lc], 1u);
                            }
                        }
                    }
                }
            }
        }
        w.hrec[j] = rec;
        w.lpack[j] = lp;
        w.meta[j] = meta;
    }
    __syncthreads();
    const int col = blk_col((int)blockIdx.x, w.nblk, w.run_stride);
    for (int b = threadIdx.x; b < w.nsub; b += blockDim.x)
        w.blk[(int64_t)col * w.nsub + b] = lh[b];
    if (st) {
        unsigned long long v;
        v = block_sum(nl, red);  if (threadIdx.x == 0) add_stats(st, 0, v);
        v = block_sum(nh, red);  if (threadIdx.x == 0) add_stats(st, 1, v);
        v = block_sum(nsk, red); if (threadIdx.x == 0) add_stats(st, 2, v);
        v = block_sum(nmi, red); if (threadIdx.x == 0) add_stats(st, 3, v);
    }
}

// Exclusive scan of get(0..n) into out[0..n) by one block (wave64 shuffles
// and one LDS pass over the wave totals); returns the total in every thread.
template <typename T, class Get, class Put>
__device__ T block_exclusive_scan_to(int n, Get get, Put put, T *sh)
{
    const int nt = (int)blockDim.x;
    const int per = (n + nt - 1) / nt;
    const int b0 = threadIdx.x * per;
    T s = 0;
    for (int i = 0; i < per && b0 + i < n; ++i) s += get(b0 + i);
    // inclusive scan within the wave
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T inc = s;
    for (int o = 1; o < 64; o <<= 1) {
        const T v = __shfl_up(inc, o, 64);
        if (lane >= o) inc += v;
    }
    if (lane == 63) sh[wid] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = 0;
        for (int i = 0; i < (nt >> 6); ++i) { const T v = sh[i]; sh[i] = acc; acc += v; }
        sh[nt >> 6] = acc;
    }
    __syncthreads();
    T acc = sh[wid] + inc - s;
    for (int i = 0; i < per && b0 + i < n; ++i) {
        const T v = get(b0 + i);
        put(b0 + i, acc);
        acc += v;
    }
    const T total = sh[nt >> 6];
    __syncthreads();
    return total;
}

template <typename T, class Get>
__device__ T block_exclusive_scan(int n, Get get, T *out, T *sh)
{
    return block_exclusive_scan_to<T>(n, get, [&](int i, T v) { out[i] = v; }, sh);
}

// The per-block counts are a matrix of block columns (rows, in run order) by
// sub-bins, so that a classification block writes, and a scatter block
// reads, one contiguous row. Each sub-bin's exclusive scan over the columns
// runs in two steps: within groups of kScanGroup columns (a thread per
// sub-bin, reading down its column, a wave reading 64 neighbouring sub-bins
// of a row at a time), then over the group sums.
__global__ void __launch_bounds__(256) k_bin_scan_groups(BinWs w)
{
    const int g = blockIdx.x;
    const int c0 = g * kScanGroup;
    const int nc = min(kScanGroup, w.nblk - c0);
    for (int s = threadIdx.x; s < w.nsub; s += blockDim.x) {
        uint32_t v[kScanGroup];
#pragma unroll
        for (int i = 0; i < kScanGroup; ++i)
            v[i] = i < nc ? w.blk[(int64_t)(c0 + i) * w.nsub + s] : 0u;
        uint32_t acc = 0;
#pragma unroll
        for (int i = 0; i < kScanGroup; ++i) {
            if (i < nc) w.boff[(int64_t)(c0 + i) * w.nsub + s] = acc;
            acc += v[i];
        }
        w.gsum[(int64_t)s * w.ngroups + g] = acc;
    }
}

// One wave per sub-bin: exclusive scan of its group sums, 64 groups at a
// time; the group offsets are written group-major (a scatter block reads its
// group's row), the total per sub-bin beside them.
__global__ void __launch_bounds__(256) k_bin_scan_sums(BinWs w)
{
    const int s = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (s >= w.nsub) return;   // whole waves
    const int lane = threadIdx.x & 63;
    uint32_t carry = 0;
    for (int g0 = 0; g0 < w.ngroups; g0 += 64) {
        const int g = g0 + lane;
        const uint32_t v = g < w.ngroups ? w.gsum[(int64_t)s * w.ngroups + g] : 0u;
        uint32_t inc = v;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        if (g < w.ngroups) w.goff[(int64_t)g * w.nsub + s] = carry + inc - v;
        carry += __shfl(inc, 63, 64);
    }
    if (lane == 0) w.sub_total[s] = carry;
}

__device__ __forceinline__ unsigned long long item_work(const BinWs &w, int sub)
{
    const int lc = sub % w.nl;
    return kWorkPerItem + (unsigned long long)lc * w.lwidth + w.lwidth / 2;
}

// Single block: sub-bin and slice starts, then the ranges: P0 = max(min_ranges,
// ceil(I / kItemsPerRange)) ranges of equal estimated work, each split again
// where it holds more than kItemsPerRange items, so that a range never adds
// more than 65535 to one 16-bit counter (an item adds at most 1 to a voxel).
__global__ void __launch_bounds__(1024) k_bin_plan(BinWs w)
{
    __shared__ unsigned long long shw[17];
    __shared__ uint32_t shu[17];
    __shared__ unsigned long long wp[kMaxSubBins];   // the work prefix, for the searches
    const int nreg = w.ntiles * w.nl;
    const uint32_t total = block_exclusive_scan<uint32_t>(
        w.nsub, [&](int i) { return w.sub_total[i]; }, w.sub_start, shu);
    if (threadIdx.x == 0) w.sub_start[w.nsub] = total;
    const unsigned long long wtot = block_exclusive_scan<unsigned long long>(
        nreg, [&](int i) { return (unsigned long long)w.sub_total[i] * item_work(w, i); },
        w.wprefix, shw);
    if (threadIdx.x == 0) w.wprefix[nreg] = wtot;
    __syncthreads();
    for (int i = threadIdx.x; i <= nreg; i += blockDim.x) wp[i] = w.wprefix[i];
    __syncthreads();
    const uint32_t I = w.sub_start[nreg];
    for (int t = threadIdx.x; t <= w.ntiles; t += blockDim.x) w.tile_start[t] = w.sub_start[t * w.nl];
    uint32_t P0 = (I + kItemsPerRange - 1) / kItemsPerRange;
    if (P0 < (uint32_t)w.min_ranges) P0 = w.min_ranges;
    // coarse bounds: first item whose work prefix reaches r * wtot / P0
    for (uint32_t r = threadIdx.x; r <= P0; r += blockDim.x) {
        uint32_t item;
        if (r == 0) item = 0;
        else if (r == P0 || wtot == 0) item = I;
        else {
            const unsigned long long X = (unsigned long long)r * wtot / P0;
            int l = 0, h = nreg;   // last sub-bin s with wprefix[s] <= X
            while (l < h) {
                const int m = (l + h + 1) >> 1;
                if (wp[m] <= X) l = m; else h = m - 1;
            }
            const unsigned long long per = item_work(w, l);
            unsigned long long k = (X - wp[l] + per - 1) / per;
            if (k > w.sub_total[l]) k = w.sub_total[l];
            item = min(w.sub_start[l] + (uint32_t)k, I);
        }
        w.range_coarse[r] = item;
    }
    __syncthreads();
    // pieces per coarse range and their starts
    auto pieces = [&](int r) {
        const uint32_t cnt = w.range_coarse[r + 1] - w.range_coarse[r];
        return cnt > (uint32_t)kItemsPerRange ? (cnt + kItemsPerRange - 1) / kItemsPerRange : 1u;
    };
    const uint32_t P = block_exclusive_scan<uint32_t>((int)P0, pieces, w.range_piece, shu);
    for (uint32_t r = threadIdx.x; r < P0; r += blockDim.x) {
        const uint32_t a = w.range_coarse[r], cnt = w.range_coarse[r + 1] - a;
        const uint32_t np = pieces((int)r), o = w.range_piece[r];
        for (uint32_t j = 0; j < np; ++j)
            w.range_start[o + j] = a + (uint32_t)((unsigned long long)cnt * j / np);
    }
    if (threadIdx.x == 0) {
        w.range_start[P] = I;
        w.ctl[kCtlRanges] = (int32_t)P;
        w.ctl[kCtlItems] = (int32_t)I;
        w.ctl[kCtlOverflowStart] = (int32_t)w.sub_start[w.nsub - 2];
        w.ctl[kCtlOverflowCount] = (int32_t)(w.sub_total[w.nsub - 2] + w.sub_total[w.nsub - 1]);
        w.ctl[kCtlOverflowLow] = (int32_t)w.sub_total[w.nsub - 2];
        w.ctl[kCtlCoarse] = (int32_t)P0;
    }
}

// Writes the items of one classification block (8192 histories) to their
// runs: an LDS cursor per sub-bin, started at where this block's run of the
// sub-bin begins. A thread takes eight histories and loads all of their meta
// words, length classes and packed records before it stores anything: vector
// memory operations retire in order, so a load issued after a scattered store
// would wait for that store, and the stores would set the pace.
__global__ void __launch_bounds__(kScatterThreads) k_bin_scatter(int64_t nb, BinWs w)
{
    __shared__ uint32_t cur[kMaxSubBins];
    const int col = blk_col((int)blockIdx.x, w.nblk, w.run_stride);
    const int64_t row = (int64_t)col * w.nsub, grow = (int64_t)(col / kScanGroup) * w.nsub;
    for (int b = threadIdx.x; b < w.nsub; b += blockDim.x)
        cur[b] = w.sub_start[b] + w.goff[grow + b] + w.boff[row + b];
    __syncthreads();
    constexpr int R = kHistPerBlock / kScatterThreads;
    const int64_t base = (int64_t)blockIdx.x * kHistPerBlock + threadIdx.x;
    uint32_t m[R], lp[R];
    uint4 rec[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t j = base + (int64_t)r * kScatterThreads;
        m[r] = j < nb ? w.meta[j] : 0u;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t j = base + (int64_t)r * kScatterThreads;
        // the record of an unclassified history is read but not used
        lp[r] = j < nb ? w.lpack[j] : 0u;
        rec[r] = j < nb ? w.hrec[j] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!(m[r] & kMetaValid)) continue;
        const int cls = (m[r] & kMetaHigh) ? 1 : 0;
        if (m[r] & kMetaOverflow) {
            // the overflow walk reads the full record by history
            const uint32_t j = (uint32_t)(base + (int64_t)r * kScatterThreads);
            w.item[atomicAdd(&cur[w.nsub - 2 + cls], 1u)] = make_uint4(j, 0u, 0u, 0u);
        } else {
            const int k0 = (int)(m[r] & 0xfffu), ns = (int)((m[r] >> 12) & 0xfffu);
            for (int k = k0; k < k0 + ns; ++k) {
                const int lc = (int)((lp[r] >> (4 * (k - k0))) & 0xfu);
                w.item[atomicAdd(&cur[(cls * w.nz + k) * w.nl + lc], 1u)] = rec[r];
            }
        }
    }
}

// Replaces the endpoints of every tile item by its slice-walk state (one item
// per lane, grid-stride over the items counted on the device), so that the
// walk's lanes only run the loop.
__global__ void __launch_bounds__(256) k_item_setup(BinWs w, int nx, int ny)
{
    extern __shared__ uint32_t ts[];   // the slice tile starts
    for (int t = threadIdx.x; t <= w.ntiles; t += blockDim.x) ts[t] = w.tile_start[t];
    __syncthreads();
    const int n = w.ctl[kCtlItems];
    const int stride = gridDim.x * blockDim.x;
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    // a thread's items increase, so its slice tile only moves forward; the
    // next item's record is in flight while the current one is set up
    int t = p < n ? count_le(ts, 0, w.ntiles, (uint32_t)p) - 1 : 0;
    int k = t % w.nz;   // the slice of tile t (tiles are class-major)
    uint4 nxt = p < n ? w.item[p] : make_uint4(0u, 0u, 0u, 0u);
    for (; p < n; p += stride) {
        const uint4 cur = nxt;
        if (p + stride < n) nxt = w.item[p + stride];
        while (ts[t + 1] <= (uint32_t)p) {   // slice tile of p
            ++t;
            k = k + 1 == w.nz ? 0 : k + 1;
        }
        int q[6];
        unpack_line(cur, q);
        SliceState st;
        slice_state_tile(q[0], q[1], q[2], q[3], q[4], q[5], nx, ny, w.stride, k, st);
        const bool nc = (st.d & 1) || corner_free(q[0], q[1], q[3] - q[0], q[4] - q[1]);
        w.item[p] = pack_state(st, nc);
    }
}

// The walk loops issue their ds_add_u32 from inline assembly, which the
// compiler's wait counting does not see: a plain barrier after them could let
// another wave read a counter before the last adds land. Every barrier that
// follows the assembly loops goes through this, which waits for the wave's
// outstanding LDS operations first.
__device__ __forceinline__ void barrier_after_asm_lds()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __syncthreads();
}

// Persistent workgroups over the coarse ranges of equal estimated work (dealt
// round-robin); a coarse range is cut at its pieces' and at slice boundaries
// into segments, each accumulated in the LDS copy of its slice and written to
// its partial slot. A workgroup walks every piece of its coarse ranges, so the
// work stays even when long ranges are split. Items carry their slice-walk
// state (k_item_setup), so a lane only runs the loop; the next item's state is
// loaded while the current one is walked.
__global__ void __launch_bounds__(kTileThreads) k_walk_tiles(BinWs w, int nx, int ny)
{
    extern __shared__ uint32_t lds[];   // tile (slot_words), then 2 control words
    uint32_t *tile = lds;
    uint32_t *seg = lds + w.slot_words;
    const int nranges = w.ctl[kCtlRanges];
    const int ncoarse = w.ctl[kCtlCoarse];
    // LDS byte address of the tile (the low 32 bits of a local pointer)
    const uint32_t tile_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint32_t *)tile;
    for (int r = blockIdx.x; r < ncoarse; r += gridDim.x) {
        uint32_t x = w.range_coarse[r];
        const uint32_t b = w.range_coarse[r + 1];
        while (x < b) {
            if (threadIdx.x == 0) {
                const int t = count_le(w.tile_start, 0, w.ntiles, x) - 1;   // slice holding x
                const int p = count_le(w.range_start, 0, nranges + 1, x) - 1;   // piece holding x
                seg[0] = min(min(b, w.tile_start[t + 1]), w.range_start[p + 1]);
                seg[1] = (uint32_t)slot_of(w, nranges, x);
            }
            for (int i = threadIdx.x; i < w.slot_words; i += blockDim.x) tile[i] = 0;
            __syncthreads();
            const uint32_t y = seg[0], slot = seg[1];
            // the workgroup takes the items S at a time, in groups of 256 for
            // each four waves: lane l of the group's wave q takes item 4 l + q,
            // so that a wave's 64 lines come from across the 256 (from about
            // twenty item runs, i.e. classification blocks and gantry angles)
            // rather than from five neighbouring runs, and fewer of its LDS
            // adds meet in one bank; each 64-byte piece of the item list is
            // still read by one group at one time. Groups of 16 waves spread
            // the lines further but read each cache line from eight waves and
            // were slower. The next item's record is in flight while the
            // current line is walked.
            const uint32_t S = blockDim.x;
            uint32_t it = x + (threadIdx.x & ~255u) + (threadIdx.x & 63) * 4 + ((threadIdx.x >> 6) & 3);
            uint4 c = make_uint4(0u, 0u, kStateEmpty, 0u);
            if (it < y) c = w.item[it];
            while (it < y) {
                const uint4 a = c;
                if (it + S < y) c = w.item[it + S];
                const bool live = !(a.z & kStateEmpty);   // a slice the line meets
                const int32_t incx = (int32_t)((a.z & 0x7ffffu) << 11);
                const int32_t incy = -(int32_t)(a.w << 11);
                const int32_t ox = (a.z >> 19) & 1u ? -2 : 2;
                const int32_t oy = (a.z >> 20) & 1u ? -2 * w.stride : 2 * w.stride;
                const int32_t off = (int32_t)(tile_base + 2 * ((a.y & 0xffffu) | ((a.z >> 22) & 1u) << 16));
                const int32_t last = (int32_t)(tile_base + 2 * ((a.y >> 16) | ((a.z >> 23) & 1u) << 16));
                // when no live lane's line can pass through a voxel corner
                // (nearly every wave), the wave takes the shorter loop
                // the first step adds to the half of the first counter's word
                const uint32_t val = (off & 2) ? 65536u : 1u;
                if (__all(!live || (a.z & kStateNoCorner))) {
                    if (live) {
                        // word-address increments of x and y steps from the starting
                        // half (first steps of a round) and from the other half
                        // (second steps): counter L + sx or L + sy S (S odd) against
                        // word L >> 1
                        const int32_t p0 = (off >> 1) & 1;
                        const int32_t S = w.stride;
                        const bool xp = ox > 0, yp = oy > 0;
                        auto dx = [&](int32_t p) { return xp ? (p ? 4 : 0) : (p ? 0 : -4); };
                        auto dy = [&](int32_t p) {
                            return yp ? (p ? 2 * (S + 1) : 2 * (S - 1)) : (p ? -2 * (S - 1) : -2 * (S + 1));
                        };
                        const bool last_first = (((last >> 1) & 1) == p0);
                        const int32_t lw = last & ~3;
                        walk_slice_lds16_nocorner_w((int32_t)a.x, off & ~3, last_first ? lw : -1,
                                                    last_first ? -1 : lw, incx, incy, dx(p0), dy(p0),
                                                    dx(1 - p0), dy(1 - p0), val, nx + ny);
                    }
                } else if (live) {
                    walk_slice_lds16((int32_t)a.x, off, last, incx, incy, ox, oy, val, nx + ny);
                }
                it += S;
            }
            barrier_after_asm_lds();
            uint4 *dst = reinterpret_cast<uint4 *>(w.partial + (int64_t)slot * w.slot_words);
            const uint4 *src = reinterpret_cast<const uint4 *>(tile);
            for (int i = threadIdx.x; i < w.slot_words / 4; i += blockDim.x) dst[i] = src[i];
            x = y;
            __syncthreads();
        }
    }
}

// Adds the partial slots of every slice into N or M; the sum of what is added
// is the number of voxel visits of the class. A thread owns four consecutive
// words (eight counters) of the tile and reads them from every slot of the
// slice as one 16-byte load (slots are padded to a multiple of four words),
// four slots in flight at a time.
__global__ void __launch_bounds__(256) k_reduce_tiles(BinWs w, int plane, int *N, int *M, hullmi_stats *st)
{
    __shared__ uint32_t slots[256];
    __shared__ int r0;
    __shared__ unsigned long long red[16];
    const int t = blockIdx.y;
    const int cls = t / w.nz, k = t % w.nz;
    const uint32_t ta = w.tile_start[t], tb = w.tile_start[t + 1];
    if (ta == tb) return;   // uniform across the block
    const int nranges = w.ctl[kCtlRanges];
    const int wd = 4 * (blockIdx.x * blockDim.x + threadIdx.x);   // first of four words
    uint32_t lo[4] = {0u, 0u, 0u, 0u}, hi[4] = {0u, 0u, 0u, 0u};
    if (threadIdx.x == 0) r0 = count_le(w.range_start, 0, nranges + 1, ta) - 1;
    __syncthreads();
    // ranges overlapping [ta, tb), 256 at a time, one per thread: the ranges
    // that start before tb are a prefix of them (starts never decrease)
    for (int rb = r0;; rb += 256) {
        const int r = rb + (int)threadIdx.x;
        const bool in = r < nranges && w.range_start[r] < tb;
        uint32_t sl = 0xffffffffu;   // empty segment: nothing to add
        if (in) {
            const uint32_t a = max(w.range_start[r], ta), b = min(w.range_start[r + 1], tb);
            if (a < b) sl = (uint32_t)slot_of(w, nranges, a);
        }
        slots[threadIdx.x] = sl;
        const int n = __syncthreads_count(in);
        if (wd < w.tile_words) {
            auto quad = [&](int s) {
                const uint32_t q = slots[s];
                return q == 0xffffffffu
                           ? make_uint4(0u, 0u, 0u, 0u)
                           : *reinterpret_cast<const uint4 *>(w.partial + (int64_t)q * w.slot_words + wd);
            };
            auto add = [&](const uint4 v) {
                lo[0] += v.x & 0xffffu; hi[0] += v.x >> 16;
                lo[1] += v.y & 0xffffu; hi[1] += v.y >> 16;
                lo[2] += v.z & 0xffffu; hi[2] += v.z >> 16;
                lo[3] += v.w & 0xffffu; hi[3] += v.w >> 16;
            };
            int s = 0;
            for (; s + 4 <= n; s += 4) {
                uint4 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = quad(s + u);
#pragma unroll
                for (int u = 0; u < 4; ++u) add(v[u]);
            }
            for (; s < n; ++s) add(quad(s));
        }
        if (n < 256) break;   // uniform: n is the same in every thread
        __syncthreads();      // slots are rewritten in the next round
    }
    int *dst = cls ? M : N;
    unsigned long long tot = 0;
    // counter c of the tile is voxel (c mod S, c / S) of the slice (S = the
    // row length, odd); counters past column nx - 1 and past the last row are
    // padding and hold 0
    auto put = [&](int c, uint32_t v) {
        const int y = c / w.stride, x = c - y * w.stride;
        if (x < w.gnx && y < w.gny) dst[(int64_t)k * plane + (int64_t)y * w.gnx + x] += (int)v;
    };
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int wu = wd + u;
        if (wu >= w.tile_words) break;
        put(2 * wu, lo[u]);
        put(2 * wu + 1, hi[u]);
        tot += (unsigned long long)lo[u] + hi[u];
    }
    if (st) {
        const unsigned long long v = block_sum(tot, red);
        if (threadIdx.x == 0) add_stats(st, 4 + cls, v);
    }
}

struct GlobalAcc3 {
    int *cnt;
    __device__ __forceinline__ void operator()(int off) const { atomicAdd(cnt + off, 1); }
};

// Lines listed in the overflow bins, walked through the whole grid with global
// atomics (grid-stride over a count known only on the device); each line is
// quantised again from its history, as classification did.
__global__ void __launch_bounds__(256)
k_walk_overflow(hullmi_histories h, int64_t h0, DevGrid g, BinWs w, int *N, int *M,
                hullmi_stats *st)
{
    __shared__ unsigned long long red[16];
    const int start = w.ctl[kCtlOverflowStart], count = w.ctl[kCtlOverflowCount];
    const int nlow = w.ctl[kCtlOverflowLow];
    unsigned long long vl = 0, vh = 0;
    uint32_t trig_bits = 0x7fc00001u;
    float tc = 1.0f, ts = 0.0f;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x) {
        const int64_t i = h0 + w.item[start + t].x;
        int q[6];
        // classification listed the line, so its quantisation succeeds
        history_line(h.x_in[i], h.y_in[i], h.z_in[i], h.x_out[i], h.y_out[i], h.z_out[i],
                     h.angle_deg[i], g, trig_bits, tc, ts, q);
        const bool high = t >= nlow;
        GlobalAcc3 acc{high ? M : N};
        const int v = walk_line(q[0], q[1], q[2], q[3], q[4], q[5], g.nx, g.ny, g.nz, acc);
        if (high) vh += (unsigned long long)v; else vl += (unsigned long long)v;
    }
    if (st) {
        unsigned long long v = block_sum(vl, red);
        if (threadIdx.x == 0) add_stats(st, 4, v);
        v = block_sum(vh, red);
        if (threadIdx.x == 0) add_stats(st, 5, v);
    }
}

}  // namespace hullmi
