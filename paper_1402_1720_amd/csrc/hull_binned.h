// Slice-binned counting: the (history, z-slice) items of a batch are sorted by
// (class, slice, length class), each a 16-byte record (the line's packed
// endpoints, then its packed slice-walk state); a persistent grid of
// workgroups takes ranges of equal estimated work from that list (two per
// workgroup, dealt round-robin) and accumulates each slice it meets in a
// 16-bit LDS copy, written out as a partial tile when its range leaves the
// slice; a reduction then adds the partials into N or M.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hull_device.h"
#include "hullmi.h"

namespace hullmi {

constexpr int kBinThreads = 256;        // classify block
constexpr int kHistPerThread = 32;
constexpr int kHistPerBlock = kBinThreads * kHistPerThread;
constexpr int kScatterThreads = 1024;   // scatter block: the same 8192 histories
constexpr int kMaxSlicesPerLine = 6;    // longer lines go to the global-atomic walk
constexpr int kMaxSubBins = 4098;       // LDS histogram of the classify / scatter blocks
constexpr int kScanGroup = 16;         // block columns per first-step scan group
constexpr int kTileThreads = 1024;      // workgroup of the LDS walk
static_assert(kTileThreads % 256 == 0, "the walk deals items in groups of four waves");
constexpr int kItemsPerRange = 65535;   // a range holds at most this many items: each adds
                                        // at most 1 to a voxel, so a 16-bit counter holds it
constexpr int kWorkPerItem = 16;        // fixed cost of an item in visit units (set-up)
// Histories per internal batch: at most kBatch (about 12 GB of workspace on a
// 256x256x64 grid), fewer when the caller's workspace is smaller, but at least
// kMinBatch (or all of them). Batches of 2^26 rather than 2^24 took the counting
// pass of a 256x256x64, 2e8-history scan from 24.7 to 23.0 ms (fewer partial
// slice tiles to reduce, fewer plans).
constexpr int64_t kBatch = int64_t(1) << 26;
constexpr int64_t kMinBatch = int64_t(1) << 16;

// meta word per history: valid | overflow | class | nslices | first slice
constexpr uint32_t kMetaValid = 1u << 31;
constexpr uint32_t kMetaOverflow = 1u << 25;
constexpr uint32_t kMetaHigh = 1u << 24;

// control words written on the device by the planning kernel
enum : int { kCtlRanges = 0, kCtlItems = 1, kCtlOverflowStart = 2, kCtlOverflowCount = 3,
             kCtlOverflowLow = 4, kCtlCoarse = 5, kCtlWords = 16 };

// A line the tile walk takes has every endpoint coordinate in
// [-kPackLimit, kPackLimit) (1/1024 voxel): its record packs into 16 bytes.
constexpr int kPackLimit = 1 << 20;

struct BinWs {
    // per-history arrays hold whole classification blocks (B rounded up)
    uint4 *hrec;            // per history: the packed endpoints of a tile line, else zeros
    uint32_t *meta;         // per history
    uint32_t *lpack;        // per history: 4-bit length class per slice
    uint32_t *blk;          // [nblk][nsub] items of each (block column, sub-bin)
    uint32_t *boff;         // [nblk][nsub] offset of a column within its scan group
    uint32_t *gsum;         // [nsub][ngroups] items per (sub-bin, scan group)
    uint32_t *goff;         // [ngroups][nsub] offset of a scan group within its sub-bin
    uint32_t *sub_total;    // [nsub]
    uint32_t *sub_start;    // [nsub + 1]
    uint32_t *tile_start;   // [ntiles + 1]
    uint32_t *range_start;  // [max_ranges + 1] item bounds of the ranges
    uint32_t *range_coarse; // [max_ranges + 1] equal-work bounds before splitting
    uint32_t *range_piece;  // [max_ranges] first final range of each coarse range
    unsigned long long *wprefix;  // [nsub + 1] work prefix of the sub-bins
    int32_t *ctl;           // kCtlWords
    uint4 *item;            // [B * kMaxSlicesPerLine] per item: a tile item's packed
                            // endpoints, replaced by its packed slice-walk state; the
                            // history of an overflow item
    uint32_t *partial;      // [max_slots][slot_words]
    int nz, nl, lwidth;     // slices, length classes per slice, class width (voxels)
    int nsub, ntiles, nblk, ngroups, tile_words, max_ranges, max_slots, min_ranges;
    int slot_words;         // tile_words rounded up to a multiple of four
    int stride, gnx, gny;   // tile row length in counters (odd), grid columns and rows
    int run_stride;         // runs of a sub-bin ordered by block modulo this
    int64_t B;
};

__global__ void k_bin_classify(hullmi_histories h, int64_t h0, int64_t nb, DevGrid g, float e_low,
                               float e_high, int use_low, int use_high, int tile_ok, BinWs w,
                               hullmi_stats *st);
__global__ void k_bin_scan_groups(BinWs w);
__global__ void k_bin_scan_sums(BinWs w);
__global__ void k_bin_plan(BinWs w);
__global__ void k_bin_scatter(int64_t nb, BinWs w);
__global__ void k_item_setup(BinWs w, int nx, int ny);
__global__ void k_walk_tiles(BinWs w, int nx, int ny);
__global__ void k_reduce_tiles(BinWs w, int plane, int *N, int *M, hullmi_stats *st);
__global__ void k_walk_overflow(hullmi_histories h, int64_t h0, DevGrid g, BinWs w, int *N,
                                int *M, hullmi_stats *st);

}  // namespace hullmi
