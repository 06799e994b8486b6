// Binned SC: silhouette carving as the paper ran it (Section 3.2, after
// Algorithm 1), on the FDK hull's (angle, u, v) bins with the per-bin WEPL
// data cuts of Section 2.2, one carve line per bin, then a W x W in-plane
// mean and a threshold.
//
// Pass structure (each pass one kernel):
//   stats    histories -> (bin, w_q) record per history; per-bin count and sum
//            of w_q = rint(WEPL * 1024), accumulated in LDS copies of the
//            detector planes of the chunk's first and last gantry angle;
//   squares  records -> per-bin sum of w_q^2 (LDS planes again);
//   bounds   per bin: the kept range [lo, hi] of w_q, from the exact integer
//            form of "not more than k standard deviations from the mean";
//   cut      records -> per-bin kept count and kept sum (LDS planes);
//   select   per bin: kept mean below E_L -> appended to the carve list;
//   carve    per listed bin: walk the line from the source through the bin
//            centre and mark its voxels in a bit volume (through an LDS
//            window of the slices the block's lines cross);
//   blur     per voxel: count of uncarved voxels in its W x W window.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hull_device.h"
#include "hull_kernels.h"
#include "hullmi.h"

namespace hullmi {

constexpr int kBscThreads = 1024;       // block of the two history passes
constexpr int kBscWide = 1 << 20;       // |w_q| below this goes through the packed LDS sums
constexpr int64_t kBscMaxChunk = int64_t(1) << 21;   // histories per block (packed-sum limit)

// Per-bin LDS word of a history pass: count in bits 42..63, sum of
// (w_q + kBscWide) below. With at most kBscMaxChunk histories per block and
// 0 < w_q + kBscWide < 2^21 the sum stays under 2^42 and the count under 2^22.
constexpr int kBscCountShift = 42;

enum : int { kBscBinned = 0, kBscCut = 1, kBscUsed = 2, kBscCarved = 3, kBscSkipped = 4,
             kBscVisits = 5, kBscStatWords = 6 };

constexpr int kBlurTx = 64, kBlurTy = 8;   // output tile of a blur block
constexpr int kCarveThreads = 1024;        // carve block, one per CU (its LDS window takes all)
constexpr int kRecUnroll = 8;              // records per lane in flight in the record passes

struct BscWs {
    int2 *rec;                       // [n] (bin or -1, w_q)
    unsigned *cnt;                   // [nb] histories binned
    unsigned long long *s1;          // [nb] sum of w_q (two's complement)
    unsigned long long *s2lo;        // [nb] sum of the low 32 bits of w_q^2
    unsigned long long *s2hi;        // [nb] sum of w_q^2 >> 32
    int2 *bnd;                       // [nb] kept range [lo, hi] of w_q
    unsigned *kept_n;                // [nb]
    unsigned long long *kept_s;      // [nb] (int64 two's complement)
    unsigned *cbits;                 // [ceil(V / 32)] carved flags, bit v % 32 of word v / 32
    unsigned long long *stats;       // kBscStatWords counters (hullmi_bsc_stats layout)
    float2 *cs;                      // [n_angles] cos, sin of each bin's gantry angle
    int *list;                       // [nb] bins to carve, then
    int *nlist;                      // their number
    int64_t nb;
};

__global__ void k_bsc_stats(hullmi_histories h, FbpDev p, BscWs w, int64_t chunk, int nplanes);
__global__ void k_bsc_squares(BscWs w, int64_t n, int plane, int64_t chunk, int nplanes);
__global__ void k_bsc_bounds(BscWs w, int ksig);
__global__ void k_bsc_cut(BscWs w, int64_t n, int plane, int64_t chunk, int nplanes,
                          const float *wepl, unsigned long long *fsum, unsigned *fcnt);
__global__ void k_bsc_trig(BscWs w, FbpDev p);
__global__ void k_bsc_select(BscWs w, FbpDev p, long long e_q, int row_first);
__global__ void k_bsc_carve(BscWs w, FbpDev p, DevGrid g, int lwords);
__global__ void k_bsc_clear(BscWs w, int64_t vwords);
__global__ void k_bsc_blur(const unsigned *cbits, uint8_t *carved, uint8_t *mask, int nx, int ny,
                           int r, long long num_w2, int den);

}  // namespace hullmi
