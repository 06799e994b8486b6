// Kernel declarations and the small parameter blocks they take by value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hull_device.h"
#include "hullmi.h"

namespace hullmi {

struct FbpDev {
    float src_dist, du, dv, u0, v0;
    float rdu, rdv, rda;        // 1/du, 1/dv, 1/dangle rounded once on the host
    float angle0, dangle, threshold, half_dth;
    int nu, nv, n_angles;
};

struct FbpGridDev {
    int nx, ny, nz;
    float dx, dy, dz, x0, y0, z0;
};

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n);
__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t n);
__global__ void k_walk_lines(const int *qin, const int *qout, int64_t n, int nx, int ny, int nz,
                             int *cnt, hullmi_stats *st);
__global__ void k_quantize(hullmi_histories h, DevGrid g, int *status, int *qin, int *qout);
__global__ void k_sc_mask(const int *N, uint8_t *mask, int64_t V);
__global__ void k_msc_mask(const int *N, uint8_t *mask, int nx, int ny, int nz, int n_t, int mode,
                           int nbr);
__global__ void k_seg_max(const int *M, unsigned long long *out, int64_t V, int64_t seg_len);
__global__ void k_seg_slope_argmax(const int *M, unsigned long long *out, int nx, int ny, int nz,
                                   int nbr, int64_t seg_len);
__global__ void k_sm_mask(const int *M, uint8_t *mask, int64_t V, int64_t seg_len, int mode,
                          int num, int den, const unsigned long long *seg);
__global__ void k_fbp_bin(hullmi_histories h, FbpDev p, unsigned long long *sum, unsigned *cnt);
constexpr int kFbpBinThreads = 1024;   // block of the LDS-binned FDK histogram
__global__ void k_fbp_bin_lds(hullmi_histories h, FbpDev p, unsigned long long *sum, unsigned *cnt,
                              int64_t chunk, int nplanes);
__global__ void k_fbp_filter(const unsigned long long *sum, const unsigned *cnt, float *q, FbpDev p);
__global__ void k_fbp_trig(float2 *cs, FbpDev p);
constexpr int kBpTile = 16;      // columns per side of a tiled-backprojection block
constexpr int kBpStage = 2048;   // floats of projection footprint staged in LDS
__global__ void k_fbp_footprint(const float2 *cs, FbpDev p, FbpGridDev g, int4 *fp, int ntx,
                                int nty, int ntz);
__global__ void k_fbp_backproject_tiles(const float *q, const float2 *cs, const int4 *fp, FbpDev p,
                                        FbpGridDev g, float *image, uint8_t *mask, int ntx, int nty);

}  // namespace hullmi
