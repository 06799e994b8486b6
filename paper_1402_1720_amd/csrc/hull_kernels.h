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

// Where a history's line crosses x = 0, decided in FP32: gantry angle bin k,
// detector bin (iu, iv) and the WEPL in fixed point (2^-16 mm). False when the
// history is not binned.
__device__ __forceinline__ bool fbp_locate_vals(float xi, float yi, float zi, float xo, float yo,
                                                float zo, float a, float w, const FbpDev &p, int &k,
                                                int &iu, int &iv, long long &fx)
{
    if (!(isfinite(xi) && isfinite(yi) && isfinite(zi) && isfinite(xo) && isfinite(yo) &&
          isfinite(zo) && isfinite(a) && isfinite(w)))
        return false;
    if (!(fabsf(w) < 65536.0f)) return false;
    const float ddx = xo - xi;
    if (ddx == 0.0f) return false;
    const float r = (0.0f - xi) / ddx;
    const float u = yi + r * (yo - yi);
    const float v = zi + r * (zo - zi);
    const float fa = (a - p.angle0) * p.rda;
    const float fu = (u - p.u0) * p.rdu;
    const float fv = (v - p.v0) * p.rdv;
    if (!(fabsf(fa) < 1.0e9f)) return false;
    if (!(fu >= 0.0f && fu < (float)p.nu && fv >= 0.0f && fv < (float)p.nv)) return false;
    // |fa| < 1e9 < 2^31: the angle index fits 32 bits, and it is almost always
    // already in [0, n_angles), where no remainder is needed
    int kk = (int)rintf(fa);
    if ((unsigned)kk >= (unsigned)p.n_angles) {
        kk %= p.n_angles;
        if (kk < 0) kk += p.n_angles;
    }
    k = kk;
    iu = (int)floorf(fu);
    iv = (int)floorf(fv);
    fx = llrint((double)w * 65536.0);
    return true;
}

__device__ __forceinline__ bool fbp_locate(const hullmi_histories &h, int64_t i, const FbpDev &p,
                                           int &k, int &iu, int &iv, long long &fx)
{
    return fbp_locate_vals(h.x_in[i], h.y_in[i], h.z_in[i], h.x_out[i], h.y_out[i], h.z_out[i],
                           h.angle_deg[i], h.wepl[i], p, k, iu, iv, fx);
}

// Angle bin of a history from its angle alone (-1 when it cannot be binned).
__device__ __forceinline__ int fbp_angle_bin(float a, const FbpDev &p)
{
    if (!isfinite(a)) return -1;
    const float fa = (a - p.angle0) * p.rda;
    if (!(fabsf(fa) < 1.0e9f)) return -1;
    long long kk = (long long)rintf(fa) % p.n_angles;
    if (kk < 0) kk += p.n_angles;
    return (int)kk;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n);
__global__ void k_fill_u8(uint8_t *p, uint8_t v, int64_t n);
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
__global__ void k_sm_edge_thin(const int *M, unsigned long long *gp, unsigned long long *seed, int nx,
                               int ny);
__global__ void k_sm_edge_trace(const int *M, const unsigned long long *gp,
                                const unsigned long long *seed, long long *mt, int *glist, int nx,
                                int ny, int num, int den, int cap);
__global__ void k_sm_edge_mask(const int *M, const long long *mt, uint8_t *mask, int64_t V,
                               int64_t plane);
__global__ void k_fbp_bin(hullmi_histories h, FbpDev p, unsigned long long *sum, unsigned *cnt);
constexpr int kFbpBinThreads = 1024;   // block of the LDS-binned FDK histogram
__global__ void k_fbp_bin_lds(hullmi_histories h, FbpDev p, unsigned long long *sum, unsigned *cnt,
                              int64_t chunk);
constexpr int kFbpFilterRows = 4;   // detector rows per filter block
__global__ void k_fbp_filter(const unsigned long long *sum, const unsigned *cnt, float *q, FbpDev p,
                             double unit);
__global__ void k_fbp_trig(float2 *cs, FbpDev p);
constexpr int kBpTile = 16;      // columns per side of a tiled-backprojection block
constexpr int kBpStage = 2048;   // floats of projection footprint staged in LDS
__global__ void k_fbp_footprint(const float2 *cs, FbpDev p, FbpGridDev g, int4 *fp, int ntx,
                                int nty, int ntz);
__global__ void k_fbp_backproject_tiles(const float *q, const float2 *cs, const int4 *fp, FbpDev p,
                                        FbpGridDev g, float *image, uint8_t *mask, int ntx, int nty);

}  // namespace hullmi
