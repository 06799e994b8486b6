// Kernels of the hull path for gfx950 (wave64): classify + geometry + walk +
// accumulate, the SC/MSC/SM rules, and the FDK hull.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hull_device.h"
#include "hull_kernels.h"

namespace hullmi {

// ---------------------------------------------------------------------------
// small utilities

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_u8(uint8_t *p, uint8_t v, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Block-wide sum of six per-thread counters into the stats struct.
__device__ __forceinline__ void flush_stats(hullmi_stats *st, unsigned long long l,
                                            unsigned long long h, unsigned long long sk,
                                            unsigned long long mi, unsigned long long vl,
                                            unsigned long long vh)
{
    __shared__ unsigned long long s[6];
    if (threadIdx.x < 6) s[threadIdx.x] = 0;
    __syncthreads();
    if (l) atomicAdd(&s[0], l);
    if (h) atomicAdd(&s[1], h);
    if (sk) atomicAdd(&s[2], sk);
    if (mi) atomicAdd(&s[3], mi);
    if (vl) atomicAdd(&s[4], vl);
    if (vh) atomicAdd(&s[5], vh);
    __syncthreads();
    if (threadIdx.x < 6 && s[threadIdx.x])
        atomicAdd(reinterpret_cast<unsigned long long *>(st) + threadIdx.x, s[threadIdx.x]);
}

struct GlobalAcc {
    int *cnt;
    __device__ __forceinline__ void operator()(int off) const { atomicAdd(cnt + off, 1); }
};

__global__ void __launch_bounds__(256)
k_walk_lines(const int *qin, const int *qout, int64_t n, int nx, int ny, int nz, int *cnt,
             hullmi_stats *st)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long nl = 0, nsk = 0, nmi = 0, vl = 0;
    if (i < n) {
        const int a0 = qin[3 * i], a1 = qin[3 * i + 1], a2 = qin[3 * i + 2];
        const int b0 = qout[3 * i], b1 = qout[3 * i + 1], b2 = qout[3 * i + 2];
        const int lim = 1 << 26;
        const bool ok = a0 > -lim && a0 < lim && a1 > -lim && a1 < lim && a2 > -lim && a2 < lim &&
                        b0 > -lim && b0 < lim && b1 > -lim && b1 < lim && b2 > -lim && b2 < lim &&
                        !(a0 == b0 && a1 == b1 && a2 == b2);
        if (!ok) {
            nsk = 1;
        } else {
            GlobalAcc acc{cnt};
            const int c = walk_line(a0, a1, a2, b0, b1, b2, nx, ny, nz, acc);
            nl = 1;
            vl = (unsigned long long)c;
            nmi = c == 0;
        }
    }
    if (st) flush_stats(st, nl, 0, nsk, nmi, vl, 0);
}

__global__ void __launch_bounds__(256)
k_quantize(hullmi_histories h, DevGrid g, int *status, int *qin, int *qout)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= h.n) return;
    const float xi = h.x_in[i], yi = h.y_in[i], zi = h.z_in[i];
    const float xo = h.x_out[i], yo = h.y_out[i], zo = h.z_out[i];
    const float a = h.angle_deg[i], w = h.wepl[i];
    int st = (isfinite(xi) && isfinite(yi) && isfinite(zi) && isfinite(xo) && isfinite(yo) &&
              isfinite(zo) && isfinite(a) && isfinite(w))
                 ? kGeoOk
                 : kGeoNonFinite;
    int q[6];
    if (st == kGeoOk) {
        float c, s;
        deg_cos_sin(a, c, s);
        st = quantize_point(c, s, xi, yi, zi, g, q[0], q[1], q[2]);
        if (st == kGeoOk) st = quantize_point(c, s, xo, yo, zo, g, q[3], q[4], q[5]);
        if (st == kGeoOk && q[0] == q[3] && q[1] == q[4] && q[2] == q[5]) st = kGeoDegenerate;
    }
    status[i] = st;
    if (st == kGeoOk || st == kGeoDegenerate) {
        qin[3 * i] = q[0]; qin[3 * i + 1] = q[1]; qin[3 * i + 2] = q[2];
        qout[3 * i] = q[3]; qout[3 * i + 1] = q[4]; qout[3 * i + 2] = q[5];
    }
}

// ---------------------------------------------------------------------------
// hull rules

__device__ __forceinline__ void voxel_ijk(int64_t v, int nx, int ny, int &i, int &j, int &k)
{
    i = (int)(v % nx);
    const int64_t r = v / nx;
    j = (int)(r % ny);
    k = (int)(r / ny);
}

__global__ void k_sc_mask(const int *N, uint8_t *mask, int64_t V)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < V) mask[v] = N[v] == 0;
}

// MSC: COUNT keeps N < n_t; NEIGHBOR_DIFF removes v when N(v) - N(w) >= n_t
// for a face neighbour w (in-plane, or 3-D with nbr == SPATIAL6).
__global__ void k_msc_mask(const int *N, uint8_t *mask, int nx, int ny, int nz, int n_t,
                           int mode, int nbr)
{
    const int64_t V = (int64_t)nx * ny * nz;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const int64_t nv = N[v];
    if (mode == HULL_MSC_COUNT) {
        mask[v] = nv < n_t;
        return;
    }
    int i, j, k;
    voxel_ijk(v, nx, ny, i, j, k);
    int64_t lo = nv;   // smallest neighbour count (v itself included)
    if (i > 0) lo = min(lo, (int64_t)N[v - 1]);
    if (i < nx - 1) lo = min(lo, (int64_t)N[v + 1]);
    if (j > 0) lo = min(lo, (int64_t)N[v - nx]);
    if (j < ny - 1) lo = min(lo, (int64_t)N[v + nx]);
    if (nbr == HULL_NBR_SPATIAL6) {
        const int64_t pl = (int64_t)nx * ny;
        if (k > 0) lo = min(lo, (int64_t)N[v - pl]);
        if (k < nz - 1) lo = min(lo, (int64_t)N[v + pl]);
    }
    mask[v] = nv - lo < n_t;
}

// Block-wide maximum (wave64 shuffles, then LDS); valid in thread 0.
__device__ __forceinline__ unsigned long long block_max(unsigned long long v)
{
    __shared__ unsigned long long sh[16];
    for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned long long)__shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long m = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) m = max(m, sh[i]);
    return m;
}

// Largest M per segment (the whole volume, or one z-slice each):
// blockIdx.y picks the segment, the blocks of a segment stride over it and
// each issues one atomicMax.
__global__ void __launch_bounds__(256)
k_seg_max(const int *M, unsigned long long *out, int64_t V, int64_t seg_len)
{
    const int64_t base = (int64_t)blockIdx.y * seg_len;
    const int64_t end = min(base + seg_len, V);
    unsigned long long m = 0;
    for (int64_t v = base + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < end;
         v += (int64_t)gridDim.x * blockDim.x)
        m = max(m, (unsigned long long)(unsigned)M[v]);
    m = block_max(m);
    if (threadIdx.x == 0) atomicMax(out + blockIdx.y, m);
}

// Algorithm 3's maximum slope: per voxel the largest M(v) - M(w) over B(v)
// (0 from w = v), packed with the voxel index so that the 64-bit maximum
// picks the largest slope and, among equal slopes, the last voxel.
__global__ void __launch_bounds__(256)
k_seg_slope_argmax(const int *M, unsigned long long *out, int nx, int ny, int nz, int nbr,
                   int64_t seg_len)
{
    const int64_t V = (int64_t)nx * ny * nz;
    const int64_t base = (int64_t)blockIdx.y * seg_len;
    const int64_t end = min(base + seg_len, V);
    const int64_t pl = (int64_t)nx * ny;
    unsigned long long best = 0;
    for (int64_t v = base + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < end;
         v += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        voxel_ijk(v, nx, ny, i, j, k);
        const int64_t mv = M[v];
        int64_t lo = mv;
        if (i > 0) lo = min(lo, (int64_t)M[v - 1]);
        if (i < nx - 1) lo = min(lo, (int64_t)M[v + 1]);
        if (j > 0) lo = min(lo, (int64_t)M[v - nx]);
        if (j < ny - 1) lo = min(lo, (int64_t)M[v + nx]);
        if (nbr == HULL_NBR_SPATIAL6) {
            if (k > 0) lo = min(lo, (int64_t)M[v - pl]);
            if (k < nz - 1) lo = min(lo, (int64_t)M[v + pl]);
        }
        best = max(best, ((unsigned long long)(mv - lo) << 32) | (unsigned long long)v);
    }
    best = block_max(best);
    if (threadIdx.x == 0) atomicMax(out + blockIdx.y, best);
}

__global__ void k_sm_mask(const int *M, uint8_t *mask, int64_t V, int64_t seg_len, int mode,
                          int num, int den, const unsigned long long *seg)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const unsigned long long s = seg[v / seg_len];
    const int64_t mv = M[v];
    if (mode == HULL_SM_FRACTION) {
        mask[v] = (int64_t)den * mv > (int64_t)num * (int64_t)s;
    } else {
        const int64_t mt = M[(int64_t)(s & 0xffffffffull)];
        mask[v] = mv > mt;
    }
}

// ---------------------------------------------------------------------------
// FDK hull

// Bin each history; WEPL sums in fixed point so the result does not depend
// on the order of the atomics. Used when a detector plane does not fit LDS.
__global__ void __launch_bounds__(256)
k_fbp_bin(hullmi_histories h, FbpDev p, unsigned long long *sum, unsigned *cnt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= h.n) return;
    int k, iu, iv;
    long long fx;
    if (!fbp_locate(h, i, p, k, iu, iv, fx)) return;
    const int64_t b = ((int64_t)k * p.nv + iv) * p.nu + iu;
    atomicAdd(sum + b, (unsigned long long)fx);
    atomicAdd(cnt + b, 1u);
}

// The same binning for a chunk of consecutive histories per block, through an
// LDS copy of one detector plane (sums and counts). The plane follows the
// histories' gantry angle: after every round of blockDim histories, when the
// angle bin of the round's last history differs from the plane's, the plane
// is added to the global sums and restarts on that angle. Histories come in
// long runs of one angle, so nearly all of them land in LDS and each block
// flushes its plane about once per angle it crosses; a history of any other
// angle goes straight to the global sums (any order of histories gives the
// same sums). The next history's fields are loaded while the current one is
// binned. Same fixed point, so the sums are identical to k_fbp_bin's.
__global__ void __launch_bounds__(kFbpBinThreads)
k_fbp_bin_lds(hullmi_histories h, FbpDev p, unsigned long long *sum, unsigned *cnt, int64_t chunk)
{
    extern __shared__ unsigned long long lsum[];   // the plane's sums, then its counts
    const int plane = p.nu * p.nv;
    unsigned *lcnt = reinterpret_cast<unsigned *>(lsum + plane);
    const int64_t base = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(base + chunk, h.n);
    if (base >= end) return;   // uniform across the block
    for (int b = threadIdx.x; b < plane; b += blockDim.x) { lsum[b] = 0ull; lcnt[b] = 0u; }
    int kcur = fbp_angle_bin(h.angle_deg[base], p);   // -1: no plane yet
    __syncthreads();
    // adds the plane's non-empty bins to angle k's global sums and clears them
    auto flush = [&](int k) {
        for (int b = threadIdx.x; b < plane; b += blockDim.x) {
            const unsigned c = lcnt[b];
            if (c) {
                const int64_t g = (int64_t)k * plane + b;
                atomicAdd(sum + g, lsum[b]);
                atomicAdd(cnt + g, c);
                lsum[b] = 0ull;
                lcnt[b] = 0u;
            }
        }
    };
    struct F8 { float xi, yi, zi, xo, yo, zo, a, w; };
    auto fetch = [&](int64_t i, F8 &f) {
        if (i < end) {
            f.xi = h.x_in[i]; f.yi = h.y_in[i]; f.zi = h.z_in[i];
            f.xo = h.x_out[i]; f.yo = h.y_out[i]; f.zo = h.z_out[i];
            f.a = h.angle_deg[i]; f.w = h.wepl[i];
        }
    };
    F8 nf{};
    fetch(base + threadIdx.x, nf);
    // the angle of each round's last history decides the plane switch; it is
    // loaded a round ahead, like the fields, so that no round waits for it
    const int64_t R = blockDim.x;
    float a_last = h.angle_deg[min(base + R, end) - 1];
    // every thread runs the same rounds: the plane switch needs the whole block
    for (int64_t i0 = base; i0 < end; i0 += R) {
        const int64_t i = i0 + threadIdx.x;
        const F8 f = nf;
        fetch(i + R, nf);
        const float a_next = i0 + R < end ? h.angle_deg[min(i0 + 2 * R, end) - 1] : 0.0f;
        int k, iu, iv;
        long long fx;
        if (i < end && fbp_locate_vals(f.xi, f.yi, f.zi, f.xo, f.yo, f.zo, f.a, f.w, p, k, iu, iv, fx)) {
            const int pb = iv * p.nu + iu;
            if (k == kcur) {
                atomicAdd(&lsum[pb], (unsigned long long)fx);
                atomicAdd(&lcnt[pb], 1u);
            } else {
                const int64_t b = (int64_t)k * plane + pb;
                atomicAdd(sum + b, (unsigned long long)fx);
                atomicAdd(cnt + b, 1u);
            }
        }
        // the same value in every thread: the round's last history
        const int kn = fbp_angle_bin(a_last, p);
        a_last = a_next;
        if (kn >= 0 && kn != kcur) {
            __syncthreads();
            if (kcur >= 0) flush(kcur);
            __syncthreads();
            kcur = kn;
        }
    }
    __syncthreads();
    if (kcur >= 0) flush(kcur);
}

// One block per detector row: bin means (sums in fixed point of `unit` mm),
// cosine pre-weight, then the
// Shepp-Logan convolution along u (FP64 accumulation in the order j = 0 ..
// nu - 1, rows taken as zero outside the detector).
constexpr int kFilterOut = 5;
constexpr int kFilterRows = kFbpFilterRows;   // one detector row per wavefront
__global__ void __launch_bounds__(64 * kFilterRows)
k_fbp_filter(const unsigned long long *sum, const unsigned *cnt, float *q, FbpDev p, double unit)
{
    extern __shared__ double sh[];
    const int nu = p.nu;
    const int64_t nrows = (int64_t)p.n_angles * p.nv;
    // ker[m + nu - 1] = h[m] for |m| < nu, with one zero before it (ker[-1]),
    // so that the sliding window below needs no bounds test
    double *ker = sh + 1;                          // 2 nu - 1 values after the zero
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *row = sh + 2 * nu + wave * nu;         // this wavefront's row
    const int64_t r = (int64_t)blockIdx.x * kFilterRows + wave;   // k * nv + iv
    const double D = p.src_dist, du = p.du;
    const double pi = 3.14159265358979323846;
    if (threadIdx.x == 0) ker[-1] = 0.0;
    for (int m = threadIdx.x; m < 2 * nu - 1; m += blockDim.x) {
        const double n = (double)(m - (nu - 1));
        ker[m] = -2.0 / (pi * pi * du * du * (4.0 * n * n - 1.0));
    }
    const int iv = (int)(r % p.nv);
    if (r < nrows) {
        const double vc = (double)p.v0 + ((double)iv + 0.5) * (double)p.dv;
        for (int iu = lane; iu < nu; iu += 64) {
            const int64_t b = r * nu + iu;
            const unsigned c = cnt[b];
            const double mean = c ? (double)(long long)sum[b] * unit / (double)c : 0.0;
            const double uc = (double)p.u0 + ((double)iu + 0.5) * du;
            row[iu] = mean * D / sqrt(D * D + uc * uc + vc * vc);
        }
    }
    __syncthreads();
    if (r >= nrows) return;
    // padded output: [n_angles][nv + 4][nu + 4], two zero bins on every side
    const int64_t k = r / p.nv;
    float *qr = q + (k * (p.nv + 4) + (iv + 2)) * (int64_t)(nu + 4) + 2;
    // kFilterOut consecutive outputs per lane: output iu + c needs
    // ker[iu + c + nu - 1 - j]; the window of kernel values slides down by one
    // per j, so each j costs one kernel load and one (broadcast) row load
    for (int iu = lane * kFilterOut; iu < nu; iu += 64 * kFilterOut) {
        double acc[kFilterOut], win[kFilterOut];
        const int top = iu + nu - 1;   // ker index of output iu at j = 0
#pragma unroll
        for (int c = 0; c < kFilterOut; ++c) {
            acc[c] = 0.0;
            win[c] = top + c < 2 * nu - 1 ? ker[top + c] : 0.0;
        }
#pragma unroll 8
        for (int j = 0; j < nu; ++j) {
            const double x = row[j];
#pragma unroll
            for (int c = 0; c < kFilterOut; ++c) acc[c] = __builtin_fma(win[c], x, acc[c]);
#pragma unroll
            for (int c = kFilterOut - 1; c > 0; --c) win[c] = win[c - 1];
            win[0] = ker[top - j - 1];   // index >= -1 (top >= nu - 1, j < nu)
        }
#pragma unroll
        for (int c = 0; c < kFilterOut; ++c)
            if (iu + c < nu) qr[iu + c] = (float)(du * acc[c]);
    }
}

__global__ void k_fbp_trig(float2 *cs, FbpDev p)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.n_angles) return;
    const double th = ((double)p.angle0 + (double)k * (double)p.dangle) * (3.14159265358979323846 / 180.0);
    cs[k] = make_float2((float)cos(th), (float)sin(th));
}

// FDK backprojection. One lane per (x, y) column and group of kFbpZ slices:
// per angle the rotation, the magnification U and the u interpolation are
// computed once and reused for every slice of the group. The filtered
// projections carry two zero bins on every side, so an index clamped into
// that border samples zeros. Threshold fused.
constexpr int kFbpZ = 8;

// One (column, angle) term for kFbpZ slices: `sample(iv, iu, row)` returns the
// padded projection values at row iv + 2 + row, bins iu + 2 and iu + 3, as a
// float2 (left, right); the same arithmetic whether they come from LDS or
// from global memory.
template <class Sample>
__device__ __forceinline__ void bp_term(float2 c, float xo, float yo, const float *zo, float *f,
                                        const FbpDev &p, float D, float rD, Sample &&sample)
{
    const float xl = c.x * xo - c.y * yo;
    const float yl = c.y * xo + c.x * yo;
    const float U = (D + xl) * rD;
    if (!(U > 0.0f)) return;   // voxel at or behind the source plane
    const float iU = __builtin_amdgcn_rcpf(U);
    const float w2 = iU * iU;
    const float fu = (yl * iU - p.u0) * p.rdu - 0.5f;
    const float fu0 = floorf(fu);
    const float au = fu - fu0;
    const int iu0 = min(max((int)fmaxf(fminf(fu0, 1.0e8f), -1.0e8f), -2), p.nu);
    const float fvs = iU * p.rdv;
#pragma unroll
    for (int z = 0; z < kFbpZ; ++z) {
        const float fv = zo[z] * fvs - p.v0 * p.rdv - 0.5f;
        const float fv0 = floorf(fv);
        const float av = fv - fv0;
        const int iv0 = min(max((int)fmaxf(fminf(fv0, 1.0e8f), -1.0e8f), -2), p.nv);
        const float2 t = sample(iv0, iu0, 0), b = sample(iv0, iu0, 1);
        const float top = t.x + au * (t.y - t.x);
        const float bot = b.x + au * (b.y - b.x);
        f[z] += (top + av * (bot - top)) * w2;
    }
}

// bp_term for a tile whose footprint is staged in LDS (`st` = the stage at
// padded bin bx and row by, rw bins per row): the same samples and weights
// with fewer instructions. The row coordinate steps by dz * fvs from slice to
// slice, the bin and row indices are clamped with one med3 each (clamped
// indices fall in the zero border, as in bp_term), and the bilinear weights
// use explicit FMAs; the image differs from bp_term's only by rounding.
__device__ __forceinline__ void bp_term_lds(float2 c, float xo, float yo, float zo0, float dz,
                                            float *f, const FbpDev &p, float D, float rD,
                                            float vbase, const float *st, int bx, int by, int rw)
{
    const float xl = c.x * xo - c.y * yo;
    const float yl = c.y * xo + c.x * yo;
    const float U = (D + xl) * rD;
    if (!(U > 0.0f)) return;   // voxel at or behind the source plane
    const float iU = __builtin_amdgcn_rcpf(U);
    const float w2 = iU * iU;
    const float fu = (yl * iU - p.u0) * p.rdu - 0.5f;
    const float fu0 = floorf(fu);
    const float au = fu - fu0;
    const int iu0 = (int)__builtin_amdgcn_fmed3f(fu0, -2.0f, (float)p.nu);
    const float fvs = iU * p.rdv;
    const float step = dz * fvs;
    float fv = __builtin_fmaf(zo0, fvs, vbase);
    const float *col = st + (iu0 + 2 - bx) - (by - 2) * rw;
#pragma unroll
    for (int z = 0; z < kFbpZ; ++z) {
        const float fv0 = floorf(fv);
        const float av = fv - fv0;
        const int iv0 = (int)__builtin_amdgcn_fmed3f(fv0, -2.0f, (float)p.nv);
        const float *s0 = col + iv0 * rw;
        const float2 t = make_float2(s0[0], s0[1]), b = make_float2(s0[rw], s0[rw + 1]);
        const float top = __builtin_fmaf(au, t.y - t.x, t.x);
        const float bot = __builtin_fmaf(au, b.y - b.x, b.x);
        f[z] = __builtin_fmaf(__builtin_fmaf(av, bot - top, top), w2, f[z]);
        fv += step;
    }
}

// The bin and row indices bp_term uses for one column at one angle: iu0 and
// the range of iv0 over the slices z_lo .. z_hi; false behind the source.
__device__ __forceinline__ bool bp_indices(float2 c, float xo, float yo, float z_lo, float z_hi,
                                           const FbpDev &p, float D, float rD, int &iu0,
                                           int &iv_min, int &iv_max)
{
    const float xl = c.x * xo - c.y * yo;
    const float yl = c.y * xo + c.x * yo;
    const float U = (D + xl) * rD;
    if (!(U > 0.0f)) return false;
    const float iU = __builtin_amdgcn_rcpf(U);
    const float fu = (yl * iU - p.u0) * p.rdu - 0.5f;
    iu0 = min(max((int)fmaxf(fminf(floorf(fu), 1.0e8f), -1.0e8f), -2), p.nu);
    const float fvs = iU * p.rdv;
    int a = min(max((int)fmaxf(fminf(floorf(z_lo * fvs - p.v0 * p.rdv - 0.5f), 1.0e8f), -1.0e8f), -2), p.nv);
    int b = min(max((int)fmaxf(fminf(floorf(z_hi * fvs - p.v0 * p.rdv - 0.5f), 1.0e8f), -1.0e8f), -2), p.nv);
    iv_min = min(a, b);
    iv_max = max(a, b);
    return true;
}

// Footprint on the padded projection of every (tile, angle) of the tiled
// backprojection: bins [x, x + z) and rows [y, y + w) hold every sample the
// tile's lanes take at that angle (extremes at the tile's corner columns and
// end slices, widened by one bin and one row for rounding); z = 0 when a
// corner lies at or behind the source (the tile then reads global memory).
__global__ void __launch_bounds__(256)
k_fbp_footprint(const float2 *cs, FbpDev p, FbpGridDev g, int4 *fp, int ntx, int nty, int ntz)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ntiles = (int64_t)ntx * nty * ntz;
    if (t >= ntiles * p.n_angles) return;
    const int a = (int)(t % p.n_angles);
    const int64_t tile = t / p.n_angles;
    const int tx = (int)(tile % ntx), ty = (int)((tile / ntx) % nty), tz = (int)(tile / ((int64_t)ntx * nty));
    const int i0 = tx * kBpTile, i1 = min(i0 + kBpTile, g.nx) - 1;
    const int j0 = ty * kBpTile, j1 = min(j0 + kBpTile, g.ny) - 1;
    const int k0 = tz * kFbpZ, k1 = min(k0 + kFbpZ, g.nz) - 1;
    const float z_lo = g.z0 + ((float)k0 + 0.5f) * g.dz, z_hi = g.z0 + ((float)k1 + 0.5f) * g.dz;
    const float D = p.src_dist, rD = __builtin_amdgcn_rcpf(p.src_dist);
    const float2 c = cs[a];
    int umin = 1 << 30, umax = -(1 << 30), vmin = 1 << 30, vmax = -(1 << 30);
    bool ok = true;
    for (int corner = 0; corner < 4; ++corner) {
        const int i = (corner & 1) ? i1 : i0, j = (corner & 2) ? j1 : j0;
        const float xo = g.x0 + ((float)i + 0.5f) * g.dx;
        const float yo = g.y0 + ((float)j + 0.5f) * g.dy;
        int iu0, a0, a1;
        if (!bp_indices(c, xo, yo, z_lo, z_hi, p, D, rD, iu0, a0, a1)) { ok = false; break; }
        umin = min(umin, iu0); umax = max(umax, iu0);
        vmin = min(vmin, a0); vmax = max(vmax, a1);
    }
    int4 r = make_int4(0, 0, 0, 0);
    if (ok) {
        // padded bins iu0 + 2 and iu0 + 3, rows iv0 + 2 and iv0 + 3, one more each side
        const int ulo = max(umin + 1, 0), uhi = min(umax + 4, p.nu + 3);
        const int vlo = max(vmin + 1, 0), vhi = min(vmax + 4, p.nv + 3);
        r = make_int4(ulo, vlo, uhi - ulo + 1, vhi - vlo + 1);
        if (r.z * r.w > kBpStage) r.z = 0;
    }
    fp[tile * p.n_angles + a] = r;
}

// Tiled backprojection: a block of kBpTile x kBpTile columns and one group of
// kFbpZ slices stages, for each angle, the footprint of the tile on the
// padded projection in LDS and samples it there; a footprint too large for
// the stage is sampled from global memory.
__global__ void __launch_bounds__(kBpTile * kBpTile)
k_fbp_backproject_tiles(const float *q, const float2 *cs, const int4 *fp, FbpDev p, FbpGridDev g,
                        float *image, uint8_t *mask, int ntx, int nty)
{
    __shared__ float stage[kBpStage];
    const int tx = blockIdx.x % ntx, ty = (blockIdx.x / ntx) % nty, tz = blockIdx.x / (ntx * nty);
    const int li = threadIdx.x % kBpTile, lj = threadIdx.x / kBpTile;
    const int i = tx * kBpTile + li, j = ty * kBpTile + lj, kz0 = tz * kFbpZ;
    const bool in = i < g.nx && j < g.ny;
    const int nzg = min(kFbpZ, g.nz - kz0);
    const float xo = g.x0 + ((float)i + 0.5f) * g.dx;
    const float yo = g.y0 + ((float)j + 0.5f) * g.dy;
    float zo[kFbpZ], f[kFbpZ];
#pragma unroll
    for (int z = 0; z < kFbpZ; ++z) {
        zo[z] = g.z0 + ((float)(kz0 + z) + 0.5f) * g.dz;
        f[z] = 0.0f;
    }
    const float D = p.src_dist, rD = __builtin_amdgcn_rcpf(p.src_dist);
    const float vbase = -p.v0 * p.rdv - 0.5f;
    const int pu = p.nu + 4;
    const int64_t pa = (int64_t)(p.nv + 4) * pu;
    const int4 *fpt = fp + (int64_t)blockIdx.x * p.n_angles;
    for (int a = 0; a < p.n_angles; ++a) {
        const int4 r = fpt[a];   // the same in every lane
        const float *qa = q + (int64_t)a * pa;
        if (r.z > 0) {
            __syncthreads();   // the previous angle's samples are taken
            const int n = r.z * r.w;
            const float rw = 1.0f / (float)r.z;
            for (int e = threadIdx.x; e < n; e += blockDim.x) {
                int row = (int)((float)e * rw);
                if (row * r.z > e) --row;
                if ((row + 1) * r.z <= e) ++row;
                stage[e] = qa[(int64_t)(r.y + row) * pu + r.x + (e - row * r.z)];
            }
            __syncthreads();
            if (in) bp_term_lds(cs[a], xo, yo, zo[0], g.dz, f, p, D, rD, vbase, stage, r.x, r.y, r.z);
        } else if (in) {
            bp_term(cs[a], xo, yo, zo, f, p, D, rD, [&](int iv0, int iu0, int rr) {
                const float *s = qa + (int64_t)(iv0 + 2 + rr) * pu + (iu0 + 2);
                return make_float2(s[0], s[1]);
            });
        }
    }
    if (!in) return;
    for (int z = 0; z < nzg; ++z) {
        const float v = f[z] * p.half_dth;
        const int64_t vox = ((int64_t)(kz0 + z) * g.ny + j) * g.nx + i;
        image[vox] = v;
        if (mask) mask[vox] = v >= p.threshold;
    }
}


// ---------------------------------------------------------------------------
// SM threshold from the strongest edge of each slice (the EDGE rule stated in
// hullmi.h). Everything is integer: gradients, thinning, the edge component
// and M_t are the same whatever the thread order.

namespace {

__device__ __forceinline__ bool sobel_at(const int *Ms, int nx, int ny, int i, int j,
                                         long long &gx, long long &gy)
{
    if (i < 1 || j < 1 || i > nx - 2 || j > ny - 2) return false;
    auto at = [&](int a, int b) { return (long long)Ms[(int64_t)b * nx + a]; };
    gx = (at(i + 1, j - 1) + 2 * at(i + 1, j) + at(i + 1, j + 1)) -
         (at(i - 1, j - 1) + 2 * at(i - 1, j) + at(i - 1, j + 1));
    gy = (at(i - 1, j + 1) + 2 * at(i, j + 1) + at(i + 1, j + 1)) -
         (at(i - 1, j - 1) + 2 * at(i, j - 1) + at(i + 1, j - 1));
    return true;
}

__device__ __forceinline__ long long grad_l1(const int *Ms, int nx, int ny, int i, int j)
{
    long long gx, gy;
    if (!sobel_at(Ms, nx, ny, i, j, gx, gy)) return 0;
    return (gx < 0 ? -gx : gx) + (gy < 0 ? -gy : gy);
}

// index of q in the sorted list idx[0, n), or -1
__device__ __forceinline__ int find_sorted(const int *idx, int n, int q)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (idx[mid] < q) lo = mid + 1; else hi = mid;
    }
    return lo < n && idx[lo] == q ? lo : -1;
}

__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v)
{
    __shared__ unsigned long long part[16];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_down(v, o, 64);
        v = w > v ? w : v;
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x + 63) / 64; ++i) v = part[i] > v ? part[i] : v;
        part[0] = v;
    }
    __syncthreads();
    const unsigned long long r = part[0];
    __syncthreads();
    return r;
}

}  // namespace

// Per pixel: the L1 gradient G and whether thinning keeps it, packed as
// (G << 1) | edge; per slice the seed key (G << 22) | pixel of the strongest
// edge pixel (ties to the larger pixel index), one atomic per block.
__global__ void __launch_bounds__(256)
k_sm_edge_thin(const int *M, unsigned long long *gp, unsigned long long *seed, int nx, int ny)
{
    const int64_t plane = (int64_t)nx * ny;
    const int k = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int *Ms = M + (int64_t)k * plane;
    unsigned long long key = 0;
    if (p < plane) {
        const int i = (int)(p % nx), j = (int)(p / nx);
        long long gx = 0, gy = 0;
        long long G = 0;
        bool edge = false;
        if (sobel_at(Ms, nx, ny, i, j, gx, gy)) {
            const long long ax = gx < 0 ? -gx : gx, ay = gy < 0 ? -gy : gy;
            G = ax + ay;
            int di, dj;
            if (5 * ay <= 2 * ax) { di = 1; dj = 0; }
            else if (5 * ax <= 2 * ay) { di = 0; dj = 1; }
            else if ((gx > 0) == (gy > 0)) { di = 1; dj = 1; }
            else { di = 1; dj = -1; }
            edge = G > 0 && G > grad_l1(Ms, nx, ny, i - di, j - dj) &&
                   G >= grad_l1(Ms, nx, ny, i + di, j + dj);
        }
        gp[(int64_t)k * plane + p] = ((unsigned long long)G << 1) | (edge ? 1ull : 0ull);
        if (edge) key = ((unsigned long long)G << 22) | (unsigned long long)p;
    }
    key = block_max_u64(key);
    if (threadIdx.x == 0 && key) atomicMax(seed + k, key);
}

// One block per slice: the edge pixels eligible for the seed's edge
// (den G >= num G(seed), and the seed itself) are listed in raster order;
// union-find over their 8-neighbourhoods labels the components; M_t = the
// largest M on the seed's component. The
// list lives in LDS when it fits `cap` entries, else in `glist` (two arrays
// of `plane` ints per slice).
__global__ void __launch_bounds__(1024)
k_sm_edge_trace(const int *M, const unsigned long long *gp, const unsigned long long *seed,
                long long *mt, int *glist, int nx, int ny, int num, int den, int cap)
{
    extern __shared__ int lsh[];
    __shared__ int wsum[16];
    __shared__ int total;
    const int64_t plane = (int64_t)nx * ny;
    const int k = blockIdx.x;
    const unsigned long long key = seed[k];
    if (key == 0) {
        if (threadIdx.x == 0) mt[k] = -1;
        return;   // uniform
    }
    const long long Gs = (long long)(key >> 22);
    const int sp = (int)(key & ((1ull << 22) - 1));
    const unsigned long long *g = gp + (int64_t)k * plane;
    auto eligible = [&](int64_t p) {
        const unsigned long long w = g[p];
        return (w & 1ull) && ((long long)den * (long long)(w >> 1) >= (long long)num * Gs || p == sp);
    };
    // raster-order compaction in coalesced chunks: lane t of the block takes
    // pixels c0 + 4t .. c0 + 4t + 3 of each chunk of 4 * blockDim pixels; a
    // block scan of the per-lane counts places them in order
    const int nt = blockDim.x, t = threadIdx.x;
    const int64_t chunk = (int64_t)4 * nt;
    // the list goes to LDS when the slice's eligible pixels fit, else to
    // global memory: count them first (coalesced as well)
    int mine = 0;
    for (int64_t c0 = 0; c0 < plane; c0 += chunk)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t p = c0 + 4 * t + u;
            mine += p < plane && eligible(p);
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mine += __shfl_down(mine, o, 64);
    if ((t & 63) == 0) wsum[t >> 6] = mine;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int w = 0; w < (nt + 63) / 64; ++w) run += wsum[w];
        total = run;
    }
    __syncthreads();
    const int L = total;
    int *idx = L <= cap ? lsh : glist + (int64_t)k * 2 * plane;
    int *lab = L <= cap ? lsh + cap : idx + plane;
    int run = 0;   // entries written by earlier chunks (the same in every lane)
    for (int64_t c0 = 0; c0 < plane; c0 += chunk) {
        bool el[4];
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t p = c0 + 4 * t + u;
            el[u] = p < plane && eligible(p);
            cnt += el[u];
        }
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if ((t & 63) >= o) incl += y;
        }
        __syncthreads();   // wsum of the previous chunk has been read
        if ((t & 63) == 63) wsum[t >> 6] = incl;
        __syncthreads();
        int before = run;
        for (int w = 0; w < (t >> 6); ++w) before += wsum[w];
        int pos = before + incl - cnt;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (el[u]) {
                idx[pos] = (int)(c0 + 4 * t + u);
                lab[pos] = pos;
                ++pos;
            }
        for (int w = 0; w < (nt + 63) / 64; ++w) run += wsum[w];
    }
    __syncthreads();
    // components by union-find over the list: every entry is united with its
    // listed neighbours that come earlier in raster order (each pair once);
    // roots hook the larger position under the smaller with a compare-and-
    // swap, so parents only decrease and every root walk ends; then each
    // entry takes its root
    volatile int *par = lab;
    auto root = [&](int x) {
        while (par[x] != x) x = par[x];
        return x;
    };
    for (int e = t; e < L; e += nt) {
        const int p = idx[e], i = p % nx, j = p / nx;
        const int nb[4][2] = {{i - 1, j - 1}, {i, j - 1}, {i + 1, j - 1}, {i - 1, j}};
#pragma unroll
        for (int n4 = 0; n4 < 4; ++n4) {
            const int a = nb[n4][0], b = nb[n4][1];
            if (a < 0 || a >= nx || b < 0) continue;
            const int f = find_sorted(idx, L, b * nx + a);
            if (f < 0) continue;
            int x = e, y = f;
            for (;;) {
                x = root(x);
                y = root(y);
                if (x == y) break;
                if (x < y) { const int tmp = x; x = y; y = tmp; }
                if (atomicCAS(lab + x, x, y) == x) break;
            }
        }
    }
    __syncthreads();
    for (int e = t; e < L; e += nt) lab[e] = root(e);
    __syncthreads();
    // the seed is an edge pixel, so it is listed
    const int s = find_sorted(idx, L, sp);
    const int ls = s >= 0 ? lab[s] : -1;
    unsigned long long best = 0;
    const int *Ms = M + (int64_t)k * plane;
    for (int e = t; e < L; e += nt)
        if (lab[e] == ls) {
            const unsigned long long v = (unsigned long long)(unsigned)Ms[idx[e]] + 1ull;
            best = v > best ? v : best;
        }
    best = block_max_u64(best);
    if (t == 0) mt[k] = (long long)best - 1;
}

__global__ void k_sm_edge_mask(const int *M, const long long *mt, uint8_t *mask, int64_t V,
                               int64_t plane)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const long long t = mt[v / plane];
    mask[v] = t >= 0 && (long long)M[v] >= t;
}

}  // namespace hullmi
