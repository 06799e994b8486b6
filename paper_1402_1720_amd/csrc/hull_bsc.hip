// Binned SC kernels (the pass structure is described in hull_bsc.h).
#include <climits>

#include "hull_bsc.h"

namespace hullmi {

namespace {

// Sum over the wavefront, then one atomic per wavefront.
__device__ __forceinline__ void wave_add(unsigned long long *dst, unsigned long long v)
{
    if (!dst) return;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, v);
}

__device__ __forceinline__ long long floor_div_pos(long long a, long long n)
{
    long long q = a / n;
    if (q * n > a) --q;
    return q;
}

__device__ __forceinline__ double u128_to_double(unsigned __int128 x)
{
    return (double)(unsigned long long)(x >> 64) * 18446744073709551616.0 +
           (double)(unsigned long long)x;
}

__device__ __forceinline__ double i128_to_double(__int128 x)
{
    return x < 0 ? -u128_to_double((unsigned __int128)(-x)) : u128_to_double((unsigned __int128)x);
}

// floor(sqrt(T)) for T < 2^126: an FP64 estimate (within about 2^10 of the
// root), one Newton step in FP64 on the exact remainder T - r^2 (then within
// a few units), and exact integer corrections.
__device__ unsigned long long isqrt_u128(unsigned __int128 T)
{
    unsigned long long r = (unsigned long long)sqrt(u128_to_double(T));
    if (r > 0) {
        const __int128 e = (__int128)T - (__int128)((unsigned __int128)r * r);
        const double step = i128_to_double(e) / (2.0 * (double)r);
        const long long d = (long long)llrint(step);
        r = (unsigned long long)((long long)r + d);
    }
    while ((unsigned __int128)r * r > T) --r;
    while ((unsigned __int128)(r + 1) * (r + 1) <= T) ++r;
    return r;
}

struct SetAcc {
    uint8_t *v;
    __device__ __forceinline__ void operator()(int off) const { v[off] = 1; }
};

}  // namespace

// Pass 1. Blocks take consecutive chunks of histories; histories arrive angle
// by angle, so most of a chunk shares the gantry angle bin of its first
// history and is summed in an LDS copy of that detector plane (packed count
// and sum, then the sum of squares); the rest goes to the global sums.
__global__ void __launch_bounds__(kBscThreads)
k_bsc_stats(hullmi_histories h, FbpDev p, BscWs w, int64_t chunk, int use_lds)
{
    extern __shared__ unsigned long long lds[];
    const int plane = p.nu * p.nv;
    unsigned long long *la = lds, *lb = lds + plane;
    const int64_t base = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(base + chunk, h.n);
    if (base >= end) return;   // uniform across the block
    int k0 = -1;
    if (use_lds) {
        for (int b = threadIdx.x; b < 2 * plane; b += blockDim.x) lds[b] = 0ull;
        k0 = fbp_angle_bin(h.angle_deg[base], p);
    }
    __syncthreads();
    struct F8 { float xi, yi, zi, xo, yo, zo, a, w; };
    auto fetch = [&](int64_t i, F8 &f) {
        if (i < end) {
            f.xi = h.x_in[i]; f.yi = h.y_in[i]; f.zi = h.z_in[i];
            f.xo = h.x_out[i]; f.yo = h.y_out[i]; f.zo = h.z_out[i];
            f.a = h.angle_deg[i]; f.w = h.wepl[i];
        }
    };
    unsigned long long binned = 0;
    F8 nf{};
    fetch(base + threadIdx.x, nf);
    for (int64_t i = base + threadIdx.x; i < end; i += blockDim.x) {
        const F8 f = nf;
        fetch(i + blockDim.x, nf);
        int k, iu, iv;
        long long fx;
        int2 r = make_int2(-1, 0);
        if (fbp_locate_vals(f.xi, f.yi, f.zi, f.xo, f.yo, f.zo, f.a, f.w, p, k, iu, iv, fx)) {
            // |WEPL| < 2^16, so WEPL * 1024 is exact in FP32 and |w_q| <= 2^26
            const int wq = (int)rintf(f.w * 1024.0f);
            const int pb = iv * p.nu + iu;
            const int bin = k * plane + pb;
            r = make_int2(bin, wq);
            ++binned;
            const unsigned long long sq = (unsigned long long)((long long)wq * wq);
            if (k == k0 && wq > -kBscWide && wq < kBscWide) {
                atomicAdd(&la[pb], (1ull << kBscCountShift) + (unsigned long long)(wq + kBscWide));
                atomicAdd(&lb[pb], sq);
            } else {
                atomicAdd(w.cnt + bin, 1u);
                atomicAdd(w.s1 + bin, (unsigned long long)(long long)wq);
                atomicAdd(w.s2lo + bin, sq & 0xffffffffull);
                atomicAdd(w.s2hi + bin, sq >> 32);
            }
        }
        w.rec[i] = r;
    }
    wave_add(w.stats ? w.stats + kBscBinned : nullptr, binned);
    if (k0 < 0) return;   // uniform: k0 depends on the block only
    __syncthreads();
    const int64_t g0 = (int64_t)k0 * plane;
    for (int b = threadIdx.x; b < plane; b += blockDim.x) {
        const unsigned long long a = la[b];
        if (!a) continue;
        const unsigned c = (unsigned)(a >> kBscCountShift);
        const long long s = (long long)(a & ((1ull << kBscCountShift) - 1)) - (long long)c * kBscWide;
        const unsigned long long q = lb[b];
        atomicAdd(w.cnt + g0 + b, c);
        atomicAdd(w.s1 + g0 + b, (unsigned long long)s);
        atomicAdd(w.s2lo + g0 + b, q & 0xffffffffull);
        atomicAdd(w.s2hi + g0 + b, q >> 32);
    }
}

// Pass 2. With n binned histories, S1 = sum w_q and S2 = sum w_q^2, a history
// lies more than k population standard deviations from the mean iff
// (n w_q - S1)^2 > k^2 (n S2 - S1^2). With r = floor(sqrt(k^2 (n S2 - S1^2)))
// that is |n w_q - S1| > r, so the kept w_q form the integer range
// [ceil((S1 - r) / n), floor((S1 + r) / n)]. Empty bins keep nothing
// (lo > hi); k = 0 keeps everything.
__global__ void __launch_bounds__(256) k_bsc_bounds(BscWs w, int ksig)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long used = 0;
    if (b < w.nb) {
        const unsigned n = w.cnt[b];
        int lo = 1, hi = 0;
        if (n > 0) {
            used = 1;
            lo = INT_MIN;
            hi = INT_MAX;
            if (ksig > 0) {
                const long long S1 = (long long)w.s1[b];
                const unsigned __int128 S2 = ((unsigned __int128)w.s2hi[b] << 32) + w.s2lo[b];
                const unsigned __int128 R =
                    (unsigned __int128)n * S2 - (unsigned __int128)((__int128)S1 * S1);
                const unsigned __int128 T = (unsigned __int128)(unsigned)(ksig * ksig) * R;
                const unsigned long long r = isqrt_u128(T);
                // |n w_q - S1| < 2^58 for every possible w_q: a larger r keeps all
                if (r < (1ull << 59)) {
                    const long long l = -floor_div_pos(-(S1 - (long long)r), (long long)n);
                    const long long u = floor_div_pos(S1 + (long long)r, (long long)n);
                    const long long lim = 1ll << 27;   // beyond every w_q (|w_q| <= 2^26)
                    lo = (int)max(-lim, min(lim, l));
                    hi = (int)max(-lim, min(lim, u));
                }
            }
        }
        w.bnd[b] = make_int2(lo, hi);
    }
    wave_add(w.stats ? w.stats + kBscUsed : nullptr, used);
}

// Pass 3. The records of a chunk are tested against their bin's kept range;
// kept ones are summed in LDS copies of the detector planes of the chunk's
// first and last record (nplanes 2, or only the first), the rest directly.
__global__ void __launch_bounds__(kBscThreads)
k_bsc_cut(BscWs w, int64_t n, int plane, int64_t chunk, int nplanes)
{
    extern __shared__ unsigned long long lk[];
    const int64_t base = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(base + chunk, n);
    if (base >= end) return;
    for (int b = threadIdx.x; b < nplanes * plane; b += blockDim.x) lk[b] = 0ull;
    // first bin of each LDS plane (-1 when unused); a record is in plane p
    // iff pbase[p] <= bin < pbase[p] + plane
    int p0 = -1, p1 = -1;
    if (nplanes > 0) {
        const int b0 = w.rec[base].x;
        if (b0 >= 0) p0 = b0 - b0 % plane;
        if (nplanes > 1) {
            const int b1 = w.rec[end - 1].x;
            if (b1 >= 0) p1 = b1 - b1 % plane;
            if (p1 == p0) p1 = -1;
        }
    }
    __syncthreads();
    unsigned long long ncut = 0;
    int2 nr = make_int2(-1, 0);
    if (base + threadIdx.x < end) nr = w.rec[base + threadIdx.x];
    for (int64_t i = base + threadIdx.x; i < end; i += blockDim.x) {
        const int2 r = nr;
        if (i + blockDim.x < end) nr = w.rec[i + blockDim.x];
        if (r.x < 0) continue;
        const int2 bd = w.bnd[r.x];
        if (r.y < bd.x || r.y > bd.y) {
            ++ncut;
            continue;
        }
        const bool narrow = r.y > -kBscWide && r.y < kBscWide;
        if (narrow && p0 >= 0 && r.x >= p0 && r.x < p0 + plane) {
            atomicAdd(&lk[r.x - p0], (1ull << kBscCountShift) + (unsigned long long)(r.y + kBscWide));
        } else if (narrow && p1 >= 0 && r.x >= p1 && r.x < p1 + plane) {
            atomicAdd(&lk[plane + r.x - p1], (1ull << kBscCountShift) + (unsigned long long)(r.y + kBscWide));
        } else {
            atomicAdd(w.kept_n + r.x, 1u);
            atomicAdd(w.kept_s + r.x, (unsigned long long)(long long)r.y);
        }
    }
    wave_add(w.stats ? w.stats + kBscCut : nullptr, ncut);
    __syncthreads();
    for (int b = threadIdx.x; b < nplanes * plane; b += blockDim.x) {
        const int pb = b < plane ? p0 : p1;
        const unsigned long long a = lk[b];
        if (pb < 0 || !a) continue;
        const unsigned c = (unsigned)(a >> kBscCountShift);
        const long long s = (long long)(a & ((1ull << kBscCountShift) - 1)) - (long long)c * kBscWide;
        const int64_t g = (int64_t)pb + (b < plane ? b : b - plane);
        atomicAdd(w.kept_n + g, c);
        atomicAdd(w.kept_s + g, (unsigned long long)s);
    }
}

// Pass 4. One lane per bin: a bin that kept histories with mean WEPL below
// E_L (kept sum < e_q * kept count, exact) carves its line. The line runs from
// the source (-D, 0, 0) through the bin centre (0, u_c, v_c) on the detector
// plane, in the lab frame at the bin's gantry angle; it is rotated, scaled
// and rounded exactly as a history is, and every voxel of its A is marked.
__global__ void __launch_bounds__(256) k_bsc_carve(BscWs w, FbpDev p, DevGrid g, long long e_q)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long carved = 0, skipped = 0, visits = 0;
    if (b < w.nb) {
        const long long n = w.kept_n[b];
        const long long s = (long long)w.kept_s[b];
        if (n > 0 && s < e_q * n) {
            carved = 1;
            const int iu = (int)(b % p.nu);
            const int iv = (int)((b / p.nu) % p.nv);
            const int k = (int)(b / ((int64_t)p.nu * p.nv));
            const float uc = p.u0 + ((float)iu + 0.5f) * p.du;
            const float vc = p.v0 + ((float)iv + 0.5f) * p.dv;
            const float th = p.angle0 + (float)k * p.dangle;
            int a0, a1, a2, b0, b1, b2;
            bool ok = isfinite(uc) && isfinite(vc) && isfinite(th);
            if (ok) {
                float c, sn;
                deg_cos_sin(th, c, sn);
                ok = quantize_point(c, sn, -p.src_dist, 0.0f, 0.0f, g, a0, a1, a2) == kGeoOk &&
                     quantize_point(c, sn, 0.0f, uc, vc, g, b0, b1, b2) == kGeoOk &&
                     !(a0 == b0 && a1 == b1 && a2 == b2);
            }
            if (ok) {
                SetAcc acc{w.carved};
                visits = (unsigned long long)walk_line(a0, a1, a2, b0, b1, b2, g.nx, g.ny, g.nz, acc);
            } else {
                skipped = 1;
            }
        }
    }
    if (w.stats) {
        wave_add(w.stats + kBscCarved, carved);
        wave_add(w.stats + kBscSkipped, skipped);
        wave_add(w.stats + kBscVisits, visits);
    }
}

// Pass 5. mask = [den * (uncarved voxels of the (2r+1)^2 window in the slice,
// the outside counting as carved) > num * (2r+1)^2].
__global__ void __launch_bounds__(256)
k_bsc_blur(const uint8_t *carved, uint8_t *mask, int nx, int ny, int nz, int r, long long num_w2,
           int den)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (int64_t)nx * ny * nz) return;
    const int i = (int)(v % nx);
    const int j = (int)((v / nx) % ny);
    const int64_t k = v / ((int64_t)nx * ny);
    const uint8_t *sl = carved + k * nx * ny;
    int sum = 0;
    for (int y = max(j - r, 0); y <= min(j + r, ny - 1); ++y)
        for (int x = max(i - r, 0); x <= min(i + r, nx - 1); ++x) sum += sl[(int64_t)y * nx + x] ? 0 : 1;
    mask[v] = (long long)den * sum > num_w2;
}

}  // namespace hullmi
