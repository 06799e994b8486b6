// Binned SC kernels (the pass structure is described in hull_bsc.h).
#include <climits>

#include "hull_bsc.h"

namespace hullmi {

namespace {

// Sum over a (one-dimensional) block, then one atomic per block: counters
// shared by the whole grid are single addresses, and atomics on one address
// serialise. Every thread of the block must call it.
__device__ __forceinline__ void block_add(unsigned long long *dst, unsigned long long v)
{
    __shared__ unsigned long long part[kBscThreads / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) t += part[i];
        if (t) atomicAdd(dst, t);
    }
    __syncthreads();
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

// floor(sqrt(T)) for T < 2^126. Below 2^104 the FP64 root is within one of
// the answer; above, one Newton step on the exact remainder brings the FP64
// estimate (within about 2^10) to within a few units. Exact corrections last.
__device__ unsigned long long isqrt_u128(unsigned __int128 T)
{
    unsigned long long r = (unsigned long long)sqrt(u128_to_double(T));
    if ((T >> 104) != 0) {
        const __int128 e = (__int128)T - (__int128)((unsigned __int128)r * r);
        const double step = i128_to_double(e) / (2.0 * (double)r);
        r = (unsigned long long)((long long)r + (long long)llrint(step));
    }
    while ((unsigned __int128)r * r > T) --r;
    while ((unsigned __int128)(r + 1) * (r + 1) <= T) ++r;
    return r;
}

// floor(a / n) for n > 0 and |a / n| < 2^40: the FP64 quotient is within one
// of it, and exact products fix the last step.
__device__ __forceinline__ long long floor_div_pos(long long a, long long n)
{
    long long q = (long long)floor((double)a / (double)n);
    while (q * n > a) --q;
    while ((q + 1) * n <= a) ++q;
    return q;
}

// First bin of the detector plane that holds `bin` (-1 for -1).
__device__ __forceinline__ int plane_base(int bin, int plane) { return bin < 0 ? -1 : bin - bin % plane; }

__device__ __forceinline__ unsigned long long packed(int wq)
{
    return (1ull << kBscCountShift) + (unsigned long long)(wq + kBscWide);
}

__device__ __forceinline__ bool narrow(int wq) { return wq > -kBscWide && wq < kBscWide; }

// Adds a block's LDS plane words (packed count and sum) into the global
// count and sum arrays of the plane starting at bin g0.
__device__ __forceinline__ void flush_packed(const unsigned long long *l, int plane, int g0,
                                             unsigned *cnt, unsigned long long *sum)
{
    if (g0 < 0) return;
    for (int b = threadIdx.x; b < plane; b += blockDim.x) {
        const unsigned long long a = l[b];
        if (!a) continue;
        const unsigned c = (unsigned)(a >> kBscCountShift);
        const long long s = (long long)(a & ((1ull << kBscCountShift) - 1)) - (long long)c * kBscWide;
        atomicAdd(cnt + g0 + b, c);
        atomicAdd(sum + g0 + b, (unsigned long long)s);
    }
}

// Marks the part of A of a line that lies in z-slice k of an nx x ny grid:
// the slice-restricted set-up gives the first voxel and the in-plane decision
// variable, the set-up of the reversed line the last voxel (A does not
// depend on the direction); between them x steps when d < 0, y when d > 0
// and both when d = 0. 64-bit d: a line from a distant source has |D| near
// 2^21 (1/1024 voxel units). Voxel g (linear index) goes to bit g - wbase of
// the LDS window when it falls inside it, else to bit g of the global bit
// volume. Returns the voxels marked.
__device__ __forceinline__ int carve_slice(int a0, int a1, int a2, int b0, int b1, int b2, int nx,
                                           int ny, int k, unsigned *win, int64_t wbase,
                                           int64_t wbits, unsigned *gbits)
{
    const int zs = k * kQ;
    int off, last;
    int64_t d, incx, incy;
    int ox, oy;
    const int lim = 1 << 23;
    if (max(max(abs(a0), abs(a1)), max(abs(a2), max(abs(b0), max(abs(b1), abs(b2))))) < lim) {
        // exact in FP64 (the same result as the integer set-up below)
        const int32_t P[3] = {a0, a1, a2 - zs}, Q[3] = {b0, b1, b2 - zs};
        const int32_t D[3] = {b0 - a0, b1 - a1, b2 - a2}, R[3] = {a0 - b0, a1 - b1, a2 - b2};
        int fx, fy, lx, ly;
        double dd;
        if (!slice_entry_f64(P, D, nx, ny, true, fx, fy, &dd) ||
            !slice_entry_f64(Q, R, nx, ny, false, lx, ly, nullptr))
            return 0;
        off = fx + nx * fy;
        last = lx + nx * ly;
        d = (int64_t)dd;
        incx = 2048 * (int64_t)abs(D[1]);
        incy = -2048 * (int64_t)abs(D[0]);
        ox = D[0] > 0 ? 1 : -1;
        oy = (D[1] > 0 ? 1 : -1) * nx;
    } else {
        WalkInit f, r;
        if (!walk_init(a0, a1, a2 - zs, b0, b1, b2 - zs, nx, ny, 1, f) ||
            !walk_init(b0, b1, b2 - zs, a0, a1, a2 - zs, nx, ny, 1, r))
            return 0;
        off = f.cx + nx * f.cy;
        last = r.cx + nx * r.cy;
        incx = 2048 * f.Ay;
        incy = -2048 * f.Ax;
        ox = f.sx;
        oy = f.sy * nx;
        d = f.dxy;
    }
    // Both steps change d by a multiple of 2048 (incx = 2048 Ay, incy = -2048
    // Ax), so d = 2048 q + r with r = d mod 2048 fixed for the line: d < 0
    // exactly when q < 0, and d = 0 exactly when q = 0 and r = 0. The walk
    // keeps q, in 32 bits (|q| <= Ax + Ay + 1 < 2^23), and a line with r != 0
    // never takes a corner step.
    int32_t q = (int32_t)(d >> 11);
    const bool ties = (d & 2047) == 0;
    const int32_t ax = (int32_t)(-incy >> 11), ay = (int32_t)(incx >> 11);
    const int64_t sl = (int64_t)k * nx * ny;
    const bool all_in = sl - wbase >= 0 && sl + (int64_t)nx * ny - wbase <= wbits;
    int cnt = 0;
    if (all_in && !ties) {
        // the slice lies inside the LDS window and the line has no corner step
        unsigned *ws = win + ((sl - wbase) >> 5);
        const int sh = (int)((sl - wbase) & 31);   // 0: the window starts on a word
        for (int it = nx + ny; it > 0; --it) {
            const int rel = off + sh;
            atomicOr(ws + (rel >> 5), 1u << (rel & 31));
            ++cnt;
            if (off == last) break;
            const bool bx = q < 0;
            q += bx ? ay : -ax;
            off += bx ? ox : oy;
        }
        return cnt;
    }
    for (int it = nx + ny; it > 0; --it) {
        const int64_t gi = sl + off, rel = gi - wbase;
        if ((uint64_t)rel < (uint64_t)wbits)
            atomicOr(win + (rel >> 5), 1u << (rel & 31));
        else
            atomicOr(gbits + (gi >> 5), 1u << (gi & 31));
        ++cnt;
        if (off == last) break;
        const bool tie = ties && q == 0, bx = q < 0;
        q += tie ? ay - ax : (bx ? ay : -ax);
        off += tie ? ox + oy : (bx ? ox : oy);
    }
    return cnt;
}

// Object-frame quantised endpoints of bin b's carve line; false when the line
// is skipped (a non-finite value, an endpoint out of range, or coincident
// endpoints).
__device__ __forceinline__ bool bin_line(const BscWs &w, const FbpDev &p, const DevGrid &g, int b,
                                         int &a0, int &a1, int &a2, int &b0, int &b1, int &b2)
{
    const int iu = b % p.nu;
    const int iv = (b / p.nu) % p.nv;
    const int k = b / (p.nu * p.nv);
    const float uc = p.u0 + ((float)iu + 0.5f) * p.du;
    const float vc = p.v0 + ((float)iv + 0.5f) * p.dv;
    const float th = p.angle0 + (float)k * p.dangle;
    if (!(isfinite(uc) && isfinite(vc) && isfinite(th))) return false;
    const float2 cs = w.cs[k];
    return quantize_point(cs.x, cs.y, -p.src_dist, 0.0f, 0.0f, g, a0, a1, a2) == kGeoOk &&
           quantize_point(cs.x, cs.y, 0.0f, uc, vc, g, b0, b1, b2) == kGeoOk &&
           !(a0 == b0 && a1 == b1 && a2 == b2);
}

}  // namespace

// Pass 1. Blocks take consecutive chunks of histories. Histories arrive angle
// by angle, so the gantry angle bins of a chunk's first and last history
// usually hold all of it: each has an LDS copy of its detector plane (packed
// count and sum, nplanes = 2, or only the first); other histories, and WEPL
// beyond 1024 mm, go straight to the global sums.
__global__ void __launch_bounds__(kBscThreads)
k_bsc_stats(hullmi_histories h, FbpDev p, BscWs w, int64_t chunk, int nplanes)
{
    extern __shared__ unsigned long long lds[];
    const int plane = p.nu * p.nv;
    const int64_t base = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(base + chunk, h.n);
    if (base >= end) return;   // uniform across the block
    for (int b = threadIdx.x; b < nplanes * plane; b += blockDim.x) lds[b] = 0ull;
    const int k0 = nplanes > 0 ? fbp_angle_bin(h.angle_deg[base], p) : -1;
    int k1 = nplanes > 1 ? fbp_angle_bin(h.angle_deg[end - 1], p) : -1;
    if (k1 == k0) k1 = -1;
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
            if ((k == k0 || k == k1) && narrow(wq)) {
                atomicAdd(&lds[(k == k0 ? 0 : plane) + pb], packed(wq));
            } else {
                atomicAdd(w.cnt + bin, 1u);
                atomicAdd(w.s1 + bin, (unsigned long long)(long long)wq);
            }
        }
        w.rec[i] = r;
    }
    block_add(w.stats + kBscBinned, binned);
    __syncthreads();
    if (nplanes > 0) flush_packed(lds, plane, k0 < 0 ? -1 : k0 * plane, w.cnt, w.s1);
    if (nplanes > 1) flush_packed(lds + plane, plane, k1 < 0 ? -1 : k1 * plane, w.cnt, w.s1);
}

// Pass 2. Sum of w_q^2 per bin from the records, with the LDS planes of the
// chunk's first and last record (a plane's sum over at most 2^21 records of
// |w_q| < 2^20 stays below 2^61); the global sum is split at bit 32 so that
// it cannot overflow.
__global__ void __launch_bounds__(kBscThreads)
k_bsc_squares(BscWs w, int64_t n, int plane, int64_t chunk, int nplanes)
{
    extern __shared__ unsigned long long lq[];
    const int64_t base = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(base + chunk, n);
    if (base >= end) return;
    for (int b = threadIdx.x; b < nplanes * plane; b += blockDim.x) lq[b] = 0ull;
    const int p0 = nplanes > 0 ? plane_base(w.rec[base].x, plane) : -1;
    int p1 = nplanes > 1 ? plane_base(w.rec[end - 1].x, plane) : -1;
    if (p1 == p0) p1 = -1;
    __syncthreads();
    // kRecUnroll records per lane are loaded before any is used, so that
    // enough bytes are in flight to cover the memory latency
    const int64_t step = (int64_t)blockDim.x * kRecUnroll;
    for (int64_t i0 = base + threadIdx.x; i0 < end; i0 += step) {
        int2 rr[kRecUnroll];
#pragma unroll
        for (int u = 0; u < kRecUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * blockDim.x;
            rr[u] = i < end ? w.rec[i] : make_int2(-1, 0);
        }
#pragma unroll
        for (int u = 0; u < kRecUnroll; ++u) {
            const int2 r = rr[u];
            if (r.x < 0) continue;
            const unsigned long long sq = (unsigned long long)((long long)r.y * r.y);
            if (narrow(r.y) && p0 >= 0 && r.x >= p0 && r.x < p0 + plane) {
                atomicAdd(&lq[r.x - p0], sq);
            } else if (narrow(r.y) && p1 >= 0 && r.x >= p1 && r.x < p1 + plane) {
                atomicAdd(&lq[plane + r.x - p1], sq);
            } else {
                atomicAdd(w.s2lo + r.x, sq & 0xffffffffull);
                atomicAdd(w.s2hi + r.x, sq >> 32);
            }
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nplanes * plane; b += blockDim.x) {
        const int pb = b < plane ? p0 : p1;
        const unsigned long long q = lq[b];
        if (pb < 0 || !q) continue;
        const int64_t g = (int64_t)pb + (b < plane ? b : b - plane);
        atomicAdd(w.s2lo + g, q & 0xffffffffull);
        atomicAdd(w.s2hi + g, q >> 32);
    }
}

// Pass 3. With n binned histories, S1 = sum w_q and S2 = sum w_q^2, a history
// lies more than k population standard deviations from the mean iff
// (n w_q - S1)^2 > k^2 (n S2 - S1^2). With r = floor(sqrt(k^2 (n S2 - S1^2)))
// that is |n w_q - S1| > r, so the kept w_q form the integer range
// [ceil((S1 - r) / n), floor((S1 + r) / n)]. Empty bins keep nothing
// (lo > hi); k = 0 keeps everything.
__global__ void __launch_bounds__(kBscThreads) k_bsc_bounds(BscWs w, int ksig)
{
    unsigned long long used = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < w.nb; b += stride) {
        const unsigned n = w.cnt[b];
        int lo = 1, hi = 0;
        if (n > 0) {
            ++used;
            lo = INT_MIN;
            hi = INT_MAX;
            if (ksig > 0) {
                const long long S1 = (long long)w.s1[b];
                const unsigned __int128 S2 = ((unsigned __int128)w.s2hi[b] << 32) + w.s2lo[b];
                // n S2 >= S1^2 (Cauchy-Schwarz); T < 2^126 for k <= 64, n < 2^31
                const unsigned __int128 R =
                    (unsigned __int128)n * S2 - (unsigned __int128)((__int128)S1 * S1);
                const unsigned __int128 T = (unsigned __int128)(unsigned)(ksig * ksig) * R;
                const unsigned long long r = isqrt_u128(T);
                // r <= k n max|w_q - mean| < 2^34 n and |S1| <= 2^26 n, so both
                // quotients are below 2^35; the test only guards the arithmetic
                if (r < (1ull << 59)) {
                    const long long l = -floor_div_pos((long long)r - S1, (long long)n);
                    const long long u = floor_div_pos(S1 + (long long)r, (long long)n);
                    const long long lim = 1ll << 27;   // beyond every w_q (|w_q| <= 2^26)
                    lo = (int)max(-lim, min(lim, l));
                    hi = (int)max(-lim, min(lim, u));
                }
            }
        }
        w.bnd[b] = make_int2(lo, hi);
    }
    block_add(w.stats + kBscUsed, used);
}

// Pass 4. The records of a chunk are tested against their bin's kept range;
// kept ones are summed in the LDS planes of the chunk's first and last record
// (nplanes 2, or only the first), the rest directly. With fsum set (the FDK
// hull after cuts) each cut history is also taken out of the FDK bin sums
// (WEPL in 2^-16 mm, from wepl) and counts.
__global__ void __launch_bounds__(kBscThreads)
k_bsc_cut(BscWs w, int64_t n, int plane, int64_t chunk, int nplanes, const float *wepl,
          unsigned long long *fsum, unsigned *fcnt)
{
    extern __shared__ unsigned long long lk[];
    const int64_t base = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(base + chunk, n);
    if (base >= end) return;
    for (int b = threadIdx.x; b < nplanes * plane; b += blockDim.x) lk[b] = 0ull;
    const int p0 = nplanes > 0 ? plane_base(w.rec[base].x, plane) : -1;
    int p1 = nplanes > 1 ? plane_base(w.rec[end - 1].x, plane) : -1;
    if (p1 == p0) p1 = -1;
    __syncthreads();
    unsigned long long ncut = 0;
    // kRecUnroll records per lane, then their kept ranges, are loaded before
    // any is used
    const int64_t step = (int64_t)blockDim.x * kRecUnroll;
    for (int64_t i0 = base + threadIdx.x; i0 < end; i0 += step) {
        int2 rr[kRecUnroll], bd[kRecUnroll];
#pragma unroll
        for (int u = 0; u < kRecUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * blockDim.x;
            rr[u] = i < end ? w.rec[i] : make_int2(-1, 0);
        }
#pragma unroll
        for (int u = 0; u < kRecUnroll; ++u) bd[u] = rr[u].x >= 0 ? w.bnd[rr[u].x] : make_int2(1, 0);
#pragma unroll
        for (int u = 0; u < kRecUnroll; ++u) {
            const int2 r = rr[u];
            if (r.x < 0) continue;
            if (r.y < bd[u].x || r.y > bd[u].y) {
                ++ncut;
                if (fsum) {
                    const long long fx = llrint((double)wepl[i0 + (int64_t)u * blockDim.x] * 65536.0);
                    atomicAdd(fsum + r.x, (unsigned long long)(-fx));
                    atomicAdd(fcnt + r.x, 0xffffffffu);
                }
                continue;
            }
            if (narrow(r.y) && p0 >= 0 && r.x >= p0 && r.x < p0 + plane) {
                atomicAdd(&lk[r.x - p0], packed(r.y));
            } else if (narrow(r.y) && p1 >= 0 && r.x >= p1 && r.x < p1 + plane) {
                atomicAdd(&lk[plane + r.x - p1], packed(r.y));
            } else {
                atomicAdd(w.kept_n + r.x, 1u);
                atomicAdd(w.kept_s + r.x, (unsigned long long)(long long)r.y);
            }
        }
    }
    block_add(w.stats + kBscCut, ncut);
    __syncthreads();
    if (nplanes > 0) flush_packed(lk, plane, p0, w.kept_n, w.kept_s);
    if (nplanes > 1) flush_packed(lk + plane, plane, p1, w.kept_n, w.kept_s);
}

// cos and sin of every bin's gantry angle angle0 + k dangle (FP32), as the
// geometry of a history takes them.
__global__ void k_bsc_trig(BscWs w, FbpDev p)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.n_angles) return;
    const float th = p.angle0 + (float)k * p.dangle;
    float c = 0.0f, s = 0.0f;
    if (isfinite(th)) deg_cos_sin(th, c, s);
    w.cs[k] = make_float2(c, s);
}

// Pass 5. A bin that kept histories with mean WEPL below E_L (kept sum <
// e_q * kept count, exact) goes on the carve list. With row_first the list
// runs over detector rows first (row iv, then gantry angle, then iu), so that
// a stretch of it holds lines of one row, which stay within a few slices
// whatever the angle; otherwise it is in bin order (angle first), which mixes
// long and short lines evenly. Each block owns a contiguous stretch of that
// order: it counts its carved bins, reserves that many list entries with one
// atomic, then writes them in order.
__device__ __forceinline__ int64_t row_major_bin(int64_t j, const FbpDev &p, int row_first)
{
    if (!row_first) return j;
    const int64_t per_row = (int64_t)p.n_angles * p.nu;
    const int64_t iv = j / per_row, rem = j - iv * per_row;
    const int64_t k = rem / p.nu, iu = rem - k * p.nu;
    return (k * p.nv + iv) * p.nu + iu;
}

__device__ __forceinline__ bool bsc_carves(const BscWs &w, int64_t b, long long e_q)
{
    const long long n = w.kept_n[b];
    return n > 0 && (long long)w.kept_s[b] < e_q * n;
}

__global__ void __launch_bounds__(kBscThreads)
k_bsc_select(BscWs w, FbpDev p, long long e_q, int row_first)
{
    __shared__ int wcnt[kBscThreads / 64];
    __shared__ int sbase;
    const int64_t per = (w.nb + gridDim.x - 1) / gridDim.x;
    const int64_t j0 = (int64_t)blockIdx.x * per, j1 = min(j0 + per, w.nb);
    unsigned long long mine = 0;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x)
        mine += bsc_carves(w, row_major_bin(j, p, row_first), e_q);
    // block total, then one reservation
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mine += __shfl_down(mine, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) / 64;
    if (lane == 0) wcnt[wave] = (int)mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < nw; ++i) t += wcnt[i];
        sbase = t ? atomicAdd(w.nlist, t) : 0;
        if (t) atomicAdd(w.stats + kBscCarved, (unsigned long long)t);
    }
    __syncthreads();
    int run = sbase;
    for (int64_t s0 = j0; s0 < j1; s0 += blockDim.x) {
        const int64_t j = s0 + threadIdx.x;
        const int64_t b = j < j1 ? row_major_bin(j, p, row_first) : 0;
        const bool c = j < j1 && bsc_carves(w, b, e_q);
        const unsigned long long m = __ballot(c);
        if (lane == 0) wcnt[wave] = __popcll(m);
        __syncthreads();
        int off = run;
        for (int i = 0; i < wave; ++i) off += wcnt[i];
        if (c) w.list[off + __popcll(m & ((1ull << lane) - 1))] = (int)b;
        for (int i = wave; i < nw; ++i) off += wcnt[i];
        run = off;   // the same for every thread: all counts of this round added
        __syncthreads();
    }
}

// Pass 6. Each block owns an equal share of the carve list (when the whole
// volume does not fit the LDS window the list runs rows first, so a share is
// mostly one detector row and its lines stay within a few slices). It first finds the slice range of its lines and
// places an LDS bit window of `lwords` words there; then its lanes take the
// next line from an LDS counter (lanes that finish short lines early take
// more) and mark every voxel of the line's A, slice by slice, in the window or
// (outside it) in the global bit volume; last the window is ORed into the
// global bits, one atomic per non-zero word. Each line runs from the source
// (-D, 0, 0) through the bin centre (0, u_c, v_c) on the detector plane, in
// the lab frame at the bin's gantry angle, rotated, scaled and rounded
// exactly as a history is.
__global__ void __launch_bounds__(kCarveThreads)
k_bsc_carve(BscWs w, FbpDev p, DevGrid g, int lwords)
{
    extern __shared__ unsigned win[];
    __shared__ int next, zlo;
    const int nl = *w.nlist;
    const int per = (int)(((int64_t)nl + gridDim.x - 1) / gridDim.x);
    const int i0 = (int)min((int64_t)blockIdx.x * per, (int64_t)nl);
    const int i1 = min(i0 + per, nl);
    if (i0 >= i1) return;   // uniform across the block
    if (threadIdx.x == 0) {
        next = i0;
        zlo = INT_MAX;
    }
    for (int j = threadIdx.x; j < lwords; j += blockDim.x) win[j] = 0u;
    __syncthreads();
    const int64_t plane = (int64_t)g.nx * g.ny;
    int a0, a1, a2, b0, b1, b2;
    // a window that holds the whole volume starts at voxel 0; a smaller one
    // starts at the lowest slice the block's lines can meet
    if ((int64_t)lwords * 32 < plane * g.nz) {
        for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
            if (!bin_line(w, p, g, w.list[i], a0, a1, a2, b0, b1, b2)) continue;
            if (!line_meets_grid(a0, a1, a2, b0, b1, b2, g.nx, g.ny, g.nz)) continue;
            int z0, z1;
            line_z_cover(a0, a1, a2, b0, b1, b2, g.nx, g.ny, g.nz, z0, z1);
            atomicMin(&zlo, z0);
        }
    } else if (threadIdx.x == 0) {
        zlo = 0;
    }
    __syncthreads();
    const int64_t wbase = zlo == INT_MAX ? 0 : ((int64_t)zlo * plane) & ~int64_t(31);
    const int64_t wbits = (int64_t)lwords * 32;
    unsigned long long skipped = 0, visits = 0;
    for (;;) {
        const int i = atomicAdd(&next, 1);
        if (i >= i1) break;
        if (!bin_line(w, p, g, w.list[i], a0, a1, a2, b0, b1, b2)) {
            ++skipped;
            continue;
        }
        // whether A is empty (from the slab where it is clear, else exactly),
        // then the slices that cover it
        LineSlab sb;
        line_slab(a0, a1, a2, b0, b1, b2, g.nx, g.ny, g.nz, sb);
        int meets = slab_meets(sb, a0, a1, a2, b0, b1, b2, g.nx, g.ny, g.nz);
        if (meets < 0) meets = line_meets_grid(a0, a1, a2, b0, b1, b2, g.nx, g.ny, g.nz);
        if (!meets) continue;
        int z0, z1;
        slab_z_cover(sb, g.nz, z0, z1);
        for (int z = z0; z <= z1; ++z)
            visits += (unsigned long long)carve_slice(a0, a1, a2, b0, b1, b2, g.nx, g.ny, z, win,
                                                      wbase, wbits, w.cbits);
    }
    __syncthreads();
    const int64_t gw0 = wbase >> 5, gwn = (plane * g.nz + 31) >> 5;
    for (int j = threadIdx.x; j < lwords; j += blockDim.x) {
        const unsigned v = win[j];
        if (v && gw0 + j < gwn) atomicOr(w.cbits + gw0 + j, v);
    }
    block_add(w.stats + kBscSkipped, skipped);
    block_add(w.stats + kBscVisits, visits);
}

// Zeroes the per-bin sums and counters, the carved bit volume (vwords
// words), the carve list length and the statistics.
__global__ void __launch_bounds__(256) k_bsc_clear(BscWs w, int64_t vwords)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t b = t0; b < w.nb; b += stride) {
        w.cnt[b] = 0u;
        w.s1[b] = 0ull;
        w.s2lo[b] = 0ull;
        w.s2hi[b] = 0ull;
        w.kept_n[b] = 0u;
        w.kept_s[b] = 0ull;
    }
    for (int64_t v = t0; v < vwords; v += stride) w.cbits[v] = 0u;
    if (t0 < kBscStatWords) w.stats[t0] = 0ull;
    if (t0 == 0) *w.nlist = 0;
}

// Pass 7. mask = [den * (uncarved voxels of the (2r+1)^2 window in the slice,
// the outside counting as carved) > num * (2r+1)^2]; carved (when not null)
// gets the carved flags as bytes. A block covers a kBlurTx x kBlurTy tile of
// one slice: the uncarved flags of the tile and its halo go to LDS, then row
// sums, then column sums.
__global__ void __launch_bounds__(kBlurTx * kBlurTy)
k_bsc_blur(const unsigned *cbits, uint8_t *carved, uint8_t *mask, int nx, int ny, int r,
           long long num_w2, int den)
{
    constexpr int kMaxR = 15;
    constexpr int kW = kBlurTx + 2 * kMaxR, kH = kBlurTy + 2 * kMaxR;
    __shared__ uint8_t u[kH][kW];
    __shared__ short rs[kH][kBlurTx];
    const int x0 = blockIdx.x * kBlurTx, y0 = blockIdx.y * kBlurTy;
    const int64_t sl = (int64_t)blockIdx.z * nx * ny;
    const int tw = kBlurTx + 2 * r, th = kBlurTy + 2 * r;
    const int t = threadIdx.y * kBlurTx + threadIdx.x;
    for (int e = t; e < tw * th; e += kBlurTx * kBlurTy) {
        const int ty = e / tw, tx = e - ty * tw;
        const int x = x0 - r + tx, y = y0 - r + ty;
        uint8_t v = 0;
        if (x >= 0 && x < nx && y >= 0 && y < ny) {
            const int64_t gi = sl + (int64_t)y * nx + x;
            v = ((cbits[gi >> 5] >> (gi & 31)) & 1u) ? 0 : 1;
        }
        u[ty][tx] = v;
    }
    __syncthreads();
    for (int e = t; e < th * kBlurTx; e += kBlurTx * kBlurTy) {
        const int ty = e / kBlurTx, tx = e - ty * kBlurTx;
        int s = 0;
        for (int a = 0; a <= 2 * r; ++a) s += u[ty][tx + a];
        rs[ty][tx] = (short)s;
    }
    __syncthreads();
    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    int s = 0;
    for (int a = 0; a <= 2 * r; ++a) s += rs[threadIdx.y + a][threadIdx.x];
    const int64_t gi = sl + (int64_t)y * nx + x;
    mask[gi] = (long long)den * s > num_w2;
    if (carved) carved[gi] = 1 - u[threadIdx.y + r][threadIdx.x + r];
}

}  // namespace hullmi
