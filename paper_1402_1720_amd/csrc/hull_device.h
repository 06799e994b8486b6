// Device-side building blocks of the hull path for gfx950: the FP32 geometry
// that turns a history into a quantised object-frame line, and the exact
// integer walk that enumerates the voxel set A_i of that line (Sections 3.2
// and 3.4 of the paper; A_i read as the half-open voxel boxes that the
// infinite line meets).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hullmi {

constexpr int kQ = 1024;            // endpoints in units of 1/1024 voxel
constexpr float kGMax = 65536.0f;   // |g| < 2^16 voxels

enum : int { kGeoOk = 0, kGeoNonFinite = 1, kGeoRange = 2, kGeoDegenerate = 3 };

struct DevGrid {
    int nx, ny, nz;
    float rdx, rdy, rdz;   // 1.0f / voxel size, rounded once on the host
    float x0, y0, z0;
};

// cos/sin of an angle in degrees: remainder modulo 360 (exact in FP64), FP64
// cos/sin, rounded to FP32.
__device__ __forceinline__ void deg_cos_sin(float a, float &c, float &s)
{
    const double th = (double)a;
    const double r = th - 360.0 * floor(th / 360.0);
    const double rad = r * 0.017453292519943295;
    c = (float)cos(rad);
    s = (float)sin(rad);
}

// Object frame (lab rotated by -theta about z), voxel units, 1/1024 rounding.
__device__ __forceinline__ int quantize_point(float c, float s, float x, float y, float z,
                                              const DevGrid &g, int &qx, int &qy, int &qz)
{
    const float xo = c * x + s * y;
    const float yo = c * y - s * x;
    const float gx = (xo - g.x0) * g.rdx;
    const float gy = (yo - g.y0) * g.rdy;
    const float gz = (z - g.z0) * g.rdz;
    if (!(fabsf(gx) < kGMax && fabsf(gy) < kGMax && fabsf(gz) < kGMax)) return kGeoRange;
    qx = (int)rintf(gx * (float)kQ);
    qy = (int)rintf(gy * (float)kQ);
    qz = (int)rintf(gz * (float)kQ);
    return kGeoOk;
}

// Exact product of two int32 values. Every factor of the set-up below fits in
// 32 bits: coordinates are below 2^26 in magnitude (2^27 after a slice
// shift, grid axes at most 2048 voxels), so differences, entry distances and
// next-crossing distances stay below 2^28 and every product below 2^56.
__device__ __forceinline__ int64_t mul64(int32_t a, int32_t b) { return (int64_t)a * (int64_t)b; }

// Voxel index on a moving axis at the entry key e / A of the entry axis:
// floor(num / (kQ A)) with num = P A + D e, or ceil(num / (kQ A)) - 1 when
// `up`; -1 when it lies outside [0, n). Once num is known to lie in range the
// quotient is below n <= 2048, and its FP32 estimate (a few 2^-24 relative
// error) is within 2^-10 of it: flooring is off by at most one, and two exact
// comparisons fix that.
__device__ __forceinline__ int entry_index(int32_t P, int32_t D, int32_t e, int32_t A, bool up, int n)
{
    const int64_t num = mul64(P, A) + mul64(D, e);
    const int64_t lim = mul64(n * kQ, A);
    if (up ? (num <= 0 || num > lim) : (num < 0 || num >= lim)) return -1;
    // up: ceil(num / den) - 1 = floor((num - 1) / den) for integers
    const int64_t a = up ? num - 1 : num;
    const float est = (float)a * __builtin_amdgcn_rcpf((float)A) * (1.0f / (float)kQ);
    int q = (int)floorf(est);
    q = max(0, min(q, n - 1));
    if (mul64(q * kQ, A) > a) --q;
    if (mul64((q + 1) * kQ, A) <= a) ++q;
    return q;
}

// Walk state after set-up: the first voxel of A_i and, per axis, the next
// crossing written as pairwise decision variables.
//
// Parameterise the line as P(t) = P0 + t D. The index on a moving axis a
// changes at plane crossings; with the half-open reading an increasing axis
// takes its new index at the crossing itself and a decreasing axis just after
// it. Order crossings by the key (t, sigma) with sigma = 0 for increasing and
// 1 for decreasing axes; crossings with equal keys happen together. With
// e_a / A_a the t of axis a's next crossing (A_a = |D_a|), the key order of
// axes a and b is the sign of d_ab = 2 (e_a A_b - e_b A_a) + (sigma_a -
// sigma_b): exact, integer, and updated by +-2048 A when an axis steps.
// A fixed axis gets e = 1, A = 0, sigma = 0, which makes it never step.
struct WalkInit {
    int cx, cy, cz;          // first voxel
    int64_t dxy, dxz, dyz;   // decision variables
    int64_t Ax, Ay, Az;      // |D|
    int sx, sy, sz;          // +-1 per axis
};

// Returns false when the line misses the grid.
__device__ __forceinline__ bool walk_init(int qix, int qiy, int qiz, int qox, int qoy, int qoz,
                                          int nx, int ny, int nz, WalkInit &w)
{
    const int32_t P[3] = {qix, qiy, qiz};
    const int32_t D[3] = {qox - qix, qoy - qiy, qoz - qiz};
    const int n[3] = {nx, ny, nz};
    int32_t A[3], en[3];
    int g[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        // a fixed axis must already lie inside the grid
        if (D[b] == 0 && (P[b] < 0 || P[b] >= kQ * n[b])) return false;
        A[b] = D[b] < 0 ? -D[b] : D[b];
        // entry key of a moving axis: t = en / A, sigma = (D < 0)
        en[b] = D[b] > 0 ? -P[b] : P[b] - kQ * n[b];
        g[b] = D[b] < 0;
    }
    // the latest entry key decides where the line enters the grid
    int wa = -1;
    int32_t ew = 0, aw = 1;
    int gw = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        if (!A[b]) continue;
        if (wa >= 0) {
            const int64_t l = mul64(en[b], aw), r = mul64(ew, A[b]);
            if (!(l > r || (l == r && g[b] > gw))) continue;
        }
        wa = b; ew = en[b]; aw = A[b]; gw = g[b];
    }
    // voxel index of each axis at the entry key
    int c[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        if (b == wa) {
            c[b] = D[b] > 0 ? 0 : n[b] - 1;
        } else if (D[b] == 0) {
            c[b] = P[b] >> 10;
        } else {
            // a decreasing axis rounds up when a decreasing axis decides the entry
            c[b] = entry_index(P[b], D[b], ew, aw, gw && D[b] < 0, n[b]);
            if (c[b] < 0) return false;
        }
    }
    // next crossing per axis (|e| < 2^28)
    int32_t e[3];
#pragma unroll
    for (int b = 0; b < 3; ++b)
        e[b] = D[b] > 0 ? kQ * (c[b] + 1) - P[b] : (D[b] < 0 ? P[b] - kQ * c[b] : 1);
    w.dxy = 2 * (mul64(e[0], A[1]) - mul64(e[1], A[0])) + (g[0] - g[1]);
    w.dxz = 2 * (mul64(e[0], A[2]) - mul64(e[2], A[0])) + (g[0] - g[2]);
    w.dyz = 2 * (mul64(e[1], A[2]) - mul64(e[2], A[1])) + (g[1] - g[2]);
    w.Ax = A[0]; w.Ay = A[1]; w.Az = A[2];
    w.cx = c[0]; w.cy = c[1]; w.cz = c[2];
    w.sx = D[0] > 0 ? 1 : -1; w.sy = D[1] > 0 ? 1 : -1; w.sz = D[2] > 0 ? 1 : -1;
    return true;
}

// Enumerates A_i from the initial voxel, calling acc(linear_index) once per
// voxel, and returns |A_i|. T holds the decision variables: int32 is exact
// when every |D| < 2^19 (then |d| <= 4096 max A + 1 < 2^31 at every step),
// int64 always.
template <typename T, class Acc>
__device__ __forceinline__ int walk_run(const WalkInit &w, int nx, int ny, int nz, Acc &acc)
{
    T dxy = (T)w.dxy, dxz = (T)w.dxz, dyz = (T)w.dyz;
    const T Kx = (T)(2048 * w.Ax), Ky = (T)(2048 * w.Ay), Kz = (T)(2048 * w.Az);
    int cx = w.cx, cy = w.cy, cz = w.cz;
    const int ox = w.sx, oy = w.sy * nx, oz = w.sz * nx * ny;
    int off = cx + nx * (cy + ny * cz);
    const int maxit = nx + ny + nz;
    int cnt = 0;
    for (int it = 0; it < maxit; ++it) {
        acc(off);
        ++cnt;
        const bool bx = (dxy <= 0) & (dxz <= 0);
        const bool by = (dxy >= 0) & (dyz <= 0);
        const bool bz = (dxz >= 0) & (dyz >= 0);
        dxy += (bx ? Ky : (T)0) - (by ? Kx : (T)0);
        dxz += (bx ? Kz : (T)0) - (bz ? Kx : (T)0);
        dyz += (by ? Kz : (T)0) - (bz ? Ky : (T)0);
        cx += bx ? w.sx : 0;
        cy += by ? w.sy : 0;
        cz += bz ? w.sz : 0;
        off += (bx ? ox : 0) + (by ? oy : 0) + (bz ? oz : 0);
        if (((unsigned)cx >= (unsigned)nx) | ((unsigned)cy >= (unsigned)ny) |
            ((unsigned)cz >= (unsigned)nz))
            break;
    }
    return cnt;
}

template <class Acc>
__device__ __forceinline__ int walk_line(int qix, int qiy, int qiz, int qox, int qoy, int qoz,
                                         int nx, int ny, int nz, Acc &acc)
{
    WalkInit w;
    if (!walk_init(qix, qiy, qiz, qox, qoy, qoz, nx, ny, nz, w)) return 0;
    const int64_t amax = max(w.Ax, max(w.Ay, w.Az));
    if (amax < (int64_t(1) << 19)) return walk_run<int32_t>(w, nx, ny, nz, acc);
    return walk_run<int64_t>(w, nx, ny, nz, acc);
}

}  // namespace hullmi

namespace hullmi {

// The part of A_i inside one z-slice. The z index is constant there, so once
// the first and the last voxel are known (the last is the first voxel of the
// reversed line, since A_i does not depend on the direction) the walk needs
// only the x/y decision variable d: x steps when d < 0, y when d > 0, both
// when d = 0 (the line passes through a voxel corner with both indices moving
// the same way; mixed directions never tie, the sigma term breaks it), and
// every step changes d by incx, incy or both.
//
// The loops are written directly in gfx950 assembly (the compiler keeps the
// loop guard and the any-lane test in vector registers; here they are
// scalar). Counters are 16 bits, two to an LDS word, in tile rows of an odd
// number S of counters: the counter of voxel (x, y) is number L = x + S y, so
// an x step (L +- 1) and a y step (L +- S) both move to the other half of a
// word, and a corner step (both) stays in the same half. The value a step
// adds to its word (1 or 65536) therefore alternates with every step that is
// not a corner step. Lanes leave the exec mask when they have visited `last`;
// the loop also ends after maxit rounds. Only LDS is touched: `off` and `last`
// are LDS byte addresses of 16-bit counters (tile base + 2 L, the base a
// multiple of 4), so the word is off & ~3; `val` is what the first step adds
// (65536 when bit 1 of off is set, else 1).
//
// General loop: 12 VALU instructions and one ds_add_u32 per step.
__device__ __forceinline__ void walk_slice_lds16(int32_t d, int32_t off, int32_t last,
                                                 int32_t incx, int32_t incy, int32_t ox,
                                                 int32_t oy, uint32_t val, int32_t maxit)
{
    const int32_t incxy = incx + incy, oxy = ox + oy;
    const uint32_t flip = 65537u;
    int32_t t0, t1, t2;
    uint64_t save, sbx, stie;
    int32_t it = maxit;
    asm volatile(
        "s_mov_b64 %[save], exec\n"
        "1:\n"
        // compares first: every SGPR a VALU writes is read at least three
        // instructions later (gfx950 needs wait states between the two)
        "v_cmp_gt_i32 %[sbx], 0, %[d]\n"
        "v_cmp_eq_u32 %[stie], 0, %[d]\n"
        "v_cmp_ne_u32 vcc, %[off], %[last]\n"
        "v_and_b32 %[t0], -4, %[off]\n"
        "v_cndmask_b32 %[t2], %[incy], %[incxy], %[stie]\n"
        "v_cndmask_b32 %[t2], %[t2], %[incx], %[sbx]\n"
        "v_add_u32 %[d], %[d], %[t2]\n"
        "ds_add_u32 %[t0], %[val]\n"
        // the next step adds to the other half unless this was a corner step
        "v_cndmask_b32 %[t1], %[flip], 0, %[stie]\n"
        "v_cndmask_b32 %[t2], %[oy], %[oxy], %[stie]\n"
        "v_cndmask_b32 %[t2], %[t2], %[ox], %[sbx]\n"
        "v_add_u32 %[off], %[off], %[t2]\n"
        "v_xor_b32 %[val], %[val], %[t1]\n"
        "s_and_b64 exec, exec, vcc\n"
        "s_cbranch_execz 2f\n"
        "s_sub_u32 %[it], %[it], 1\n"
        "s_cmp_eq_u32 %[it], 0\n"
        "s_cbranch_scc0 1b\n"
        "2:\n"
        "s_mov_b64 exec, %[save]\n"
        : [d] "+v"(d), [off] "+v"(off), [val] "+v"(val), [it] "+s"(it), [t0] "=&v"(t0),
          [t1] "=&v"(t1), [t2] "=&v"(t2), [save] "=&s"(save), [sbx] "=&s"(sbx),
          [stie] "=&s"(stie)
        : [last] "v"(last), [incx] "v"(incx), [incy] "v"(incy), [incxy] "v"(incxy),
          [ox] "v"(ox), [oy] "v"(oy), [oxy] "v"(oxy), [flip] "v"(flip)
        : "vcc", "scc", "memory");
}

// walk_slice_lds16 for lines whose decision variable is never zero in the
// slice, so that each step is an x step (d < 0) or a y step (d > 0) and the
// added value alternates at every step: two steps per round, the first
// adding `val`, the second val ^ 65537, each step 7 VALU instructions and one
// ds_add_u32; the same voxels. d = 0 means that the next x and y crossings
// coincide, i.e. the line passes through a voxel corner with both indices
// moving the same way. That never happens when d is odd (both increments of d
// are even, so an odd d stays odd: the x and y steps go in opposite
// directions), nor when the projected line holds no lattice corner at all
// (corner_free below). maxit bounds the steps (rounds of two).
__device__ __forceinline__ void walk_slice_lds16_nocorner(int32_t d, int32_t off, int32_t last,
                                                          int32_t incx, int32_t incy, int32_t ox,
                                                          int32_t oy, uint32_t val, int32_t maxit)
{
    const uint32_t val2 = val ^ 65537u;
    int32_t t0, t1, t2;
    uint64_t save, sbx, sdone;
    int32_t it = (maxit + 1) >> 1;
    asm volatile(
        "s_mov_b64 %[save], exec\n"
        "1:\n"
        "v_cmp_gt_i32 %[sbx], 0, %[d]\n"
        "v_cmp_ne_u32 %[sdone], %[off], %[last]\n"
        "v_and_b32 %[t0], -4, %[off]\n"
        "v_cndmask_b32 %[t2], %[incy], %[incx], %[sbx]\n"
        "v_add_u32 %[d], %[d], %[t2]\n"
        "ds_add_u32 %[t0], %[val]\n"
        "v_cndmask_b32 %[t2], %[oy], %[ox], %[sbx]\n"
        "v_add_u32 %[off], %[off], %[t2]\n"
        "s_and_b64 exec, exec, %[sdone]\n"
        "s_cbranch_execz 2f\n"
        "v_cmp_gt_i32 %[sbx], 0, %[d]\n"
        "v_cmp_ne_u32 %[sdone], %[off], %[last]\n"
        "v_and_b32 %[t1], -4, %[off]\n"
        "v_cndmask_b32 %[t2], %[incy], %[incx], %[sbx]\n"
        "v_add_u32 %[d], %[d], %[t2]\n"
        "ds_add_u32 %[t1], %[val2]\n"
        "v_cndmask_b32 %[t2], %[oy], %[ox], %[sbx]\n"
        "v_add_u32 %[off], %[off], %[t2]\n"
        "s_and_b64 exec, exec, %[sdone]\n"
        "s_cbranch_execz 2f\n"
        "s_sub_u32 %[it], %[it], 1\n"
        "s_cmp_eq_u32 %[it], 0\n"
        "s_cbranch_scc0 1b\n"
        "2:\n"
        "s_mov_b64 exec, %[save]\n"
        : [d] "+v"(d), [off] "+v"(off), [it] "+s"(it), [t0] "=&v"(t0), [t1] "=&v"(t1),
          [t2] "=&v"(t2), [save] "=&s"(save), [sbx] "=&s"(sbx), [sdone] "=&s"(sdone)
        : [last] "v"(last), [incx] "v"(incx), [incy] "v"(incy), [ox] "v"(ox), [oy] "v"(oy),
          [val] "v"(val), [val2] "v"(val2)
        : "scc", "memory");
}

// walk_slice_lds16_nocorner on word addresses. Every step of a corner-free
// line moves its counter to the other half of a word, so the first step of
// each round is always on the half the line starts on and the second on the
// other one: the word-address change of an x step and of a y step at each of
// the two positions is fixed for the line (dxa, dya for the first, dxb, dyb
// for the second), and the loop keeps the word address itself instead of
// masking a counter address at every step. The last voxel is reached at a
// first step when its half is the starting half, else at a second step, so
// each position compares with the last voxel's word only where it can be
// reached (last_a, last_b; -1 where it cannot, which no word address equals;
// a line visits each voxel once, so a match at that position is the last
// voxel). The same voxels in the same order; 6 VALU instructions and one
// ds_add_u32 per step.
__device__ __forceinline__ void walk_slice_lds16_nocorner_w(int32_t d, int32_t w, int32_t last_a,
                                                            int32_t last_b, int32_t incx,
                                                            int32_t incy, int32_t dxa,
                                                            int32_t dya, int32_t dxb, int32_t dyb,
                                                            uint32_t val, int32_t maxit)
{
    const uint32_t val2 = val ^ 65537u;
    int32_t t2, t3, w2;
    uint64_t save, sbx, sdone;
    int32_t it = (maxit + 1) >> 1;
    // the two steps of a round keep the word address in alternate registers
    // (w, then w2), so no register is written right after a ds_add_u32 that
    // reads it
    asm volatile(
        "s_mov_b64 %[save], exec\n"
        "1:\n"
        // compares first: every SGPR a VALU writes is read at least three
        // instructions later
        "v_cmp_gt_i32 %[sbx], 0, %[d]\n"
        "v_cmp_ne_u32 %[sdone], %[w], %[la]\n"
        "ds_add_u32 %[w], %[val]\n"
        "v_cndmask_b32 %[t2], %[incy], %[incx], %[sbx]\n"
        "v_cndmask_b32 %[t3], %[dya], %[dxa], %[sbx]\n"
        "v_add_u32 %[d], %[d], %[t2]\n"
        "v_add_u32 %[w2], %[w], %[t3]\n"
        "s_and_b64 exec, exec, %[sdone]\n"
        "s_cbranch_execz 2f\n"
        "v_cmp_gt_i32 %[sbx], 0, %[d]\n"
        "v_cmp_ne_u32 %[sdone], %[w2], %[lb]\n"
        "ds_add_u32 %[w2], %[val2]\n"
        "v_cndmask_b32 %[t2], %[incy], %[incx], %[sbx]\n"
        "v_cndmask_b32 %[t3], %[dyb], %[dxb], %[sbx]\n"
        "v_add_u32 %[d], %[d], %[t2]\n"
        "v_add_u32 %[w], %[w2], %[t3]\n"
        "s_and_b64 exec, exec, %[sdone]\n"
        "s_cbranch_execz 2f\n"
        "s_sub_u32 %[it], %[it], 1\n"
        "s_cmp_eq_u32 %[it], 0\n"
        "s_cbranch_scc0 1b\n"
        "2:\n"
        "s_mov_b64 exec, %[save]\n"
        : [d] "+v"(d), [w] "+v"(w), [it] "+s"(it), [t2] "=&v"(t2), [t3] "=&v"(t3),
          [w2] "=&v"(w2), [save] "=&s"(save), [sbx] "=&s"(sbx), [sdone] "=&s"(sdone)
        : [la] "v"(last_a), [lb] "v"(last_b), [incx] "v"(incx), [incy] "v"(incy),
          [dxa] "v"(dxa), [dya] "v"(dya), [dxb] "v"(dxb), [dyb] "v"(dyb), [val] "v"(val),
          [val2] "v"(val2)
        : "scc", "memory");
}

// Whether the line's projection on the x-y plane passes through no voxel
// corner (no point with both coordinates multiples of kQ): a corner
// (kQ i, kQ j) on P + t D needs kQ (Dy i - Dx j) = Dy Px - Dx Py, so it
// cannot exist when Dy Px - Dx Py is not a multiple of kQ. Only the low ten
// bits of that product are needed, and 32-bit wrap-around keeps them.
// Sufficient, not necessary: lines it cannot clear walk the general loop.
__device__ __forceinline__ bool corner_free(int32_t px, int32_t py, int32_t dx, int32_t dy)
{
    const uint32_t c = (uint32_t)dy * (uint32_t)px - (uint32_t)dx * (uint32_t)py;
    return (c & (uint32_t)(kQ - 1)) != 0u;
}

// Walk state of A_i inside z-slice k for walk_slice_lds16, set up once per
// (line, slice) by walk_init's entry rule restricted to the slice (the line
// for the first voxel and d, the reversed line for the last voxel): the
// decision variable, the first and the last voxel (in-plane index x + stride
// y, stride >= nx being the length of a tile row), |D| on x
// and y (d changes by 2048 Ay per x step and by -2048 Ax per y step) and the
// step directions. first = last = -1 when the line does not meet the slice
// inside the grid. Exact when |D| < 2^19 on x and y (the int32 condition of
// the loop).
struct SliceState {
    int32_t d, first, last, ax, ay, sx, sy;
};

// The slice set-up in FP64. For endpoint coordinates below 2^23 in magnitude
// (2^24 after the slice shift of at most 2047 slices) every entry distance is
// below 2^25 and every |D| below 2^24, so every product below is below 2^49
// and every sum below 2^51: all exact in a double, and the results equal
// those of the integer set-up. FP64 operations issue at half the FP32 rate,
// 64-bit integer multiplies at a quarter of it. The binned SC's carve lines
// (from a source far outside the grid) use this form; tile lines use the
// 24-bit integer one below.
__device__ __forceinline__ bool slice_entry_f64(const int32_t P[3], const int32_t D[3], int nx,
                                                int ny, bool check_z, int &cx, int &cy,
                                                double *dxy)
{
    // Every lane computes every case and selects: the per-lane branches
    // (axis not moving, entry axis, range checks) would otherwise cost a
    // divergent branch each.
    const int n[3] = {nx, ny, 1};
    double A[3], en[3];
    int g[3];
    bool ok = true;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        ok &= !((D[b] == 0) & ((P[b] < 0) | (P[b] >= kQ * n[b])));
        A[b] = (double)(D[b] < 0 ? -D[b] : D[b]);
        en[b] = (double)(D[b] > 0 ? -P[b] : P[b] - kQ * n[b]);
        g[b] = D[b] < 0;
    }
    // entry axis: the moving axis whose slab is entered last (largest en / A),
    // ties to the axis that steps down
    int wa = -1;
    double ew = 0.0, aw = 1.0;
    int gw = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const double l = en[b] * aw, r = ew * A[b];
        const bool take = (D[b] != 0) & ((wa < 0) | (l > r) | ((l == r) & (g[b] > gw)));
        wa = take ? b : wa;
        ew = take ? en[b] : ew;
        aw = take ? A[b] : aw;
        gw = take ? g[b] : gw;
    }
    // products and sums below are exact in a double, so an FMA gives the same values
    if (check_z) {
        const double num = __builtin_fma((double)P[2], aw, (double)D[2] * ew);
        const double lim = (double)kQ * aw;
        const bool up = (gw != 0) & (D[2] < 0);
        const bool bad = (up & ((num <= 0.0) | (num > lim))) | (!up & ((num < 0.0) | (num >= lim)));
        ok &= !((wa != 2) & (D[2] != 0) & bad);
    }
    const double den = (double)kQ * aw;
    const double rden = __builtin_amdgcn_rcp(den);
    int c[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const double num = __builtin_fma((double)P[b], aw, (double)D[b] * ew);
        const double lim = (double)n[b] * den;
        const bool up = (gw != 0) & (D[b] < 0);
        const bool bad = (up & ((num <= 0.0) | (num > lim))) | (!up & ((num < 0.0) | (num >= lim)));
        // up: ceil(num / den) - 1 = floor((num - 1) / den); the estimate is
        // off by at most one, fixed by two exact comparisons (clamped first,
        // so that the conversion stays in range where the line misses)
        const double a = up ? num - 1.0 : num;
        const double e = fmin(fmax(floor(a * rden), 0.0), (double)(n[b] - 1));
        int q = (int)e;
        q -= (double)q * den > a ? 1 : 0;
        q += (double)(q + 1) * den <= a ? 1 : 0;
        const bool moving = (D[b] != 0) & (b != wa);
        ok &= !(moving & bad);
        c[b] = b == wa ? (D[b] > 0 ? 0 : n[b] - 1) : (D[b] == 0 ? P[b] >> 10 : q);
    }
    cx = c[0];
    cy = c[1];
    if (dxy) {
        const int32_t ex = D[0] > 0 ? kQ * (c[0] + 1) - P[0] : (D[0] < 0 ? P[0] - kQ * c[0] : 1);
        const int32_t ey = D[1] > 0 ? kQ * (c[1] + 1) - P[1] : (D[1] < 0 ? P[1] - kQ * c[1] : 1);
        *dxy = 2.0 * __builtin_fma((double)ex, A[1], -((double)ey * A[0])) + (double)(g[0] - g[1]);
    }
    return ok;
}

// Exact 48-bit product of two integers of magnitude below 2^23, from the
// full-rate 24-bit multiplies (low 32 bits, then bits 32..47 sign-extended);
// written out because the compiler otherwise falls back to quarter-rate 64-bit
// multiplies where it cannot prove the operands' range.
__device__ __forceinline__ int64_t mul_i24(int32_t a, int32_t b)
{
    int32_t lo, hi;
    asm("v_mul_i32_i24 %0, %1, %2" : "=v"(lo) : "v"(a), "v"(b));
    asm("v_mul_hi_i32_i24 %0, %1, %2" : "=v"(hi) : "v"(a), "v"(b));
    return (int64_t)((uint64_t)(uint32_t)hi << 32 | (uint32_t)lo);
}

// Low 32 bits of the product of two integers below 2^24 (full rate).
__device__ __forceinline__ uint32_t mul_u24(uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// slice_entry_f64 in integers, for tile lines: every endpoint coordinate below
// 2^20 in magnitude and |D| < 2^19 on x and y, slice k < 2048, so that P
// (below 2^21 + 2^20 on z after the slice shift), D, A and the entry
// distances all stay below 2^23 and every product is an exact 24 x 24-bit one.
// The floor division by den = 1024 aw is (num >> 10) / aw for num >= 0, whose
// quotient is below n <= 2048 and whose dividend then fits 32 bits: an FP32
// estimate (off by at most one) fixed by two exact comparisons. Same
// decisions as slice_entry_f64, at full-rate integer instructions instead of
// half-rate FP64 ones. dxy is the decision variable in 32-bit wrap-around
// arithmetic: exact whenever its value fits 32 bits, as it does on a tile line.
__device__ __forceinline__ bool slice_entry_i24(const int32_t P[3], const int32_t D[3], int nx,
                                                int ny, bool check_z, int &cx, int &cy,
                                                int32_t *dxy)
{
    const int n[3] = {nx, ny, 1};
    int32_t A[3], en[3];
    int g[3];
    bool ok = true;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        // an axis the line does not move along must hold the point; the
        // reversed line from the other endpoint has the same such axes, at the
        // same coordinates, so only the first call (check_z) tests them
        if (check_z) ok &= !((D[b] == 0) & ((P[b] < 0) | (P[b] >= kQ * n[b])));
        A[b] = D[b] < 0 ? -D[b] : D[b];
        en[b] = D[b] > 0 ? -P[b] : P[b] - kQ * n[b];
        g[b] = D[b] < 0;
    }
    int wa = -1;
    int32_t ew = 0, aw = 1;
    int gw = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int64_t l = mul_i24(en[b], aw), r = mul_i24(ew, A[b]);
        const bool take = (D[b] != 0) & ((wa < 0) | (l > r) | ((l == r) & (g[b] > gw)));
        wa = take ? b : wa;
        ew = take ? en[b] : ew;
        aw = take ? A[b] : aw;
        gw = take ? g[b] : gw;
    }
    // The entry point's coordinate on a non-entry axis is num / den with den =
    // 1024 aw; the voxel is floor(num / den), or ceil(num / den) - 1 =
    // floor((num - 1) / den) where the walk steps down (up). With a = num or
    // num - 1, it lies in [0, n) exactly when a >= 0 and floor(a / 1024) < n aw
    // (the half-open range test on num, [0, n den) or (0, n den], restated).
    if (check_z) {
        const bool up = (gw != 0) & (D[2] < 0);
        const int64_t a = mul_i24(P[2], aw) + mul_i24(D[2], ew) - (up ? 1 : 0);
        const bool bad = (a < 0) | ((a >> 10) >= (int64_t)aw);
        ok &= !((wa != 2) & (D[2] != 0) & bad);
    }
    const float raw = __builtin_amdgcn_rcpf((float)aw);
    int c[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const bool up = (gw != 0) & (D[b] < 0);
        const int64_t a = mul_i24(P[b], aw) + mul_i24(D[b], ew) - (up ? 1 : 0);
        const bool bad = (a < 0) | ((a >> 10) >= mul_i24(n[b], aw));
        // where the axis is in range, m = floor(a / 1024) < n aw <= 2^32; a
        // lane whose line misses computes a bounded q that is never used
        const uint32_t m = (uint32_t)(a >> 10);
        int q = (int)fminf((float)m * raw, 4096.0f);
        q = min(q, n[b] - 1);
        const uint32_t qa = mul_u24((uint32_t)q, (uint32_t)aw);   // q aw < n aw <= 2^32: exact
        q -= qa > m ? 1 : 0;
        q += mul_u24((uint32_t)(q + 1), (uint32_t)aw) <= m ? 1 : 0;
        ok &= !(((D[b] != 0) & (b != wa)) & bad);
        c[b] = b == wa ? (D[b] > 0 ? 0 : n[b] - 1) : (D[b] == 0 ? P[b] >> 10 : q);
    }
    cx = c[0];
    cy = c[1];
    if (dxy) {
        const int32_t ex = D[0] > 0 ? kQ * (c[0] + 1) - P[0] : (D[0] < 0 ? P[0] - kQ * c[0] : 1);
        const int32_t ey = D[1] > 0 ? kQ * (c[1] + 1) - P[1] : (D[1] < 0 ? P[1] - kQ * c[1] : 1);
        const uint32_t cross = (uint32_t)mul_i24(ex, A[1]) - (uint32_t)mul_i24(ey, A[0]);
        *dxy = (int32_t)(2u * cross + (uint32_t)(g[0] - g[1]));
    }
    return ok;
}

__device__ __forceinline__ void slice_state_tile(int qix, int qiy, int qiz, int qox, int qoy, int qoz,
                                                 int nx, int ny, int stride, int k, SliceState &s)
{
    const int zs = k * kQ;
    const int32_t P[3] = {qix, qiy, qiz - zs}, Q[3] = {qox, qoy, qoz - zs};
    const int32_t D[3] = {qox - qix, qoy - qiy, qoz - qiz};
    const int32_t R[3] = {-D[0], -D[1], -D[2]};
    int fx, fy, lx, ly;
    int32_t d;
    const bool in_first = slice_entry_i24(P, D, nx, ny, true, fx, fy, &d);
    const bool in_last = slice_entry_i24(Q, R, nx, ny, false, lx, ly, nullptr);
    // selected rather than branched on: a line that misses the slice gets
    // first = last = -1 and zeros
    const bool in = in_first & in_last;
    s.d = in ? d : 0;
    s.first = in ? fx + (int)mul_u24((uint32_t)stride, (uint32_t)fy) : -1;
    s.last = in ? lx + (int)mul_u24((uint32_t)stride, (uint32_t)ly) : -1;
    s.ax = in ? (D[0] < 0 ? -D[0] : D[0]) : 0;
    s.ay = in ? (D[1] < 0 ? -D[1] : D[1]) : 0;
    s.sx = (in & (D[0] <= 0)) ? -1 : 1;
    s.sy = (in & (D[1] <= 0)) ? -1 : 1;
}

// Whether A_i is not empty, exactly when walk_init returns true: the entry key
// as walk_init picks it, then every axis only range-checked, which needs no
// division (for den > 0, floor(num / den) lies in [0, n) iff
// 0 <= num < n den, and ceil(num / den) - 1 lies in [0, n) iff
// 0 < num <= n den).
__device__ __forceinline__ bool line_meets_grid(int qix, int qiy, int qiz, int qox, int qoy, int qoz,
                                                int nx, int ny, int nz)
{
    const int32_t P[3] = {qix, qiy, qiz};
    const int32_t D[3] = {qox - qix, qoy - qiy, qoz - qiz};
    const int n[3] = {nx, ny, nz};
    int wa = -1;
    int32_t ew = 0, aw = 1;
    int gw = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int32_t L = kQ * n[b];
        if (D[b] == 0) {
            if (P[b] < 0 || P[b] >= L) return false;
            continue;
        }
        const int32_t A = D[b] < 0 ? -D[b] : D[b];
        const int32_t en = D[b] > 0 ? -P[b] : P[b] - L;
        const int g = D[b] < 0;
        if (wa >= 0) {
            const int64_t l = mul64(en, aw), r = mul64(ew, A);
            if (!(l > r || (l == r && g > gw))) continue;
        }
        wa = b; ew = en; aw = A; gw = g;
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        if (b == wa || D[b] == 0) continue;
        const int64_t num = mul64(P[b], aw) + mul64(D[b], ew);
        const int64_t lim = mul64(kQ * n[b], aw);
        const bool up = gw && D[b] < 0;
        if (up ? (num <= 0 || num > lim) : (num < 0 || num >= lim)) return false;
    }
    return true;
}

// A range of z-slices that holds every slice A_i meets (for a line that meets
// the grid): the z extent of the line's part inside the grid box in FP32,
// widened by far more than its rounding error. Slices it adds that the line
// does not meet are found empty by the exact slice set-up.
// The FP32 slab of a line against the grid box: p and d in voxel units, and
// the entry and exit parameters tlo, thi of P(t) = p + t d over the moving
// axes (an axis with D = 0 is left out: it bounds nothing). err bounds the
// FP32 error of tlo and thi, with room to spare: per moving axis t = (c - p)
// times the hardware reciprocal of d (p, d, c - p and the product each
// rounded once, the reciprocal within 1 ulp: below 5.5 2^-24 relative) is off
// by less than (n + 2 |p|) / |d| 2^-21, and err is 16 times the largest such
// bound.
struct LineSlab {
    float p[3], d[3];
    float tlo, thi, err;
};

__device__ __forceinline__ void line_slab(int qix, int qiy, int qiz, int qox, int qoy, int qoz,
                                          int nx, int ny, int nz, LineSlab &b)
{
    const float s = 1.0f / (float)kQ;
    b.p[0] = qix * s; b.p[1] = qiy * s; b.p[2] = qiz * s;
    b.d[0] = (float)((int64_t)qox - qix) * s;
    b.d[1] = (float)((int64_t)qoy - qiy) * s;
    b.d[2] = (float)((int64_t)qoz - qiz) * s;
    const float n[3] = {(float)nx, (float)ny, (float)nz};
    float tlo = -3.0e38f, thi = 3.0e38f, e = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (b.d[a] != 0.0f) {
            const float r = __builtin_amdgcn_rcpf(b.d[a]);
            const float t0 = (0.0f - b.p[a]) * r, t1 = (n[a] - b.p[a]) * r;
            tlo = fmaxf(tlo, fminf(t0, t1));
            thi = fminf(thi, fmaxf(t0, t1));
            e = fmaxf(e, (n[a] + 2.0f * fabsf(b.p[a])) * fabsf(r));
        }
    }
    b.tlo = tlo;
    b.thi = thi;
    b.err = e * (1.0f / 131072.0f);
}

// Whether A_i is not empty, decided from the slab where the margin is clear:
// 1 when the line passes through the inside of the box (tlo < thi by more
// than twice the error bound), 0 when it clearly misses it or a fixed axis
// lies outside the grid (exact, in integers), -1 when only the exact test
// (line_meets_grid) can tell: a line that touches an edge, a face or a corner.
__device__ __forceinline__ int slab_meets(const LineSlab &b, int qix, int qiy, int qiz, int qox,
                                          int qoy, int qoz, int nx, int ny, int nz)
{
    if (qox == qix && (qix < 0 || qix >= kQ * nx)) return 0;
    if (qoy == qiy && (qiy < 0 || qiy >= kQ * ny)) return 0;
    if (qoz == qiz && (qiz < 0 || qiz >= kQ * nz)) return 0;
    if (b.tlo < b.thi - 2.0f * b.err) return 1;
    if (b.tlo > b.thi + 2.0f * b.err) return 0;
    return -1;
}

// A range of z-slices that holds every slice A_i meets, from the slab.
__device__ __forceinline__ void slab_z_cover(const LineSlab &b, int nz, int &k0, int &k1)
{
    const float nzf = (float)nz;
    float za = b.p[2], zb = b.p[2];
    if (b.d[2] != 0.0f) {
        za = b.p[2] + b.tlo * b.d[2];
        zb = b.p[2] + b.thi * b.d[2];
    }
    const float lo = fminf(za, zb), hi = fmaxf(za, zb);
    const float m = (fabsf(b.p[2]) + fabsf(lo) + fabsf(hi) + nzf) * (1.0f / 65536.0f) + 1.0f / 1024.0f;
    k0 = (int)fmaxf(floorf(lo - m), 0.0f);
    k1 = (int)fminf(floorf(hi + m), nzf - 1.0f);
    if (k1 < k0) k1 = k0;   // cannot happen for a line that meets the grid
}

__device__ __forceinline__ void line_z_cover(int qix, int qiy, int qiz, int qox, int qoy, int qoz,
                                             int nx, int ny, int nz, int &k0, int &k1)
{
    LineSlab b;
    line_slab(qix, qiy, qiz, qox, qoy, qoz, nx, ny, nz, b);
    slab_z_cover(b, nz, k0, k1);
}

}  // namespace hullmi
