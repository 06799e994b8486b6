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

// floor(a / b) for b > 0 when the quotient is known to satisfy |a / b| < 2^12:
// an FP32 estimate (relative error a few 2^-24, so within 2^-10 of a / b) is
// off by at most one after flooring, and two exact integer comparisons fix it.
__device__ __forceinline__ int64_t floor_div_small(int64_t a, int64_t b)
{
    int64_t q = (int64_t)floorf((float)a * __builtin_amdgcn_rcpf((float)b));
    if (q * b > a) --q;
    if ((q + 1) * b <= a) ++q;
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
    const int64_t Px = qix, Py = qiy, Pz = qiz;
    const int64_t Dx = (int64_t)qox - qix, Dy = (int64_t)qoy - qiy, Dz = (int64_t)qoz - qiz;
    const int64_t Lx = (int64_t)kQ * nx, Ly = (int64_t)kQ * ny, Lz = (int64_t)kQ * nz;
    // a fixed axis must already lie inside the grid
    if (Dx == 0 && (Px < 0 || Px >= Lx)) return false;
    if (Dy == 0 && (Py < 0 || Py >= Ly)) return false;
    if (Dz == 0 && (Pz < 0 || Pz >= Lz)) return false;
    const int64_t Ax = Dx < 0 ? -Dx : Dx, Ay = Dy < 0 ? -Dy : Dy, Az = Dz < 0 ? -Dz : Dz;
    // entry key of each moving axis: t = en / A, sigma = (D < 0)
    const int64_t enx = Dx > 0 ? -Px : Px - Lx;
    const int64_t eny = Dy > 0 ? -Py : Py - Ly;
    const int64_t enz = Dz > 0 ? -Pz : Pz - Lz;
    const int gx = Dx < 0, gy = Dy < 0, gz = Dz < 0;
    // the latest entry key decides where the line enters the grid
    int wa = -1;
    int64_t ew = 0, aw = 1;
    int gw = 0;
    if (Ax) { wa = 0; ew = enx; aw = Ax; gw = gx; }
    if (Ay) {
        const int64_t l = eny * aw, r = ew * Ay;
        if (wa < 0 || l > r || (l == r && gy > gw)) { wa = 1; ew = eny; aw = Ay; gw = gy; }
    }
    if (Az) {
        const int64_t l = enz * aw, r = ew * Az;
        if (wa < 0 || l > r || (l == r && gz > gw)) { wa = 2; ew = enz; aw = Az; gw = gz; }
    }
    const int64_t den = (int64_t)kQ * aw;
    // voxel index of each axis at the entry key
    int64_t c[3];
    const int64_t P[3] = {Px, Py, Pz}, D[3] = {Dx, Dy, Dz};
    const int n[3] = {nx, ny, nz};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        if (b == wa) {
            c[b] = D[b] > 0 ? 0 : n[b] - 1;
        } else if (D[b] == 0) {
            c[b] = P[b] >> 10;
        } else {
            // c = floor(num / den), or ceil(num / den) - 1 for a decreasing axis
            // when a decreasing axis decides the entry; checked against [0, n)
            // before dividing (den > 0), so the quotient is small
            const int64_t num = P[b] * aw + D[b] * ew;
            const bool up = gw && D[b] < 0;
            if (up ? (num <= 0 || num > (int64_t)n[b] * den) : (num < 0 || num >= (int64_t)n[b] * den))
                return false;
            c[b] = up ? -floor_div_small(-num, den) - 1 : floor_div_small(num, den);
        }
    }
    // next crossing per axis
    const int64_t ex = Dx > 0 ? (int64_t)kQ * (c[0] + 1) - Px : (Dx < 0 ? Px - (int64_t)kQ * c[0] : 1);
    const int64_t ey = Dy > 0 ? (int64_t)kQ * (c[1] + 1) - Py : (Dy < 0 ? Py - (int64_t)kQ * c[1] : 1);
    const int64_t ez = Dz > 0 ? (int64_t)kQ * (c[2] + 1) - Pz : (Dz < 0 ? Pz - (int64_t)kQ * c[2] : 1);
    w.dxy = 2 * (ex * Ay - ey * Ax) + (gx - gy);
    w.dxz = 2 * (ex * Az - ez * Ax) + (gx - gz);
    w.dyz = 2 * (ey * Az - ez * Ay) + (gy - gz);
    w.Ax = Ax; w.Ay = Ay; w.Az = Az;
    w.cx = (int)c[0]; w.cy = (int)c[1]; w.cz = (int)c[2];
    w.sx = Dx > 0 ? 1 : -1; w.sy = Dy > 0 ? 1 : -1; w.sz = Dz > 0 ? 1 : -1;
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
// The loop is written directly in gfx950 assembly (the compiler keeps the loop
// guard and the any-lane test in vector registers; here they are scalar): per
// step 12 VALU instructions and one ds_add_u32 into the 16-bit LDS tile. Lanes
// leave the exec mask when they have visited `last`; the loop also ends after
// maxit rounds. Only LDS is touched: `off` and `last` are LDS byte addresses
// of 16-bit counters (tile base + 2 * voxel, the base a multiple of 4), so the
// word is off & ~3 and the half is bit 1 of off.
__device__ __forceinline__ void walk_slice_lds16(int32_t d, int32_t off, int32_t last,
                                                 int32_t incx, int32_t incy, int32_t ox,
                                                 int32_t oy, int32_t maxit)
{
    const int32_t incxy = incx + incy, oxy = ox + oy;
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
        "v_bfe_u32 %[t1], %[off], 1, 1\n"
        "v_cndmask_b32 %[t2], %[incy], %[incxy], %[stie]\n"
        "v_cndmask_b32 %[t2], %[t2], %[incx], %[sbx]\n"
        "v_add_u32 %[d], %[d], %[t2]\n"
        "v_mad_u32_u24 %[t1], %[t1], %[k16], 1\n"
        "ds_add_u32 %[t0], %[t1]\n"
        "v_cndmask_b32 %[t2], %[oy], %[oxy], %[stie]\n"
        "v_cndmask_b32 %[t2], %[t2], %[ox], %[sbx]\n"
        "v_add_u32 %[off], %[off], %[t2]\n"
        "s_and_b64 exec, exec, vcc\n"
        "s_cbranch_execz 2f\n"
        "s_sub_u32 %[it], %[it], 1\n"
        "s_cmp_eq_u32 %[it], 0\n"
        "s_cbranch_scc0 1b\n"
        "2:\n"
        "s_mov_b64 exec, %[save]\n"
        : [d] "+v"(d), [off] "+v"(off), [it] "+s"(it), [t0] "=&v"(t0), [t1] "=&v"(t1),
          [t2] "=&v"(t2), [save] "=&s"(save), [sbx] "=&s"(sbx), [stie] "=&s"(stie)
        : [last] "v"(last), [incx] "v"(incx), [incy] "v"(incy), [incxy] "v"(incxy),
          [ox] "v"(ox), [oy] "v"(oy), [oxy] "v"(oxy), [k16] "s"(65535)
        : "vcc", "scc", "memory");
}

// Walk state of A_i inside z-slice k for walk_slice_lds16, set up once per
// (line, slice) from two walk_init calls restricted to the slice (forward for
// the first voxel and d, reversed for the last voxel): the decision
// variable, the byte offsets 2 * voxel of the first and the last
// voxel, the changes of d per x and per y step, and the byte steps per x step
// (low 16 bits of `steps`, signed) and per y step (high 16 bits, signed).
// first = last = -1 when the line does not meet the slice inside the grid.
// Exact when |D| < 2^19 on x and y (the int32 condition of the loop).
struct SliceState {
    int32_t d, first, last, incx, incy, steps;
};

__device__ __forceinline__ void slice_state(int qix, int qiy, int qiz, int qox, int qoy, int qoz,
                                            int nx, int ny, int k, SliceState &s)
{
    const int zs = k * kQ;
    WalkInit a, b;
    if (!walk_init(qix, qiy, qiz - zs, qox, qoy, qoz - zs, nx, ny, 1, a) ||
        !walk_init(qox, qoy, qoz - zs, qix, qiy, qiz - zs, nx, ny, 1, b)) {
        s.d = 0; s.first = -1; s.last = -1; s.incx = 0; s.incy = 0; s.steps = 0;
        return;
    }
    s.d = (int32_t)a.dxy;
    s.first = 2 * (a.cx + nx * a.cy);
    s.last = 2 * (b.cx + nx * b.cy);
    s.incx = (int32_t)(2048 * a.Ay);
    s.incy = (int32_t)(-2048 * a.Ax);
    const int32_t ox = 2 * a.sx, oy = 2 * a.sy * nx;
    s.steps = (int32_t)(((uint32_t)oy << 16) | ((uint32_t)ox & 0xffffu));
}

// Whether A_i is not empty, exactly when walk_init returns true: the entry key
// as walk_init picks it, then every axis only range-checked, which needs no
// division (for den > 0, floor(num / den) lies in [0, n) iff
// 0 <= num < n den, and ceil(num / den) - 1 lies in [0, n) iff
// 0 < num <= n den).
__device__ __forceinline__ bool line_meets_grid(int qix, int qiy, int qiz, int qox, int qoy, int qoz,
                                                int nx, int ny, int nz)
{
    const int64_t P[3] = {qix, qiy, qiz};
    const int64_t D[3] = {(int64_t)qox - qix, (int64_t)qoy - qiy, (int64_t)qoz - qiz};
    const int n[3] = {nx, ny, nz};
    int wa = -1;
    int64_t ew = 0, aw = 1;
    int gw = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int64_t L = (int64_t)kQ * n[b];
        if (D[b] == 0) {
            if (P[b] < 0 || P[b] >= L) return false;
            continue;
        }
        const int64_t A = D[b] < 0 ? -D[b] : D[b];
        const int64_t en = D[b] > 0 ? -P[b] : P[b] - L;
        const int g = D[b] < 0;
        if (wa >= 0) {
            const int64_t l = en * aw, r = ew * A;
            if (!(l > r || (l == r && g > gw))) continue;
        }
        wa = b; ew = en; aw = A; gw = g;
    }
    const int64_t den = (int64_t)kQ * aw;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        if (b == wa || D[b] == 0) continue;
        const int64_t num = P[b] * aw + D[b] * ew;
        const bool up = gw && D[b] < 0;
        if (up ? (num <= 0 || num > (int64_t)n[b] * den) : (num < 0 || num >= (int64_t)n[b] * den))
            return false;
    }
    return true;
}

// A range of z-slices that holds every slice A_i meets (for a line that meets
// the grid): the z extent of the line's part inside the grid box in FP32,
// widened by far more than its rounding error. Slices it adds that the line
// does not meet are found empty by the exact slice set-up.
__device__ __forceinline__ void line_z_cover(int qix, int qiy, int qiz, int qox, int qoy, int qoz,
                                             int nx, int ny, int nz, int &k0, int &k1)
{
    const float s = 1.0f / (float)kQ;
    const float p[3] = {qix * s, qiy * s, qiz * s};
    const float d[3] = {(float)((int64_t)qox - qix) * s, (float)((int64_t)qoy - qiy) * s,
                        (float)((int64_t)qoz - qiz) * s};
    const float n[3] = {(float)nx, (float)ny, (float)nz};
    float tlo = -3.0e38f, thi = 3.0e38f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0f) {
            const float t0 = (0.0f - p[a]) / d[a], t1 = (n[a] - p[a]) / d[a];
            tlo = fmaxf(tlo, fminf(t0, t1));
            thi = fminf(thi, fmaxf(t0, t1));
        }
    }
    float za = p[2], zb = p[2];
    if (d[2] != 0.0f) {
        za = p[2] + tlo * d[2];
        zb = p[2] + thi * d[2];
    }
    const float lo = fminf(za, zb), hi = fmaxf(za, zb);
    const float m = (fabsf(p[2]) + fabsf(lo) + fabsf(hi) + n[2]) * (1.0f / 65536.0f) + 1.0f / 1024.0f;
    k0 = (int)fmaxf(floorf(lo - m), 0.0f);
    k1 = (int)fminf(floorf(hi + m), n[2] - 1.0f);
    if (k1 < k0) k1 = k0;   // cannot happen for a line that meets the grid
}

}  // namespace hullmi
