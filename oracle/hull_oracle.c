/*
 * CPU oracle for proton-CT hull detection (Schultze, Witt, Censor, Schulte,
 * Schubert, "Performance of Hull-Detection Algorithms for Proton Computed
 * Tomography Reconstruction", arXiv:1402.1720).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline of the benchmark call this library. It shares no source, header,
 * table or constant with the GPU library, and the GPU library never calls it.
 *
 * What it computes, in the paper's order:
 *   1. Classification (Section 3.2, eq. for I_L; Section 3.4, eq. for I_H):
 *      low  <=> WEPL <  E_L,   high <=> WEPL > E_H   (FP32 compares).
 *   2. Straight line per history (Sections 3.2-3.4: L_i joins the entry and
 *      exit points), moved into the object frame: the object turns by theta
 *      in front of a fixed horizontal beam (Section 2.2), so object = R(-theta)
 *      * lab. FP32 arithmetic, one rounding per operation, then the endpoints
 *      are rounded to 1/1024 voxel.
 *   3. The voxel set A_i = { v : d(L_i, v) <= d0 } (Sections 3.2 and 3.4).
 *      Reading: d0 = 0 against half-open voxel boxes, L_i the infinite line;
 *      v is in A_i iff some point of the line lies in [v, v+1) on every axis
 *      (in voxel units). The membership test below decides this exactly with
 *      integer arithmetic; it is the test of Algorithms 1-3's inner loop.
 *   4. Counts N(v) = |C(v)| over low histories (Section 3.3) and M(v) over
 *      high histories (Section 3.4).
 *   5. Hull rules: SC  H1 = V minus the union of A_i (Section 3.2),
 *      MSC H2 by the neighbour-difference rule (Section 3.3) or a plain count
 *      threshold, SM H3 = {M > M_t} with M_t from Algorithm 3's maximum slope
 *      or from a fraction of max M (Section 3.4).
 *   6. FDK cone-beam FBP hull (Section 3.1): bin, cosine weight, Shepp-Logan
 *      filter, weighted backprojection, threshold RSP >= 0.6. FP64 throughout,
 *      except that the bin a history falls in is decided in FP32.
 *   7. Binned SC (Section 3.2 as the paper ran it, with Section 2.2's data
 *      cuts): per-bin WEPL cuts at k standard deviations, one carve line per
 *      bin whose kept mean WEPL is below E_L, then a W x W averaging filter
 *      and a threshold. Integer statistics in 1/1024 mm fixed point.
 *
 * Every function here is pinned by the test suite to something other than
 * itself (brute force with exact fractions, hand-derived cases, closed forms,
 * invariants); none is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_ABI 1

/* Status of one history's geometry. */
enum { OR_OK = 0, OR_SKIP_NONFINITE = 1, OR_SKIP_RANGE = 2, OR_SKIP_DEGENERATE = 3 };

/* Fixed-point fraction of the quantised endpoints: 1/1024 voxel. */
#define OR_QBITS 10
#define OR_QONE 1024
/* Endpoints further than 2^16 voxels from the grid origin are rejected. */
#define OR_GMAX 65536.0f

typedef struct {
    int32_t nx, ny, nz;
    float dx, dy, dz;
    float x0, y0, z0; /* lower corner of voxel (0,0,0), object frame, mm */
} or_grid;

typedef struct {
    const float *x_in, *y_in, *z_in, *x_out, *y_out, *z_out, *angle_deg, *wepl;
    int64_t n;
} or_hist;

typedef struct {
    int64_t n_low, n_high, n_skipped, n_missed_grid, n_visits_low, n_visits_high;
} or_stats;

typedef struct {
    float src_dist_mm, du_mm, dv_mm, u0_mm, v0_mm;
    int32_t nu, nv, n_angles;
    float angle0_deg, dangle_deg;
    int32_t filter; /* 0 = Shepp-Logan */
    float threshold;
} or_fbp_params;

int or_abi(void) { return OR_ABI; }

/* ------------------------------------------------------------------------ */
/* Step 2: object-frame endpoints, rounded to 1/1024 voxel.                  */

/* cos/sin of an angle in degrees: exact remainder modulo 360 in FP64, FP64
 * libm cos/sin, then rounded to FP32. */
static void or_trig(float angle_deg, float *c, float *s)
{
    const double th = (double)angle_deg;
    const double r = th - 360.0 * floor(th / 360.0);
    const double rad = r * 0.017453292519943295;
    *c = (float)cos(rad);
    *s = (float)sin(rad);
}

void or_trig_table(const float *angle_deg, int64_t n, float *c, float *s)
{
    for (int64_t i = 0; i < n; ++i) or_trig(angle_deg[i], &c[i], &s[i]);
}

static int or_point(float c, float s, float x, float y, float z, const or_grid *g, int32_t q[3])
{
    /* object frame = lab frame rotated by -theta about z */
    const float xo = c * x + s * y;
    const float yo = c * y - s * x;
    const float zo = z;
    /* voxel units with a once-rounded reciprocal of the voxel size */
    const float gx = (xo - g->x0) * (1.0f / g->dx);
    const float gy = (yo - g->y0) * (1.0f / g->dy);
    const float gz = (zo - g->z0) * (1.0f / g->dz);
    if (!(fabsf(gx) < OR_GMAX && fabsf(gy) < OR_GMAX && fabsf(gz) < OR_GMAX)) return OR_SKIP_RANGE;
    q[0] = (int32_t)rintf(gx * (float)OR_QONE);
    q[1] = (int32_t)rintf(gy * (float)OR_QONE);
    q[2] = (int32_t)rintf(gz * (float)OR_QONE);
    return OR_OK;
}

int or_quantize(const or_hist *h, const or_grid *g, int64_t i, int32_t qin[3], int32_t qout[3])
{
    const float f[8] = {h->x_in[i], h->y_in[i], h->z_in[i], h->x_out[i],
                        h->y_out[i], h->z_out[i], h->angle_deg[i], h->wepl[i]};
    for (int k = 0; k < 8; ++k)
        if (!isfinite(f[k])) return OR_SKIP_NONFINITE;
    float c, s;
    or_trig(f[6], &c, &s);
    int st = or_point(c, s, f[0], f[1], f[2], g, qin);
    if (st == OR_OK) st = or_point(c, s, f[3], f[4], f[5], g, qout);
    if (st != OR_OK) return st;
    if (qin[0] == qout[0] && qin[1] == qout[1] && qin[2] == qout[2]) return OR_SKIP_DEGENERATE;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Step 3: v in A_i, decided exactly.                                        */

/* The line is P(t) = P0 + t*D in units of 1/1024 voxel. On a moving axis the
 * points with 1024 v <= P(t) < 1024 (v+1) form one t-interval whose ends are
 * fractions; on a fixed axis the coordinate is in the slab or not. A family of
 * intervals on the real line meets iff every pair meets (Helly's theorem in one
 * dimension), so the test compares every lower end with every upper end. */
int or_line_meets_cell(const int64_t P0[3], const int64_t D[3], const int32_t v[3])
{
    int64_t ln[3], ld[3], un[3], ud[3];
    int lc[3], uc[3], na = 0;
    for (int a = 0; a < 3; ++a) {
        const int64_t lo = (int64_t)OR_QONE * v[a] - P0[a]; /* P(t)_a = 1024 v     at t = lo / D */
        const int64_t hi = lo + OR_QONE;                    /* P(t)_a = 1024 v + 1024 at t = hi / D */
        if (D[a] == 0) {
            if (!(lo <= 0 && 0 < hi)) return 0;
            continue;
        }
        if (D[a] > 0) { /* t in [lo/D, hi/D) */
            ln[na] = lo; ld[na] = D[a]; lc[na] = 1;
            un[na] = hi; ud[na] = D[a]; uc[na] = 0;
        } else {        /* t in (hi/D, lo/D], written with positive denominators */
            ln[na] = -hi; ld[na] = -D[a]; lc[na] = 0;
            un[na] = -lo; ud[na] = -D[a]; uc[na] = 1;
        }
        ++na;
    }
    for (int a = 0; a < na; ++a)
        for (int b = 0; b < na; ++b) {
            if (a == b) continue;
            const __int128 L = (__int128)ln[a] * ud[b];
            const __int128 U = (__int128)un[b] * ld[a];
            if (L > U) return 0;
            if (L == U && !(lc[a] && uc[b])) return 0;
        }
    return 1;
}

static int or_cmp_i32(const void *a, const void *b)
{
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Visits every voxel that can possibly be in A_i and keeps those that pass the
 * exact test. Candidates: the line is cut into the slabs of its major axis m
 * (largest |D|); inside slab i_m each other coordinate moves between its values
 * at the two slab faces, so its voxel index lies in [floor(min), floor(max)].
 * Those ends are computed in FP64 (error far below 1e-6 voxel) and widened by
 * one voxel each way, so the candidate set contains A_i. If `all` is set every
 * voxel of the grid is tested instead (Algorithm 1's loop as written).
 * Writes up to `cap` linear indices (x fastest), sorted, and returns |A_i|. */
static int64_t or_cells(const int64_t P0[3], const int64_t D[3], const or_grid *g,
                        int all, int32_t *out, int64_t cap, int32_t *counts)
{
    const int32_t n[3] = {g->nx, g->ny, g->nz};
    int64_t cnt = 0;
    int32_t v[3];
    if (all) {
        for (v[2] = 0; v[2] < n[2]; ++v[2])
            for (v[1] = 0; v[1] < n[1]; ++v[1])
                for (v[0] = 0; v[0] < n[0]; ++v[0])
                    if (or_line_meets_cell(P0, D, v)) {
                        const int32_t lin = v[0] + n[0] * (v[1] + n[1] * v[2]);
                        if (out && cnt < cap) out[cnt] = lin;
                        if (counts) {
#pragma omp atomic
                            counts[lin] += 1;
                        }
                        ++cnt;
                    }
        return cnt;
    }
    int m = 0;
    for (int a = 1; a < 3; ++a)
        if (llabs(D[a]) > llabs(D[m])) m = a;
    const int b1 = (m + 1) % 3, b2 = (m + 2) % 3;
    for (int32_t im = 0; im < n[m]; ++im) {
        const double t0 = ((double)OR_QONE * im - (double)P0[m]) / (double)D[m];
        const double t1 = ((double)OR_QONE * (im + 1) - (double)P0[m]) / (double)D[m];
        int64_t lo[3], hi[3];
        int empty = 0;
        const int bs[2] = {b1, b2};
        for (int k = 0; k < 2; ++k) {
            const int b = bs[k];
            const double c0 = ((double)P0[b] + t0 * (double)D[b]) / OR_QONE;
            const double c1 = ((double)P0[b] + t1 * (double)D[b]) / OR_QONE;
            int64_t l = (int64_t)floor(fmin(c0, c1)) - 1;
            int64_t h = (int64_t)floor(fmax(c0, c1)) + 1;
            if (l < 0) l = 0;
            if (h > n[b] - 1) h = n[b] - 1;
            if (l > h) empty = 1;
            lo[b] = l;
            hi[b] = h;
        }
        if (empty) continue;
        v[m] = im;
        for (int64_t j = lo[b1]; j <= hi[b1]; ++j)
            for (int64_t k = lo[b2]; k <= hi[b2]; ++k) {
                v[b1] = (int32_t)j;
                v[b2] = (int32_t)k;
                if (or_line_meets_cell(P0, D, v)) {
                    const int32_t lin = v[0] + n[0] * (v[1] + n[1] * v[2]);
                    if (out && cnt < cap) out[cnt] = lin;
                    if (counts) {
#pragma omp atomic
                        counts[lin] += 1;
                    }
                    ++cnt;
                }
            }
    }
    if (out) qsort(out, (size_t)(cnt < cap ? cnt : cap), sizeof(int32_t), or_cmp_i32);
    return cnt;
}

/* A_i for one quantised line: sorted linear indices, returns |A_i|. */
int64_t or_line_cells(const int32_t qin[3], const int32_t qout[3], const or_grid *g,
                      int all, int32_t *out, int64_t cap)
{
    const int64_t P0[3] = {qin[0], qin[1], qin[2]};
    const int64_t D[3] = {(int64_t)qout[0] - qin[0], (int64_t)qout[1] - qin[1],
                          (int64_t)qout[2] - qin[2]};
    if (D[0] == 0 && D[1] == 0 && D[2] == 0) return 0;
    return or_cells(P0, D, g, all, out, cap, NULL);
}

/* counts[v] += |{lines i : v in A_i}| for n quantised lines given as [n][3].
 * Lines with q_in == q_out or a coordinate of magnitude 2^26 or more are
 * skipped (the same bound that endpoints within 2^16 voxels satisfy). */
void or_count_lines(const int32_t *qin, const int32_t *qout, int64_t n, const or_grid *g,
                    int32_t *counts)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        const int64_t P0[3] = {qin[3 * i], qin[3 * i + 1], qin[3 * i + 2]};
        const int64_t P1[3] = {qout[3 * i], qout[3 * i + 1], qout[3 * i + 2]};
        int ok = 1;
        for (int a = 0; a < 3; ++a)
            ok &= llabs(P0[a]) < (1LL << 26) && llabs(P1[a]) < (1LL << 26);
        if (!ok) continue;
        const int64_t D[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
        if (D[0] == 0 && D[1] == 0 && D[2] == 0) continue;
        or_cells(P0, D, g, 0, NULL, 0, counts);
    }
}

/* Steps 1-4 over histories [0, n): N counts low histories (WEPL < e_low),
 * M counts high ones (WEPL > e_high). Either output may be NULL, which also
 * switches its class off. Counts are added to what N and M hold.
 * Skipped (and counted in n_skipped): a history whose WEPL is not finite, and
 * a history of an active class with another field not finite, an endpoint
 * with |g| >= 2^16, or endpoints that coincide after rounding. */
void or_counts(const or_hist *h, const or_grid *g, float e_low, float e_high,
               int32_t *N, int32_t *M, or_stats *st)
{
    int64_t s_low = 0, s_high = 0, s_skip = 0, s_miss = 0, s_vl = 0, s_vh = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : s_low, s_high, s_skip, s_miss, s_vl, s_vh)
    for (int64_t i = 0; i < h->n; ++i) {
        const float w = h->wepl[i];
        if (!isfinite(w)) { ++s_skip; continue; }
        const int low = N != NULL && w < e_low;
        const int high = M != NULL && w > e_high;
        if (!low && !high) continue;
        int32_t qin[3], qout[3];
        if (or_quantize(h, g, i, qin, qout) != OR_OK) { ++s_skip; continue; }
        const int64_t P0[3] = {qin[0], qin[1], qin[2]};
        const int64_t D[3] = {(int64_t)qout[0] - qin[0], (int64_t)qout[1] - qin[1],
                              (int64_t)qout[2] - qin[2]};
        const int64_t c = or_cells(P0, D, g, 0, NULL, 0, low ? N : M);
        if (low) { ++s_low; s_vl += c; }
        else { ++s_high; s_vh += c; }
        if (c == 0) ++s_miss;
    }
    if (st) {
        st->n_low = s_low; st->n_high = s_high; st->n_skipped = s_skip;
        st->n_missed_grid = s_miss; st->n_visits_low = s_vl; st->n_visits_high = s_vh;
    }
}

/* ------------------------------------------------------------------------ */
/* Step 5: hull rules.                                                       */

enum { OR_MSC_COUNT = 0, OR_MSC_NEIGHBOR_DIFF = 1 };
enum { OR_SM_FRACTION = 0, OR_SM_MAX_SLOPE = 1, OR_SM_EDGE = 2 };
enum { OR_SCOPE_VOLUME = 0, OR_SCOPE_SLICE = 1 };
enum { OR_NBR_INPLANE4 = 0, OR_NBR_SPATIAL6 = 1 };

/* B(v) = { w : d(v, w) <= 1 } (Section 3.3) read in voxel-index units: v itself
 * and its face neighbours inside the grid, in the slice (INPLANE4) or in 3-D
 * (SPATIAL6). Writes up to 7 linear indices, returns how many. */
static int or_nbrs(const or_grid *g, int nbr, int64_t v, int64_t w[7])
{
    const int64_t nx = g->nx, ny = g->ny, nz = g->nz;
    const int64_t i = v % nx, j = (v / nx) % ny, k = v / (nx * ny);
    int c = 0;
    w[c++] = v;
    if (i > 0) w[c++] = v - 1;
    if (i < nx - 1) w[c++] = v + 1;
    if (j > 0) w[c++] = v - nx;
    if (j < ny - 1) w[c++] = v + nx;
    if (nbr == OR_NBR_SPATIAL6) {
        if (k > 0) w[c++] = v - nx * ny;
        if (k < nz - 1) w[c++] = v + nx * ny;
    }
    return c;
}

/* SC, Algorithm 1: start from all ones and clear every voxel a low line
 * crosses. With N(v) the number of low lines through v that is H1 = [N == 0]. */
void or_sc(const int32_t *N, int64_t V, uint8_t *mask)
{
    for (int64_t v = 0; v < V; ++v) mask[v] = (uint8_t)(N[v] == 0);
}

/* MSC. NEIGHBOR_DIFF follows Algorithm 2's final loop: H2(v) starts at 1 and
 * becomes 0 when some w in B(v) has N(v) - N(w) >= N_t. COUNT keeps v when
 * N(v) < N_t. Returns 0, or -1 on a bad mode. */
int or_msc(const int32_t *N, const or_grid *g, int32_t n_t, int mode, int nbr, uint8_t *mask)
{
    const int64_t V = (int64_t)g->nx * g->ny * g->nz;
    if (mode == OR_MSC_COUNT) {
        for (int64_t v = 0; v < V; ++v) mask[v] = (uint8_t)(N[v] < n_t);
        return 0;
    }
    if (mode != OR_MSC_NEIGHBOR_DIFF) return -1;
    for (int64_t v = 0; v < V; ++v) {
        int64_t w[7];
        const int nw = or_nbrs(g, nbr, v, w);
        mask[v] = 1;
        for (int k = 0; k < nw; ++k)
            if ((int64_t)N[v] - (int64_t)N[w[k]] >= n_t) mask[v] = 0;
    }
    return 0;
}

/* SM. MAX_SLOPE follows Algorithm 3: scan v in linear order, w over B(v);
 * whenever M(v) - M(w) >= MaxSlope, take it as MaxSlope and remember v; then
 * M_t = M(index) and H3 = [M > M_t]. FRACTION sets H3 = [den*M > num*max M].
 * With scope SLICE each z-slice gets its own statistic (the paper thresholds
 * slice by slice, Section 3.4). mt_out (optional) receives M_t per slice (or
 * once) for MAX_SLOPE and max M for FRACTION. Returns 0 or -1. */
/* SM threshold from the strongest edge of M in one slice (Section 3.4: the
 * edge with the largest gradient of M is found in each slice and the largest
 * M on it is the slice's threshold; voxels with M >= M_t are kept). The paper
 * used an unstated modification of Canny's detector; this one is stated in
 * full and is integer-exact:
 *   gradient  Sobel: gx = [M(i+1,j-1) + 2M(i+1,j) + M(i+1,j+1)]
 *                       - [M(i-1,j-1) + 2M(i-1,j) + M(i-1,j+1)], gy likewise
 *             along j; G = |gx| + |gy| for 1 <= i <= nx-2, 1 <= j <= ny-2,
 *             G = 0 on the slice border;
 *   direction d = (1,0) if 5|gy| <= 2|gx|, (0,1) if 5|gx| <= 2|gy|, else (1,1)
 *             when gx and gy have the same sign and (1,-1) otherwise;
 *   thinning  p is an edge pixel iff G(p) > 0, G(p) > G(p - d), G(p) >= G(p + d)
 *             (G = 0 outside the slice);
 *   the edge  seed = the edge pixel of largest G (ties: largest index); the
 *             edge is the 8-connected set of edge pixels q with
 *             den G(q) >= num G(seed) that contains the seed;
 *   threshold M_t = max of M over the edge; mask = [M >= M_t]; a slice
 *             without edge pixels keeps nothing.
 * Writes the slice's mask and returns M_t (-1 when there is no edge). */
static int64_t or_sm_edge_slice(const int32_t *M, int64_t nx, int64_t ny, int32_t num, int32_t den,
                                 uint8_t *mask)
{
    const int64_t P = nx * ny;
    int64_t *G = (int64_t *)calloc((size_t)P, sizeof(int64_t));
    int8_t *dir = (int8_t *)calloc((size_t)P, 1);
    uint8_t *edge = (uint8_t *)calloc((size_t)P, 1);
    uint8_t *seen = (uint8_t *)calloc((size_t)P, 1);
    int64_t *stack = (int64_t *)malloc((size_t)P * sizeof(int64_t));
#define AT(i, j) ((int64_t)M[(j) * nx + (i)])
    for (int64_t j = 1; j + 1 < ny; ++j)
        for (int64_t i = 1; i + 1 < nx; ++i) {
            const int64_t gx = (AT(i + 1, j - 1) + 2 * AT(i + 1, j) + AT(i + 1, j + 1)) -
                               (AT(i - 1, j - 1) + 2 * AT(i - 1, j) + AT(i - 1, j + 1));
            const int64_t gy = (AT(i - 1, j + 1) + 2 * AT(i, j + 1) + AT(i + 1, j + 1)) -
                               (AT(i - 1, j - 1) + 2 * AT(i, j - 1) + AT(i + 1, j - 1));
            const int64_t ax = llabs(gx), ay = llabs(gy);
            G[j * nx + i] = ax + ay;
            dir[j * nx + i] = 5 * ay <= 2 * ax ? 0 : (5 * ax <= 2 * ay ? 1 : ((gx > 0) == (gy > 0) ? 2 : 3));
        }
#undef AT
    static const int DI[4] = {1, 0, 1, 1}, DJ[4] = {0, 1, 1, -1};
    int64_t seed = -1;
    for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
            const int64_t p = j * nx + i;
            if (G[p] <= 0) continue;
            const int d = dir[p];
            const int64_t ib = i - DI[d], jb = j - DJ[d], ia = i + DI[d], ja = j + DJ[d];
            const int64_t gb = (ib >= 0 && ib < nx && jb >= 0 && jb < ny) ? G[jb * nx + ib] : 0;
            const int64_t ga = (ia >= 0 && ia < nx && ja >= 0 && ja < ny) ? G[ja * nx + ia] : 0;
            if (G[p] > gb && G[p] >= ga) {
                edge[p] = 1;
                if (seed < 0 || G[p] >= G[seed]) seed = p;
            }
        }
    int64_t mt = -1;
    if (seed >= 0) {
        const int64_t gs = G[seed];
        int64_t top = 0;
        stack[top++] = seed;
        seen[seed] = 1;
        mt = M[seed];
        while (top > 0) {
            const int64_t p = stack[--top];
            const int64_t i = p % nx, j = p / nx;
            if (M[p] > mt) mt = M[p];
            for (int64_t b = j - 1; b <= j + 1; ++b)
                for (int64_t a = i - 1; a <= i + 1; ++a) {
                    if (a < 0 || a >= nx || b < 0 || b >= ny) continue;
                    const int64_t q = b * nx + a;
                    if (seen[q] || !edge[q] || (int64_t)den * G[q] < (int64_t)num * gs) continue;
                    seen[q] = 1;
                    stack[top++] = q;
                }
        }
    }
    for (int64_t p = 0; p < P; ++p) mask[p] = (uint8_t)(mt >= 0 && (int64_t)M[p] >= mt);
    free(G); free(dir); free(edge); free(seen); free(stack);
    return mt;
}

int or_sm(const int32_t *M, const or_grid *g, int32_t num, int32_t den, int mode, int scope,
          int nbr, uint8_t *mask, int64_t *mt_out)
{
    if (mode == OR_SM_EDGE) {
        /* per slice by definition; num / den is the edge's hysteresis fraction */
        if (scope != OR_SCOPE_SLICE || den <= 0 || num < 0) return -1;
        const int64_t plane = (int64_t)g->nx * g->ny;
        for (int64_t k = 0; k < g->nz; ++k) {
            const int64_t mt = or_sm_edge_slice(M + k * plane, g->nx, g->ny, num, den, mask + k * plane);
            if (mt_out) mt_out[k] = mt;
        }
        return 0;
    }
    const int64_t plane = (int64_t)g->nx * g->ny;
    const int64_t V = plane * g->nz;
    const int64_t nseg = scope == OR_SCOPE_SLICE ? g->nz : 1;
    const int64_t seg = scope == OR_SCOPE_SLICE ? plane : V;
    if (mode != OR_SM_FRACTION && mode != OR_SM_MAX_SLOPE) return -1;
    if (scope != OR_SCOPE_VOLUME && scope != OR_SCOPE_SLICE) return -1;
    for (int64_t sgi = 0; sgi < nseg; ++sgi) {
        const int64_t b = sgi * seg, e = b + seg;
        if (mode == OR_SM_FRACTION) {
            int64_t mmax = 0;
            for (int64_t v = b; v < e; ++v)
                if (M[v] > mmax) mmax = M[v];
            for (int64_t v = b; v < e; ++v)
                mask[v] = (uint8_t)((int64_t)den * M[v] > (int64_t)num * mmax);
            if (mt_out) mt_out[sgi] = mmax;
        } else {
            int64_t max_slope = 0, index = b;
            for (int64_t v = b; v < e; ++v) {
                int64_t w[7];
                const int nw = or_nbrs(g, nbr, v, w);
                for (int k = 0; k < nw; ++k) {
                    const int64_t d = (int64_t)M[v] - (int64_t)M[w[k]];
                    if (d >= max_slope) { max_slope = d; index = v; }
                }
            }
            const int64_t mt = M[index];
            for (int64_t v = b; v < e; ++v) mask[v] = (uint8_t)(M[v] > mt);
            if (mt_out) mt_out[sgi] = mt;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Step 6: FDK hull (Section 3.1). Virtual detector on the lab plane x = 0    */
/* (through the isocentre), u along lab y, v along lab z; source at          */
/* (-src_dist, 0, 0).                                                        */

/* Bin histories by (gantry angle, u, v) where their line crosses x = 0 and
 * average the WEPL of each bin (an empty bin is 0). The bin is decided in FP32,
 * everything else is FP64. Histories with a non-finite field, |WEPL| >= 2^16 mm
 * (far beyond any proton range) or x_out == x_in are not binned.
 * proj: [n_angles][nv][nu]. Returns the number of histories binned. */
/* The bin of history i: -1 when it is not binned, else (k nv + iv) nu + iu. */
static int64_t or_bin_of(const or_hist *h, int64_t i, const or_fbp_params *p)
{
    const float rdu = 1.0f / p->du_mm, rdv = 1.0f / p->dv_mm, rda = 1.0f / p->dangle_deg;
    const float xi = h->x_in[i], yi = h->y_in[i], zi = h->z_in[i];
    const float xo = h->x_out[i], yo = h->y_out[i], zo = h->z_out[i];
    const float a = h->angle_deg[i], w = h->wepl[i];
    if (!(isfinite(xi) && isfinite(yi) && isfinite(zi) && isfinite(xo) && isfinite(yo) &&
          isfinite(zo) && isfinite(a) && isfinite(w)))
        return -1;
    if (!(fabsf(w) < 65536.0f)) return -1;
    const float ddx = xo - xi;
    if (ddx == 0.0f) return -1;
    const float r = (0.0f - xi) / ddx;
    const float u = yi + r * (yo - yi);
    const float v = zi + r * (zo - zi);
    const float fa = (a - p->angle0_deg) * rda;
    const float fu = (u - p->u0_mm) * rdu;
    const float fv = (v - p->v0_mm) * rdv;
    if (!(fabsf(fa) < 1.0e9f)) return -1;
    if (!(fu >= 0.0f && fu < (float)p->nu && fv >= 0.0f && fv < (float)p->nv)) return -1;
    long k = lrintf(fa) % p->n_angles;
    if (k < 0) k += p->n_angles;
    const int64_t iu = (int64_t)floorf(fu), iv = (int64_t)floorf(fv);
    return ((int64_t)k * p->nv + iv) * p->nu + iu;
}

int64_t or_fbp_bin(const or_hist *h, const or_fbp_params *p, double *proj)
{
    const int64_t nb = (int64_t)p->n_angles * p->nv * p->nu;
    double *cnt = (double *)calloc((size_t)nb, sizeof(double));
    for (int64_t b = 0; b < nb; ++b) proj[b] = 0.0;
    int64_t used = 0;
    for (int64_t i = 0; i < h->n; ++i) {
        const int64_t b = or_bin_of(h, i, p);
        if (b < 0) continue;
        proj[b] += (double)h->wepl[i];
        cnt[b] += 1.0;
        ++used;
    }
    for (int64_t b = 0; b < nb; ++b) proj[b] = cnt[b] > 0.0 ? proj[b] / cnt[b] : 0.0;
    free(cnt);
    return used;
}

/* Cosine pre-weight D / sqrt(D^2 + u^2 + v^2) at bin centres, then the
 * Shepp-Logan filter along each detector row: q[i] = du * sum_j h[i-j] p[j],
 * h[n] = -2 / (pi^2 du^2 (4 n^2 - 1)), the row taken as zero outside. In place. */
void or_fbp_filter(const or_fbp_params *p, double *proj)
{
    const int64_t nu = p->nu, nv = p->nv;
    const double D = p->src_dist_mm, du = p->du_mm, dv = p->dv_mm;
    const double pi = 3.14159265358979323846;
    double *row = (double *)malloc((size_t)nu * sizeof(double));
    double *h = (double *)malloc((size_t)(2 * nu - 1) * sizeof(double));
    for (int64_t n = -(nu - 1); n <= nu - 1; ++n)
        h[n + nu - 1] = -2.0 / (pi * pi * du * du * (4.0 * (double)n * (double)n - 1.0));
    for (int64_t k = 0; k < p->n_angles; ++k)
        for (int64_t iv = 0; iv < nv; ++iv) {
            double *pr = proj + (k * nv + iv) * nu;
            const double vc = p->v0_mm + ((double)iv + 0.5) * dv;
            for (int64_t iu = 0; iu < nu; ++iu) {
                const double uc = p->u0_mm + ((double)iu + 0.5) * du;
                row[iu] = pr[iu] * D / sqrt(D * D + uc * uc + vc * vc);
            }
            for (int64_t i = 0; i < nu; ++i) {
                double acc = 0.0;
                for (int64_t j = 0; j < nu; ++j) acc += h[i - j + nu - 1] * row[j];
                pr[i] = du * acc;
            }
        }
    free(h);
    free(row);
}

/* FDK backprojection onto voxel centres: for each angle theta_k the voxel's
 * lab position is R(theta_k) times its object position; with U = (D + x_L)/D
 * the ray from the source meets the detector at (y_L/U, z/U); the filtered
 * projection is sampled there bilinearly between bin centres (zero outside)
 * and added with weight (dtheta/2) / U^2. image: [nz][ny][nx]. */
void or_fbp_backproject(const or_grid *g, const or_fbp_params *p, const double *q, double *image)
{
    const double D = p->src_dist_mm, du = p->du_mm, dv = p->dv_mm;
    const double pi = 3.14159265358979323846;
    const double half_dth = 0.5 * (double)p->dangle_deg * pi / 180.0;
    const int64_t nu = p->nu, nv = p->nv, nx = g->nx, ny = g->ny, nz = g->nz;
    double *cs = (double *)malloc((size_t)p->n_angles * 2 * sizeof(double));
    for (int64_t k = 0; k < p->n_angles; ++k) {
        const double th = ((double)p->angle0_deg + (double)k * (double)p->dangle_deg) * pi / 180.0;
        cs[2 * k] = cos(th);
        cs[2 * k + 1] = sin(th);
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t kz = 0; kz < nz; ++kz)
        for (int64_t jy = 0; jy < ny; ++jy)
            for (int64_t ix = 0; ix < nx; ++ix) {
                const double xo = (double)g->x0 + ((double)ix + 0.5) * (double)g->dx;
                const double yo = (double)g->y0 + ((double)jy + 0.5) * (double)g->dy;
                const double zo = (double)g->z0 + ((double)kz + 0.5) * (double)g->dz;
                double f = 0.0;
                for (int64_t k = 0; k < p->n_angles; ++k) {
                    const double c = cs[2 * k], s = cs[2 * k + 1];
                    const double xl = c * xo - s * yo;
                    const double yl = s * xo + c * yo;
                    const double U = (D + xl) / D;
                    const double us = yl / U, vs = zo / U;
                    const double fu = (us - p->u0_mm) / du - 0.5;
                    const double fv = (vs - p->v0_mm) / dv - 0.5;
                    const double iu0 = floor(fu), iv0 = floor(fv);
                    const double a = fu - iu0, b = fv - iv0;
                    double val = 0.0;
                    for (int dj = 0; dj < 2; ++dj)
                        for (int di = 0; di < 2; ++di) {
                            const double iu = iu0 + di, iv = iv0 + dj;
                            if (iu < 0.0 || iu >= (double)nu || iv < 0.0 || iv >= (double)nv) continue;
                            const double wgt = (di ? a : 1.0 - a) * (dj ? b : 1.0 - b);
                            val += wgt * q[(k * nv + (int64_t)iv) * nu + (int64_t)iu];
                        }
                    f += half_dth * val / (U * U);
                }
                image[(kz * ny + jy) * nx + ix] = f;
            }
    free(cs);
}

/* The whole FDK hull: bin, weight and filter, backproject, mask = [f >= thr].
 * proj (optional) receives the filtered projections. Returns histories binned. */
int64_t or_fbp(const or_hist *h, const or_grid *g, const or_fbp_params *p, double *proj,
               double *image, uint8_t *mask)
{
    const int64_t nb = (int64_t)p->n_angles * p->nv * p->nu;
    double *q = proj ? proj : (double *)malloc((size_t)nb * sizeof(double));
    const int64_t used = or_fbp_bin(h, p, q);
    or_fbp_filter(p, q);
    or_fbp_backproject(g, p, q, image);
    const int64_t V = (int64_t)g->nx * g->ny * g->nz;
    if (mask)
        for (int64_t v = 0; v < V; ++v) mask[v] = (uint8_t)(image[v] >= (double)p->threshold);
    if (!proj) free(q);
    return used;
}

/* ------------------------------------------------------------------------ */
/* Binned SC with data cuts and a blur: the form in which the paper ran SC   */
/* (Section 3.2, after Algorithm 1; the data cuts of Section 2.2).           */
/*   1. Bin histories by (gantry angle, u, v) where their line crosses x = 0, */
/*      the bins of the FDK hull (decided in FP32 by or_bin_of).              */
/*   2. Per bin: mean and standard deviation of WEPL; drop each history      */
/*      whose WEPL lies more than k standard deviations from its bin's mean  */
/*      (the record has no angles, so only WEPL is cut).                      */
/*   3. A bin whose remaining histories have mean WEPL below E_L is taken as  */
/*      a miss: the voxels of its line are carved. The bin's line runs from  */
/*      the source through the bin centre on the detector plane, and its     */
/*      voxels are A of that line (steps 2-3 above, the same rounding).      */
/*   4. A W x W in-plane averaging filter over the uncarved image (voxels    */
/*      outside the grid count as carved), then keep a voxel iff its window  */
/*      mean exceeds num/den.                                                */
/* Reading for exactness: WEPL enters the statistics in fixed point,         */
/* w_q = rint(WEPL * 1024) (1/1024 mm), as does the cutoff e_q; sums are     */
/* exact integers, sigma is the population deviation, and "more than k sigma"*/
/* is (n w_q - S1)^2 > k^2 (n S2 - S1^2) with S1 = sum w_q, S2 = sum w_q^2.  */
/* A bin is carved iff it keeps at least one history and S1' < e_q n'.       */

typedef struct {
    float wepl_low;            /* E_L, mm: a bin with kept mean WEPL below it is carved */
    int32_t cut_sigmas;        /* k; 0 turns the data cuts off */
    int32_t window;            /* W, odd */
    int32_t thr_num, thr_den;  /* keep iff window mean > num / den */
} or_bsc_params;

typedef struct {
    int64_t n_binned, n_cut, n_bins_used, n_bins_carved, n_lines_skipped, n_visits;
} or_bsc_stats;

/* The carve line of bin (k, iu, iv) as quantised object-frame endpoints:
 * source (-D, 0, 0) and bin centre (0, u_c, v_c) in the lab frame at gantry
 * angle theta_k = angle0 + k dangle, all in FP32. Returns OR_OK or a skip
 * reason (as for a history). */
int or_bsc_line(const or_fbp_params *p, const or_grid *g, int32_t k, int32_t iu, int32_t iv,
                int32_t qin[3], int32_t qout[3])
{
    const float uc = p->u0_mm + ((float)iu + 0.5f) * p->du_mm;
    const float vc = p->v0_mm + ((float)iv + 0.5f) * p->dv_mm;
    const float th = p->angle0_deg + (float)k * p->dangle_deg;
    if (!(isfinite(uc) && isfinite(vc) && isfinite(th))) return OR_SKIP_NONFINITE;
    float c, s;
    or_trig(th, &c, &s);
    int st = or_point(c, s, -p->src_dist_mm, 0.0f, 0.0f, g, qin);
    if (st == OR_OK) st = or_point(c, s, 0.0f, uc, vc, g, qout);
    if (st != OR_OK) return st;
    if (qin[0] == qout[0] && qin[1] == qout[1] && qin[2] == qout[2]) return OR_SKIP_DEGENERATE;
    return OR_OK;
}

/* Step 4: mask[v] = [den * (number of uncarved voxels of the W x W window
 * around v in its slice) > num * W^2]. */
void or_bsc_blur(const uint8_t *carved, const or_grid *g, int32_t W, int32_t num, int32_t den,
                 uint8_t *mask)
{
    const int64_t nx = g->nx, ny = g->ny, nz = g->nz, r = W / 2;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t sum = 0;
                for (int64_t b = j - r; b <= j + r; ++b)
                    for (int64_t a = i - r; a <= i + r; ++a)
                        if (a >= 0 && a < nx && b >= 0 && b < ny)
                            sum += carved[(k * ny + b) * nx + a] ? 0 : 1;
                mask[(k * ny + j) * nx + i] =
                    (uint8_t)((int64_t)den * sum > (int64_t)num * W * W);
            }
}

/* Steps 1 and 2 for histories [0, n): bin[i] (-1 when not binned) and
 * keep[i] (binned and not more than k standard deviations from its bin's
 * mean; every binned history when k = 0). Adds to *binned and *cut. */
void or_bsc_cut(const or_hist *h, const or_fbp_params *p, int32_t k, int64_t *bin, uint8_t *keep,
                int64_t *binned, int64_t *cut)
{
    const int64_t nb = (int64_t)p->n_angles * p->nv * p->nu;
    const __int128 k2 = (__int128)k * k;
    int64_t *n = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
    int64_t *s1 = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
    __int128 *s2 = (__int128 *)calloc((size_t)nb, sizeof(__int128));
    int64_t *wq = (int64_t *)malloc((size_t)(h->n > 0 ? h->n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < h->n; ++i) {
        keep[i] = 0;
        bin[i] = or_bin_of(h, i, p);
        if (bin[i] < 0) continue;
        wq[i] = llrint((double)h->wepl[i] * 1024.0);
        n[bin[i]] += 1;
        s1[bin[i]] += wq[i];
        s2[bin[i]] += (__int128)wq[i] * wq[i];
        ++*binned;
    }
    for (int64_t i = 0; i < h->n; ++i) {
        const int64_t b = bin[i];
        if (b < 0) continue;
        const __int128 dev = (__int128)n[b] * wq[i] - s1[b];
        const __int128 var = (__int128)n[b] * s2[b] - (__int128)s1[b] * s1[b];
        if (k2 > 0 && dev * dev > k2 * var) {
            ++*cut;
            continue;
        }
        keep[i] = 1;
    }
    free(n); free(s1); free(s2); free(wq);
}

/* Steps 1-4. kept_n, kept_sum (both [n_angles][nv][nu], sums in 1/1024 mm),
 * carved and mask may each be NULL. Returns 0, or 1 for a bad argument. */
int or_bsc(const or_hist *h, const or_grid *g, const or_fbp_params *p, const or_bsc_params *bp,
           uint32_t *kept_n, int64_t *kept_sum, uint8_t *carved, uint8_t *mask, or_bsc_stats *st)
{
    if (!(isfinite(bp->wepl_low) && fabsf(bp->wepl_low) < 65536.0f)) return 1;
    if (bp->cut_sigmas < 0 || bp->cut_sigmas > 64) return 1;
    if (bp->window < 1 || bp->window % 2 == 0 || bp->thr_den <= 0) return 1;
    const int64_t nb = (int64_t)p->n_angles * p->nv * p->nu;
    const int64_t V = (int64_t)g->nx * g->ny * g->nz;
    const int64_t e_q = llrint((double)bp->wepl_low * 1024.0);
    int64_t *bin = (int64_t *)malloc((size_t)(h->n > 0 ? h->n : 1) * sizeof(int64_t));
    uint8_t *keep = (uint8_t *)malloc((size_t)(h->n > 0 ? h->n : 1));
    int64_t *n = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
    int64_t *n_k = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
    int64_t *s1_k = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
    int32_t *hits = (int32_t *)calloc((size_t)V, sizeof(int32_t));
    or_bsc_stats s;
    memset(&s, 0, sizeof s);
    or_bsc_cut(h, p, bp->cut_sigmas, bin, keep, &s.n_binned, &s.n_cut);
    for (int64_t i = 0; i < h->n; ++i) {
        if (bin[i] < 0) continue;
        ++n[bin[i]];
        if (!keep[i]) continue;
        n_k[bin[i]] += 1;
        s1_k[bin[i]] += llrint((double)h->wepl[i] * 1024.0);
    }
    /* step 3: carve the lines of the bins that missed the object */
    int64_t used = 0, ncarved = 0, nskip = 0, visits = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : used, ncarved, nskip, visits)
    for (int64_t b = 0; b < nb; ++b) {
        if (n[b] > 0) ++used;
        if (!(n_k[b] > 0 && s1_k[b] < e_q * n_k[b])) continue;
        ++ncarved;
        const int32_t iu = (int32_t)(b % p->nu), iv = (int32_t)((b / p->nu) % p->nv);
        const int32_t k = (int32_t)(b / ((int64_t)p->nu * p->nv));
        int32_t qin[3], qout[3];
        if (or_bsc_line(p, g, k, iu, iv, qin, qout) != OR_OK) { ++nskip; continue; }
        const int64_t P0[3] = {qin[0], qin[1], qin[2]};
        const int64_t D[3] = {(int64_t)qout[0] - qin[0], (int64_t)qout[1] - qin[1],
                              (int64_t)qout[2] - qin[2]};
        visits += or_cells(P0, D, g, 0, NULL, 0, hits);
    }
    s.n_bins_used = used;
    s.n_bins_carved = ncarved;
    s.n_lines_skipped = nskip;
    s.n_visits = visits;
    /* step 4 */
    uint8_t *cv = carved ? carved : (uint8_t *)malloc((size_t)(V > 0 ? V : 1));
    for (int64_t v = 0; v < V; ++v) cv[v] = (uint8_t)(hits[v] > 0);
    if (mask) or_bsc_blur(cv, g, bp->window, bp->thr_num, bp->thr_den, mask);
    if (kept_n)
        for (int64_t b = 0; b < nb; ++b) kept_n[b] = (uint32_t)n_k[b];
    if (kept_sum)
        for (int64_t b = 0; b < nb; ++b) kept_sum[b] = s1_k[b];
    if (st) *st = s;
    if (!carved) free(cv);
    free(bin); free(keep); free(n); free(n_k); free(s1_k); free(hits);
    return 0;
}

/* FDK hull after the data cuts (Section 3.1: the FBP hull was computed from
 * the histories left after the cuts of Section 2.2): the bins of step 1, the
 * cut of step 2 (k standard deviations, k = 0 keeps all), then the FDK steps
 * with each bin's mean WEPL taken over its kept histories (FP64; an empty bin
 * is 0). proj (optional, [n_angles][nv][nu]) receives the kept bin means
 * before weighting and filtering. Returns histories kept, or -1 for a bad k. */
int64_t or_fbp_cut(const or_hist *h, const or_grid *g, const or_fbp_params *p, int32_t k,
                   double *proj, double *image, uint8_t *mask)
{
    if (k < 0 || k > 64) return -1;
    const int64_t nb = (int64_t)p->n_angles * p->nv * p->nu;
    int64_t *bin = (int64_t *)malloc((size_t)(h->n > 0 ? h->n : 1) * sizeof(int64_t));
    uint8_t *keep = (uint8_t *)malloc((size_t)(h->n > 0 ? h->n : 1));
    double *q = (double *)calloc((size_t)nb, sizeof(double));
    double *cnt = (double *)calloc((size_t)nb, sizeof(double));
    int64_t binned = 0, cut = 0;
    or_bsc_cut(h, p, k, bin, keep, &binned, &cut);
    for (int64_t i = 0; i < h->n; ++i) {
        if (bin[i] < 0 || !keep[i]) continue;
        q[bin[i]] += (double)h->wepl[i];
        cnt[bin[i]] += 1.0;
    }
    for (int64_t b = 0; b < nb; ++b) q[b] = cnt[b] > 0.0 ? q[b] / cnt[b] : 0.0;
    if (proj) memcpy(proj, q, (size_t)nb * sizeof(double));
    or_fbp_filter(p, q);
    or_fbp_backproject(g, p, q, image);
    const int64_t V = (int64_t)g->nx * g->ny * g->nz;
    if (mask)
        for (int64_t v = 0; v < V; ++v) mask[v] = (uint8_t)(image[v] >= (double)p->threshold);
    free(bin); free(keep); free(q); free(cnt);
    return binned - cut;
}

/* Step 2 for histories [0, n): status per history (OR_OK or a skip reason)
 * and the quantised endpoints as [n][3]. */
void or_quantize_all(const or_hist *h, const or_grid *g, int32_t *status, int32_t *qin,
                     int32_t *qout)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < h->n; ++i) status[i] = or_quantize(h, g, i, qin + 3 * i, qout + 3 * i);
}

/* ------------------------------------------------------------------------
 * Whole-call mirrors of the GPU library's per-scan calls: the same argument
 * layouts (grid, histories, stats, parameters, FDK geometry) with host
 * pointers and no stream or workspace. Counts are overwritten; masks, stats
 * and the FDK mask may be NULL. The FDK image is FP64 here. Return 0, or 1
 * when a required pointer is missing. */

typedef struct {
    float wepl_low, wepl_high;
    int32_t msc_n_t, msc_mode;
    int32_t sm_frac_num, sm_frac_den, sm_mode, sm_scope;
    int32_t nbr;
} or_params;

static void or_stats_out(or_stats *dst, const or_stats *src)
{
    if (dst) *dst = *src;
}

int oracle_hull_sc(const or_hist *h, const or_grid *g, float wepl_low, int32_t *N, uint8_t *mask,
                   or_stats *st)
{
    if (!h || !g || !N) return 1;
    const int64_t V = (int64_t)g->nx * g->ny * g->nz;
    or_stats s;
    memset(N, 0, (size_t)V * sizeof(int32_t));
    or_counts(h, g, wepl_low, 0.0f, N, NULL, &s);
    if (mask) or_sc(N, V, mask);
    or_stats_out(st, &s);
    return 0;
}

int oracle_hull_msc(const or_hist *h, const or_grid *g, float wepl_low, int32_t n_t, int mode,
                    int nbr, int32_t *N, uint8_t *mask, or_stats *st)
{
    if (!h || !g || !N) return 1;
    const int64_t V = (int64_t)g->nx * g->ny * g->nz;
    or_stats s;
    memset(N, 0, (size_t)V * sizeof(int32_t));
    or_counts(h, g, wepl_low, 0.0f, N, NULL, &s);
    if (mask && or_msc(N, g, n_t, mode, nbr, mask) != 0) return 1;
    or_stats_out(st, &s);
    return 0;
}

int oracle_hull_sm(const or_hist *h, const or_grid *g, float wepl_high, int32_t num, int32_t den,
                   int mode, int scope, int nbr, int32_t *M, uint8_t *mask, or_stats *st)
{
    if (!h || !g || !M) return 1;
    const int64_t V = (int64_t)g->nx * g->ny * g->nz;
    or_stats s;
    memset(M, 0, (size_t)V * sizeof(int32_t));
    or_counts(h, g, 0.0f, wepl_high, NULL, M, &s);
    if (mask && or_sm(M, g, num, den, mode, scope, nbr, mask, NULL) != 0) return 1;
    or_stats_out(st, &s);
    return 0;
}

int oracle_hull_all(const or_hist *h, const or_grid *g, const or_params *p, int32_t *N,
                    int32_t *M, uint8_t *sc_mask, uint8_t *msc_mask, uint8_t *sm_mask,
                    or_stats *st)
{
    if (!h || !g || !p || !N || !M) return 1;
    const int64_t V = (int64_t)g->nx * g->ny * g->nz;
    or_stats s;
    memset(N, 0, (size_t)V * sizeof(int32_t));
    memset(M, 0, (size_t)V * sizeof(int32_t));
    or_counts(h, g, p->wepl_low, p->wepl_high, N, M, &s);
    if (sc_mask) or_sc(N, V, sc_mask);
    if (msc_mask && or_msc(N, g, p->msc_n_t, p->msc_mode, p->nbr, msc_mask) != 0) return 1;
    if (sm_mask && or_sm(M, g, p->sm_frac_num, p->sm_frac_den, p->sm_mode, p->sm_scope, p->nbr,
                         sm_mask, NULL) != 0)
        return 1;
    or_stats_out(st, &s);
    return 0;
}

int oracle_hull_fbp(const or_hist *h, const or_grid *g, const or_fbp_params *p, double *image,
                    uint8_t *mask)
{
    if (!h || !g || !p || !image) return 1;
    or_fbp(h, g, p, NULL, image, mask);
    return 0;
}

int oracle_hull_sc_binned(const or_hist *h, const or_grid *g, const or_fbp_params *p,
                          const or_bsc_params *bp, uint32_t *kept_n, int64_t *kept_sum,
                          uint8_t *carved, uint8_t *mask, or_bsc_stats *st)
{
    if (!h || !g || !p || !bp || !mask) return 1;
    return or_bsc(h, g, p, bp, kept_n, kept_sum, carved, mask, st);
}
