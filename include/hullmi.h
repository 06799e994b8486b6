/*
 * hullmi: proton-CT hull detection on AMD Instinct MI355X (gfx950).
 *
 * The method is that of Schultze, Witt, Censor, Schulte and Schubert,
 * "Performance of Hull-Detection Algorithms for Proton Computed Tomography
 * Reconstruction" (arXiv:1402.1720): every proton history is a straight line
 * through the image grid; low-WEPL lines feed silhouette/space carving (SC,
 * Section 3.2, Algorithm 1) and modified SC (MSC, Section 3.3, Algorithm 2),
 * high-WEPL lines feed space modelling (SM, Section 3.4, Algorithm 3), and a
 * cone-beam FDK reconstruction thresholded at RSP 0.6 gives the FBP hull
 * (Section 3.1).
 *
 * Conventions shared by every entry point
 *   - Frames. Lab frame in mm: the beam runs along +x, z is the rotation axis.
 *     The object turns by the gantry angle theta (degrees) in front of the
 *     fixed beam (Section 2.2), so object coordinates are the lab coordinates
 *     rotated by -theta about z. Grids live in the object frame.
 *   - Geometry, decided bit-exactly: c, s = FP32 rounding of the FP64 cosine
 *     and sine of (theta mod 360 computed exactly in FP64) * pi/180; each
 *     endpoint becomes x_o = c*x + s*y, y_o = c*y - s*x, z_o = z (FP32, one
 *     rounding per operation, no fused multiply-add), then voxel units
 *     g = (x_o - x0) * (1.0f/dx), then q = rint(g * 1024) (round half to even).
 *   - The voxel set A_i of a line (Sections 3.2 and 3.4, d0 read as 0 against
 *     half-open voxel boxes, L_i read as the infinite line): voxel v belongs to
 *     A_i when some point of the line through q_in and q_out lies in
 *     [1024 v, 1024 (v+1)) on every axis. Integer arithmetic decides it.
 *   - Classes (Section 3.2 eq. for I_L, Section 3.4 eq. for I_H): low when
 *     WEPL < wepl_low, high when WEPL > wepl_high (FP32 compares).
 *   - A history is skipped (counted in n_skipped, never an error) when its WEPL
 *     is not finite, or when it belongs to a class being counted and another
 *     field is not finite, an endpoint has |g| >= 2^16, or q_in == q_out.
 *   - Volumes are [nz][ny][nx] with x fastest: v = i + nx*(j + ny*k).
 *     Counts are int32, masks uint8 0/1.
 *
 * Memory and streams
 *   - Histories, counts, masks, images, stats and workspace are DEVICE
 *     pointers owned by the caller. Grid and parameter structs are host
 *     pointers read before the call returns. Outputs must not alias inputs.
 *   - Calls enqueue work on `stream` (a hipStream_t; NULL is the null stream)
 *     and return without waiting. They allocate no device memory: the
 *     workspace is passed in, sized by hull_workspace_bytes(). Calls on
 *     different streams with disjoint outputs and workspaces may overlap.
 *   - hull_sc, hull_msc, hull_sm and hull_all may also run part of their
 *     work on a second stream that the library creates once per device
 *     (non-blocking, default priority, kept until the process ends): when
 *     the histories need more than one internal batch of the workspace (see
 *     hull_workspace_bytes), unless `stream` is being captured into a graph.
 *     That work starts after everything enqueued on `stream` before the call
 *     and is joined back into `stream` before the call's last work on it, so
 *     the call is ordered on `stream` as if it ran there alone.
 *
 * Errors
 *   - Argument errors return HULL_EINVAL before anything is enqueued: a NULL
 *     pointer that the call needs, n < 0 or n >= 2^31, a grid axis outside
 *     [1, 2048] or with more than 2^31 - 1 voxels, a voxel size or origin that
 *     is not finite or not positive, a non-finite threshold, n_t < 1,
 *     frac_den <= 0, frac_num < 0, an unknown mode, scope or neighbourhood.
 *   - A workspace smaller than hull_workspace_bytes() returns HULL_ENOMEM
 *     (for the counting ops, smaller than their minimum; see there).
 *   - A failed launch returns HULL_EDEVICE.
 */
#ifndef HULLMI_H
#define HULLMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HULLMI_ABI_VERSION 3

typedef enum hull_status {
    HULL_OK = 0,
    HULL_EINVAL = 1,
    HULL_ENOMEM = 2,
    HULL_EDEVICE = 3,
    HULL_EBUSY = 4,
    HULL_ENOTSUP = 5,
    HULL_ETIMEDOUT = 6
} hull_status;

/* Voxel grid in the object frame (mm): (x0, y0, z0) is the lower corner of
 * voxel (0, 0, 0); voxel (i, j, k) spans [x0 + i dx, x0 + (i+1) dx) etc. */
typedef struct hullmi_grid {
    int32_t nx, ny, nz;
    float dx, dy, dz;
    float x0, y0, z0;
} hullmi_grid;

/* Proton histories as eight FP32 device arrays of length n (structure of
 * arrays): tracker entry and exit points (lab frame, mm), gantry angle
 * (degrees) and water-equivalent path length (mm). */
typedef struct hullmi_histories {
    const float *x_in, *y_in, *z_in;
    const float *x_out, *y_out, *z_out;
    const float *angle_deg;
    const float *wepl;
    int64_t n;
} hullmi_histories;

/* Optional per-call counters (device memory). n_visits_* = sum of |A_i| over
 * the counted low / high lines; n_missed_grid = counted lines with A_i empty. */
typedef struct hullmi_stats {
    int64_t n_low, n_high, n_skipped, n_missed_grid, n_visits_low, n_visits_high;
} hullmi_stats;

/* flags */
#define HULL_ACCUMULATE 1u /* add to the counts (and stats) instead of overwriting */

/* MSC rule. NEIGHBOR_DIFF is the paper's: keep v unless N(v) - N(w) >= n_t
 * for some w in B(v) (Section 3.3, equation for H2 and Algorithm 2).
 * COUNT keeps v when N(v) < n_t. */
enum hull_msc_mode { HULL_MSC_COUNT = 0, HULL_MSC_NEIGHBOR_DIFF = 1 };
/* SM threshold. MAX_SLOPE follows Algorithm 3: M_t = M at the last voxel (in
 * linear order) whose slope max_{w in B(v)} M(v) - M(w) is largest; FRACTION
 * sets M_t by frac_den * M > frac_num * max M. H3 = {M > M_t} (Section 3.4). */
enum hull_sm_mode { HULL_SM_FRACTION = 0, HULL_SM_MAX_SLOPE = 1, HULL_SM_EDGE = 2 };
/* EDGE (scope SLICE only) follows the per-slice rule of Section 3.4's text:
 * M_t is the largest M on the slice's strongest edge and H3 = {M >= M_t}. The
 * paper's edge detector (a modified Canny) is not given; this one is, exactly
 * in integers: Sobel gx, gy on the slice, G = |gx| + |gy| (0 on the slice
 * border); direction (1,0) if 5|gy| <= 2|gx|, (0,1) if 5|gx| <= 2|gy|, else
 * (1,1) when gx and gy share a sign and (1,-1) otherwise; p is an edge pixel
 * iff G(p) > 0, G(p) > G(p - d) and G(p) >= G(p + d); the seed is the edge
 * pixel of largest G (ties: largest index); the edge is the 8-connected set of
 * edge pixels q with frac_den * G(q) >= frac_num * G(seed) that holds the
 * seed; a slice without edge pixels keeps nothing. */
/* statistic of the SM threshold over the whole volume or per z-slice */
enum hull_scope { HULL_SCOPE_VOLUME = 0, HULL_SCOPE_SLICE = 1 };
/* B(v) = {w : d(v, w) <= 1} (Section 3.3) in voxel units: v and its face
 * neighbours in the slice (INPLANE4) or in 3-D (SPATIAL6) */
enum hull_nbr { HULL_NBR_INPLANE4 = 0, HULL_NBR_SPATIAL6 = 1 };

/* operations for hull_workspace_bytes */
enum hull_op {
    HULL_OP_SC = 0,
    HULL_OP_MSC = 1,
    HULL_OP_SM = 2,
    HULL_OP_ALL = 3,
    HULL_OP_FBP = 4,
    HULL_OP_COUNT_LINES = 5,
    HULL_OP_SC_BINNED = 6,
    HULL_OP_FBP_CUT = 7
};

/* All parameters of the one-pass call. The paper's values: wepl_low 1.0 mm
 * (Sections 3.2, 3.3), wepl_high 5.0 mm (Section 3.4), msc_n_t 50 with
 * NEIGHBOR_DIFF (Section 3.3). */
typedef struct hullmi_params {
    float wepl_low, wepl_high;
    int32_t msc_n_t, msc_mode;
    int32_t sm_frac_num, sm_frac_den, sm_mode, sm_scope;
    int32_t nbr;
} hullmi_params;

/* FDK geometry (Section 3.1): virtual detector on the lab plane x = 0, u along
 * lab y, v along lab z, nu x nv bins of du x dv mm starting at (u0, v0); the
 * point source sits at (-src_dist, 0, 0); n_angles gantry angle bins of
 * dangle degrees from angle0 covering the full turn; nu <= 2048 and
 * nu * nv * n_angles < 2^31. filter 0 = Shepp-Logan.
 * threshold: RSP at or above it belongs to the hull (0.6 in the paper). */
typedef struct hullmi_fbp_params {
    float src_dist_mm, du_mm, dv_mm, u0_mm, v0_mm;
    int32_t nu, nv, n_angles;
    float angle0_deg, dangle_deg;
    int32_t filter;
    float threshold;
} hullmi_fbp_params;

/* HULLMI_ABI_VERSION of the loaded library. */
int hull_abi_version(void);

/* Static description of a status code; never NULL. */
const char *hull_strerror(int status);

/* Device workspace (bytes, 256-byte aligned start expected) that `op` needs
 * for a grid and n histories (fbp may be NULL unless op is HULL_OP_FBP,
 * HULL_OP_FBP_CUT or HULL_OP_SC_BINNED, where it gives the bins).
 * Returns 0 when nothing is needed, or (size_t)-1 on invalid arguments.
 * The counting ops (SC, MSC, SM, ALL) take their histories in internal
 * batches of at most 2^26: for n <= 2^26 this is the size for one batch of
 * n, about 150 bytes per history on large scans; above 2^26, the size for two
 * halves that each hold a batch of n / k histories (k the smallest even
 * number of batches of at most 2^25), which the two-stream pass below takes
 * two at a time. They also run in any smaller
 * workspace of at least hull_workspace_bytes(op, grid, min(n, 65536)), in
 * smaller batches (the largest that fit): the same results, with more
 * launches. When the histories need more than one batch of the workspace
 * passed, the per-scan calls split its counting part in two halves and run
 * batches of equal size (whole blocks of 8192 histories) that fit a half,
 * alternately on `stream` and on the library's second stream, so that one
 * batch's classification and scatter overlap the other's walk; a workspace
 * whose half cannot hold 65536 histories keeps the batches on `stream`. */
size_t hull_workspace_bytes(int op, const hullmi_grid *grid, int64_t n,
                            const hullmi_fbp_params *fbp);

/* SC (Section 3.2, Algorithm 1): N[v] = number of low lines whose A_i holds v;
 * mask[v] = (N[v] == 0). N (required) and mask (may be NULL) are device
 * arrays of nx*ny*nz elements. stats may be NULL. */
int hull_sc(const hullmi_histories *hist, const hullmi_grid *grid, float wepl_low,
            int32_t *N, uint8_t *mask, uint32_t flags, hullmi_stats *stats,
            void *ws, size_t ws_bytes, void *stream);

/* MSC (Section 3.3, Algorithm 2): the same N, then the MSC mask by `mode`
 * (hull_msc_mode) with threshold n_t and neighbourhood `nbr` (hull_nbr). */
int hull_msc(const hullmi_histories *hist, const hullmi_grid *grid, float wepl_low,
             int32_t n_t, int mode, int nbr, int32_t *N, uint8_t *mask, uint32_t flags,
             hullmi_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* SM (Section 3.4, Algorithm 3): M[v] = number of high lines whose A_i holds
 * v; mask by `mode` (hull_sm_mode), `scope` (hull_scope) and `nbr`. FRACTION
 * uses frac_num / frac_den (for example 3 / 5 keeps M > 0.6 max M). */
int hull_sm(const hullmi_histories *hist, const hullmi_grid *grid, float wepl_high,
            int32_t frac_num, int32_t frac_den, int mode, int scope, int nbr, int32_t *M,
            uint8_t *mask, uint32_t flags, hullmi_stats *stats, void *ws, size_t ws_bytes,
            void *stream);

/* One pass over the histories for all three rules: low lines count into N,
 * high lines into M, then the SC, MSC and SM masks (each may be NULL). */
int hull_all(const hullmi_histories *hist, const hullmi_grid *grid, const hullmi_params *params,
             int32_t *N, int32_t *M, uint8_t *sc_mask, uint8_t *msc_mask, uint8_t *sm_mask,
             uint32_t flags, hullmi_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* FDK hull (Section 3.1). Every history with finite fields, |WEPL| < 2^16 mm
 * and x_out != x_in is binned by (gantry angle, u, v) where its line crosses
 * x = 0 (decided in FP32: r = (0 - x_in)/(x_out - x_in), u = y_in + r*(y_out -
 * y_in), v likewise, k = rint((theta - angle0) * (1/dangle)) mod n_angles,
 * iu = floor((u - u0) * (1/du)), iv likewise); bins average their WEPL
 * (empty bins are 0), are weighted by D / sqrt(D^2 + u^2 + v^2), filtered
 * along u with the Shepp-Logan kernel -2 / (pi^2 du^2 (4 n^2 - 1)) times du,
 * and backprojected onto voxel centres with weight (dtheta/2) / U^2, U =
 * (D + x_L)/D, sampling bilinearly (zero off the detector). image (FP32,
 * required) gets the RSP estimate, mask (may be NULL) = image >= threshold. */
int hull_fbp(const hullmi_histories *hist, const hullmi_grid *grid, const hullmi_fbp_params *fbp,
             float *image, uint8_t *mask, void *ws, size_t ws_bytes, void *stream);

/* FDK hull after the data cuts (Section 3.1 computes its FBP hull from the
 * histories that survive the cuts of Section 2.2): histories are binned as in
 * hull_fbp, each bin drops its histories more than cut_sigmas population
 * standard deviations from its mean WEPL (decided exactly on WEPL in 1/1024
 * mm, as hull_sc_binned does; 0 keeps all), and the bin means are taken over
 * the kept histories (WEPL summed in 2^-16 mm, as hull_fbp sums it); then the
 * FDK steps of hull_fbp. EINVAL also for cut_sigmas outside [0, 64].
 * Workspace: op HULL_OP_FBP_CUT. */
int hull_fbp_cut(const hullmi_histories *hist, const hullmi_grid *grid, const hullmi_fbp_params *fbp,
                 int32_t cut_sigmas, float *image, uint8_t *mask, void *ws, size_t ws_bytes,
                 void *stream);

/* Binned SC: SC as the paper ran it (Section 3.2, after Algorithm 1) with the
 * data cuts of Section 2.2, on the FDK hull's bins (`bins`, as hull_fbp takes
 * them; its threshold is not used).
 *   1. Every history with finite fields, |WEPL| < 2^16 mm and x_out != x_in
 *      that lands on the detector is binned exactly as in hull_fbp; its WEPL
 *      enters the statistics as w_q = rint(WEPL * 1024) (1/1024 mm).
 *   2. Data cut: with n, S1 = sum w_q and S2 = sum w_q^2 over the bin, a
 *      history is dropped when (n w_q - S1)^2 > k^2 (n S2 - S1^2), i.e. when
 *      it lies more than k population standard deviations from the bin mean
 *      (k = params->cut_sigmas; 0 keeps every history). Integer-exact.
 *   3. A bin whose kept histories have mean WEPL below E_L (kept sum <
 *      rint(E_L * 1024) * kept count, at least one kept) carves its line: from
 *      the source (-src_dist, 0, 0) through the bin centre (0, u0 + (iu + 0.5)
 *      du, v0 + (iv + 0.5) dv) in the lab frame at gantry angle angle0 + k
 *      dangle (FP32), moved to the object frame and rounded like a history;
 *      carved[v] = 1 for every v of its A.
 *   4. mask[v] = 1 iff den * (uncarved voxels of the W x W window around v in
 *      its slice; voxels outside the grid count as carved) > num * W^2, which
 *      keeps voxels whose window mean exceeds num/den (0.4 in the paper).
 * Outputs (device): kept_n [n_angles][nv][nu] uint32 and kept_sum (int64,
 * 1/1024 mm) per bin after the cut (each may be NULL: the workspace then holds
 * it), carved uint8[V] 0/1 (may be NULL). mask uint8[V] is required. stats (device, may be
 * NULL) is overwritten. EINVAL also for a non-finite wepl_low or |wepl_low| >=
 * 2^16, cut_sigmas outside [0, 64], an even window or one outside [1, 31],
 * thr_den <= 0 or thr_num < 0. */
typedef struct hullmi_bsc_params {
    float wepl_low;           /* E_L, mm (1.0 in the paper) */
    int32_t cut_sigmas;       /* k (3 in the paper), 0 = no data cuts */
    int32_t window;           /* W, odd (5 in the paper) */
    int32_t thr_num, thr_den; /* keep iff the window mean exceeds num/den (2/5) */
} hullmi_bsc_params;

typedef struct hullmi_bsc_stats {
    int64_t n_binned;         /* histories that landed in a bin */
    int64_t n_cut;            /* of those, dropped by the data cut */
    int64_t n_bins_used;      /* bins with at least one history */
    int64_t n_bins_carved;    /* bins taken as misses */
    int64_t n_lines_skipped;  /* of those, lines out of range or degenerate */
    int64_t n_visits;         /* sum of |A| over the carved lines */
} hullmi_bsc_stats;

int hull_sc_binned(const hullmi_histories *hist, const hullmi_grid *grid,
                   const hullmi_fbp_params *bins, const hullmi_bsc_params *params,
                   uint32_t *kept_n, int64_t *kept_sum, uint8_t *carved, uint8_t *mask,
                   hullmi_bsc_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* The accumulate step alone, for lines already in quantised object-frame form
 * (for example one line per bin): q_in and q_out are device arrays [n][3] of
 * int32 in 1/1024-voxel units; counts[v] gets the number of lines whose A_i
 * holds v (added to when flags has HULL_ACCUMULATE). Lines with q_in == q_out
 * or a coordinate of magnitude 2^26 or more are skipped. */
int hull_count_lines(const int32_t *q_in, const int32_t *q_out, int64_t n,
                     const hullmi_grid *grid, int32_t *counts, uint32_t flags,
                     hullmi_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* Kernels (or short groups of launches) as hull_count_profile and
 * hull_fbp_profile report them. */
enum hull_prof_kernel {
    HULL_PROF_CLASSIFY = 0,       /* classes, geometry, slice ranges, per-block bin counts */
    HULL_PROF_SCAN = 1,           /* per-bin offsets of every block */
    HULL_PROF_PLAN = 2,           /* bin and slice starts, equal-work ranges */
    HULL_PROF_SCATTER = 3,        /* (history, slice) items in bin order */
    HULL_PROF_SETUP = 4,          /* slice-walk state of every item */
    HULL_PROF_WALK = 5,           /* the voxel walk into LDS slice tiles */
    HULL_PROF_REDUCE = 6,         /* partial tiles summed into N and M */
    HULL_PROF_OVERFLOW = 7,       /* lines over many slices, global atomics */
    HULL_PROF_FBP_CLEAR = 8,      /* FDK: zero the bin sums and counts */
    HULL_PROF_FBP_BIN = 9,        /* FDK: bin every history on the detector */
    HULL_PROF_FBP_FILTER = 10,    /* FDK: weight and Shepp-Logan filter every row */
    HULL_PROF_FBP_GEOMETRY = 11,  /* FDK: per-angle trig and per-tile footprints */
    HULL_PROF_FBP_BACKPROJECT = 12, /* FDK: backprojection and threshold */
    HULL_PROF_KERNELS = 13
};

/* Measurement aid: the counting pass of hull_all (no masks) with a HIP event
 * pair recorded around every kernel launch on `stream`. Arguments, flags and
 * errors as hull_all (N and M required). The call waits for the stream;
 * then ms[k] (host, HULL_PROF_KERNELS entries) holds the summed duration of
 * kernel k over every internal batch and launches[k] (host, may be NULL) the
 * number of its launches. The batches are hull_all's with the same workspace,
 * run one after another on `stream`. The counts equal hull_all's.
 * HULL_EDEVICE also when an event cannot be created or read. */
int hull_count_profile(const hullmi_histories *hist, const hullmi_grid *grid,
                       const hullmi_params *params, int32_t *N, int32_t *M, uint32_t flags,
                       hullmi_stats *stats, void *ws, size_t ws_bytes, void *stream, float *ms,
                       int32_t *launches);

/* Measurement aid: hull_fbp with a HIP event pair around every kernel launch
 * (or group of launches) on `stream`; waits for the stream and fills ms and
 * launches as hull_count_profile does (entries HULL_PROF_FBP_*). Arguments
 * and errors as hull_fbp. */
int hull_fbp_profile(const hullmi_histories *hist, const hullmi_grid *grid,
                     const hullmi_fbp_params *fbp, float *image, uint8_t *mask, void *ws,
                     size_t ws_bytes, void *stream, float *ms, int32_t *launches);

/* For callers that cannot allocate device memory or pass a workspace (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): hull_fbp with its workspace in a fixed device array of the
 * library, HULLMI_NOALLOC_SCRATCH_BYTES long. Each device that runs the
 * library holds its own copy until the process ends (set up on the first
 * call on that device). The call allocates nothing; arguments, outputs and
 * results are those of hull_fbp. HULL_EINVAL also when the geometry's
 * workspace (hull_workspace_bytes(HULL_OP_FBP, ...)) exceeds the array, and
 * HULL_EDEVICE when the array's address cannot be found. Every call on one
 * device shares that device's array: calls that overlap in time on one
 * device (other streams, other host threads) race and must be serialised by
 * the caller; calls in sequence on one stream are safe (each call clears what
 * it accumulates before using it). */
#define HULLMI_NOALLOC_SCRATCH_BYTES (256u << 20)
int hull_fbp_noalloc(const hullmi_histories *hist, const hullmi_grid *grid,
                     const hullmi_fbp_params *fbp, float *image, uint8_t *mask, void *stream);

/* The geometry step alone: per history status (0 ok, 1 non-finite field,
 * 2 endpoint out of range, 3 degenerate) and the quantised endpoints [n][3]
 * (int32, 1/1024 voxel; left unwritten for status 1 and 2). */
int hull_quantize(const hullmi_histories *hist, const hullmi_grid *grid, int32_t *status,
                  int32_t *q_in, int32_t *q_out, void *stream);

/* Device bytes that one request of `op` (HULL_OP_SC, _MSC, _SM, _ALL, _FBP,
 * _FBP_CUT or _SC_BINNED) occupies when the library holds everything itself,
 * as the server does: the eight input arrays (n values each), every output of
 * the op (counts, masks, FBP image), the two counter blocks and the op's
 * workspace, each piece 256-byte aligned. fbp may be NULL unless op is one of
 * the three that bin on the detector. (size_t)-1 on invalid arguments.
 * Servers admit requests by this figure against their budget. */
size_t hull_footprint_bytes(int op, const hullmi_grid *grid, int64_t n,
                            const hullmi_fbp_params *fbp);

/* ------------------------------------------------------------------------
 * Sessions: online accumulation.
 *
 * MSC and SM need no binning, so each path can be carved as soon as it is
 * measured, during the scan, with the hull available right after it
 * (Section 5). A session keeps N and M resident on one device and adds chunks
 * of histories to them as they arrive; the masks of all three rules can be
 * read at any time and equal those of one call over every history pushed so
 * far (counts are integers, so the order and chunking of pushes do not
 * matter). Pushed chunks are appended to a device buffer of
 * max(max_chunk, 2^22) histories; a full buffer is counted while the next
 * chunks fill a second one, and a read counts what is buffered, so the
 * session's rate stays near that of one call over the whole scan however
 * small the chunks. A session owns its device memory (counts, masks, the two
 * buffers and a workspace, allocated at creation) and two streams of default
 * priority. Calls on one session serialise; sessions are independent.
 * ---------------------------------------------------------------------- */

typedef struct hullmi_session hullmi_session;

/* New session for a grid and the rules' parameters (hullmi_params, checked as
 * hull_all checks them), for chunks of at most max_chunk (1 .. 2^31 - 1)
 * histories, on HIP device `device`. EINVAL for bad arguments, ENOMEM when the
 * device memory cannot be allocated. */
int hull_session_create(const hullmi_grid *grid, const hullmi_params *params, int64_t max_chunk,
                        int device, hullmi_session **out);

/* Adds a chunk (n <= max_chunk) of histories: its eight arrays are host
 * memory (host = 1; pinned memory copies fastest) or device memory (host = 0,
 * already written). They are copied into the session's buffer, while earlier
 * chunks are counted, and the call returns once the copy is done: the caller
 * may then reuse the arrays. */
int hull_session_push(hullmi_session *s, const hullmi_histories *chunk, int host);

/* Counts what is buffered, waits for every count so far, computes the masks
 * asked for and copies the
 * asked-for outputs (each may be NULL): N, M (int32[V]), the SC, MSC and SM
 * masks (uint8[V]) and the accumulated counters. host = 1: the outputs are
 * host memory, else device memory. Returns when they are written. */
int hull_session_read(hullmi_session *s, int32_t *N, int32_t *M, uint8_t *sc_mask,
                      uint8_t *msc_mask, uint8_t *sm_mask, hullmi_stats *stats, int host);

/* Zeroes the counts and counters (a new scan). */
int hull_session_reset(hullmi_session *s);

/* Waits for pending work and frees the session. */
int hull_session_destroy(hullmi_session *s);

/* ------------------------------------------------------------------------
 * Batches: many scans, planned once and launched as one unit.
 *
 * The scans are independent (every history is its own line, Section 3), so a
 * plan spreads its jobs over several internal streams, longest first onto the
 * least loaded stream, each stream with a workspace of its own, and on the
 * first launch captures the whole fork/join into a HIP graph that later
 * launches replay. A job is one per-scan call with device pointers exactly
 * as hull_sc / hull_msc / hull_sm / hull_all / hull_fbp / hull_fbp_cut /
 * hull_sc_binned take them.
 * ---------------------------------------------------------------------- */

/* One scan of a batch. op selects the call; only the fields that call reads
 * matter: SC reads params.wepl_low and writes N (+ sc_mask); MSC reads
 * params.wepl_low / msc_n_t / msc_mode / nbr and writes N (+ msc_mask); SM
 * reads params.wepl_high / sm_* / nbr and writes M (+ sm_mask); ALL is
 * hull_all; FBP reads fbp and writes image (+ fbp_mask); FBP_CUT is
 * hull_fbp_cut with bsc.cut_sigmas and writes image (+ fbp_mask); SC_BINNED
 * is hull_sc_binned with fbp as its bins and bsc as its parameters, and
 * writes bsc_mask (required) and bsc_stats (may be NULL). stats belongs to
 * the counting ops (SC, MSC, SM, ALL) and is ignored by the others. Pointers
 * are device pointers owned by the caller and must stay valid until the plan
 * is destroyed; their contents may change between launches. HULL_ACCUMULATE
 * in flags applies to the counting ops only. */
typedef struct hullmi_job {
    int32_t op;
    uint32_t flags;
    hullmi_histories hist;
    hullmi_grid grid;
    hullmi_params params;
    hullmi_fbp_params fbp;
    int32_t *N, *M;
    uint8_t *sc_mask, *msc_mask, *sm_mask;
    float *image;
    uint8_t *fbp_mask;
    hullmi_stats *stats;
    hullmi_bsc_params bsc;
    uint8_t *bsc_mask;
    hullmi_bsc_stats *bsc_stats;
} hullmi_job;

/* Launch choices of a plan; counts and masks do not depend on any of them.
 * streams: concurrent internal streams (1..16);
 * use_graph: capture on the first launch and replay afterwards (0 / 1);
 * walk_blocks: cap on the workgroups of each persistent walk (0 = one per
 *   resident slot of the device);
 * ranges_per_group: ranges of equal estimated work dealt to each walk
 *   workgroup (0..64; 0 = 2 where two walk workgroups share a CU, 8 where one
 *   fills it; never more than 2048 / walk workgroups);
 * length_classes: line-length classes per z-slice by which the walk's items
 *   are grouped so that a wavefront walks lines of similar length (0..16;
 *   0 = 16, or fewer on grids of more than 128 slices); with two or more, the
 *   last class holds the lines that may pass through a voxel corner, which
 *   need the walk's longer loop;
 * run_stride: the item runs of one (class, slice, length) bin are ordered
 *   by classification block modulo this stride, so that neighbouring runs
 *   come from histories of different gantry angles (0..256; 0 = the internal
 *   batch's classification blocks of 8192 histories over 128, at least 1). */
typedef struct hullmi_tuning {
    int32_t streams;
    int32_t use_graph;
    int32_t walk_blocks;
    int32_t ranges_per_group;
    int32_t length_classes;
    int32_t run_stride;
} hullmi_tuning;

typedef struct hullmi_plan hullmi_plan;

/* Checks every job as its per-scan call would (HULL_EINVAL on the first bad
 * one, nothing enqueued), allocates one workspace per internal stream and
 * assigns jobs to streams. With tuning == NULL the choice comes from a
 * per-process cache keyed by the job shapes; on a miss, when no job has
 * HULL_ACCUMULATE, a few candidate tunings are timed by running the batch
 * (outputs are written), else a fixed default is used. Must be called with
 * the device of the job pointers current. */
int hull_batch_plan(const hullmi_job *jobs, int n_jobs, const hullmi_tuning *tuning,
                    hullmi_plan **plan);

/* Enqueues every job of the plan on `stream`: work starts after what is
 * already on `stream` and everything the plan does is complete before later
 * work on `stream` starts. Launches of one plan must not overlap. */
int hull_batch_launch(hullmi_plan *plan, void *stream);

/* The tuning the plan uses. */
int hull_batch_tuning(const hullmi_plan *plan, hullmi_tuning *out);

/* Waits for the plan's streams, frees its memory. NULL is ignored. */
int hull_batch_destroy(hullmi_plan *plan);

/* ------------------------------------------------------------------------
 * Serving: scans arrive one by one from the host and leave as masks on the
 * host.
 *
 * A server owns one device arena of hbm_budget bytes and max_slots worker
 * threads, each with its own stream. Requests queue in arrival order; a free
 * worker admits the request at the head of the queue as soon as its
 * footprint (hull_footprint_bytes) fits in the arena, copies its histories
 * in, runs its call, copies the outputs out and frees its space, so new
 * requests join while others are still running. Requests never share device
 * memory, so a request's result does not depend on what else is running.
 * ---------------------------------------------------------------------- */

/* One request. Histories and outputs are HOST pointers owned by the caller,
 * valid until hull_server_wait has returned for the ticket (pinned host
 * memory gives the full copy rate; pageable works). Outputs may be NULL when
 * not wanted; op and parameters as in hullmi_job. */
typedef struct hullmi_request {
    int32_t op;
    hullmi_histories hist;
    hullmi_grid grid;
    hullmi_params params;
    hullmi_fbp_params fbp;
    int32_t *N, *M;
    uint8_t *sc_mask, *msc_mask, *sm_mask;
    float *image;
    uint8_t *fbp_mask;
    hullmi_bsc_params bsc;
    uint8_t *bsc_mask;
} hullmi_request;

/* Outcome of a request. Times are steady-clock nanoseconds of the host:
 * arrival (submit), admission (space granted), done (outputs on the host).
 * device_ms runs from the first input copy to the last output copy on the
 * worker's stream; compute_ms covers the call alone. */
typedef struct hullmi_result {
    int32_t status;
    hullmi_stats stats;          /* counting ops; zero for the others */
    hullmi_bsc_stats bsc_stats;  /* HULL_OP_SC_BINNED; zero for the others */
    int64_t t_arrive_ns, t_admit_ns, t_done_ns;
    float device_ms, h2d_ms, compute_ms, d2h_ms;
} hullmi_result;

typedef struct hullmi_server_stats {
    int64_t submitted, completed, failed, queued, running;
    int64_t histories_done;
    uint64_t bytes_budget, bytes_in_use, bytes_peak;
} hullmi_server_stats;

typedef struct hullmi_server hullmi_server;

/* Creates a server on `device` with an arena of hbm_budget bytes (allocated
 * here, once) and max_slots (1..64) workers. HULL_ENOMEM when the arena cannot
 * be allocated, HULL_EDEVICE when the device cannot be used. */
int hull_server_create(size_t hbm_budget, int max_slots, int device, hullmi_server **srv);

/* Validates and queues a request; returns at once with its ticket.
 * HULL_EINVAL for bad arguments, HULL_ENOMEM when its footprint exceeds the
 * whole budget (it could never be admitted), HULL_EBUSY after destroy began. */
int hull_server_submit(hullmi_server *srv, const hullmi_request *req, uint64_t *ticket);

/* Waits up to timeout_us microseconds (negative: no limit) for a ticket.
 * HULL_OK with *result filled (result->status is the call's own status) and
 * the ticket retired; HULL_ETIMEDOUT when it is still queued or running;
 * HULL_EINVAL for an unknown or retired ticket. */
int hull_server_wait(hullmi_server *srv, uint64_t ticket, hullmi_result *result,
                     int64_t timeout_us);

int hull_server_stats(hullmi_server *srv, hullmi_server_stats *out);

/* Finishes the requests already admitted, drops the ones still queued and
 * frees everything. NULL is ignored. */
int hull_server_destroy(hullmi_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* HULLMI_H */
