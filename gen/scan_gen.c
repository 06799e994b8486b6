/*
 * Seeded synthetic proton-CT scans: a cone beam from a point source crossing a
 * phantom made of nested, axis-aligned ellipsoids.
 *
 * This module only makes inputs. It holds none of the hull-detection
 * arithmetic: both the CPU oracle and the GPU library read what it writes.
 *
 * Geometry (lab frame, mm): the beam runs along +x from a source at
 * (-src_dist, 0, 0); z is the rotation axis. The paper rotates the object in
 * front of a fixed horizontal beam (Section 2.2), so object coordinates are the
 * lab coordinates rotated by -theta about z. Entry/exit points are where the
 * ray crosses the tracker planes x = -tracker_x and x = +tracker_x.
 *
 * WEPL is the exact line integral of relative stopping power along the straight
 * line through the (FP32-rounded) entry and exit points: a sum of closed-form
 * ellipsoid chords weighted by each ellipsoid's RSP increment. The paper's
 * simulated sets also assume straight lines between entry and exit points
 * (Section 2.1). Multiple Coulomb scattering is not simulated.
 *
 * Random numbers are counter based: SplitMix64's output mix (Steele, Lea and
 * Flood, OOPSLA 2014) applied to seed + (8*h + stream + 1) * golden gamma, so
 * history h gets the same draws whatever range or thread count produces it.
 * Gaussian noise uses the Box-Muller transform.
 */
#include <math.h>
#include <stdint.h>

typedef struct {
    double cx, cy, cz;   /* centre (object frame, mm) */
    double a, b, c;      /* semi-axes (mm) */
    double drho;         /* RSP added inside this ellipsoid */
} gen_ellipsoid;

typedef struct {
    int64_t n_hist;       /* histories in the whole scan */
    int32_t n_angles;     /* gantry angles, uniform over 360 degrees */
    int32_t n_ellipsoids;
    double angle0_deg;    /* first gantry angle */
    double src_dist;      /* source to isocentre (mm) */
    double tracker_x;     /* tracker planes at lab x = -tracker_x / +tracker_x */
    double fan_y, fan_z;  /* aim points uniform in |y| <= fan_y, |z| <= fan_z at x = 0 */
    double sigma;         /* additive Gaussian WEPL noise (mm) */
    double outlier_frac;  /* probability that a history is an outlier */
    double outlier_max;   /* outlier WEPL ~ U[0, outlier_max) */
    uint64_t seed;
    const gen_ellipsoid *ell;
} gen_scan_config;

static inline uint64_t gen_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Uniform double in [0, 1) for history h, stream s. */
static inline double gen_u01(uint64_t seed, int64_t h, int s)
{
    uint64_t ctr = (uint64_t)h * 8u + (uint64_t)s + 1u;
    return (double)(gen_mix64(seed + ctr * 0x9E3779B97F4A7C15ULL) >> 11) * 0x1.0p-53;
}

/* Length of the chord that the infinite line p + t*u (|u| = 1) cuts from an
 * axis-aligned ellipsoid: the distance between the two roots of the quadratic
 * obtained by substituting the line into sum((x_i - c_i)^2 / a_i^2) = 1. */
double gen_chord(const gen_ellipsoid *e, const double p[3], const double u[3])
{
    const double ax[3] = {e->a, e->b, e->c};
    const double ce[3] = {e->cx, e->cy, e->cz};
    double A = 0.0, B = 0.0, C = -1.0;
    for (int i = 0; i < 3; ++i) {
        double w = u[i] / ax[i];
        double r = (p[i] - ce[i]) / ax[i];
        A += w * w;
        B += 2.0 * w * r;
        C += r * r;
    }
    double disc = B * B - 4.0 * A * C;
    if (!(disc > 0.0)) return 0.0;
    return sqrt(disc) / A;
}

/* Exact WEPL of the straight line through two lab-frame points at gantry angle
 * theta (degrees): the object frame is the lab frame rotated by -theta. */
double gen_line_wepl(const gen_scan_config *cfg, double theta_deg,
                     const double pin[3], const double pout[3])
{
    const double th = theta_deg * (3.14159265358979323846 / 180.0);
    const double c = cos(th), s = sin(th);
    double a[3], b[3], u[3];
    a[0] = c * pin[0] + s * pin[1];
    a[1] = -s * pin[0] + c * pin[1];
    a[2] = pin[2];
    b[0] = c * pout[0] + s * pout[1];
    b[1] = -s * pout[0] + c * pout[1];
    b[2] = pout[2];
    double len = 0.0;
    for (int i = 0; i < 3; ++i) { u[i] = b[i] - a[i]; len += u[i] * u[i]; }
    len = sqrt(len);
    if (!(len > 0.0)) return 0.0;
    for (int i = 0; i < 3; ++i) u[i] /= len;
    double w = 0.0;
    for (int k = 0; k < cfg->n_ellipsoids; ++k) w += cfg->ell[k].drho * gen_chord(&cfg->ell[k], a, u);
    return w;
}

/* Fills histories [h0, h1) of the scan into arrays indexed from 0.
 * wepl_true (optional, may be NULL) receives the noise-free WEPL in FP64.
 * Returns 0, or -1 on bad arguments. */
int gen_scan(const gen_scan_config *cfg, int64_t h0, int64_t h1,
             float *x_in, float *y_in, float *z_in,
             float *x_out, float *y_out, float *z_out,
             float *angle_deg, float *wepl, double *wepl_true)
{
    if (!cfg || h0 < 0 || h1 < h0 || h1 > cfg->n_hist || cfg->n_angles < 1) return -1;
    const double D = cfg->src_dist, T = cfg->tracker_x;
    const double step = 360.0 / (double)cfg->n_angles;
    const int64_t n = h1 - h0;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        const int64_t h = h0 + j;
        const int64_t k = (int64_t)(((__int128)h * cfg->n_angles) / cfg->n_hist);
        const float theta = (float)(cfg->angle0_deg + (double)k * step);
        const double ya = cfg->fan_y * (2.0 * gen_u01(cfg->seed, h, 0) - 1.0);
        const double za = cfg->fan_z * (2.0 * gen_u01(cfg->seed, h, 1) - 1.0);
        /* ray from (-D,0,0) through (0,ya,za) evaluated at x = -T and x = +T */
        const float xi = (float)(-T), xo = (float)T;
        const float yi = (float)(ya * (D - T) / D), zi = (float)(za * (D - T) / D);
        const float yo = (float)(ya * (D + T) / D), zo = (float)(za * (D + T) / D);
        const double pin[3] = {xi, yi, zi}, pout[3] = {xo, yo, zo};
        const double wt = gen_line_wepl(cfg, (double)theta, pin, pout);
        double w = wt;
        if (cfg->sigma > 0.0) {
            const double u1 = 1.0 - gen_u01(cfg->seed, h, 2);   /* (0, 1] */
            const double u2 = gen_u01(cfg->seed, h, 3);
            w += cfg->sigma * sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2);
        }
        if (cfg->outlier_frac > 0.0 && gen_u01(cfg->seed, h, 4) < cfg->outlier_frac)
            w = cfg->outlier_max * gen_u01(cfg->seed, h, 5);
        x_in[j] = xi; y_in[j] = yi; z_in[j] = zi;
        x_out[j] = xo; y_out[j] = yo; z_out[j] = zo;
        angle_deg[j] = theta;
        wepl[j] = (float)w;
        if (wepl_true) wepl_true[j] = wt;
    }
    return 0;
}
