/*
 * mxo.c -- plain, slow, scalar CPU oracle for the per-ray X-ray Monte Carlo
 * tracer.  TEST INFRASTRUCTURE ONLY: it exists so that tests, the smoke check
 * and the CPU-baseline leg of the benchmark can check the HIP library.  The
 * product path never links, loads or calls it, and it shares no code, header,
 * table or constant generator with the HIP library.
 *
 * What it computes (the paper's method, sections 2-3): independent photon
 * packets ("rays") are emitted by a source component and carried, in order,
 * through a sequential list of components (section 2: an instrument is a
 * sequential list of components; rays are generated at the source and
 * propagated through the list).  Each ray carries position, direction, energy
 * and a Monte Carlo weight (section 2.2.2, the particle struct).  Monitors
 * accumulate histograms of the weights of the rays that reach them (section
 * 2.2.2, monitor arrays).  Every random draw comes from a counter-based
 * generator keyed by (seed, ray id), so a ray's fate is a pure function of
 * its id (section 2.2.2 asks for a per-thread generator; a counter-based one
 * makes that independent of the thread layout).
 *
 * The paper prints no component equations.  Each component below is the
 * textbook definition of the physics it names, in the readings listed in the
 * design notes; the voxel phantom (section 3.3, the 3-D segmented sample)
 * uses Siddon's exact radiological path in its original merge form
 * (R. L. Siddon, Med. Phys. 12 (1985) 252): all plane crossings are listed,
 * sorted, and each consecutive pair is one voxel segment whose voxel is found
 * from its midpoint.
 *
 * Floating point: binary64, round to nearest, compiled with
 * -ffp-contract=off so every expression rounds exactly as written.
 *
 * Parity pins: see the header of oracle/__init__.py.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- types -- */

enum {
    MXO_SRC_RECT_CONE = 0,
    MXO_SRC_CONE_BEAM = 1,
    MXO_SRC_GAUSSIAN = 2,
    MXO_SLIT = 3,
    MXO_BOX = 4,
    MXO_PHANTOM = 5,
    MXO_MIRROR_ELLIPTIC = 6,
    MXO_DCM = 7,
    MXO_POWDER = 8,
    MXO_DETECTOR = 9,
    MXO_LENS_CRL = 10
};

enum { MXO_ALIVE = 0, MXO_EXITED = 1, MXO_ABSORBED = 2 };

#define MXO_SLIT_CIRCULAR 1u
#define MXO_DET_WAVELENGTH 1u

/* One component as the oracle sees it.  The parameter slots are the oracle's
 * own; oracle/__init__.py fills them from the neutral instrument dict. */
typedef struct {
    int32_t type;
    uint32_t flags;
    double pos[3];
    double rot[9]; /* row major: local = rot * (lab - pos) */
    double par[24];
    const void *data0;
    const void *data1;
    int64_t n0, n1;
    int64_t dims[4];
} mxo_comp;

typedef struct {
    double r[3], d[3], E, w;
    int32_t status, dead_at;
    int64_t bin;
} mxo_ray;

/* per-detector tally (caller-owned host arrays) */
typedef struct {
    uint64_t *count;
    double *sum_w;
    double *sum_w2;
    int64_t n_bins;
} mxo_tally;

/* ------------------------------------------------------- Philox4x32-10 -- */
/* Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
 * (SC'11): a 4x32-bit counter and a 2x32-bit key; ten rounds of two 32x32
 * multiplies (multipliers 0xD2511F53 and 0xCD9E8D57) whose high halves are
 * xored with the other counter words and the round key; the key is advanced
 * by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds. */
void mxo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t a_hi = (uint32_t)(prod_a >> 32), a_lo = (uint32_t)prod_a;
        uint32_t b_hi = (uint32_t)(prod_b >> 32), b_lo = (uint32_t)prod_b;
        uint32_t y0 = b_hi ^ x1 ^ k0;
        uint32_t y1 = b_lo;
        uint32_t y2 = a_hi ^ x3 ^ k1;
        uint32_t y3 = a_lo;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The stream of one ray: counter = (block j, ray id low, ray id high,
 * purpose << 24 | job), key = (seed low, seed high).  Block j yields
 * uniforms 2j (from words 1:0) and 2j+1 (from words 3:2). */
typedef struct {
    uint32_t key[2];
    uint32_t ctr_hi[3];
    int64_t cached_block;
    uint32_t words[4];
} mxo_stream;

static void stream_init(mxo_stream *s, uint64_t seed, uint64_t ray, uint32_t purpose, uint32_t job)
{
    s->key[0] = (uint32_t)seed;
    s->key[1] = (uint32_t)(seed >> 32);
    s->ctr_hi[0] = (uint32_t)ray;
    s->ctr_hi[1] = (uint32_t)(ray >> 32);
    s->ctr_hi[2] = (purpose << 24) | (job & 0xFFFFFFu);
    s->cached_block = -1;
}

/* 52 random bits mapped to the open interval: ((w >> 12) + 1/2) * 2^-52,
 * exact in binary64 and strictly inside (0, 1). */
static double u01_from_word(uint64_t w)
{
    return ((double)(w >> 12) + 0.5) * 0x1.0p-52;
}

static double stream_uniform(mxo_stream *s, int index)
{
    int64_t block = index / 2;
    if (block != s->cached_block) {
        uint32_t ctr[4] = {(uint32_t)block, s->ctr_hi[0], s->ctr_hi[1], s->ctr_hi[2]};
        mxo_philox4x32_10(ctr, s->key, s->words);
        s->cached_block = block;
    }
    uint64_t w;
    if ((index & 1) == 0)
        w = ((uint64_t)s->words[1] << 32) | s->words[0];
    else
        w = ((uint64_t)s->words[3] << 32) | s->words[2];
    return u01_from_word(w);
}

/* exported for the known-answer and uniformity tests */
double mxo_uniform(uint64_t seed, uint64_t ray, uint32_t purpose, uint32_t job, int index)
{
    mxo_stream s;
    stream_init(&s, seed, ray, purpose, job);
    return stream_uniform(&s, index);
}

/* ------------------------------------------------------------ frames ---- */

static void to_local(const mxo_comp *c, const double r[3], const double d[3], double q[3], double dl[3])
{
    double v[3] = {r[0] - c->pos[0], r[1] - c->pos[1], r[2] - c->pos[2]};
    for (int i = 0; i < 3; ++i) {
        const double *R = c->rot + 3 * i;
        q[i] = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
        dl[i] = R[0] * d[0] + R[1] * d[1] + R[2] * d[2];
    }
}

static void to_lab(const mxo_comp *c, const double q[3], const double dl[3], double r[3], double d[3])
{
    const double *R = c->rot;
    for (int i = 0; i < 3; ++i) {
        r[i] = R[i] * q[0] + R[3 + i] * q[1] + R[6 + i] * q[2] + c->pos[i];
        d[i] = R[i] * dl[0] + R[3 + i] * dl[1] + R[6 + i] * dl[2];
    }
}

/* Propagate to the local plane z = 0.  A ray that moves away from the plane
 * or would have to go back in time cannot reach it. */
static int to_plane_z0(double q[3], const double dl[3])
{
    if (!(dl[2] > 0.0))
        return 0;
    double t = -q[2] / dl[2];
    if (!(t >= 0.0))
        return 0;
    q[0] = q[0] + t * dl[0];
    q[1] = q[1] + t * dl[1];
    q[2] = 0.0;
    return 1;
}

static double cross_dot_norm(const double a[3])
{
    return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
}

/* ----------------------------------------------------------- sources ---- */

static const double HC_KEV_ANGSTROM = 12.398419843320026; /* CODATA 2018 */

/* Square emitter with a cone uniform in solid angle about +z.  Uniform in
 * solid angle inside half-angle alpha: 1 - cos(theta) = U (1 - cos(alpha)),
 * i.e. sin(theta/2) = sqrt(U) sin(alpha/2). */
static void src_rect_cone(const mxo_comp *c, mxo_stream *s, mxo_ray *ray)
{
    double wx = c->par[0], wy = c->par[1], alpha = c->par[2], emin = c->par[3], emax = c->par[4];
    double q[3], dl[3];
    q[0] = (stream_uniform(s, 0) - 0.5) * wx;
    q[1] = (stream_uniform(s, 1) - 0.5) * wy;
    q[2] = 0.0;
    double theta = 2.0 * asin(sqrt(stream_uniform(s, 2)) * sin(0.5 * alpha));
    double phi = (2.0 * M_PI) * stream_uniform(s, 3);
    dl[0] = sin(theta) * cos(phi);
    dl[1] = sin(theta) * sin(phi);
    dl[2] = cos(theta);
    ray->E = emin + (emax - emin) * stream_uniform(s, 4);
    ray->w = 1.0;
    to_lab(c, q, dl, ray->r, ray->d);
}

/* Number of strata per side actually used for n_total rays: the largest
 * g <= G with 16 g*g <= n_total (1 if none), so that every stratum holds at
 * least 16 rays. */
uint64_t mxo_strata_side(uint64_t G, uint64_t n_total)
{
    uint64_t g = G < 1 ? 1 : G;
    while (g > 1 && 16 * g * g > n_total)
        g -= 1;
    return g;
}

/* Gaussian line profile normalised over the real line. */
static double gauss_pdf(double E, double mean, double sigma)
{
    double z = (E - mean) / sigma;
    return exp(-0.5 * z * z) / (sigma * sqrt(2.0 * M_PI));
}

/* Tube spectrum as a photon-number density on [emin, emax]: a Kramers
 * continuum proportional to (E0 - E)/E carrying fraction fc, plus two
 * Gaussian lines carrying f1 and f2. */
double mxo_spectrum(const double *par, double E)
{
    double emin = par[1], emax = par[2], E0 = par[3];
    double fc = par[4], E1 = par[5], f1 = par[6], E2 = par[7], f2 = par[8], sig = par[9];
    double K = E0 * log(emax / emin) - (emax - emin);
    return fc * ((E0 - E) / E) / K + f1 * gauss_pdf(E, E1, sig) + f2 * gauss_pdf(E, E2, sig);
}

/* Cone-beam point source: direction uniform in solid angle inside
 * half-angle alpha, stratified over G x G equal-area cells of the unit
 * square mapped to the disk by the concentric map (Shirley and Chiu 1997),
 * energy uniform on [emin, emax] with the spectrum carried in the weight:
 * w0 = (emax - emin) S(E) * (n_total / G^2) / n_cell. */
static void src_cone_beam(const mxo_comp *c, mxo_stream *s, mxo_ray *ray, uint64_t ray_id, uint64_t n_total)
{
    double alpha = c->par[0], emin = c->par[1], emax = c->par[2];
    uint64_t G = mxo_strata_side((uint64_t)c->dims[0], n_total);
    uint64_t G2 = G * G;
    uint64_t cell = (ray_id * G2) / n_total;
    uint64_t first = (cell * n_total + G2 - 1) / G2;
    uint64_t next = ((cell + 1) * n_total + G2 - 1) / G2;
    uint64_t n_cell = next - first;
    double cell_factor = ((double)n_total / (double)G2) / (double)n_cell;
    double u = ((double)(cell % G) + stream_uniform(s, 0)) / (double)G;
    double v = ((double)(cell / G) + stream_uniform(s, 1)) / (double)G;

    /* concentric square -> disk map */
    double a = 2.0 * u - 1.0, b = 2.0 * v - 1.0;
    double rad, ang;
    if (a == 0.0 && b == 0.0) {
        rad = 0.0;
        ang = 0.0;
    } else if (fabs(a) > fabs(b)) {
        rad = a;
        ang = (M_PI / 4.0) * (b / a);
    } else {
        rad = b;
        ang = (M_PI / 2.0) - (M_PI / 4.0) * (a / b);
    }
    double px = rad * cos(ang), py = rad * sin(ang);
    double rho = fabs(rad);

    double theta = 2.0 * asin(rho * sin(0.5 * alpha));
    double psi = atan2(py, px);
    double q[3] = {0.0, 0.0, 0.0}, dl[3];
    dl[0] = sin(theta) * cos(psi);
    dl[1] = sin(theta) * sin(psi);
    dl[2] = cos(theta);
    ray->E = emin + (emax - emin) * stream_uniform(s, 2);
    ray->w = ((emax - emin) * mxo_spectrum(c->par, ray->E)) * cell_factor;
    to_lab(c, q, dl, ray->r, ray->d);
}

/* ------------------------------------------------ learned proposal ---- */
/* Inverse of the standard normal distribution function: Wichura's
 * algorithm AS 241 (PPND16, Applied Statistics 37 (1988) 477), rational
 * approximations on a central region and two tail regions, accurate to about
 * 1e-16. */
double mxo_ppnd16(double p)
{
    double q = p - 0.5, r;
    if (fabs(q) <= 0.425) {
        r = 0.180625 - q * q;
        return q * (((((((2.5090809287301226727e+3 * r + 3.3430575583588128105e+4) * r +
                          6.7265770927008700853e+4) * r + 4.5921953931549871457e+4) * r +
                        1.3731693765509461125e+4) * r + 1.9715909503065514427e+3) * r +
                      1.3314166789178437745e+2) * r + 3.3871328727963666080e+0) /
               (((((((5.2264952788528545610e+3 * r + 2.8729085735721942674e+4) * r +
                     3.9307895800092710610e+4) * r + 2.1213794301586595867e+4) * r +
                   5.3941960214247511077e+3) * r + 6.8718700749205790830e+2) * r +
                 4.2313330701600911252e+1) * r + 1.0);
    }
    r = q < 0.0 ? p : 1.0 - p;
    r = sqrt(-log(r));
    double x;
    if (r <= 5.0) {
        r -= 1.6;
        x = (((((((7.74545014278341407640e-4 * r + 2.27238449892691845833e-2) * r +
                  2.41780725177450611770e-1) * r + 1.27045825245236838258e+0) * r +
                3.64784832476320460504e+0) * r + 5.76949722146069140550e+0) * r +
              4.63033784615654529590e+0) * r + 1.42343711074968357734e+0) /
            (((((((1.05075007164441684324e-9 * r + 5.47593808499534494600e-4) * r +
                  1.51986665636164571966e-2) * r + 1.48103976427480074590e-1) * r +
                6.89767334985100004550e-1) * r + 1.67638483018380384940e+0) * r +
              2.05319162663775882187e+0) * r + 1.0);
    } else {
        r -= 5.0;
        x = (((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r +
                  1.24266094738807843860e-3) * r + 2.65321895265761230930e-2) * r +
                2.96560571828504891230e-1) * r + 1.78482653991729133580e+0) * r +
              5.46378491116411436990e+0) * r + 6.65790464350110377720e+0) /
            (((((((2.04426310338993978564e-15 * r + 1.42151175831644588870e-7) * r +
                  1.84631831751005468180e-5) * r + 7.86869131145613259100e-4) * r +
                1.48753612908506148525e-2) * r + 1.36929880922735805310e-1) * r +
              5.99832206555887937690e-1) * r + 1.0);
    }
    return q < 0.0 ? -x : x;
}

/* Standard normal distribution function and its upper tail. */
static double norm_cdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }
static double norm_sf(double z) { return 0.5 * erfc(z / sqrt(2.0)); }

/* A standard normal truncated to [za, zb], by inversion of the distribution
 * function at the point that leaves mass U of the interval below it.  The
 * target is written as a lower-tail probability Pa + U (Pb - Pa) when that
 * is at most 1/2, else as the upper-tail probability Qb + (1 - U)(Qa - Qb)
 * (P lower tails, Q upper tails of za and zb), so no probability near 1 is
 * inverted and neither form cancels in the tail it serves. */
double mxo_truncnorm(double za, double zb, double U)
{
    double Pa = norm_cdf(za), Pb = norm_cdf(zb);
    double pl = Pa + U * (Pb - Pa);
    if (pl <= 0.5)
        return mxo_ppnd16(pl);
    double Qa = norm_sf(za), Qb = norm_sf(zb);
    return -mxo_ppnd16(Qb + (1.0 - U) * (Qa - Qb));
}

/* Density of the proposal mixture q = alpha q_plain + (1 - alpha) q_gmm at
 * y = (u, v, E), u = dx/dz, v = dy/dz, and the physical density p of the
 * plain source at y.  The plain source is uniform in solid angle inside the
 * cone (solid angle Omega; in (u, v) its density is
 * (1 + u^2 + v^2)^(-3/2) / Omega) and uniform in energy; the physical
 * source has the spectrum S(E) instead.  q_gmm is the 8-component diagonal
 * Gaussian mixture truncated to the box [-t, t]^2 x [emin, emax], t = tan
 * alpha: sum_k pi_k prod_d phi(z_kd)/sigma_kd divided by sum_k pi_k Z_k, Z_k
 * the box mass of component k.  gmm holds per component (pi, mu_u, mu_v,
 * mu_E, sigma_u, sigma_v, sigma_E). */
double mxo_proposal_density(const double *par, const double *gmm, double alpha_def, double u, double v, double E,
                            double *p_phys)
{
    double alpha = par[0], emin = par[1], emax = par[2];
    double t = tan(alpha);
    double lo[3] = {-t, -t, emin}, hi[3] = {t, t, emax}, y[3] = {u, v, E};
    double omega = 2.0 * M_PI * (1.0 - cos(alpha));
    double J = pow(1.0 + u * u + v * v, -1.5);
    int in_cone = u * u + v * v <= t * t && E >= emin && E <= emax;
    double q_plain = in_cone ? J / omega / (emax - emin) : 0.0;
    *p_phys = in_cone ? mxo_spectrum(par, E) * J / omega : 0.0;
    double num = 0.0, norm = 0.0;
    for (int k = 0; k < 8; ++k) {
        const double *g = gmm + 7 * k;
        double dens = g[0], Z = g[0];
        for (int d = 0; d < 3; ++d) {
            double mu = g[1 + d], sg = g[4 + d];
            double z = (y[d] - mu) / sg;
            dens *= exp(-0.5 * z * z) / (sg * sqrt(2.0 * M_PI));
            Z *= norm_cdf((hi[d] - mu) / sg) - norm_cdf((lo[d] - mu) / sg);
        }
        num += dens;
        norm += Z;
    }
    int in_box = u >= lo[0] && u <= hi[0] && v >= lo[1] && v <= hi[1] && E >= emin && E <= emax;
    double q_gmm = in_box ? num / norm : 0.0;
    return alpha_def * q_plain + (1.0 - alpha_def) * q_gmm;
}

/* Branch boundaries of an n_total-ray proposal run: rays [0, B[0]) take
 * the plain source, rays [B[k], B[k+1]) component k; B[0] = round(alpha
 * n_total), B[k+1] - B[0] = round((n_total - B[0]) cum_k / total) with cum_k
 * the running sum of the box masses pi_j Z_j, B[8] = n_total. */
void mxo_proposal_bounds(const double *par, const double *gmm, double alpha_def, uint64_t n_total, uint64_t *B)
{
    double alpha = par[0], emin = par[1], emax = par[2];
    double t = tan(alpha);
    double lo[3] = {-t, -t, emin}, hi[3] = {t, t, emax};
    double mass[8], total = 0.0;
    for (int k = 0; k < 8; ++k) {
        const double *g = gmm + 7 * k;
        double Z = g[0];
        for (int d = 0; d < 3; ++d)
            Z *= norm_cdf((hi[d] - g[1 + d]) / g[4 + d]) - norm_cdf((lo[d] - g[1 + d]) / g[4 + d]);
        mass[k] = Z;
        total += Z;
    }
    uint64_t n_plain = (uint64_t)floor(alpha_def * (double)n_total + 0.5);
    if (n_plain > n_total)
        n_plain = n_total;
    B[0] = n_plain;
    double cum = 0.0;
    for (int k = 0; k < 8; ++k) {
        cum += mass[k];
        uint64_t b = total > 0.0 ? n_plain + (uint64_t)floor((double)(n_total - n_plain) * (cum / total) + 0.5) : n_total;
        B[k + 1] = b > n_total ? n_total : b;
    }
    B[8] = n_total;
}

/* Importance weight p(y) / q(y) of a proposal draw at y = (u, v, E) in an
 * n_total-ray run, q the realised mixture density sum_b (n_b / n_total)
 * q_b(y) (q_b the plain density or component b's truncated density); 0
 * outside the cone. */
double mxo_proposal_weight(const double *par, const double *gmm, double alpha_def, uint64_t n_total, double u,
                           double v, double E)
{
    double alpha = par[0], emin = par[1], emax = par[2];
    double t = tan(alpha);
    double lo[3] = {-t, -t, emin}, hi[3] = {t, t, emax}, y[3] = {u, v, E};
    uint64_t B[9];
    mxo_proposal_bounds(par, gmm, alpha_def, n_total, B);
    double omega = 2.0 * M_PI * (1.0 - cos(alpha));
    double J = pow(1.0 + u * u + v * v, -1.5);
    int in_cone = u * u + v * v <= t * t && E >= emin && E <= emax;
    int in_box = u >= lo[0] && u <= hi[0] && v >= lo[1] && v <= hi[1] && E >= emin && E <= emax;
    double q = in_cone ? ((double)B[0] / (double)n_total) * (J / omega / (emax - emin)) : 0.0;
    for (int k = 0; k < 8; ++k) {
        uint64_t nk = B[k + 1] - B[k];
        if (nk == 0 || !in_box)
            continue;
        const double *g = gmm + 7 * k;
        double dens = 1.0, Fk = 1.0;
        for (int d = 0; d < 3; ++d) {
            double mu = g[1 + d], sg = g[4 + d];
            double z = (y[d] - mu) / sg;
            dens *= exp(-0.5 * z * z) / (sg * sqrt(2.0 * M_PI));
            Fk *= norm_cdf((hi[d] - mu) / sg) - norm_cdf((lo[d] - mu) / sg);
        }
        q += ((double)nk / (double)n_total) * (dens / Fk);
    }
    double p_phys = in_cone ? mxo_spectrum(par, E) * J / omega : 0.0;
    return p_phys > 0.0 ? p_phys / q : 0.0;
}

/* Cone-beam point source drawing from the proposal as a stratified
 * deterministic mixture.  The n_total rays are split into contiguous id
 * ranges, one per branch (plain source, then components 0..7, sizes from
 * mxo_proposal_bounds); within its branch a ray's first two uniforms are
 * stratified over G x G cells of the unit square exactly like the plain
 * stratified source (cell of local index i among n: floor(i G^2 / n), cell
 * factor (n / G^2) / n_cell), so neighbouring ids leave in neighbouring
 * directions.  The plain branch maps the stratified pair to the cone with the
 * concentric map; a component inverts a truncated normal per coordinate (u
 * from the first, v from the second, E from the third uniform).  The weight
 * is the physical density over the realised mixture density,
 * p(y) / (sum_b (n_b / n_total) q_b(y)), times the cell factor: the balance
 * heuristic of multiple importance sampling, unbiased for any split.  A draw
 * outside the cone has weight 0 and is absorbed at the source. */
static int src_cone_proposal(const mxo_comp *c, mxo_stream *s, mxo_ray *ray, uint64_t ray_id, uint64_t n_total,
                             const double *gmm, double alpha_def)
{
    double alpha = c->par[0], emin = c->par[1], emax = c->par[2];
    double t = tan(alpha);
    double lo[3] = {-t, -t, emin}, hi[3] = {t, t, emax};
    uint64_t B[9];
    mxo_proposal_bounds(c->par, gmm, alpha_def, n_total, B);
    int branch = -1; /* -1 plain, else the component */
    uint64_t start = 0, count = B[0];
    if (ray_id >= B[0]) {
        for (int k = 0; k < 8; ++k) {
            if (ray_id >= B[k] && ray_id < B[k + 1]) {
                branch = k;
                start = B[k];
                count = B[k + 1] - B[k];
                break;
            }
        }
    }
    uint64_t G = mxo_strata_side((uint64_t)c->dims[0], count);
    uint64_t G2 = G * G, i = ray_id - start;
    uint64_t cell = (i * G2) / count;
    uint64_t first = (cell * count + G2 - 1) / G2;
    uint64_t next = ((cell + 1) * count + G2 - 1) / G2;
    double cell_factor = ((double)count / (double)G2) / (double)(next - first);
    double su = ((double)(cell % G) + stream_uniform(s, 0)) / (double)G;
    double sv = ((double)(cell / G) + stream_uniform(s, 1)) / (double)G;
    double y[3];
    if (branch < 0) {
        double a = 2.0 * su - 1.0, b = 2.0 * sv - 1.0;
        double rad, ang;
        if (a == 0.0 && b == 0.0) {
            rad = 0.0;
            ang = 0.0;
        } else if (fabs(a) > fabs(b)) {
            rad = a;
            ang = (M_PI / 4.0) * (b / a);
        } else {
            rad = b;
            ang = (M_PI / 2.0) - (M_PI / 4.0) * (a / b);
        }
        double theta = 2.0 * asin(fabs(rad) * sin(0.5 * alpha));
        double psi = atan2(rad * sin(ang), rad * cos(ang));
        double dz = cos(theta);
        y[0] = sin(theta) * cos(psi) / dz;
        y[1] = sin(theta) * sin(psi) / dz;
        y[2] = emin + (emax - emin) * stream_uniform(s, 2);
    } else {
        const double *g = gmm + 7 * branch;
        double U[3] = {su, sv, stream_uniform(s, 2)};
        for (int d = 0; d < 3; ++d) {
            double mu = g[1 + d], sg = g[4 + d];
            y[d] = mu + sg * mxo_truncnorm((lo[d] - mu) / sg, (hi[d] - mu) / sg, U[d]);
        }
    }
    double wgt = mxo_proposal_weight(c->par, gmm, alpha_def, n_total, y[0], y[1], y[2]);
    double n = sqrt(1.0 + y[0] * y[0] + y[1] * y[1]);
    double qz[3] = {0.0, 0.0, 0.0}, dl[3] = {y[0] / n, y[1] / n, 1.0 / n};
    ray->E = y[2];
    ray->w = wgt > 0.0 ? wgt * cell_factor : 0.0;
    to_lab(c, qz, dl, ray->r, ray->d);
    return wgt > 0.0;
}

/* Gaussian (undulator-like) source: position and angle normal in both
 * planes (Box-Muller on consecutive uniform pairs), energy flat within a
 * relative half-width. */
static void src_gaussian(const mxo_comp *c, mxo_stream *s, mxo_ray *ray)
{
    double sx = c->par[0], sy = c->par[1], sxp = c->par[2], syp = c->par[3];
    double E0 = c->par[4], hw = c->par[5];
    double r1 = sqrt(-2.0 * log(stream_uniform(s, 0)));
    double a1 = (2.0 * M_PI) * stream_uniform(s, 1);
    double r2 = sqrt(-2.0 * log(stream_uniform(s, 2)));
    double a2 = (2.0 * M_PI) * stream_uniform(s, 3);
    double q[3], dl[3];
    q[0] = sx * (r1 * cos(a1));
    q[1] = sy * (r1 * sin(a1));
    q[2] = 0.0;
    double tx = tan(sxp * (r2 * cos(a2)));
    double ty = tan(syp * (r2 * sin(a2)));
    double nrm = sqrt(tx * tx + ty * ty + 1.0);
    dl[0] = tx / nrm;
    dl[1] = ty / nrm;
    dl[2] = 1.0 / nrm;
    ray->E = E0 * ((1.0 - hw) + 2.0 * hw * stream_uniform(s, 4));
    ray->w = 1.0;
    to_lab(c, q, dl, ray->r, ray->d);
}

/* -------------------------------------------------- absorbers and optics -- */

/* Slab method chord through the box |x| < hx, |y| < hy, |z| < hz for the
 * ray q + a dl, a >= 0. */
static double box_chord(const double h[3], const double q[3], const double dl[3])
{
    double a_in = 0.0, a_out = INFINITY;
    for (int i = 0; i < 3; ++i) {
        if (dl[i] == 0.0) {
            if (!(q[i] > -h[i] && q[i] < h[i]))
                return 0.0;
        } else {
            double inv = 1.0 / dl[i];
            double a0 = (-h[i] - q[i]) * inv, a1 = (h[i] - q[i]) * inv;
            double lo = a0 < a1 ? a0 : a1, hi = a0 < a1 ? a1 : a0;
            if (lo > a_in) a_in = lo;
            if (hi < a_out) a_out = hi;
        }
    }
    return a_out > a_in ? a_out - a_in : 0.0;
}

/* Homogeneous box, Beer-Lambert: w *= exp(-mu(E) L), mu = a E^-3 + b in
 * 1/cm, L in mm. */
static void comp_box(const mxo_comp *c, mxo_ray *ray)
{
    double q[3], dl[3];
    to_local(c, ray->r, ray->d, q, dl);
    double L = box_chord(c->par, q, dl);
    double E = ray->E;
    double mu = c->par[3] / (E * E * E) + c->par[4];
    ray->w = ray->w * exp(-(mu * L) / 10.0);
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Siddon's exact radiological path, merge form.  Volume of nx*ny*nz voxels
 * of edge v (mm), centred on the local origin, voxel (i,j,k) at byte
 * i + nx*(j + ny*k) holding a material id; mu table [material][energy bin]
 * in 1/cm on a uniform energy grid.  Returns tau = sum mu * length / 10.
 * When seg is non-null the segments (voxel index, length) are written out,
 * in traversal order, up to max_seg of them. */
typedef struct {
    const uint8_t *vol;
    const double *mu;
    int64_t n[3];
    double v;
    double corner[3];
    int64_t n_mat, n_ebin;
    double t_emin, t_emax;
} mxo_volume;

static void volume_from(const mxo_comp *c, mxo_volume *V)
{
    V->vol = (const uint8_t *)c->data0;
    V->mu = (const double *)c->data1;
    for (int i = 0; i < 3; ++i)
        V->n[i] = c->dims[i];
    V->v = c->par[0];
    for (int i = 0; i < 3; ++i)
        V->corner[i] = -0.5 * ((double)V->n[i] * V->v);
    V->t_emin = c->par[1];
    V->t_emax = c->par[2];
    V->n_mat = c->dims[3];
    /* a scattering phantom's table holds three channels (total, Rayleigh,
     * Compton), each n_mat x n_ebin */
    int64_t channels = (c->flags & 2u) ? 3 : 1;
    V->n_ebin = c->n1 / ((c->dims[3] > 0 ? c->dims[3] : 1) * channels);
}

static int64_t floor_index(double x, int64_t n)
{
    double f = floor(x);
    if (f < 0.0)
        return 0;
    if (f > (double)(n - 1))
        return n - 1;
    return (int64_t)f;
}

double mxo_siddon(const mxo_volume *V, const double q[3], const double dl[3], double E,
                  int64_t *seg_voxel, double *seg_len, int64_t max_seg, int64_t *n_seg)
{
    if (n_seg)
        *n_seg = 0;
    double inv[3];
    double a_in = 0.0, a_out = INFINITY;
    for (int i = 0; i < 3; ++i) {
        double lo_plane = V->corner[i];
        double hi_plane = V->corner[i] + (double)V->n[i] * V->v;
        if (dl[i] == 0.0) {
            inv[i] = 0.0;
            if (!(q[i] > lo_plane && q[i] < hi_plane))
                return 0.0;
        } else {
            inv[i] = 1.0 / dl[i];
            double a0 = (lo_plane - q[i]) * inv[i], a1 = (hi_plane - q[i]) * inv[i];
            double lo = a0 < a1 ? a0 : a1, hi = a0 < a1 ? a1 : a0;
            if (lo > a_in) a_in = lo;
            if (hi < a_out) a_out = hi;
        }
    }
    if (!(a_out > a_in))
        return 0.0;

    /* every plane crossing strictly inside (a_in, a_out), plus the ends */
    int64_t cap = V->n[0] + V->n[1] + V->n[2] + 5;
    double *alpha = (double *)malloc((size_t)cap * sizeof(double));
    int64_t m = 0;
    alpha[m++] = a_in;
    for (int i = 0; i < 3; ++i) {
        if (dl[i] == 0.0)
            continue;
        for (int64_t p = 0; p <= V->n[i]; ++p) {
            double plane = V->corner[i] + (double)p * V->v;
            double a = (plane - q[i]) * inv[i];
            if (a > a_in && a < a_out)
                alpha[m++] = a;
        }
    }
    alpha[m++] = a_out;
    qsort(alpha, (size_t)m, sizeof(double), cmp_double);

    double ebin_scale = (double)V->n_ebin / (V->t_emax - V->t_emin);
    int64_t e = floor_index((E - V->t_emin) * ebin_scale, V->n_ebin);
    double tau = 0.0;
    int64_t ns = 0;
    for (int64_t k = 0; k + 1 < m; ++k) {
        double len = alpha[k + 1] - alpha[k];
        if (!(len > 0.0))
            continue;
        double mid = 0.5 * (alpha[k] + alpha[k + 1]);
        int64_t idx[3];
        for (int i = 0; i < 3; ++i)
            idx[i] = floor_index((q[i] + mid * dl[i] - V->corner[i]) / V->v, V->n[i]);
        int64_t voxel = idx[0] + V->n[0] * (idx[1] + V->n[1] * idx[2]);
        int64_t mat = V->vol[voxel];
        if (mat >= V->n_mat)
            mat = V->n_mat - 1;
        tau = tau + V->mu[mat * V->n_ebin + e] * len / 10.0;
        if (seg_voxel && ns < max_seg) {
            seg_voxel[ns] = voxel;
            seg_len[ns] = len;
        }
        ns++;
    }
    free(alpha);
    if (n_seg)
        *n_seg = ns;
    return tau;
}

/* exported debug entry: segments of one ray through a volume given in
 * local coordinates */
double mxo_siddon_debug(const mxo_comp *c, const double q[3], const double dl[3], double E,
                        int64_t *seg_voxel, double *seg_len, int64_t max_seg, int64_t *n_seg)
{
    mxo_volume V;
    volume_from(c, &V);
    return mxo_siddon(&V, q, dl, E, seg_voxel, seg_len, max_seg, n_seg);
}

/* The paper's own model of the voxel sample (section 3.3, Phantom_sample3D):
 * the ray advances in fixed increments h (one third of a voxel by default);
 * after each increment the voxel holding the new position gives the material
 * and the weight is attenuated over the increment.  Readings: the chord is
 * the same as Siddon's (entry a_in, exit a_out along the unit direction);
 * step j (j = 1, 2, ...) ends at alpha_j = a_in + j h and covers
 * [alpha_(j-1), min(alpha_j, a_out)], so the last step is clipped at the
 * exit; its position is taken unclipped, in voxel units,
 * u_j = u_in + j (h d / v) with u_in = (entry point - corner) / v (evaluated
 * as one correctly rounded fused multiply-add per axis), and the voxel index
 * is floor(u_j) clamped into the volume (so the clipped last step reads the
 * voxel at the exit).  tau = sum mu(voxel of step j) * length
 * of step j / 10.  *n_steps receives the number of steps. */
double mxo_step_tau(const mxo_volume *V, const double q[3], const double dl[3], double E, double h,
                    int64_t *n_steps)
{
    if (n_steps)
        *n_steps = 0;
    double a_in = 0.0, a_out = INFINITY;
    for (int i = 0; i < 3; ++i) {
        double lo_plane = V->corner[i];
        double hi_plane = V->corner[i] + (double)V->n[i] * V->v;
        if (dl[i] == 0.0) {
            if (!(q[i] > lo_plane && q[i] < hi_plane))
                return 0.0;
        } else {
            double inv = 1.0 / dl[i];
            double a0 = (lo_plane - q[i]) * inv, a1 = (hi_plane - q[i]) * inv;
            double lo = a0 < a1 ? a0 : a1, hi = a0 < a1 ? a1 : a0;
            if (lo > a_in) a_in = lo;
            if (hi < a_out) a_out = hi;
        }
    }
    if (!(a_out > a_in))
        return 0.0;
    double u_in[3], du[3];
    for (int i = 0; i < 3; ++i) {
        u_in[i] = ((q[i] + a_in * dl[i]) - V->corner[i]) / V->v;
        du[i] = (h * dl[i]) / V->v;
    }
    double ebin_scale = (double)V->n_ebin / (V->t_emax - V->t_emin);
    int64_t e = floor_index((E - V->t_emin) * ebin_scale, V->n_ebin);
    double tau = 0.0, a_prev = a_in;
    int64_t j = 0;
    for (;;) {
        j++;
        double a_j = a_in + (double)j * h;
        double end = a_j < a_out ? a_j : a_out;
        int64_t idx[3];
        for (int i = 0; i < 3; ++i)
            idx[i] = floor_index(fma((double)j, du[i], u_in[i]), V->n[i]);
        int64_t mat = V->vol[idx[0] + V->n[0] * (idx[1] + V->n[1] * idx[2])];
        if (mat >= V->n_mat)
            mat = V->n_mat - 1;
        tau = tau + V->mu[mat * V->n_ebin + e] * (end - a_prev) / 10.0;
        a_prev = end;
        if (!(a_j < a_out))
            break;
    }
    if (n_steps)
        *n_steps = j;
    return tau;
}

double mxo_step_debug(const mxo_comp *c, const double q[3], const double dl[3], double E, int64_t *n_steps)
{
    mxo_volume V;
    volume_from(c, &V);
    return mxo_step_tau(&V, q, dl, E, c->par[3], n_steps);
}

/* ------------------------------------------------ scattering phantom ---- */
/* Scattering in the voxel sample (section 3.3: the sample models absorption
 * and scattering; scattering prolongs the paths).  Estimator: the image is
 * split by scatter order.  A run of order K traces, for every source ray,
 * the contribution of photons that interact exactly K times in the volume,
 * each interaction forced:
 *   - along the current direction the chord's optical depth tau_tot (total
 *     attenuation, channel 0) is computed; the interaction depth is drawn
 *     from the truncated exponential, tau* = -log(1 - u1 (1 - e^-tau_tot)),
 *     and located on the segment list (the point where the running optical
 *     depth reaches tau*); the weight takes the factor 1 - e^-tau_tot;
 *   - at that point the scatter albedo (mu_R + mu_C) / mu_tot of the voxel's
 *     material multiplies the weight; Rayleigh is chosen with probability
 *     mu_R / (mu_R + mu_C) (u2), Compton otherwise;
 *   - the new direction is drawn uniformly on the sphere (cos theta = 2 u3 - 1,
 *     phi = 2 pi u4 about the old direction, in the frame e1 = (d x a) / |d x a|,
 *     e2 = d x e1, a = y unless |d_y| >= 1/2, then x) and the weight takes
 *     4 pi times the normalised angular density: Rayleigh as Thomson
 *     scattering, 3 (1 + cos^2) / 4 (no form factor); Compton as
 *     Klein-Nishina for free electrons, rho^2 (rho + 1/rho - sin^2) / f(k)
 *     with k = E / m_e c^2, rho = E' / E = 1 / (1 + k (1 - cos theta)) and
 *     2 pi f(k) r_e^2 the Klein-Nishina total cross section; Compton scattering
 *     lowers the energy to E' = rho E;
 * and after the K-th interaction the ray leaves the volume along its new
 * direction attenuated by e^-tau_exit at its new energy.
 * Aimed last scatter (flags bit 2, a next-event form for a monitor of
 * known extent): the K-th direction points instead at a point drawn
 * uniformly on a target rectangle (centre par[5..7], half-axes par[8..10]
 * and par[11..13], lab frame; the point is centre + (2 u3 - 1) a +
 * (2 u4 - 1) b), whose density per steradian is dist^2 / (|n . d'| area),
 * and the weight takes the ratio of the scattering density per steradian
 * (Thomson 3 (1 + cos^2) / 16 pi, Klein-Nishina rho^2 (rho + 1/rho -
 * sin^2) / 4 pi f(k)) to it; photons scattered off the target are not
 * followed, so the estimator serves tallies on the target.  The ray reported
 * by the component sits at the last interaction point.  Order 0 is the
 * plain (uncollided) run; the orders add up to the image.  A ray that meets
 * no material (tau_tot = 0) or no scattering material (mu_R + mu_C = 0)
 * carries no weight in this estimator and is absorbed here.
 * Draws: four per order (u1 .. u4). */
static const double ME_C2_KEV = 510.99895;

/* Klein-Nishina total cross section over 2 pi r_e^2 */
static double kn_f(double k)
{
    double l = log1p(2.0 * k);
    return ((1.0 + k) / (k * k)) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k) + l / (2.0 * k) -
           (1.0 + 3.0 * k) / ((1.0 + 2.0 * k) * (1.0 + 2.0 * k));
}

/* segments of the chord in traversal order: start and end alpha and the
 * voxel of each (zero-length segments dropped), from the sorted list of all
 * plane crossings as in mxo_siddon */
static int64_t chord_segments(const mxo_volume *V, const double q[3], const double dl[3], double *a0, double *a1,
                              int64_t *vox, int64_t cap)
{
    double inv[3];
    double a_in = 0.0, a_out = INFINITY;
    for (int i = 0; i < 3; ++i) {
        double lo_plane = V->corner[i];
        double hi_plane = V->corner[i] + (double)V->n[i] * V->v;
        if (dl[i] == 0.0) {
            inv[i] = 0.0;
            if (!(q[i] > lo_plane && q[i] < hi_plane))
                return 0;
        } else {
            inv[i] = 1.0 / dl[i];
            double b0 = (lo_plane - q[i]) * inv[i], b1 = (hi_plane - q[i]) * inv[i];
            double lo = b0 < b1 ? b0 : b1, hi = b0 < b1 ? b1 : b0;
            if (lo > a_in) a_in = lo;
            if (hi < a_out) a_out = hi;
        }
    }
    if (!(a_out > a_in))
        return 0;
    int64_t m = 0;
    double *alpha = (double *)malloc((size_t)(V->n[0] + V->n[1] + V->n[2] + 5) * sizeof(double));
    alpha[m++] = a_in;
    for (int i = 0; i < 3; ++i) {
        if (dl[i] == 0.0)
            continue;
        for (int64_t p = 0; p <= V->n[i]; ++p) {
            double a = ((V->corner[i] + (double)p * V->v) - q[i]) * inv[i];
            if (a > a_in && a < a_out)
                alpha[m++] = a;
        }
    }
    alpha[m++] = a_out;
    qsort(alpha, (size_t)m, sizeof(double), cmp_double);
    int64_t ns = 0;
    for (int64_t k = 0; k + 1 < m && ns < cap; ++k) {
        if (!(alpha[k + 1] - alpha[k] > 0.0))
            continue;
        double mid = 0.5 * (alpha[k] + alpha[k + 1]);
        int64_t idx[3];
        for (int i = 0; i < 3; ++i)
            idx[i] = floor_index((q[i] + mid * dl[i] - V->corner[i]) / V->v, V->n[i]);
        a0[ns] = alpha[k];
        a1[ns] = alpha[k + 1];
        vox[ns] = idx[0] + V->n[0] * (idx[1] + V->n[1] * idx[2]);
        ns++;
    }
    free(alpha);
    return ns;
}

/* one forced interaction along dl from q: returns 0 if the chord holds no
 * attenuating material, else moves q to the interaction point and gives the
 * weight factor 1 - e^-tau_tot and the material there */
static int forced_interaction(const mxo_volume *V, double q[3], const double dl[3], int64_t e, double u1,
                              double *p_int, int64_t *mat_out)
{
    int64_t cap = V->n[0] + V->n[1] + V->n[2] + 5;
    double *a0 = (double *)malloc((size_t)cap * sizeof(double));
    double *a1 = (double *)malloc((size_t)cap * sizeof(double));
    int64_t *vox = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    int64_t ns = chord_segments(V, q, dl, a0, a1, vox, cap);
    double tau_tot = 0.0;
    for (int64_t j = 0; j < ns; ++j)
        tau_tot = tau_tot + V->mu[V->vol[vox[j]] * V->n_ebin + e] * (a1[j] - a0[j]) / 10.0;
    int ok = 0;
    if (tau_tot > 0.0) {
        double p = -expm1(-tau_tot);
        double tau_star = -log1p(-u1 * p);
        double tc = 0.0, s = 0.0;
        int64_t m = -1;
        for (int64_t j = 0; j < ns; ++j) {
            int64_t mj = V->vol[vox[j]];
            double mu = V->mu[mj * V->n_ebin + e] / 10.0;
            if (!(mu > 0.0))
                continue;
            double d = mu * (a1[j] - a0[j]);
            m = mj;
            s = a1[j];
            if (tc + d >= tau_star) {
                s = a0[j] + (tau_star - tc) / mu;
                break;
            }
            tc = tc + d;
        }
        for (int i = 0; i < 3; ++i)
            q[i] = q[i] + s * dl[i];
        *p_int = p;
        *mat_out = m;
        ok = 1;
    }
    free(a0);
    free(a1);
    free(vox);
    return ok;
}

static int comp_phantom_scatter(const mxo_comp *c, mxo_stream *st, int draw0, mxo_ray *ray)
{
    double q[3], dl[3];
    to_local(c, ray->r, ray->d, q, dl);
    mxo_volume V;
    volume_from(c, &V);
    const int64_t K = (int64_t)c->par[4];
    const int64_t plane = V.n_mat * V.n_ebin;
    double E = ray->E, w = ray->w;
    double ebin_scale = (double)V.n_ebin / (V.t_emax - V.t_emin);
    for (int64_t k = 0; k < K; ++k) {
        int64_t e = floor_index((E - V.t_emin) * ebin_scale, V.n_ebin);
        double p_int;
        int64_t m;
        if (!forced_interaction(&V, q, dl, e, stream_uniform(st, draw0 + 4 * (int)k), &p_int, &m))
            return 0;
        double mu_t = V.mu[m * V.n_ebin + e];
        double mu_r = V.mu[plane + m * V.n_ebin + e];
        double mu_c = V.mu[2 * plane + m * V.n_ebin + e];
        if (!(mu_r + mu_c > 0.0))
            return 0;
        double albedo = (mu_r + mu_c) / mu_t;
        int rayleigh = stream_uniform(st, draw0 + 4 * (int)k + 1) < mu_r / (mu_r + mu_c);
        double ct = 2.0 * stream_uniform(st, draw0 + 4 * (int)k + 2) - 1.0;
        double phi = 2.0 * M_PI * stream_uniform(st, draw0 + 4 * (int)k + 3);
        double nd[3], dens_ratio = 4.0 * M_PI; /* isotropic: 1 / density = 4 pi */
        if ((c->flags & 4u) && k == K - 1) {
            /* aimed: a point on the target rectangle, in the local frame */
            double tl[3], ta[3], tb[3], tw[3];
            for (int i = 0; i < 3; ++i)
                tw[i] = c->par[5 + i] - c->pos[i];
            for (int i = 0; i < 3; ++i) {
                tl[i] = c->rot[3 * i] * tw[0] + c->rot[3 * i + 1] * tw[1] + c->rot[3 * i + 2] * tw[2];
                ta[i] = c->rot[3 * i] * c->par[8] + c->rot[3 * i + 1] * c->par[9] + c->rot[3 * i + 2] * c->par[10];
                tb[i] = c->rot[3 * i] * c->par[11] + c->rot[3 * i + 1] * c->par[12] + c->rot[3 * i + 2] * c->par[13];
            }
            double sa = 2.0 * stream_uniform(st, draw0 + 4 * (int)k + 2) - 1.0;
            double sb = 2.0 * stream_uniform(st, draw0 + 4 * (int)k + 3) - 1.0;
            double r[3];
            for (int i = 0; i < 3; ++i)
                r[i] = (tl[i] + sa * ta[i] + sb * tb[i]) - q[i];
            double dist2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            double dist = sqrt(dist2);
            double nrm[3] = {ta[1] * tb[2] - ta[2] * tb[1], ta[2] * tb[0] - ta[0] * tb[2], ta[0] * tb[1] - ta[1] * tb[0]};
            double area4 = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]); /* |a x b| */
            if (!(dist > 0.0) || !(area4 > 0.0))
                return 0;
            for (int i = 0; i < 3; ++i)
                nd[i] = r[i] / dist;
            double cosn = fabs(nd[0] * nrm[0] + nd[1] * nrm[1] + nd[2] * nrm[2]) / area4;
            if (!(cosn > 0.0))
                return 0;
            /* density of the aimed direction: dist^2 / (cos_n * 4 |a x b|) */
            dens_ratio = (cosn * 4.0 * area4) / dist2;
            ct = dl[0] * nd[0] + dl[1] * nd[1] + dl[2] * nd[2];
        } else {
            double a[3] = {0.0, 1.0, 0.0};
            if (!(fabs(dl[1]) < 0.5)) {
                a[0] = 1.0;
                a[1] = 0.0;
            }
            double e1[3] = {dl[1] * a[2] - dl[2] * a[1], dl[2] * a[0] - dl[0] * a[2], dl[0] * a[1] - dl[1] * a[0]};
            double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
            for (int i = 0; i < 3; ++i)
                e1[i] = e1[i] / n1;
            double e2[3] = {dl[1] * e1[2] - dl[2] * e1[1], dl[2] * e1[0] - dl[0] * e1[2],
                            dl[0] * e1[1] - dl[1] * e1[0]};
            double sn = sqrt(1.0 - ct * ct), cp = cos(phi), sp = sin(phi);
            for (int i = 0; i < 3; ++i)
                nd[i] = ct * dl[i] + sn * (cp * e1[i] + sp * e2[i]);
        }
        /* scattering density per steradian at cos theta = ct */
        double st2 = 1.0 - ct * ct, dens;
        if (rayleigh) {
            dens = 3.0 * (1.0 + ct * ct) / (16.0 * M_PI);
        } else {
            double kk = E / ME_C2_KEV;
            double rho = 1.0 / (1.0 + kk * (1.0 - ct));
            dens = rho * rho * (rho + 1.0 / rho - st2) / (4.0 * M_PI * kn_f(kk));
            E = rho * E;
        }
        w = w * (p_int * albedo * (dens * dens_ratio));
        for (int i = 0; i < 3; ++i)
            dl[i] = nd[i];
    }
    /* leave the volume along the last direction at the last energy */
    double tau = mxo_siddon(&V, q, dl, E, NULL, NULL, 0, NULL);
    ray->E = E;
    ray->w = w * exp(-tau);
    to_lab(c, q, dl, ray->r, ray->d);
    return 1;
}

/* exported debug entry: the Klein-Nishina f(k) */
double mxo_kn_f(double k) { return kn_f(k); }

/* flags bit 0: the fixed-step model with step length par[3] (mm) instead of
 * Siddon's exact path */
static void comp_phantom(const mxo_comp *c, mxo_ray *ray)
{
    double q[3], dl[3];
    to_local(c, ray->r, ray->d, q, dl);
    mxo_volume V;
    volume_from(c, &V);
    double tau = (c->flags & 1u) ? mxo_step_tau(&V, q, dl, ray->E, c->par[3], NULL)
                                 : mxo_siddon(&V, q, dl, ray->E, NULL, NULL, 0, NULL);
    ray->w = ray->w * exp(-tau);
}

/* Compound refractive lens: a stack of N identical bi-concave parabolic
 * lenses (section 3.2, the focusing instrument: sixteen double-sided
 * parabolic beryllium lenses of 200 um apex radius).  Local frame: z along
 * the stack axis, origin at the stack centre; lens k (k = 0 .. N-1) is
 * centred at c_k = (k - (N-1)/2) p.  Its material lies between the front
 * surface z = c_k - w/2 - rho^2 / 2R and the back surface
 * z = c_k + w/2 + rho^2 / 2R (rho^2 = x^2 + y^2; on-axis thickness w, the
 * thickness at rho is w + rho^2 / R), inside the aperture radius r_a; the
 * frame beyond r_a is opaque.  Refractive index n = 1 - delta with
 * delta(E) = delta_ref (E_ref / E)^2; attenuation mu(E) = a / E^3 + b (1/cm).
 *
 * At every surface the ray meets the paraboloid at the root of the
 * intersection quadratic nearest to -C/B (the stable form C / q'), is
 * absorbed if it cannot reach it moving forward or meets it outside the
 * aperture, and is refracted by the vector form of Snell's law,
 * d' = eta d + (sqrt(k) - eta cos_i) m (m the unit normal pointing into the
 * second medium, cos_i = d . m, eta = n_1 / n_2, k = 1 - eta^2 (1 - cos_i^2);
 * k < 0, total reflection, absorbs).  sqrt(k) - eta cos_i is evaluated as
 * (1 - eta^2) / (sqrt(k) + eta cos_i), the same number without cancellation,
 * with 1 - eta^2 written out for each side: -delta (2 - delta) / (1 - delta)^2
 * entering the lens, delta (2 - delta) leaving it.  The weight is multiplied
 * once by exp(-mu L / 10), L the summed path length inside the material (mm). */
static int lens_surface(double q[3], double dl[3], double z0, double s, double R, double ra2, double eta,
                        double one_m_eta2, double *t_out)
{
    double A = -s * (dl[0] * dl[0] + dl[1] * dl[1]) / (2.0 * R);
    double B = dl[2] - s * (q[0] * dl[0] + q[1] * dl[1]) / R;
    double C = (q[2] - z0) - s * (q[0] * q[0] + q[1] * q[1]) / (2.0 * R);
    double disc = B * B - 4.0 * A * C;
    if (!(disc >= 0.0))
        return 0;
    double qq = -0.5 * (B + copysign(sqrt(disc), B));
    if (qq == 0.0)
        return 0;
    double t = C / qq;
    if (!(t >= 0.0))
        return 0;
    for (int i = 0; i < 3; ++i)
        q[i] = q[i] + t * dl[i];
    if (q[0] * q[0] + q[1] * q[1] > ra2)
        return 0;
    /* gradient of z - z0 - s rho^2 / 2R: (-s x / R, -s y / R, 1), downstream */
    double g[3] = {-s * q[0] / R, -s * q[1] / R, 1.0};
    double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    double m[3] = {g[0] / gn, g[1] / gn, g[2] / gn};
    double cos_i = dl[0] * m[0] + dl[1] * m[1] + dl[2] * m[2];
    if (!(cos_i > 0.0))
        return 0;
    double k = 1.0 - eta * eta * (1.0 - cos_i * cos_i);
    if (!(k >= 0.0))
        return 0;
    double gcoef = one_m_eta2 / (sqrt(k) + eta * cos_i);
    for (int i = 0; i < 3; ++i)
        dl[i] = eta * dl[i] + gcoef * m[i];
    *t_out = t;
    return 1;
}

static int comp_lens(const mxo_comp *c, mxo_ray *ray)
{
    double q[3], dl[3];
    to_local(c, ray->r, ray->d, q, dl);
    const double R = c->par[0], w = c->par[2], pitch = c->par[3], ra2 = c->par[4] * c->par[4];
    const int64_t N = (int64_t)c->par[1];
    const double E = ray->E;
    const double delta = c->par[5] * ((c->par[6] / E) * (c->par[6] / E));
    const double mu = c->par[7] / (E * E * E) + c->par[8];
    const double eta_in = 1.0 / (1.0 - delta), eta_out = 1.0 - delta;
    const double ome_in = -delta * (2.0 - delta) / ((1.0 - delta) * (1.0 - delta));
    const double ome_out = delta * (2.0 - delta);
    double L = 0.0, t;
    for (int64_t k = 0; k < N; ++k) {
        double ck = ((double)k - 0.5 * (double)(N - 1)) * pitch;
        if (!lens_surface(q, dl, ck - 0.5 * w, -1.0, R, ra2, eta_in, ome_in, &t))
            return 0;
        if (!lens_surface(q, dl, ck + 0.5 * w, 1.0, R, ra2, eta_out, ome_out, &t))
            return 0;
        L = L + t;
    }
    ray->w = ray->w * exp(-(mu * L) / 10.0);
    to_lab(c, q, dl, ray->r, ray->d);
    return 1;
}

/* exported debug entry: one ray given in the lens frame (the component's
 * pos and rot are ignored); returns 0 if absorbed, else the ray after the
 * stack in q, dl and the weight factor in *w */
int mxo_lens_debug(const mxo_comp *c, const double q[3], const double dl[3], double E, double q_out[3],
                   double dl_out[3], double *w)
{
    mxo_comp cc = *c;
    memset(cc.pos, 0, sizeof cc.pos);
    memset(cc.rot, 0, sizeof cc.rot);
    cc.rot[0] = cc.rot[4] = cc.rot[8] = 1.0;
    mxo_ray ray;
    memcpy(ray.r, q, sizeof ray.r);
    memcpy(ray.d, dl, sizeof ray.d);
    ray.E = E;
    ray.w = 1.0;
    int ok = comp_lens(&cc, &ray);
    memcpy(q_out, ray.r, sizeof ray.r);
    memcpy(dl_out, ray.d, sizeof ray.d);
    *w = ray.w;
    return ok;
}

/* Rectangular (or circular) aperture in the local plane z = 0; edges pass. */
static int comp_slit(const mxo_comp *c, mxo_ray *ray)
{
    double q[3], dl[3];
    to_local(c, ray->r, ray->d, q, dl);
    if (!to_plane_z0(q, dl))
        return 0;
    if (c->flags & MXO_SLIT_CIRCULAR) {
        double rr = c->par[2];
        if (!(q[0] * q[0] + q[1] * q[1] <= rr * rr))
            return 0;
    } else {
        if (!(fabs(q[0]) <= 0.5 * c->par[0] && fabs(q[1]) <= 0.5 * c->par[1]))
            return 0;
    }
    to_lab(c, q, dl, ray->r, ray->d);
    return 1;
}

/* Elliptic-cylinder mirror (meridional focusing).  Local frame: origin at
 * the mirror pole P, z along the incoming central ray, y towards the
 * reflected side.  Foci F1 = (0, 0, -p) and F2 = q (0, sin 2t0, cos 2t0);
 * semi-axes a = (p + q)/2 and b^2 = p q sin^2 t0; half focal distance
 * c = |F2 - F1|/2.  Reflectivity from a table on n nodes over [0, tmax]
 * by linear interpolation, zero beyond. */
static int comp_mirror(const mxo_comp *c, mxo_ray *ray)
{
    double p = c->par[0], qd = c->par[1], t0 = c->par[2];
    double len = c->par[3], wid = c->par[4], tmax = c->par[5];
    const double *table = (const double *)c->data0;
    int64_t nt = c->n0;

    double a = 0.5 * (p + qd);
    double b2 = p * qd * (sin(t0) * sin(t0));
    double F2y = qd * sin(2.0 * t0), F2z = qd * cos(2.0 * t0);
    double fy = F2y, fz = F2z + p;
    double two_c = sqrt(fy * fy + fz * fz);
    double uy = fy / two_c, uz = fz / two_c; /* major axis (y,z) */
    double vy = uz, vz = -uy;                /* minor axis (y,z) */
    double Cy = 0.5 * F2y, Cz = 0.5 * (F2z - p);

    double q[3], dl[3];
    to_local(c, ray->r, ray->d, q, dl);
    double gy = q[1] - Cy, gz = q[2] - Cz;
    double s0 = gy * uy + gz * uz, n0 = gy * vy + gz * vz;
    double ds = dl[1] * uy + dl[2] * uz, dn = dl[1] * vy + dl[2] * vz;
    double ia2 = 1.0 / (a * a), ib2 = 1.0 / b2;
    double A = ds * ds * ia2 + dn * dn * ib2;
    double B = 2.0 * (s0 * ds * ia2 + n0 * dn * ib2);
    double C = s0 * s0 * ia2 + n0 * n0 * ib2 - 1.0;
    double disc = B * B - 4.0 * A * C;
    if (!(disc >= 0.0))
        return 0;
    double t = (-B + sqrt(disc)) / (2.0 * A);
    if (!(t > 0.0))
        return 0;
    double X[3] = {q[0] + t * dl[0], q[1] + t * dl[1], q[2] + t * dl[2]};
    double along = X[1] * sin(t0) + X[2] * cos(t0);
    if (!(fabs(X[0]) <= 0.5 * wid && fabs(along) <= 0.5 * len))
        return 0;
    double hy = X[1] - Cy, hz = X[2] - Cz;
    double hs = (hy * uy + hz * uz) * ia2, hn = (hy * vy + hz * vz) * ib2;
    double N[3] = {0.0, hs * uy + hn * vy, hs * uz + hn * vz};
    double nn = cross_dot_norm(N);
    N[1] = N[1] / nn;
    N[2] = N[2] / nn;
    double dd = dl[0] * N[0] + dl[1] * N[1] + dl[2] * N[2];
    if (dd > 0.0) {
        N[1] = -N[1];
        N[2] = -N[2];
        dd = -dd;
    }
    double theta = asin(-dd);
    double R = 0.0;
    double h = tmax / (double)(nt - 1);
    double uu = theta / h;
    if (uu <= (double)(nt - 1)) {
        int64_t k = (int64_t)floor(uu);
        if (k > nt - 2)
            k = nt - 2;
        double f = uu - (double)k;
        R = table[k] * (1.0 - f) + table[k + 1] * f;
    }
    double out[3];
    for (int i = 0; i < 3; ++i)
        out[i] = dl[i] - 2.0 * dd * N[i];
    ray->w = ray->w * R;
    to_lab(c, X, out, ray->r, ray->d);
    return 1;
}

/* Darwin reflectivity of a thick perfect crystal without absorption, as a
 * function of x = offset / (half plateau width): 1 on the plateau, and
 * (|x| - sqrt(x^2 - 1))^2 = 1 / (|x| + sqrt(x^2 - 1))^2 outside. */
static double darwin(double x)
{
    double ax = fabs(x);
    if (ax <= 1.0)
        return 1.0;
    double den = ax + sqrt(ax * ax - 1.0);
    return 1.0 / (den * den);
}

/* Bragg reflection off the crystal plane through point P with unit normal
 * N (facing the incoming ray). */
static int bragg_bounce(double q[3], double dl[3], const double P[3], const double N[3],
                        double dspace, double width, double E, double *R)
{
    double dn = dl[0] * N[0] + dl[1] * N[1] + dl[2] * N[2];
    if (!(dn < 0.0))
        return 0;
    double rel[3] = {q[0] - P[0], q[1] - P[1], q[2] - P[2]};
    double t = -(rel[0] * N[0] + rel[1] * N[1] + rel[2] * N[2]) / dn;
    if (!(t >= 0.0))
        return 0;
    for (int i = 0; i < 3; ++i)
        q[i] = q[i] + t * dl[i];
    double theta_in = asin(-dn);
    double theta_b = asin(HC_KEV_ANGSTROM / (2.0 * dspace * E));
    double x = (theta_in - theta_b) / (0.5 * width);
    *R = darwin(x);
    for (int i = 0; i < 3; ++i)
        dl[i] = dl[i] - 2.0 * dn * N[i];
    return 1;
}

/* Two-bounce monochromator of parallel crystals.  Local frame: origin at
 * the first crystal's pole, z along the incoming beam axis, y up.  Crystal
 * 1 normal n1 = (0, cos tc, -sin tc) at the setting angle tc; crystal 2 is
 * the parallel plane through g n1 facing -n1. */
static int comp_dcm(const mxo_comp *c, mxo_ray *ray)
{
    double dsp = c->par[0], tc = c->par[1], wd = c->par[2], g = c->par[3];
    double n1[3] = {0.0, cos(tc), -sin(tc)};
    double n2[3] = {-n1[0], -n1[1], -n1[2]};
    double P1[3] = {0.0, 0.0, 0.0};
    double P2[3] = {g * n1[0], g * n1[1], g * n1[2]};
    double q[3], dl[3], R1, R2;
    to_local(c, ray->r, ray->d, q, dl);
    if (!bragg_bounce(q, dl, P1, n1, dsp, wd, ray->E, &R1))
        return 0;
    if (!bragg_bounce(q, dl, P2, n2, dsp, wd, ray->E, &R2))
        return 0;
    ray->w = ray->w * R1;
    ray->w = ray->w * R2;
    to_lab(c, q, dl, ray->r, ray->d);
    return 1;
}

/* Thin powder plate in the local plane z = 0: one of the tabulated
 * d-spacings is picked uniformly, the ray is turned by the Bragg angle 2
 * theta = 2 asin(lambda / 2d) onto the Debye-Scherrer cone at a uniform
 * azimuth.  Draws: index then azimuth. */
static int comp_powder(const mxo_comp *c, mxo_stream *s, int draw0, mxo_ray *ray)
{
    const double *dsp = (const double *)c->data0;
    int64_t nd = c->n0;
    double q[3], dl[3];
    to_local(c, ray->r, ray->d, q, dl);
    if (!to_plane_z0(q, dl))
        return 0;
    if (!(fabs(q[0]) <= 0.5 * c->par[0] && fabs(q[1]) <= 0.5 * c->par[1]))
        return 0;
    int64_t j = (int64_t)floor((double)nd * stream_uniform(s, draw0));
    if (j > nd - 1)
        j = nd - 1;
    double lambda = HC_KEV_ANGSTROM / ray->E;
    double sarg = lambda / (2.0 * dsp[j]);
    if (!(sarg <= 1.0))
        return 0;
    double tth = 2.0 * asin(sarg);
    double eta = (2.0 * M_PI) * stream_uniform(s, draw0 + 1);
    /* e1 = normalize(dl x y_hat), e2 = dl x e1 */
    double e1[3] = {-dl[2], 0.0, dl[0]};
    double n1 = cross_dot_norm(e1);
    e1[0] = e1[0] / n1;
    e1[2] = e1[2] / n1;
    double e2[3] = {dl[1] * e1[2] - dl[2] * e1[1], dl[2] * e1[0] - dl[0] * e1[2],
                    dl[0] * e1[1] - dl[1] * e1[0]};
    double ct = cos(tth), st = sin(tth), ce = cos(eta), se = sin(eta);
    double out[3];
    for (int i = 0; i < 3; ++i)
        out[i] = ct * dl[i] + st * (ce * e1[i] + se * e2[i]);
    to_lab(c, q, out, ray->r, ray->d);
    return 1;
}

/* half-open bin of x on [lo, hi) with n bins, or -1 */
static int64_t bin_of(double x, double lo, double hi, int64_t n)
{
    double f = floor((x - lo) * ((double)n / (hi - lo)));
    if (!(f >= 0.0 && f < (double)n))
        return -1;
    return (int64_t)f;
}

/* Ideal energy/position-sensitive monitor in the local plane z = 0: bins
 * (x, y, E) -- or wavelength when flagged -- with the tally index
 * (iy * nx + ix) * ne + ie.  Monitors do not absorb. */
static int comp_detector(const mxo_comp *c, mxo_ray *ray, int64_t *bin)
{
    double q[3], dl[3];
    to_local(c, ray->r, ray->d, q, dl);
    if (!to_plane_z0(q, dl))
        return 0;
    int64_t nx = c->dims[0], ny = c->dims[1], ne = c->dims[2];
    double ev = (c->flags & MXO_DET_WAVELENGTH) ? HC_KEV_ANGSTROM / ray->E : ray->E;
    int64_t ix = bin_of(q[0], c->par[0], c->par[1], nx);
    int64_t iy = bin_of(q[1], c->par[2], c->par[3], ny);
    int64_t ie = bin_of(ev, c->par[4], c->par[5], ne);
    if (ix >= 0 && iy >= 0 && ie >= 0)
        *bin = (iy * nx + ix) * ne + ie;
    else
        *bin = -1;
    to_lab(c, q, dl, ray->r, ray->d);
    return 1;
}

static int draws_of(const mxo_comp *c)
{
    switch (c->type) {
    case MXO_SRC_RECT_CONE: return 5;
    case MXO_SRC_CONE_BEAM: return 3;
    case MXO_SRC_GAUSSIAN: return 5;
    case MXO_POWDER: return 2;
    case MXO_PHANTOM: return (c->flags & 2u) ? 4 * (int)c->par[4] : 0;
    default: return 0;
    }
}

/* ------------------------------------------------------------ ledger ---- */
/* Neumaier-compensated sums of weight: per component k, slots
 * [0] weight entering (for the source: weight emitted), [1] weight of rays
 * absorbed at k, [2] weight removed by attenuation at k, [3] weight tallied
 * at k; one last slot [4K] holds the weight of rays leaving the instrument. */
typedef struct {
    double s, c;
} ksum;

static void kadd(ksum *k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x))
        k->c += (k->s - t) + x;
    else
        k->c += (x - t) + k->s;
    k->s = t;
}

/* ---------------------------------------------------- one ray, in order -- */

typedef struct {
    const mxo_comp *comps;
    int ncomp;
    uint64_t seed, n_total;
    uint32_t purpose, job;
    const double *gmm; /* proposal mixture of the cone-beam source, or NULL */
    double alpha_def;  /* weight of the plain source in the proposal mixture */
} mxo_instr;

/* Carry one ray through components [k0, ncomp): k0 = 0 draws it at the
 * source, k0 = 1 continues a ray whose source state the caller set. */
static void trace_from(const mxo_instr *I, uint64_t ray_id, int k0, mxo_ray *ray, mxo_tally *tallies, ksum *ledger)
{
    mxo_stream s;
    stream_init(&s, I->seed, ray_id, I->purpose, I->job);
    ray->status = MXO_ALIVE;
    ray->dead_at = -1;
    ray->bin = -1;
    int draw = 0, det = 0;
    for (int k = 0; k < k0; ++k)
        draw += draws_of(&I->comps[k]);
    for (int k = k0; k < I->ncomp; ++k) {
        const mxo_comp *c = &I->comps[k];
        double w_in = ray->w;
        mxo_ray before = *ray;
        int ok = 1;
        int64_t bin = -1;
        switch (c->type) {
        case MXO_SRC_RECT_CONE: src_rect_cone(c, &s, ray); w_in = ray->w; break;
        case MXO_SRC_CONE_BEAM:
            if (I->gmm)
                ok = src_cone_proposal(c, &s, ray, ray_id, I->n_total, I->gmm, I->alpha_def);
            else
                src_cone_beam(c, &s, ray, ray_id, I->n_total);
            w_in = ray->w;
            break;
        case MXO_SRC_GAUSSIAN: src_gaussian(c, &s, ray); w_in = ray->w; break;
        case MXO_SLIT: ok = comp_slit(c, ray); break;
        case MXO_BOX: comp_box(c, ray); break;
        case MXO_PHANTOM:
            if (c->flags & 2u)
                ok = comp_phantom_scatter(c, &s, draw, ray);
            else
                comp_phantom(c, ray);
            break;
        case MXO_MIRROR_ELLIPTIC: ok = comp_mirror(c, ray); break;
        case MXO_DCM: ok = comp_dcm(c, ray); break;
        case MXO_POWDER: ok = comp_powder(c, &s, draw, ray); break;
        case MXO_DETECTOR: ok = comp_detector(c, ray, &bin); break;
        case MXO_LENS_CRL: ok = comp_lens(c, ray); break;
        default: ok = 0; break;
        }
        draw += draws_of(c);
        if (ledger)
            kadd(&ledger[4 * k + 0], w_in);
        if (!ok && k == 0) {
            /* a proposal draw outside the cone: emitted with weight 0 */
            ray->status = MXO_ABSORBED;
            ray->dead_at = 0;
            if (ledger)
                kadd(&ledger[1], ray->w);
            return;
        }
        if (!ok) {
            *ray = before;
            ray->status = MXO_ABSORBED;
            ray->dead_at = k;
            if (ledger)
                kadd(&ledger[4 * k + 1], w_in);
            return;
        }
        if (ledger && c->type != MXO_SRC_RECT_CONE && c->type != MXO_SRC_CONE_BEAM &&
            c->type != MXO_SRC_GAUSSIAN)
            kadd(&ledger[4 * k + 2], w_in - ray->w);
        if (c->type == MXO_DETECTOR) {
            if (bin >= 0) {
                ray->bin = bin;
                if (tallies) {
                    tallies[det].count[bin] += 1;
                    tallies[det].sum_w[bin] += ray->w;
                    tallies[det].sum_w2[bin] += ray->w * ray->w;
                }
                if (ledger)
                    kadd(&ledger[4 * k + 3], ray->w);
            }
            det++;
        }
    }
    ray->status = MXO_EXITED;
    if (ledger)
        kadd(&ledger[4 * I->ncomp], ray->w);
}

static void trace_one(const mxo_instr *I, uint64_t ray_id, mxo_ray *ray, mxo_tally *tallies, ksum *ledger)
{
    trace_from(I, ray_id, 0, ray, tallies, ledger);
}

/* ----------------------------------------------------- exported runs ---- */

typedef struct {
    const mxo_instr *I;
    uint64_t begin, end;
    mxo_tally *tallies;
    int n_det;
    ksum *ledger;
} worker_arg;

static void *worker(void *p)
{
    worker_arg *a = (worker_arg *)p;
    mxo_ray ray;
    for (uint64_t r = a->begin; r < a->end; ++r) {
        memset(&ray, 0, sizeof ray);
        trace_one(a->I, r, &ray, a->tallies, a->ledger);
    }
    return NULL;
}

static int count_detectors(const mxo_comp *comps, int ncomp)
{
    int n = 0;
    for (int k = 0; k < ncomp; ++k)
        n += comps[k].type == MXO_DETECTOR;
    return n;
}

/* Trace rays [first, first + n) of an n_total-ray run (with the cone-beam
 * source drawing from the proposal mixture gmm when it is non-null), adding their
 * histograms into the caller's tallies (one per detector, in order) and,
 * when ledger is non-null, their weight ledger (4 * ncomp + 1 doubles).
 * The work is split over n_threads threads by contiguous ray ranges, each
 * with private histograms that are summed at the end. */
int mxo_run(const mxo_comp *comps, int ncomp, uint64_t seed, uint64_t first, uint64_t n,
            uint64_t n_total, uint32_t purpose, uint32_t job, const double *gmm, double alpha_def,
            mxo_tally *tallies, double *ledger, int n_threads)
{
    if (n_threads < 1)
        n_threads = 1;
    mxo_instr I = {comps, ncomp, seed, n_total, purpose, job, gmm, alpha_def};
    int n_det = count_detectors(comps, ncomp);
    int n_slots = 4 * ncomp + 1;
    worker_arg *args = (worker_arg *)calloc((size_t)n_threads, sizeof(worker_arg));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    for (int t = 0; t < n_threads; ++t) {
        args[t].I = &I;
        args[t].begin = first + (n * (uint64_t)t) / (uint64_t)n_threads;
        args[t].end = first + (n * (uint64_t)(t + 1)) / (uint64_t)n_threads;
        args[t].n_det = n_det;
        args[t].tallies = (mxo_tally *)calloc((size_t)(n_det > 0 ? n_det : 1), sizeof(mxo_tally));
        for (int d = 0; d < n_det; ++d) {
            int64_t nb = tallies[d].n_bins;
            args[t].tallies[d].n_bins = nb;
            args[t].tallies[d].count = (uint64_t *)calloc((size_t)nb, sizeof(uint64_t));
            args[t].tallies[d].sum_w = (double *)calloc((size_t)nb, sizeof(double));
            args[t].tallies[d].sum_w2 = (double *)calloc((size_t)nb, sizeof(double));
        }
        args[t].ledger = (ksum *)calloc((size_t)n_slots, sizeof(ksum));
        pthread_create(&th[t], NULL, worker, &args[t]);
    }
    ksum *total = (ksum *)calloc((size_t)n_slots, sizeof(ksum));
    for (int t = 0; t < n_threads; ++t) {
        pthread_join(th[t], NULL);
        for (int d = 0; d < n_det; ++d) {
            for (int64_t b = 0; b < tallies[d].n_bins; ++b) {
                tallies[d].count[b] += args[t].tallies[d].count[b];
                tallies[d].sum_w[b] += args[t].tallies[d].sum_w[b];
                tallies[d].sum_w2[b] += args[t].tallies[d].sum_w2[b];
            }
            free(args[t].tallies[d].count);
            free(args[t].tallies[d].sum_w);
            free(args[t].tallies[d].sum_w2);
        }
        for (int i = 0; i < n_slots; ++i) {
            kadd(&total[i], args[t].ledger[i].s);
            kadd(&total[i], args[t].ledger[i].c);
        }
        free(args[t].tallies);
        free(args[t].ledger);
    }
    if (ledger)
        for (int i = 0; i < n_slots; ++i)
            ledger[i] += total[i].s + total[i].c;
    free(total);
    free(args);
    free(th);
    return 0;
}

/* Trace the listed rays one by one and report their final states. */
int mxo_trace_rays(const mxo_comp *comps, int ncomp, uint64_t seed, uint64_t n_total, uint32_t purpose,
                   uint32_t job, const double *gmm, double alpha_def, const uint64_t *ids, int64_t n,
                   double *r_out, double *d_out, double *E_out, double *w_out, int32_t *status_out,
                   int32_t *dead_out, int64_t *bin_out)
{
    mxo_instr I = {comps, ncomp, seed, n_total, purpose, job, gmm, alpha_def};
    for (int64_t i = 0; i < n; ++i) {
        mxo_ray ray;
        memset(&ray, 0, sizeof ray);
        trace_one(&I, ids[i], &ray, NULL, NULL);
        for (int k = 0; k < 3; ++k) {
            r_out[3 * i + k] = ray.r[k];
            d_out[3 * i + k] = ray.d[k];
        }
        E_out[i] = ray.E;
        w_out[i] = ray.w;
        status_out[i] = ray.status;
        dead_out[i] = ray.dead_at;
        bin_out[i] = ray.bin;
    }
    return 0;
}

/* Continue the listed rays from a given state after the source (position
 * r, direction d, energy E, weight w per ray; the random streams of later
 * components are the rays' own) and report their final states. */
int mxo_trace_after_source(const mxo_comp *comps, int ncomp, uint64_t seed, uint64_t n_total, uint32_t purpose,
                           uint32_t job, const uint64_t *ids, int64_t n, const double *r_in, const double *d_in,
                           const double *E_in, const double *w_in, double *r_out, double *d_out, double *E_out,
                           double *w_out, int32_t *status_out, int32_t *dead_out, int64_t *bin_out)
{
    mxo_instr I = {comps, ncomp, seed, n_total, purpose, job, NULL, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        mxo_ray ray;
        memset(&ray, 0, sizeof ray);
        for (int k = 0; k < 3; ++k) {
            ray.r[k] = r_in[3 * i + k];
            ray.d[k] = d_in[3 * i + k];
        }
        ray.E = E_in[i];
        ray.w = w_in[i];
        trace_from(&I, ids[i], 1, &ray, NULL, NULL);
        for (int k = 0; k < 3; ++k) {
            r_out[3 * i + k] = ray.r[k];
            d_out[3 * i + k] = ray.d[k];
        }
        E_out[i] = ray.E;
        w_out[i] = ray.w;
        status_out[i] = ray.status;
        dead_out[i] = ray.dead_at;
        bin_out[i] = ray.bin;
    }
    return 0;
}
