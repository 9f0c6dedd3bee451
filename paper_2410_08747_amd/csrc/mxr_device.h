// mxr_device.h -- per-ray device code for gfx950: counter-based RNG, ray
// state in registers, the component models and the voxel traversal.
//
// One lane carries one ray from the source to the end of the component list
// (paper, section 2.2: rays are independent; every per-ray intermediate is
// local).  Component parameters live in a small device block read with
// wave-uniform (scalar) loads; the only shared writable state is the monitor
// histograms, updated with FP64 atomics (paper, section 2.2.2: the monitor
// arrays are the one structure threads must share).
//
// The library is compiled with -ffp-contract=off: every expression rounds as
// written, so wherever a formula is the same as in an independent
// implementation the two agree bit for bit; FMA is spelled out only in the
// traversal's inner loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mxr.h"

namespace mxr {

constexpr double kHc = 12.398419843320026;  // keV * Angstrom (CODATA 2018)
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 2.0 * 3.14159265358979323846;
constexpr double kInf = __builtin_huge_val();

enum RayStatus : int32_t { kAlive = 0, kExited = 1, kAbsorbed = 2 };

// Device copy of one component: the caller's parameters plus constants the
// host derives once (aux), the first uniform index it draws, and for a
// monitor its tally slot.
struct DevComp {
    uint32_t type, flags, draw0, slot;
    double pos[3];
    double rot[9];
    double par[16];
    double aux[16];
    const void *data0;
    const void *data1;
    uint64_t n0, n1;
    uint32_t dims[4];
};

struct DevInstr {
    uint32_t ncomp;
    int32_t phantom;  // index of the phantom component or -1
    uint32_t n_mat, n_ebin;
    DevComp c[MXR_MAX_COMPONENTS];
    // the phantom's attenuation table as the kernels stage it in LDS: mu / 10
    // (per mm), energy-major (row e holds every material), n_ebin x n_mat.
    // (After the components, which keep their 16-byte alignment.)
    const double *mu_em;
};

struct TallyPtrs {
    unsigned long long *count[MXR_MAX_DETECTORS];
    double *sum_w[MXR_MAX_DETECTORS];
    double *sum_w2[MXR_MAX_DETECTORS];
};

// Proposal mixture of a cone-beam source, prepared on the host from the
// caller's 8 x (pi, mu[3], sigma[3]) table: per component the normal
// distribution function (P) and its upper tail (Q) at the box edges, in
// standard units, the box masses pi_k Z_k, and the prefactor of the
// component's own truncated density, 1 / (sigma_u sigma_v sigma_E
// (2 pi)^(3/2) F_k) with F_k its box mass without pi_k (0 for an empty
// component).
struct PropTable {
    double kcoef[8];
    double mu[8][3], sigma[8][3], inv_sigma[8][3];
    double Pa[8][3], Pb[8][3], Qa[8][3], Qb[8][3];
    double mass[8];
    double norm;       // sum_k pi_k Z_k
    double alpha;      // share of the plain source in the mixture
    double t2;         // tan^2 of the cone half-angle
    double inv_omega;  // 1 / solid angle of the cone
    double lo[3], hi[3];
};

// Where a hit-collecting run writes the rays that reach a monitor.
struct HitSink {
    float *ctx;                  // n x 6
    double *y;                   // n x 3: u = dx/dz, v = dy/dz (source frame), E
    double *w;                   // n
    int64_t *bin;                // n
    unsigned long long *count;   // rows written (may exceed capacity: then truncated)
    uint64_t capacity;
    float c[6];                  // context of this run
};

// Divisors of a stratified range of n rays over G x G cells, prepared on the
// host: ray i of the range lies in cell floor(i G^2 / n), and a cell holds
// c0 = floor(n / G^2) or c0 + 1 rays (r = n mod G^2 of the cells hold one
// more), so the cell factor (n / G^2) / count takes one of the two values f0
// and f1, each the same division the factor is defined by.  rn, rG and rG2
// are 1/n, 1/G and 1/G^2 rounded, for the quotient estimates.
struct StratDiv {
    uint64_t n, G2, c0, r;
    uint32_t G, pad;
    double rn, rG, rG2, f0, f1;
};

struct RunArgs {
    const DevInstr *ins;
    uint64_t first, n, n_total, seed;
    uint64_t G, G2;  // strata per side used, and its square
    StratDiv sd;     // the same strata's divisors
    uint32_t word3;  // purpose << 24 | job
    uint32_t blocks_per_xcd;
    uint32_t compact_rounds;  // compacting kernel: 64-ray rounds per wave
    uint32_t xcd_order;       // tiles per XCD: 0 the x-th eighth of the range, 1 launch order, 2 runs of 64 tiles
    TallyPtrs tally;
    double *ledger;
    const uint64_t *ids;  // trace mode: ray ids
    mxr_ray_soa dump;     // trace mode: outputs
    const PropTable *prop;  // proposal of the cone-beam source, or null
    // proposal runs: branch b (plain, then components 0..7) takes ray ids
    // [pb[b], pb[b+1]) (pb[0] = 0 is implicit: pb here holds the 9 upper
    // bounds), stratified over psd[b].G^2 cells; pc[b] = its share of the rays
    uint64_t pb[9];
    StratDiv psd[9];
    double pc[9];
    HitSink hits;  // hit-collecting runs
};

// ------------------------------------------------------------- Philox ----
// Philox4x32-10 (Salmon et al., SC'11).  The 32x32->64 products map to
// v_mad_u64_u32.
struct Philox {
    uint32_t k0, k1, c1, c2, c3;

    __device__ __forceinline__ void block(uint32_t j, uint32_t out[4]) const {
        uint32_t x0 = j, x1 = c1, x2 = c2, x3 = c3, a = k0, b = k1;
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            uint64_t pa = (uint64_t)0xD2511F53u * x0;
            uint64_t pb = (uint64_t)0xCD9E8D57u * x2;
            uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ a;
            uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ b;
            x1 = (uint32_t)pb;
            x3 = (uint32_t)pa;
            x0 = y0;
            x2 = y2;
            a += 0x9E3779B9u;
            b += 0xBB67AE85u;
        }
        out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
    }
};

__device__ __forceinline__ double u01(uint32_t lo, uint32_t hi) {
    uint64_t w = ((uint64_t)hi << 32) | lo;
    return ((double)(w >> 12) + 0.5) * 0x1.0p-52;
}

// Uniforms of one ray, produced two at a time on demand.
struct Stream {
    Philox ph;
    int blk;
    uint32_t w[4];

    __device__ __forceinline__ void init(uint64_t seed, uint64_t ray, uint32_t word3) {
        ph.k0 = (uint32_t)seed;
        ph.k1 = (uint32_t)(seed >> 32);
        ph.c1 = (uint32_t)ray;
        ph.c2 = (uint32_t)(ray >> 32);
        ph.c3 = word3;
        blk = -1;
    }
    __device__ __forceinline__ double u(int index) {
        int b = index >> 1;
        if (b != blk) {
            ph.block((uint32_t)b, w);
            blk = b;
        }
        return (index & 1) ? u01(w[2], w[3]) : u01(w[0], w[1]);
    }
};

// ---------------------------------------------------------------- ray ----
struct Ray {
    double r[3], d[3];
    double E, w;
};

__device__ __forceinline__ void to_local(const DevComp &c, const Ray &ray, double q[3], double dl[3]) {
    double v0 = ray.r[0] - c.pos[0], v1 = ray.r[1] - c.pos[1], v2 = ray.r[2] - c.pos[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double *R = c.rot + 3 * i;
        q[i] = R[0] * v0 + R[1] * v1 + R[2] * v2;
        dl[i] = R[0] * ray.d[0] + R[1] * ray.d[1] + R[2] * ray.d[2];
    }
}

__device__ __forceinline__ void to_lab(const DevComp &c, const double q[3], const double dl[3], Ray &ray) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ray.r[i] = c.rot[i] * q[0] + c.rot[3 + i] * q[1] + c.rot[6 + i] * q[2] + c.pos[i];
        ray.d[i] = c.rot[i] * dl[0] + c.rot[3 + i] * dl[1] + c.rot[6 + i] * dl[2];
    }
}

// A ray leaving the component's origin: position pos, direction R dl (what
// to_lab gives for q = 0, since R 0 + pos = pos for a finite rotation).
__device__ __forceinline__ void from_origin(const DevComp &c, const double dl[3], Ray &ray) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ray.r[i] = c.pos[i];
        ray.d[i] = c.rot[i] * dl[0] + c.rot[3 + i] * dl[1] + c.rot[6 + i] * dl[2];
    }
}

__device__ __forceinline__ bool plane_z0(double q[3], const double dl[3]) {
    if (!(dl[2] > 0.0)) return false;
    double t = -q[2] / dl[2];
    if (!(t >= 0.0)) return false;
    q[0] = q[0] + t * dl[0];
    q[1] = q[1] + t * dl[1];
    q[2] = 0.0;
    return true;
}

// ------------------------------------------------------------ sources ----
// Square emitter, cone uniform in solid angle: with s = sqrt(U) sin(a/2) =
// sin(theta/2), sin(theta) = 2 s sqrt(1 - s^2) and cos(theta) = 1 - 2 s^2,
// free of the cancellation of 1 - cos at small angles.
__device__ __forceinline__ void src_rect_cone(const DevComp &c, Stream &s, Ray &ray) {
    double q[3], dl[3];
    q[0] = (s.u(0) - 0.5) * c.par[0];
    q[1] = (s.u(1) - 0.5) * c.par[1];
    q[2] = 0.0;
    double sh = sqrt(s.u(2)) * c.aux[0];
    double ch = sqrt(1.0 - sh * sh);
    double sinp, cosp;
    sincos(kTwoPi * s.u(3), &sinp, &cosp);
    double st = 2.0 * sh * ch;
    dl[0] = st * cosp;
    dl[1] = st * sinp;
    dl[2] = 1.0 - 2.0 * (sh * sh);
    ray.E = c.par[3] + c.aux[1] * s.u(4);
    ray.w = 1.0;
    to_lab(c, q, dl, ray);
}

// Tube spectrum (section 3.4's source: Kramers continuum plus two Gaussian
// lines), per keV and normalised; the constant divisors come as host-side
// reciprocals and quotients: aux[4] = 1/sigma, aux[5] = 1/(sigma sqrt(2 pi)),
// aux[6] = continuum weight / continuum integral.
__device__ __forceinline__ double spectrum(const DevComp &c, double E) {
    double z1 = (E - c.par[5]) * c.aux[4];
    double z2 = (E - c.par[7]) * c.aux[4];
    double g1 = exp(-0.5 * z1 * z1) * c.aux[5];
    double g2 = exp(-0.5 * z2 * z2) * c.aux[5];
    return c.aux[6] * ((c.par[3] - E) / E) + c.par[6] * g1 + c.par[8] * g2;
}

// floor(x / d) from the rounded estimate x * rd (rd = 1/d rounded), for a
// quotient below 2^32 and at most q_max with q_max d < 2^64: the estimate's
// relative error is a few 2^-53, so it lies within 1 of the quotient, and
// one product decides a step down or up.
__device__ __forceinline__ uint64_t div_est(uint64_t x, uint64_t d, double rd, uint64_t q_max) {
    uint64_t q = (uint64_t)((double)x * rd);
    q = q > q_max ? q_max : q;
    const uint64_t p = q * d;
    if (p > x) q -= 1;
    else if (x - p >= d) q += 1;
    return q;
}
__device__ __forceinline__ uint32_t div_est32(uint32_t x, uint32_t d, double rd, uint32_t q_max) {
    uint32_t q = (uint32_t)((double)x * rd);
    q = q > q_max ? q_max : q;
    const uint32_t p = q * d;
    if (p > x) q -= 1;
    else if (x - p >= d) q += 1;
    return q;
}

// Cell (cx, cy) of ray i of a stratified range and its factor (n / G^2) /
// count.  cell = floor(i G^2 / n) < G^2 <= 2^32; the count is c0 plus the
// difference of ceil(j r / G^2) at the cell's two ends (its first ray is
// ceil(cell n / G^2) = cell c0 + ceil(cell r / G^2)).
struct StratCell {
    uint32_t cx, cy;
    double factor;
};
__device__ __forceinline__ StratCell strat_cell(const StratDiv &s, uint64_t i) {
    const uint64_t cell = div_est(i * s.G2, s.n, s.rn, s.G2 - 1);
    const uint32_t cy = div_est32((uint32_t)cell, s.G, s.rG, s.G - 1);
    const uint32_t cx = (uint32_t)cell - cy * s.G;
    uint64_t count = s.c0;
    if (s.r != 0)
        count += div_est((cell + 1) * s.r + s.G2 - 1, s.G2, s.rG2, s.G2 - 1) -
                 div_est(cell * s.r + s.G2 - 1, s.G2, s.rG2, s.G2 - 1);
    return {cx, cy, count == s.c0 ? s.f0 : s.f1};
}

// sin y and cos y for |y| <= pi/4 from their Maclaurin series through y^17
// and y^18 (the first omitted terms, y^19/19! and y^20/20!, are below 1e-19
// there), evaluated by Horner's rule in fused multiply-adds.
__device__ __forceinline__ void sincos_quarter(double y, double &sn, double &cs) {
    const double y2 = y * y;
    double p = -1.0 / 355687428096000.0;
    p = fma(y2, p, 1.0 / 1307674368000.0);
    p = fma(y2, p, -1.0 / 6227020800.0);
    p = fma(y2, p, 1.0 / 39916800.0);
    p = fma(y2, p, -1.0 / 362880.0);
    p = fma(y2, p, 1.0 / 5040.0);
    p = fma(y2, p, -1.0 / 120.0);
    p = fma(y2, p, 1.0 / 6.0);
    sn = fma(-(y * y2), p, y);
    double q = 1.0 / 6402373705728000.0;
    q = fma(y2, q, -1.0 / 20922789888000.0);
    q = fma(y2, q, 1.0 / 87178291200.0);
    q = fma(y2, q, -1.0 / 479001600.0);
    q = fma(y2, q, 1.0 / 3628800.0);
    q = fma(y2, q, -1.0 / 40320.0);
    q = fma(y2, q, 1.0 / 720.0);
    q = fma(y2, q, -1.0 / 24.0);
    q = fma(y2, q, 0.5);
    cs = fma(-y2, q, 1.0);
}

// Concentric map of (ca, cb) in [-1, 1]^2 onto the unit disk: radius rad
// and the angle's sine and cosine.  The angle is (pi/4) x with x = cb/ca,
// or pi/2 - (pi/4) x with x = ca/cb, |x| <= 1; both come from sin and cos
// of y = (pi/4) x (swapped for the second form).
__device__ __forceinline__ void concentric(double ca, double cb, double &rad, double &sa, double &cs) {
    double y = 0.0;
    bool swap = false;
    if (ca == 0.0 && cb == 0.0) {
        rad = 0.0;
    } else if (fabs(ca) > fabs(cb)) {
        rad = ca;
        y = (kPi / 4.0) * (cb / ca);
    } else {
        rad = cb;
        y = (kPi / 4.0) * (ca / cb);
        swap = true;
    }
    double sn, cn;
    sincos_quarter(y, sn, cn);
    sa = swap ? cn : sn;
    cs = swap ? sn : cn;
}

// Cone-beam point source, stratified: ray r lies in cell floor(r G^2 / N);
// the cell's square is mapped to the unit disk by the concentric map and the
// disk radius rho to the cone by sin(theta/2) = rho sin(alpha/2).  Then
// (dx, dy) = sin(theta) (px, py) / rho = 2 sin(alpha/2) cos(theta/2) (px, py).
__device__ __forceinline__ void src_cone_beam(const DevComp &c, Stream &s, Ray &ray, uint64_t ray_id,
                                              const RunArgs &a) {
    const StratCell sc = strat_cell(a.sd, ray_id);
    const double factor = sc.factor;
    double u = ((double)sc.cx + s.u(0)) * a.sd.rG;
    double v = ((double)sc.cy + s.u(1)) * a.sd.rG;
    double ca = 2.0 * u - 1.0, cb = 2.0 * v - 1.0;
    double rad, sa, cs;
    concentric(ca, cb, rad, sa, cs);
    double px = rad * cs, py = rad * sa;
    double sh = fabs(rad) * c.aux[0];
    double ch = sqrt(1.0 - sh * sh);
    double k = 2.0 * c.aux[0] * ch;
    double dl[3] = {k * px, k * py, 1.0 - 2.0 * (sh * sh)};
    ray.E = c.par[1] + c.aux[1] * s.u(2);
    ray.w = (c.aux[1] * spectrum(c, ray.E)) * factor;
    from_origin(c, dl, ray);
}

// Standard normal truncated to [za, zb] by inversion: the point leaving
// mass U of the interval below it, written as a lower-tail probability
// Pa + U (Pb - Pa) when that is at most 1/2 and as the upper-tail
// probability Qb + (1 - U)(Qa - Qb) otherwise, so that no probability near 1
// is inverted.  Phi^-1(p) = -sqrt(2) erfcinv(2p).
__device__ __forceinline__ double trunc_normal(double Pa, double Pb, double Qa, double Qb, double U) {
    const double pl = Pa + U * (Pb - Pa);
    if (pl <= 0.5) return -1.4142135623730951 * erfcinv(2.0 * pl);
    return 1.4142135623730951 * erfcinv(2.0 * (Qb + (1.0 - U) * (Qa - Qb)));
}

// Cone-beam point source drawing y = (u, v, E), u = dx/dz, v = dy/dz, from
// the proposal as a stratified deterministic mixture: the run's ray ids are
// split into contiguous ranges, one per branch (the plain source, then the 8
// truncated-normal components, sized by alpha and the box masses); within its
// range a ray's first two uniforms are stratified over G x G cells like the
// plain source, so the rays of a wave leave in neighbouring directions.  The
// plain branch maps the pair to the cone (concentric map), a component
// inverts a truncated normal per coordinate (E from the third uniform).  The
// weight is p(y) over the realised mixture density sum_b (n_b / n) q_b(y)
// (balance heuristic: unbiased for any split) times the cell factor.  A draw
// outside the cone gets weight 0 and the source returns false.
__device__ __forceinline__ bool src_cone_proposal(const DevComp &c, const PropTable *__restrict__ P, Stream &s,
                                                  Ray &ray, uint64_t ray_id, const RunArgs &a) {
    int branch = -1;
    uint64_t start = 0;
    if (ray_id >= a.pb[0]) {
        for (int k = 0; k < 8; ++k) {
            if (ray_id < a.pb[k + 1]) {
                branch = k;
                start = a.pb[k];
                break;
            }
        }
    }
    const StratDiv &sd = a.psd[branch + 1];
    const StratCell sc = strat_cell(sd, ray_id - start);
    const double factor = sc.factor;
    const double su = ((double)sc.cx + s.u(0)) * sd.rG;
    const double sv = ((double)sc.cy + s.u(1)) * sd.rG;
    double y[3];
    if (branch < 0) {
        double ca = 2.0 * su - 1.0, cb = 2.0 * sv - 1.0;
        double rad, sa, cs;
        concentric(ca, cb, rad, sa, cs);
        double sh = fabs(rad) * c.aux[0];
        double ch = sqrt(1.0 - sh * sh);
        double k = 2.0 * c.aux[0] * ch;
        double dz = 1.0 - 2.0 * (sh * sh);
        y[0] = (k * (rad * cs)) / dz;
        y[1] = (k * (rad * sa)) / dz;
        y[2] = c.par[1] + c.aux[1] * s.u(2);
    } else {
        const double U[3] = {su, sv, s.u(2)};
        for (int d = 0; d < 3; ++d) {
            double z = trunc_normal(P->Pa[branch][d], P->Pb[branch][d], P->Qa[branch][d], P->Qb[branch][d], U[d]);
            y[d] = P->mu[branch][d] + P->sigma[branch][d] * z;
        }
    }
    const double r2 = y[0] * y[0] + y[1] * y[1];
    const bool in_cone = r2 <= P->t2 && y[2] >= P->lo[2] && y[2] <= P->hi[2];
    const bool in_box = y[0] >= P->lo[0] && y[0] <= P->hi[0] && y[1] >= P->lo[1] && y[1] <= P->hi[1] &&
                        y[2] >= P->lo[2] && y[2] <= P->hi[2];
    // the Jacobian (1 + r2)^(-3/2) of the map from (u, v) to directions, from
    // the square root the direction needs anyway (pow would cost ~200
    // instructions per ray; the two forms differ by a few units in the last
    // place)
    const double w2 = 1.0 + r2;
    const double n = sqrt(w2);
    const double J = 1.0 / (w2 * n);
    double q = in_cone ? a.pc[0] * (J * P->inv_omega * c.aux[7]) : 0.0;
    if (in_box) {
        for (int k = 0; k < 8; ++k) {
            if (a.pc[k + 1] == 0.0) continue;
            double zu = (y[0] - P->mu[k][0]) * P->inv_sigma[k][0];
            double zv = (y[1] - P->mu[k][1]) * P->inv_sigma[k][1];
            double ze = (y[2] - P->mu[k][2]) * P->inv_sigma[k][2];
            q += a.pc[k + 1] * (P->kcoef[k] * exp(-0.5 * (zu * zu + zv * zv + ze * ze)));
        }
    }
    const double p_phys = in_cone ? spectrum(c, y[2]) * J * P->inv_omega : 0.0;
    double dl[3] = {y[0] / n, y[1] / n, 1.0 / n};
    ray.E = y[2];
    ray.w = p_phys > 0.0 ? (p_phys / q) * factor : 0.0;
    from_origin(c, dl, ray);
    return p_phys > 0.0;
}

// tan(x): for |x| < 2^-7 the Maclaurin series x + x^3/3 + 2x^5/15 +
// 17x^7/315 + 62x^9/2835 (the first omitted term is below 1e-23 of x there),
// else the library tan.  Beam divergences are micro- to milliradians, so a
// wave normally skips the library call and its argument reduction.
__device__ __forceinline__ double tan_small(double x) {
    if (fabs(x) < 0.0078125) {
        const double x2 = x * x;
        const double p = 1.0 / 3.0 + x2 * (2.0 / 15.0 + x2 * (17.0 / 315.0 + x2 * (62.0 / 2835.0)));
        return x + x * (x2 * p);
    }
    return tan(x);
}

__device__ __forceinline__ void src_gaussian(const DevComp &c, Stream &s, Ray &ray) {
    double r1 = sqrt(-2.0 * log(s.u(0)));
    double s1, c1, s2, c2;
    sincos(kTwoPi * s.u(1), &s1, &c1);
    double r2 = sqrt(-2.0 * log(s.u(2)));
    sincos(kTwoPi * s.u(3), &s2, &c2);
    double q[3], dl[3];
    q[0] = c.par[0] * (r1 * c1);
    q[1] = c.par[1] * (r1 * s1);
    q[2] = 0.0;
    double tx = tan_small(c.par[2] * (r2 * c2));
    double ty = tan_small(c.par[3] * (r2 * s2));
    double nrm = sqrt(tx * tx + ty * ty + 1.0);
    dl[0] = tx / nrm;
    dl[1] = ty / nrm;
    dl[2] = 1.0 / nrm;
    ray.E = c.par[4] * ((1.0 - c.par[5]) + 2.0 * c.par[5] * s.u(4));
    ray.w = 1.0;
    to_lab(c, q, dl, ray);
}

// ---------------------------------------------------------- apertures ----
__device__ __forceinline__ bool comp_slit(const DevComp &c, Ray &ray) {
    double q[3], dl[3];
    to_local(c, ray, q, dl);
    if (!plane_z0(q, dl)) return false;
    if (c.flags & 1u) {
        if (!(q[0] * q[0] + q[1] * q[1] <= c.aux[2])) return false;
    } else {
        if (!(fabs(q[0]) <= c.aux[0] && fabs(q[1]) <= c.aux[1])) return false;
    }
    to_lab(c, q, dl, ray);
    return true;
}

__device__ __forceinline__ void comp_box(const DevComp &c, Ray &ray) {
    double q[3], dl[3];
    to_local(c, ray, q, dl);
    double a_in = 0.0, a_out = kInf;
    bool miss = false;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double h = c.par[i];
        if (dl[i] == 0.0) {
            if (!(q[i] > -h && q[i] < h)) miss = true;
        } else {
            double inv = 1.0 / dl[i];
            double a0 = (-h - q[i]) * inv, a1 = (h - q[i]) * inv;
            double lo = a0 < a1 ? a0 : a1, hi = a0 < a1 ? a1 : a0;
            if (lo > a_in) a_in = lo;
            if (hi < a_out) a_out = hi;
        }
    }
    double L = (!miss && a_out > a_in) ? a_out - a_in : 0.0;
    double E = ray.E;
    double mu = c.par[3] / (E * E * E) + c.par[4];
    ray.w = ray.w * exp(-(mu * L) / 10.0);
}

// --------------------------------------------------------------- lens ----
// Compound refractive lens (section 3.2): N identical bi-concave parabolic
// lenses; lens k (centre c_k = (k - (N-1)/2) p on the local z axis) holds
// material between z = c_k - w/2 - rho^2/2R and z = c_k + w/2 + rho^2/2R
// inside the aperture radius.  Per surface: the intersection quadratic's
// root nearest -C/B in the stable form C / q', the aperture test, the unit
// normal into the next medium, and Snell's law in vector form with the
// normal coefficient sqrt(k) - eta cos_i written as
// (1 - eta^2) / (sqrt(k) + eta cos_i) (no cancellation; 1 - eta^2 comes
// in closed form from delta).  The path inside the material is summed and
// the weight attenuated once.  S = -1 front surface, +1 back surface.
template <int S>
__device__ __forceinline__ bool lens_surface(double q[3], double dl[3], double z0, double inv_R, double inv_2R,
                                             double ra2, double eta, double one_m_eta2, double &t_out) {
    const double A = (double)(-S) * ((dl[0] * dl[0] + dl[1] * dl[1]) * inv_2R);
    const double B = dl[2] - (double)S * ((q[0] * dl[0] + q[1] * dl[1]) * inv_R);
    const double C = (q[2] - z0) - (double)S * ((q[0] * q[0] + q[1] * q[1]) * inv_2R);
    const double disc = B * B - 4.0 * A * C;
    if (!(disc >= 0.0)) return false;
    const double qq = -0.5 * (B + copysign(sqrt(disc), B));
    if (qq == 0.0) return false;
    const double t = C / qq;
    if (!(t >= 0.0)) return false;
#pragma unroll
    for (int i = 0; i < 3; ++i) q[i] = q[i] + t * dl[i];
    if (q[0] * q[0] + q[1] * q[1] > ra2) return false;
    const double g0 = (double)(-S) * (q[0] * inv_R), g1 = (double)(-S) * (q[1] * inv_R);
    const double inv_gn = 1.0 / sqrt(g0 * g0 + g1 * g1 + 1.0);
    const double m0 = g0 * inv_gn, m1 = g1 * inv_gn, m2 = inv_gn;
    const double cos_i = dl[0] * m0 + dl[1] * m1 + dl[2] * m2;
    if (!(cos_i > 0.0)) return false;
    const double k = 1.0 - eta * eta * (1.0 - cos_i * cos_i);
    if (!(k >= 0.0)) return false;
    const double gc = one_m_eta2 / (sqrt(k) + eta * cos_i);
    dl[0] = eta * dl[0] + gc * m0;
    dl[1] = eta * dl[1] + gc * m1;
    dl[2] = eta * dl[2] + gc * m2;
    t_out = t;
    return true;
}

// aux: 0 1/R, 1 1/(2R), 2 aperture radius^2
__device__ __forceinline__ bool comp_lens(const DevComp &c, Ray &ray) {
    double q[3], dl[3];
    to_local(c, ray, q, dl);
    const double inv_R = c.aux[0], inv_2R = c.aux[1], ra2 = c.aux[2];
    const double w = c.par[2], pitch = c.par[3];
    const int N = (int)c.par[1];
    const double E = ray.E;
    const double er = c.par[6] / E;
    const double delta = c.par[5] * (er * er);
    const double mu = c.par[7] / (E * E * E) + c.par[8];
    const double eta_in = 1.0 / (1.0 - delta), eta_out = 1.0 - delta;
    const double ome_in = -delta * (2.0 - delta) / ((1.0 - delta) * (1.0 - delta));
    const double ome_out = delta * (2.0 - delta);
    const double half_n1 = 0.5 * (double)(N - 1);
    double L = 0.0, t;
    for (int k = 0; k < N; ++k) {
        const double ck = ((double)k - half_n1) * pitch;
        if (!lens_surface<-1>(q, dl, ck - 0.5 * w, inv_R, inv_2R, ra2, eta_in, ome_in, t)) return false;
        if (!lens_surface<1>(q, dl, ck + 0.5 * w, inv_R, inv_2R, ra2, eta_out, ome_out, t)) return false;
        L = L + t;
    }
    ray.w = ray.w * exp(-(mu * L) / 10.0);
    to_lab(c, q, dl, ray);
    return true;
}

// ------------------------------------------------------------ phantom ----
// Exact radiological path through the voxel grid.
//
// The ray is walked along its dominant axis D (largest |d|): every step
// crosses one D plane; with cubic voxels and |d_A|, |d_B| <= |d_D| at most
// one plane of each other axis lies between two D planes, so those rarer
// crossings are taken in a branch that coherent waves mostly skip.  Every
// crossing parameter is a fixed function of the exact plane coordinate
// (fma(plane, inv, -q inv), or (plane - q) inv, with inv = 1/d and q fixed
// per ray and axis), so a plane's alpha is the same number in whatever order
// the planes are visited and in the set-up that finds the first plane
// (negative directions are mirrored so every axis steps by +v, which
// leaves both forms unchanged).  The optical depth is accumulated per material run:
// segment lengths between crossings telescope, so a run of voxels of one
// material adds mu * (alpha_end - alpha_start) -- the same sum of
// mu * length as segment by segment, up to rounding -- and the mu table is
// read only where the material changes.  Voxels are read with buffer loads
// (hardware range check: an out-of-range offset reads 0 instead of
// faulting).  The walk is bounded by nx + ny + nz + 3 steps.
#ifndef MXR_WALK_ROUND
#define MXR_WALK_ROUND 4
#endif
#ifndef MXR_LOCATE_ROUND
#define MXR_LOCATE_ROUND 3
#endif
constexpr int kWalkRound = MXR_WALK_ROUND;      // crossings per round of loads
constexpr int kLocateRound = MXR_LOCATE_ROUND;  // the same for the locate walks

struct PhantomGeo {
    const uint8_t *vol;
    uint32_t nvox;
    int n[3];
    double v, rv;  // voxel edge and its reciprocal
    double corner[3];
    // the occupied box: every voxel outside the planes blo[i] .. bhi[i] holds
    // material bg; box = false when every voxel does
    double blo[3], bhi[3];
    uint32_t bg;
    bool box;
};

// The loaded byte goes through an empty asm so that it stays a plain 32-bit
// value: the compiler otherwise narrows the walk's materials to 16 bits and
// masks the loads with extra instructions.
__device__ __forceinline__ uint32_t load_voxel(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    uint32_t m = (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, off, 0, 0);
    asm("" : "+v"(m));
    return m;
}

template <class T>
__device__ __forceinline__ T pick3(int k, T a0, T a1, T a2) {
    return k == 0 ? a0 : (k == 1 ? a1 : a2);
}

// alpha of the plane at coordinate P on an axis with start q, reciprocal
// direction inv and offset nq = -q inv.  ONE_ROUNDING: fma(P, inv, nq), one
// instruction, one rounding after the exact product; otherwise
// (P - q) * inv, the reference definition's rounding.  The walks that
// locate interaction points keep the latter: a scattering chain feeds each
// located point into the next walk, so it stays on the reference's
// roundings, while a plain optical depth only sums the crossings' alphas.
template <bool ONE_ROUNDING>
__device__ __forceinline__ double plane_alpha(double P, double q, double inv, double nq) {
    if constexpr (ONE_ROUNDING) return fma(P, inv, nq);
    else return (P - q) * inv;
}

// Per-axis walk state, one entry per axis; roles D, A, B pick from it with
// selects (registers cannot be indexed by a per-lane value).
struct AxisSet {
    double P[3], q[3], nq[3], inv[3], c[3];  // c: corner, mirrored (-corner) for negative directions
    int k[3], doff[3];
};

// Minimum of two doubles that are never NaN, as the one VALU instruction
// v_min_f64.  The ternary a < b ? a : b compiles to a compare and two
// selects, and fmin() adds canonicalising instructions for operands the
// compiler cannot prove canonical; the walk's alphas are finite or +inf and
// positive, so a tie returns the same number either way.
__device__ __forceinline__ double min_f64(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// The divergent event's updates, written so that each new value takes the
// register of the value it replaces (tied operands).  The uniform D step
// leaves the A and B state untouched; with in-place updates on the other
// path the two paths meet without register copies (the compiler otherwise
// gives the new values fresh registers and copies the old ones on the
// uniform path, five to six moves per event).  Same arithmetic as
// P = fma(f, v, P), a = fma(P, inv, nq) and m = min(a, b).
__device__ __forceinline__ void step_in_place(double &P, double f, double v) {
    asm("v_fma_f64 %0, %1, %2, %0" : "+v"(P) : "v"(f), "s"(v));
}
__device__ __forceinline__ void alpha_in_place(double &a, double P, double inv, double nq) {
    asm("v_fma_f64 %0, %1, %2, %3" : "+v"(a) : "v"(P), "v"(inv), "v"(nq));
}
__device__ __forceinline__ void min_in_place(double &m, double a, double b) {
    asm("v_min_f64 %0, %1, %2" : "+v"(m) : "v"(a), "v"(b));
}

// clamp(x, 0, hi) for hi >= 0 as one v_med3_i32, and a * b + c on the low
// 24 bits of a and b as one full-rate v_mad_u32_u24.  Written out because
// the compiler emits max + min for the first and folds the second into a
// 64-bit multiply-add.  hi and a are wave-uniform here (the phantom's
// dimensions) and stay in scalar registers.
__device__ __forceinline__ int clamp0_i32(int x, int hi) {
    int r;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(x), "s"(hi));
    return r;
}
__device__ __forceinline__ uint32_t mad_u24(int a, int b, int c) {
    uint32_t r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "s"(a), "v"(b), "v"(c));
    return r;
}

// The walk in rounds of K crossings ("events").  Each event is the nearest
// of the next D, A and B crossings (D first on ties with the others, A before
// B); its alpha is computed from the plane coordinate, so it is the same
// number the merged order of all crossings would see.  The nearer of the A
// and B crossings is kept (mAB), so one compare tells whether a lane's next
// event is a D step.  When no lane of the wave has an A or B crossing next,
// the event is a D step for the whole wave (the common case).  Otherwise
// every lane steps one axis without branching: each axis's plane advances
// by a factor of 1 or 0 times v (an exact fma), and all three alphas are
// recomputed from their planes, which leaves the two unchanged ones bit for
// bit as they were.  An axis the ray runs parallel to has inv = 0 and
// nq = +inf, so its alpha is +inf and it never steps.  The K voxel loads of
// a round are issued together and then folded into the material runs in
// order.  Events are not clipped to the exit: a lane past its exit keeps
// stepping, and the fold clips each closing alpha to a_out, so runs past the
// exit have zero length and add nothing (their voxels are read through the
// range-checked buffer).
//
// LOCATE: also find where the running optical depth reaches tau_star.  Within
// a material run mu is constant, so the point is checked when a run closes:
// a_start + (tau_star - tau_before) / mu in the first attenuating run whose
// closing depth reaches tau_star (hit.found); hit.last_end / last_m keep the
// end and material of the last attenuating run for a tau_star that rounding
// leaves beyond the total.  A wave leaves the walk once every lane has found
// its point or passed its exit.
struct WalkHit {
    double s = 0.0, last_end = 0.0;
    uint32_t m = 0, last_m = 0;
    bool found = false;
};

// Close the material run [a_start, tc] of material m (attenuation mu) onto
// the optical depth tau; LOCATE: and check it for the depth tau_star.
template <bool LOCATE>
__device__ __forceinline__ void close_run(double tc, double mu, uint32_t m, double &tau, double a_start,
                                          double tau_star, WalkHit *hit) {
    const double closed = fma(mu, tc - a_start, tau);
    if constexpr (LOCATE) {
        if (mu > 0.0 && tc > a_start) {
            if (!hit->found && closed >= tau_star) {
                hit->found = true;
                hit->s = a_start + (tau_star - tau) / mu;
                hit->m = m;
            }
            hit->last_end = tc;
            hit->last_m = m;
        }
    }
    tau = closed;
}

// a_vol <= a_in: the path enters the volume at a_vol and the walk at a_in,
// the first voxel (off) lying just past a_in; before it the path runs in
// material bg (bg < 0: a_vol = a_in).  The walk stops once every lane's events
// reach a_stop <= a_out; runs still close at a_out.
template <bool EXACT, int K, bool LOCATE = false>
__device__ __forceinline__ double siddon_walk(const PhantomGeo &g, const AxisSet &S, int D, int A, int B,
                                              uint32_t off, double a_vol, double a_in, double a_stop, double a_out,
                                              int bg, const double *__restrict__ mu_row, double tau_star = 0.0,
                                              WalkHit *hit = nullptr) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)g.vol, (short)0, (int)g.nvox, 0x00020000);
    const double v = g.v;
    double PD = pick3(D, S.P[0], S.P[1], S.P[2]), PA = pick3(A, S.P[0], S.P[1], S.P[2]);
    double PB = pick3(B, S.P[0], S.P[1], S.P[2]);
    constexpr bool ONE = !LOCATE;
    const double nD = pick3(D, S.nq[0], S.nq[1], S.nq[2]);
    const double nA = pick3(A, S.nq[0], S.nq[1], S.nq[2]), nB = pick3(B, S.nq[0], S.nq[1], S.nq[2]);
    const double qD = pick3(D, S.q[0], S.q[1], S.q[2]);
    const double qA = pick3(A, S.q[0], S.q[1], S.q[2]), qB = pick3(B, S.q[0], S.q[1], S.q[2]);
    const double iD = pick3(D, S.inv[0], S.inv[1], S.inv[2]);
    const double iA = pick3(A, S.inv[0], S.inv[1], S.inv[2]), iB = pick3(B, S.inv[0], S.inv[1], S.inv[2]);
    int kD = pick3(D, S.k[0], S.k[1], S.k[2]), kA = pick3(A, S.k[0], S.k[1], S.k[2]);
    int kB = pick3(B, S.k[0], S.k[1], S.k[2]);
    const int oD = pick3(D, S.doff[0], S.doff[1], S.doff[2]), oA = pick3(A, S.doff[0], S.doff[1], S.doff[2]);
    const int oB = pick3(B, S.doff[0], S.doff[1], S.doff[2]);
    const int dA = oA - oD, dB = oB - oD;  // offset change of an A or B step in place of the D step
    // plane k of a mirrored axis sits at -corner + k v
    const double cD = pick3(D, S.c[0], S.c[1], S.c[2]);
    const double cA = pick3(A, S.c[0], S.c[1], S.c[2]), cB = pick3(B, S.c[0], S.c[1], S.c[2]);
    double aD = plane_alpha<ONE>(PD, qD, iD, nD);
    double aA = plane_alpha<ONE>(PA, qA, iA, nA);
    double aB = plane_alpha<ONE>(PB, qB, iB, nB);
    double mAB = min_f64(aA, aB);

    uint32_t run_m = load_voxel(rs, off);
    double a_start = a_vol, tau = 0.0;
    if (bg >= 0 && run_m != (uint32_t)bg) {
        // the background run ends where the walk enters its first voxel
        close_run<LOCATE>(a_in, mu_row[bg], (uint32_t)bg, tau, a_vol, tau_star, hit);
        a_start = a_in;
    }
    const int max_rounds = __builtin_amdgcn_readfirstlane((g.n[0] + g.n[1] + g.n[2] + 3) / K + 2);
    for (int round = 0; round < max_rounds; ++round) {
        uint32_t o[K];
        double t[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const bool side = mAB < aD;
            t[j] = min_f64(aD, mAB);
            // every lane takes the D step; a lane whose next crossing is an
            // A or B plane takes that one instead: in an exec-masked block it
            // advances that plane, adds the stride difference and moves its
            // D plane back by v (exact), so the step leaves it in place
            off += (uint32_t)oD;
            if constexpr (EXACT) PD = PD + v;
            else ++kD;
            const uint64_t wside = __builtin_amdgcn_ballot_w64(side);
            if (LOCATE && wside != 0) {
                // the locate walks (scattering chains, whose kernel runs
                // short of registers): every lane advances each axis's plane
                // by a 0/1 factor times v (branch-free, no exec changes)
                const bool tA = side && aA <= aB;
                const bool tB = side && !tA;
                off += (uint32_t)(tA ? dA : (tB ? dB : 0));
                if constexpr (EXACT) {
                    PD = fma(side ? -1.0 : 0.0, v, PD);
                    PA = fma(tA ? 1.0 : 0.0, v, PA);
                    PB = fma(tB ? 1.0 : 0.0, v, PB);
                } else {
                    kD -= side;
                    kA += tA;
                    kB += tB;
                    PA = cA + (double)kA * v;
                    PB = cB + (double)kB * v;
                }
                aA = plane_alpha<ONE>(PA, qA, iA, nA);
                aB = plane_alpha<ONE>(PB, qB, iB, nB);
                mAB = min_f64(aA, aB);
            } else if (wside != 0) {
                // the A/B order as a lane mask straight from the compare, so
                // the wave can skip a block that none of its lanes takes
                const uint64_t wle = __builtin_amdgcn_fcmp(aA, aB, 5);  // FCMP_OLE: ordered <=
                const bool AfirstB = aA <= aB;
                if (__builtin_expect((wside & wle) != 0, 0)) {
                    if (side && AfirstB) {
                        off += (uint32_t)dA;
                        PA = EXACT ? PA + v : cA + (double)(++kA) * v;
                        aA = plane_alpha<ONE>(PA, qA, iA, nA);
                        if constexpr (EXACT) PD = PD - v;
                        else kD -= 1;
                    }
                }
                if (__builtin_expect((wside & ~wle) != 0, 0)) {
                    if (side && !AfirstB) {
                        off += (uint32_t)dB;
                        PB = EXACT ? PB + v : cB + (double)(++kB) * v;
                        aB = plane_alpha<ONE>(PB, qB, iB, nB);
                        if constexpr (EXACT) PD = PD - v;
                        else kD -= 1;
                    }
                }
                mAB = min_f64(aA, aB);
            }
            if constexpr (!EXACT) PD = cD + (double)kD * v;
            aD = plane_alpha<ONE>(PD, qD, iD, nD);
            o[j] = off;
        }
        uint32_t m[K];
#pragma unroll
        for (int j = 0; j < K; ++j) m[j] = load_voxel(rs, o[j]);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            // a material change closes the run (a wave with no change skips
            // the block on its empty execution mask)
            if (m[j] != run_m) {
                const double tc = min_f64(t[j], a_out);
                close_run<LOCATE>(tc, mu_row[run_m], run_m, tau, a_start, tau_star, hit);
                a_start = tc;
                run_m = m[j];
            }
        }
        // every lane is past its exit once its last event lies at or beyond a_out
        if constexpr (LOCATE) {
            if (__builtin_amdgcn_ballot_w64(t[K - 1] < a_out && !hit->found) == 0) break;
        } else {
            if (__builtin_amdgcn_ballot_w64(t[K - 1] < a_stop) == 0) break;
        }
    }
    close_run<LOCATE>(a_out, mu_row[run_m], run_m, tau, a_start, tau_star, hit);
    return tau;
}

// EXACT: every plane coordinate corner + i v is reached exactly by adding v
// (true for dyadic voxel sizes such as 1 mm); decided once per instrument.
// BOX (optical depths only): the walk covers the path's stretch inside the
// occupied box.  Outside it every voxel holds the background material, so
// the run that enters the volume there stays open up to the box, and the
// box's faces are crossed at the alphas the full walk computes for those
// planes (fma(plane, inv, -q inv)): the same runs and sums, except that a
// path touching the box only along an edge or a face takes its background run
// in one piece (a zero-length run less, a rounding of the sum).
template <bool EXACT, bool LOCATE = false, bool BOX = false, int KW = kWalkRound>
__device__ __forceinline__ double siddon_tau(const PhantomGeo &g, const double q[3], const double dl[3],
                                             const double *__restrict__ mu_row, double tau_star = 0.0,
                                             WalkHit *hit = nullptr) {
    double inv[3];
    double a_in = 0.0, a_out = kInf;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double lo_p = g.corner[i];
        double hi_p = g.corner[i] + (double)g.n[i] * g.v;
        if (dl[i] == 0.0) {
            inv[i] = 0.0;
            if (!(q[i] > lo_p && q[i] < hi_p)) return 0.0;
        } else {
            inv[i] = 1.0 / dl[i];
            double a0 = (lo_p - q[i]) * inv[i], a1 = (hi_p - q[i]) * inv[i];
            double lo = a0 < a1 ? a0 : a1, hi = a0 < a1 ? a1 : a0;
            if (lo > a_in) a_in = lo;
            if (hi < a_out) a_out = hi;
        }
    }
    if (!(a_out > a_in)) return 0.0;
    const double a_vol = a_in;
    double a_stop = a_out;
    int bg = -1;
    if constexpr (BOX && !LOCATE) {
        bool miss = !g.box;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (dl[i] == 0.0) {
                // the voxel slab the walk would keep (as in the set-up below)
                const double f = floor((q[i] - g.corner[i]) / g.v);
                const int idx = (int)fmin(fmax(f, 0.0), (double)(g.n[i] - 1));
                const int lo = (int)rint((g.blo[i] - g.corner[i]) * g.rv);
                const int hi = (int)rint((g.bhi[i] - g.corner[i]) * g.rv);
                if (idx < lo || idx >= hi) miss = true;
            } else {
                const double nq = -(q[i] * inv[i]);
                const double b0 = fma(g.blo[i], inv[i], nq), b1 = fma(g.bhi[i], inv[i], nq);
                a_in = fmax(a_in, fmin(b0, b1));
                a_stop = fmin(a_stop, fmax(b0, b1));
            }
        }
        if (miss || !(a_stop > a_in)) return fma(mu_row[g.bg], a_out - a_vol, 0.0);
        bg = (int)g.bg;
    }

    // Per axis: the voxel holding the start of the walk and the first plane
    // crossed after a_in.  Planes are mirrored for negative directions
    // (coordinate -x, plane index counted downwards), so that the next plane
    // is always reached by adding v; alpha keeps its value (with -P, -q and
    // -inv the product P inv and the difference (P - q) inv are the same
    // numbers, -q inv unchanged).  An axis the ray runs parallel to gets an
    // alpha of +inf: inv = 0 and nq = +inf for the one-rounding form, a
    // plane ahead of q and inv = +inf for the other.
    constexpr bool ONE = !LOCATE;
    int idx[3];
    AxisSet S;
    const int nx = g.n[0], nxy = g.n[0] * g.n[1];
    const int stride[3] = {1, nx, nxy};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int n = g.n[i];
        const double c = g.corner[i], v = g.v;
        if (dl[i] == 0.0) {
            double f = floor((q[i] - c) / v);
            idx[i] = (int)fmin(fmax(f, 0.0), (double)(n - 1));
            S.k[i] = 0;
            S.P[i] = ONE ? 0.0 : q[i] + 1.0;
            S.q[i] = q[i];
            S.nq[i] = kInf;
            S.inv[i] = ONE ? 0.0 : kInf;
            S.c[i] = c;
            S.doff[i] = 0;
            continue;
        }
        const double nq = -(q[i] * inv[i]);
        const double x_in = q[i] + a_in * dl[i];
        const double f = (x_in - c) * g.rv;  // an estimate: p is corrected below
        int p;
        if (dl[i] > 0.0) {
            // first plane p in [1, n] with alpha(p) > a_in
            p = (int)fmin(fmax(floor(f) + 1.0, 1.0), (double)n);
            if (p > 1 && plane_alpha<ONE>(c + (double)(p - 1) * v, q[i], inv[i], nq) > a_in) p -= 1;
            if (p < n && !(plane_alpha<ONE>(c + (double)p * v, q[i], inv[i], nq) > a_in)) p += 1;
            idx[i] = p - 1;
            S.k[i] = p;
            S.P[i] = c + (double)p * v;
            S.q[i] = q[i];
            S.nq[i] = nq;
            S.inv[i] = inv[i];
            S.c[i] = c;
            S.doff[i] = stride[i];
        } else {
            // last plane p in [0, n - 1] with alpha(p) > a_in, walked downwards
            p = (int)fmin(fmax(ceil(f) - 1.0, 0.0), (double)(n - 1));
            if (p < n - 1 && plane_alpha<ONE>(c + (double)(p + 1) * v, q[i], inv[i], nq) > a_in) p += 1;
            if (p > 0 && !(plane_alpha<ONE>(c + (double)p * v, q[i], inv[i], nq) > a_in)) p -= 1;
            idx[i] = p;
            // mirrored: plane index k = -p, coordinate -(c + p v), -q, -inv
            S.k[i] = -p;
            S.P[i] = -(c + (double)p * v);
            S.q[i] = -q[i];
            S.nq[i] = nq;
            S.inv[i] = -inv[i];
            S.c[i] = -c;
            S.doff[i] = -stride[i];
        }
    }
    // dominant axis (largest |d|, lowest index on ties) and the other two
    const double ax = fabs(dl[0]), ay = fabs(dl[1]), az = fabs(dl[2]);
    int D, A, B;
    if (ax >= ay && ax >= az) { D = 0; A = 1; B = 2; }
    else if (ay >= az) { D = 1; A = 0; B = 2; }
    else { D = 2; A = 0; B = 1; }
    const uint32_t off = (uint32_t)(idx[0] + nx * idx[1] + nxy * idx[2]);
    return siddon_walk<EXACT, LOCATE ? kLocateRound : KW, LOCATE>(g, S, D, A, B, off, a_vol, a_in, a_stop,
                                                                         a_out, bg, mu_row, tau_star, hit);
}

// ------------------------------------------------- scattering phantom ----
// Photons scattered exactly K times in the volume (section 3.3: the voxel
// sample models absorption and scattering), each interaction forced: on the
// chord ahead the total optical depth tau is taken by the exact walk, the
// depth tau* = -log(1 - u1 (1 - e^-tau)) is located by the same walk (in
// the material run where the running depth reaches tau*, at
// a_start + (tau* - tau_before) / mu), and the weight takes 1 - e^-tau,
// the scatter albedo
// (mu_R + mu_C) / mu_tot of the voxel's material and the angular factor;
// Rayleigh (Thomson law, no form factor) is chosen with probability
// mu_R / (mu_R + mu_C) (u2), Compton (Klein-Nishina, free electrons)
// otherwise, lowering E to E / (1 + k (1 - cos)).  Directions: uniform on
// the sphere (cos = 2 u3 - 1, phi = 2 pi u4 about the old direction, frame
// e1 = d x a / |d x a| with a = y unless |d_y| >= 1/2, then x, e2 = d x e1),
// weight 4 pi x the density per steradian; or, for the last interaction of
// an aimed phantom (flags bit 2), towards the point c + (2 u3 - 1) a +
// (2 u4 - 1) b of a target rectangle, weight = density / (dist^2 /
// (|n . d| 4 |a x b|)).  After the K-th interaction the walk to the exit
// attenuates at the final energy.  The total-attenuation channel is read
// from LDS (mu / 10 per mm, as for the plain phantom), the Rayleigh and
// Compton channels from the table in global memory at each interaction.
constexpr double kMeC2Kev = 510.99895;

// Klein-Nishina total cross section over 2 pi r_e^2
__device__ __forceinline__ double kn_f(double k) {
    const double l = log1p(2.0 * k);
    return ((1.0 + k) / (k * k)) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k) + l / (2.0 * k) -
           (1.0 + 3.0 * k) / ((1.0 + 2.0 * k) * (1.0 + 2.0 * k));
}

// Walk the chord from q along dl voxel by voxel (every plane crossing at
// alpha = (plane - q) / d with plane = corner + p v, as in the exact walk),
// summing mu * length segment by segment until the running optical depth
// reaches tau_star.  Returns true with the interaction distance s and the
// voxel's material (if rounding leaves tau_star beyond the last attenuating
// segment: the end of that segment); with tau_star = infinity it walks the
// whole chord and tau_out is the chord's optical depth.  False if the ray
// misses the volume.  Bounded by nx + ny + nz + 3 steps.
__device__ __forceinline__ bool siddon_locate(const PhantomGeo &g, const double q[3], const double dl[3],
                                              const double *__restrict__ mu_row, double tau_star, double &s_out,
                                              uint32_t &m_out, double &tau_out) {
    double inv[3], a_in = 0.0, a_out = kInf;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double lo_p = g.corner[i], hi_p = g.corner[i] + (double)g.n[i] * g.v;
        if (dl[i] == 0.0) {
            inv[i] = 0.0;
            if (!(q[i] > lo_p && q[i] < hi_p)) return false;
        } else {
            inv[i] = 1.0 / dl[i];
            const double a0 = (lo_p - q[i]) * inv[i], a1 = (hi_p - q[i]) * inv[i];
            const double lo = a0 < a1 ? a0 : a1, hi = a0 < a1 ? a1 : a0;
            if (lo > a_in) a_in = lo;
            if (hi < a_out) a_out = hi;
        }
    }
    if (!(a_out > a_in)) return false;
    int idx[3], p[3], st[3];
    double na[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int n = g.n[i];
        const double c = g.corner[i], v = g.v;
        if (dl[i] == 0.0) {
            const double f = floor((q[i] - c) / v);
            idx[i] = (int)fmin(fmax(f, 0.0), (double)(n - 1));
            p[i] = 0;
            st[i] = 0;
            na[i] = kInf;
            continue;
        }
        const double f = ((q[i] + a_in * dl[i]) - c) / v;
        if (dl[i] > 0.0) {
            int pp = (int)fmin(fmax(floor(f) + 1.0, 1.0), (double)n);
            if (pp > 1 && ((c + (double)(pp - 1) * v) - q[i]) * inv[i] > a_in) pp -= 1;
            if (pp < n && !(((c + (double)pp * v) - q[i]) * inv[i] > a_in)) pp += 1;
            idx[i] = pp - 1;
            p[i] = pp;
            st[i] = 1;
        } else {
            int pp = (int)fmin(fmax(ceil(f) - 1.0, 0.0), (double)(n - 1));
            if (pp < n - 1 && ((c + (double)(pp + 1) * v) - q[i]) * inv[i] > a_in) pp += 1;
            if (pp > 0 && !(((c + (double)pp * v) - q[i]) * inv[i] > a_in)) pp -= 1;
            idx[i] = pp;
            p[i] = pp;
            st[i] = -1;
        }
        na[i] = ((c + (double)p[i] * v) - q[i]) * inv[i];
    }
    // per-axis state in scalars (an array indexed by the crossing axis
    // would live in scratch memory)
    const int nx = g.n[0], nxy = g.n[0] * g.n[1];
    int i0 = idx[0], i1 = idx[1], i2 = idx[2];
    int p0 = p[0], p1 = p[1], p2 = p[2];
    double n0 = na[0], n1 = na[1], n2 = na[2];
    double a_prev = a_in, tc = 0.0, last_end = a_in;
    uint32_t last_m = 0;
    // the next voxel's load is issued before the current segment is summed
    // (its index does not depend on the material), hiding its latency
    uint32_t m = g.vol[i0 + nx * i1 + nxy * i2];
    const int max_steps = g.n[0] + g.n[1] + g.n[2] + 3;
    for (int step = 0; step < max_steps; ++step) {
        const int ax = (n1 < n0) ? ((n2 < n1) ? 2 : 1) : ((n2 < n0) ? 2 : 0);
        const double nmin = min_f64(n0, min_f64(n1, n2));  // the value of axis ax
        const double a_next = min_f64(nmin, a_out);
        const bool more = nmin < a_out;
        if (more) {
            // cross the plane: the next voxel along that axis (clamped)
            if (ax == 0) {
                i0 = clamp0_i32(i0 + st[0], g.n[0] - 1);
                p0 += st[0];
                n0 = ((g.corner[0] + (double)p0 * g.v) - q[0]) * inv[0];
            } else if (ax == 1) {
                i1 = clamp0_i32(i1 + st[1], g.n[1] - 1);
                p1 += st[1];
                n1 = ((g.corner[1] + (double)p1 * g.v) - q[1]) * inv[1];
            } else {
                i2 = clamp0_i32(i2 + st[2], g.n[2] - 1);
                p2 += st[2];
                n2 = ((g.corner[2] + (double)p2 * g.v) - q[2]) * inv[2];
            }
        }
        const uint32_t m_next = g.vol[i0 + nx * i1 + nxy * i2];
        const double mu = mu_row[m];
        if (mu > 0.0 && a_next > a_prev) {
            const double d = mu * (a_next - a_prev);
            last_m = m;
            last_end = a_next;
            if (tc + d >= tau_star) {
                s_out = a_prev + (tau_star - tc) / mu;
                m_out = m;
                tau_out = tc + d;
                return true;
            }
            tc = tc + d;
        }
        if (!more) break;
        m = m_next;
        a_prev = a_next;
    }
    s_out = last_end;
    m_out = last_m;
    tau_out = tc;
    return true;
}

// The scattering phantom component: par 4 = K; flags bit 2 aims the last
// interaction at the rectangle par 5..7 (centre), 8..10 and 11..13 (half
// axes), lab frame.  T: the three-channel table (1/cm) in global memory.
// The 2K + 1 walks (optical depth ahead, interaction point, ..., exit) run
// as passes of one loop: the event walk in locate mode (tau_star infinite for
// the depth and exit passes) for the coherent chords, the voxel-by-voxel
// walk for the chords after an isotropic scatter.
template <bool EXACT>
__device__ __forceinline__ bool comp_phantom_scatter(const DevComp &c, Stream &s, Ray &ray, const double *mu_lds,
                                                     uint32_t n_mat, uint32_t n_ebin) {
    double q[3], dl[3];
    to_local(c, ray, q, dl);
    PhantomGeo g;
    g.vol = (const uint8_t *)c.data0;
    g.n[0] = (int)c.dims[0];
    g.n[1] = (int)c.dims[1];
    g.n[2] = (int)c.dims[2];
    g.v = c.par[0];
    g.rv = c.aux[6];
    g.corner[0] = c.aux[0];
    g.corner[1] = c.aux[1];
    g.corner[2] = c.aux[2];
    g.nvox = (uint32_t)c.n0;
    const double *__restrict__ T = (const double *)c.data1;
    const uint32_t plane = n_mat * n_ebin;
    const int K = (int)c.par[4];
    const bool aimed = (c.flags & 4u) != 0;
    double E = ray.E, w = ray.w, tau_star = kInf, pint = 0.0;
    int e = 0;
    for (int pass = 0; pass <= 2 * K; ++pass) {
        const int k = pass >> 1;
        const bool locate = (pass & 1) != 0;
        if (!locate) {
            const double f = floor((E - c.par[1]) * c.aux[3]);
            e = (int)fmin(fmax(f, 0.0), (double)(n_ebin - 1));
            tau_star = kInf;
        }
        // chords along the primary or towards the target are coherent
        // across a wave and take the event walk; chords after an isotropic
        // scatter go voxel by voxel
        const bool coherent = k == 0 || (k == K && aimed);
        WalkHit hit;
        double tau = 0.0;
        if (coherent) {
            tau = siddon_tau<EXACT, true>(g, q, dl, mu_lds + e * n_mat, tau_star, &hit);
        } else {
            double sl = 0.0;
            uint32_t ml = 0;
            if (siddon_locate(g, q, dl, mu_lds + e * n_mat, tau_star, sl, ml, tau)) {
                hit.found = sl >= 0.0 && tau_star < kInf;
                hit.s = sl;
                hit.m = ml;
                hit.last_end = sl;
                hit.last_m = ml;
            }
        }
        if (pass == 2 * K) {  // the exit walk
            ray.E = E;
            ray.w = w * exp(-tau);
            break;
        }
        if (!locate) {
            // optical depth ahead: draw the forced interaction depth
            if (!(tau > 0.0)) return false;
            pint = -expm1(-tau);
            tau_star = -log1p(-s.u((int)c.draw0 + 4 * k) * pint);
            continue;
        }
        const double sint = hit.found ? hit.s : hit.last_end;
        const uint32_t m = hit.found ? hit.m : hit.last_m;
#pragma unroll
        for (int i = 0; i < 3; ++i) q[i] = q[i] + sint * dl[i];
        const double mu_t = T[m * n_ebin + e];
        const double mu_r = T[plane + m * n_ebin + e];
        const double mu_c = T[2 * plane + m * n_ebin + e];
        if (!(mu_r + mu_c > 0.0)) return false;
        const double albedo = (mu_r + mu_c) / mu_t;
        const bool rayleigh = s.u((int)c.draw0 + 4 * k + 1) < mu_r / (mu_r + mu_c);
        double ct = 2.0 * s.u((int)c.draw0 + 4 * k + 2) - 1.0;
        const double phi = kTwoPi * s.u((int)c.draw0 + 4 * k + 3);
        double nd[3], dens_ratio = 4.0 * kPi;
        if (aimed && k == K - 1) {
            double tw[3], tl[3], ta[3], tb[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) tw[i] = c.par[5 + i] - c.pos[i];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                tl[i] = c.rot[3 * i] * tw[0] + c.rot[3 * i + 1] * tw[1] + c.rot[3 * i + 2] * tw[2];
                ta[i] = c.rot[3 * i] * c.par[8] + c.rot[3 * i + 1] * c.par[9] + c.rot[3 * i + 2] * c.par[10];
                tb[i] = c.rot[3 * i] * c.par[11] + c.rot[3 * i + 1] * c.par[12] + c.rot[3 * i + 2] * c.par[13];
            }
            const double sa = 2.0 * s.u((int)c.draw0 + 4 * k + 2) - 1.0;
            const double sb = 2.0 * s.u((int)c.draw0 + 4 * k + 3) - 1.0;
            double r[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) r[i] = (tl[i] + sa * ta[i] + sb * tb[i]) - q[i];
            const double dist2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const double dist = sqrt(dist2);
            const double nrm0 = ta[1] * tb[2] - ta[2] * tb[1], nrm1 = ta[2] * tb[0] - ta[0] * tb[2],
                         nrm2 = ta[0] * tb[1] - ta[1] * tb[0];
            const double area4 = sqrt(nrm0 * nrm0 + nrm1 * nrm1 + nrm2 * nrm2);
            if (!(dist > 0.0) || !(area4 > 0.0)) return false;
#pragma unroll
            for (int i = 0; i < 3; ++i) nd[i] = r[i] / dist;
            const double cosn = fabs(nd[0] * nrm0 + nd[1] * nrm1 + nd[2] * nrm2) / area4;
            if (!(cosn > 0.0)) return false;
            dens_ratio = (cosn * 4.0 * area4) / dist2;
            ct = dl[0] * nd[0] + dl[1] * nd[1] + dl[2] * nd[2];
        } else {
            double a0 = 0.0, a1 = 1.0;
            if (!(fabs(dl[1]) < 0.5)) {
                a0 = 1.0;
                a1 = 0.0;
            }
            // e1 = d x a with a = (a0, a1, 0)
            double e1[3] = {dl[1] * 0.0 - dl[2] * a1, dl[2] * a0 - dl[0] * 0.0, dl[0] * a1 - dl[1] * a0};
            const double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
#pragma unroll
            for (int i = 0; i < 3; ++i) e1[i] = e1[i] / n1;
            const double e2[3] = {dl[1] * e1[2] - dl[2] * e1[1], dl[2] * e1[0] - dl[0] * e1[2],
                                  dl[0] * e1[1] - dl[1] * e1[0]};
            const double sn = sqrt(1.0 - ct * ct);
            double sp, cp;
            sincos(phi, &sp, &cp);
#pragma unroll
            for (int i = 0; i < 3; ++i) nd[i] = ct * dl[i] + sn * (cp * e1[i] + sp * e2[i]);
        }
        const double st2 = 1.0 - ct * ct;
        double dens;
        if (rayleigh) {
            dens = 3.0 * (1.0 + ct * ct) / (16.0 * kPi);
        } else {
            const double kk = E / kMeC2Kev;
            const double rho = 1.0 / (1.0 + kk * (1.0 - ct));
            dens = rho * rho * (rho + 1.0 / rho - st2) / (4.0 * kPi * kn_f(kk));
            E = rho * E;
        }
        w = w * (pint * albedo * (dens * dens_ratio));
#pragma unroll
        for (int i = 0; i < 3; ++i) dl[i] = nd[i];
    }
    to_lab(c, q, dl, ray);
    return true;
}

// ---------------------------------------------------- fixed-step model ----
// The paper's own way through the voxel sample (section 3.3): fixed steps of
// length h, each reading the voxel that holds its end position and
// attenuating over its length.  The chord is the exact walk's; step j covers
// [a_in + (j-1) h, min(a_in + j h, a_out)] (the last step is clipped at the
// exit) and reads the voxel at u_in + j (h d / v) in voxel units (one fused
// multiply-add per axis), taken unclipped and clamped into the volume.  Both numbers come from j directly,
// with no running sum, so the steps are independent: kStepRound voxel loads
// are issued per round.  The optical depth is summed per material run as in
// the exact walk.  jmax (volume diagonal / h + 2, from the host) bounds every
// loop; a voxel index is clamped per axis, so every load is in range.
constexpr int kStepRound = 4;

__device__ __forceinline__ double step_tau(const PhantomGeo &g, const double q[3], const double dl[3], double h,
                                           int jmax, const double *__restrict__ mu_row) {
    double a_in = 0.0, a_out = kInf;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double lo_p = g.corner[i];
        const double hi_p = g.corner[i] + (double)g.n[i] * g.v;
        if (dl[i] == 0.0) {
            if (!(q[i] > lo_p && q[i] < hi_p)) return 0.0;
        } else {
            const double inv = 1.0 / dl[i];
            const double a0 = (lo_p - q[i]) * inv, a1 = (hi_p - q[i]) * inv;
            const double lo = a0 < a1 ? a0 : a1, hi = a0 < a1 ? a1 : a0;
            if (lo > a_in) a_in = lo;
            if (hi < a_out) a_out = hi;
        }
    }
    if (!(a_out > a_in)) return 0.0;
    double u0[3], du[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        u0[i] = ((q[i] + a_in * dl[i]) - g.corner[i]) / g.v;
        du[i] = (h * dl[i]) / g.v;
    }
    // this lane's step count: the first j with a_in + j h >= a_out
    // (a_in + j h is non-decreasing in j, so the fix-ups end at that j)
    int J = (int)fmin(fmax(ceil((a_out - a_in) / h), 1.0), (double)jmax);
    while (J > 1 && !(a_in + (double)(J - 1) * h < a_out)) --J;
    while (J < jmax && a_in + (double)J * h < a_out) ++J;

    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)g.vol, (short)0, (int)g.nvox, 0x00020000);
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    // voxel of step j: truncation then clamping at 0 equals floor then
    // clamping, for every value in int range.  The host admits the model
    // only for ny nz < 2^24, so the offset takes two 24-bit multiply-adds
    // (full rate) instead of 32-bit multiplies (quarter rate).
    auto voxel_of = [&](int j) -> uint32_t {
        const double dj = (double)j;
        int ix = (int)fma(dj, du[0], u0[0]);
        int iy = (int)fma(dj, du[1], u0[1]);
        int iz = (int)fma(dj, du[2], u0[2]);
        ix = clamp0_i32(ix, nx - 1);
        iy = clamp0_i32(iy, ny - 1);
        iz = clamp0_i32(iz, nz - 1);
        return mad_u24(nx, mad_u24(ny, iz, iy), ix);
    };
    uint32_t run_m = load_voxel(rs, voxel_of(1));
    double a_start = a_in, tau = 0.0;
    const int max_rounds = (jmax + kStepRound - 1) / kStepRound + 1;
    int j0 = 2;
    for (int round = 0; round < max_rounds; ++round, j0 += kStepRound) {
        if (__builtin_amdgcn_ballot_w64(j0 <= J) == 0) break;
        uint32_t m[kStepRound];
#pragma unroll
        for (int k = 0; k < kStepRound; ++k) m[k] = load_voxel(rs, voxel_of(j0 + k));
#pragma unroll
        for (int k = 0; k < kStepRound; ++k) {
            // a step past this lane's last one starts at or beyond a_out:
            // clamped there, it closes the open run exactly as the final
            // term would and adds zero-length runs after it, so no per-step
            // j <= J test is needed
            if (m[k] != run_m) {
                const double a = min_f64(a_in + (double)(j0 + k - 1) * h, a_out);
                tau = fma(mu_row[run_m], a - a_start, tau);
                a_start = a;
                run_m = m[k];
            }
        }
    }
    return fma(mu_row[run_m], a_out - a_start, tau);
}

// ------------------------------------------------------------- mirror ----
__device__ __forceinline__ bool comp_mirror(const DevComp &c, Ray &ray) {
    // aux: 0 Cy, 1 Cz, 2 uy, 3 uz, 4 vy, 5 vz, 6 1/a^2, 7 1/b^2,
    //      8 sin t0, 9 cos t0, 10 length/2, 11 width/2, 12 node step
    double q[3], dl[3];
    to_local(c, ray, q, dl);
    const double Cy = c.aux[0], Cz = c.aux[1], uy = c.aux[2], uz = c.aux[3], vy = c.aux[4], vz = c.aux[5];
    const double ia2 = c.aux[6], ib2 = c.aux[7];
    double gy = q[1] - Cy, gz = q[2] - Cz;
    double s0 = gy * uy + gz * uz, n0 = gy * vy + gz * vz;
    double ds = dl[1] * uy + dl[2] * uz, dn = dl[1] * vy + dl[2] * vz;
    double A = ds * ds * ia2 + dn * dn * ib2;
    double B = 2.0 * (s0 * ds * ia2 + n0 * dn * ib2);
    double C = s0 * s0 * ia2 + n0 * n0 * ib2 - 1.0;
    double disc = B * B - 4.0 * A * C;
    if (!(disc >= 0.0)) return false;
    double t = (-B + sqrt(disc)) / (2.0 * A);
    if (!(t > 0.0)) return false;
    double X[3] = {q[0] + t * dl[0], q[1] + t * dl[1], q[2] + t * dl[2]};
    double along = X[1] * c.aux[8] + X[2] * c.aux[9];
    if (!(fabs(X[0]) <= c.aux[11] && fabs(along) <= c.aux[10])) return false;
    double hy = X[1] - Cy, hz = X[2] - Cz;
    double hs = (hy * uy + hz * uz) * ia2, hn = (hy * vy + hz * vz) * ib2;
    double N1 = hs * uy + hn * vy, N2 = hs * uz + hn * vz;
    double nn = sqrt(0.0 * 0.0 + N1 * N1 + N2 * N2);
    N1 = N1 / nn;
    N2 = N2 / nn;
    double dd = dl[0] * 0.0 + dl[1] * N1 + dl[2] * N2;
    if (dd > 0.0) {
        N1 = -N1;
        N2 = -N2;
        dd = -dd;
    }
    double theta = asin(-dd);
    const double *tab = (const double *)c.data0;
    const int64_t nt = (int64_t)c.n0;
    double R = 0.0;
    double uu = theta / c.aux[12];
    if (uu <= (double)(nt - 1)) {
        int64_t k = (int64_t)floor(uu);
        if (k > nt - 2) k = nt - 2;
        double f = uu - (double)k;
        R = tab[k] * (1.0 - f) + tab[k + 1] * f;
    }
    double out[3] = {dl[0] - 2.0 * dd * 0.0, dl[1] - 2.0 * dd * N1, dl[2] - 2.0 * dd * N2};
    ray.w = ray.w * R;
    to_lab(c, X, out, ray);
    return true;
}

// --------------------------------------------------------- crystals ----
__device__ __forceinline__ double darwin(double x) {
    double ax = fabs(x);
    if (ax <= 1.0) return 1.0;
    double den = ax + sqrt(ax * ax - 1.0);
    return 1.0 / (den * den);
}

__device__ __forceinline__ bool bragg(double q[3], double dl[3], const double P[3], const double N[3],
                                      double two_d, double half_w, double E, double &R) {
    double dn = dl[0] * N[0] + dl[1] * N[1] + dl[2] * N[2];
    if (!(dn < 0.0)) return false;
    double rel0 = q[0] - P[0], rel1 = q[1] - P[1], rel2 = q[2] - P[2];
    double t = -(rel0 * N[0] + rel1 * N[1] + rel2 * N[2]) / dn;
    if (!(t >= 0.0)) return false;
#pragma unroll
    for (int i = 0; i < 3; ++i) q[i] = q[i] + t * dl[i];
    double th_in = asin(-dn);
    double th_b = asin(kHc / (two_d * E));
    R = darwin((th_in - th_b) / half_w);
#pragma unroll
    for (int i = 0; i < 3; ++i) dl[i] = dl[i] - 2.0 * dn * N[i];
    return true;
}

__device__ __forceinline__ bool comp_dcm(const DevComp &c, Ray &ray) {
    // aux: 0..2 n1, 3..5 n2 = -n1, 6..8 crystal-2 point, 9 2d, 10 width/2
    double q[3], dl[3], R1, R2;
    to_local(c, ray, q, dl);
    const double P1[3] = {0.0, 0.0, 0.0};
    if (!bragg(q, dl, P1, c.aux + 0, c.aux[9], c.aux[10], ray.E, R1)) return false;
    if (!bragg(q, dl, c.aux + 6, c.aux + 3, c.aux[9], c.aux[10], ray.E, R2)) return false;
    ray.w = ray.w * R1;
    ray.w = ray.w * R2;
    to_lab(c, q, dl, ray);
    return true;
}

// ------------------------------------------------------------- powder ----
__device__ __forceinline__ bool comp_powder(const DevComp &c, Stream &s, Ray &ray) {
    double q[3], dl[3];
    to_local(c, ray, q, dl);
    if (!plane_z0(q, dl)) return false;
    if (!(fabs(q[0]) <= c.aux[0] && fabs(q[1]) <= c.aux[1])) return false;
    const double *dsp = (const double *)c.data0;
    const int64_t nd = (int64_t)c.n0;
    int64_t j = (int64_t)floor((double)nd * s.u((int)c.draw0));
    if (j > nd - 1) j = nd - 1;
    double lambda = kHc / ray.E;
    double sarg = lambda / (2.0 * dsp[j]);
    if (!(sarg <= 1.0)) return false;
    double tth = 2.0 * asin(sarg);
    double eta = kTwoPi * s.u((int)c.draw0 + 1);
    double e1x = -dl[2], e1z = dl[0];
    double n1 = sqrt(e1x * e1x + 0.0 * 0.0 + e1z * e1z);
    e1x = e1x / n1;
    e1z = e1z / n1;
    const double e1y = 0.0;
    double e2x = dl[1] * e1z - dl[2] * e1y;
    double e2y = dl[2] * e1x - dl[0] * e1z;
    double e2z = dl[0] * e1y - dl[1] * e1x;
    double st, ct, se, ce;
    sincos(tth, &st, &ct);
    sincos(eta, &se, &ce);
    double out[3] = {ct * dl[0] + st * (ce * e1x + se * e2x), ct * dl[1] + st * (ce * e1y + se * e2y),
                     ct * dl[2] + st * (ce * e1z + se * e2z)};
    to_lab(c, q, out, ray);
    return true;
}

// ----------------------------------------------------------- monitors ----
__device__ __forceinline__ int64_t bin_of(double x, double lo, double scale, uint32_t n) {
    double f = floor((x - lo) * scale);
    if (!(f >= 0.0 && f < (double)n)) return -1;
    return (int64_t)f;
}

// returns false if the ray cannot reach the plane; bin = -1 outside
__device__ __forceinline__ bool comp_detector(const DevComp &c, Ray &ray, int64_t &bin) {
    // aux: 0 nx/(xmax-xmin), 1 ny/(ymax-ymin), 2 ne/(emax-emin)
    double q[3], dl[3];
    to_local(c, ray, q, dl);
    if (!plane_z0(q, dl)) return false;
    double ev = (c.flags & 1u) ? kHc / ray.E : ray.E;
    int64_t ix = bin_of(q[0], c.par[0], c.aux[0], c.dims[0]);
    int64_t iy = bin_of(q[1], c.par[2], c.aux[1], c.dims[1]);
    int64_t ie = bin_of(ev, c.par[4], c.aux[2], c.dims[2]);
    bin = (ix >= 0 && iy >= 0 && ie >= 0) ? (iy * (int64_t)c.dims[0] + ix) * (int64_t)c.dims[2] + ie : -1;
    to_lab(c, q, dl, ray);
    return true;
}

}  // namespace mxr
