/*
 * mxr.h -- C ABI of the MI355X (gfx950) Monte Carlo X-ray ray tracer.
 *
 * The library carries independent photon packets ("rays") from a source
 * through a sequential list of components into energy/position-resolving
 * monitors, one GPU lane per ray (paper, section 2: an instrument is a
 * sequential list of components; rays are generated at the source and
 * propagated through the list; section 2.2: the problem is embarrassingly
 * parallel over rays; monitor arrays are the only shared state).
 *
 * Conventions
 *   - Lengths in mm, energies in keV, angles in rad, attenuation in 1/cm.
 *   - Every component has a frame: local = rot * (lab - pos), rot row major.
 *   - All array arguments named "device" are caller-owned device pointers
 *     (hipMalloc or torch allocations on the device that is current when the
 *     instrument is created).  The library never frees caller memory.
 *   - Calls validate synchronously and execute asynchronously on the HIP
 *     stream passed in (NULL = the null stream); the caller synchronises.
 *   - Every function returns an mxr_status; a negative value is an error and
 *     mxr_last_error() then holds a message.  No exception or abort crosses
 *     the ABI.
 *   - Results are a pure function of (instrument, seed, n_total, purpose,
 *     job, ray id): rays [a, b) of an n_total-ray run are the same rays in
 *     any chunking, launch shape or thread layout.
 *
 * Random numbers (paper, section 2.2.2, a per-thread generator): ray r of a
 * run draws from Philox4x32-10 (Salmon et al., SC'11) with key (seed low,
 * seed high) and counter (j, r low, r high, purpose << 24 | job); block j
 * gives uniforms 2j (words 1:0) and 2j+1 (words 3:2) as
 * ((w >> 12) + 1/2) * 2^-52.  Components draw in instrument order; the
 * number of draws per component type is listed below.
 *
 * Threads: one instrument handle per host thread, or external locking.
 */
#ifndef MXR_H
#define MXR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MXR_ABI_VERSION 1u
#define MXR_MAX_COMPONENTS 16u
#define MXR_MAX_DETECTORS 4u

typedef enum {
    MXR_OK = 0,
    MXR_E_INVALID = -1,     /* malformed argument or descriptor */
    MXR_E_UNSUPPORTED = -2, /* valid but outside what the library supports */
    MXR_E_NOMEM = -3,       /* device allocation failed */
    MXR_E_HIP = -4,         /* a HIP runtime call failed */
    MXR_E_STATE = -5        /* wrong device current, or handle misuse */
} mxr_status;

/* Component types and their parameter slots (par[]), data arrays
 * (data[], element counts in data_len[]) and dims[].
 *
 * MXR_SRC_RECT_CONE (5 draws) -- square emitter in the local plane z = 0,
 *   direction uniform in solid angle inside a cone about +z, energy flat,
 *   weight 1 (paper, section 3.1: point/flat sources emitting a cone).
 *   par: 0 width x, 1 width y, 2 cone half-angle, 3 E min, 4 E max.
 * MXR_SRC_CONE_BEAM (3 draws) -- point source at the local origin, direction
 *   uniform in solid angle inside a cone about +z, stratified over
 *   G x G equal-area cells (concentric square-to-disk map, Shirley & Chiu
 *   1997; G is reduced to the largest value with G^2 <= n_total), energy
 *   flat on [E min, E max] with the tube spectrum carried in the weight
 *   w0 = (E max - E min) S(E) (n_total / G^2) / n_cell (paper, section 3.3:
 *   a tube source illuminating the whole detector).  S is a Kramers
 *   continuum (E0 - E)/E with fraction f_c plus two Gaussian lines.
 *   par: 0 half-angle, 1 E min, 2 E max, 3 E0, 4 f_c, 5 E line 1,
 *   6 f line 1, 7 E line 2, 8 f line 2, 9 line sigma.  dims: 0 G.
 * MXR_SRC_GAUSSIAN (5 draws) -- Gaussian position and angle in both planes,
 *   energy flat within a relative half-width (paper, section 3.2, an
 *   undulator source).  par: 0 sigma x, 1 sigma y, 2 sigma x', 3 sigma y',
 *   4 E0, 5 relative half-width.
 * MXR_SLIT -- aperture in the local plane z = 0; edges pass; rays that
 *   cannot reach the plane or miss the opening are absorbed.
 *   par: 0 width, 1 height; flags bit 0 = circular with par 2 = radius.
 * MXR_BOX -- homogeneous box |x|<hx, |y|<hy, |z|<hz, Beer-Lambert weight
 *   factor exp(-mu(E) L / 10) with mu = a / E^3 + b (1/cm).
 *   par: 0 hx, 1 hy, 2 hz, 3 a, 4 b.
 * MXR_PHANTOM -- voxel volume centred on the local origin (paper, section
 *   3.3, a 3-D segmented sample of material indices), exact path lengths by
 *   Siddon-type traversal, weight factor exp(-sum mu_m(E) l / 10).
 *   data[0] (device, uint8, nx*ny*nz): material id of voxel (i, j, k) at
 *   i + nx (j + ny k).  data[1] (device, double, n_mat * n_ebin): mu in 1/cm,
 *   material-major, energy bins uniform on [table E min, table E max),
 *   looked up piecewise constant.  par: 0 voxel edge, 1 table E min,
 *   2 table E max.  dims: 0 nx, 1 ny, 2 nz, 3 n_mat (1..16), n_ebin =
 *   data_len[1] / n_mat (1..256).  A volume holding an id >= n_mat is
 *   rejected at create (the volume is scanned once on the device).  At most
 *   one phantom per instrument.
 * MXR_MIRROR_ELLIPTIC -- elliptic-cylinder mirror; local origin at the pole,
 *   z along the incoming axis, y to the reflected side; foci at (0,0,-p)
 *   and q (0, sin 2t0, cos 2t0).  Specular reflection, weight times the
 *   reflectivity at the glancing angle by linear interpolation of data[0]
 *   (device, double, n >= 2 nodes on [0, t max]), zero beyond; rays missing
 *   the length x width surface are absorbed.
 *   par: 0 p, 1 q, 2 t0, 3 length, 4 width, 5 t max.
 * MXR_DCM -- two parallel crystals; local origin at crystal 1, z along the
 *   incoming axis, y up; crystal 1 normal (0, cos tc, -sin tc), crystal 2
 *   the parallel plane through g n1.  Each bounce reflects specularly with
 *   the Darwin-curve weight of (theta_in - asin(hc / 2dE)) / (width / 2).
 *   par: 0 d-spacing (Angstrom), 1 tc, 2 Darwin full width, 3 gap g.
 * MXR_POWDER (2 draws) -- thin plate in the local plane z = 0; a hit picks
 *   one of data[0] (device, double, d-spacings in Angstrom) uniformly and
 *   turns the ray onto its Debye-Scherrer cone 2 asin(lambda / 2d) at a
 *   uniform azimuth; misses are absorbed.  par: 0 width, 1 height.
 * MXR_DETECTOR -- ideal monitor in the local plane z = 0 with half-open
 *   bins (x, y, E) (flags bit 0: wavelength hc/E instead of E); tally index
 *   (iy * nx + ix) * ne + ie.  Monitors do not absorb; rays that cannot
 *   reach the plane are absorbed.  par: 0 x min, 1 x max, 2 y min, 3 y max,
 *   4 E min, 5 E max.  dims: 0 nx, 1 ny, 2 ne.
 */
typedef enum {
    MXR_SRC_RECT_CONE = 0,
    MXR_SRC_CONE_BEAM = 1,
    MXR_SRC_GAUSSIAN = 2,
    MXR_SLIT = 3,
    MXR_BOX = 4,
    MXR_PHANTOM = 5,
    MXR_MIRROR_ELLIPTIC = 6,
    MXR_DCM = 7,
    MXR_POWDER = 8,
    MXR_DETECTOR = 9
} mxr_component_type;

typedef struct {
    uint32_t type;
    uint32_t flags;
    double pos[3];
    double rot[9];
    double par[16];
    const void *data[2];
    uint64_t data_len[2];
    uint32_t dims[4];
} mxr_component_desc;

/* The first component must be a source and no other may be one. */
typedef struct {
    uint32_t abi_version; /* MXR_ABI_VERSION */
    uint32_t n_components;
    const mxr_component_desc *components;
} mxr_instrument_desc;

/* One monitor's histogram: three device arrays of n_bins entries, added to
 * (+=), so the caller zeroes them before the first run. */
typedef struct {
    uint64_t *count;
    double *sum_w;
    double *sum_w2;
    uint64_t n_bins;
} mxr_tally;

/* Final per-ray state (device arrays of n entries each).  status: 1 left
 * the instrument, 2 absorbed; dead_at: index of the absorbing component or
 * -1; bin: tally index at the last monitor the ray hit, or -1.  An absorbed
 * ray reports its state on entering the absorbing component. */
typedef struct {
    double *x, *y, *z, *dx, *dy, *dz, *E, *w;
    int32_t *status;
    int32_t *dead_at;
    int64_t *bin;
} mxr_ray_soa;

typedef struct mxr_instrument mxr_instrument;

/* Returns MXR_ABI_VERSION. */
uint32_t mxr_abi_version(void);

/* Message of the last error on this host thread; valid until the next call
 * on this thread.  Never NULL. */
const char *mxr_last_error(void);

/* Validates desc, derives per-component constants and copies them to the
 * current device (one small allocation, owned by the handle).  The data
 * arrays are referenced, not copied: they must stay alive and unchanged
 * while the handle is used.  Errors: MXR_E_INVALID (null pointers, wrong
 * version, bad component order, non-finite or out-of-range parameters),
 * MXR_E_UNSUPPORTED (limits above), MXR_E_NOMEM, MXR_E_HIP. */
mxr_status mxr_instrument_create(const mxr_instrument_desc *desc, mxr_instrument **out);

/* Frees the handle and its device copy (synchronises the device first).
 * NULL is accepted. */
void mxr_instrument_destroy(mxr_instrument *ins);

/* Traces rays [first_ray, first_ray + n_rays) of an n_total-ray run and
 * adds their histograms into tallies[0 .. n_tallies) (one per monitor, in
 * instrument order, n_bins = nx*ny*ne each).  ledger (nullable, device,
 * 4 * n_components + 1 doubles, added to): per component k, [4k] weight
 * entering (for the source: emitted), [4k+1] weight absorbed at k,
 * [4k+2] weight removed by attenuation at k, [4k+3] weight tallied at k;
 * [4K] weight leaving the instrument.  Errors: MXR_E_INVALID (null handle
 * or tallies, tally count or size mismatch, first_ray + n_rays > n_total,
 * n_total * G^2 >= 2^64), MXR_E_STATE (another device current), MXR_E_HIP. */
mxr_status mxr_run(mxr_instrument *ins, uint64_t first_ray, uint64_t n_rays, uint64_t n_total, uint64_t seed,
                   uint32_t purpose, uint32_t job, const mxr_tally *tallies, uint32_t n_tallies, double *ledger,
                   void *hip_stream);

/* Traces the listed rays (ray_ids: device, n entries, each < n_total) of an
 * n_total-ray run and writes their final states into out (no tallies).
 * The same per-ray code as mxr_run.  Errors as mxr_run. */
mxr_status mxr_trace_rays(mxr_instrument *ins, const uint64_t *ray_ids, uint64_t n, uint64_t n_total,
                          uint64_t seed, uint32_t purpose, uint32_t job, const mxr_ray_soa *out,
                          void *hip_stream);

/* ------------------------------------------------------------------------
 * Batched runs: many projections (angles) of many phantoms in one launch.
 *
 * A CT acquisition repeats one instrument for every projection angle of
 * every sample (paper, section 3.3: a simulation per imaged line and
 * rotational position; section 5.1: hundreds of projections per data set).
 * A batch traces all jobs in one launch over a table of (job, ray range)
 * tiles, longest jobs first, so phantoms of very different size share the
 * GPU without one launch per job: either one work-group per tile (grid
 * form) or persistent work-groups that pop tiles from a device counter.  The
 * launch is captured once into a HIP graph and replayed by every
 * mxr_batch_run.
 */
typedef struct mxr_batch mxr_batch;

/* One job: trace rays [0, n_rays) of an n_rays-ray run of `instrument` with
 * the given seed and RNG job field, adding into `tallies` (one per monitor,
 * device arrays, as in mxr_run).  The result equals
 * mxr_run(instrument, 0, n_rays, n_rays, seed, 0, job, tallies, ...) up to
 * the order of the atomic additions. */
typedef struct {
    const mxr_instrument *instrument;
    uint64_t n_rays;
    uint64_t seed;
    uint32_t job; /* < 2^24 */
    mxr_tally tallies[MXR_MAX_DETECTORS];
} mxr_batch_job;

/* Launch shape of a batch.  It changes the order in which tiles are traced,
 * never the set of rays or their results. */
typedef struct {
    /* 0: grid form -- one work-group per tile of 256 rays over a 2-D grid of
     *    the whole batch, no loops, balanced by the hardware dispatcher;
     * 1..8: persistent form -- that many work-groups per compute unit pop
     *    tiles from a device counter until it passes the last tile. */
    uint32_t groups_per_cu;
    uint32_t tile_rays; /* persistent form: rays per tile, a multiple of 256 in
                           [256, 2^24] (0 = 65536); grid form: 256 (0 = 256) */
} mxr_batch_schedule;

/* Validates the jobs (all instruments on the current device with the same
 * component types in the same order; tally sizes; n_rays >= 1) and builds
 * the job and tile tables on the device (owned by the handle).  schedule is
 * nullable (grid form until tuned).  The
 * instruments and tallies must outlive the handle.  Errors: MXR_E_INVALID,
 * MXR_E_UNSUPPORTED (more than 2^31 tiles), MXR_E_NOMEM, MXR_E_HIP,
 * MXR_E_STATE. */
mxr_status mxr_batch_create(const mxr_batch_job *jobs, uint32_t n_jobs, const mxr_batch_schedule *schedule,
                            mxr_batch **out);

/* Traces every job once (tallies added to).  The first call on a handle
 * captures the launch into a HIP graph; later calls replay it.  Asynchronous
 * on hip_stream.  Calls on one handle must not overlap.  Errors: MXR_E_HIP,
 * MXR_E_STATE. */
mxr_status mxr_batch_run(mxr_batch *batch, void *hip_stream);

/* Current launch shape. */
mxr_status mxr_batch_get_schedule(const mxr_batch *batch, mxr_batch_schedule *out);

/* Replaces the launch shape (the captured graph is rebuilt on the next run).
 * Errors: MXR_E_INVALID for an out-of-range shape. */
mxr_status mxr_batch_set_schedule(mxr_batch *batch, const mxr_batch_schedule *schedule);

/* Synchronises the device, frees the handle and its device tables.  NULL is
 * accepted. */
void mxr_batch_destroy(mxr_batch *batch);

/* Autotuner: times candidate launch shapes (the grid form, and persistent
 * forms of 2/4/6/8 groups per CU x 16K/64K/256K-ray tiles) on
 * the batch with every job's ray count scaled by rays_fraction (0 < f <= 1),
 * keeps the fastest and records it under a key describing the batch (its
 * component chain, job count, total rays and work estimate) in the text
 * file cache_path (nullable: no cache), which later calls consult before
 * timing anything.  The chosen shape is set on the batch and returned in
 * out (nullable).  Timing runs ADD into the jobs' tallies: zero them before
 * the production run.  Synchronous.  Errors: MXR_E_INVALID, MXR_E_HIP. */
mxr_status mxr_batch_autotune(mxr_batch *batch, double rays_fraction, const char *cache_path,
                              mxr_batch_schedule *out);

#ifdef __cplusplus
}
#endif

#endif /* MXR_H */
