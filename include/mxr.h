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

#define MXR_ABI_VERSION 2u
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
 *   1997; G is reduced to the largest value with 16 G^2 <= n_total, 1 if
 *   none, so that a cell holds at least 16 rays), energy
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
 *   one phantom per instrument.  flags bit 0: the paper's fixed-step model
 *   instead (section 3.3: the ray advances by a fixed increment, the voxel
 *   holding the new position gives the material, the weight is attenuated
 *   over the increment) with par 3 = step length h (mm, > 0; the paper's
 *   default is a third of the voxel edge): step j covers [a_in + (j-1) h,
 *   min(a_in + j h, a_out)] of the chord and reads the voxel holding
 *   u_in + j h d / v (voxel units, j h d / v + u_in as one fused
 *   multiply-add per axis, clamped into the volume).  MXR_E_UNSUPPORTED
 *   when the longest chord needs more than 2^26 steps or ny * nz >= 2^24.
 *   flags bit 1: scattering (section 3.3: the sample models absorption and
 *   scattering): the run traces the photons scattered exactly K = par 4
 *   (1..3) times in the volume instead of the uncollided ones; the image is
 *   the sum of the order-0 (plain) and the order-K runs.  data[1] then holds
 *   three channels, 3 * n_mat * n_ebin doubles (total attenuation, Rayleigh,
 *   Compton, each material-major; n_ebin = data_len[1] / (3 n_mat)), with
 *   Rayleigh + Compton <= total expected of the caller.  Each interaction is
 *   forced on the chord ahead: depth -log(1 - u (1 - e^-tau)), weight times
 *   1 - e^-tau, the scatter albedo (mu_R + mu_C) / mu_tot, and the angular
 *   density (Rayleigh: Thomson; Compton: Klein-Nishina for free electrons,
 *   E' = E / (1 + (E / 510.99895 keV)(1 - cos))) over the sampling density:
 *   directions uniform on the sphere, or, with flags bit 2, the last
 *   interaction aimed at a point drawn uniformly on the rectangle with
 *   centre par 5..7 and half-axes par 8..10, par 11..13 (lab frame; for a
 *   monitor of that extent).  Four uniforms per interaction.  The ray leaves
 *   the component at its last interaction point, attenuated along its new
 *   direction at its new energy; a chord without attenuating or scattering
 *   material absorbs it.  Bits 0 and 1 exclude each other; bit 2 needs bit
 *   1; other bits are rejected.
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
 * MXR_LENS_CRL -- compound refractive lens (paper, section 3.2: a stack of
 *   double-sided parabolic beryllium lenses): N bi-concave lenses on the
 *   local z axis, lens k centred at (k - (N-1)/2) pitch, its material between
 *   the paraboloids z = c_k - w/2 - rho^2/2R and z = c_k + w/2 + rho^2/2R
 *   inside the aperture radius (the frame beyond it is opaque: a surface
 *   met outside it absorbs the ray, as does a surface the ray cannot reach
 *   moving forward, or total reflection).  Refraction by Snell's law with
 *   n = 1 - delta, delta(E) = delta_ref (E_ref / E)^2; weight times
 *   exp(-mu(E) L / 10) with L the path inside the material (mm) and
 *   mu = a / E^3 + b (1/cm).  par: 0 R, 1 N (integer, 1..1024), 2 on-axis
 *   thickness w, 3 pitch (>= w + r_a^2 / R), 4 aperture radius r_a,
 *   5 delta_ref (0 <= delta_ref < 0.5), 6 E_ref, 7 a, 8 b.
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
    MXR_DETECTOR = 9,
    MXR_LENS_CRL = 10
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

/* Returns MXR_ABI_VERSION (library bookkeeping; no passage of the paper). */
uint32_t mxr_abi_version(void);

/* Message of the last error on this host thread; valid until the next call
 * on this thread.  Never NULL.  (Library bookkeeping.) */
const char *mxr_last_error(void);

/* Validates desc, derives per-component constants and copies them to the
 * current device (small allocations owned by the handle: the constants and,
 * for a phantom, a copy of its attenuation table per mm and energy-major,
 * the form the kernels stage in LDS): the
 * instrument as a sequence of components placed in the lab frame (paper,
 * section 2.1), its component data held in structs and made available on
 * the device once (section 2.2.2).  The data
 * arrays are referenced, not copied: they must stay alive and unchanged
 * while the handle is used.  Errors: MXR_E_INVALID (null pointers, wrong
 * version, bad component order, non-finite or out-of-range parameters),
 * MXR_E_UNSUPPORTED (limits above), MXR_E_NOMEM, MXR_E_HIP. */
mxr_status mxr_instrument_create(const mxr_instrument_desc *desc, mxr_instrument **out);

/* Frees the handle and its device copy (synchronises the device first).
 * NULL is accepted.  (Library bookkeeping.) */
void mxr_instrument_destroy(mxr_instrument *ins);

/* Launch shape of an instrument's plain runs (mxr_run without a ledger or a
 * proposal).  It changes how rays are mapped onto the device, never which
 * rays are traced or their results (per bin up to the order of the atomic
 * additions): the rays are independent (paper, section 2.2), so their
 * mapping onto threads is free.
 *   occupancy  waves per SIMD the run kernel is compiled for: 0 the chain's
 *              own, or 4, 6, 8 (fixed chains only; others ignore it)
 *   compact    1: chains with a crop right after the source run the
 *              survivor-compacting kernel; 0: one ray per lane
 *   rounds     compacting kernel: 64-ray rounds per wave, 1..64 (0 = 64)
 *   xcd_order  which 256-ray tiles each of the eight XCDs traces: 0, the
 *              i-th XCD the i-th eighth of the ray range; 1, launch order;
 *              2, runs of 64 consecutive tiles dealt to the XCDs in turn.
 *              The default is 1 for instruments with a phantom (the
 *              stratified source sends each block of ray ids through one
 *              band of the cone, so order 0 leaves XCDs idle where the
 *              bands' paths cost unequally) and 0 otherwise (neighbouring
 *              rays keep their tally updates in one XCD's L2).  Runs with a
 *              ledger, a ray trace, a proposal or hit collection use the
 *              default. */
typedef struct {
    uint32_t occupancy;
    uint32_t compact;
    uint32_t rounds;
    uint32_t xcd_order;
} mxr_launch_shape;

/* Traces rays [first_ray, first_ray + n_rays) of an n_total-ray run and
 * adds their histograms into tallies[0 .. n_tallies) (one per monitor, in
 * instrument order, n_bins = nx*ny*ne each).  The method of the paper:
 * independent rays, each carried from the source through every component
 * into the monitors (Introduction; section 2.2), the monitor arrays updated
 * atomically (section 2.2.2), a run split into ray ranges as the MPI
 * scatter-gather splits it (section 2.2.1).  ledger (nullable, device,
 * 4 * n_components + 1 doubles, added to): per component k, [4k] weight
 * entering (for the source: emitted), [4k+1] weight absorbed at k,
 * [4k+2] weight removed by attenuation at k, [4k+3] weight tallied at k;
 * [4K] weight leaving the instrument.  Errors: MXR_E_INVALID (null handle
 * or tallies, tally count or size mismatch, first_ray + n_rays > n_total,
 * n_total G^2 + G^2 - 1 >= 2^64), MXR_E_STATE (another device current), MXR_E_HIP. */
mxr_status mxr_run(mxr_instrument *ins, uint64_t first_ray, uint64_t n_rays, uint64_t n_total, uint64_t seed,
                   uint32_t purpose, uint32_t job, const mxr_tally *tallies, uint32_t n_tallies, double *ledger,
                   void *hip_stream);

/* Traces the listed rays (ray_ids: device, n entries, each < n_total) of an
 * n_total-ray run and writes their final states into out (no tallies): the
 * particle state of section 2.2.2 (position, wavevector as direction and
 * energy, weight) at the end of each ray.  The same per-ray code as
 * mxr_run.  Errors as mxr_run. */
mxr_status mxr_trace_rays(mxr_instrument *ins, const uint64_t *ray_ids, uint64_t n, uint64_t n_total,
                          uint64_t seed, uint32_t purpose, uint32_t job, const mxr_ray_soa *out,
                          void *hip_stream);

/* Current launch shape of the instrument's plain runs (see
 * mxr_autotune_instrument). */
mxr_status mxr_get_launch_shape(const mxr_instrument *ins, mxr_launch_shape *out);

/* Sets the launch shape (validated: occupancy in {0, 4, 6, 8}, compact in
 * {0, 1}, rounds <= 64, xcd_order in {0, 1, 2}).  Errors: MXR_E_INVALID. */
mxr_status mxr_set_launch_shape(mxr_instrument *ins, const mxr_launch_shape *shape);

/* Autotuner of an instrument's plain runs (paper, section 2.2: the
 * simulation is parallel over rays, so the mapping of rays onto the device
 * is free; the kernels' occupancy and ray order are the levers measured
 * here): times each candidate shape -- occupancy 0/4/6/8 for fixed chains,
 * both XCD ray orders, and for chains with a crop after the source the
 * compacting kernel at 64 or 16 rounds or none -- on rays [0, n) of an
 * n_total-ray run, n = max(1, rays_fraction n_total), after one untimed run
 * each; keeps the fastest and records it under a key of the instrument
 * (component chain, exactness of the phantom's planes, phantom and monitor
 * sizes, the run size's power of two) in the text file cache_path
 * (nullable), which later calls consult before timing anything.  The chosen
 * shape is set on the instrument and returned in out (nullable).  The
 * timing runs ADD into tallies: zero them before the production run.
 * Synchronous.  Errors: as mxr_run, MXR_E_INVALID for rays_fraction outside
 * (0, 1]. */
mxr_status mxr_autotune_instrument(mxr_instrument *ins, uint64_t n_total, double rays_fraction, const mxr_tally *tallies,
                                   uint32_t n_tallies, const char *cache_path, mxr_launch_shape *out);

/* ------------------------------------------------------------------------
 * Importance sampling of the cone-beam source by a learned proposal.
 *
 * The Monte Carlo weight a ray carries (paper, section 2.2.2: the particle
 * state includes a statistical weight) lets rays be drawn from any density
 * q that covers the physical one p, each weighted by p/q, without bias.  The
 * proposal is a defensive mixture q = alpha q_plain + (1 - alpha) q_gmm over
 * y = (u, v, E), u = dx/dz and v = dy/dz in the source frame:
 *   q_plain  the plain source (uniform in solid angle inside the cone,
 *            uniform energy);
 *   q_gmm    8 diagonal Gaussians truncated to the box
 *            [-tan a, tan a]^2 x [emin, emax] (a the cone half-angle), with
 *            density sum_k pi_k prod_d N(y_d; mu_kd, sigma_kd) / sum_k pi_k Z_k,
 *            Z_k the box mass of component k.
 * Rays are drawn as a stratified deterministic mixture: the n_total ray ids
 * of a run are split into contiguous ranges, [0, B0) for the plain source
 * (B0 = round(alpha n_total)) and one per component, sized by the rounded
 * running sums of the box masses pi_k Z_k.  Within its range a ray's first
 * two uniforms are stratified over G x G cells (G the source's strata,
 * reduced so 16 G^2 <= the range size) exactly like the plain source; the plain
 * branch maps them to the cone with the concentric map and draws E from the
 * third uniform, a component inverts a truncated normal per coordinate (u,
 * v from the stratified pair, E from the third uniform).  The ray's weight is
 * p(y) / sum_b (n_b / n_total) q_b(y) times the cell factor (n_b / G^2) /
 * n_cell: the balance heuristic of multiple importance sampling, unbiased
 * for any split.  A draw outside the cone is absorbed at the source with
 * weight 0.  The source still draws 3 uniforms per ray. */

/* Makes later mxr_run / mxr_trace_rays / mxr_collect calls on this
 * instrument draw its cone-beam source from the proposal.  gmm: DEVICE array of 56 doubles, per component
 * (pi, mu_u, mu_v, mu_E, sigma_u, sigma_v, sigma_E); pi >= 0 (need not sum
 * to 1), sigma > 0; it is copied (synchronously, after the device is idle),
 * so it may be freed afterwards.  alpha in [0, 1].  gmm NULL switches the
 * proposal off.  Errors: MXR_E_INVALID (values), MXR_E_UNSUPPORTED (the
 * first component is not a cone-beam source), MXR_E_STATE, MXR_E_NOMEM,
 * MXR_E_HIP. */
mxr_status mxr_proposal_set(mxr_instrument *ins, const double *gmm, double alpha);

/* The box of the proposal coordinates of the instrument's cone-beam source
 * (host arrays of 3): lo = (-tan a, -tan a, E min), hi = (tan a, tan a,
 * E max), a the cone half-angle; the mixture head and the training loss
 * below take it.  Errors: MXR_E_INVALID (null pointers), MXR_E_UNSUPPORTED
 * (the first component is not a cone-beam source). */
mxr_status mxr_proposal_box(const mxr_instrument *ins, double lo[3], double hi[3]);

/* Rows of training data: one per ray that reaches the monitor.  All arrays
 * are DEVICE arrays of `capacity` rows; *count (device) is advanced by the
 * rows found (rows past capacity are dropped, so count > capacity means
 * truncation: zero *count before the first run).  Row order is not
 * specified. */
typedef struct {
    float *ctx;        /* capacity x 6: `context` of the run, copied per row */
    double *y;         /* capacity x 3: u, v (source frame), E of the ray */
    double *w;         /* capacity: weight at the monitor */
    int64_t *bin;      /* capacity: monitor bin */
    uint64_t capacity;
    uint64_t *count;
    float context[6];  /* the run's context (e.g. focal spot, angle, size) */
} mxr_hits;

/* mxr_run that also appends every ray reaching the monitor to hits: the
 * particle state at the monitor (section 2.2.2) as training data for the
 * learned proposal (this library's addition; the paper has no learned
 * component).  The instrument must be a cone-beam source, then slits /
 * boxes / phantoms (which keep direction and energy), then one monitor.  Errors as mxr_run,
 * plus MXR_E_UNSUPPORTED for other instruments. */
mxr_status mxr_collect(mxr_instrument *ins, uint64_t first_ray, uint64_t n_rays, uint64_t n_total, uint64_t seed,
                       uint32_t purpose, uint32_t job, const mxr_tally *tallies, uint32_t n_tallies,
                       const mxr_hits *hits, void *hip_stream);

/* ------------------------------------------------------------------------
 * The proposal network (this library's addition, not the paper's: its
 * output enters the method only through the statistical weight of section
 * 2.2.2, which the importance weights of the proposal keep unbiased).
 *
 * An MLP maps a 6-number context c (e.g. focal-spot position, projection
 * angle as cos / sin, phantom size) to the mixture above:
 *   z1 = c W1 + b1, h1 = silu(z1), z2 = h1 W2 + b2, h2 = silu(z2),
 *   o = h2 W3 + b3 (56 numbers), silu(z) = z / (1 + exp(-z)).
 * Head, component k reading o[7k .. 7k+6]: pi = softmax of the logits
 * o[7k], mu_d = centre_d + half_d tanh(o[7k+1+d]), sigma_d = half_d
 * (1e-3 + softplus(o[7k+4+d])), with the box of the source (centre, half
 * width).  Parameters are packed W1 (6 x 128, row-major), b1, W2 (128 x
 * 128), b2, W3 (128 x 56), b3: MXR_MLP_PARAMS numbers, held as float32
 * master weights and a bfloat16 working copy (uint16_t bit patterns).
 * Products run in bfloat16 with float32 accumulation; the head and its loss
 * in float32.
 *
 * Training loss over a batch: L = -sum_i omega_i log q_gmm(y_i | c_i) /
 * sum_i omega_i.  All arrays below are DEVICE arrays owned by the caller;
 * every call is asynchronous on hip_stream.
 */
#define MXR_MLP_IN 6
#define MXR_MLP_HIDDEN 128
#define MXR_MLP_OUT 56
#define MXR_MLP_PARAMS 24632

/* Regions of the workspace of a batch of n rows (offsets in bytes from
 * mxr_mlp_workspace_layout; row-major, row stride = the row width):
 * X context (n x 6 bf16), Z1 / H1 (n x 128 f32 / bf16), Z2 / H2, O (n x 56
 * f32), DO / DOH gradient of O (f32 / bf16), DZ2 / DZ2H, DZ1 / DZ1H
 * gradients of the pre-activations, PARTIAL per-split gradient partials,
 * Y (n x 3 f64) and W (n f64) gathered targets and weights, ROWLOSS (n f64),
 * SCALARS (reduction scratch), WT (the weight matrices transposed, bf16,
 * out x in row-major, at the parameter offsets of W1, W2, W3), COLS
 * (per-tile column sums for the bias gradients). */
#define MXR_MLP_WS_X 0
#define MXR_MLP_WS_Z1 1
#define MXR_MLP_WS_H1 2
#define MXR_MLP_WS_Z2 3
#define MXR_MLP_WS_H2 4
#define MXR_MLP_WS_O 5
#define MXR_MLP_WS_DO 6
#define MXR_MLP_WS_DOH 7
#define MXR_MLP_WS_DZ2 8
#define MXR_MLP_WS_DZ2H 9
#define MXR_MLP_WS_DZ1 10
#define MXR_MLP_WS_DZ1H 11
#define MXR_MLP_WS_PARTIAL 12
#define MXR_MLP_WS_Y 13
#define MXR_MLP_WS_W 14
#define MXR_MLP_WS_ROWLOSS 15
#define MXR_MLP_WS_SCALARS 16
#define MXR_MLP_WS_WT 17
#define MXR_MLP_WS_COLS 18
#define MXR_MLP_WS_REGIONS 19

typedef struct {
    float lr, beta1, beta2, eps; /* Adam (Kingma and Ba 2015) */
    uint32_t batch;              /* rows per step */
    uint32_t epochs;
    uint64_t seed;               /* per-epoch row shuffles */
    uint32_t first_step;         /* Adam steps already taken (0 for a fresh start) */
} mxr_train_cfg;

/* Bytes of workspace for batches of up to `batch` rows (network section
 * above). */
uint64_t mxr_mlp_workspace_bytes(uint64_t batch);

/* Byte offsets of the MXR_MLP_WS_REGIONS workspace regions for a batch of
 * n rows (offsets[MXR_MLP_WS_REGIONS], host; network section above).
 * Errors: MXR_E_INVALID. */
mxr_status mxr_mlp_workspace_layout(uint64_t batch, uint64_t *offsets);

/* y[i] = bfloat16(x[i]), round to nearest even (the network's working copy,
 * network section above). */
mxr_status mxr_mlp_to_bf16(const float *x, uint64_t n, uint16_t *y, void *hip_stream);

/* Network outputs o (n x 56 f32) of contexts ctx (n x 6 f32) under the
 * bfloat16 parameters w (the forward of the network section above); the layer values stay in ws (ws_bytes >=
 * mxr_mlp_workspace_bytes(n)).  Errors: MXR_E_INVALID, MXR_E_HIP. */
mxr_status mxr_mlp_forward(const uint16_t *w, const float *ctx, uint64_t n, float *out, void *ws, uint64_t ws_bytes,
                           void *hip_stream);

/* mxr_mlp_forward for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): no workspace
 * argument and no allocation; the layer values live in a static device array
 * of 8 MiB that the library holds on each device it runs on until the
 * process ends (its address is looked up once per device, on the first
 * call).  At most MXR_MLP_NOALLOC_ROWS rows per call.  Calls on one device
 * share that array: calls that overlap on one device (on different streams,
 * or from several host threads) race and must not be issued.  No part of the
 * array needs clearing between calls.  Errors: MXR_E_INVALID (null arrays,
 * n above the limit), MXR_E_HIP. */
#define MXR_MLP_NOALLOC_ROWS 4096u
mxr_status mxr_mlp_forward_noalloc(const uint16_t *w, const float *ctx, uint64_t n, float *out, void *hip_stream);

/* Mixture tables for mxr_proposal_set from outputs (the head of the network
 * section above): gmm (n x 56 f64, per row 8 x (pi, mu[3], sigma[3])),
 * with the source's box lo / hi (host, 3 doubles each: -tan a, -tan a,
 * emin / tan a, tan a, emax; mxr_proposal_box). */
mxr_status mxr_mlp_mixture(const float *out, uint64_t n, const double lo[3], const double hi[3], double *gmm,
                           void *hip_stream);

/* Loss L of the network section above (loss: device double, nullable) and
 * its gradient with respect to the parameters (grad: MXR_MLP_PARAMS f32, overwritten) over n rows
 * (ctx n x 6 f32, y n x 3 f64, omega n f64 >= 0 with a positive sum).
 * The weight gradients are reduced over splits of 1024 rows in a fixed
 * order (deterministic).  Errors: MXR_E_INVALID, MXR_E_HIP. */
mxr_status mxr_mlp_loss_grad(const uint16_t *w, const float *ctx, const double *y, const double *omega, uint64_t n,
                             const double lo[3], const double hi[3], float *grad, double *loss, void *ws,
                             uint64_t ws_bytes, void *hip_stream);

/* One Adam step (Kingma and Ba 2015) on master (f32) with moments m, v
 * (f32), writing the bfloat16 copy w; step counts from 1 (bias
 * correction). */
mxr_status mxr_adam_step(float *master, uint16_t *w, const float *grad, float *m, float *v, uint64_t n_params,
                         uint32_t step, float lr, float beta1, float beta2, float eps, void *hip_stream);

/* Training weights of collected rows (mxr_collect): omega_i = w_i /
 * max(I_b, floor_frac * mean of I over bins with hits), I = sum_w of the
 * collecting run's monitor (n_bins), so every live bin carries equal total
 * weight -- the proposal that equalises per-bin errors, the statistic the
 * paper sizes its runs by (section 5.1: rays per pixel and energy bin).
 * scratch: 2 * 256 + 1 doubles. */
mxr_status mxr_train_weights(const double *w, const int64_t *bin, uint64_t n, const double *sum_w, uint64_t n_bins,
                             double floor_frac, double *omega, double *scratch, void *hip_stream);

/* Adam training of the network section above over n_rows rows (< 2^32)
 * for cfg->epochs epochs of batches of cfg->batch rows, each epoch in its
 * own shuffled order.  grad
 * (MXR_MLP_PARAMS f32) is scratch; loss_log (nullable, epochs *
 * ceil(n_rows / batch) doubles) receives each step's loss.  Errors:
 * MXR_E_INVALID, MXR_E_UNSUPPORTED, MXR_E_HIP. */
mxr_status mxr_mlp_train(const float *ctx, const double *y, const double *omega, uint64_t n_rows,
                         const mxr_train_cfg *cfg, const double lo[3], const double hi[3], float *master, uint16_t *w,
                         float *m, float *v, float *grad, void *ws, uint64_t ws_bytes, double *loss_log,
                         void *hip_stream);

/* Training rows gathered by one or more collecting runs (mxr_collect), as
 * DEVICE arrays of n_rows entries; rows [run_first[r], run_first[r + 1])
 * came from run r, whose monitor image (sum_w, DEVICE, n_bins doubles) is
 * run_image[r].  run_first and run_image are HOST arrays of n_runs + 1 and
 * n_runs entries; run_first[0] = 0 and run_first[n_runs] = n_rows. */
typedef struct {
    const float *ctx;
    const double *y;
    const double *w;
    const int64_t *bin;
    uint64_t n_rows;
    uint32_t n_runs;
    const uint64_t *run_first;
    const double *const *run_image;
    uint64_t n_bins;
    double floor_frac; /* of mxr_train_weights */
} mxr_train_rows;

/* The learned proposal from collected rows in one call: the training
 * weights of each run's rows from that run's image (mxr_train_weights,
 * written to omega: DEVICE, n_rows doubles), then Adam training of the
 * network (mxr_mlp_train) in the box of the instrument's source
 * (mxr_proposal_box).  master, w, m, v, grad, ws, ws_bytes and loss_log as
 * in mxr_mlp_train (ws also serves the weight statistics before the
 * training steps).  Asynchronous on hip_stream.  Errors: MXR_E_INVALID
 * (null arrays, run table not covering the rows, n_runs = 0),
 * MXR_E_UNSUPPORTED (the source is not a cone-beam source, 2^32 rows or
 * more), MXR_E_HIP. */
mxr_status mxr_proposal_train(const mxr_instrument *ins, const mxr_train_rows *rows, const mxr_train_cfg *cfg,
                              float *master, uint16_t *w, float *m, float *v, float *grad, double *omega, void *ws,
                              uint64_t ws_bytes, double *loss_log, void *hip_stream);

/* Sets the instrument's proposal from the network: one forward at the
 * host `context` (6 floats) under the bfloat16 parameters w (DEVICE), the
 * mixture in the source's box, then mxr_proposal_set(ins, ., alpha).  ws:
 * DEVICE, at least mxr_mlp_workspace_bytes(1) + 1024 bytes.  Synchronises
 * the device (as mxr_proposal_set).  Errors: as mxr_mlp_forward and
 * mxr_proposal_set. */
mxr_status mxr_proposal_apply(mxr_instrument *ins, const uint16_t *w, const float context[6], double alpha, void *ws,
                              uint64_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Per-bin error of a detector image by batch means.  The paper sizes runs by
 * the statistics each pixel and energy bin receives (section 5.1) and judges
 * images by contrast over noise; it gives no per-bin estimator, so this one
 * is a reading: independent replicas, which stay valid for stratified and
 * importance-weighted sources.
 *
 * sums: DEVICE array of R x n_bins doubles, row r the summed weights
 * (mxr_tally.sum_w) of replica r, an independent run of rays_per_replica
 * rays (e.g. purpose 3 + r).  Writes per bin the image mean_b = (1/R)
 * sum_r sums_rb / rays_per_replica and its relative standard error rel_b =
 * sd_r / (sqrt(R) mean_b) (sd with R - 1 degrees of freedom; +inf where
 * mean_b = 0).  The estimate holds for stratified and importance-weighted
 * runs alike.  Errors: MXR_E_INVALID (R < 2, no rays, null arrays),
 * MXR_E_HIP. */
mxr_status mxr_batch_means(const double *sums, uint32_t R, uint64_t n_bins, uint64_t rays_per_replica,
                           double *mean, double *rel, void *hip_stream);

/* ------------------------------------------------------------------------
 * Batched runs: many projections (angles) of many phantoms in one launch.
 *
 * A CT acquisition repeats one instrument for every projection angle of
 * every sample (paper, section 3.3: a simulation per imaged line and
 * rotational position; section 5.1: hundreds of projections per data set).
 * A batch traces all jobs, longest first, from one HIP graph that is
 * captured once and replayed by every mxr_batch_run: either one kernel over
 * a table of (job, ray range) tiles (one work-group per tile, or persistent
 * work-groups that pop tiles from a device counter), or the jobs' own
 * kernels on parallel graph branches so that one job's tail overlaps the
 * next job.
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

/* Launch shape of a batch.  It changes the order in which rays are traced,
 * never the set of rays or their results. */
#define MXR_BATCH_GRID 0u       /* one work-group per tile of 256 rays over one 2-D grid */
#define MXR_BATCH_PERSISTENT 1u /* groups_per_cu work-groups per CU pop tiles from a counter */
#define MXR_BATCH_LAUNCHES 2u   /* one mxr_run-shaped launch per job, on `branches` graph branches */
typedef struct {
    uint32_t form;
    uint32_t groups_per_cu; /* persistent: 1..8 */
    uint32_t tile_rays;     /* persistent: a multiple of 256 in [256, 2^24] (0 = 65536) */
    uint32_t branches;      /* launches: 1..4 (0 = 1); jobs dealt longest-first round-robin */
} mxr_batch_schedule;

/* Validates the jobs (all instruments on the current device with the same
 * component types in the same order; tally sizes; n_rays >= 1) and builds
 * the job and tile tables on the device (owned by the handle).  schedule is
 * nullable (one launch per job on one branch until tuned).  The
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

/* Current launch shape (batch section above). */
mxr_status mxr_batch_get_schedule(const mxr_batch *batch, mxr_batch_schedule *out);

/* Replaces the launch shape (batch section above; the captured graph is
 * rebuilt on the next run).
 * Errors: MXR_E_INVALID for an out-of-range shape. */
mxr_status mxr_batch_set_schedule(mxr_batch *batch, const mxr_batch_schedule *schedule);

/* Synchronises the device, frees the handle and its device tables.  NULL is
 * accepted.  (Library bookkeeping.) */
void mxr_batch_destroy(mxr_batch *batch);

/* Autotuner of a batch (the rays of all jobs are independent, paper section
 * 2.2, so their order and grouping on the device are free): times candidate
 * launch shapes (the grid form; persistent forms
 * of 2/4/8 groups per CU x 16K/64K-ray tiles; launches on 1/2/4 branches) on
 * the batch with every job's ray count scaled by rays_fraction (0 < f <= 1),
 * keeps the fastest and records it under a key describing the batch (its
 * component chain, job count, total rays and work estimate) in the text
 * file cache_path (nullable: no cache), which later calls consult before
 * timing anything.  The chosen shape is set on the batch and returned in
 * out (nullable).  Timing runs ADD into the jobs' tallies: zero them before
 * the production run.  Synchronous.  Errors: MXR_E_INVALID, MXR_E_HIP. */
mxr_status mxr_batch_autotune(mxr_batch *batch, double rays_fraction, const char *cache_path,
                              mxr_batch_schedule *out);

/* ------------------------------------------------------------------------
 * Micro-benchmarks: the achievable rates that bound the tracing kernels, for
 * roofline denominators measured on the device beside the vendor figures
 * (measurement infrastructure, not part of the method; the paper's own
 * procedure, section 3.4, times whole runs).
 * Not part of tracing.  One launch of groups x 256 lanes on hip_stream
 * (asynchronous; the caller times it with events on that stream); *work
 * receives the operations (bytes for the read) the launch performs.
 *   MXR_PEAK_FP64_FMA  -- iters x 8 independent FP64 fma chains per lane;
 *                         *work = flops (2 per fma).  buf: one double per
 *                         lane (sink).
 *   MXR_PEAK_U32_MULHI -- iters x 8 chains of 32-bit multiply-high (the
 *                         Philox rounds' product); *work = multiplies.
 *   MXR_PEAK_FP64_EXP  -- iters x 4 chains of FP64 exp; *work = exps.
 *   MXR_PEAK_READ      -- a grid-stride read of the buffer beyond the first
 *                         groups x 256 doubles (the sink), in 16-byte
 *                         elements; *work = bytes read.
 *   MXR_PEAK_ATOMIC_F64 -- every lane adds 1.0 iters times into buf[0 ..
 *                         spread) (addresses hashed per lane, consecutive
 *                         per iteration); *work = atomics.  The buffer then
 *                         holds the counts (sum = *work).
 * buf: device buffer of bytes bytes.  Errors: MXR_E_INVALID (null
 * pointers, groups not in [1, 2^20], iters not in [1, 2^32], a buffer too
 * small, spread not in [1, bytes / 8], unknown kind), MXR_E_HIP. */
#define MXR_PEAK_FP64_FMA 0u
#define MXR_PEAK_U32_MULHI 1u
#define MXR_PEAK_FP64_EXP 2u
#define MXR_PEAK_READ 3u
#define MXR_PEAK_ATOMIC_F64 4u
mxr_status mxr_peak_launch(uint32_t kind, void *buf, uint64_t bytes, uint64_t spread, uint64_t iters, uint32_t groups,
                           double *work, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MXR_H */
