// mxr.hip -- fused per-ray tracing kernels and the C ABI of include/mxr.h.
//
// One kernel launch traces a contiguous range of ray ids.  Each lane takes a
// ray from the source through every component to the monitors with all
// state in registers (paper, section 2.2: independent rays, local
// intermediates; the monitor arrays are the only shared data and are updated
// atomically).  The launch is XCD-aware: work-groups are dealt to the eight
// XCDs round-robin, so work-group b works on the (b mod 8)-th eighth of the
// ray range and neighbouring ray ids -- which the stratified cone-beam
// source sends through neighbouring voxels -- share one XCD's L2.
//
// Component sequences that the library knows are compiled as fixed chains
// (no per-component dispatch); any other sequence of supported components
// runs through a generic chain that dispatches on the component type, which
// is wave-uniform.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "mxr.h"
#include "mxr_device.h"

using namespace mxr;

namespace {

// The device's constant address space, for tables that no kernel writes
// while they are read (in the host pass, where kernel bodies are only
// parsed, it is the ordinary one).
#if defined(__HIP_DEVICE_COMPILE__)
#define MXR_CONSTANT __attribute__((address_space(4)))
#else
#define MXR_CONSTANT
#endif
// The same space for a kernel's pointer parameter, in both passes: a
// parameter's type is part of the kernel's mangled name, by which the host
// stub finds the device code, so host and device must spell it alike.
#define MXR_CONSTANT_PARAM __attribute__((address_space(4)))

constexpr int kBlock = 256;
// The HSA dispatch packet gives the grid size in work-items as a 32-bit count:
// a launch of 256-item groups holds at most 2^24 - 1 of them.  2^24 - 8 keeps
// the count a multiple of the 8 XCDs.
constexpr uint64_t kMaxLaunchGroups = (1ull << 24) - 8;
constexpr int kDynamic = -1;
constexpr uint32_t kMaxBranches = 4;  // graph branches of a batch in the launches form
// internal component kinds (not in the public enum): the cone-beam source
// drawing from a proposal mixture, and a monitor that also records its hits
constexpr int kSrcConeProposal = 100;
constexpr int kDetectorCollect = 101;
// the phantom component (same descriptor) under the fixed-step model
constexpr int kPhantomStep = 102;
// a monitor whose histogram may be accumulated in a work-group private LDS
// copy (small monitors of the compacting kernel), flushed once per group
constexpr int kDetectorLds = 103;
// the phantom component (same descriptor) tracing photons scattered K times
constexpr int kPhantomScatter = 104;

constexpr bool is_detector(int T) { return T == MXR_DETECTOR || T == kDetectorCollect || T == kDetectorLds; }

// ---------------------------------------------------------------- state --

struct RayEnd {
    int32_t status, dead_at;
    int64_t bin;
};

struct LedgerLds {
    double *slots;  // 4 * ncomp + 1 doubles in LDS, or null
    // work-group private monitors (kDetectorLds): the LDS block, and per
    // tally slot the first word of the monitor's block (-1: not private)
    // and its bin count; the block holds count (u64), sum w, sum w^2
    double *tl = nullptr;
    const int32_t *tl_off = nullptr;
    const uint32_t *tl_nb = nullptr;
};

template <bool LEDGER>
__device__ __forceinline__ void ledger_add(const LedgerLds &L, int slot, double v) {
    if constexpr (LEDGER) atomicAdd(L.slots + slot, v);
}

// Append (context, y, w, bin) of the lanes whose flag is set to the hit
// sink: one atomic per wave reserves the rows, each lane writes at its rank
// among the flagged lanes.  y is the direction in the source's frame as
// (dx/dz, dy/dz) and the energy: the collecting chains leave both as the
// source drew them.
__device__ __forceinline__ void append_hit(const RunArgs &a, const DevComp &src, const Ray &ray, int64_t bin,
                                           bool flag) {
    const uint64_t mask = __builtin_amdgcn_ballot_w64(flag);
    if (!flag) return;
    const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const int leader = __builtin_ctzll(mask);
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    unsigned long long base = 0;
    if ((int)lane == leader) base = atomicAdd(a.hits.count, (unsigned long long)__builtin_popcountll(mask));
    base = __shfl(base, leader, 64);
    const uint64_t row = base + rank;
    if (row >= a.hits.capacity) return;
    double q[3], dl[3];
    to_local(src, ray, q, dl);
#pragma unroll
    for (int i = 0; i < 6; ++i) a.hits.ctx[row * 6 + i] = a.hits.c[i];
    a.hits.y[row * 3 + 0] = dl[0] / dl[2];
    a.hits.y[row * 3 + 1] = dl[1] / dl[2];
    a.hits.y[row * 3 + 2] = ray.E;
    a.hits.w[row] = ray.w;
    a.hits.bin[row] = bin;
}

// Apply component k of type T.  Returns false when the ray is absorbed.
template <int T, bool LEDGER, bool TRACE, bool EXACT, int KW = kWalkRound>
__device__ __forceinline__ bool apply(const DevComp &c, int k, Ray &ray, Stream &s, uint64_t ray_id,
                                      const RunArgs &a, const double *mu_lds, uint32_t n_mat, uint32_t n_ebin,
                                      RayEnd &end, const LedgerLds &L) {
    if constexpr (T == MXR_SRC_RECT_CONE || T == MXR_SRC_CONE_BEAM || T == MXR_SRC_GAUSSIAN ||
                  T == kSrcConeProposal) {
        if constexpr (T == MXR_SRC_RECT_CONE) src_rect_cone(c, s, ray);
        if constexpr (T == MXR_SRC_CONE_BEAM) src_cone_beam(c, s, ray, ray_id, a);
        if constexpr (T == MXR_SRC_GAUSSIAN) src_gaussian(c, s, ray);
        if constexpr (T == kSrcConeProposal) {
            const bool ok = src_cone_proposal(c, a.prop, s, ray, ray_id, a);
            ledger_add<LEDGER>(L, 4 * k, ray.w);
            if (!ok) {  // drawn outside the cone: emitted with weight 0
                end.status = kAbsorbed;
                end.dead_at = k;
                ledger_add<LEDGER>(L, 4 * k + 1, ray.w);
                return false;
            }
            return true;
        }
        ledger_add<LEDGER>(L, 4 * k, ray.w);
        return true;
    } else {
        const double w_in = ray.w;
        Ray before = ray;
        bool ok = true;
        int64_t bin = -1;
        if constexpr (T == MXR_SLIT) ok = comp_slit(c, ray);
        if constexpr (T == MXR_BOX) comp_box(c, ray);
        if constexpr (T == MXR_LENS_CRL) ok = comp_lens(c, ray);
        if constexpr (T == kPhantomScatter) ok = comp_phantom_scatter<EXACT>(c, s, ray, mu_lds, n_mat, n_ebin);
        if constexpr (T == MXR_PHANTOM || T == kPhantomStep) {
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
            for (int i = 0; i < 3; ++i) {
                g.blo[i] = c.aux[8 + i];
                g.bhi[i] = c.aux[11 + i];
            }
            g.bg = (uint32_t)c.aux[14];
            g.box = c.aux[15] != 0.0;
            double f = floor((ray.E - c.par[1]) * c.aux[3]);
            int e = (int)fmin(fmax(f, 0.0), (double)(n_ebin - 1));
            double tau;
            if constexpr (T == kPhantomStep)
                tau = step_tau(g, q, dl, c.par[3], (int)c.aux[5], mu_lds + e * n_mat);
            else
                tau = siddon_tau<EXACT, false, true, KW>(g, q, dl, mu_lds + e * n_mat);
            ray.w = ray.w * exp(-tau);
        }
        if constexpr (T == MXR_MIRROR_ELLIPTIC) ok = comp_mirror(c, ray);
        if constexpr (T == MXR_DCM) ok = comp_dcm(c, ray);
        if constexpr (T == MXR_POWDER) ok = comp_powder(c, s, ray);
        if constexpr (is_detector(T)) ok = comp_detector(c, ray, bin);
        ledger_add<LEDGER>(L, 4 * k, w_in);
        if (!ok) {
            ray = before;
            end.status = kAbsorbed;
            end.dead_at = k;
            ledger_add<LEDGER>(L, 4 * k + 1, w_in);
            return false;
        }
        ledger_add<LEDGER>(L, 4 * k + 2, w_in - ray.w);
        if constexpr (T == kDetectorCollect) append_hit(a, a.ins->c[0], ray, bin, bin >= 0);
        if constexpr (is_detector(T)) {
            if (bin >= 0) {
                end.bin = bin;
                if constexpr (!TRACE) {
                    const uint32_t sl = c.slot;
                    bool done = false;
                    if constexpr (T == kDetectorLds) {
                        const int32_t o = L.tl_off[sl];
                        if (o >= 0) {
                            const uint32_t nb = L.tl_nb[sl];
                            atomicAdd((unsigned long long *)(L.tl + o) + bin, 1ull);
                            atomicAdd(L.tl + o + nb + bin, ray.w);
                            atomicAdd(L.tl + o + 2 * nb + bin, ray.w * ray.w);
                            done = true;
                        }
                    }
                    if (!done) {
                        atomicAdd(a.tally.count[sl] + bin, 1ull);
                        atomicAdd(a.tally.sum_w[sl] + bin, ray.w);
                        atomicAdd(a.tally.sum_w2[sl] + bin, ray.w * ray.w);
                    }
                }
                ledger_add<LEDGER>(L, 4 * k + 3, ray.w);
            }
        }
        return true;
    }
}

template <bool LEDGER, bool TRACE, bool EXACT, int KW = kWalkRound>
__device__ __forceinline__ bool apply_dynamic(const DevComp &c, int k, Ray &ray, Stream &s, uint64_t ray_id,
                                              const RunArgs &a, const double *mu_lds, uint32_t n_mat,
                                              uint32_t n_ebin, RayEnd &end, const LedgerLds &L) {
#define MXR_CASE(T) \
    case T: return apply<T, LEDGER, TRACE, EXACT, KW>(c, k, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L);
    switch (c.type) {
        MXR_CASE(MXR_SRC_RECT_CONE)
        case MXR_SRC_CONE_BEAM:
            if (a.prop) return apply<kSrcConeProposal, LEDGER, TRACE, EXACT, KW>(c, k, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L);
            return apply<MXR_SRC_CONE_BEAM, LEDGER, TRACE, EXACT, KW>(c, k, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L);
        MXR_CASE(MXR_SRC_GAUSSIAN)
        MXR_CASE(MXR_SLIT)
        MXR_CASE(MXR_BOX)
        case MXR_PHANTOM:
            if (c.flags & 2u) return apply<kPhantomScatter, LEDGER, TRACE, EXACT, KW>(c, k, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L);
            if (c.flags & 1u) return apply<kPhantomStep, LEDGER, TRACE, EXACT, KW>(c, k, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L);
            return apply<MXR_PHANTOM, LEDGER, TRACE, EXACT, KW>(c, k, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L);
        MXR_CASE(MXR_MIRROR_ELLIPTIC)
        MXR_CASE(MXR_DCM)
        MXR_CASE(MXR_POWDER)
        MXR_CASE(MXR_LENS_CRL)
        case MXR_DETECTOR:
            if (a.hits.count) return apply<kDetectorCollect, LEDGER, TRACE, EXACT, KW>(c, k, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L);
            return apply<MXR_DETECTOR, LEDGER, TRACE, EXACT, KW>(c, k, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L);
        default: break;
    }
#undef MXR_CASE
    end.status = kAbsorbed;
    end.dead_at = k;
    return false;
}

// Fixed chains: the component types in instrument order.
template <int... Ts>
struct Chain {};

// Occupancy hint per chain (waves per SIMD the compiler must fit).  The
// projection chain is latency-bound in its voxel walk: 8 waves (64 VGPRs,
// a few bytes of scratch for the ray state held across the walk) measured
// faster than the 6 its natural 76 VGPRs allow.
template <class C>
struct WavesHint {
    static constexpr int value = 1;
};
#ifndef MXR_PROJ_WAVES
#define MXR_PROJ_WAVES 8
#endif
template <>
struct WavesHint<Chain<MXR_SRC_CONE_BEAM, MXR_PHANTOM, MXR_DETECTOR>> {
    static constexpr int value = MXR_PROJ_WAVES;
};
template <>
struct WavesHint<Chain<MXR_SRC_CONE_BEAM, MXR_PHANTOM, kDetectorCollect>> {
    static constexpr int value = 8;
};
template <>
struct WavesHint<Chain<kSrcConeProposal, MXR_PHANTOM, MXR_DETECTOR>> {
    static constexpr int value = 8;
};
template <>
struct WavesHint<Chain<MXR_SRC_CONE_BEAM, MXR_SLIT, MXR_PHANTOM, MXR_DETECTOR>> {
    static constexpr int value = 8;
};
template <>
struct WavesHint<Chain<MXR_SRC_CONE_BEAM, kPhantomStep, MXR_DETECTOR>> {
    static constexpr int value = 8;
};
// the scattering chain holds three walks: 6 waves (at most 80 VGPRs)
// measured 17 % faster than its natural 141 VGPRs at 3 waves, and than 4 or 8
template <>
struct WavesHint<Chain<MXR_SRC_CONE_BEAM, kPhantomScatter, MXR_DETECTOR>> {
    static constexpr int value = 6;
};
// Crossings per round of the optical-depth walk, per chain.  The projection's
// own kernel takes 5 (2-3 % faster than 4 at every angle measured, 12 B of
// scratch); the chains whose kernels spill more at 5 keep 4 (the early-out
// projection's kernel ran 1.4x slower at 5, the batch grid 3 % slower).
template <class C>
struct WalkRound {
    static constexpr int value = kWalkRound;
};
template <>
struct WalkRound<Chain<MXR_SRC_CONE_BEAM, MXR_PHANTOM, MXR_DETECTOR>> {
    static constexpr int value = 5;
};

// The batch kernels read their per-job arguments from memory rather than the
// kernel-argument segment and hold more live values: the projection chain
// fits 4 waves per SIMD without spilling there.
template <class C>
struct BatchWavesHint {
    static constexpr int value = 1;
};
#ifndef MXR_BATCH_WAVES
#define MXR_BATCH_WAVES 8
#endif
template <>
struct BatchWavesHint<Chain<MXR_SRC_CONE_BEAM, MXR_PHANTOM, MXR_DETECTOR>> {
    static constexpr int value = MXR_BATCH_WAVES;
};

template <bool LEDGER, bool TRACE, bool EXACT, int KW, int T, int... Rest>
__device__ __forceinline__ bool run_fixed(const DevInstr *ins, int k, Ray &ray, Stream &s, uint64_t ray_id,
                                          const RunArgs &a, const double *mu_lds, uint32_t n_mat,
                                          uint32_t n_ebin, RayEnd &end, const LedgerLds &L) {
    if (!apply<T, LEDGER, TRACE, EXACT, KW>(ins->c[k], k, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L)) return false;
    if constexpr (sizeof...(Rest) > 0)
        return run_fixed<LEDGER, TRACE, EXACT, KW, Rest...>(ins, k + 1, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L);
    return true;
}

template <bool LEDGER, bool TRACE, bool EXACT, int KW = kWalkRound, int... Ts>
__device__ __forceinline__ bool run_chain(Chain<Ts...>, const DevInstr *ins, Ray &ray, Stream &s, uint64_t ray_id,
                                          const RunArgs &a, const double *mu_lds, uint32_t n_mat,
                                          uint32_t n_ebin, RayEnd &end, const LedgerLds &L) {
    if constexpr (sizeof...(Ts) == 1 && ((Ts == kDynamic) && ...)) {
        const uint32_t n = ins->ncomp;
        for (uint32_t k = 0; k < n; ++k)
            if (!apply_dynamic<LEDGER, TRACE, EXACT, KW>(ins->c[k], (int)k, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L))
                return false;
        return true;
    } else {
        return run_fixed<LEDGER, TRACE, EXACT, KW, Ts...>(ins, 0, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L);
    }
}

// Ray tile of work-group b of a launch of 8 * per_xcd work-groups.  The
// hardware deals work-groups to the eight XCDs round-robin (XCD b mod 8), so
// the order decides which tiles an XCD traces: 0, the (b mod 8)-th eighth of
// the range (each XCD a contiguous block of ray ids); 1, launch order (tile
// b); 2, runs of kXcdRun consecutive tiles, the runs dealt to the XCDs in
// turn.  The stratified source sends a block of ray ids through one band of
// the cone, whose paths can be longer or shorter than the others', so order
// 0 leaves XCDs idle at the end; orders 1 and 2 spread every band over all
// eight.  Each order is a bijection of [0, 8 per_xcd).
constexpr uint32_t kXcdRun = 64;
__device__ __forceinline__ uint64_t tile_of(uint32_t b, uint32_t order, uint32_t per_xcd) {
    const uint32_t x = b & 7u, slot = b >> 3;
    if (order == 1) return b;
    if (order == 2) {
        const uint32_t full = per_xcd / kXcdRun * kXcdRun;
        if (slot < full) return (uint64_t)(slot / kXcdRun) * (8 * kXcdRun) + x * kXcdRun + slot % kXcdRun;
        return 8ull * full + (uint64_t)x * (per_xcd - full) + (slot - full);
    }
    return (uint64_t)x * per_xcd + slot;
}

// The instrument block is read-only for the whole launch; passing it as its
// own restrict-qualified argument lets its wave-uniform fields be read with
// scalar loads even though the kernel stores to the histograms.
//
// One lane traces exactly one ray.  (A loop over several rays per lane lets
// the compiler hoist every loop-invariant constant -- the polynomial
// coefficients of exp, sin, cos -- into registers for the whole kernel, which
// costs occupancy.)  Which tiles of the ray range a work-group traces is
// tile_of's choice (launch order unless the launch shape picks another).
template <class C, bool LEDGER, bool TRACE, bool EXACT, int WAVES = WavesHint<C>::value>
__global__ __launch_bounds__(kBlock, WAVES) void k_trace(const MXR_CONSTANT_PARAM DevInstr *__restrict__ insc,
                                                         RunArgs a) {
    // the instrument block through the constant address space: nothing writes
    // it during a launch, so its wave-uniform fields may be loaded again near
    // each use instead of being held in scalar registers across the walk
    const DevInstr *ins = (const DevInstr *)insc;
    extern __shared__ double smem[];
    const uint32_t n_mat = ins->n_mat, n_ebin = ins->n_ebin;
    double *mu_lds = smem;
    const uint32_t n_mu = (ins->phantom >= 0) ? n_mat * n_ebin : 0u;
    if (n_mu) {
        // stage the table as prepared at create (mu / 10, energy-major)
        const double *T = ins->mu_em;
        for (uint32_t i = threadIdx.x; i < n_mu; i += kBlock) mu_lds[i] = T[i];
    }
    LedgerLds L{nullptr};
    const uint32_t n_slots = 4 * ins->ncomp + 1;
    if constexpr (LEDGER) {
        L.slots = smem + n_mu;
        for (uint32_t i = threadIdx.x; i < n_slots; i += kBlock) L.slots[i] = 0.0;
    }
    __syncthreads();

    const uint64_t logical = tile_of(blockIdx.x, a.xcd_order, a.blocks_per_xcd);
    const uint64_t i = logical * kBlock + threadIdx.x;
    if (i < a.n) {
        const uint64_t ray_id = TRACE ? a.ids[i] : a.first + i;
        Stream s;
        s.init(a.seed, ray_id, a.word3);
        Ray ray;
        ray.r[0] = ray.r[1] = ray.r[2] = 0.0;
        ray.d[0] = ray.d[1] = ray.d[2] = 0.0;
        ray.E = 0.0;
        ray.w = 0.0;
        RayEnd end{kExited, -1, -1};
        bool alive = run_chain<LEDGER, TRACE, EXACT, WalkRound<C>::value>(C{}, ins, ray, s, ray_id, a, mu_lds, n_mat,
                                                                          n_ebin, end, L);
        if constexpr (LEDGER) {
            if (alive) atomicAdd(L.slots + 4 * ins->ncomp, ray.w);
        }
        if constexpr (TRACE) {
            a.dump.x[i] = ray.r[0];
            a.dump.y[i] = ray.r[1];
            a.dump.z[i] = ray.r[2];
            a.dump.dx[i] = ray.d[0];
            a.dump.dy[i] = ray.d[1];
            a.dump.dz[i] = ray.d[2];
            a.dump.E[i] = ray.E;
            a.dump.w[i] = ray.w;
            a.dump.status[i] = end.status;
            a.dump.dead_at[i] = end.dead_at;
            a.dump.bin[i] = end.bin;
        }
        (void)alive;
    }
    if constexpr (LEDGER) {
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < n_slots; k += kBlock) {
            double v = L.slots[k];
            if (v != 0.0) atomicAdd(a.ledger + k, v);
        }
    }
}

// ------------------------------------------------- survivor compaction --
// Chains whose first components discard most rays (a crop aperture right
// after the source: 87 % of the focusing instrument's rays, 98.7 % of the
// basic absorber's) would run their costly later components on waves that
// are mostly idle.  The compacting kernel runs only the cheap prefix
// (components 0 .. CompactCut) per ray id, collects the ids of the rays that
// survive it in a per-wave LDS queue (ballot + rank), and whenever 64 are
// queued traces those 64 through the whole chain -- source again included,
// which redraws exactly the same ray -- with every lane busy.  Used for plain
// runs (no ledger, no per-ray output); the result is the same set of rays,
// tallied in another order.
template <class C>
struct CompactCut {
    static constexpr int value = -1;  // no compaction
};

// 64-ray rounds per wave: at most kCompactRounds, fewer for small runs so
// that a launch still has several work-groups per compute unit
constexpr int kCompactRounds = 64;

// Monitors of the compacting kernel with at most kLdsTallyBins bins (and at
// most kLdsTallyTotal bins over all of them, in instrument order) are
// accumulated in a work-group private LDS histogram and added to the
// caller's tallies once per work-group: a small monitor (e.g. 130 energy
// bins) hit by every surviving ray would otherwise serialise its global
// atomics on a few hundred addresses.  Layout per private monitor: count
// (u64), sum w, sum w^2, n_bins each.  Returns the LDS bytes; off[slot] is
// the private monitor's first bin in units of 8 bytes, or -1.
__host__ __device__ inline uint32_t lds_tally_layout(const DevInstr &d, int32_t off[MXR_MAX_DETECTORS]) {
    constexpr uint64_t kLdsTallyBins = 1024, kLdsTallyTotal = 2048;
    uint64_t used = 0;
    for (uint32_t s = 0; s < MXR_MAX_DETECTORS; ++s) off[s] = -1;
    for (uint32_t k = 0; k < d.ncomp; ++k) {
        const DevComp &c = d.c[k];
        if (c.type != MXR_DETECTOR) continue;
        const uint64_t nb = (uint64_t)c.dims[0] * c.dims[1] * c.dims[2];
        if (nb <= kLdsTallyBins && used + nb <= kLdsTallyTotal) {
            off[c.slot] = (int32_t)(3 * used);
            used += nb;
        }
    }
    return (uint32_t)(3 * used * 8);
}

template <bool EXACT, int CUT, int I, int T, int... Rest>
__device__ __forceinline__ bool run_prefix(const DevInstr *ins, Ray &ray, Stream &s, uint64_t ray_id,
                                           const RunArgs &a, RayEnd &end, const LedgerLds &L) {
    static_assert(!is_detector(T), "the compaction prefix must end before the first monitor");
    if (!apply<T, false, false, EXACT>(ins->c[I], I, ray, s, ray_id, a, nullptr, 0u, 1u, end, L)) return false;
    if constexpr (I < CUT) return run_prefix<EXACT, CUT, I + 1, Rest...>(ins, ray, s, ray_id, a, end, L);
    return true;
}

template <bool EXACT, int CUT, int... Ts>
__device__ __forceinline__ bool run_prefix_chain(Chain<Ts...>, const DevInstr *ins, Ray &ray, Stream &s,
                                                 uint64_t ray_id, const RunArgs &a, RayEnd &end,
                                                 const LedgerLds &L) {
    return run_prefix<EXACT, CUT, 0, Ts...>(ins, ray, s, ray_id, a, end, L);
}

__device__ __forceinline__ void fresh_ray(Ray &ray) {
    ray.r[0] = ray.r[1] = ray.r[2] = 0.0;
    ray.d[0] = ray.d[1] = ray.d[2] = 0.0;
    ray.E = 0.0;
    ray.w = 0.0;
}

// Each wave owns 64 * a.compact_rounds consecutive ray ids of the launch
// (work-groups remapped to XCDs as in k_trace); the queue never holds more
// than 127 ids (it is drained as soon as it reaches 64), every loop is
// bounded by the wave's id count, and every wave reaches the two barriers.
// The chains compacted here hold no phantom, so no attenuation table is
// staged; the dynamic LDS holds the private monitors.
template <class C, bool EXACT>
__global__ __launch_bounds__(kBlock, WavesHint<C>::value) void k_trace_compact(const MXR_CONSTANT_PARAM DevInstr *__restrict__ insc,
                                                                               RunArgs a) {
    const DevInstr *ins = (const DevInstr *)insc;  // as in k_trace
    constexpr int CUT = CompactCut<C>::value;
    static_assert(CUT >= 0, "chain without a compaction prefix");
    extern __shared__ double smem[];
    __shared__ uint64_t queue[kBlock / 64][128];
    // the private monitors' layout, set up once per work-group
    __shared__ int32_t tl_off[MXR_MAX_DETECTORS];
    __shared__ uint32_t tl_nb[MXR_MAX_DETECTORS];
    __shared__ uint32_t lds_words;
    if (threadIdx.x == 0) {
        lds_words = lds_tally_layout(*ins, tl_off) / 8;
        for (uint32_t sl = 0; sl < MXR_MAX_DETECTORS; ++sl) tl_nb[sl] = 0;
        for (uint32_t k = 0; k < ins->ncomp; ++k) {
            const DevComp &c = ins->c[k];
            if (c.type == MXR_DETECTOR) tl_nb[c.slot] = c.dims[0] * c.dims[1] * c.dims[2];
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < lds_words; i += kBlock) smem[i] = 0.0;
    __syncthreads();
    LedgerLds L{nullptr};
    L.tl = smem;
    L.tl_off = tl_off;
    L.tl_nb = tl_nb;
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    uint64_t *Q = queue[wave];
    const uint64_t logical = tile_of(blockIdx.x, a.xcd_order, a.blocks_per_xcd);
    const uint64_t per_wave = 64ull * a.compact_rounds;
    const uint64_t wbase = (logical * (kBlock / 64) + wave) * per_wave;
    const uint64_t wend = wbase + per_wave < a.n ? wbase + per_wave : a.n;
    uint32_t qn = 0;  // wave-uniform
    for (uint64_t i0 = wbase; i0 < wend; i0 += 64) {
        const uint64_t i = i0 + lane;
        bool pass = false;
        if (i < wend) {
            Stream s;
            s.init(a.seed, a.first + i, a.word3);
            Ray ray;
            fresh_ray(ray);
            RayEnd end{kExited, -1, -1};
            pass = run_prefix_chain<EXACT, CUT>(C{}, ins, ray, s, a.first + i, a, end, L);
        }
        const uint64_t mask = __builtin_amdgcn_ballot_w64(pass);
        if (pass) {
            const uint32_t rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            Q[qn + rank] = a.first + i;
        }
        qn += (uint32_t)__builtin_popcountll(mask);
        __builtin_amdgcn_wave_barrier();
        if (qn >= 64) {
            const uint64_t ray_id = Q[lane];
            Stream s;
            s.init(a.seed, ray_id, a.word3);
            Ray ray;
            fresh_ray(ray);
            RayEnd end{kExited, -1, -1};
            (void)run_chain<false, false, EXACT>(C{}, ins, ray, s, ray_id, a, nullptr, 0u, 1u, end, L);
            const uint32_t rest = qn - 64;
            const uint64_t carry = lane < rest ? Q[64 + lane] : 0ull;
            __builtin_amdgcn_wave_barrier();
            if (lane < rest) Q[lane] = carry;
            __builtin_amdgcn_wave_barrier();
            qn = rest;
        }
    }
    if (lane < qn) {
        const uint64_t ray_id = Q[lane];
        Stream s;
        s.init(a.seed, ray_id, a.word3);
        Ray ray;
        fresh_ray(ray);
        RayEnd end{kExited, -1, -1};
        (void)run_chain<false, false, EXACT>(C{}, ins, ray, s, ray_id, a, nullptr, 0u, 1u, end, L);
    }
    // add the private monitors to the caller's tallies (bins nobody hit skipped)
    __syncthreads();
    for (uint32_t sl = 0; sl < MXR_MAX_DETECTORS; ++sl) {
        const int32_t o = tl_off[sl];
        if (o < 0) continue;
        const uint32_t nb = tl_nb[sl];
        for (uint32_t b = threadIdx.x; b < nb; b += kBlock) {
            const unsigned long long n = ((const unsigned long long *)(smem + o))[b];
            if (n == 0) continue;
            atomicAdd(a.tally.count[sl] + b, n);
            atomicAdd(a.tally.sum_w[sl] + b, smem[o + nb + b]);
            atomicAdd(a.tally.sum_w2[sl] + b, smem[o + 2 * nb + b]);
        }
    }
}

// ---------------------------------------------------------------- batch --

// One job of a batch: its instrument and the arguments of its run (read in
// place from the job table, so their wave-uniform fields stay scalar loads).
struct BatchJob {
    RunArgs args;    // args.ins, n = n_total = rays of the job, seed, strata, tallies
    uint64_t tile0;  // first tile of this job in the launch's tile order
};

__global__ void k_batch_reset(unsigned long long *counter) { *counter = 0ull; }

// Persistent batched launch: each work-group pops tiles (job, range of
// tile_rays ray ids) from one device counter until the counter passes the
// last tile -- every work-group reaches that exit.  Jobs are stored
// longest-first, so the costly tiles go out early and the short ones fill
// the end.  The mu table is restaged in LDS when a work-group moves to a job
// with another table.
template <class C, bool EXACT>
__global__ __launch_bounds__(kBlock, BatchWavesHint<C>::value) void k_batch(const BatchJob *__restrict__ jobs,
                                                                     uint32_t n_jobs, uint64_t n_tiles,
                                                                     uint32_t tile_rays,
                                                                     unsigned long long *counter) {
    extern __shared__ double smem[];
    __shared__ unsigned long long s_tile;
    double *mu_lds = smem;
    const double *staged = nullptr;
    const LedgerLds L{nullptr};
    for (uint64_t iter = 0; iter <= n_tiles; ++iter) {
        if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1ull);
        __syncthreads();
        // the popped tile is the same for every lane: make that explicit so
        // the job lookup and the job's arguments stay scalar
        const uint64_t t_lds = s_tile;
        const uint64_t tile = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(t_lds >> 32)) << 32) |
                              (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)t_lds);
        __syncthreads();
        if (tile >= n_tiles) break;
        // job of this tile: the last job whose first tile is <= tile
        uint32_t lo = 0, hi = n_jobs;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (jobs[mid].tile0 <= tile) lo = mid;
            else hi = mid;
        }
        // the job through the constant address space (see k_batch_grid)
        const MXR_CONSTANT BatchJob &J = ((const MXR_CONSTANT BatchJob *)jobs)[lo];
        const MXR_CONSTANT RunArgs &a = J.args;
        const DevInstr *ins = a.ins;
        const uint32_t n_mat = ins->n_mat, n_ebin = ins->n_ebin;
        if (ins->phantom >= 0) {
            const double *T = ins->mu_em;
            if (T != staged) {
                const uint32_t n_mu = n_mat * n_ebin;
                for (uint32_t i = threadIdx.x; i < n_mu; i += kBlock) mu_lds[i] = T[i];
                staged = T;
                __syncthreads();
            }
        }
        const uint64_t r0 = (tile - J.tile0) * tile_rays;
        const uint64_t r1 = r0 + tile_rays < a.n ? r0 + tile_rays : a.n;
        for (uint64_t ray_id = r0 + threadIdx.x; ray_id < r1; ray_id += kBlock) {
            Stream s;
            s.init(a.seed, ray_id, a.word3);
            Ray ray;
            ray.r[0] = ray.r[1] = ray.r[2] = 0.0;
            ray.d[0] = ray.d[1] = ray.d[2] = 0.0;
            ray.E = 0.0;
            ray.w = 0.0;
            RayEnd end{kExited, -1, -1};
            run_chain<false, false, EXACT>(C{}, ins, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L);
        }
        // the next tile may restage the table: everyone must be done with it
        __syncthreads();
    }
}


// Grid form of a batch: one work-group per tile of 256 rays, one ray per
// lane and no loop (the whole batch is one 2-D grid; the hardware dispatcher
// balances the uneven jobs).  Tiles are numbered longest job first; within
// groups of 8 x 64 consecutive tiles, each XCD gets 64 consecutive tiles.
template <class C, bool EXACT>
__global__ __launch_bounds__(kBlock, BatchWavesHint<C>::value) void k_batch_grid(const BatchJob *__restrict__ jobs,
                                                                          uint32_t n_jobs, uint64_t n_tiles) {
    extern __shared__ double smem[];
    constexpr uint64_t kRun = 64;
    const uint64_t b = (uint64_t)blockIdx.y * gridDim.x + blockIdx.x;
    const uint64_t group = b / (8 * kRun), in = b % (8 * kRun);
    const uint64_t tile = group * (8 * kRun) + (in & 7) * kRun + (in >> 3);
    if (tile >= n_tiles) return;  // whole work-group
    uint32_t lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (jobs[mid].tile0 <= tile) lo = mid;
        else hi = mid;
    }
    // the job's arguments through the constant address space: the job table
    // does not change during the launch, and loads from that space may be
    // repeated near each use (like the kernel-argument segment's) instead of
    // held in registers for the whole chain (which spilled 172 B per lane)
    const MXR_CONSTANT RunArgs &a = ((const MXR_CONSTANT BatchJob *)jobs)[lo].args;
    const DevInstr *ins = a.ins;
    const uint32_t n_mat = ins->n_mat, n_ebin = ins->n_ebin;
    double *mu_lds = smem;
    if (ins->phantom >= 0) {
        const double *T = ins->mu_em;
        const uint32_t n_mu = n_mat * n_ebin;
        for (uint32_t i = threadIdx.x; i < n_mu; i += kBlock) mu_lds[i] = T[i];
    }
    __syncthreads();
    const uint64_t ray_id = (tile - jobs[lo].tile0) * kBlock + threadIdx.x;
    if (ray_id >= a.n) return;
    const LedgerLds L{nullptr};
    Stream s;
    s.init(a.seed, ray_id, a.word3);
    Ray ray;
    ray.r[0] = ray.r[1] = ray.r[2] = 0.0;
    ray.d[0] = ray.d[1] = ray.d[2] = 0.0;
    ray.E = 0.0;
    ray.w = 0.0;
    RayEnd end{kExited, -1, -1};
    run_chain<false, false, EXACT>(C{}, ins, ray, s, ray_id, a, mu_lds, n_mat, n_ebin, end, L);
}

// The phantom's attenuation table in the form the kernels stage (run once at
// create): out[e n_mat + m] = T[m n_ebin + e] / 10, per mm and energy-major.
__global__ __launch_bounds__(kBlock) void k_mu_energy_major(const double *T, uint32_t n_mat, uint32_t n_ebin,
                                                            double *out) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_mat * n_ebin) return;
    const uint32_t m = i / n_ebin, e = i - m * n_ebin;
    out[e * n_mat + m] = T[i] * 0.1;
}

// One pass over a phantom (run once at create), one row of x per lane: the
// largest material id, and the box of the voxels whose material differs from
// the corner voxel's.  out[0] = largest id, out[1..3] = least x, y, z of such
// a voxel, out[4..6] = largest x, y, z + 1, out[7] = the corner's material
// (out[1..3] start at ~0 and out[0], out[4..6] at 0).
__global__ __launch_bounds__(kBlock) void k_phantom_scan(const uint8_t *vol, uint32_t nx, uint32_t ny, uint32_t nz,
                                                        unsigned int *out) {
    __shared__ unsigned int red[7];
    if (threadIdx.x < 7) red[threadIdx.x] = (threadIdx.x >= 1 && threadIdx.x <= 3) ? ~0u : 0u;
    __syncthreads();
    const uint32_t bg = vol[0];
    const uint32_t rows = ny * nz;
    unsigned int mx = 0, lo[3] = {~0u, ~0u, ~0u}, hi[3] = {0u, 0u, 0u};
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < rows; r += gridDim.x * kBlock) {
        const uint8_t *row = vol + (uint64_t)r * nx;
        uint32_t first = nx, last = 0;
        for (uint32_t x = 0; x < nx; ++x) {
            const uint32_t m = row[x];
            mx = m > mx ? m : mx;
            if (m != bg) {
                first = x < first ? x : first;
                last = x + 1;
            }
        }
        if (last > 0) {
            const uint32_t z = r / ny, y = r - z * ny;
            lo[0] = first < lo[0] ? first : lo[0];
            hi[0] = last > hi[0] ? last : hi[0];
            lo[1] = y < lo[1] ? y : lo[1];
            hi[1] = y + 1 > hi[1] ? y + 1 : hi[1];
            lo[2] = z < lo[2] ? z : lo[2];
            hi[2] = z + 1 > hi[2] ? z + 1 : hi[2];
        }
    }
    atomicMax(&red[0], mx);
    for (int d = 0; d < 3; ++d) {
        atomicMin(&red[1 + d], lo[d]);
        atomicMax(&red[4 + d], hi[d]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMax(out, red[0]);
        for (int d = 0; d < 3; ++d) {
            atomicMin(out + 1 + d, red[1 + d]);
            atomicMax(out + 4 + d, red[4 + d]);
        }
        if (blockIdx.x == 0) out[7] = bg;
    }
}

// ------------------------------------------------------------- recipes --

using ChainGeneric = Chain<kDynamic>;
using ChainBasic = Chain<MXR_SRC_RECT_CONE, MXR_SLIT, MXR_BOX, MXR_DETECTOR>;
using ChainEdct = Chain<MXR_SRC_CONE_BEAM, MXR_PHANTOM, MXR_DETECTOR>;
using ChainBeamline = Chain<MXR_SRC_GAUSSIAN, MXR_MIRROR_ELLIPTIC, MXR_DCM, MXR_POWDER, MXR_DETECTOR>;
// the projection behind an aperture that passes exactly the rays bound for the
// detector (a geometric early-out: the others end before the phantom)
using ChainEdctAimed = Chain<MXR_SRC_CONE_BEAM, MXR_SLIT, MXR_PHANTOM, MXR_DETECTOR>;
using ChainEdctProposal = Chain<kSrcConeProposal, MXR_PHANTOM, MXR_DETECTOR>;
using ChainEdctCollect = Chain<MXR_SRC_CONE_BEAM, MXR_PHANTOM, kDetectorCollect>;
using ChainEdctStep = Chain<MXR_SRC_CONE_BEAM, kPhantomStep, MXR_DETECTOR>;
using ChainEdctScatter = Chain<MXR_SRC_CONE_BEAM, kPhantomScatter, MXR_DETECTOR>;
using ChainCrl = Chain<MXR_SRC_GAUSSIAN, MXR_SLIT, MXR_LENS_CRL, MXR_SLIT, MXR_DETECTOR, MXR_DETECTOR>;

// their compacting forms: compaction after the crop aperture (component 1),
// small monitors in work-group private LDS
using ChainCrlCompact = Chain<MXR_SRC_GAUSSIAN, MXR_SLIT, MXR_LENS_CRL, MXR_SLIT, kDetectorLds, kDetectorLds>;
using ChainBasicCompact = Chain<MXR_SRC_RECT_CONE, MXR_SLIT, MXR_BOX, kDetectorLds>;
template <>
struct CompactCut<ChainCrlCompact> {
    static constexpr int value = 1;
};
template <>
struct CompactCut<ChainBasicCompact> {
    static constexpr int value = 1;
};

enum Recipe {
    kRecipeGeneric = 0,
    kRecipeBasic,
    kRecipeEdct,
    kRecipeBeamline,
    kRecipeEdctStep,
    kRecipeCrl,
    kRecipeEdctScatter,
    kRecipeEdctAimed,
    kNumRecipes
};

typedef void (*KernelFn)(const MXR_CONSTANT_PARAM DevInstr *, RunArgs);

template <class C, bool EXACT>
struct KernelSet {
    static KernelFn get(bool ledger, bool trace) {
        if (trace) return ledger ? k_trace<C, true, true, EXACT> : k_trace<C, false, true, EXACT>;
        return ledger ? k_trace<C, true, false, EXACT> : k_trace<C, false, false, EXACT>;
    }
    // the plain run kernel compiled for another occupancy (waves per SIMD;
    // 0: the chain's own)
    static KernelFn plain(uint32_t waves) {
        switch (waves) {
            case 4: return k_trace<C, false, false, EXACT, 4>;
            case 6: return k_trace<C, false, false, EXACT, 6>;
            case 8: return k_trace<C, false, false, EXACT, 8>;
            default: return k_trace<C, false, false, EXACT>;
        }
    }
};

// plain run kernel of a fixed chain at an occupancy, or nullptr (generic chain)
KernelFn pick_plain(int recipe, bool exact, uint32_t waves) {
    switch (recipe) {
        case kRecipeBasic: return KernelSet<ChainBasic, true>::plain(waves);
        case kRecipeEdct: return exact ? KernelSet<ChainEdct, true>::plain(waves) : KernelSet<ChainEdct, false>::plain(waves);
        case kRecipeBeamline: return KernelSet<ChainBeamline, true>::plain(waves);
        case kRecipeEdctStep: return KernelSet<ChainEdctStep, true>::plain(waves);
        case kRecipeCrl: return KernelSet<ChainCrl, true>::plain(waves);
        case kRecipeEdctScatter:
            return exact ? KernelSet<ChainEdctScatter, true>::plain(waves) : KernelSet<ChainEdctScatter, false>::plain(waves);
        case kRecipeEdctAimed: return exact ? KernelSet<ChainEdctAimed, true>::plain(waves) : nullptr;
        default: return nullptr;
    }
}

enum RunMode { kModePlain = 0, kModeProposal, kModeCollect, kModeProposalCollect };

// exact: the phantom's planes are reached exactly by adding the voxel edge
// (chains without a phantom ignore it)
KernelFn pick_kernel(int recipe, bool ledger, bool trace, bool exact, int mode) {
    if (mode != kModePlain) {
        if (recipe == kRecipeEdct && mode == kModeProposal)
            return exact ? KernelSet<ChainEdctProposal, true>::get(ledger, trace)
                         : KernelSet<ChainEdctProposal, false>::get(ledger, trace);
        if (recipe == kRecipeEdct && mode == kModeCollect && !trace)
            return exact ? KernelSet<ChainEdctCollect, true>::get(ledger, false)
                         : KernelSet<ChainEdctCollect, false>::get(ledger, false);
        // any other combination (e.g. a proposal while collecting) dispatches
        // both on the run's arguments
        return exact ? KernelSet<ChainGeneric, true>::get(ledger, trace) : KernelSet<ChainGeneric, false>::get(ledger, trace);
    }
    switch (recipe) {
        case kRecipeBasic: return KernelSet<ChainBasic, true>::get(ledger, trace);
        case kRecipeEdct:
            return exact ? KernelSet<ChainEdct, true>::get(ledger, trace) : KernelSet<ChainEdct, false>::get(ledger, trace);
        case kRecipeBeamline: return KernelSet<ChainBeamline, true>::get(ledger, trace);
        case kRecipeEdctStep: return KernelSet<ChainEdctStep, true>::get(ledger, trace);
        case kRecipeCrl: return KernelSet<ChainCrl, true>::get(ledger, trace);
        case kRecipeEdctScatter:
            return exact ? KernelSet<ChainEdctScatter, true>::get(ledger, trace)
                         : KernelSet<ChainEdctScatter, false>::get(ledger, trace);
        case kRecipeEdctAimed:
            // plain runs only; ledgers and ray traces take the generic chain
            if (exact && !ledger && !trace) return k_trace<ChainEdctAimed, false, false, true>;
            return exact ? KernelSet<ChainGeneric, true>::get(ledger, trace)
                         : KernelSet<ChainGeneric, false>::get(ledger, trace);
        default:
            return exact ? KernelSet<ChainGeneric, true>::get(ledger, trace)
                         : KernelSet<ChainGeneric, false>::get(ledger, trace);
    }
}

// the compacting kernel for plain runs of a chain with a compaction prefix,
// or nullptr
KernelFn pick_compact(int recipe) {
    switch (recipe) {
        case kRecipeBasic: return k_trace_compact<ChainBasicCompact, true>;
        case kRecipeCrl: return k_trace_compact<ChainCrlCompact, true>;
        default: return nullptr;
    }
}

typedef void (*BatchKernelFn)(const BatchJob *, uint32_t, uint64_t, uint32_t, unsigned long long *);
typedef void (*BatchGridFn)(const BatchJob *, uint32_t, uint64_t);

BatchGridFn pick_batch_grid(int recipe, bool exact) {
    switch (recipe) {
        case kRecipeBasic: return k_batch_grid<ChainBasic, true>;
        case kRecipeEdct: return exact ? k_batch_grid<ChainEdct, true> : k_batch_grid<ChainEdct, false>;
        case kRecipeBeamline: return k_batch_grid<ChainBeamline, true>;
        default: return exact ? k_batch_grid<ChainGeneric, true> : k_batch_grid<ChainGeneric, false>;
    }
}

BatchKernelFn pick_batch_kernel(int recipe, bool exact) {
    switch (recipe) {
        case kRecipeBasic: return k_batch<ChainBasic, true>;
        case kRecipeEdct: return exact ? k_batch<ChainEdct, true> : k_batch<ChainEdct, false>;
        case kRecipeBeamline: return k_batch<ChainBeamline, true>;
        default: return exact ? k_batch<ChainGeneric, true> : k_batch<ChainGeneric, false>;
    }
}

int match_recipe(const DevInstr &d) {
    auto is = [&](std::initializer_list<int> seq) {
        if (d.ncomp != seq.size()) return false;
        int k = 0;
        for (int t : seq)
            if ((int)d.c[k++].type != t) return false;
        return true;
    };
    if (is({MXR_SRC_RECT_CONE, MXR_SLIT, MXR_BOX, MXR_DETECTOR})) return kRecipeBasic;
    if (is({MXR_SRC_CONE_BEAM, MXR_PHANTOM, MXR_DETECTOR}))
        return (d.c[1].flags & 2u) ? kRecipeEdctScatter : ((d.c[1].flags & 1u) ? kRecipeEdctStep : kRecipeEdct);
    if (is({MXR_SRC_CONE_BEAM, MXR_SLIT, MXR_PHANTOM, MXR_DETECTOR}) && d.c[2].flags == 0) return kRecipeEdctAimed;
    if (is({MXR_SRC_GAUSSIAN, MXR_MIRROR_ELLIPTIC, MXR_DCM, MXR_POWDER, MXR_DETECTOR})) return kRecipeBeamline;
    if (is({MXR_SRC_GAUSSIAN, MXR_SLIT, MXR_LENS_CRL, MXR_SLIT, MXR_DETECTOR, MXR_DETECTOR})) return kRecipeCrl;
    return kRecipeGeneric;
}

// --------------------------------------------------------------- errors --

thread_local std::string g_error = "no error";

mxr_status fail(mxr_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

mxr_status hip_fail(hipError_t e, const char *what) {
    return fail(MXR_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool finite_all(const double *p, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

bool is_source(uint32_t t) { return t == MXR_SRC_RECT_CONE || t == MXR_SRC_CONE_BEAM || t == MXR_SRC_GAUSSIAN; }

int draws_of(const mxr_component_desc &s) {
    switch (s.type) {
        case MXR_SRC_RECT_CONE: return 5;
        case MXR_SRC_CONE_BEAM: return 3;
        case MXR_SRC_GAUSSIAN: return 5;
        case MXR_POWDER: return 2;
        case MXR_PHANTOM: return (s.flags & 2u) ? 4 * (int)s.par[4] : 0;  // four per forced interaction
        default: return 0;
    }
}

}  // namespace

// error reporting shared with the other translation units of the library
namespace mxr_host {
mxr_status set_error(mxr_status st, const char *msg) {
    g_error = msg;
    return st;
}
}  // namespace mxr_host

struct mxr_instrument {
    mxr_launch_shape shape{0, 1, 0, 0};  // plain runs' launch shape (see mxr_set_launch_shape)
    uint32_t order = 0;                  // XCD order of the other runs (see tile_of)
    int device;
    DevInstr host;
    DevInstr *dev;
    int recipe;
    uint32_t n_det;
    uint64_t det_bins[MXR_MAX_DETECTORS];
    uint64_t strata;      // G of the cone-beam source, 0 if none
    int n_cu;             // compute units of the device
    PropTable *prop_dev;  // proposal mixture (device), allocated on first use
    double *mu_dev;       // the phantom's staged attenuation table (device), or null
    PropTable prop_host;  // its host copy (branch sizes are set per run)
    bool prop_on;
};

// Derive per-component constants on the host (glibc), validate ranges.
static mxr_status derive(const mxr_component_desc &s, DevComp &c, int k, uint32_t &n_mat, uint32_t &n_ebin) {
    c.type = s.type;
    c.flags = s.flags;
    std::memcpy(c.pos, s.pos, sizeof c.pos);
    std::memcpy(c.rot, s.rot, sizeof c.rot);
    std::memcpy(c.par, s.par, sizeof c.par);
    std::memset(c.aux, 0, sizeof c.aux);
    c.data0 = s.data[0];
    c.data1 = s.data[1];
    c.n0 = s.data_len[0];
    c.n1 = s.data_len[1];
    std::memcpy(c.dims, s.dims, sizeof c.dims);
    if (!finite_all(s.pos, 3) || !finite_all(s.rot, 9) || !finite_all(s.par, 16))
        return fail(MXR_E_INVALID, "component %d: non-finite position, rotation or parameter", k);
    const double *p = s.par;
    switch (s.type) {
        case MXR_SRC_RECT_CONE:
            if (!(p[0] >= 0 && p[1] >= 0 && p[2] > 0 && p[2] < kPi && p[4] > p[3] && p[3] > 0))
                return fail(MXR_E_INVALID, "component %d: bad rectangular source parameters", k);
            c.aux[0] = std::sin(0.5 * p[2]);
            c.aux[1] = p[4] - p[3];
            break;
        case MXR_SRC_CONE_BEAM:
            if (!(p[0] > 0 && p[0] < kPi && p[2] > p[1] && p[1] > 0 && p[3] >= p[2] && p[9] > 0))
                return fail(MXR_E_INVALID, "component %d: bad cone-beam source parameters", k);
            if (s.dims[0] < 1 || s.dims[0] > 65536)
                return fail(MXR_E_INVALID, "component %d: strata per side must be in [1, 65536]", k);
            c.aux[0] = std::sin(0.5 * p[0]);
            c.aux[1] = p[2] - p[1];
            c.aux[2] = p[3] * std::log(p[2] / p[1]) - (p[2] - p[1]);
            c.aux[3] = p[9] * std::sqrt(2.0 * M_PI);
            c.aux[4] = 1.0 / p[9];
            c.aux[5] = 1.0 / c.aux[3];
            c.aux[6] = p[4] / c.aux[2];
            c.aux[7] = 1.0 / c.aux[1];
            break;
        case MXR_SRC_GAUSSIAN:
            if (!(p[0] >= 0 && p[1] >= 0 && p[2] >= 0 && p[3] >= 0 && p[4] > 0 && p[5] >= 0 && p[5] < 1))
                return fail(MXR_E_INVALID, "component %d: bad Gaussian source parameters", k);
            break;
        case MXR_SLIT:
            if (s.flags & 1u) {
                if (!(p[2] >= 0)) return fail(MXR_E_INVALID, "component %d: bad slit radius", k);
                c.aux[2] = p[2] * p[2];
            } else {
                if (!(p[0] >= 0 && p[1] >= 0)) return fail(MXR_E_INVALID, "component %d: bad slit size", k);
                c.aux[0] = 0.5 * p[0];
                c.aux[1] = 0.5 * p[1];
            }
            break;
        case MXR_BOX:
            if (!(p[0] > 0 && p[1] > 0 && p[2] > 0)) return fail(MXR_E_INVALID, "component %d: bad box size", k);
            break;
        case MXR_PHANTOM: {
            if (!s.data[0] || !s.data[1]) return fail(MXR_E_INVALID, "component %d: phantom needs volume and mu table", k);
            uint64_t nvox = (uint64_t)s.dims[0] * s.dims[1] * s.dims[2];
            if (s.dims[0] < 1 || s.dims[1] < 1 || s.dims[2] < 1 || nvox != s.data_len[0])
                return fail(MXR_E_INVALID, "component %d: volume size does not match dims", k);
            if (nvox >= (1ull << 31) || s.dims[0] + s.dims[1] + s.dims[2] > (1u << 20))
                return fail(MXR_E_UNSUPPORTED, "component %d: volume too large", k);
            if (s.dims[3] < 1 || s.dims[3] > 16) return fail(MXR_E_UNSUPPORTED, "component %d: 1..16 materials", k);
            if (s.flags & ~7u) return fail(MXR_E_INVALID, "component %d: unknown phantom flags", k);
            if ((s.flags & 3u) == 3u || (s.flags & 6u) == 4u)
                return fail(MXR_E_INVALID, "component %d: phantom flags: scattering excludes the fixed-step model, aiming needs scattering", k);
            // a scattering phantom's table holds three channels (total, Rayleigh, Compton)
            const uint64_t per_mat = (s.flags & 2u) ? 3ull * s.dims[3] : (uint64_t)s.dims[3];
            if (s.data_len[1] % per_mat != 0 || s.data_len[1] / per_mat < 1 || s.data_len[1] / per_mat > 256)
                return fail(MXR_E_UNSUPPORTED, "component %d: 1..256 energy bins per material", k);
            if (!(p[0] > 0 && p[2] > p[1])) return fail(MXR_E_INVALID, "component %d: bad voxel size or table range", k);
            if (s.flags & 2u) {
                if (!(p[4] >= 1 && p[4] <= 3 && p[4] == std::floor(p[4])))
                    return fail(MXR_E_INVALID, "component %d: scatter order must be 1, 2 or 3", k);
                if (s.flags & 4u) {
                    const double *a = p + 8, *b = p + 11;
                    const double n0 = a[1] * b[2] - a[2] * b[1], n1 = a[2] * b[0] - a[0] * b[2],
                                 n2 = a[0] * b[1] - a[1] * b[0];
                    if (!(n0 * n0 + n1 * n1 + n2 * n2 > 0))
                        return fail(MXR_E_INVALID, "component %d: degenerate scatter target", k);
                }
            }
            if (s.flags & 1u) {
                // fixed-step model: bound the steps of the longest chord
                if (!(p[3] > 0)) return fail(MXR_E_INVALID, "component %d: step length must be positive", k);
                const double diag = p[0] * std::sqrt((double)s.dims[0] * s.dims[0] + (double)s.dims[1] * s.dims[1] +
                                                     (double)s.dims[2] * s.dims[2]);
                const double jmax = std::ceil(diag / p[3]) + 2.0;
                if (!(jmax <= (double)(1 << 26)))
                    return fail(MXR_E_UNSUPPORTED, "component %d: more than 2^26 steps per chord", k);
                if ((uint64_t)s.dims[1] * s.dims[2] >= (1ull << 24))
                    return fail(MXR_E_UNSUPPORTED, "component %d: fixed-step model needs ny * nz < 2^24", k);
                c.aux[5] = jmax;
            }
            n_mat = s.dims[3];
            n_ebin = (uint32_t)(s.data_len[1] / per_mat);
            for (int i = 0; i < 3; ++i) c.aux[i] = -0.5 * ((double)s.dims[i] * p[0]);
            c.aux[3] = (double)n_ebin / (p[2] - p[1]);
            c.aux[6] = 1.0 / p[0];
            // can the walk step planes by adding v and stay exact?
            bool exact = true;
            for (int i = 0; i < 3 && exact; ++i) {
                double P = c.aux[i];
                for (uint32_t k = 1; k <= s.dims[i]; ++k) {
                    P = P + p[0];
                    if (P != c.aux[i] + (double)k * p[0]) {
                        exact = false;
                        break;
                    }
                }
            }
            c.aux[4] = exact ? 1.0 : 0.0;
            break;
        }
        case MXR_LENS_CRL: {
            // 0 R, 1 N, 2 on-axis thickness w, 3 pitch, 4 aperture radius,
            // 5 delta at 6 E ref, 7-8 mu = a / E^3 + b
            if (!(p[0] > 0 && p[1] >= 1 && p[1] <= 1024 && p[1] == std::floor(p[1]) && p[2] >= 0 && p[4] > 0 &&
                  p[5] >= 0 && p[5] < 0.5 && p[6] > 0 && p[7] >= 0 && p[8] >= 0))
                return fail(MXR_E_INVALID, "component %d: bad lens parameters", k);
            if (!(p[3] >= p[2] + p[4] * p[4] / p[0]))
                return fail(MXR_E_INVALID, "component %d: lens pitch below w + r_a^2 / R (lenses would overlap)", k);
            c.aux[0] = 1.0 / p[0];
            c.aux[1] = 1.0 / (2.0 * p[0]);
            c.aux[2] = p[4] * p[4];
            break;
        }
        case MXR_MIRROR_ELLIPTIC: {
            double P = p[0], Q = p[1], t0 = p[2];
            if (!(P > 0 && Q > 0 && t0 > 0 && t0 < 0.5 && p[3] > 0 && p[4] > 0 && p[5] > 0) || !s.data[0] ||
                s.data_len[0] < 2)
                return fail(MXR_E_INVALID, "component %d: bad mirror parameters", k);
            double a = 0.5 * (P + Q);
            double b2 = P * Q * (std::sin(t0) * std::sin(t0));
            double F2y = Q * std::sin(2.0 * t0), F2z = Q * std::cos(2.0 * t0);
            double fy = F2y, fz = F2z + P;
            double two_c = std::sqrt(fy * fy + fz * fz);
            double uy = fy / two_c, uz = fz / two_c;
            c.aux[0] = 0.5 * F2y;
            c.aux[1] = 0.5 * (F2z - P);
            c.aux[2] = uy;
            c.aux[3] = uz;
            c.aux[4] = uz;
            c.aux[5] = -uy;
            c.aux[6] = 1.0 / (a * a);
            c.aux[7] = 1.0 / b2;
            c.aux[8] = std::sin(t0);
            c.aux[9] = std::cos(t0);
            c.aux[10] = 0.5 * p[3];
            c.aux[11] = 0.5 * p[4];
            c.aux[12] = p[5] / (double)(s.data_len[0] - 1);
            break;
        }
        case MXR_DCM: {
            if (!(p[0] > 0 && p[1] > 0 && p[1] < 0.5 * kPi && p[2] > 0 && p[3] > 0))
                return fail(MXR_E_INVALID, "component %d: bad monochromator parameters", k);
            double n1[3] = {0.0, std::cos(p[1]), -std::sin(p[1])};
            for (int i = 0; i < 3; ++i) {
                c.aux[i] = n1[i];
                c.aux[3 + i] = -n1[i];
                c.aux[6 + i] = p[3] * n1[i];
            }
            c.aux[9] = 2.0 * p[0];
            c.aux[10] = 0.5 * p[2];
            break;
        }
        case MXR_POWDER:
            if (!(p[0] >= 0 && p[1] >= 0) || !s.data[0] || s.data_len[0] < 1)
                return fail(MXR_E_INVALID, "component %d: bad powder parameters", k);
            c.aux[0] = 0.5 * p[0];
            c.aux[1] = 0.5 * p[1];
            break;
        case MXR_DETECTOR:
            if (s.dims[0] < 1 || s.dims[1] < 1 || s.dims[2] < 1 || !(p[1] > p[0] && p[3] > p[2] && p[5] > p[4]))
                return fail(MXR_E_INVALID, "component %d: bad monitor binning", k);
            c.aux[0] = (double)s.dims[0] / (p[1] - p[0]);
            c.aux[1] = (double)s.dims[1] / (p[3] - p[2]);
            c.aux[2] = (double)s.dims[2] / (p[5] - p[4]);
            break;
        default:
            return fail(MXR_E_INVALID, "component %d: unknown type %u", k, s.type);
    }
    return MXR_OK;
}

// Box of the proposal coordinates y = (u, v, E) of a cone-beam source:
// u = dx/dz and v = dy/dz reach tan(half-angle) on the cone's rim, and the
// energy is drawn on [E min, E max].
static void proposal_box(const DevComp &c, double lo[3], double hi[3]) {
    const double t = std::tan(c.par[0]);
    lo[0] = lo[1] = -t;
    hi[0] = hi[1] = t;
    lo[2] = c.par[1];
    hi[2] = c.par[2];
}

extern "C" {

uint32_t mxr_abi_version(void) { return MXR_ABI_VERSION; }

const char *mxr_last_error(void) { return g_error.c_str(); }

mxr_status mxr_instrument_create(const mxr_instrument_desc *desc, mxr_instrument **out) {
    if (!desc || !out) return fail(MXR_E_INVALID, "null descriptor or output pointer");
    *out = nullptr;
    if (desc->abi_version != MXR_ABI_VERSION)
        return fail(MXR_E_INVALID, "descriptor ABI version %u, library %u", desc->abi_version, MXR_ABI_VERSION);
    if (desc->n_components < 1 || desc->n_components > MXR_MAX_COMPONENTS || !desc->components)
        return fail(MXR_E_INVALID, "need 1..%u components", MXR_MAX_COMPONENTS);
    mxr_instrument *ins = new (std::nothrow) mxr_instrument();
    if (!ins) return fail(MXR_E_NOMEM, "host allocation failed");
    std::memset(&ins->host, 0, sizeof ins->host);
    DevInstr &d = ins->host;
    d.ncomp = desc->n_components;
    d.phantom = -1;
    uint32_t draw = 0, n_det = 0, n_phantom = 0;
    for (uint32_t k = 0; k < desc->n_components; ++k) {
        const mxr_component_desc &s = desc->components[k];
        if ((k == 0) != is_source(s.type)) {
            delete ins;
            return fail(MXR_E_INVALID, "component %u: the first component, and only it, must be a source", k);
        }
        uint32_t nm = 0, ne = 0;
        mxr_status st = derive(s, d.c[k], (int)k, nm, ne);
        if (st != MXR_OK) {
            delete ins;
            return st;
        }
        d.c[k].draw0 = draw;
        draw += draws_of(s);
        if (s.type == MXR_PHANTOM) {
            if (++n_phantom > 1) {
                delete ins;
                return fail(MXR_E_UNSUPPORTED, "at most one phantom per instrument");
            }
            d.phantom = (int32_t)k;
            d.n_mat = nm;
            d.n_ebin = ne;
        }
        if (s.type == MXR_DETECTOR) {
            if (n_det >= MXR_MAX_DETECTORS) {
                delete ins;
                return fail(MXR_E_UNSUPPORTED, "at most %u monitors", MXR_MAX_DETECTORS);
            }
            d.c[k].slot = n_det;
            ins->det_bins[n_det] = (uint64_t)s.dims[0] * s.dims[1] * s.dims[2];
            n_det++;
        }
        if (s.type == MXR_SRC_CONE_BEAM) ins->strata = s.dims[0];
    }
    ins->n_det = n_det;
    ins->recipe = match_recipe(d);
    // launch order spreads a phantom's bands of unequal path length over the
    // XCDs; without a phantom the per-XCD blocks of neighbouring rays keep
    // their tally updates in one L2 and measured faster
    ins->order = d.phantom >= 0 ? 1u : 0u;
    ins->shape.xcd_order = ins->order;
    hipError_t e = hipGetDevice(&ins->device);
    if (e != hipSuccess) {
        delete ins;
        return hip_fail(e, "hipGetDevice");
    }
    if (hipDeviceGetAttribute(&ins->n_cu, hipDeviceAttributeMultiprocessorCount, ins->device) != hipSuccess ||
        ins->n_cu < 1)
        ins->n_cu = 256;
    ins->mu_dev = nullptr;
    if (d.phantom >= 0) {
        const uint32_t n_mu = d.n_mat * d.n_ebin;
        e = hipMalloc((void **)&ins->mu_dev, (size_t)n_mu * sizeof(double));
        if (e != hipSuccess) {
            delete ins;
            return fail(MXR_E_NOMEM, "hipMalloc of the attenuation table: %s", hipGetErrorString(e));
        }
        hipLaunchKernelGGL(k_mu_energy_major, dim3((n_mu + kBlock - 1) / kBlock), dim3(kBlock), 0, 0,
                           (const double *)d.c[d.phantom].data1, d.n_mat, d.n_ebin, ins->mu_dev);
        e = hipGetLastError();
        if (e != hipSuccess) {
            (void)hipFree(ins->mu_dev);
            delete ins;
            return hip_fail(e, "attenuation table launch");
        }
        d.mu_em = ins->mu_dev;
    }
    if (d.phantom >= 0) {
        // one pass over the volume: every material id must index the mu
        // table, and the box of voxels unlike the corner bounds the walk
        DevComp &c = d.c[d.phantom];
        unsigned int *dscan = nullptr, hs[8] = {0u, ~0u, ~0u, ~0u, 0u, 0u, 0u, 0u};
        e = hipMalloc((void **)&dscan, sizeof hs);
        if (e == hipSuccess) e = hipMemcpy(dscan, hs, sizeof hs, hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            const uint64_t rows = (uint64_t)c.dims[1] * c.dims[2];
            const uint64_t nb = std::min<uint64_t>((rows + kBlock - 1) / kBlock, 4096);
            hipLaunchKernelGGL(k_phantom_scan, dim3((unsigned)nb), dim3(kBlock), 0, 0, (const uint8_t *)c.data0,
                               c.dims[0], c.dims[1], c.dims[2], dscan);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpy(hs, dscan, sizeof hs, hipMemcpyDeviceToHost);
        if (dscan) (void)hipFree(dscan);
        if (e != hipSuccess) {
            (void)hipFree(ins->mu_dev);
            delete ins;
            return hip_fail(e, "phantom scan");
        }
        if (hs[0] >= d.n_mat) {
            (void)hipFree(ins->mu_dev);
            delete ins;
            return fail(MXR_E_INVALID, "phantom holds material id %u but the table has %u materials", hs[0], d.n_mat);
        }
        // box planes as the walk places them: corner + k v
        const bool any = hs[4] > 0;
        for (int i = 0; i < 3; ++i) {
            c.aux[8 + i] = c.aux[i] + (double)(any ? hs[1 + i] : 0u) * c.par[0];
            c.aux[11 + i] = c.aux[i] + (double)(any ? hs[4 + i] : 0u) * c.par[0];
        }
        c.aux[14] = (double)hs[7];
        c.aux[15] = any ? 1.0 : 0.0;
    }
    e = hipMalloc((void **)&ins->dev, sizeof(DevInstr));
    if (e != hipSuccess) {
        if (ins->mu_dev) (void)hipFree(ins->mu_dev);
        delete ins;
        return fail(MXR_E_NOMEM, "hipMalloc of the instrument block: %s", hipGetErrorString(e));
    }
    e = hipMemcpy(ins->dev, &d, sizeof(DevInstr), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(ins->dev);
        if (ins->mu_dev) (void)hipFree(ins->mu_dev);
        delete ins;
        return hip_fail(e, "hipMemcpy of the instrument block");
    }
    *out = ins;
    return MXR_OK;
}

void mxr_instrument_destroy(mxr_instrument *ins) {
    if (!ins) return;
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != ins->device) (void)hipSetDevice(ins->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(ins->dev);
    if (ins->prop_dev) (void)hipFree(ins->prop_dev);
    if (ins->mu_dev) (void)hipFree(ins->mu_dev);
    if (cur >= 0 && cur != ins->device) (void)hipSetDevice(cur);
    delete ins;
}

static mxr_status launch(mxr_instrument *ins, const RunArgs &base, uint64_t n, bool ledger, bool trace,
                         hipStream_t stream) {
    const bool exact = ins->host.phantom < 0 || ins->host.c[ins->host.phantom].aux[4] != 0.0;
    const int mode = base.hits.count ? (base.prop ? kModeProposalCollect : kModeCollect)
                                     : (base.prop ? kModeProposal : kModePlain);
    const bool plain = !ledger && !trace && mode == kModePlain;
    KernelFn k = pick_kernel(ins->recipe, ledger, trace, exact, mode);
    if (plain && ins->shape.occupancy) {
        KernelFn ko = pick_plain(ins->recipe, exact, ins->shape.occupancy);
        if (ko) k = ko;
    }
    KernelFn kc = (plain && ins->shape.compact) ? pick_compact(ins->recipe) : nullptr;
    size_t shmem = 0;
    if (ins->host.phantom >= 0) shmem += (size_t)ins->host.n_mat * ins->host.n_ebin * sizeof(double);
    if (ledger) shmem += (size_t)(4 * ins->host.ncomp + 1) * sizeof(double);
    if (kc) {
        int32_t off[MXR_MAX_DETECTORS];
        shmem = lds_tally_layout(ins->host, off);
    }
    // one lane per ray; a launch's grid is counted in work-items with 32 bits,
    // so a launch takes at most kMaxLaunchGroups work-groups and longer ray
    // ranges are split into several launches
    const uint64_t max_rays = kMaxLaunchGroups * kBlock;
    for (uint64_t done = 0; done < n;) {
        const uint64_t m = std::min(n - done, max_rays);
        RunArgs a = base;
        a.n = m;
        if (trace) {
            a.ids = base.ids + done;
            a.dump.x = base.dump.x + done;
            a.dump.y = base.dump.y + done;
            a.dump.z = base.dump.z + done;
            a.dump.dx = base.dump.dx + done;
            a.dump.dy = base.dump.dy + done;
            a.dump.dz = base.dump.dz + done;
            a.dump.E = base.dump.E + done;
            a.dump.w = base.dump.w + done;
            a.dump.status = base.dump.status + done;
            a.dump.dead_at = base.dump.dead_at + done;
            a.dump.bin = base.dump.bin + done;
        } else {
            a.first = base.first + done;
        }
        // compacting kernel: as many rounds as keep >= 4 work-groups per CU
        // (at most the shape's rounds, when it sets them)
        a.compact_rounds = (uint32_t)std::max<uint64_t>(
            1, std::min<uint64_t>(ins->shape.rounds ? ins->shape.rounds : kCompactRounds,
                                  m / ((uint64_t)kBlock * 4 * ins->n_cu)));
        a.xcd_order = plain ? ins->shape.xcd_order : ins->order;
        const uint64_t rays_per_group = kc ? (uint64_t)kBlock * a.compact_rounds : (uint64_t)kBlock;
        const uint64_t groups = (m + rays_per_group - 1) / rays_per_group;
        a.blocks_per_xcd = (uint32_t)((groups + 7) / 8);
        const uint64_t blocks = (uint64_t)a.blocks_per_xcd * 8;
        hipLaunchKernelGGL(kc ? kc : k, dim3((unsigned)blocks), dim3(kBlock), shmem, stream,
                           (const MXR_CONSTANT_PARAM DevInstr *)ins->dev, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        done += m;
    }
    return MXR_OK;
}


// Strata per side used for n rays: the largest g <= G with 16 g^2 <= n (1 if
// none).  Every cell then holds at least 16 rays, so the 64 consecutive rays
// of a wave fall in a few neighbouring cells and leave the source in nearly
// one direction (with one ray per cell a wave would span 64 cells).
static uint64_t strata_side(uint64_t G, uint64_t n) {
    uint64_t g = G < 1 ? 1 : G;
    while (g > 1 && 16 * g * g > n) g -= 1;
    return g;
}

// Divisors of n rays stratified over G x G cells (the device's strat_cell).
static StratDiv strat_div(uint64_t n, uint64_t G) {
    StratDiv d{};
    d.n = n;
    d.G = (uint32_t)G;
    d.G2 = G * G;
    d.c0 = n / d.G2;
    d.r = n % d.G2;
    d.rn = n ? 1.0 / (double)n : 0.0;
    d.rG = 1.0 / (double)G;
    d.rG2 = 1.0 / (double)d.G2;
    const double per = (double)n / (double)d.G2;
    d.f0 = d.c0 ? per / (double)d.c0 : 0.0;
    d.f1 = per / (double)(d.c0 + 1);
    return d;
}
static mxr_status common_args(mxr_instrument *ins, uint64_t n_total, uint64_t seed, uint32_t purpose, uint32_t job,
                              RunArgs &a) {
    if (!ins) return fail(MXR_E_INVALID, "null instrument");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != ins->device) return fail(MXR_E_STATE, "instrument lives on device %d, device %d is current", ins->device, cur);
    if (purpose > 255 || job > 0xFFFFFFu) return fail(MXR_E_INVALID, "purpose must be < 256 and job < 2^24");
    if (n_total < 1) return fail(MXR_E_INVALID, "n_total must be positive");
    std::memset(&a, 0, sizeof a);
    a.ins = ins->dev;
    a.n_total = n_total;
    a.seed = seed;
    a.word3 = (purpose << 24) | job;
    a.xcd_order = ins->order;
    const uint64_t G = strata_side(ins->strata, n_total);
    a.G = G;
    a.G2 = G * G;
    // the last cell's bound (cell + 1) n_total + G^2 - 1 must not wrap
    if (a.G2 > 1 && n_total > (~0ull - (a.G2 - 1)) / a.G2)
        return fail(MXR_E_INVALID, "n_total * strata^2 + strata^2 - 1 must stay below 2^64");
    a.sd = strat_div(n_total, G);
    a.prop = ins->prop_on ? ins->prop_dev : nullptr;
    if (ins->prop_on) {
        // branch ranges of this run: plain share round(alpha n), then the
        // components by their box masses (rounded running sums)
        const PropTable &P = ins->prop_host;
        uint64_t n_plain = (uint64_t)std::floor(P.alpha * (double)n_total + 0.5);
        if (n_plain > n_total) n_plain = n_total;
        a.pb[0] = n_plain;
        double cum = 0.0;
        for (int k = 0; k < 8; ++k) {
            cum += P.mass[k];
            uint64_t b = P.norm > 0.0 ? n_plain + (uint64_t)std::floor((double)(n_total - n_plain) * (cum / P.norm) + 0.5)
                                      : n_total;
            a.pb[k + 1] = b > n_total ? n_total : b;
        }
        a.pb[8] = n_total;
        const uint64_t gmax = ins->strata ? ins->strata : 1;
        for (int b = 0; b < 9; ++b) {
            const uint64_t cnt = a.pb[b] - (b ? a.pb[b - 1] : 0);
            const uint64_t g = strata_side(gmax, cnt);
            a.psd[b] = strat_div(cnt, g);
            a.pc[b] = (double)cnt / (double)n_total;
        }
    }
    return MXR_OK;
}

static mxr_status check_tallies(mxr_instrument *ins, const mxr_tally *tallies, uint32_t n_tallies, RunArgs &a) {
    if (n_tallies != ins->n_det) return fail(MXR_E_INVALID, "%u tallies given, instrument has %u monitors", n_tallies, ins->n_det);
    if (n_tallies && !tallies) return fail(MXR_E_INVALID, "null tallies");
    for (uint32_t i = 0; i < n_tallies; ++i) {
        if (!tallies[i].count || !tallies[i].sum_w || !tallies[i].sum_w2)
            return fail(MXR_E_INVALID, "tally %u has a null array", i);
        if (tallies[i].n_bins != ins->det_bins[i])
            return fail(MXR_E_INVALID, "tally %u has %llu bins, monitor needs %llu", i,
                        (unsigned long long)tallies[i].n_bins, (unsigned long long)ins->det_bins[i]);
        a.tally.count[i] = (unsigned long long *)tallies[i].count;
        a.tally.sum_w[i] = tallies[i].sum_w;
        a.tally.sum_w2[i] = tallies[i].sum_w2;
    }
    return MXR_OK;
}

mxr_status mxr_run(mxr_instrument *ins, uint64_t first_ray, uint64_t n_rays, uint64_t n_total, uint64_t seed,
                   uint32_t purpose, uint32_t job, const mxr_tally *tallies, uint32_t n_tallies, double *ledger,
                   void *hip_stream) {
    RunArgs a;
    mxr_status st = common_args(ins, n_total, seed, purpose, job, a);
    if (st != MXR_OK) return st;
    if (first_ray > n_total || n_rays > n_total - first_ray)
        return fail(MXR_E_INVALID, "rays [%llu, %llu) exceed n_total %llu", (unsigned long long)first_ray,
                    (unsigned long long)(first_ray + n_rays), (unsigned long long)n_total);
    st = check_tallies(ins, tallies, n_tallies, a);
    if (st != MXR_OK) return st;
    if (n_rays == 0) return MXR_OK;
    a.first = first_ray;
    a.n = n_rays;
    a.ledger = ledger;
    return launch(ins, a, n_rays, ledger != nullptr, false, (hipStream_t)hip_stream);
}

mxr_status mxr_collect(mxr_instrument *ins, uint64_t first_ray, uint64_t n_rays, uint64_t n_total, uint64_t seed,
                       uint32_t purpose, uint32_t job, const mxr_tally *tallies, uint32_t n_tallies,
                       const mxr_hits *hits, void *hip_stream) {
    RunArgs a;
    mxr_status st = common_args(ins, n_total, seed, purpose, job, a);
    if (st != MXR_OK) return st;
    if (first_ray > n_total || n_rays > n_total - first_ray)
        return fail(MXR_E_INVALID, "rays [%llu, %llu) exceed n_total %llu", (unsigned long long)first_ray,
                    (unsigned long long)(first_ray + n_rays), (unsigned long long)n_total);
    st = check_tallies(ins, tallies, n_tallies, a);
    if (st != MXR_OK) return st;
    if (!hits || !hits->ctx || !hits->y || !hits->w || !hits->bin || !hits->count)
        return fail(MXR_E_INVALID, "null hit sink array");
    const DevInstr &d = ins->host;
    if (d.c[0].type != MXR_SRC_CONE_BEAM) return fail(MXR_E_UNSUPPORTED, "hit collection needs a cone-beam source");
    if (ins->n_det != 1 || d.c[d.ncomp - 1].type != MXR_DETECTOR)
        return fail(MXR_E_UNSUPPORTED, "hit collection needs exactly one monitor, the last component");
    for (uint32_t k = 1; k + 1 < d.ncomp; ++k) {
        const uint32_t t = d.c[k].type;
        if ((t != MXR_SLIT && t != MXR_BOX && t != MXR_PHANTOM) || (t == MXR_PHANTOM && (d.c[k].flags & 2u)))
            return fail(MXR_E_UNSUPPORTED, "hit collection: component %u changes direction or energy", k);
    }
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(hits->context[i])) return fail(MXR_E_INVALID, "non-finite context");
    if (n_rays == 0) return MXR_OK;
    a.hits.ctx = hits->ctx;
    a.hits.y = hits->y;
    a.hits.w = hits->w;
    a.hits.bin = hits->bin;
    a.hits.count = (unsigned long long *)hits->count;
    a.hits.capacity = hits->capacity;
    for (int i = 0; i < 6; ++i) a.hits.c[i] = hits->context[i];
    a.first = first_ray;
    a.n = n_rays;
    return launch(ins, a, n_rays, false, false, (hipStream_t)hip_stream);
}

mxr_status mxr_proposal_box(const mxr_instrument *ins, double lo[3], double hi[3]) {
    if (!ins || !lo || !hi) return fail(MXR_E_INVALID, "null instrument or box");
    if (ins->host.c[0].type != MXR_SRC_CONE_BEAM) return fail(MXR_E_UNSUPPORTED, "a proposal needs a cone-beam source");
    proposal_box(ins->host.c[0], lo, hi);
    return MXR_OK;
}

mxr_status mxr_proposal_set(mxr_instrument *ins, const double *gmm, double alpha) {
    if (!ins) return fail(MXR_E_INVALID, "null instrument");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != ins->device) return fail(MXR_E_STATE, "instrument lives on device %d, device %d is current", ins->device, cur);
    if (!gmm) {
        ins->prop_on = false;
        return MXR_OK;
    }
    const DevInstr &d = ins->host;
    if (d.c[0].type != MXR_SRC_CONE_BEAM) return fail(MXR_E_UNSUPPORTED, "a proposal needs a cone-beam source");
    if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(MXR_E_INVALID, "alpha must be in [0, 1]");
    double g[56];
    e = hipMemcpy(g, gmm, sizeof g, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "copy of the mixture table");
    const DevComp &c = d.c[0];
    PropTable P;
    std::memset(&P, 0, sizeof P);
    double lo[3], hi[3];
    proposal_box(c, lo, hi);
    const double t = hi[0];
    double run = 0.0;
    for (int k = 0; k < 8; ++k) {
        const double *gk = g + 7 * k;
        if (!std::isfinite(gk[0]) || gk[0] < 0.0) return fail(MXR_E_INVALID, "component %d: bad weight", k);
        double Z = gk[0], F = 1.0, sprod = 1.0;
        for (int dd = 0; dd < 3; ++dd) {
            const double mu = gk[1 + dd], sg = gk[4 + dd];
            if (!std::isfinite(mu) || !std::isfinite(sg) || !(sg > 0.0))
                return fail(MXR_E_INVALID, "component %d: non-finite mean or non-positive width", k);
            const double za = (lo[dd] - mu) / sg, zb = (hi[dd] - mu) / sg;
            P.mu[k][dd] = mu;
            P.sigma[k][dd] = sg;
            P.inv_sigma[k][dd] = 1.0 / sg;
            P.Pa[k][dd] = 0.5 * std::erfc(-za / std::sqrt(2.0));
            P.Pb[k][dd] = 0.5 * std::erfc(-zb / std::sqrt(2.0));
            P.Qa[k][dd] = 0.5 * std::erfc(za / std::sqrt(2.0));
            P.Qb[k][dd] = 0.5 * std::erfc(zb / std::sqrt(2.0));
            Z *= P.Pb[k][dd] - P.Pa[k][dd];
            F *= P.Pb[k][dd] - P.Pa[k][dd];
            sprod *= sg;
        }
        P.kcoef[k] = F > 0.0 ? 1.0 / (sprod * std::pow(2.0 * M_PI, 1.5) * F) : 0.0;
        P.mass[k] = Z;
        run += Z;
    }
    P.norm = run;
    if (!(run > 0.0) && alpha < 1.0) return fail(MXR_E_INVALID, "the mixture has no mass inside the box");
    P.alpha = alpha;
    P.t2 = t * t;
    P.inv_omega = 1.0 / (2.0 * M_PI * (1.0 - std::cos(c.par[0])));
    for (int dd = 0; dd < 3; ++dd) {
        P.lo[dd] = lo[dd];
        P.hi[dd] = hi[dd];
    }
    if (!ins->prop_dev) {
        e = hipMalloc((void **)&ins->prop_dev, sizeof(PropTable));
        if (e != hipSuccess) {
            ins->prop_dev = nullptr;
            return fail(MXR_E_NOMEM, "hipMalloc of the proposal table: %s", hipGetErrorString(e));
        }
    }
    // runs still in flight read the previous table
    e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(ins->prop_dev, &P, sizeof P, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload of the proposal table");
    ins->prop_host = P;
    ins->prop_on = true;
    return MXR_OK;
}

mxr_status mxr_get_launch_shape(const mxr_instrument *ins, mxr_launch_shape *out) {
    if (!ins || !out) return fail(MXR_E_INVALID, "null instrument or shape");
    *out = ins->shape;
    return MXR_OK;
}

mxr_status mxr_set_launch_shape(mxr_instrument *ins, const mxr_launch_shape *shape) {
    if (!ins || !shape) return fail(MXR_E_INVALID, "null instrument or shape");
    const mxr_launch_shape &s = *shape;
    if (!(s.occupancy == 0 || s.occupancy == 4 || s.occupancy == 6 || s.occupancy == 8) || s.compact > 1 ||
        s.rounds > kCompactRounds || s.xcd_order > 2)
        return fail(MXR_E_INVALID, "launch shape out of range (occupancy %u, compact %u, rounds %u, xcd order %u)",
                    s.occupancy, s.compact, s.rounds, s.xcd_order);
    ins->shape = s;
    return MXR_OK;
}

// Tuning-cache key of an instrument's plain runs of about n_total rays.
static std::string instrument_key(const mxr_instrument *ins, uint64_t n_total) {
    const DevInstr &d = ins->host;
    std::string k = "instrument recipe " + std::to_string(ins->recipe) + " chain";
    for (uint32_t c = 0; c < d.ncomp; ++c) {
        k += " " + std::to_string(d.c[c].type) + "/" + std::to_string(d.c[c].flags);
        if (d.c[c].type == MXR_PHANTOM || d.c[c].type == MXR_DETECTOR)
            k += ":" + std::to_string(d.c[c].dims[0]) + "x" + std::to_string(d.c[c].dims[1]) + "x" +
                 std::to_string(d.c[c].dims[2]);
    }
    const bool exact = d.phantom < 0 || d.c[d.phantom].aux[4] != 0.0;
    int lg = 0;
    while (lg < 63 && (1ull << (lg + 1)) <= n_total) ++lg;
    return k + " exact " + std::to_string(exact ? 1 : 0) + " log2n " + std::to_string(lg);
}

mxr_status mxr_autotune_instrument(mxr_instrument *ins, uint64_t n_total, double rays_fraction, const mxr_tally *tallies,
                                   uint32_t n_tallies, const char *cache_path, mxr_launch_shape *out) {
    if (!ins) return fail(MXR_E_INVALID, "null instrument");
    if (!(rays_fraction > 0.0 && rays_fraction <= 1.0)) return fail(MXR_E_INVALID, "rays_fraction must be in (0, 1]");
    if (n_total < 1) return fail(MXR_E_INVALID, "n_total must be positive");
    const std::string key = instrument_key(ins, n_total);
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "r")) {
            char line[1024];
            bool found = false;
            mxr_launch_shape hit{};
            while (std::fgets(line, sizeof line, f)) {
                char *tab = std::strchr(line, '\t');
                if (!tab) continue;
                *tab = 0;
                mxr_launch_shape sh{};
                if (key == line &&
                    std::sscanf(tab + 1, "%u %u %u %u", &sh.occupancy, &sh.compact, &sh.rounds, &sh.xcd_order) == 4) {
                    hit = sh;
                    found = true;
                }
            }
            std::fclose(f);
            if (found && mxr_set_launch_shape(ins, &hit) == MXR_OK) {
                if (out) *out = ins->shape;
                return MXR_OK;
            }
        }
    }
    const bool fixed = pick_plain(ins->recipe, true, 0) != nullptr;
    const bool compactable = pick_compact(ins->recipe) != nullptr;
    std::vector<mxr_launch_shape> cand;
    for (uint32_t occ : {0u, 4u, 6u, 8u}) {
        if (occ && !fixed) continue;
        for (uint32_t xo : {0u, 1u, 2u}) {
            if (compactable) {
                cand.push_back({occ, 1, 0, xo});
                cand.push_back({occ, 1, 16, xo});
            }
            cand.push_back({occ, 0, 0, xo});
        }
    }
    const uint64_t n = std::max<uint64_t>(1, (uint64_t)((double)n_total * rays_fraction));
    const mxr_launch_shape saved = ins->shape;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipStreamCreate(&st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    mxr_status status = e == hipSuccess ? MXR_OK : hip_fail(e, "autotune stream and events");
    float best_ms = 0.f;
    mxr_launch_shape best = saved;
    for (size_t c = 0; status == MXR_OK && c < cand.size(); ++c) {
        ins->shape = cand[c];
        float ms = 0.f;
        for (int rep = 0; status == MXR_OK && rep < 2; ++rep) {  // the first run warms up
            e = hipEventRecord(e0, st);
            if (e == hipSuccess)
                status = mxr_run(ins, 0, n, n_total, 1, 0, 0, tallies, n_tallies, nullptr, st);
            if (status == MXR_OK) {
                e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) status = hip_fail(e, "autotune timing");
            }
        }
        if (status == MXR_OK && (best_ms == 0.f || ms < best_ms)) {
            best_ms = ms;
            best = cand[c];
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (status != MXR_OK) {
        ins->shape = saved;
        return status;
    }
    ins->shape = best;
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "a")) {
            std::fprintf(f, "%s\t%u %u %u %u\n", key.c_str(), best.occupancy, best.compact, best.rounds, best.xcd_order);
            std::fclose(f);
        }
    }
    if (out) *out = best;
    return MXR_OK;
}

mxr_status mxr_trace_rays(mxr_instrument *ins, const uint64_t *ray_ids, uint64_t n, uint64_t n_total, uint64_t seed,
                          uint32_t purpose, uint32_t job, const mxr_ray_soa *out, void *hip_stream) {
    RunArgs a;
    mxr_status st = common_args(ins, n_total, seed, purpose, job, a);
    if (st != MXR_OK) return st;
    if (n == 0) return MXR_OK;
    if (!ray_ids || !out) return fail(MXR_E_INVALID, "null ray ids or output");
    const mxr_ray_soa &o = *out;
    if (!o.x || !o.y || !o.z || !o.dx || !o.dy || !o.dz || !o.E || !o.w || !o.status || !o.dead_at || !o.bin)
        return fail(MXR_E_INVALID, "null output array");
    a.n = n;
    a.ids = ray_ids;
    a.dump = o;
    return launch(ins, a, n, false, true, (hipStream_t)hip_stream);
}

}  // extern "C"

// ---------------------------------------------------------------- batch --

struct mxr_batch {
    int device;
    int recipe;
    bool exact;
    uint32_t n_jobs;
    uint64_t total_rays, total_cost;
    std::vector<BatchJob> host_jobs;  // longest-first
    BatchJob *dev_jobs;
    unsigned long long *counter;
    size_t shmem;
    mxr_batch_schedule sched;  // normalised launch shape
    uint64_t n_tiles;
    int n_cu;
    std::string key;  // describes the batch for the tuning cache
    hipStream_t capture_stream;
    hipStream_t branch[kMaxBranches];  // graph branches of the launches form
    hipEvent_t fork, join[kMaxBranches];
    hipGraph_t graph;
    hipGraphExec_t exec;
    bool graph_ready;
};

static uint64_t batch_tiles(const std::vector<BatchJob> &jobs, uint32_t tile_rays, std::vector<uint64_t> *first) {
    uint64_t t = 0;
    for (const BatchJob &j : jobs) {
        if (first) first->push_back(t);
        t += (j.args.n + tile_rays - 1) / tile_rays;
    }
    return t;
}

static void batch_drop_graph(mxr_batch *b) {
    if (b->graph_ready) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->graph_ready = false;
    }
}

static void batch_free(mxr_batch *b) {
    batch_drop_graph(b);
    if (b->dev_jobs) (void)hipFree(b->dev_jobs);
    if (b->counter) (void)hipFree(b->counter);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    for (uint32_t i = 0; i < kMaxBranches; ++i) {
        if (b->branch[i]) (void)hipStreamDestroy(b->branch[i]);
        if (b->join[i]) (void)hipEventDestroy(b->join[i]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
}

// Lays out the tiles for the current tile size and uploads the job table.
static mxr_status batch_layout(mxr_batch *b) {
    // a replay still in flight reads the table being replaced
    hipError_t w = hipDeviceSynchronize();
    if (w != hipSuccess) return hip_fail(w, "hipDeviceSynchronize before the job table upload");
    std::vector<uint64_t> first;
    const uint64_t n_tiles = batch_tiles(b->host_jobs, b->sched.tile_rays, &first);
    if (n_tiles >= (1ull << 31)) return fail(MXR_E_UNSUPPORTED, "batch needs %llu tiles (limit 2^31)", (unsigned long long)n_tiles);
    for (size_t i = 0; i < first.size(); ++i) b->host_jobs[i].tile0 = first[i];
    b->n_tiles = n_tiles;
    hipError_t e = hipMemcpy(b->dev_jobs, b->host_jobs.data(), b->host_jobs.size() * sizeof(BatchJob), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy of the batch job table");
    batch_drop_graph(b);
    return MXR_OK;
}

// Checks a launch shape and fills the fields its form ignores: the grid
// form's tiles are one work-group (256 rays), the launches form keeps the
// 256-ray tile table unused.
static bool schedule_normalise(const mxr_batch_schedule &in, mxr_batch_schedule &out) {
    out = in;
    switch (in.form) {
        case MXR_BATCH_GRID:
            out.groups_per_cu = 0;
            out.tile_rays = kBlock;
            out.branches = 0;
            return true;
        case MXR_BATCH_PERSISTENT:
            out.branches = 0;
            if (out.tile_rays == 0) out.tile_rays = 65536;
            return in.groups_per_cu >= 1 && in.groups_per_cu <= 8 && out.tile_rays >= (uint32_t)kBlock &&
                   out.tile_rays <= (1u << 24) && out.tile_rays % kBlock == 0;
        case MXR_BATCH_LAUNCHES:
            out.groups_per_cu = 0;
            out.tile_rays = kBlock;
            if (out.branches == 0) out.branches = 1;
            return out.branches <= kMaxBranches;
        default: return false;
    }
}

static const char *kScheduleRule =
    "schedule: form 0 (grid), 1 (persistent: groups_per_cu 1..8, tile_rays a multiple of 256 in [256, 2^24]) "
    "or 2 (launches: branches 1..4)";

// One job's rays as k_trace launches of at most kMaxLaunchGroups work-groups
// (the same kernels and launch shape as mxr_run).
static hipError_t launch_job(KernelFn k, const RunArgs &job, size_t shmem, hipStream_t st) {
    const uint64_t max_rays = kMaxLaunchGroups * kBlock;
    for (uint64_t done = 0; done < job.n;) {
        const uint64_t m = std::min(job.n - done, max_rays);
        RunArgs a = job;
        a.first = done;
        a.n = m;
        const uint64_t groups = (m + kBlock - 1) / kBlock;
        a.blocks_per_xcd = (uint32_t)((groups + 7) / 8);
        hipLaunchKernelGGL(k, dim3((unsigned)((uint64_t)a.blocks_per_xcd * 8)), dim3(kBlock), shmem, st,
                           (const MXR_CONSTANT_PARAM DevInstr *)job.ins, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        done += m;
    }
    return hipSuccess;
}

// Capture the batch's launch into a graph (once per shape): the grid kernel,
// or counter reset + persistent kernel, or the per-job launches.
static mxr_status batch_capture(mxr_batch *b) {
    hipError_t e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t launch_err = hipSuccess;
    if (b->sched.form == MXR_BATCH_LAUNCHES) {
        // jobs dealt longest-first round-robin over the branches, which fork
        // from and join back into the capture stream
        const uint32_t nb = b->sched.branches;
        KernelFn k = pick_kernel(b->recipe, false, false, b->exact, kModePlain);
        launch_err = hipEventRecord(b->fork, b->capture_stream);
        for (uint32_t i = 0; launch_err == hipSuccess && i < nb; ++i)
            launch_err = hipStreamWaitEvent(b->branch[i], b->fork, 0);
        for (uint32_t j = 0; launch_err == hipSuccess && j < b->n_jobs; ++j)
            launch_err = launch_job(k, b->host_jobs[j].args, b->shmem, b->branch[j % nb]);
        for (uint32_t i = 0; launch_err == hipSuccess && i < nb; ++i) {
            launch_err = hipEventRecord(b->join[i], b->branch[i]);
            if (launch_err == hipSuccess) launch_err = hipStreamWaitEvent(b->capture_stream, b->join[i], 0);
        }
    } else if (b->sched.form == MXR_BATCH_GRID) {
        // grid form: one work-group per 256-ray tile, 2-D grid
        const uint64_t groups = (b->n_tiles + 511) / 512 * 512;
        const uint32_t gx = (uint32_t)std::min<uint64_t>(groups, 1u << 16);
        const uint32_t gy = (uint32_t)((groups + gx - 1) / gx);
        hipLaunchKernelGGL(pick_batch_grid(b->recipe, b->exact), dim3(gx, gy), dim3(kBlock), b->shmem,
                           b->capture_stream, (const BatchJob *)b->dev_jobs, b->n_jobs, b->n_tiles);
    } else {
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, b->capture_stream, b->counter);
        BatchKernelFn k = pick_batch_kernel(b->recipe, b->exact);
        const unsigned grid = (unsigned)(b->sched.groups_per_cu * (uint32_t)b->n_cu);
        hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), b->shmem, b->capture_stream, (const BatchJob *)b->dev_jobs,
                           b->n_jobs, b->n_tiles, b->sched.tile_rays, b->counter);
    }
    hipError_t launch = launch_err != hipSuccess ? launch_err : hipGetLastError();
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->capture_stream, &g);
    if (launch != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(launch, "batch kernel launch during capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    b->graph = g;
    b->exec = x;
    b->graph_ready = true;
    return MXR_OK;
}

extern "C" {

mxr_status mxr_batch_create(const mxr_batch_job *jobs, uint32_t n_jobs, const mxr_batch_schedule *schedule,
                            mxr_batch **out) {
    if (!jobs || !out || n_jobs == 0) return fail(MXR_E_INVALID, "null jobs or output, or no jobs");
    *out = nullptr;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const mxr_instrument *i0 = jobs[0].instrument;
    if (!i0) return fail(MXR_E_INVALID, "job 0 has no instrument");
    std::vector<std::pair<uint64_t, uint32_t>> order;  // (cost, index)
    std::vector<BatchJob> hj(n_jobs);
    uint64_t total_rays = 0, total_cost = 0;
    for (uint32_t k = 0; k < n_jobs; ++k) {
        const mxr_batch_job &j = jobs[k];
        const mxr_instrument *ins = j.instrument;
        if (!ins) return fail(MXR_E_INVALID, "job %u has no instrument", k);
        if (ins->device != cur) return fail(MXR_E_STATE, "job %u: instrument on device %d, device %d current", k, ins->device, cur);
        if (ins->prop_on) return fail(MXR_E_UNSUPPORTED, "job %u: batches trace the plain source (clear the proposal)", k);
        if (ins->host.ncomp != i0->host.ncomp) return fail(MXR_E_INVALID, "job %u: component chain differs from job 0", k);
        for (uint32_t c = 0; c < ins->host.ncomp; ++c)
            if (ins->host.c[c].type != i0->host.c[c].type) return fail(MXR_E_INVALID, "job %u: component chain differs from job 0", k);
        if (ins->recipe != i0->recipe) return fail(MXR_E_INVALID, "job %u: phantom model differs from job 0", k);
        if (j.n_rays < 1) return fail(MXR_E_INVALID, "job %u: n_rays must be positive", k);
        if (j.job > 0xFFFFFFu) return fail(MXR_E_INVALID, "job %u: RNG job field must be < 2^24", k);
        BatchJob &bj = hj[k];
        std::memset(&bj, 0, sizeof bj);
        RunArgs &b = bj.args;
        b.ins = ins->dev;
        b.first = 0;
        b.n = j.n_rays;
        b.n_total = j.n_rays;
        b.seed = j.seed;
        b.word3 = j.job;
        const uint64_t G = strata_side(ins->strata, j.n_rays);
        if (G * G > 1 && j.n_rays > (~0ull - (G * G - 1)) / (G * G))
            return fail(MXR_E_INVALID, "job %u: n_rays * strata^2 + strata^2 - 1 must stay below 2^64", k);
        b.G = G;
        b.G2 = G * G;
        b.sd = strat_div(j.n_rays, G);
        for (uint32_t d = 0; d < ins->n_det; ++d) {
            const mxr_tally &t = j.tallies[d];
            if (!t.count || !t.sum_w || !t.sum_w2) return fail(MXR_E_INVALID, "job %u: tally %u has a null array", k, d);
            if (t.n_bins != ins->det_bins[d])
                return fail(MXR_E_INVALID, "job %u: tally %u has %llu bins, monitor needs %llu", k, d,
                            (unsigned long long)t.n_bins, (unsigned long long)ins->det_bins[d]);
            b.tally.count[d] = (unsigned long long *)t.count;
            b.tally.sum_w[d] = t.sum_w;
            b.tally.sum_w2[d] = t.sum_w2;
        }
        // work estimate per ray: a walk through the phantom visits ~ (nx + ny + nz) voxels
        uint64_t per_ray = 1;
        if (ins->host.phantom >= 0) {
            const DevComp &c = ins->host.c[ins->host.phantom];
            per_ray += (uint64_t)c.dims[0] + c.dims[1] + c.dims[2];
        }
        const uint64_t cost = j.n_rays * per_ray;
        order.push_back({cost, k});
        total_rays += j.n_rays;
        total_cost += cost;
    }
    std::stable_sort(order.begin(), order.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
    mxr_batch *b = new (std::nothrow) mxr_batch();
    if (!b) return fail(MXR_E_NOMEM, "host allocation failed");
    b->device = cur;
    b->recipe = i0->recipe;
    b->exact = true;
    size_t mu_bytes = 0;
    for (uint32_t k = 0; k < n_jobs; ++k) {
        const mxr_instrument *ins = jobs[k].instrument;
        if (ins->host.phantom >= 0) {
            b->exact = b->exact && ins->host.c[ins->host.phantom].aux[4] != 0.0;
            mu_bytes = std::max(mu_bytes, (size_t)ins->host.n_mat * ins->host.n_ebin * sizeof(double));
        }
    }
    b->shmem = mu_bytes;
    b->n_jobs = n_jobs;
    b->total_rays = total_rays;
    b->total_cost = total_cost;
    for (const auto &o : order) b->host_jobs.push_back(hj[o.second]);
    e = hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, cur);
    if (e != hipSuccess || b->n_cu < 1) b->n_cu = 256;
    // one launch per job, one branch, until tuned
    const mxr_batch_schedule dflt{MXR_BATCH_LAUNCHES, 0, 0, 1};
    if (!schedule_normalise(schedule ? *schedule : dflt, b->sched)) {
        delete b;
        return fail(MXR_E_INVALID, "%s", kScheduleRule);
    }
    char key[256];
    std::string chain;
    for (uint32_t c = 0; c < i0->host.ncomp; ++c) chain += std::to_string(i0->host.c[c].type) + (c + 1 < i0->host.ncomp ? "-" : "");
    snprintf(key, sizeof key, "chain=%s jobs=%u rays=%llu cost=%llu cu=%d", chain.c_str(), n_jobs,
             (unsigned long long)total_rays, (unsigned long long)total_cost, b->n_cu);
    b->key = key;
    b->graph_ready = false;
    b->dev_jobs = nullptr;
    b->counter = nullptr;
    b->capture_stream = nullptr;
    b->fork = nullptr;
    for (uint32_t i = 0; i < kMaxBranches; ++i) {
        b->branch[i] = nullptr;
        b->join[i] = nullptr;
    }
    e = hipMalloc((void **)&b->dev_jobs, n_jobs * sizeof(BatchJob));
    if (e == hipSuccess) e = hipMalloc((void **)&b->counter, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
    for (uint32_t i = 0; e == hipSuccess && i < kMaxBranches; ++i) e = hipStreamCreateWithFlags(&b->branch[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (uint32_t i = 0; e == hipSuccess && i < kMaxBranches; ++i) e = hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming);
    mxr_status st = e == hipSuccess ? batch_layout(b) : fail(MXR_E_NOMEM, "batch allocation: %s", hipGetErrorString(e));
    if (st != MXR_OK) {
        batch_free(b);
        return st;
    }
    *out = b;
    return MXR_OK;
}

mxr_status mxr_batch_run(mxr_batch *b, void *hip_stream) {
    if (!b) return fail(MXR_E_INVALID, "null batch");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != b->device) return fail(MXR_E_STATE, "batch lives on device %d, device %d is current", b->device, cur);
    if (!b->graph_ready) {
        mxr_status st = batch_capture(b);
        if (st != MXR_OK) return st;
    }
    e = hipGraphLaunch(b->exec, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return MXR_OK;
}

mxr_status mxr_batch_get_schedule(const mxr_batch *b, mxr_batch_schedule *out) {
    if (!b || !out) return fail(MXR_E_INVALID, "null batch or output");
    *out = b->sched;
    return MXR_OK;
}

mxr_status mxr_batch_set_schedule(mxr_batch *b, const mxr_batch_schedule *s) {
    if (!b || !s) return fail(MXR_E_INVALID, "null batch or schedule");
    mxr_batch_schedule n;
    if (!schedule_normalise(*s, n)) return fail(MXR_E_INVALID, "%s", kScheduleRule);
    const bool relayout = n.tile_rays != b->sched.tile_rays;
    b->sched = n;
    batch_drop_graph(b);
    return relayout ? batch_layout(b) : MXR_OK;
}

void mxr_batch_destroy(mxr_batch *b) {
    if (!b) return;
    const int b_device = b->device;
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != b_device) (void)hipSetDevice(b_device);
    (void)hipDeviceSynchronize();
    batch_free(b);
    if (cur >= 0 && cur != b_device) (void)hipSetDevice(cur);
}

// Tuning cache: one line per batch, "<key>\t<form> <groups_per_cu> <tile_rays> <branches>".
static bool cache_lookup(const char *path, const std::string &key, mxr_batch_schedule &out) {
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char *tab = std::strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        mxr_batch_schedule s{}, n{};
        if (key == line && std::sscanf(tab + 1, "%u %u %u %u", &s.form, &s.groups_per_cu, &s.tile_rays, &s.branches) == 4 &&
            schedule_normalise(s, n)) {
            out = n;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

static void cache_store(const char *path, const std::string &key, const mxr_batch_schedule &s) {
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s\t%u %u %u %u\n", key.c_str(), s.form, s.groups_per_cu, s.tile_rays, s.branches);
    std::fclose(f);
}

mxr_status mxr_batch_autotune(mxr_batch *b, double rays_fraction, const char *cache_path, mxr_batch_schedule *out) {
    if (!b) return fail(MXR_E_INVALID, "null batch");
    if (!(rays_fraction > 0.0 && rays_fraction <= 1.0)) return fail(MXR_E_INVALID, "rays_fraction must be in (0, 1]");
    mxr_batch_schedule cached;
    if (cache_lookup(cache_path, b->key, cached)) {
        mxr_status st = mxr_batch_set_schedule(b, &cached);
        if (st == MXR_OK && out) *out = b->sched;
        return st;
    }
    // timing copy of the job table with every job's rays scaled down (the
    // random streams and tallies are the real ones)
    std::vector<BatchJob> saved = b->host_jobs;
    for (BatchJob &j : b->host_jobs) {
        j.args.n = std::max<uint64_t>(1, (uint64_t)(j.args.n * rays_fraction));
        j.args.n_total = j.args.n;
        const uint64_t G = strata_side(j.args.G, j.args.n_total);
        j.args.G = G;
        j.args.G2 = G * G;
        j.args.sd = strat_div(j.args.n_total, G);
    }
    mxr_status lay = batch_layout(b);
    if (lay != MXR_OK) {
        b->host_jobs = saved;
        (void)batch_layout(b);
        return lay;
    }
    std::vector<mxr_batch_schedule> cand;
    cand.push_back({MXR_BATCH_GRID, 0, 0, 0});
    for (uint32_t g : {2u, 4u, 8u})
        for (uint32_t t : {16384u, 65536u}) cand.push_back({MXR_BATCH_PERSISTENT, g, t, 0});
    for (uint32_t br : {1u, 2u, 4u}) cand.push_back({MXR_BATCH_LAUNCHES, 0, 0, br});
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best_ms = 0.f;
    mxr_batch_schedule best = b->sched;
    mxr_status st = e == hipSuccess ? MXR_OK : hip_fail(e, "hipEventCreate");
    for (size_t c = 0; st == MXR_OK && c < cand.size(); ++c) {
        st = mxr_batch_set_schedule(b, &cand[c]);
        for (int rep = 0; st == MXR_OK && rep < 2; ++rep) {  // first replay warms up
            e = hipEventRecord(e0, b->capture_stream);
            if (e == hipSuccess) st = mxr_batch_run(b, b->capture_stream);
            if (st == MXR_OK) e = hipEventRecord(e1, b->capture_stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e != hipSuccess) st = hip_fail(e, "autotune timing");
        }
        float ms = 0.f;
        if (st == MXR_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && (best_ms == 0.f || ms < best_ms)) {
            best_ms = ms;
            best = b->sched;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    // back to the real ray counts, with the fastest shape
    b->host_jobs = saved;
    b->sched = best;
    mxr_status st2 = batch_layout(b);
    if (st != MXR_OK) return st;
    if (st2 != MXR_OK) return st2;
    cache_store(cache_path, b->key, best);
    if (out) *out = best;
    return MXR_OK;
}

}  // extern "C"
