// lsm_internal.h -- shared definitions of the host runtime and the HIP
// kernels of liblsm.so (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lsm.h"

namespace lsm {

constexpr int kTileX = 64;  // one wavefront covers 64 consecutive sites of a row
constexpr int kTileY = 4;   // four rows per workgroup
constexpr int kBlock = kTileX * kTileY;
constexpr int kMaxTypes = 2 * LSM_MAX_PHASES * LSM_MAX_PHASES;  // (geometry, phase, phase)
constexpr uint8_t kVoid = 0xFF;
constexpr int kNumPartials = 24;  // virial[9], kinetic[9], pe, ke, nonfinite, 3 spare
constexpr int kSweepCols = 62;    // owned columns per wavefront in the 2D row sweep
constexpr int kSweepCols2 = 60;   // owned columns per wavefront of the two-step sweep
// The row sweeps address 16-byte site records with 32-bit byte offsets:
// lattices and batches they run hold fewer sites than this (one more, the
// sentinel site, follows the last).
constexpr int64_t kSweepMaxSites = (int64_t(1) << 28) - 1;

// Site flag byte: bits 0-3 phase, bits 4-5 grip (1 left column, 2 right column).
__host__ __device__ inline int flag_phase(uint8_t f) { return f & 0x0F; }
__host__ __device__ inline int flag_grip(uint8_t f) { return (f >> 4) & 3; }

// Spring type record: constant, rest length and critical length for a
// (geometry class, phase a, phase b) triple, in both precisions.
struct TypeRec {
    float k32, kr0_32, rc2_32, r0_32;  // k, k r0, rc^2, r0 rounded to FP32
    double k64, r0_64, rc64, pad;
};

// Loop control kept in device memory so captured graphs can be replayed
// across increments.
struct Ctl {
    double eps;
    int32_t inc;
    int32_t step_base;  // steps already done inside the current increment
    uint32_t n_events;
    int32_t rate_s0;    // constant-rate loading: step inside the increment at which
    double rate_eps0;   // the strain was rate_eps0, advancing rate_de per step
    double rate_de;
};

// Device record (same layout as lsm_record).
typedef lsm_record DevRecord;

enum Mode { kStart = 0, kMid = 1, kEnd = 2, kEval = 3 };

// One wavefront work item of the 2D row sweep over a batch of specimens:
// specimen s (site block [base, base + nx*ny)), strip of columns starting at
// i0 = strip * kSweepCols - 1, owned rows [j0, j1).  End-of-relax partials of
// row j go to pbase + j * strips + strip.
struct SweepItem {
    int32_t base, nx, ny, i0;
    int32_t j0, j1, strip, strips;
    int32_t pbase, spec, pad0, pad1;
};

// Per-specimen reduction range and reference volume.
struct SpecDesc {
    int32_t pbase, npart;
    double omega;
};

struct StepParams {
    int32_t nx, ny, nz;
    int32_t tiles_x, tiles_y, ntiles, nblocks;
    int32_t nphase;
    int64_t nsites;
    double a;
    double dt, gamma;
    double mass[LSM_MAX_PHASES];
    const uint8_t *flags;
    void *mask;            // uint8 (2D) or uint32 (3D) broken bits per site and direction
    const uint32_t *sbase; // canonical id of the first forward spring of a site
    void *u_in;            // displacement state read this step
    void *u_out;           // displacement state written this step
    void *v;               // velocity (updated in place)
    void *acc;             // acceleration at the last full step
    const TypeRec *types;
    Ctl *ctl;
    lsm_event *events;
    int64_t ev_cap;
    double *partials;      // kNumPartials per workgroup (end-of-relax reductions)
    double *f64;           // force output of the evaluation mode
    int32_t commit;        // evaluation mode: apply the break rule to the state
    int32_t red_blocks;    // workgroups that wrote partials in the last end-of-relax step
    // row-sweep decomposition of the 2D lattice: each wavefront owns 62
    // columns of a strip and sw_rows rows, sweeping upward
    int32_t sw_strips, sw_rows, sw_nwork, sw_nblocks;
    int32_t sw_pf;          // rows prefetched ahead by each wavefront (1..3)
    // particle-list mode of the gather kernel (3D): one thread per particle,
    // plist[p] = i | j << 10 | k << 21 of particle p (raster order)
    int32_t n_part;
    const uint32_t *plist;  // null: one thread per grid site
    int32_t c_blocks;       // workgroups of the particle-list grid (multiple of 8)
    // two-step sweep: 60-column strips; velocities and break bits are read
    // from v / mask and written to v_out / mask_out
    int32_t sw2_strips, sw2_nwork, sw2_nblocks;
    void *v_out;
    void *mask_out;
    const SweepItem *items2;   // batch work items of the two-step sweep (60-column strips)
    const int32_t *n_items2;   // their number (device)
    // batch of specimens (2D sweep only)
    const SweepItem *items;  // active work items
    const int32_t *n_items;  // number of active work items (device)
    uint32_t *spec_broken;   // broken-spring count per specimen
    // compact 3D layout: per grid site (plus a sentinel) a row-table entry:
    // bits 32-63 the number of solid sites before it in raster order (= the
    // particle index of a solid site), bit 12 whether it is solid, bits 0-3,
    // 4-7, 8-11 the phases of the sites at x - 1, x, x + 1 of its row (0 if
    // void or off the grid) -- or, for single-phase lattices, 32-bit entries
    // (solid sites before it << 1 | solid); per particle the directions
    // (bits 0-17) whose neighbour is void or off the grid
    const uint64_t *crow;
    const uint32_t *cabs;
    // LDS-window variant (single-phase lattices): per workgroup of
    // kC3WinBlock particles (c_wblocks workgroups, a multiple of 8),
    // cwin[8 lb ..] = first particle of the windows of plane
    // offsets -1, 0, +1, then their lengths; per particle crel = eight
    // 16-bit entries (offset in the plane's window << 1 | solid) of the
    // off-row grid rows, slots (dj + 1) * 3 + (dk + 1) without the own row
    const uint32_t *cwin;
    const void *crel;
    int32_t c_wblocks;
    // spring law (LSM_SPRING_*) and the cubic coefficient; only the gather
    // kernel (and the local fields) take a law other than the linear one
    int32_t law;
    double law_c;
    // constant-rate loading in the one-step 2D sweep's interior steps: the
    // sweep places the grips of the rows it loads itself (no grip kernel)
    int32_t grip_rate;
};

// Launchers (lsm_kernels.hip).  All are asynchronous on `stream`.
hipError_t launch_increment(const StepParams &p, int dim, int prec, hipStream_t stream,
                            double eps_new, double d_eps, int inc, int affine);
hipError_t launch_step(const StepParams &p, int dim, int prec, int mode, hipStream_t stream,
                       int step_local);
// Small 2D lattices: nsteps interior steps (step_local ..) in one launch of
// one workgroup holding the state in LDS (same results as nsteps launches
// of launch_step); reads u_in, writes u_out, velocities and break bits in
// place.  Lattices whose state needs more than kSmallLdsBytes are rejected.
constexpr int kSmallBlock = 1024;
constexpr size_t kSmallLdsBytes = 56 * 1024;
size_t small_lds_bytes(int64_t nsites, int prec);
hipError_t launch_small_mid(const StepParams &p, int prec, hipStream_t stream, int nsteps, int step_local);
// 2D row-sweep variant of the start/mid/end steps (same semantics as launch_step).
hipError_t launch_sweep2d(const StepParams &p, int prec, int mode, hipStream_t stream,
                          int step_local);
// Two interior steps (step_local and step_local + 1) in one launch of the
// 2D row sweep; reads u_in, writes u_out.
hipError_t launch_sweep2d_x2(const StepParams &p, int prec, hipStream_t stream, int step_local);
// Wavefronts of the interior-step row sweep (two-step or one-step kernel)
// resident per CU; 0 if the runtime cannot tell.
int sweep_waves_per_cu(int two_step, int prec, int pf);
// Batch version over capacity2 two-step work items (items beyond *p.n_items2 exit at once).
hipError_t launch_sweep2d_x2_batch(const StepParams &p, int prec, hipStream_t stream, int step_local,
                                   int capacity2);
hipError_t launch_kick_drift(const StepParams &p, int dim, int prec, hipStream_t stream);
// 3D compact layout: one interior step (P's state pointers, flags and break
// bits point at the compact arrays, P.nsites is their particle stride), and
// the copies between the site-grid and compact states (cn: compact stride).
// kind 0: 64-bit row table; 1: 32-bit row table (particles before << 1 |
// solid) of a single-phase lattice; 2: LDS windows (cwin / crel) of a
// single-phase lattice
hipError_t launch_step_c3(const StepParams &p, int prec, hipStream_t stream, int step_local, int kind);
// particles per workgroup of the window variant (eight wavefronts: 4.3
// window records per particle on the C3 lattice against 5.6 for 256), and
// the records of the three plane windows it stages in LDS (66 KB: two
// workgroups per CU)
constexpr int kC3WinBlock = 512;
constexpr int kC3PoolF64 = 2816;
constexpr int kC3PoolF32 = 2816;
hipError_t launch_pack_c3(const StepParams &p, int prec, hipStream_t stream, int to_compact, void *u_grid,
                          void *v_grid, uint32_t *m_grid, void *u_c, void *v_c, uint32_t *m_c, int64_t cn);
// Local fields of the state in u_in / v / mask (particle order, FP64
// [n][dim][dim]): virial stress over the radius-0 or radius-1 domain per
// site volume vsite, and the Lagrangian strain (NaN where undefined).
hipError_t launch_local_fields(const StepParams &p, int dim, int prec, hipStream_t stream, const int32_t *site_of,
                               const int32_t *part_of, int radius, double vsite, double *stress, double *strain);
// Constant-rate loading: places the grips of u_in at the strain of step
// step_local of the increment (rate fields of the loop control) and records
// that strain; launched before every step kernel while a rate is set.
hipError_t launch_grips(const StepParams &p, int dim, int prec, hipStream_t stream, int step_local);
// Batch versions: the grid covers `capacity` work items; items beyond
// *p.n_items exit at once.
hipError_t launch_sweep2d_batch(const StepParams &p, int prec, int mode, hipStream_t stream,
                                int step_local, int capacity);
hipError_t launch_increment_batch(const StepParams &p, int prec, hipStream_t stream, double eps_new,
                                  double d_eps, int inc, int affine, int capacity);
hipError_t launch_finalize_batch(const StepParams &p, int dim, hipStream_t stream, DevRecord *recs,
                                 const SpecDesc *specs, int nspec, int nsteps);
hipError_t launch_finalize(const StepParams &p, int dim, hipStream_t stream, DevRecord *rec,
                           double omega, int nsteps);

}  // namespace lsm
