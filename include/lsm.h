/*
 * lsm.h -- C ABI of the MI355X lattice spring model (LSM) library, liblsm.so.
 *
 * The calls follow the paper's statement of the problem (arXiv 2201.04565):
 * an image with a number of particle types becomes a particle-spring network
 * (Introduction, Img2Particle); a displacement-controlled mechanical test is
 * run on it (Introduction; Section 3.1) by velocity Verlet time integration
 * (Section 2.2, Eq. 3-5) of the truncated harmonic spring forces (Section
 * 2.1, Eq. 1-2) with irreversible critical-stretch breaking (Section 2.3,
 * Section 4); energies and the virial stress (Eq. 7) are reported.
 *
 * Conventions
 *  - Every call returns an int status: LSM_OK (0) or a negative LSM_E* code.
 *    No exception crosses the ABI.  lsm_last_error() gives the text of the
 *    last failure on a handle.
 *  - A handle is single-threaded and bound to one HIP stream.  Calls that
 *    launch GPU work are asynchronous on that stream unless stated otherwise.
 *  - Host arrays passed in are caller-owned and only read during the call.
 *    Host arrays passed out are caller-allocated with the stated size.
 *  - Device memory is caller-owned: the caller allocates
 *    lsm_workspace_bytes() bytes (256-byte aligned) and hands the pointer to
 *    lsm_bind(); it must stay valid until lsm_destroy().  The library itself
 *    never allocates device memory.  Host-side objects (HIP graphs, events)
 *    are owned by the handle.
 *  - Particles are numbered in raster order of the non-void sites (x
 *    fastest); springs are numbered by owner particle and then by forward
 *    direction in canonical order (2D: east, upper-left, upper-right; 3D:
 *    (1,0,0) (0,1,0) (0,0,1) (1,1,0) (-1,1,0) (1,0,1) (-1,0,1) (0,1,1)
 *    (0,-1,1)).
 */
#ifndef LSM_H
#define LSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define LSM_OK 0
#define LSM_EINVAL (-1)    /* bad argument (null pointer, size, range) */
#define LSM_ENOMEM (-2)    /* workspace too small / host allocation failed */
#define LSM_EHIP (-3)      /* a HIP runtime call failed; see lsm_last_error */
#define LSM_EUNSTABLE (-4) /* non-finite stress or energy detected */
#define LSM_ESTATE (-5)    /* call made in the wrong order */

/* ---- enumerations ---- */
#define LSM_LATTICE_TRI2D 0 /* 2D triangular packing, 6 nearest neighbours */
#define LSM_LATTICE_SC3D 1  /* 3D simple cubic, 6 face + 12 edge neighbours */
#define LSM_FP64 0          /* FP64 displacements, velocities and forces */
#define LSM_FP32_KAHAN 1    /* FP32 forces, compensated FP32 displacements */
#define LSM_PRED_AFFINE 0     /* free particles follow the strain increment */
#define LSM_PRED_GRIPS_ONLY 1 /* only the grips move at an increment */
#define LSM_MAX_PHASES 8
#define LSM_KERNEL_AUTO 0   /* 2D: LSM_KERNEL_SMALL where the lattice fits it, else the
                               two-step (FP32-compensated) or one-step (FP64) row sweep;
                               3D: LSM_KERNEL_COMPACT (the gather kernel under
                               constant-rate loading or beyond 2^28 particles) */
#define LSM_KERNEL_GATHER 1 /* one thread per site, all incident springs */
#define LSM_KERNEL_SWEEP 2  /* 2D: wavefronts sweep rows, forward springs once */
#define LSM_KERNEL_SWEEP2 3 /* 2D, FP32-compensated: row sweep advancing two interior
                               steps per launch (same results as LSM_KERNEL_SWEEP, about
                               half the memory traffic); LSM_EINVAL for FP64 lattices */
#define LSM_KERNEL_SMALL 4  /* 2D lattices whose state fits one workgroup's LDS (about
                               1,100 sites in FP64, 1,300 FP32-compensated): all
                               interior steps of a relaxation chunk in one launch of one
                               workgroup (same results as LSM_KERNEL_GATHER, whose kernel
                               runs the start and end steps); LSM_EINVAL for 3D or larger
                               lattices (a lattice built later and too large runs the
                               gather kernel) */
#define LSM_KERNEL_COMPACT 5 /* 3D: interior steps on a compact copy of the state (one
                               record per particle instead of per grid site, neighbours
                               found through a per-site prefix count), copied in and out
                               around every chunk of interior steps; same results as
                               LSM_KERNEL_GATHER, whose kernel runs the start and end
                               steps.  Single-phase lattices stage each workgroup's
                               neighbour records in LDS (where every window holds fewer
                               than 2^15 particles; else, and for several phases, it runs
                               as LSM_KERNEL_COMPACT_DIRECT, which lsm_get_launch then
                               reports).  LSM_EINVAL for 2D lattices and for lattices of
                               2^28 particles or more.  Not under constant-rate loading
                               (the gather kernel runs those steps) */
#define LSM_KERNEL_COMPACT_DIRECT 6 /* LSM_KERNEL_COMPACT with every neighbour record read
                               from global memory (no LDS staging); same results and
                               rules */

/* Model and integration parameters.
 *  k[P*P], break_stretch[P*P]: row-major, symmetric spring constant and
 *    critical stretch s_c (rc = r0 (1 + s_c)) of a spring joining phases
 *    (a, b) -- Section 2.3 assigns spring parameters by particle type, the
 *    paper's Table "Constants of linear fracture spring" gives one such
 *    table.  A non-finite off-diagonal entry selects the series rule
 *    k_ab = 2 k_a k_b / (k_a + k_b), s_ab = min(s_a k_a, s_b k_b) / k_ab.
 *  k_face, k_diag: 3D multipliers of face and edge-diagonal springs.
 *  mass[P]: particle mass per phase (Section 2.3: mass by type).
 *  dt: time step; damping: viscous coefficient gamma of the force -gamma v
 *    (0 gives undamped velocity Verlet).
 *  void_value: pixel value of empty sites, or -1 for none.              */
typedef struct {
    int32_t lattice;
    int32_t nphase;
    double a;
    double k[LSM_MAX_PHASES * LSM_MAX_PHASES];
    double break_stretch[LSM_MAX_PHASES * LSM_MAX_PHASES];
    double k_face;
    double k_diag;
    double mass[LSM_MAX_PHASES];
    double dt;
    double damping;
    int32_t precision;
    int32_t predictor;
    int32_t void_value;
    int32_t spring_law;   /* LSM_SPRING_* (0: the linear spring of Eq. 1-2) */
    double law_c;         /* cubic coefficient c of LSM_SPRING_CUBIC */
} lsm_config;

/* Spring laws.  The paper's closing section keeps broken springs in the
 * list so that their stiffness may recover under compression, and names
 * non-linear elasticity among the extensions of the linear spring:
 *   LSM_SPRING_LINEAR: U = k (r - r0)^2 / 2 (Eq. 1), broken springs inert;
 *   LSM_SPRING_RECOVER: as linear, and a broken spring shorter than its rest
 *     length acts with its intact stiffness (contact of crack faces);
 *   LSM_SPRING_CUBIC: U = k d^2 / 2 + k c d^4 / (4 r0^2), d = r - r0, force
 *     magnitude k d (1 + c d^2 / r0^2) (c > 0 stiffening, c < 0 softening).
 * The break rule is the same for all.  Lattices with a law other than
 * LSM_SPRING_LINEAR run the gather kernel, except for the interior steps
 * of single-phase 3D lattices with LDS windows, which run the LSM_KERNEL_COMPACT
 * form (LSM_KERNEL_AUTO resolves to that where it applies; asking for a
 * kernel other than LSM_KERNEL_AUTO, LSM_KERNEL_GATHER or
 * LSM_KERNEL_COMPACT is LSM_EINVAL); batches take the linear law only.    */
#define LSM_SPRING_LINEAR 0
#define LSM_SPRING_RECOVER 1
#define LSM_SPRING_CUBIC 2

/* State record at the end of a relaxation.
 *  eps: applied engineering strain (sum of increments).
 *  sigma: virial stress (Eq. 7), row-major 3x3 (2D uses the upper 2x2),
 *    tension positive, over the reference volume N * (site area or volume).
 *  ke, pe: kinetic energy and Eq. 1 potential energy.  n_broken: broken
 *  springs so far.  increment, step: loading increment and step inside it.
 *  status: LSM_OK or LSM_EUNSTABLE.                                       */
typedef struct {
    double eps;
    double sigma[9];
    double ke;
    double pe;
    int64_t n_broken;
    int32_t increment;
    int32_t step;
    int32_t status;
    int32_t reserved;
} lsm_record;

/* One spring break: loading increment, step inside it (0 = the force
 * evaluation right after the increment), canonical spring id, and the
 * relative overshoot (r - rc) / rc at detection.                          */
typedef struct {
    int32_t increment;
    int32_t step;
    int64_t spring_id;
    double margin;
} lsm_event;

/* One launch configuration of the step kernel and its measured time. */
typedef struct {
    int32_t variant;          /* LSM_KERNEL_*; from lsm_get_launch the kernel that
                                 runs the interior steps (AUTO resolved) */
    int32_t rows_per_wave;    /* sweep row chunk */
    int32_t prefetch;         /* sweep rows prefetched ahead */
    int32_t steps_per_launch; /* interior steps per launch: 2 for the two-step
                                 sweep, else 1 (lsm_get_launch; 0 from tuners) */
    double us_per_step;       /* measured (lsm_autotune), 0 otherwise */
} lsm_tuning;

typedef struct lsm_handle lsm_handle;

/* Creates a handle from a copy of *cfg.  Errors: LSM_EINVAL for an invalid
 * configuration (lattice kind, 1 <= nphase <= 8, a > 0, dt > 0,
 * damping >= 0, masses > 0, finite non-negative diagonal k and s).        */
int lsm_create(const lsm_config *cfg, lsm_handle **out);

/* Frees the handle and its host-side objects; never touches the caller's
 * workspace.  Synchronises the bound stream first.  Null is ignored.      */
void lsm_destroy(lsm_handle *h);

/* Image -> particles and typed springs (Introduction, Img2Particle).
 * phase: host array of nx*ny*nz pixel values, x fastest (nz = 1 for 2D);
 * each value is a phase index < nphase or the void value.  The first and
 * last image columns (x = 0 and x = nx-1) are the grips of the uniaxial
 * test (Section 3.1 boundary particles).  Host-only: may be called before
 * lsm_bind, and not after it.                                              */
int lsm_build_lattice(lsm_handle *h, const uint8_t *phase, int64_t nx, int64_t ny, int64_t nz);

/* Particle and spring counts of the built lattice (LSM_ESTATE before it).  */
int lsm_counts(const lsm_handle *h, int64_t *n_particles, int64_t *n_springs);

/* Device workspace size in bytes for the built lattice.                   */
int lsm_workspace_bytes(const lsm_handle *h, size_t *bytes);

/* Binds caller-owned device memory (dptr, 256-byte aligned, at least
 * lsm_workspace_bytes) and a HIP stream (hipStream_t, not the null stream
 * so that relaxation loops can be captured into HIP graphs), then uploads
 * the lattice and sets x = X0, v = 0 on that stream.  LSM_ENOMEM when the
 * workspace is too small.                                                 */
int lsm_bind(lsm_handle *h, void *dptr, size_t bytes, void *hip_stream);

/* One displacement-controlled loading increment (Section 3.1): the strain
 * becomes eps + d_eps, the grips move to X0_x + eps * i * a (all other
 * components clamped, v = 0), free particles get the affine predictor
 * d_eps * i * a along x (LSM_PRED_AFFINE), then the forces are evaluated
 * with the break test (step 0) and the first half kick and drift of the
 * integrator are applied.  LSM_ESTATE if called twice without lsm_relax.  */
int lsm_apply_strain_increment(lsm_handle *h, double d_eps);

/* nsteps >= 1 velocity Verlet steps (Eq. 3-5, half-step velocity form)
 * with the spring forces of Eq. 2, the break test each step, and viscous
 * damping; ends on a full step and computes the record (Eq. 7 stress,
 * energies).  Launched as HIP graphs of the step kernel.                  */
int lsm_relax(lsm_handle *h, int64_t nsteps);

/* Constant strain-rate loading, the paper's protocol (Section 3.1: the
 * boundary particles are displaced apart along x at a fixed strain rate;
 * Section 2.3: the boundary displacement is the first operation of every
 * time step).  rate is per unit time (the paper's 1e-6 with its dt = 1).
 * From the next step on, step S of the increment first places the grips at
 * X0_x + eps_S i a, eps_S = eps0 + (S - S0) (rate dt), where eps0 is the
 * strain at this call (step S0) or at the next lsm_apply_strain_increment
 * (S0 = 0), which continues at the same rate from its new strain; free
 * particles move only by integration.  The record's eps is eps_S of its
 * last step.  rate = 0 stops the grips.  While a rate is set the interior
 * steps run one step per launch (the two-step sweep and the one-workgroup
 * kernel are not used).  Bound handles only; synchronises.  LSM_EINVAL
 * for a non-finite rate.                                                   */
int lsm_set_strain_rate(lsm_handle *h, double rate);

/* lsm_relax in chunks of `every` steps (the last may be shorter) with a
 * record after each chunk -- the paper's periodic callbacks that report the
 * potential and kinetic energies (Section 2.3) -- written to out[0 ..
 * cap-1] (host); *n (may be NULL) receives the number written.  A chunk
 * ending on a non-finite state stops the run with LSM_EUNSTABLE (its record
 * is written).  Synchronises after every chunk.                            */
int lsm_relax_trace(lsm_handle *h, int64_t nsteps, int64_t every, lsm_record *out, int64_t cap,
                    int64_t *n);

/* Synchronises the stream and copies the record of the last relaxation.
 * Returns LSM_EUNSTABLE (with *out filled) if the state was not finite.   */
int lsm_read_state(lsm_handle *h, lsm_record *out);

/* Synchronises and copies broken-spring events first .. first+cap-1, in
 * (increment, step, spring_id) order; *n receives the number copied.      */
int lsm_read_broken(lsm_handle *h, int64_t first, int64_t cap, lsm_event *out, int64_t *n);

/* Total number of broken springs (synchronises).                          */
int lsm_n_broken(lsm_handle *h, int64_t *n);

/* Canonical spring list: endpoints p < q, spring constant k, rest length
 * r0, critical length rc, broken flag (synchronises).  Arrays of
 * n_springs entries; any pointer may be null to skip that field.          */
int lsm_get_springs(lsm_handle *h, int64_t *p, int64_t *q, double *k, double *r0, double *rc,
                    uint8_t *broken);

/* Reference positions X0 (host, n_particles x dim, canonical order).     */
int lsm_get_reference(lsm_handle *h, double *X0);

/* Current positions X0 + u and velocities as FP64 (host, n_particles x
 * dim).  Synchronises.  Velocities are full-step values after lsm_relax. */
int lsm_get_positions(lsm_handle *h, double *x);
int lsm_get_velocities(lsm_handle *h, double *v);

/* Overwrites positions or velocities (host, n_particles x dim).  Only
 * between relaxations (LSM_ESTATE otherwise); synchronises.               */
int lsm_set_positions(lsm_handle *h, const double *x);
int lsm_set_velocities(lsm_handle *h, const double *v);

/* One force evaluation (Eq. 2 with the break test) at the current
 * positions, returned as FP64 (host, n_particles x dim).  commit_breaks != 0
 * marks springs found beyond rc as broken and logs them at the current
 * (increment, step); 0 leaves the state untouched (such springs still give
 * no force).  Synchronises.                                               */
int lsm_eval_forces(lsm_handle *h, double *f, int commit_breaks);

/* Local fields of the current state (Section 3.1: the virial stress of
 * Eq. 7 over a neighbourhood domain and the Lagrangian strain of the field
 * figure, Eq. 8), FP64, written asynchronously on the bound stream to
 * caller-owned DEVICE arrays stress and strain, each [n_particles][dim][dim]
 * in particle order (both required).
 *   stress: sigma = (1 / (|D| V)) sum_{k in D} s^k with
 *     s^k_ab = 1/2 sum over k's intact springs (x_l - x_k)_a f^{kl}_b
 *              - m_k v_a v_b  (f^{kl}: Eq. 2 force on k from l; tension
 *     positive), V the site area (sqrt3/2 a^2) or volume (a^3), and D = {k}
 *     for radius 0 or k and every particle it shares a spring with (broken
 *     or not) for radius 1;
 *   strain: (J^T J - I) / 2 (the Green-Lagrange reading of Eq. 8) with J the
 *     least-squares map (sum d d0^T)(sum d0 d0^T)^-1 of the vectors to the
 *     first nearest neighbours (2D: the six lattice neighbours, 3D: the six
 *     face neighbours; broken springs included) from the reference to the
 *     current configuration; NaN where those vectors do not span the space.
 * With radius 1 the strain array also serves as the temporary of the
 * per-particle sums.  LSM_EINVAL for other radii or null arrays; LSM_ESTATE
 * between lsm_apply_strain_increment and lsm_relax (velocities are then
 * half-step values).                                                      */
int lsm_local_fields(lsm_handle *h, int radius, double *stress, double *strain);

/* Bitwise checkpoint of the dynamic state (displacements, velocities,
 * broken flags, clock, events).  lsm_save_state with buf == NULL returns
 * the size in *n; otherwise *n must hold the buffer size.  lsm_load_state
 * requires a handle built from the same image and configuration.          */
int lsm_save_state(lsm_handle *h, void *buf, size_t *n);
int lsm_load_state(lsm_handle *h, const void *buf, size_t n);

/* Measurement hooks.  lsm_set_timing(h, 1) brackets every graph of step
 * kernels with HIP events on the bound stream; lsm_read_timing returns the
 * summed event time in ms and the number of step kernels it covered
 * (synchronises).  lsm_step_bytes gives the algorithmic bytes one launch of
 * the interior step kernel in use must move: state read and written once,
 * site flags, break masks (and the particle list in 3D); one launch
 * advances lsm_tuning.steps_per_launch steps.                             */
int lsm_set_timing(lsm_handle *h, int enable);
int lsm_read_timing(lsm_handle *h, double *ms, int64_t *steps);
int lsm_step_bytes(const lsm_handle *h, int64_t *bytes);

/* Launch shape of the step kernel (used by the autotuner).  variant is one
 * of LSM_KERNEL_*; rows_per_wave (2..4096, 0 = keep) sets the row chunk of
 * the 2D sweep (lattices of fewer than 2^28 sites; larger 2D lattices
 * run the gather kernel, and asking for a sweep there is LSM_EINVAL).
 * Until a row chunk is set, the sweep picks one per kernel
 * and prefetch depth from the bound device's compute units and the
 * kernel's occupancy (wavefronts of nearly equal work filling whole rounds
 * of resident slots).  Results are bitwise independent of rows_per_wave.
 * LSM_KERNEL_SMALL is LSM_EINVAL for 3D lattices and for built lattices
 * whose state exceeds its LDS budget.
 * Only between relaxations (LSM_ESTATE otherwise); drops cached graphs.  */
int lsm_set_launch(lsm_handle *h, int variant, int rows_per_wave);

/* Rows the 2D sweep prefetches ahead of the row it computes (1..3).
 * Results are bitwise independent of it.  Same call-order rules as
 * lsm_set_launch.                                                         */
int lsm_set_prefetch(lsm_handle *h, int rows_ahead);

/* Autotuner: times every candidate launch of the interior step kernel on
 * the bound lattice (steps_per_trial even, 2..1000, replayed from a HIP
 * graph and timed with HIP events), keeps the fastest and writes up to cap
 * results (n_results = number of candidates).  The dynamic state is
 * checkpointed to host memory before the trials and restored after them,
 * so tuning never changes results.  Only between relaxations (LSM_ESTATE
 * otherwise).  Synchronises.                                              */
int lsm_autotune(lsm_handle *h, int steps_per_trial, lsm_tuning *results, int cap, int *n_results);

/* Current launch configuration.                                           */
int lsm_get_launch(const lsm_handle *h, lsm_tuning *out);

const char *lsm_last_error(const lsm_handle *h);
const char *lsm_strerror(int status);

/* ---------------------------------------------------------------------
 * Batches of independent 2D specimens, each taken to failure.
 *
 * The paper motivates the code by high-throughput data generation for
 * machine learning (Abstract; Section 4): many specimens run the same
 * displacement-controlled test.  A batch shares one configuration and
 * loading history; every step is one launch over all specimens still
 * running.  Specimen s stops after the first increment past its stress peak
 * whose sigma_xx is below drop_fraction * peak, a non-finite state, or
 * max_inc increments.  The modulus is the least-squares slope through the
 * origin of sigma_xx against strain over the increments that ended with no
 * broken spring (at least the first one); the strength is the peak.
 * Device memory and stream ownership follow the single-lattice rules.
 * --------------------------------------------------------------------- */
typedef struct lsm_batch lsm_batch;

typedef struct {
    double drop_fraction; /* failure threshold relative to the peak (0.01) */
} lsm_fail_rule;

/* imgs[s]: host image of specimen s (x fastest); dims[3 s .. 3 s + 2] =
 * (nx, ny, 1).  2D triangular lattices only, fewer than 2^28 sites in all
 * (LSM_EINVAL otherwise).                                                */
int lsm_batch_create(const lsm_config *cfg, int64_t n, const uint8_t *const *imgs,
                     const int64_t *dims, lsm_batch **out);
void lsm_batch_destroy(lsm_batch *b);
const char *lsm_batch_last_error(const lsm_batch *b);
int lsm_batch_counts(const lsm_batch *b, int64_t *n_particles, int64_t *n_springs);
int lsm_batch_workspace_bytes(const lsm_batch *b, size_t *bytes);
int lsm_batch_bind(lsm_batch *b, void *dptr, size_t bytes, void *hip_stream);

/* Kernel, row chunk and prefetch depth of the batched sweep (before the
 * run; results do not depend on them).  variant: LSM_KERNEL_SWEEP (one
 * step per launch), LSM_KERNEL_SWEEP2 (two interior steps per launch,
 * FP32-compensated batches only) or LSM_KERNEL_AUTO (SWEEP2 where it
 * applies, the default).  After binding, a row chunk whose work items
 * exceed the bound workspace is LSM_EINVAL.                               */
int lsm_batch_set_launch(lsm_batch *b, int variant, int rows_per_wave, int prefetch);
int lsm_batch_get_launch(const lsm_batch *b, lsm_tuning *out);

/* Picks the kernel (two-step sweep for FP32-compensated batches, and the
 * one-step sweep), rows_per_wave and prefetch for this batch by timing
 * candidate launches (rows 4..32 per wavefront x prefetch 1..2, those the
 * bound workspace holds) on the live specimens, each over about
 * steps_per_trial (2..1000) interior steps, and keeps the fastest.  Bound,
 * before the run.  The trials read the state at rest and write only the
 * second displacement, velocity and break-bit buffers (rewritten before
 * they are read) and the velocities (zeroed afterwards), so the run's
 * results are unchanged.  results (cap entries, may be NULL when cap = 0)
 * receives {variant, rows, prefetch, 0, mean microseconds per step} per
 * candidate; *n_results their number.  Synchronises the stream.         */
int lsm_batch_autotune(lsm_batch *b, int steps_per_trial, lsm_tuning *results, int cap,
                       int *n_results);

/* Runs every specimen to failure (rule may be NULL for drop 0.01).  Once
 * per batch; synchronises after every increment to apply the rule.        */
int lsm_batch_run(lsm_batch *b, double d_eps, int64_t steps_per_inc, int32_t max_inc,
                  const lsm_fail_rule *rule);

/* Results: sigma_xx (n x max_inc, NaN after the specimen stopped),
 * increments run, modulus, strength and broken springs per specimen; any
 * output pointer may be NULL.                                             */
int lsm_batch_read(lsm_batch *b, int32_t max_inc, double *sigma_xx, int32_t *n_inc,
                   double *modulus, double *strength, int64_t *n_broken);

/* HIP-event timing of the step graphs (as lsm_set_timing); site_steps is
 * the sum over timed steps of the particles of the specimens running.     */
int lsm_batch_set_timing(lsm_batch *b, int enable);
int lsm_batch_read_timing(lsm_batch *b, double *ms, int64_t *steps, double *site_steps);

/* ---------------------------------------------------------------------
 * Surrogate network: a small CNN from a two-phase image to the batched
 * model's stress-strain curve and modulus (the paper's motivation of fast
 * data generation for machine-learning materials design: Abstract,
 * Section 4).  Five 3x3 convolutions (ReLU; 2x2 average pooling after the
 * first four; channels[l] outputs), global average pooling, a ReLU dense
 * layer of `hidden` units and a linear layer of `outputs`.  Convolutions
 * with >= 32 input channels run on BF16 matrix cores with FP32
 * accumulation; master weights, gradients, Adam moments and dense layers
 * are FP32.  Parameters are one FP32 vector: for each conv layer l the
 * weights [Cout][3][3][Cin] then the bias [Cout]; then the dense layers
 * [out][in] weights and bias (offsets: lsm_cnn_layout).  Device pointers
 * below (x, y, target, dy, loss) are caller-owned device memory; the
 * workspace follows the single-lattice rules.
 * --------------------------------------------------------------------- */
typedef struct {
    int32_t batch;       /* largest batch */
    int32_t height;      /* image side, multiple of 16 */
    int32_t width;       /* equal to height */
    int32_t channels[5]; /* conv output channels: 32, 64, 128 or 256 each */
    int32_t hidden;
    int32_t outputs;
} lsm_cnn_config;

typedef struct lsm_cnn lsm_cnn;

int lsm_cnn_create(const lsm_cnn_config *cfg, lsm_cnn **out);
void lsm_cnn_destroy(lsm_cnn *c);
const char *lsm_cnn_last_error(const lsm_cnn *c);
int lsm_cnn_param_count(const lsm_cnn *c, int64_t *n);
/* offsets and sizes of each layer's weights and bias in the parameter
 * vector (7 entries: 5 conv, 2 dense; w_n = weight count)                 */
int lsm_cnn_layout(const lsm_cnn *c, int64_t *w_off, int64_t *b_off, int64_t *w_n);
int lsm_cnn_workspace_bytes(const lsm_cnn *c, size_t *bytes);
int lsm_cnn_bind(lsm_cnn *c, void *dptr, size_t bytes, void *hip_stream);
/* host FP32 parameter vector in / out (set also clears the Adam moments);
 * synchronise                                                             */
int lsm_cnn_set_params(lsm_cnn *c, const float *host);
int lsm_cnn_get_params(lsm_cnn *c, float *host);
int lsm_cnn_get_grads(lsm_cnn *c, float *host);
/* x: device uint8 images [batch][height][width] (phase 0/1); y (may be
 * NULL): device FP32 [batch][outputs].  Keeps activations for backward.   */
int lsm_cnn_forward(lsm_cnn *c, const uint8_t *x, int64_t batch, float *y);
/* mean squared error of the last forward against device target
 * [batch][outputs]; writes the output gradient (device, may be NULL) and
 * the loss (device float, may be NULL)                                    */
int lsm_cnn_mse(lsm_cnn *c, const float *target, float *dy, float *loss);
/* For callers that cannot allocate device memory (code under stream
 * capture, serving loops, harnesses that forbid allocation): lsm_cnn_mse
 * with its per-workgroup loss partials in a fixed static device array (one
 * per GPU, 256 KB, held until the process ends) instead of the bound
 * workspace; calls no allocating routine.  dy (device FP32 [batch][outputs])
 * and loss (device float) are required and are the only outputs: the
 * network's own gradient buffer is not touched, so pass dy to
 * lsm_cnn_backward.  Bitwise the same values as lsm_cnn_mse.  LSM_EINVAL
 * when batch x outputs exceeds 65536 x 256; LSM_EHIP if the array's address
 * cannot be obtained.  All calls on one GPU share its array: calls that
 * overlap in time on the same GPU (other streams or threads) race.        */
int lsm_cnn_mse_noalloc(lsm_cnn *c, const float *target, float *dy, float *loss);
/* gradients of all parameters for output gradient dy (device; NULL uses
 * the one from lsm_cnn_mse); overwrites the gradient vector               */
int lsm_cnn_backward(lsm_cnn *c, const float *dy);
int lsm_cnn_adam_step(lsm_cnn *c, float lr, float beta1, float beta2, float eps, int64_t t);
/* Test hook: copies one internal buffer of the last forward / backward pass
 * to host memory (synchronises), so each kernel can be checked on its own
 * inputs.  layer counts conv layers from 0; sizes are for the configured
 * batch (the first `batch` images of the last call are meaningful) and H_l
 * is the side of conv layer l's input (H_0 = height, halved after each
 * pooled layer).  host == NULL returns the size in *bytes; otherwise *bytes
 * is the host capacity (LSM_ENOMEM if short) and receives the size copied.
 * LSM_EINVAL for a buffer or layer that does not exist.                   */
#define LSM_CNN_BUF_POOLED 0  /* l = 0..3: pooled ReLU output, BF16 [B][H_l/2][H_l/2][C_l] */
#define LSM_CNN_BUF_MASK 1    /* l = 1..3: ReLU signs of the four pixels under each pooled
                                 pixel, bit d = (d / 2, d mod 2), uint8 [B][H_l/2][H_l/2][C_l] */
#define LSM_CNN_BUF_ACT 2     /* last conv output after ReLU, BF16 [B][H_4][H_4][C_4] */
#define LSM_CNN_BUF_DACT 3    /* l = 1..4: gradient of conv output l (after the ReLU
                                 mask), BF16 [B][H_l][H_l][C_l] */
#define LSM_CNN_BUF_DPOOL0 4  /* gradient of the first pooled map, BF16 [B][H_0/2][H_0/2][C_0] */
#define LSM_CNN_BUF_GAP 5     /* global average pool, FP32 [B][C_4] */
#define LSM_CNN_BUF_DGAP 6    /* its gradient */
#define LSM_CNN_BUF_HIDDEN 7  /* dense layer 1 after ReLU, FP32 [B][hidden] */
#define LSM_CNN_BUF_DHIDDEN 8 /* its gradient (after the ReLU mask) */
#define LSM_CNN_BUF_OUT 9     /* network output, FP32 [B][outputs] */
#define LSM_CNN_BUF_DOUT 10   /* output gradient of lsm_cnn_mse or lsm_cnn_backward */
int lsm_cnn_read_buffer(lsm_cnn *c, int buffer, int layer, void *host, size_t *bytes);
/* one implicit-GEMM convolution (layers 1..4, bias + ReLU) on device BF16
 * NHWC buffers with this network's weights (kernel tests)                 */
int lsm_cnn_conv_forward(lsm_cnn *c, int layer, const void *in, void *out, int64_t batch);

#ifdef __cplusplus
}
#endif
#endif /* LSM_H */
