/*
 * lbem.h -- C ABI of liblbem, an MI355X (gfx950) implementation of the
 * pseudo-vector lattice-BGK scheme for Maxwell's equations in heterogeneous
 * media (Hanasoge, Succi & Orszag, "Lattice Boltzmann Method for
 * Electromagnetic Wave Propagation", arXiv:1108.2651).
 *
 * The calls follow the paper's statement of the problem: given the medium
 * (permittivity and permeability, Section "The Maxwell Equations"), initial
 * E and B, and a current density j(x,t) (the forcing of Subsection
 * "Homogeneous media"), advance the lattice-BGK equation (eq. LBE: collision
 * eq. COLLI then streaming eq. STREAM) on a periodic box and report E, B
 * (moments, eqs. relate.1-2) and the electromagnetic energy (Subsection
 * "Heterogeneous media").
 *
 * Conventions shared by all calls
 *  - Lattice units: dx = dt = 1.  A box is nx*ny*nz cells, periodic in every
 *    direction; 2D means nz == 1 and the TM polarisation (E_z, B_x, B_y).
 *  - Cell index c = x + nx*(y + ny*z).  Vector fields are component-major
 *    arrays of 3*n doubles: component k of cell c at [k*n + c].
 *  - Every call returns an lbem_status (0 on success, negative on error);
 *    nothing throws across the ABI.  A handle must not be used by two host
 *    threads at once.  Distinct handles are independent.
 *  - Host input arrays are copied before the call returns; the caller keeps
 *    ownership.  Device memory is owned by the handle unless the caller passes
 *    an arena (lbem_config.dev_mem); then the caller frees the arena after
 *    lbem_destroy.  Small per-handle tables (source lists, reduction
 *    partials, upload staging) are always allocated by the handle.
 *  - Asynchrony: lbem_step only enqueues work on the handle's stream.
 *    lbem_moments and lbem_energy synchronise that stream.
 */
#ifndef LBEM_H
#define LBEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbem_s* lbem_t;

typedef enum {
    LBEM_OK = 0,
    LBEM_EINVAL = -1,     /* bad argument (null, out of range, wrong shape)      */
    LBEM_ENOMEM = -2,     /* device allocation failed or arena too small          */
    LBEM_EUNSTABLE = -3,  /* medium gives a rest weight w0(x) outside [0,1)       */
    LBEM_ENONFINITE = -4, /* a diagnostic sum is NaN or Inf                       */
    LBEM_EDEVICE = -5,    /* HIP runtime error (no device, launch failure, ...)   */
    LBEM_ESTATE = -6,     /* call out of order (e.g. step before init_fields)     */
    LBEM_ETOOBIG = -7     /* lattice exceeds a fixed static buffer
                             (lbem_energy_noalloc)                               */
} lbem_status;

/* Storage / arithmetic formats of the populations. */
typedef enum {
    LBEM_F64 = 0,      /* FP64 populations, FP64 medium, FP64 arithmetic          */
    LBEM_F32 = 1,      /* FP32 populations, FP32 medium, FP32 arithmetic          */
    LBEM_F16DEV = 2,   /* FP32 conserved moments + FP16 deviations from the local
                          equilibrium, scaled by a power of two per velocity;
                          all collision arithmetic in FP32                        */
    LBEM_BF16DEV = 3,  /* as LBEM_F16DEV with BF16 deviations.  NOT within the
                          1e-3 relative field error of the FP16 formats: BF16
                          keeps an 8-bit significand, and the measured error
                          against the FP64 solution is 1.2e-3 - 3.6e-3 per
                          field (1000-2000 steps, smooth media with sources)   */
    LBEM_F16GHOST = 4, /* FP32 conserved moments + FP16 ghost coordinates: only the
                          (Q-1)P - D moving deviations that the zero-moment
                          constraints leave free are stored (2D 2 of 5, 3D 15 of
                          21 per cell); the rest follow from the constraints    */
    LBEM_BF16GHOST = 5, /* as LBEM_F16GHOST with BF16 ghost coordinates; NOT
                          within 1e-3 (same band as LBEM_BF16DEV)               */
    LBEM_F16 = 6       /* plain FP16 populations, FP32 medium and arithmetic
                          (rounded to nearest on store); single steps, pull or
                          AA.  A bandwidth reference: its rounding is relative
                          to the whole population, so it misses the 1e-3 bar
                          the deviation formats meet                            */
} lbem_prec;

/* Kind of the two faces of one axis (lbem_set_boundary). */
typedef enum {
    LBEM_BC_PERIODIC = 0, /* the paper's periodic box                            */
    LBEM_BC_PEC = 1,      /* perfectly conducting walls: tangential E = 0        */
    LBEM_BC_PMC = 2       /* perfectly magnetic walls: tangential B = 0          */
} lbem_boundary;

/* Streaming pattern (eq. STREAM) of the stored populations. */
typedef enum {
    LBEM_STREAM_AUTO = 0, /* pull (the multi-step fused kernels need two copies),
                             except 3D F64, and 3D F32 below 1e6 cells, which
                             run single steps and take AA                       */
    LBEM_STREAM_PULL = 1, /* two copies; each step gathers from x - c_i           */
    LBEM_STREAM_AA = 2    /* one copy updated in place, alternating even/odd steps
                             (F64/F32 only)                                       */
} lbem_streaming;

typedef struct {
    int dim;            /* 2 (TM) or 3                                           */
    int prec;           /* lbem_prec                                             */
    int64_t nx, ny, nz; /* box; nz must be 1 when dim == 2; nx*ny*nz < 2^31      */
    double tau;         /* BGK relaxation time; the paper's choice is 0.5        */
    double w0_vac;      /* rest weight where eps_r*mu_r == 1, in [0,1); 1/3 is the
                           usual choice.  Sets the lattice light speed:
                           c_L^2(x) = (1 - w0_vac)/(dim eps_r mu_r)              */
    int streaming;      /* lbem_streaming                                        */
    int mu_varies;      /* 1: reserve room for a non-uniform permeability (adds
                           the B x grad(ln mu) part of the source); 0: mu == 1    */
    void* stream;       /* hipStream_t to enqueue on; NULL = the null stream     */
    void* dev_mem;      /* optional caller-owned device arena, 256-byte aligned  */
    size_t dev_bytes;   /* its size; must be >= lbem_required_bytes(cfg)         */
} lbem_config;

/* Device bytes the handle needs for cfg (populations, medium, field scratch);
 * 0 if cfg is invalid. */
size_t lbem_required_bytes(const lbem_config* cfg);

/* Create a solver.  On success *out is a new handle (state: no medium, no
 * fields).  Errors: EINVAL (bad cfg), ENOMEM, EDEVICE. */
int lbem_create(const lbem_config* cfg, lbem_t* out);

/* Destroy a handle (NULL is accepted).  Synchronises its stream first. */
int lbem_destroy(lbem_t h);

/* Set the medium: relative permittivity eps_r[n] > 0 and, if mu_r != NULL,
 * relative permeability mu_r[n] > 0 (host arrays).  The light speed enters
 * through the rest weight w0(x) = 1 - dim*c_L^2(x) (weights of Section
 * "Lattice BGK formulation"); EUNSTABLE if some w0 falls outside [0,1), i.e.
 * eps_r*mu_r < 1 - w0_vac.  A non-uniform mu_r needs cfg.mu_varies (else
 * EINVAL).  Clears the fields: lbem_init_fields must follow. */
int lbem_set_medium(lbem_t h, const double* eps_r, const double* mu_r);

/* Set E(0), B(0) (host arrays of 3*n doubles); the populations start at the
 * local equilibrium (eq. distrib.func) of these fields.  2D accepts only the
 * TM components: EINVAL if E_x, E_y or B_z is non-zero.  Resets time to 0.
 * ESTATE before lbem_set_medium. */
int lbem_init_fields(lbem_t h, const double* E, const double* B);

/* Current-density footprint: j_comp(cells[k], t) = weight[k] * amp[t] for the
 * m listed cells (host arrays; repeated cells add up).  comp in {0,1,2}; 2D
 * accepts comp == 2 only.  m == 0 removes the source.  The source enters the
 * collision as the tensor term T_i = -(w_i/c^2) eps S with S = -j/eps_abs
 * (eq. LBE), eps_abs = eps_r/c_vac^2.  ESTATE before lbem_set_medium. */
int lbem_set_source(lbem_t h, int comp, const int64_t* cells, const double* weight, int64_t m);

/* Enqueue nsteps time steps of the lattice-BGK equation (eq. LBE): each step
 * forms the moments (eqs. relate.1-2), relaxes to the equilibrium (eq.
 * distrib.func) with the BGK collision and the tensor source (eq. COLLI), and
 * streams (eq. STREAM).  amp (host, nsteps doubles, may be NULL = no
 * source) gives the source amplitude of each step: step k of this call uses
 * amp[k] at time t0 + k.  ESTATE before lbem_init_fields.  Periodic handles in
 * the plain formats with pull streaming advance several steps per launch
 * where the kernels allow (lbem_steps_per_launch); walls, an absorber,
 * dispersion or anisotropy make every launch a single step.  The result does
 * not depend on this choice (bit for bit). */
int lbem_step(lbem_t h, int64_t nsteps, const double* amp);

/* E and B at the current time (3*n doubles each, component-major), recovered
 * from the zeroth and first moments of the populations (eqs. relate.1-2: E
 * from Lambda = c^2 sum_i g_i by the Levi-Civita contraction of the Maxwell
 * section, B = K, the contracted first moment).  With
 * on_device == 0 they are host pointers, else device pointers on the
 * handle's device.  Either pointer may be NULL to skip it.  Synchronises. */
int lbem_moments(lbem_t h, double* E, double* B, int on_device);

/* FP64 diagnostics at the current time (synchronises):
 *   out[0]  EM energy  sum_x eps_abs |E|^2 + |B|^2/mu_r  (the energy of
 *           Subsection "Heterogeneous media", sum of B^2 + E^2/c^2, with the
 *           local light speed and permeability)
 *   out[1]  Q_c = sum_x c_L^2 sum_i sum_p g_ip^2 / w_i  (exact invariant of
 *           the scheme at tau = 1/2 with mu == 1, no source, no absorber or
 *           dispersion, periodic or walled faces, uniform anisotropy ratios)
 *   out[2]  sum_x (div_h B)^2, periodic central differences (also with walls):
 *           the solenoidal constraint of the Maxwell section, div B = 0
 *   out[3]  sum_x |B|^2
 * ENONFINITE if any of them is NaN or Inf (the values are still written). */
int lbem_energy(lbem_t h, double out[4]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * diagnostics as lbem_energy, bit for bit, with the FP64 B field and the
 * reduction partials in a static device array of the library (64 MiB per GPU,
 * held until the process ends) instead of the handle's scratch.  The call
 * allocates and frees nothing.  Lattices above LBEM_NOALLOC_MAX_CELLS cells
 * return LBEM_ETOOBIG before any work is enqueued.  All calls on one GPU share
 * the array: calls that overlap in time on the same GPU (from two threads, or
 * on two streams without an ordering between them) race and give undefined
 * results.  Synchronises the handle's stream; other errors as lbem_energy. */
#define LBEM_NOALLOC_MAX_CELLS 2781712   /* 3n + 4 ceil(n/256) + 4 doubles <= 64 MiB */
int lbem_energy_noalloc(lbem_t h, double out[4]);

/* Completed steps since lbem_init_fields (-1 for an invalid handle). */
int64_t lbem_time(lbem_t h);

/* Time steps advanced per kernel launch by lbem_step on this handle (1, or 2-4
 * when several steps are fused into one pass through LDS: the plain formats by
 * default, the 3D 16-bit formats two steps when the environment variable
 * LBEM_DEV3F=1 is set at creation; the result is identical to single steps).
 * EINVAL for NULL. */
int lbem_steps_per_launch(lbem_t h);

/* ---- exact checkpoint / resume ----
 * Not an operation of the paper: it lets a long solve stop and continue bit
 * for bit.  The blob is a 128-byte header (magic "LBEMST01", dim, format,
 * streaming, storage layout, nx, ny, nz, time, payload size) followed by the
 * handle's population state exactly as stored (format- and streaming-
 * specific; it is not converted).  The medium and the current source are not
 * in the blob: the resuming handle is created with the same configuration and
 * given the same walls, medium, anisotropy, absorber, dispersion parameters
 * and source (lbem_set_boundary ... lbem_set_source) before lbem_set_state;
 * the dispersion's auxiliary fields are in the blob. */

/* Size in bytes of the state blob of this handle (0 for NULL). */
size_t lbem_state_bytes(lbem_t h);

/* Write the state blob into buf (bytes >= lbem_state_bytes).  on_device == 0:
 * host memory, else device memory on the handle's device.  Synchronises.  The
 * blob is a function of the handle's state alone: alignment padding inside it
 * is zero, so two handles at the same state write the same bytes.
 * Errors: EINVAL (NULL, too small), ESTATE (no fields yet), EDEVICE. */
int lbem_get_state(lbem_t h, void* buf, size_t bytes, int on_device);

/* Restore a blob written by lbem_get_state on a handle of the same dim,
 * format, streaming and box: populations, storage layout and time.  Requires
 * lbem_set_medium first (ESTATE); EINVAL for a blob of another configuration
 * or a bad header.  Synchronises; afterwards the handle is initialised. */
int lbem_set_state(lbem_t h, const void* buf, size_t bytes, int on_device);

/* ---- non-periodic faces and absorbing layer ----
 * Not in the paper, which uses periodic boxes and leaves other boundaries to
 * future work.  Walls sit half a cell outside the first and last cell of an
 * axis.  A population that would stream in from beyond a wall is the cell's
 * own outgoing population along the opposite velocity, reflected as a tensor
 * under the mirror of that axis: the box then evolves exactly like the
 * periodic box of twice the length holding the box and its mirror image, with
 * tangential E odd about a PEC wall (even about a PMC wall).  Beside a wall
 * the ln mu gradient uses the mirrored medium.  The diagnostic sum of
 * (div_h B)^2 keeps periodic differences. */

/* Faces of `axis` (0..dim-1) become walls of the given kind (or periodic
 * again).  Pull streaming only (EINVAL for AA: create the handle with
 * LBEM_STREAM_PULL, since AUTO takes AA for small 3D FP32 and all 3D FP64
 * boxes); before lbem_set_medium (ESTATE after).  With walls or an absorber
 * the solver runs single steps. */
int lbem_set_boundary(lbem_t h, int axis, int kind);

/* Absorbing layer: after every collision the populations of cell x are
 * multiplied by 1 - sigma[x] (n host doubles in [0,1); EINVAL otherwise).
 * E and B decay at the same rate, so electric and magnetic losses keep the
 * ratio eps : mu and the layer is impedance-matched.  NULL removes it.  Pull
 * streaming only.  The handle copies sigma; synchronises. */
int lbem_set_absorber(lbem_t h, const double* sigma);

/* ---- anisotropic media ----
 * The lattice section notes that different weights for particles moving
 * along different axes model anisotropic media.  Factors fac[a*n + x] > 0
 * (a = 0..dim-1) scale the isotropic c_L^2(x) of the medium along axis a:
 * per-axis second moments s_a = fac_a c_L^2, rest weight 1 - sum_a s_a (in
 * [0,1), else EUNSTABLE and nothing changes), c^2 = mean_a s_a.  The
 * equilibrium keeps the paper's form with these weights and
 * Bbar_b = K_b / sum_{a != b} r_a (r_a = s_a/c^2; K/(D-1) when isotropic):
 * the orthogonal projection onto the conserved moments, so the collision
 * stays an isometry.  A wave along axis a travels at s_a (2D) and at
 * s_a^2/(s_a + s_b) polarised along b (3D); the medium is birefringent in 3D.
 * eps_abs becomes (D-1)/(mu c^2).  Plain formats (F64, F32) with pull
 * streaming only (EINVAL otherwise); after lbem_set_medium (ESTATE before;
 * lbem_set_medium again makes the medium isotropic).  The fields must be
 * initialised afterwards.  Synchronises; the solver then runs single steps. */
int lbem_set_anisotropy(lbem_t h, const double* fac);

/* ---- frequency-dispersive permittivity ----
 * The convolution term of the Maxwell source (Section "The Maxwell
 * Equations"), which the paper leaves to auxiliary differential equations:
 * one Lorentz pole per cell, chi(w) = wp2 / (w02 - w^2 - i gamma w) relative
 * to the cell's permittivity, in lattice units (time step 1).  Auxiliary
 * fields P (polarisation in units of E) at integer and J = dP/dt at
 * half-integer times: J(t+1/2) = [(1-gamma/2) J(t-1/2) + wp2 E(t) - w02 P(t)]
 * / (1+gamma/2), P(t+1) = P(t) + J(t+1/2); the source -J(t+1/2) of step t
 * enters the rest particle only (the w_i-weighted form of the other sources
 * filters S(t) but not S(t-1) and would pump one polariton branch).
 * wp2: n host doubles >= 0 (NULL removes the dispersion); w02, gamma: n
 * doubles >= 0 or NULL for zeros (Drude, lossless).  EINVAL on negative or
 * non-finite values or AA streaming.  P and J restart from zero here and at
 * lbem_init_fields; they are part of the checkpoint blob.  Stability of
 * large wp2 or w02 is the caller's (lattice units: keep them well below 1).
 * Synchronises; the solver then runs single steps. */
int lbem_set_dispersion(lbem_t h, const double* wp2, const double* w02, const double* gamma);

/* Static description of a status code. */
const char* lbem_strerror(int code);

/* ---- batched stepping of many resident lattices (continuous-batching serving) ----
 *
 * A batch advances several independent handles together: each step of a tick
 * is one persistent launch per (dim, format) class that strides over all
 * (lattice, tile) work items of the handles in that class.  A tick is
 * steps_per_tick such steps; each class's steps are captured once, when the
 * batch is created, as a HIP graph, and the classes present are replayed; the per-lattice table it reads is uploaded before each
 * tick, so lattices can join and leave between ticks.  Results are bit-for-bit
 * those of lbem_step on each handle alone.
 */
typedef struct lbem_batch_s* lbem_batch_t;

/* max_lattices: capacity of one tick (1..65536); steps_per_tick: K (1..4096);
 * stream: the hipStream_t the ticks run on (not NULL: it is captured).
 * Member handles may live on other streams: each tick waits for the work
 * already enqueued on a member's stream, and later work on that stream
 * (lbem_moments, lbem_destroy) waits for the tick.  Errors: EINVAL, ENOMEM. */
int lbem_batch_create(int max_lattices, int steps_per_tick, void* stream, lbem_batch_t* out);

/* Enqueue one tick on the batch stream: handle k advances by nsteps[k] steps
 * (0 <= nsteps[k] <= steps_per_tick; 0 leaves it untouched), each step the
 * lattice-BGK update of lbem_step (eqs. LBE, COLLI, STREAM), current source
 * and non-uniform mu term included.  Members must be distinct, initialised
 * (ESTATE otherwise), periodic with none of the cell extras (walls, absorber,
 * dispersion, anisotropy), created with pull streaming (or AA for the plain
 * formats LBEM_F64, LBEM_F32, LBEM_F16), any format (EINVAL otherwise).  A
 * member's current source runs at amplitude 0 here (as lbem_step with
 * amp == NULL); lbem_batch_run_amp gives the amplitudes.  The members of a
 * 3D class run in groups whose state touched per step fits a cache-sized
 * budget (environment LBEM_BATCH_GROUP_MIB, default 224 MiB; 0 turns it off),
 * each group for all its steps; the results are the same bits either way.
 * Returns once enqueued; lbem_moments on a member synchronises.  Each group's
 * table is uploaded through one of eight pinned staging slots: a call waits
 * only when a slot's previous upload has not executed yet. */
int lbem_batch_run(lbem_batch_t b, const lbem_t* handles, const int64_t* nsteps, int count);

/* lbem_batch_run with source amplitudes: amp (host, count * steps_per_tick
 * doubles, row k for handle k) gives amp[k*steps_per_tick + j] to the j-th
 * step of handle k in this tick, as lbem_step's amp does for a solo call (the
 * current density of the forcing of Subsection "Homogeneous media").  Rows of
 * handles without a source are ignored; amp == NULL is lbem_batch_run. */
int lbem_batch_run_amp(lbem_batch_t b, const lbem_t* handles, const int64_t* nsteps, const double* amp,
                       int count);

/* Destroy a batch (NULL accepted); synchronises its stream. */
int lbem_batch_destroy(lbem_batch_t b);

#ifdef __cplusplus
}
#endif
#endif /* LBEM_H */
