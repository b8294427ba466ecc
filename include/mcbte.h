/*
 * mcbte.h -- C ABI of the MI355X (gfx950) deviational phonon Monte Carlo tracer.
 *
 * The library runs the hot path of the linearized, deviational, energy-based
 * Monte Carlo solution of the phonon Boltzmann transport equation of Pathak et
 * al. ("MCBTE", Computer Physics Communications): deviational energy bundles are
 * emitted from sources (section 3.2), fly exponential free paths (section 3.3),
 * relax by redrawing frequency and direction (section 3.5.2), reflect, are
 * absorbed or are reinserted at boundaries (sections 3.5.3-3.5.5), and are scored
 * into temperature and heat-flux detectors (sections 3.4 and 3.6).
 *
 * Conventions of the whole interface:
 *   - every function returns an int status: MCBTE_OK (0) or a negative MCBTE_E*
 *     code; nothing throws across the ABI; mcbte_strerror() names the code;
 *   - SI units (m, s, rad/s, J, K);
 *   - "device pointer" = memory of the HIP device the tables were built for
 *     (e.g. a torch.cuda tensor's data_ptr()); "host pointer" = CPU memory;
 *   - "stream" = a hipStream_t passed as void* (NULL = the null stream); device
 *     work is enqueued asynchronously unless a function says it synchronizes;
 *   - tables are library-owned and opaque; particle-state, tally and event-log
 *     buffers are caller-owned device memory; the library allocates nothing per
 *     call (device memory is allocated only by mcbte_build_tables);
 *   - calls on distinct table handles and distinct tally buffers are
 *     thread-safe; calls sharing a tally buffer must be ordered on one stream.
 */
#ifndef MCBTE_H
#define MCBTE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MCBTE_OK 0
#define MCBTE_EINVAL (-1)   /* an argument is out of range or inconsistent            */
#define MCBTE_ENOMEM (-2)   /* host or device allocation failed                       */
#define MCBTE_EHIP (-3)     /* a HIP runtime call failed                              */
#define MCBTE_ENODEV (-4)   /* host-only tables (device = -1) passed to a device call */
#define MCBTE_ETABLE (-5)   /* a distribution or the source list has zero weight      */
#define MCBTE_EGEOM (-6)    /* geometry not closed / periodic faces not paired / pore outside */
#define MCBTE_ESIZE (-7)    /* a caller buffer is smaller than required               */
#define MCBTE_ERANGE (-8)   /* a sensitivity term was not finite (mcbte_adjoint_finalize) */
#define MCBTE_ELIMIT (-9)   /* more instances than mcbte_trace_batch_static's fixed scratch holds */

/* boundary types (order of the paper's boundary table, section 4.3) */
#define MCBTE_ISOTHERMAL 1  /* data[0] = wall temperature T_b                       */
#define MCBTE_ADIABATIC 2   /* data[0] = specularity d in [0, 1]                    */
#define MCBTE_PERIODIC 3    /* data = translation vector (must map the face onto its partner) */

/* tally component mask bits */
#define MCBTE_TALLY_T 1
#define MCBTE_TALLY_QX 2
#define MCBTE_TALLY_QY 4
#define MCBTE_TALLY_QZ 8

#define MCBTE_MAX_PORES 8
#define MCBTE_MAX_WALLS 16

/* Sensitivity estimators (mcbte_adjoint). */
#define MCBTE_SENS_SCORE 0          /* likelihood ratio: any steady problem                     */
#define MCBTE_SENS_PATHWISE 1       /* flight lengths differentiated along the trajectory       */
#define MCBTE_SENS_LOCAL 2          /* a flight's own flux through its length, the rest scored   */
#define MCBTE_PATHWISE_MAX_FLIGHTS 16 /* pathwise: n_scat_max must lie in [1, this]             */
#define MCBTE_N_COUNTS 16

/* counters, indices into the counts array of the tally buffer (all uint64) */
enum {
    MCBTE_CNT_PARTICLES = 0, MCBTE_CNT_FLIGHTS = 1, MCBTE_CNT_RELAXATIONS = 2, MCBTE_CNT_SPECULAR = 3,
    MCBTE_CNT_DIFFUSE = 4, MCBTE_CNT_PERIODIC = 5, MCBTE_CNT_ABSORBED = 6, MCBTE_CNT_TIMEOUT = 7,
    MCBTE_CNT_NSCAT_END = 8, MCBTE_CNT_CAP_END = 9, MCBTE_CNT_ESCAPED = 10, MCBTE_CNT_REJECTIONS = 11,
    MCBTE_CNT_TWO_PHONON = 12
};

/* One material row (section 4.1).  First format: omega, dos (s rad^-1 m^-3), v, domega, tau;
   the heat capacity is then dos * domega * de/dT(omega, T_lin) (Eq. BE_derivative with the
   half argument, x = hbar omega / k_B T: k_B (x/2)^2 / sinh^2(x/2)).  Second format: omega, v,
   tau and C (J m^-3 K^-1) given directly; dos / domega ignored.  tau is the three-phonon
   relaxation time.  tau_imp > 0 (finite) gives the row the separate two-phonon (impurity)
   process of section 3.3 with its own clock: both times to scattering are drawn from Eq.
   time_to_scat, the earlier one fires (a tie goes to the three-phonon one); a two-phonon event
   keeps the phonon and draws a new isotropic direction and a new two-phonon time (section
   3.5.1) while the three-phonon clock runs on; a three-phonon event redraws the phonon and both
   times; N_scat^max counts three-phonon events only.  The two-phonon time drawn at the j-th
   random-number-drawing event (j = 0 at emission) uses words W0W1 of record 0x60000000 + j.
   tau_imp = 0: no two-phonon process (Matthiessen's rule, if wanted, is then folded into tau).
   bin: frequency-bin index (for per-bin outputs). */
typedef struct {
    double omega, dos, v, domega, tau, C, tau_imp;
    int32_t bin, branch;
} mcbte_mode;

/* boundary-table row (section 4.2): isothermal data[0] = T_b; periodic data = the translation
   vector; adiabatic data[0] = d (degree of specularity, section 3.5.3) and data[1] = a cutoff
   angular frequency (rad/s, >= 0): a phonon with omega below it reflects specularly whatever d
   is (the frequency-dependent specularity of the paper's nanomesh, phonons below 2 THz
   specular); 0 = none.
   Specularity per phonon (section 3.5.3: d depends on the wavelength): an adiabatic boundary
   whose spec_table is k >= 1 reflects a phonon of table row m specularly with probability
   problem->spec_table[(k - 1) * n_modes + m]; its own d and cutoff must then be 0.  The cutoff is
   the special case of a table holding 1 below the cutoff and d above it.  spec_table = 0: none;
   other boundary types must have 0. */
typedef struct {
    int32_t type;               /* MCBTE_ISOTHERMAL / _ADIABATIC / _PERIODIC */
    int32_t spec_table;         /* adiabatic: 1-based specularity table of the problem, 0 = none */
    double data[3];
} mcbte_face;

/* internal boundary: a cylindrical pore with axis along z through (cx, cy), adiabatic wall */
typedef struct {
    double cx, cy, r;
    int32_t id;                 /* boundary id, >= 7, strictly increasing over the array */
    int32_t type;               /* MCBTE_ADIABATIC */
    double specularity;
    double spec_omega;          /* cutoff angular frequency below which reflection is specular (0: none) */
    int32_t spec_table;         /* 1-based specularity table of the problem (0: none), as for faces */
    int32_t reserved;           /* must be 0 */
} mcbte_pore;

/* internal line wall (the paper's In_bnd rows, section 4.2): the segment (x1, y1)-(x2, y2) in the
   x-y plane extended through the thickness, (nx, ny) its normal pointing into the domain (unit
   length within 1e-9; normalized by the library).  A wall is met only from the side its normal
   points to.  Adiabatic (data = specularity d, optional cutoff angular frequency): it reflects like
   a pore.  Isothermal (data = T_b): it absorbs, and emits like an isothermal face (energy
   A |T_b - T_lin| sum C v / 4, A = length x thickness, directions about its normal).  Ids
   continue after the pores' (> every pore id, strictly increasing).  Emission leaves out the
   inside of every closed loop of walls (consecutive walls each starting where the previous one
   ends, the last ending where the first starts); walls in no loop exclude nothing. */
typedef struct {
    double x1, y1, x2, y2, nx, ny;
    int32_t id;
    int32_t type;               /* MCBTE_ADIABATIC or MCBTE_ISOTHERMAL */
    double data;                /* adiabatic: specularity d; isothermal: T_b (K) */
    double spec_omega;
    int32_t spec_table;         /* adiabatic: 1-based specularity table of the problem (0: none) */
    int32_t reserved;           /* must be 0 */
} mcbte_wall;

/* Box [0, L0] x [0, L1] x [0, L2] (one corner at the origin, section 4.2).  face[id - 1] holds
   boundary id 1..6 in the paper's order: 1 y=0, 2 x=L0, 3 y=L1, 4 x=0, 5 z=0, 6 z=L2.  An axis
   with unbounded[a] != 0 has no faces (translation-invariant direction, lengths taken as 1 m
   for areas and volumes; positions along it start at 0).  gradT is the uniform temperature
   gradient of the spatially varying control (section 2.6); volume is the solid volume
   (section 4.4; <= 0: box volume minus the pores; must be given when there are line walls). */
typedef struct {
    double L[3];
    int32_t unbounded[3];
    int32_t n_pores;
    mcbte_face face[6];
    mcbte_pore pore[MCBTE_MAX_PORES];
    double gradT[3];
    double volume;
    int32_t n_walls;
    int32_t reserved_w;
    mcbte_wall wall[MCBTE_MAX_WALLS];
} mcbte_geometry;

/* Detector grid (section 4.5): the cuboid [lo, hi] split into n[a] equal cells along each axis
   with n[a] > 0; axes with n[a] == 0 are not binned.  mask selects the accumulated components
   (MCBTE_TALLY_*).  Cells are numbered x-major: ((ix * ny) + iy) * nz + iz (n == 0 counts as 1). */
typedef struct {
    double lo[3], hi[3];
    int32_t n[3];
    int32_t mask;
} mcbte_detectors;

/* Run parameters (sections 4.4-4.5).  N: number of computational particles that share the
   total deviational energy (effective energy E_tot / N).  transient: snapshot tallies at the
   n_times sorted times t_meas (< t_max), particles end at t_max; wall and gradient sources
   emit uniformly over [0, t_max).  Steady: track-length tallies, one column per mode.
   Initial condition (transient only): n_ic cells along axis ic_axis with edges ic_edges[0..n_ic]
   and cell-averaged temperature deviations ic_dT[0..n_ic-1].  n_scat_max: relaxations after
   which a particle ends (0 = unlimited).  max_events: cap on segments per particle (counted in
   MCBTE_CNT_CAP_END).  score_axis: flux component used for kappa and its standard error.
   spec_table: n_spec_tables tables of n_modes degrees of specularity in [0, 1] each (row-major),
   referenced by the boundaries' spec_table numbers (section 3.5.3); may be NULL when
   n_spec_tables = 0.
   External heat source (transient only; the phonon generation by an external source that the
   summary section names for time-domain thermoreflectance): deviational power density heat_P[k]
   (W m^-3, either sign) over [heat_t[k], heat_t[k+1]), k < n_heat, in the cuboid
   [heat_lo, heat_hi] (bounded axes; an unbounded axis takes its whole 1 m).  Interval k is a
   source of energy |heat_P[k]| V_heat (heat_t[k+1] - heat_t[k]) and sign that of heat_P[k]; its
   particles start at a time uniform in the interval, at a position uniform in the cuboid, with a
   row drawn by heat capacity (the equilibrium distribution of a temperature rise, as for the
   initial condition) and an isotropic direction (emission record 2, words W2W3, gives the time).
   The cuboid lies inside the box and inside the solid (no pore or line wall reaches into it);
   0 <= heat_t[0] < ... <= t_max.  n_heat = 0: none.  Regions of any shape (section 3.2 builds them
   from tetrahedra): with n_heat_tet > 0 the region is instead the union of the tetrahedra heat_tet
   (4 vertices x 3 coordinates each, inside the box, positive volume, the x-y bounding rectangle
   of each clear of every pore); a particle's tetrahedron is drawn by volume (emission record 2,
   words W4W5) and its point uniformly inside it from the three position uniforms (the folding of
   the unit cube onto the tetrahedron of Rocchini and Cignoni, 2000).
   All pointers are host pointers, read during mcbte_build_tables only. */
typedef struct {
    int64_t N, max_events;
    double T_lin, t_max;
    int32_t n_scat_max, format, transient, score_axis;
    int32_t n_times, ic_axis, n_ic, n_spec_tables;
    const double* t_meas;
    const double* ic_edges;
    const double* ic_dT;
    const double* spec_table;
    int32_t n_heat, n_heat_tet;
    double heat_lo[3], heat_hi[3];
    const double* heat_t;
    const double* heat_P;
    const double* heat_tet;
} mcbte_problem;

typedef struct mcbte_tables mcbte_tables;

/* Derived quantities of a table set. */
typedef struct {
    double C_tot;        /* sum of the per-mode heat capacities (J m^-3 K^-1)              */
    double sum_Cv;       /* sum_m C_m v_m                                                  */
    double E_tot;        /* total deviational energy (transient, J) or energy rate (steady, W) */
    double e_eff;        /* E_tot / N                                                      */
    double V_solid;      /* solid volume (m^3)                                             */
    double kappa_bulk;   /* sum_m C_m v_m^2 tau_m / 3                                      */
    int64_t n_modes, n_sources, n_cells, n_cols;
    int64_t tally_bytes; /* size of the tally buffer mcbte_trace needs                     */
    int64_t n_bins;      /* frequency bins (1 + largest mcbte_mode.bin)                    */
    int64_t adj_doubles; /* doubles of the buffer mcbte_adjoint needs (n_bins + 3)         */
    int32_t device;      /* HIP device ordinal, -1 for host-only tables                    */
    int32_t reserved;
} mcbte_info;

/* Trace options. */
typedef struct {
    uint64_t seed;        /* Philox key                                                     */
    uint32_t instance;    /* fourth counter word of every Philox draw                       */
    int32_t precision;    /* 64: FP64 trajectories; 32: FP32 trajectories, FP64 tables and sums */
    int32_t block;        /* threads per workgroup: multiple of 64, <= 256 (0 = 256); <= 1024
                             (0 = 1024) for an FP32 trace whose FP64 tally is too large for a
                             per-workgroup LDS copy while its FP32 tally fits the whole LDS: those
                             run wide workgroups, the mode tables read from HBM */
    int32_t refill;       /* flights between refills of finished lanes (>= 1; 0 = default)  */
    int32_t grid;         /* workgroups (0 = enough to fill every compute unit)             */
    int32_t log_stride;   /* uint32 words per event-log row (>= 2)                          */
    int64_t n_log;        /* particles logged (first_pid .. first_pid + n_log - 1)          */
    uint32_t* event_log;  /* device pointer, n_log * log_stride uint32, or NULL             */
    double* particle_F;   /* device pointer, n doubles, or NULL: mcbte_trace writes each particle's
                             flux score F (sum of s l Omega_score over its segments) at index
                             pid - first_pid, the input of mcbte_adjoint                     */
    int32_t flags;        /* MCBTE_RUN_* bits (0: defaults)                                 */
    int32_t reserved;     /* must be 0                                                      */
} mcbte_run;

/* mcbte_run.flags.  MCBTE_RUN_SEGMENTS: trace a periodic pore lattice one segment at a time in the
   FP32 form too.  By default an FP32 steady trace of a cell that is periodic in x and y (periodic or
   unbounded in z) with one pore and no line walls follows a particle with a long free path from pore
   to pore with its whole wave, in the lattice's unfolded coordinates (a transfer through a periodic
   face reinserts the particle unchanged at the partner face, Eq. periodic_lin_final, which is flying
   on through the lattice): the same events and counts, the FP32 positions rounded differently.  The
   FP64 form always steps one segment at a time (its event sequences are the oracle's).  A sensitivity
   replay must use the flags of the forward trace that wrote particle_F. */
#define MCBTE_RUN_SEGMENTS 1

/* Finalized results (mcbte_tally). */
typedef struct {
    uint64_t counts[MCBTE_N_COUNTS];
    double moments[4];    /* sum c_T, sum c_T^2, sum c_q, sum c_q^2 over particles          */
    double e_eff;         /* E_tot / particles traced                                        */
    double V_cell;        /* detector cell volume used for the normalization                */
    double T_mean, T_mean_sigma;     /* steady: solid-averaged temperature deviation (K)    */
    double q_score, q_score_sigma;   /* steady: solid-averaged flux along score_axis (W/m^2) */
    double kappa, kappa_sigma;       /* steady: -q_score / gradT[score_axis] (0 if no gradient) */
    double kappa_cell_avg;           /* kappa * V_solid / box volume                         */
} mcbte_result;

/* Build the tables of one problem (section 3.1: source energies and effective energy; section
   3.2: the cumulative distributions of Eq. cumul_freq for emission from initial conditions
   (weight C_m), walls and the gradient source (weight C_m v_m, Eqs. iso_flux and grad_flux),
   and relaxation (weight C_m / tau_m, Eqs. norm_post_coll and n_scatt)).  Host FP64; then, if
   device >= 0, uploads the tables to that device (synchronous).  device = -1 builds host-only
   tables for inspection (mcbte_table_info / mcbte_table_export).  All input pointers are host
   pointers and are not retained.  Errors: MCBTE_EINVAL (bad row, detector or run parameter),
   MCBTE_EGEOM, MCBTE_ETABLE, MCBTE_ENOMEM, MCBTE_EHIP.  *out is NULL on error. */
int mcbte_build_tables(const mcbte_mode* modes, int32_t n_modes, const mcbte_geometry* geometry,
                       const mcbte_detectors* detectors, const mcbte_problem* problem, int32_t device,
                       mcbte_tables** out);

/* Release tables and their device memory (NULL is ignored).  Synchronizes the device first. */
void mcbte_free_tables(mcbte_tables* tables);

/* Copy the derived quantities into *info (host). */
int mcbte_table_info(const mcbte_tables* tables, mcbte_info* info);

/* Copy one host-side table into host_out (n elements available): which = 0 C_m (double[M]),
   1/2/3 initial-condition / wall / relaxation thresholds (uint64[M]), 4 source energies
   (double[S]), 5 source thresholds (uint64[S]), 6 source signs (int32[S]).  Threshold j is
   floor(F_j 2^64) saturated at 2^64 - 1; a 64-bit key K selects the first j with K < threshold. */
int mcbte_table_export(const mcbte_tables* tables, int32_t which, void* host_out, int64_t n);

/* Bytes of the particle-state buffer for `capacity` particles at `precision` (32 or 64); < 0 on
   a bad argument.  Layout (structure of arrays, each array 256-byte aligned): x, y, z, ox, oy, oz,
   t, dt_rem (real; dt_rem is the time left until the next scattering), then mode, sign, n_rel,
   segments, draws, source, rejections (int32 / uint32), then lead (real: with two clocks, how
   much later the other clock fires, sign bit set when the next one is the two-phonon clock). */
int64_t mcbte_state_bytes(int32_t precision, int64_t capacity);

/* Emit particles first_pid .. first_pid + n - 1 (section 3.2: source chosen by deviational
   energy, position, frequency, direction, sign, start time, first free flight of Eq.
   time_to_scat) into the device state buffer `state` (mcbte_state_bytes(run->precision,
   capacity) bytes, capacity >= n); slot i holds particle first_pid + i.  Async on `stream`.
   Errors: MCBTE_EINVAL, MCBTE_ENODEV, MCBTE_EHIP. */
int mcbte_emit(const mcbte_tables* tables, const mcbte_run* run, int64_t first_pid, int64_t n, void* state,
               int64_t capacity, void* stream);

/* Trace particles first_pid .. first_pid + n - 1 to termination and add their scores to the
   device tally buffer `tally` (mcbte_table_info().tally_bytes bytes, zeroed by the caller before
   the first trace; successive traces accumulate).  With state == NULL the particles are emitted
   inside the trace kernel (same draws as mcbte_emit); otherwise `state` holds them as written by
   mcbte_emit with the same run->precision and first_pid and with capacity == n (the layout of
   the state buffer depends on its capacity).  Flight loop: section 3.3 (free flight,
   boundary interruption of case iii), events of section 3.5, termination of section 3.5.6;
   tallies: Eq. sampling (transient) or Eqs. temp_steady / flux_x_steady (steady).  Async on
   `stream`.  Errors: MCBTE_EINVAL, MCBTE_ENODEV, MCBTE_EHIP.
   Tally buffer layout (bytes): [0,128) counts uint64[16]; [128,160) moments double[4];
   [192,256) library scratch (work counters); [256, ...) raw sums double[n_cells][n_cols][4] with
   components (sum s l / v | sum s, sum s l Omega_x | sum s v Omega_x, ... y, ... z); for a pore
   lattice (see MCBTE_RUN_SEGMENTS) the FP32 trace also keeps, after the raw sums, a list of the
   particles whose first free flight exceeds 1000 cell widths, which it starts before the others
   (an order that changes no result; more than 4096 of them and it takes every particle in order).
   Event log rows (if run->event_log): word 0 = number of entries, then entries
   (type << 28) | (min(boundary id or source index, 255) << 20) | mode, types 0 emit (sign +),
   9 emit (sign -), 1 relaxation (new mode), 2 specular, 3 diffuse, 4 periodic, 5 absorbed,
   6 time horizon, 7 N_scat^max reached, 8 segment cap, 10 escaped, 11 two-phonon scattering. */
int mcbte_trace(const mcbte_tables* tables, const mcbte_run* run, int64_t first_pid, int64_t n,
                const void* state, void* tally, void* stream);

/* Batched form: instance i traces particles 0 .. n_particles[i] - 1 of tables[i] with Philox
   instance word instance_ids[i] into tallies[i], all in one persistent launch whose workgroups
   pull (instance, particle chunk) work items from a shared queue.  All tables must be built for
   the same device with the same transient flag; run->instance is ignored; the event log is not
   supported (run->event_log must be NULL).  `queue` is a caller-owned device buffer of at least
   mcbte_batch_queue_bytes(n_inst) bytes (its contents are overwritten); the work table is
   uploaded into it and `stream` is synchronized once before the launch, which is then async. */
int64_t mcbte_batch_queue_bytes(int32_t n_inst);
int mcbte_trace_batch(const mcbte_tables* const* tables, int32_t n_inst, const int64_t* n_particles,
                      const uint32_t* instance_ids, void* const* tallies, const mcbte_run* run, void* queue,
                      void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
   that forbid hipMalloc): mcbte_trace_batch without the queue argument.  The work queue lives in a
   file-scope static device array of the library (about 206 KB, enough for
   MCBTE_STATIC_MAX_INSTANCES instances), which each device holds from its first use until the
   process ends; the work table reaches it through a setup kernel's arguments on `stream`, so the
   call allocates nothing, copies nothing from the host and does not synchronize (fully
   asynchronous on `stream`).  Every call on a device shares that one array: calls that overlap on
   one device (other streams, other threads) race and must be ordered by the caller; a call's
   queue counter is cleared by its own setup kernel.  Same arguments and results as
   mcbte_trace_batch (run->particle_F must be NULL as well).  Errors: as mcbte_trace_batch, and
   MCBTE_ELIMIT when n_inst > MCBTE_STATIC_MAX_INSTANCES. */
#define MCBTE_STATIC_MAX_INSTANCES 64
int mcbte_trace_batch_static(const mcbte_tables* const* tables, int32_t n_inst, const int64_t* n_particles,
                             const uint32_t* instance_ids, void* const* tallies, const mcbte_run* run, void* stream);

/* Launch-shape autotuner.  The launch shape -- threads per workgroup and the refill period
   (flights between refills of finished lanes) -- changes no result (every integer count and
   trajectory is the same; only the order of floating-point tally sums moves), only the speed.
   The candidates are block in {64, 128, 192, 256, 512, 1024} x refill in {1, 2, 4, 8, 16, 32},
   numbered block-major (candidate c: block {64, 128, 192, 256, 512, 1024}[c / 6], refill
   2^(c % 6)); a block size the problem's kernel cannot take (above 256 except for the wide FP32
   kernel, see mcbte_run) counts as +inf.  Each is timed (HIP events on
   `stream`) over `reps` launches after one warm-up launch, on a calibration run of the caller's
   problem: n_inst == 1, particles 0 .. n_probe - 1 of tables[0] (mcbte_trace); n_inst > 1, the
   batched form (mcbte_trace_batch) with every instance's particle count scaled by
   n_probe / sum(n_particles) (at least one particle each), keeping the mix of instances.
   *out = *base with the fastest block and refill (grid left as in *base).  timings (optional,
   host, n_timings >= MCBTE_TUNE_CANDIDATES) receives the fastest time of each candidate in ms
   (+inf for one that cannot launch).  tallies / queue: caller-owned device buffers as for
   mcbte_trace / mcbte_trace_batch (instance_ids and queue are ignored when n_inst == 1); their
   contents are meaningless afterwards.  base->event_log and base->particle_F must be NULL.
   Synchronizes `stream`.  Errors: MCBTE_EINVAL, MCBTE_ENODEV, MCBTE_EHIP, MCBTE_ESIZE. */
#define MCBTE_TUNE_CANDIDATES 36
int mcbte_autotune(const mcbte_tables* const* tables, int32_t n_inst, const int64_t* n_particles,
                   const uint32_t* instance_ids, void* const* tallies, void* queue, const mcbte_run* base,
                   int64_t n_probe, int32_t reps, mcbte_run* out, double* timings, int32_t n_timings, void* stream);

/* Sensitivity of kappa to a relative change of the relaxation times of each frequency bin,
   dkappa / dln tau_i (steady runs with a gradient), by one of two estimators.
   MCBTE_SENS_SCORE (likelihood ratio): every random quantity whose law depends on tau contributes
   its score times the part of the particle's flux score that follows it -- a free flight (Eq.
   time_to_scat) that ends in a relaxation scores T/tau - 1, one cut short (absorbed, segment cap)
   T/tau, both for the flying mode's bin; a relaxation draw of row j (Eq. norm_post_coll) scores
   -[bin(j) = i] + P_i, P_i the bin's share of the post-scattering distribution.
   MCBTE_SENS_PATHWISE: a flight's distance L = v tau E is stretched by dL / dln tau = L with its
   random numbers E fixed, the change carried along the rest of the trajectory with the event
   sequence held fixed (boundary hits slide along the surface, reflections off the cylinder turn
   with its normal) into the change of the particle's net displacement along the scored axis; the
   relaxation draws keep their likelihood-ratio terms.  Lower variance; unbiased where a
   stretched flight cannot change the event sequence on average -- adiabatic walls and periodic
   faces -- but not at isothermal walls (a flight ending just before or just after one changes
   what follows).  Requires 1 <= n_scat_max <= MCBTE_PATHWISE_MAX_FLIGHTS.  Its variance grows with
   the mean free path against the geometry: a stretch moves a flight's end by L Omega, and between
   convex pores (a dispersing billiard) the shifts grow geometrically with the number of
   reflections, so for mean free paths beyond the pore size the terms can overflow; a particle
   term that is not finite is left out of the sums and counted, and mcbte_adjoint_finalize then
   reports MCBTE_ERANGE.
   MCBTE_SENS_LOCAL: for modes whose mean free path v tau is at most lambda_split (<= 0: the
   smallest bounded extent of the cell or pore diameter; every mode of the unbounded bulk), a
   flight ended by a relaxation adds its own flux's change s L Omega_a (L = v tau E stretched with
   E fixed, Omega its last direction) plus (T/tau - 1) times the flux score that follows it, a flight
   cut short adds nothing; longer modes and the relaxation draws as for MCBTE_SENS_SCORE.  Unbiased
   everywhere (the own flux is continuous in the flight time, what follows is scored), with lower
   variance where short flights carry the flux; nothing is propagated, so no growth.
   mcbte_adjoint replays particles first_pid .. first_pid + n - 1 with the same random streams
   (run->seed, run->instance, run->precision as the forward trace that filled particle_F, a
   device array of n doubles) and adds the sums to `adj` (device, adj_doubles doubles, zeroed by
   the caller; successive calls with one estimator accumulate): adj[0, n_bins) the per-bin sums,
   adj[n_bins] the relaxation-draw sum B, adj[n_bins + 1] the count of terms left out as not
   finite, adj[n_bins + 2] library scratch.  Async on `stream`.  Errors: MCBTE_EINVAL (transient run, event log set, unknown
   estimator, n_scat_max outside the pathwise range, tables with a two-phonon clock, a specular
   cutoff frequency or internal line walls, the pathwise estimator in the FP32 form on a pore lattice
   without MCBTE_RUN_SEGMENTS: the replay follows the forward trace segment by segment and the
   pathwise tangents are carried through every transfer), MCBTE_ENODEV, MCBTE_EHIP. */
int mcbte_adjoint(const mcbte_tables* tables, const mcbte_run* run, int32_t estimator, double lambda_split,
                  int64_t first_pid, int64_t n, const double* particle_F, double* adj, void* stream);

/* Copy `adj` to the host (synchronizes `stream`) and write dkappa / dln tau_i, i < n_bins, into
   host_out (n_out >= n_bins) for n_particles traced particles, with the normalisation of kappa
   (-E_tot / (V_solid gradT_score n_particles)).  dkappa / dtau_i = host_out[i] / tau_i.  Returns
   MCBTE_ERANGE (host_out still written) when terms were left out as not finite. */
int mcbte_adjoint_finalize(const mcbte_tables* tables, const double* adj, int64_t n_particles, double* host_out,
                           int64_t n_out, void* stream);

/* Copy the device tally buffer to the host (synchronizes `stream`) and finalize it (Eqs.
   sampling, temp_steady, flux_x_steady): host_out[n_cells][n_cols][4] receives the deviational
   temperature T_dev = e (C_tot V_cell)^-1 raw_T and fluxes q_a = e V_cell^-1 raw_a with
   e = E_tot / particles traced; V_cell = V_solid when no axis is binned.  host_out may be NULL
   (n_out ignored); otherwise n_out must be >= n_cells * n_cols * 4.  *result (host) receives
   counters, moments and, for steady runs, kappa with its standard error. */
int mcbte_tally(const mcbte_tables* tables, const void* tally, double* host_out, int64_t n_out,
                mcbte_result* result, void* stream);

/* Batch-mean statistics of tallies: the per-detector output of section 4.5 with its error bar.
   Trajectories are independent (section 6), so separately traced particle groups are independent
   samples of it.  tallies[b], b < n_tallies, are device tally
   buffers of these tables, each filled by its own range of particles (each its own trace calls:
   disjoint ranges of one seed, or other seeds).  Each is finalized as by mcbte_tally; host_mean
   receives the particle-weighted mean over the batches (the finalized sum of all of them) and
   host_sigma its batch-mean standard error sqrt(sum_b n_b (X_b - X)^2 / ((B - 1) N)) per element,
   B the buffers that traced particles (a buffer without particles weighs nothing; NaN for fewer
   than two such buffers; with none at all the mean is 0), both laid out [n_cells][n_cols][4] (n_out >= n_cells * n_cols * 4;
   either may be NULL, not both).  Synchronizes `stream`.  Errors: MCBTE_EINVAL (a NULL buffer,
   n_tallies < 1), MCBTE_ESIZE, MCBTE_ENODEV, MCBTE_EHIP. */
int mcbte_tally_batches(const mcbte_tables* tables, const void* const* tallies, int32_t n_tallies, double* host_mean,
                        double* host_sigma, int64_t n_out, void* stream);

/* Cumulative thermal conductivity (the frequency-resolved flux output of section 4.5, accumulated as
   in section 5.6).  Orders for mcbte_kappa_cumulative: */
#define MCBTE_CUM_MFP 0    /* by table row, rows in ascending mean free path v tau, two clocks
                              combined by Matthiessen's rule (ties by row)                         */
#define MCBTE_CUM_OMEGA 1  /* by frequency bin, bins in ascending lowest angular frequency of their
                              rows (ties by bin; a bin without rows last)                         */
/* For a steady problem with one detector cell (no axis binned) whose mask holds the score axis'
   flux: each row's (bin's) kappa_i = -q_score,i / gradT_score, summed in the order: kappa_cum[k] is
   the sum over the first k + 1 rows (bins), so the last entry is kappa.  keys[k] (may be NULL)
   receives the k-th row's mean free path (m) or bin's angular frequency (rad/s).  With several
   tallies (particle groups, as for mcbte_tally_batches), kappa_cum is the particle-weighted mean
   over them and kappa_cum_sigma (may be NULL) its batch-mean standard error, both as there.
   n_out >= n_modes (MCBTE_CUM_MFP) or n_bins (MCBTE_CUM_OMEGA).  Synchronizes `stream`.  Errors: MCBTE_EINVAL
   (transient or binned tallies, zero gradient along the score axis, flux not tallied, unknown
   order, NULL buffers), MCBTE_ESIZE, MCBTE_ENODEV, MCBTE_EHIP. */
int mcbte_kappa_cumulative(const mcbte_tables* tables, const void* const* tallies, int32_t n_tallies, int32_t order,
                           double* keys, double* kappa_cum, double* kappa_cum_sigma, int64_t n_out, void* stream);

/* Static text for a status code. */
const char* mcbte_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
