/*
 * CPU oracle for the deviational phonon Monte Carlo tracer (test infrastructure).
 *
 * This is a plain, slow, FP64 implementation of the linearized deviational
 * energy-based Monte Carlo method of Pathak et al., "MCBTE: A variance-reduced
 * Monte Carlo solution of the linearized Boltzmann transport equation for
 * phonons" (sections 2.4-2.6 for the equations, section 3 for the particle
 * method).  It exists only to check the HIP library: only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or constant with the library.
 *
 * Every function that can be pinned to something other than itself is pinned
 * by the CPU test suite (closed forms, invariants, brute force); see the tests.
 */
#ifndef MCBTE_ORACLE_H
#define MCBTE_ORACLE_H
#include <stdint.h>

#define ORC_MAX_CYL 8
#define ORC_MAX_WALL 16
#define ORC_N_COUNTS 16
#define ORC_N_MOMENTS 4

/* one material row: first format uses dos/domega, second format gives C */
typedef struct { double omega, dos, v, domega, tau, C, tau_imp; int32_t bin, branch; } orc_mode;
/* spec_table (faces, pores, adiabatic walls): k >= 1 reads the phonon's specularity from row m of
   the problem's k-th per-row table (the boundary's own d and cutoff are then 0); 0 = none */
typedef struct { int32_t type, spec_table; double data[3]; } orc_face;
/* pore: spec is the degree of specularity d; spec_wc > 0 makes phonons with omega < spec_wc reflect
   specularly whatever d is (frequency-dependent specularity, as in the paper's nanomesh with the
   phonons below 2 THz specular).  Adiabatic faces carry the same cutoff in data[1]. */
typedef struct { double cx, cy, r; int32_t id, type; double spec, spec_wc; int32_t spec_table, pad; } orc_cyl;
/* internal line wall (the paper's In_bnd rows): the segment (x1, y1)-(x2, y2) in the x-y plane,
   extended through the thickness, normal (nx, ny) pointing into the domain; adiabatic (spec = the
   specularity, spec_wc the cutoff, as for pores) or isothermal (spec = T_b: it absorbs and
   emits); ids above the pores' */
typedef struct { double x1, y1, x2, y2, nx, ny; int32_t id, type; double spec, spec_wc; int32_t spec_table, pad; } orc_wall;
typedef struct {
    double L[3];
    int32_t unbounded[3];
    int32_t n_cyl;
    orc_face face[6];          /* face[id - 1], ids in the paper's boundary-table order */
    orc_cyl cyl[ORC_MAX_CYL];
    double gradT[3];
    double volume;             /* solid volume; <= 0 means: computed from the geometry */
    int32_t n_wall, pad_w;
    orc_wall wall[ORC_MAX_WALL];
} orc_geom;
typedef struct { double lo[3], hi[3]; int32_t n[3]; int32_t mask; } orc_det;
typedef struct {
    int64_t N, max_events;
    double T_lin, t_max;
    int32_t n_scat_max, format, transient, score_axis;
    int32_t n_times, ic_axis, n_ic, n_spec_tables;
    const double* t_meas;
    const double* ic_edges;
    const double* ic_dT;
    const double* spec_table;  /* n_spec_tables x M degrees of specularity, table-major */
    /* external heat source (transient): power density heat_P[k] (W/m^3, signed) over
       [heat_t[k], heat_t[k+1]) in the cuboid [heat_lo, heat_hi] (bounded axes), or, when
       n_heat_tet > 0, in the union of the tetrahedra heat_tet (4 vertices x 3 coordinates each) */
    int32_t n_heat, n_heat_tet;
    double heat_lo[3], heat_hi[3];
    const double* heat_t;
    const double* heat_P;
    const double* heat_tet;
} orc_problem;

typedef struct orc_tables orc_tables;

/* counters (indices into the uint64 counts array) */
enum {
    ORC_C_PARTICLES = 0, ORC_C_FLIGHTS, ORC_C_RELAX, ORC_C_SPECULAR, ORC_C_DIFFUSE, ORC_C_PERIODIC,
    ORC_C_ABSORBED, ORC_C_TIMEOUT, ORC_C_NSCAT_END, ORC_C_CAP_END, ORC_C_ESCAPED, ORC_C_REJECT,
    ORC_C_TWO
};
/* event-log entry types */
enum {
    ORC_EV_EMIT_POS = 0, ORC_EV_RELAX = 1, ORC_EV_SPECULAR = 2, ORC_EV_DIFFUSE = 3,
    ORC_EV_PERIODIC = 4, ORC_EV_ABSORB = 5, ORC_EV_TIMEOUT = 6, ORC_EV_NSCAT_END = 7,
    ORC_EV_CAP_END = 8, ORC_EV_EMIT_NEG = 9, ORC_EV_ESCAPE = 10, ORC_EV_TWO = 11
};

int orc_build(const orc_mode* modes, int32_t M, const orc_geom* g, const orc_det* det,
              const orc_problem* pr, orc_tables** out);
void orc_free(orc_tables* t);
/* doubles: C_tot, sum C v, e_eff, V_solid, E_tot, kappa_bulk; ints: M, S, n_cells, n_cols, n_bins */
void orc_info(const orc_tables* t, double* d6, int64_t* i5);
/* which: 0 C, 1 thr_ic, 2 thr_wall, 3 thr_rel, 4 src_E, 5 thr_src, 6 src_sign, 7 last-index x4,
   8 relaxation probability per bin, 9 bin of each mode */
int orc_get(const orc_tables* t, int32_t which, void* out, int64_t n);
int orc_trace(const orc_tables* t, uint64_t seed, uint32_t instance, int64_t first_pid, int64_t n,
              double* raw, uint64_t* counts, double* moments,
              uint32_t* log, int64_t n_log, int32_t log_stride);

/* sensitivity sums for dkappa / dln tau_i over particles first_pid .. first_pid + n - 1 (steady
   runs).  kind 0, score function: sparse[n_bins] += sum_e g_e (F - F_before_e) over the flights and
   relaxation draws; kind 1, pathwise: sparse[n_bins] += the tangent terms s dx_a of the flights plus
   the draw terms; kind 2, local pathwise: for modes with v tau <= lambda_split a flight ended by a
   relaxation adds s L Omega_a + (T/tau - 1) (F - F at its end) and one cut short adds nothing,
   other modes and the draws as for kind 0.  All: *dense += sum over relaxation draws of
   (F - F_before).  F_out[i] (optional) = flux contribution of each particle; pp_out[i * n_bins +
   bin] (optional, kind 1) += the tangent terms of particle i.  A tangent term that is not finite is
   left out of the sums and counted in *n_bad (optional). */
int orc_adjoint(const orc_tables* t, uint64_t seed, uint32_t instance, int64_t first_pid, int64_t n,
                int32_t kind, double lambda_split, double* sparse, double* dense, double* F_out, double* pp_out,
                int64_t* n_bad);

/* building blocks exposed for the pins */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_record(uint64_t seed, uint32_t instance, int64_t pid, uint32_t rec, uint32_t W[8]);
int64_t orc_cdf_pick(const uint64_t* thr, int64_t n, int64_t last, uint64_t K);
void orc_cdf_build(const double* w, int64_t n, uint64_t* thr, int64_t* last);
void orc_dir_iso(double u1, double u2, double out[3]);
void orc_dir_cos(double u1, double u2, const double n[3], double out[3]);
double orc_dedT(double omega, double T);
/* emitted state of one particle: d8 = x, y, z, ox, oy, oz, t, dt_rem; i4 = mode, sign, source, rejections */
int orc_emit_state(const orc_tables* t, uint64_t seed, uint32_t instance, int64_t pid, double* d8, int32_t* i4);
/* its two clocks (tables with a two-phonon process): lead of the later one, and 1 if the next
   scattering is the two-phonon one */
int orc_emit_clocks(const orc_tables* t, uint64_t seed, uint32_t instance, int64_t pid, double* lead, int32_t* nx2);
/* nearest boundary along a ray: distance and boundary id (0: none) */
double orc_next_boundary(const orc_tables* t, const double x[3], const double o[3], int32_t* hit);
/* tally one straight steady segment into raw (testing the detector clipping) */
void orc_tally_segment(const orc_tables* t, const double x0[3], const double o[3], double d, int32_t m,
                       double s, double* raw);

#endif
