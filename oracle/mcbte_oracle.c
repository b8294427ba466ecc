/*
 * CPU oracle (test infrastructure only) for the linearized deviational
 * energy-based phonon Monte Carlo method of Pathak et al. (MCBTE).
 *
 * Plain FP64, one particle at a time, no blocking or reordering beyond what the
 * method states.  Build with -O2 -ffp-contract=off (no fused multiply-adds, no
 * fast-math) so that every arithmetic step rounds exactly as written.
 *
 * Conventions fixed where the paper is silent:
 *   - random numbers: Philox4x32-10, key = seed, counter = (block, pid, instance);
 *     a "record" is two consecutive blocks (eight 32-bit words W0..W7);
 *   - discrete draws invert cumulative distributions held as 64-bit integer
 *     thresholds (the paper's rule F_{j-1} <= R < F_j with a 64-bit R);
 *   - uniforms for continuous draws are 53-bit: u = (K >> 11) 2^-53 in [0, 1);
 *     a free flight uses 1 - u in (0, 1] so that the logarithm is finite;
 *   - ties: the time horizon beats boundaries and relaxations, boundaries beat
 *     relaxations (the segment (x0, x1] is tested), lower boundary id first.
 */
#include "mcbte_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define HBAR 1.054571817e-34     /* J s  */
#define KB 1.380649e-23          /* J/K  */
#define TWO_PI 6.283185307179586
#define PI 3.141592653589793
#define TWO64 18446744073709551616.0

enum { B_ISO = 1, B_ADIA = 2, B_PERI = 3 };
/* S_IWALL: isothermal line wall; S_HEAT: one time interval of the external heat source */
enum { S_WALL = 0, S_GRAD = 1, S_IC = 2, S_IWALL = 3, S_HEAT = 4 };
enum { E_OK = 0, E_INVAL = -1, E_NOMEM = -2, E_TABLE = -5, E_GEOM = -6 };

/* boundary-table order: 1 y=0, 2 x=Lx, 3 y=Ly, 4 x=0, 5 z=0, 6 z=Lz */
static const int FACE_AXIS[6] = {1, 0, 1, 0, 2, 2};
static const int FACE_SIDE[6] = {0, 1, 1, 0, 0, 1};

struct orc_tables {
    int32_t M;
    double *C, *v, *tau;
    double* omega;       /* angular frequency of each row (frequency-dependent specularity) */
    double* spec_tab;    /* per-row specularity tables (n_spec x M), or NULL */
    double* tau2;        /* two-phonon (impurity) relaxation time of each row; 0: no such process */
    int32_t two;         /* some row has a two-phonon clock */
    double C_tot, Wv, kappa_bulk;
    uint64_t *thr_ic, *thr_wall, *thr_rel;
    int64_t last_ic, last_wall, last_rel;
    int32_t S;
    int32_t *src_kind, *src_ref, *src_sign;
    double* src_E;
    uint64_t* thr_src;
    int64_t last_src;
    double E_tot, e_eff, V_solid, gnorm, ngrad[3];
    orc_geom g;
    orc_det det;
    orc_problem pr;
    double *t_meas, *ic_edges, *ic_dT;
    double *heat_t, *heat_P;   /* external heat source: interval edges and power densities */
    double* heat_tet;          /* its tetrahedra (vertex 0 and the three edges from it, 12 per one) */
    uint64_t* thr_tet;         /* choice of a tetrahedron by volume */
    int64_t last_tet;
    int64_t n_cells;
    int32_t n_cols;
    int32_t n_bins;
    int32_t* bin;        /* frequency bin of each mode row */
    double* P_bin;       /* relaxation probability mass of each bin */
};

/* ------------------------------------------------------------------------------------------ */
/* Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).                          */
/* ------------------------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {                       /* Weyl key schedule between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* record rec of particle pid: blocks 2 rec and 2 rec + 1 */
void orc_record(uint64_t seed, uint32_t instance, int64_t pid, uint32_t rec, uint32_t W[8])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint64_t up = (uint64_t)pid;
    uint32_t ctr[4] = {2u * rec, (uint32_t)up, (uint32_t)(up >> 32), instance};
    orc_philox4x32_10(ctr, key, W);
    ctr[0] = 2u * rec + 1u;
    orc_philox4x32_10(ctr, key, W + 4);
}

static uint64_t key64(const uint32_t* W, int i) { return ((uint64_t)W[i] << 32) | (uint64_t)W[i + 1]; }
static double unif(const uint32_t* W, int i) { return (double)(key64(W, i) >> 11) * 0x1p-53; }

/* ------------------------------------------------------------------------------------------ */
/* Cumulative distributions (section 3.2, Eq. cumul_freq): F_j = sum_{i<=j} w_i / sum_i w_i.   */
/* ------------------------------------------------------------------------------------------ */

void orc_cdf_build(const double* w, int64_t n, uint64_t* thr, int64_t* last)
{
    double tot = 0.0;
    int64_t ln = -1;
    for (int64_t i = 0; i < n; ++i) {
        tot += w[i];
        if (w[i] > 0.0) ln = i;
    }
    double run = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        run += w[i];
        double F = run / tot;
        thr[i] = (F >= 1.0) ? UINT64_MAX : (uint64_t)(F * TWO64);
    }
    *last = ln;
}

/* smallest j with K < thr_j, else the last positive-weight index */
int64_t orc_cdf_pick(const uint64_t* thr, int64_t n, int64_t last, uint64_t K)
{
    int64_t lo = 0, hi = n;            /* thr[j] <= K for j < lo, thr[j] > K for j >= hi */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (K < thr[mid]) hi = mid;
        else lo = mid + 1;
    }
    return lo < n ? lo : last;
}

/* ------------------------------------------------------------------------------------------ */
/* Directions.                                                                                 */
/* ------------------------------------------------------------------------------------------ */

/* uniform on the sphere (Eqs. prob_angle, angle_gen): cos(theta) = 1 - 2 R4, phi = 2 pi R5 */
void orc_dir_iso(double u1, double u2, double out[3])
{
    double mu = 1.0 - 2.0 * u1;
    double s2 = (1.0 - mu) * (1.0 + mu);
    double s = sqrt(s2 > 0.0 ? s2 : 0.0);
    double phi = TWO_PI * u2;
    out[0] = s * cos(phi);
    out[1] = s * sin(phi);
    out[2] = mu;
}

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* cosine-weighted hemisphere about the unit vector n (Eq. wall_dir): cos(theta) = sqrt(R6) */
void orc_dir_cos(double u1, double u2, const double n[3], double out[3])
{
    double mu = sqrt(u1);
    double st = sqrt(1.0 - u1);
    double phi = TWO_PI * u2;
    double a = st * cos(phi);
    double b = st * sin(phi);
    int j = 0;
    if (fabs(n[1]) < fabs(n[j])) j = 1;
    if (fabs(n[2]) < fabs(n[j])) j = 2;
    double e[3] = {0.0, 0.0, 0.0};
    e[j] = 1.0;
    double c[3], t1[3], t2[3];
    cross3(e, n, c);
    double len = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    t1[0] = c[0] / len; t1[1] = c[1] / len; t1[2] = c[2] / len;
    cross3(n, t1, t2);
    for (int i = 0; i < 3; ++i) out[i] = mu * n[i] + a * t1[i] + b * t2[i];
}

/* ------------------------------------------------------------------------------------------ */
/* Derivative of the equilibrium energy ħω f_BE with respect to T (Eq. BE_derivative, with the */
/* half argument in the hyperbolic sine): k_B (x/2)^2 / sinh^2(x/2), x = ħω/(k_B T).           */
/* ------------------------------------------------------------------------------------------ */

double orc_dedT(double omega, double T)
{
    double x = (HBAR * omega) / (KB * T);
    double h = 0.5 * x;
    double sh = sinh(h);
    return (KB * (h * h)) / (sh * sh);
}

/* ------------------------------------------------------------------------------------------ */
/* Table build: per-mode heat capacity, the three mode distributions, the source list.        */
/* ------------------------------------------------------------------------------------------ */

static double extent(const orc_geom* g, int a) { return g->unbounded[a] ? 1.0 : g->L[a]; }

/* volume of the tetrahedron with vertices v[0..2], v[3..5], v[6..8], v[9..11]: |det(e1 e2 e3)| / 6 */
static double tet_volume(const double* v)
{
    double e[3][3];
    for (int q = 0; q < 3; ++q)
        for (int a = 0; a < 3; ++a) e[q][a] = v[3 * (q + 1) + a] - v[a];
    const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                       e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                       e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    return fabs(det) / 6.0;
}

/* a point uniform in the tetrahedron v0 + b0 e1 + b1 e2 + b2 e3 (b >= 0, b0 + b1 + b2 <= 1) from three
   uniforms, by folding the unit cube onto the tetrahedron (Rocchini and Cignoni, "Generating random
   points in a tetrahedron", Journal of Graphics Tools 5(4), 2000): the cube's two halves across
   s + t = 1 map onto each other, then the triangular prism's three parts onto the tetrahedron */
static void tet_point(double s, double t, double u, double b[3])
{
    if (s + t > 1.0) {
        s = 1.0 - s;
        t = 1.0 - t;
    }
    if (t + u > 1.0) {
        const double w = u;
        u = 1.0 - s - t;
        t = 1.0 - w;
    } else if (s + t + u > 1.0) {
        const double w = u;
        u = s + t + u - 1.0;
        s = 1.0 - t - w;
    }
    b[0] = s;
    b[1] = t;
    b[2] = u;
}

void orc_free(orc_tables* t)
{
    if (!t) return;
    free(t->C); free(t->v); free(t->tau); free(t->tau2); free(t->omega);
    free(t->thr_ic); free(t->thr_wall); free(t->thr_rel);
    free(t->src_kind); free(t->src_ref); free(t->src_sign); free(t->src_E); free(t->thr_src);
    free(t->t_meas); free(t->ic_edges); free(t->ic_dT);
    free(t->bin); free(t->P_bin); free(t->spec_tab); free(t->heat_t); free(t->heat_P);
    free(t->heat_tet); free(t->thr_tet);
    free(t);
}

int orc_build(const orc_mode* modes, int32_t M, const orc_geom* g, const orc_det* det,
              const orc_problem* pr, orc_tables** out)
{
    *out = NULL;
    if (M < 1 || pr->N < 1 || pr->T_lin <= 0.0 || (pr->format != 1 && pr->format != 2)) return E_INVAL;
    const int32_t NT = pr->n_spec_tables;
    if (NT < 0 || (NT > 0 && !pr->spec_table)) return E_INVAL;
    for (int64_t i = 0; i < (int64_t)NT * M; ++i)
        if (!(pr->spec_table[i] >= 0.0 && pr->spec_table[i] <= 1.0)) return E_INVAL;
    for (int a = 0; a < 3; ++a)
        if (!g->unbounded[a] && !(g->L[a] > 0.0)) return E_GEOM;
    for (int id = 1; id <= 6; ++id) {
        int a = FACE_AXIS[id - 1];
        if (g->unbounded[a]) continue;
        int ty = g->face[id - 1].type;
        if (ty < B_ISO || ty > B_PERI) return E_GEOM;
        if (ty == B_ADIA && (!(g->face[id - 1].data[1] >= 0.0) || !isfinite(g->face[id - 1].data[1])))
            return E_GEOM;   /* the specular cutoff frequency */
        const int32_t k = g->face[id - 1].spec_table;
        if (k < 0 || k > NT || (k > 0 && (ty != B_ADIA || g->face[id - 1].data[0] != 0.0 || g->face[id - 1].data[1] != 0.0)))
            return E_GEOM;   /* a per-row table replaces the face's own specularity */
    }
    for (int a = 0; a < 3; ++a) {          /* periodic faces come in pairs on one axis */
        if (g->unbounded[a]) continue;
        int lo_id = 0, hi_id = 0;
        for (int id = 1; id <= 6; ++id)
            if (FACE_AXIS[id - 1] == a) { if (FACE_SIDE[id - 1]) hi_id = id; else lo_id = id; }
        if ((g->face[lo_id - 1].type == B_PERI) != (g->face[hi_id - 1].type == B_PERI)) return E_GEOM;
    }
    if (g->n_cyl < 0 || g->n_cyl > ORC_MAX_CYL) return E_GEOM;
    for (int c = 0; c < g->n_cyl; ++c) {
        const orc_cyl* y = &g->cyl[c];
        if (g->unbounded[0] || g->unbounded[1] || !(y->r > 0.0)) return E_GEOM;
        if (y->type != B_ADIA) return E_GEOM;
        if (!(y->spec_wc >= 0.0) || !isfinite(y->spec_wc)) return E_GEOM;
        if (y->spec_table < 0 || y->spec_table > NT || (y->spec_table > 0 && (y->spec != 0.0 || y->spec_wc != 0.0)))
            return E_GEOM;
        if (y->cx - y->r < 0.0 || y->cx + y->r > g->L[0] || y->cy - y->r < 0.0 || y->cy + y->r > g->L[1])
            return E_GEOM;
        if (y->id < 7 || (c > 0 && y->id <= g->cyl[c - 1].id)) return E_GEOM;
    }
    if (g->n_wall < 0 || g->n_wall > ORC_MAX_WALL) return E_GEOM;
    for (int k = 0; k < g->n_wall; ++k) {
        const orc_wall* wl = &g->wall[k];
        const int prev = k > 0 ? g->wall[k - 1].id : (g->n_cyl > 0 ? g->cyl[g->n_cyl - 1].id : 6);
        if (g->unbounded[0] || g->unbounded[1] || (wl->type != B_ADIA && wl->type != B_ISO) || wl->id <= prev)
            return E_GEOM;
        if (!(wl->spec_wc >= 0.0) || !isfinite(wl->spec_wc)) return E_GEOM;
        if (wl->spec_table < 0 || wl->spec_table > NT ||
            (wl->spec_table > 0 && (wl->type != B_ADIA || wl->spec != 0.0 || wl->spec_wc != 0.0)))
            return E_GEOM;
        if (wl->type == B_ADIA && !(wl->spec >= 0.0 && wl->spec <= 1.0)) return E_GEOM;
        if (wl->type == B_ISO && !(wl->spec > 0.0 && isfinite(wl->spec))) return E_GEOM;   /* T_b */
        const double pts[4] = {wl->x1, wl->y1, wl->x2, wl->y2};
        for (int q = 0; q < 4; ++q)
            if (!(pts[q] >= 0.0 && pts[q] <= g->L[q & 1])) return E_GEOM;
        if (wl->x1 == wl->x2 && wl->y1 == wl->y2) return E_GEOM;
        const double nn = sqrt(wl->nx * wl->nx + wl->ny * wl->ny);
        if (!(fabs(nn - 1.0) <= 1e-9)) return E_GEOM;
    }
    if (g->n_wall > 0 && !(g->volume > 0.0)) return E_INVAL;   /* the solid volume must be given */
    for (int a = 0; a < 3; ++a)
        if (det->n[a] < 0 || (det->n[a] > 0 && !(det->hi[a] > det->lo[a]))) return E_INVAL;
    if (pr->transient) {
        if (!(pr->t_max > 0.0) || pr->n_times < 1) return E_INVAL;
        for (int k = 1; k < pr->n_times; ++k)
            if (!(pr->t_meas[k] >= pr->t_meas[k - 1])) return E_INVAL;
    } else if (pr->n_ic > 0) {
        return E_INVAL;
    }
    if (pr->n_ic > 0 && (pr->ic_axis < 0 || pr->ic_axis > 2 || g->n_cyl > 0 || g->n_wall > 0)) return E_INVAL;
    if (pr->score_axis < 0 || pr->score_axis > 2 || pr->max_events < 1 || pr->max_events > 0x3FFFFFF0LL)
        return E_INVAL;
    /* the external heat source: transient, intervals ascending in [0, t_max], a cuboid inside the
       box that no pore or line wall reaches into */
    if (pr->n_heat < 0) return E_INVAL;
    if (pr->n_heat > 0) {
        if (!pr->transient || g->n_wall > 0 || !pr->heat_t || !pr->heat_P) return E_INVAL;
        if (!(pr->heat_t[0] >= 0.0) || !(pr->heat_t[pr->n_heat] <= pr->t_max)) return E_INVAL;
        for (int k = 0; k < pr->n_heat; ++k)
            if (!(pr->heat_t[k + 1] > pr->heat_t[k]) || !isfinite(pr->heat_P[k])) return E_INVAL;
        for (int a = 0; a < 3; ++a)
            if (!g->unbounded[a] && !(pr->heat_lo[a] >= 0.0 && pr->heat_hi[a] > pr->heat_lo[a] &&
                                      pr->heat_hi[a] <= g->L[a]))
                return E_INVAL;
        for (int c = 0; c < g->n_cyl; ++c) {     /* nearest point of the rectangle to the pore axis */
            double nx = fmin(fmax(g->cyl[c].cx, pr->heat_lo[0]), pr->heat_hi[0]);
            double ny = fmin(fmax(g->cyl[c].cy, pr->heat_lo[1]), pr->heat_hi[1]);
            double dx = nx - g->cyl[c].cx, dy = ny - g->cyl[c].cy;
            if (dx * dx + dy * dy < g->cyl[c].r * g->cyl[c].r) return E_INVAL;
        }
        /* tetrahedra: vertices inside the box (bounded axes), positive volume, the x-y bounding
           rectangle of each clear of every pore */
        if (pr->n_heat_tet < 0 || (pr->n_heat_tet > 0 && !pr->heat_tet)) return E_INVAL;
        for (int k = 0; k < pr->n_heat_tet; ++k) {
            const double* v = pr->heat_tet + 12 * k;
            double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int q = 0; q < 4; ++q)
                for (int a = 0; a < 3; ++a) {
                    const double x = v[3 * q + a];
                    if (!isfinite(x) || (!g->unbounded[a] && !(x >= 0.0 && x <= g->L[a]))) return E_INVAL;
                    lo[a] = fmin(lo[a], x);
                    hi[a] = fmax(hi[a], x);
                }
            if (!(tet_volume(v) > 0.0)) return E_INVAL;
            for (int c = 0; c < g->n_cyl; ++c) {
                double nx = fmin(fmax(g->cyl[c].cx, lo[0]), hi[0]);
                double ny = fmin(fmax(g->cyl[c].cy, lo[1]), hi[1]);
                double dx = nx - g->cyl[c].cx, dy = ny - g->cyl[c].cy;
                if (dx * dx + dy * dy < g->cyl[c].r * g->cyl[c].r) return E_INVAL;
            }
        }
    } else if (pr->n_heat_tet != 0) {
        return E_INVAL;
    }

    orc_tables* t = (orc_tables*)calloc(1, sizeof(orc_tables));
    if (!t) return E_NOMEM;
    t->M = M;
    t->g = *g;
    for (int k = 0; k < t->g.n_wall; ++k) {         /* unit normals */
        orc_wall* wl = &t->g.wall[k];
        const double nn = sqrt(wl->nx * wl->nx + wl->ny * wl->ny);
        wl->nx = wl->nx / nn;
        wl->ny = wl->ny / nn;
    }
    t->det = *det;
    t->pr = *pr;
    t->C = (double*)malloc(sizeof(double) * M);
    t->v = (double*)malloc(sizeof(double) * M);
    t->tau = (double*)malloc(sizeof(double) * M);
    t->tau2 = (double*)malloc(sizeof(double) * M);
    t->omega = (double*)malloc(sizeof(double) * M);
    t->thr_ic = (uint64_t*)malloc(sizeof(uint64_t) * M);
    t->thr_wall = (uint64_t*)malloc(sizeof(uint64_t) * M);
    t->thr_rel = (uint64_t*)malloc(sizeof(uint64_t) * M);
    double* w = (double*)malloc(sizeof(double) * M);
    if (!t->C || !t->v || !t->tau || !t->tau2 || !t->omega || !t->thr_ic || !t->thr_wall || !t->thr_rel || !w) {
        free(w); orc_free(t); return E_NOMEM;
    }
    /* per-mode heat capacity: given (second format) or DOS * delta-omega * de/dT (first format) */
    for (int m = 0; m < M; ++m) {
        const orc_mode* r = &modes[m];
        if (!(r->v > 0.0) || !(r->tau > 0.0)) { free(w); orc_free(t); return E_INVAL; }
        if (!(r->tau_imp >= 0.0) || !isfinite(r->tau_imp)) { free(w); orc_free(t); return E_INVAL; }
        t->v[m] = r->v;
        t->tau[m] = r->tau;
        t->tau2[m] = r->tau_imp;
        t->omega[m] = r->omega;
        if (r->tau_imp > 0.0) t->two = 1;
        if (pr->format == 1) {
            if (r->dos < 0.0 || r->domega < 0.0 || !(r->omega > 0.0)) { free(w); orc_free(t); return E_INVAL; }
            t->C[m] = (r->dos * r->domega) * orc_dedT(r->omega, pr->T_lin);
        } else {
            if (r->C < 0.0) { free(w); orc_free(t); return E_INVAL; }
            t->C[m] = r->C;
        }
    }
    t->C_tot = 0.0; t->Wv = 0.0; t->kappa_bulk = 0.0;
    for (int m = 0; m < M; ++m) {
        t->C_tot += t->C[m];
        t->Wv += t->C[m] * t->v[m];
        /* both processes relax the odd part of the deviation: their rates add */
        const double tau_eff = t->tau2[m] > 0.0 ? 1.0 / (1.0 / t->tau[m] + 1.0 / t->tau2[m]) : t->tau[m];
        t->kappa_bulk += ((t->C[m] * t->v[m]) * t->v[m]) * tau_eff;
    }
    t->kappa_bulk = t->kappa_bulk / 3.0;
    if (!(t->C_tot > 0.0)) { free(w); orc_free(t); return E_TABLE; }
    /* initial condition: proportional to C (Eq. Nbin); walls and gradient: C v (Eqs. iso_flux,
       grad_flux_sim); relaxation: C / tau (Eqs. norm_post_coll, n_scatt) */
    for (int m = 0; m < M; ++m) w[m] = t->C[m];
    orc_cdf_build(w, M, t->thr_ic, &t->last_ic);
    for (int m = 0; m < M; ++m) w[m] = t->C[m] * t->v[m];
    orc_cdf_build(w, M, t->thr_wall, &t->last_wall);
    for (int m = 0; m < M; ++m) w[m] = t->C[m] / t->tau[m];
    orc_cdf_build(w, M, t->thr_rel, &t->last_rel);
    free(w);
    if (t->last_ic < 0 || t->last_wall < 0 || t->last_rel < 0) { orc_free(t); return E_TABLE; }

    /* solid volume */
    if (g->volume > 0.0) {
        t->V_solid = g->volume;
    } else {
        double V = (extent(g, 0) * extent(g, 1)) * extent(g, 2);
        for (int c = 0; c < g->n_cyl; ++c) V = V - (PI * (g->cyl[c].r * g->cyl[c].r)) * extent(g, 2);
        t->V_solid = V;
    }
    t->gnorm = sqrt((g->gradT[0] * g->gradT[0] + g->gradT[1] * g->gradT[1]) + g->gradT[2] * g->gradT[2]);
    for (int a = 0; a < 3; ++a) t->ngrad[a] = t->gnorm > 0.0 ? -g->gradT[a] / t->gnorm : 0.0;

    /* per-row specularity tables */
    t->pr.spec_table = NULL;
    if (NT > 0) {
        t->spec_tab = (double*)malloc(sizeof(double) * (size_t)NT * (size_t)M);
        if (!t->spec_tab) { orc_free(t); return E_NOMEM; }
        memcpy(t->spec_tab, pr->spec_table, sizeof(double) * (size_t)NT * (size_t)M);
    }
    /* transient arrays */
    if (pr->transient) {
        t->t_meas = (double*)malloc(sizeof(double) * pr->n_times);
        if (!t->t_meas) { orc_free(t); return E_NOMEM; }
        memcpy(t->t_meas, pr->t_meas, sizeof(double) * pr->n_times);
        t->pr.t_meas = t->t_meas;
    } else {
        t->pr.n_times = 0;
        t->pr.t_meas = NULL;
    }
    if (pr->n_ic > 0) {
        t->ic_edges = (double*)malloc(sizeof(double) * (pr->n_ic + 1));
        t->ic_dT = (double*)malloc(sizeof(double) * pr->n_ic);
        if (!t->ic_edges || !t->ic_dT) { orc_free(t); return E_NOMEM; }
        memcpy(t->ic_edges, pr->ic_edges, sizeof(double) * (pr->n_ic + 1));
        memcpy(t->ic_dT, pr->ic_dT, sizeof(double) * pr->n_ic);
        for (int c = 0; c < pr->n_ic; ++c)
            if (!(t->ic_edges[c + 1] > t->ic_edges[c])) { orc_free(t); return E_INVAL; }
        t->pr.ic_edges = t->ic_edges;
        t->pr.ic_dT = t->ic_dT;
    }

    /* sources (section 3.1, Eqs. dev_tot and source_energy), in the order: isothermal faces by
       id, gradient source, initial-condition cells */
    int Smax = 6 + g->n_wall + 1 + (pr->n_ic > 0 ? pr->n_ic : 0) + (pr->n_heat > 0 ? pr->n_heat : 0);
    t->src_kind = (int32_t*)malloc(sizeof(int32_t) * Smax);
    t->src_ref = (int32_t*)malloc(sizeof(int32_t) * Smax);
    t->src_sign = (int32_t*)malloc(sizeof(int32_t) * Smax);
    t->src_E = (double*)malloc(sizeof(double) * Smax);
    t->thr_src = (uint64_t*)malloc(sizeof(uint64_t) * Smax);
    if (!t->src_kind || !t->src_ref || !t->src_sign || !t->src_E || !t->thr_src) { orc_free(t); return E_NOMEM; }
    int S = 0;
    for (int id = 1; id <= 6; ++id) {
        int a = FACE_AXIS[id - 1];
        if (g->unbounded[a] || g->face[id - 1].type != B_ISO) continue;
        double dT = g->face[id - 1].data[0] - pr->T_lin;
        if (dT == 0.0) continue;
        int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
        double area = extent(g, b) * extent(g, c);
        /* Eq. iso_flux: A / 4 sum_p V_g |e_b| D delta-omega = A |T_b - T_lin| sum_m C_m v_m / 4 */
        double E = ((area * fabs(dT)) * t->Wv) / 4.0;
        if (pr->transient) E = E * pr->t_max;
        t->src_kind[S] = S_WALL; t->src_ref[S] = id; t->src_sign[S] = dT > 0.0 ? 1 : -1; t->src_E[S] = E;
        ++S;
    }
    for (int k = 0; k < g->n_wall; ++k) {        /* isothermal line walls, by id */
        const orc_wall* wl = &g->wall[k];
        if (wl->type != B_ISO) continue;
        double dT = wl->spec - pr->T_lin;
        if (dT == 0.0) continue;
        const double ex = wl->x2 - wl->x1, ey = wl->y2 - wl->y1;
        double area = sqrt(ex * ex + ey * ey) * extent(g, 2);
        double E = ((area * fabs(dT)) * t->Wv) / 4.0;
        if (pr->transient) E = E * pr->t_max;
        t->src_kind[S] = S_IWALL; t->src_ref[S] = k; t->src_sign[S] = dT > 0.0 ? 1 : -1; t->src_E[S] = E;
        ++S;
    }
    if (t->gnorm > 0.0) {
        /* Eq. grad_flux integrated over all directions: V |grad T| sum_m C_m v_m / 2 */
        double E = ((t->V_solid * t->gnorm) * t->Wv) / 2.0;
        if (pr->transient) E = E * pr->t_max;
        t->src_kind[S] = S_GRAD; t->src_ref[S] = 0; t->src_sign[S] = 0; t->src_E[S] = E;
        ++S;
    }
    for (int c = 0; c < pr->n_ic; ++c) {
        int a = pr->ic_axis;
        int b = (a == 0) ? 1 : 0, cc = (a == 2) ? 1 : 2;
        double Vc = ((t->ic_edges[c + 1] - t->ic_edges[c]) * extent(g, b)) * extent(g, cc);
        /* Eq. Nbin summed over modes: |T_init - T_eq| sum_m C_m per unit volume */
        double E = (t->C_tot * fabs(t->ic_dT[c])) * Vc;
        t->src_kind[S] = S_IC; t->src_ref[S] = c; t->src_sign[S] = t->ic_dT[c] > 0.0 ? 1 : -1; t->src_E[S] = E;
        ++S;
    }
    /* the external heat source: the energy of interval k is |P_k| times the cuboid's volume times
       the interval's length */
    t->pr.heat_t = NULL;
    t->pr.heat_P = NULL;
    t->pr.heat_tet = NULL;
    if (pr->n_heat > 0) {
        t->heat_t = (double*)malloc(sizeof(double) * (pr->n_heat + 1));
        t->heat_P = (double*)malloc(sizeof(double) * pr->n_heat);
        if (!t->heat_t || !t->heat_P) { orc_free(t); return E_NOMEM; }
        memcpy(t->heat_t, pr->heat_t, sizeof(double) * (pr->n_heat + 1));
        memcpy(t->heat_P, pr->heat_P, sizeof(double) * pr->n_heat);
        double Vh = 1.0;
        for (int a = 0; a < 3; ++a) Vh *= g->unbounded[a] ? 1.0 : pr->heat_hi[a] - pr->heat_lo[a];
        if (pr->n_heat_tet > 0) {        /* the union of the tetrahedra: a tetrahedron by volume */
            const int nt = pr->n_heat_tet;
            t->heat_tet = (double*)malloc(sizeof(double) * 12 * nt);
            t->thr_tet = (uint64_t*)malloc(sizeof(uint64_t) * nt);
            double* vol = (double*)malloc(sizeof(double) * nt);
            if (!t->heat_tet || !t->thr_tet || !vol) { free(vol); orc_free(t); return E_NOMEM; }
            Vh = 0.0;
            for (int k = 0; k < nt; ++k) {
                const double* v = pr->heat_tet + 12 * k;
                for (int a = 0; a < 3; ++a) {
                    t->heat_tet[12 * k + a] = v[a];
                    for (int q = 1; q < 4; ++q) t->heat_tet[12 * k + 3 * q + a] = v[3 * q + a] - v[a];
                }
                vol[k] = tet_volume(v);
                Vh += vol[k];
            }
            orc_cdf_build(vol, nt, t->thr_tet, &t->last_tet);
            free(vol);
        }
        for (int k = 0; k < pr->n_heat; ++k) {
            if (t->heat_P[k] == 0.0) continue;
            double E = (fabs(t->heat_P[k]) * Vh) * (t->heat_t[k + 1] - t->heat_t[k]);
            t->src_kind[S] = S_HEAT; t->src_ref[S] = k; t->src_sign[S] = t->heat_P[k] > 0.0 ? 1 : -1;
            t->src_E[S] = E;
            ++S;
        }
    }
    t->S = S;
    if (S == 0) { orc_free(t); return E_TABLE; }
    t->E_tot = 0.0;
    for (int s = 0; s < S; ++s) t->E_tot += t->src_E[s];
    orc_cdf_build(t->src_E, S, t->thr_src, &t->last_src);
    if (t->last_src < 0) { orc_free(t); return E_TABLE; }
    t->e_eff = t->E_tot / (double)pr->N;

    t->n_cells = 1;
    for (int a = 0; a < 3; ++a) t->n_cells *= det->n[a] > 0 ? det->n[a] : 1;
    t->n_cols = pr->transient ? pr->n_times : M;

    /* frequency bins (the parameters of the sensitivity dkappa / dln tau_i) and the share of the
       relaxation distribution in each bin */
    t->bin = (int32_t*)malloc(sizeof(int32_t) * M);
    if (!t->bin) { orc_free(t); return E_NOMEM; }
    t->n_bins = 0;
    for (int m = 0; m < M; ++m) {
        if (modes[m].bin < 0) { orc_free(t); return E_INVAL; }
        t->bin[m] = modes[m].bin;
        if (modes[m].bin + 1 > t->n_bins) t->n_bins = modes[m].bin + 1;
    }
    t->P_bin = (double*)calloc(t->n_bins, sizeof(double));
    if (!t->P_bin) { orc_free(t); return E_NOMEM; }
    {
        double W = 0.0;
        for (int m = 0; m < M; ++m) W += t->C[m] / t->tau[m];
        for (int m = 0; m < M; ++m) t->P_bin[t->bin[m]] += (t->C[m] / t->tau[m]) / W;
    }
    *out = t;
    return E_OK;
}

void orc_info(const orc_tables* t, double* d6, int64_t* i4)
{
    d6[0] = t->C_tot; d6[1] = t->Wv; d6[2] = t->e_eff; d6[3] = t->V_solid; d6[4] = t->E_tot;
    d6[5] = t->kappa_bulk;
    i4[0] = t->M; i4[1] = t->S; i4[2] = t->n_cells; i4[3] = t->n_cols; i4[4] = t->n_bins;
}

int orc_get(const orc_tables* t, int32_t which, void* out, int64_t n)
{
    switch (which) {
    case 0: if (n < t->M) return E_INVAL; memcpy(out, t->C, sizeof(double) * t->M); return 0;
    case 1: if (n < t->M) return E_INVAL; memcpy(out, t->thr_ic, 8 * t->M); return 0;
    case 2: if (n < t->M) return E_INVAL; memcpy(out, t->thr_wall, 8 * t->M); return 0;
    case 3: if (n < t->M) return E_INVAL; memcpy(out, t->thr_rel, 8 * t->M); return 0;
    case 4: if (n < t->S) return E_INVAL; memcpy(out, t->src_E, sizeof(double) * t->S); return 0;
    case 5: if (n < t->S) return E_INVAL; memcpy(out, t->thr_src, 8 * t->S); return 0;
    case 6: if (n < t->S) return E_INVAL; memcpy(out, t->src_sign, 4 * t->S); return 0;
    case 8: if (n < t->n_bins) return E_INVAL; memcpy(out, t->P_bin, sizeof(double) * t->n_bins); return 0;
    case 9: if (n < t->M) return E_INVAL; memcpy(out, t->bin, 4 * t->M); return 0;
    case 7: {
        if (n < 4) return E_INVAL;
        int64_t* o = (int64_t*)out;
        o[0] = t->last_ic; o[1] = t->last_wall; o[2] = t->last_rel; o[3] = t->last_src;
        return 0;
    }
    default: return E_INVAL;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Detectors (section 3.4 and the output request of section 4).                               */
/* ------------------------------------------------------------------------------------------ */

static double cell_width(const orc_det* d, int a) { return (d->hi[a] - d->lo[a]) / (double)d->n[a]; }

/* flat cell index of a point, or -1 outside the detector region (binned axes only) */
static int64_t cell_of(const orc_det* d, const double x[3])
{
    int64_t idx = 0;
    for (int a = 0; a < 3; ++a) {
        int n = d->n[a] > 0 ? d->n[a] : 1;
        int64_t i = 0;
        if (d->n[a] > 0) {
            if (x[a] < d->lo[a] || x[a] > d->hi[a]) return -1;
            double f = floor((x[a] - d->lo[a]) / cell_width(d, a));
            i = (int64_t)f;
            if (i < 0) i = 0;
            if (i > n - 1) i = n - 1;
        }
        idx = idx * n + i;
    }
    return idx;
}

static int cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* steady track-length estimator (Eqs. temp_steady and flux_x_steady): for every detector cell
   the segment crosses, T += s l / V_g and q_a += s l Omega_a with l the length inside the cell */
static void tally_steady(const orc_tables* t, const double x0[3], const double o[3], double d, int32_t m,
                         double s, double* raw, double* pts)
{
    const orc_det* det = &t->det;
    if (!(d > 0.0)) return;
    double s_lo = 0.0, s_hi = d;
    for (int a = 0; a < 3; ++a) {
        if (det->n[a] <= 0) continue;
        if (o[a] == 0.0) {
            if (x0[a] < det->lo[a] || x0[a] > det->hi[a]) return;
        } else {
            double s1 = (det->lo[a] - x0[a]) / o[a];
            double s2 = (det->hi[a] - x0[a]) / o[a];
            if (s1 > s2) { double tmp = s1; s1 = s2; s2 = tmp; }
            if (s1 > s_lo) s_lo = s1;
            if (s2 < s_hi) s_hi = s2;
        }
    }
    if (!(s_hi > s_lo)) return;
    int np = 0;
    pts[np++] = s_lo;
    pts[np++] = s_hi;
    for (int a = 0; a < 3; ++a) {
        if (det->n[a] <= 1 || o[a] == 0.0) continue;
        double w = cell_width(det, a);
        for (int j = 1; j < det->n[a]; ++j) {
            double plane = det->lo[a] + (double)j * w;
            double sc = (plane - x0[a]) / o[a];
            if (sc > s_lo && sc < s_hi) pts[np++] = sc;
        }
    }
    qsort(pts, np, sizeof(double), cmp_double);
    double v = t->v[m];
    int mask = det->mask;
    for (int i = 0; i + 1 < np; ++i) {
        double l = pts[i + 1] - pts[i];
        if (!(l > 0.0)) continue;
        double mid = 0.5 * (pts[i] + pts[i + 1]);
        double x[3];
        for (int a = 0; a < 3; ++a) x[a] = x0[a] + o[a] * mid;
        int64_t cell = 0;
        {   /* clamp the midpoint's cell on binned axes */
            int64_t idx = 0;
            for (int a = 0; a < 3; ++a) {
                int n = det->n[a] > 0 ? det->n[a] : 1;
                int64_t ci = 0;
                if (det->n[a] > 0) {
                    ci = (int64_t)floor((x[a] - det->lo[a]) / cell_width(det, a));
                    if (ci < 0) ci = 0;
                    if (ci > n - 1) ci = n - 1;
                }
                idx = idx * n + ci;
            }
            cell = idx;
        }
        double* r = raw + (cell * t->n_cols + m) * 4;
        if (mask & 1) r[0] += s * (l / v);
        if (mask & 2) r[1] += s * (l * o[0]);
        if (mask & 4) r[2] += s * (l * o[1]);
        if (mask & 8) r[3] += s * (l * o[2]);
    }
}

void orc_tally_segment(const orc_tables* t, const double x0[3], const double o[3], double d, int32_t m,
                       double s, double* raw)
{
    int cap = 2;
    for (int a = 0; a < 3; ++a) cap += t->det.n[a];
    double* pts = (double*)malloc(sizeof(double) * cap);
    if (!pts) return;
    tally_steady(t, x0, o, d, m, s, raw, pts);
    free(pts);
}

/* transient snapshot estimator (Eq. sampling): at every measurement time t_k in [t0, t1) the
   particle sits at x0 + Omega V_g (t_k - t0) and adds s to T and s V_g Omega_a to q_a */
static void tally_transient(const orc_tables* t, const double x0[3], const double o[3], double t0, double t1,
                            int32_t m, double s, double* raw)
{
    double v = t->v[m];
    int mask = t->det.mask;
    for (int k = 0; k < t->pr.n_times; ++k) {
        double tk = t->t_meas[k];
        if (tk < t0 || !(tk < t1)) continue;
        double dist = v * (tk - t0);
        double x[3];
        for (int a = 0; a < 3; ++a) x[a] = x0[a] + o[a] * dist;
        int64_t cell = cell_of(&t->det, x);
        if (cell < 0) continue;
        double* r = raw + (cell * t->n_cols + k) * 4;
        if (mask & 1) r[0] += s;
        if (mask & 2) r[1] += s * (v * o[0]);
        if (mask & 4) r[2] += s * (v * o[1]);
        if (mask & 8) r[3] += s * (v * o[2]);
    }
}

/* ------------------------------------------------------------------------------------------ */
/* One particle: emission (section 3.2) and the flight loop (sections 3.3, 3.5).               */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    double x[3], o[3];
    double t, dtr;       /* time, time left until the next scattering event */
    double lead;         /* two clocks: how much later the other clock fires (+inf: never) */
    int32_t nx2;         /* two clocks: the next scattering is the two-phonon one */
    double cT, cq;       /* per-particle contributions for the variance estimate */
    int32_t m, s, nrel;
    uint32_t k;          /* segments so far (bounded by max_events) */
    uint32_t j;          /* events so far that drew random numbers; the j-th one draws record 2 + j */
} prt;

/* Section 3.3 draws two times to scattering, one per process, from Eq. time_to_scat; both run
   down together with the particle's time, so what is kept is the earlier one (dtr) and the
   other's lead over it.  A tie goes to the three-phonon clock. */
static void set_clocks(prt* p, double t2, double t3)
{
    if (t2 < t3) {
        p->dtr = t2;
        p->lead = t3 - t2;
        p->nx2 = 1;
    } else {
        p->dtr = t3;
        p->lead = t2 - t3;
        p->nx2 = 0;
    }
}

/* the two-phonon clock of row m drawn at the j-th drawing event (j = 0: emission): words W0W1
   of record 0x60000000 + j; +inf for a row without the process */
static double draw_t2(const orc_tables* t, uint64_t seed, uint32_t inst, int64_t pid, uint32_t j, int32_t m)
{
    if (!(t->tau2[m] > 0.0)) return INFINITY;
    uint32_t Q[8];
    orc_record(seed, inst, pid, 0x60000000u + j, Q);
    return -t->tau2[m] * log(1.0 - unif(Q, 0));
}

static int outside_solid(const orc_geom* g, const double x[3]);

static int emit(const orc_tables* t, uint64_t seed, uint32_t inst, int64_t pid, prt* p, uint64_t* counts,
                int64_t* src_out)
{
    const orc_geom* g = &t->g;
    uint32_t R0[8], R1[8], R2[8];
    orc_record(seed, inst, pid, 0, R0);
    orc_record(seed, inst, pid, 1, R1);
    int64_t src = orc_cdf_pick(t->thr_src, t->S, t->last_src, key64(R0, 0));
    int kind = t->src_kind[src];
    double up[3] = {unif(R1, 2), unif(R1, 4), unif(R1, 6)};
    double ud1 = unif(R0, 4), ud2 = unif(R0, 6);
    if (kind == S_GRAD || (t->pr.transient && kind != S_IC)) orc_record(seed, inst, pid, 2, R2);
    memset(p, 0, sizeof(*p));
    if (kind == S_WALL) {
        int id = t->src_ref[src];
        int a = FACE_AXIS[id - 1], side = FACE_SIDE[id - 1];
        int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
        p->x[b] = g->unbounded[b] ? 0.0 : up[0] * g->L[b];
        p->x[c] = g->unbounded[c] ? 0.0 : up[1] * g->L[c];
        p->x[a] = side ? g->L[a] : 0.0;
        double n[3] = {0.0, 0.0, 0.0};
        n[a] = side ? -1.0 : 1.0;
        orc_dir_cos(ud1, ud2, n, p->o);
        p->s = t->src_sign[src];
        p->m = (int32_t)orc_cdf_pick(t->thr_wall, t->M, t->last_wall, key64(R1, 0));
    } else if (kind == S_IWALL) {
        /* a point of the wall (along the segment, then through the thickness), directions
           cosine-weighted about its normal (Eq. wall_dir) */
        const orc_wall* wl = &g->wall[t->src_ref[src]];
        p->x[0] = wl->x1 + up[0] * (wl->x2 - wl->x1);
        p->x[1] = wl->y1 + up[0] * (wl->y2 - wl->y1);
        p->x[2] = g->unbounded[2] ? 0.0 : up[1] * g->L[2];
        double n[3] = {wl->nx, wl->ny, 0.0};
        orc_dir_cos(ud1, ud2, n, p->o);
        p->s = t->src_sign[src];
        p->m = (int32_t)orc_cdf_pick(t->thr_wall, t->M, t->last_wall, key64(R1, 0));
    } else if (kind == S_GRAD) {
        for (int a = 0; a < 3; ++a) p->x[a] = g->unbounded[a] ? 0.0 : up[a] * g->L[a];
        for (uint32_t attempt = 1;; ++attempt) {      /* positions outside the solid are redrawn */
            if (!outside_solid(g, p->x)) break;
            if (attempt > 4096) return -1;
            counts[ORC_C_REJECT] += 1;
            uint32_t RA[8];
            orc_record(seed, inst, pid, 0x40000000u + attempt, RA);
            double ua[3] = {unif(RA, 2), unif(RA, 4), unif(RA, 6)};
            for (int a = 0; a < 3; ++a) p->x[a] = g->unbounded[a] ? 0.0 : ua[a] * g->L[a];
        }
        orc_dir_cos(ud1, ud2, t->ngrad, p->o);
        /* Eq. grad_flux: either sign equally likely; a negative particle travels reversed */
        p->s = (R2[0] >> 31) ? -1 : 1;
        if (p->s < 0) { p->o[0] = -p->o[0]; p->o[1] = -p->o[1]; p->o[2] = -p->o[2]; }
        p->m = (int32_t)orc_cdf_pick(t->thr_wall, t->M, t->last_wall, key64(R1, 0));
    } else if (kind == S_HEAT) {
        /* the external heat source: a point of its cuboid (or of one of its tetrahedra, chosen by
           volume with words W4W5 of record 2), an isotropic direction and the row of a local
           temperature rise (weights C, as for the initial condition) */
        if (t->pr.n_heat_tet > 0) {
            const int64_t k = orc_cdf_pick(t->thr_tet, t->pr.n_heat_tet, t->last_tet, key64(R2, 4));
            double b[3];
            tet_point(up[0], up[1], up[2], b);
            const double* v = t->heat_tet + 12 * k;
            for (int a = 0; a < 3; ++a) p->x[a] = ((v[a] + b[0] * v[3 + a]) + b[1] * v[6 + a]) + b[2] * v[9 + a];
        } else {
            for (int a = 0; a < 3; ++a)
                p->x[a] = g->unbounded[a] ? 0.0 : t->pr.heat_lo[a] + up[a] * (t->pr.heat_hi[a] - t->pr.heat_lo[a]);
        }
        orc_dir_iso(ud1, ud2, p->o);
        p->s = t->src_sign[src];
        p->m = (int32_t)orc_cdf_pick(t->thr_ic, t->M, t->last_ic, key64(R1, 0));
    } else {
        int c = t->src_ref[src];
        int ia = t->pr.ic_axis;
        for (int a = 0; a < 3; ++a) p->x[a] = g->unbounded[a] ? 0.0 : up[a] * g->L[a];
        double e0 = t->ic_edges[c], width = t->ic_edges[c + 1] - t->ic_edges[c];
        p->x[ia] = e0 + up[ia] * width;
        orc_dir_iso(ud1, ud2, p->o);
        p->s = t->src_sign[src];
        p->m = (int32_t)orc_cdf_pick(t->thr_ic, t->M, t->last_ic, key64(R1, 0));
    }
    if (kind == S_HEAT) {              /* a time uniform in the source's interval */
        const double t0 = t->heat_t[t->src_ref[src]], t1 = t->heat_t[t->src_ref[src] + 1];
        p->t = t0 + unif(R2, 2) * (t1 - t0);
    } else {
        p->t = (t->pr.transient && kind != S_IC) ? unif(R2, 2) * t->pr.t_max : 0.0;
    }
    p->dtr = -t->tau[p->m] * log(1.0 - unif(R0, 2));
    if (t->two) set_clocks(p, draw_t2(t, seed, inst, pid, 0u, p->m), p->dtr);
    *src_out = src;
    return 0;
}

/* distance along the ray x + d o to the nearest boundary (box faces in id order, then the
   cylinders); ties go to the lower id.  Returns +inf and hit = 0 when the ray meets nothing. */
static double next_boundary(const orc_geom* g, const double x[3], const double o[3], int* hit_out)
{
    double db = INFINITY;
    int hit = 0;
    for (int id = 1; id <= 6; ++id) {
        int a = FACE_AXIS[id - 1], side = FACE_SIDE[id - 1];
        if (g->unbounded[a]) continue;
        double d;
        if (side == 1 && o[a] > 0.0) d = (g->L[a] - x[a]) / o[a];
        else if (side == 0 && o[a] < 0.0) d = (0.0 - x[a]) / o[a];
        else continue;
        if (d < db) { db = d; hit = id; }
    }
    for (int c = 0; c < g->n_cyl; ++c) {
        const orc_cyl* y = &g->cyl[c];
        double dx = x[0] - y->cx, dy = x[1] - y->cy;
        double qa = o[0] * o[0] + o[1] * o[1];
        double qb = dx * o[0] + dy * o[1];
        double qc = dx * dx + dy * dy - y->r * y->r;
        if (!(qb < 0.0)) continue;                /* moving away from the axis: no hit */
        double disc = qb * qb - qa * qc;
        if (!(disc >= 0.0)) continue;
        double d = (qc < 0.0) ? 0.0 : qc / (-qb + sqrt(disc));
        if (d < db) { db = d; hit = y->id; }
    }
    /* internal line walls (ids after the pores'), met from the side their normal points to:
       x + d o = P1 + s (P2 - P1) in the x-y plane, d >= 0, 0 <= s <= 1 */
    for (int k = 0; k < g->n_wall; ++k) {
        const orc_wall* wl = &g->wall[k];
        if (!(o[0] * wl->nx + o[1] * wl->ny < 0.0)) continue;
        const double ex = wl->x2 - wl->x1, ey = wl->y2 - wl->y1;
        const double den = o[0] * ey - o[1] * ex;
        if (den == 0.0) continue;
        const double wx = wl->x1 - x[0], wy = wl->y1 - x[1];
        const double d = (wx * ey - wy * ex) / den;
        const double sp = (wx * o[1] - wy * o[0]) / den;
        if (d >= 0.0 && sp >= 0.0 && sp <= 1.0 && d < db) { db = d; hit = wl->id; }
    }
    *hit_out = hit;
    return db;
}

/* a point of the box outside the solid: inside a pore, or inside a closed loop of line walls
   (consecutive walls each starting where the previous one ends, the last ending where the first
   starts; crossing-number test with half-open edges).  Walls outside such loops exclude nothing. */
static int outside_solid(const orc_geom* g, const double x[3])
{
    for (int c = 0; c < g->n_cyl; ++c) {
        double dx = x[0] - g->cyl[c].cx, dy = x[1] - g->cyl[c].cy;
        if (dx * dx + dy * dy < g->cyl[c].r * g->cyl[c].r) return 1;
    }
    int k = 0;
    while (k < g->n_wall) {
        int j = k;
        while (j + 1 < g->n_wall && g->wall[j + 1].x1 == g->wall[j].x2 && g->wall[j + 1].y1 == g->wall[j].y2) ++j;
        if (g->wall[j].x2 == g->wall[k].x1 && g->wall[j].y2 == g->wall[k].y1) {
            int in = 0;
            for (int e = k; e <= j; ++e) {
                const orc_wall* wl = &g->wall[e];
                if ((wl->y1 > x[1]) != (wl->y2 > x[1]) &&
                    x[0] < wl->x1 + (x[1] - wl->y1) * (wl->x2 - wl->x1) / (wl->y2 - wl->y1))
                    in = !in;
            }
            if (in) return 1;
        }
        k = j + 1;
    }
    return 0;
}

double orc_next_boundary(const orc_tables* t, const double x[3], const double o[3], int32_t* hit)
{
    int h = 0;
    double d = next_boundary(&t->g, x, o, &h);
    *hit = h;
    return d;
}

int orc_emit_state(const orc_tables* t, uint64_t seed, uint32_t instance, int64_t pid, double* d8, int32_t* i4)
{
    prt p;
    int64_t src = 0;
    uint64_t counts[ORC_N_COUNTS] = {0};
    if (emit(t, seed, instance, pid, &p, counts, &src) != 0) return E_INVAL;
    d8[0] = p.x[0]; d8[1] = p.x[1]; d8[2] = p.x[2];
    d8[3] = p.o[0]; d8[4] = p.o[1]; d8[5] = p.o[2];
    d8[6] = p.t; d8[7] = p.dtr;
    i4[0] = p.m; i4[1] = p.s; i4[2] = (int32_t)src; i4[3] = (int32_t)counts[ORC_C_REJECT];
    return E_OK;
}

int orc_emit_clocks(const orc_tables* t, uint64_t seed, uint32_t instance, int64_t pid, double* lead, int32_t* nx2)
{
    prt p;
    int64_t src = 0;
    uint64_t counts[ORC_N_COUNTS] = {0};
    if (emit(t, seed, instance, pid, &p, counts, &src) != 0) return E_INVAL;
    *lead = p.lead;
    *nx2 = p.nx2;
    return E_OK;
}

/* Score-function (likelihood-ratio) terms of one particle, for the sensitivity of kappa to a
   relative change of the relaxation times of one frequency bin, dkappa / dln tau_i.  Each
   random quantity whose law depends on tau contributes its score times the part of the
   particle's flux contribution F that comes after it (earlier parts cannot depend on it):
     - a free flight of mode m (Eq. time_to_scat, time T ~ Exp(tau_m)) that ends in a relaxation:
       d ln[(1/tau) e^{-T/tau}] / d ln tau = T/tau - 1, for bin(m), with F after the flight's start;
       one cut short (absorbed, time horizon, segment cap) survives: d ln e^{-T/tau} / d ln tau = T/tau;
     - a relaxation draw of row j from p_j = (C_j/tau_j) / sum_r (C_r/tau_r) (Eq. norm_post_coll):
       d ln p_j / d ln tau_i = -[bin(j) = i] + P_i, with F after the draw; the P_i part is the same
       for every draw and is summed into one number B per run. */
typedef struct { int32_t bin, dense; double g, F_before, c0; } adj_ev;   /* adds c0 + g (F - F_before) */

/* Pathwise (reparametrisation) form: a free flight of mode m covers the distance
   L = v_m tau_m E with E = -ln(1 - u) fixed by its random numbers, so dL / dln tau_m = L.  With
   the sequence of events held fixed, the first-order change of the trajectory caused by that
   stretch is a tangent (dx, dO, b): the shift of the current position and direction, and b, the
   change of the distance left in the current flight.  It is born at the start of its flight with
   b = L, carried through every later segment end (a boundary hit moves along the surface, a
   reflection turns dO, a relaxation spends b and forgets dO because the new direction is drawn
   independently of the position), and at the particle's end it changes F = s (x_end - x_start)_a
   (the flux score is the net unwrapped displacement along the scored axis) by s dx_a.  The
   relaxation draws still enter through their scores (-[bin(j) = i] + P_i) times the F that
   follows them. */
typedef struct { int32_t bin; double dx[3], dO[3], b; } tangent;

typedef struct {
    adj_ev* ev; int64_t n, cap; int failed;
    int pathwise;               /* 1: tangents for the flights, scores only for the draws */
    tangent* tg; int64_t nt, tcap;
    int32_t sign;               /* the particle's sign s */
    double dline;               /* straight distance since the last tangent update (periodic
                                   transfers do not interrupt the line) */
    int local;                  /* 1: local pathwise form for modes with v tau <= lambda_split */
    double lambda_split;
} adj_list;

static void adj_push(adj_list* al, int32_t bin, double g, double F_before, int dense)
{
    if (!al) return;
    if (al->pathwise && !dense) return;       /* flight scores: replaced by the tangents */
    if (al->n == al->cap) {
        int64_t cap = al->cap ? 2 * al->cap : 64;
        adj_ev* e = (adj_ev*)realloc(al->ev, sizeof(adj_ev) * cap);
        if (!e) { al->failed = 1; return; }
        al->ev = e;
        al->cap = cap;
    }
    adj_ev* e = &al->ev[al->n++];
    e->bin = bin;
    e->g = g;
    e->F_before = F_before;
    e->dense = dense;
    e->c0 = 0.0;
}

/* Local pathwise form, for a mode whose mean free path v tau is at most lambda_split: a flight's
   own flux A(T) = s (x_end - x_start)_a is continuous in its time T and depends on tau only through
   T = tau E, so its part is the pathwise s L Omega_a (L = v T, Omega the direction of its last
   segment; zero for a flight cut short, whose end does not move); what follows the flight, B(T),
   keeps the likelihood ratio (T/tau - 1) (F - F at the flight's end) of an uncensored flight (zero
   after a cut-short one, which ends the particle).  A per-mode choice of the form keeps the sum
   unbiased: each flight time is differentiated one way. */
static int adj_local(const adj_list* al, const orc_tables* t, int32_t m)
{
    return al && al->local && t->v[m] * t->tau[m] <= al->lambda_split;
}

static void adj_push_local(adj_list* al, int32_t bin, double c0, double g, double F_before)
{
    adj_push(al, bin, g, F_before, 0);
    if (al && !al->failed) al->ev[al->n - 1].c0 = c0;
}

/* a new flight of mode row m, distance L: its tangent; every earlier one has spent its b and
   forgotten its direction shift at the relaxation that started this flight */
static void tan_birth(adj_list* al, int32_t bin, double L)
{
    if (!al || !al->pathwise) return;
    if (al->nt == al->tcap) {
        int64_t cap = al->tcap ? 2 * al->tcap : 16;
        tangent* e = (tangent*)realloc(al->tg, sizeof(tangent) * cap);
        if (!e) { al->failed = 1; return; }
        al->tg = e;
        al->tcap = cap;
    }
    tangent* q = &al->tg[al->nt++];
    memset(q, 0, sizeof(*q));
    q->bin = bin;
    q->b = L;
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* the segment x -> x + d o ended on a surface with unit normal n at the hit point: the hit point
   stays on the surface, n . (dx + dd o + d dO) = 0, and the flight has dd less distance left */
static void tan_hit(adj_list* al, const double o[3], double d, const double n[3])
{
    if (!al || !al->pathwise) return;
    const double on = dot3(o, n);
    for (int64_t i = 0; i < al->nt; ++i) {
        tangent* q = &al->tg[i];
        const double dd = -(dot3(n, q->dx) + d * dot3(n, q->dO)) / on;
        for (int a = 0; a < 3; ++a) q->dx[a] = q->dx[a] + dd * o[a] + d * q->dO[a];
        q->b = q->b - dd;
    }
}

/* the segment x -> x + d o ended in a relaxation: the end point moves with the distance left and
   with the direction; the next direction is drawn afresh */
static void tan_relax(adj_list* al, const double o[3], double d)
{
    if (!al || !al->pathwise) return;
    for (int64_t i = 0; i < al->nt; ++i) {
        tangent* q = &al->tg[i];
        for (int a = 0; a < 3; ++a) q->dx[a] = q->dx[a] + q->b * o[a] + d * q->dO[a];
        q->b = 0.0;
        q->dO[0] = q->dO[1] = q->dO[2] = 0.0;
    }
}

/* reflection off a plane with normal along axis fa: specular negates that direction component,
   diffuse draws a direction that does not depend on the hit point */
static void tan_plane(adj_list* al, int fa, int specular)
{
    if (!al || !al->pathwise) return;
    for (int64_t i = 0; i < al->nt; ++i) {
        tangent* q = &al->tg[i];
        if (specular) q->dO[fa] = -q->dO[fa];
        else q->dO[0] = q->dO[1] = q->dO[2] = 0.0;
    }
}

/* reflection off the cylinder of radius r: the normal n = (x_h - c)_xy / r turns with the hit
   point, dn = (dx_h)_xy / r.  Specular: o' = o - 2 (o.n) n (o before the reflection).  Diffuse:
   o' = mu n + a t1 + c t2 with mu, a, c fixed by the random numbers and the frame of the
   cosine-weighted draw, t1 = (e_j x n) / |e_j x n|, t2 = n x t1 (o = o' after the reflection). */
static void tan_cyl(adj_list* al, const double o[3], const double n[3], double r, int specular)
{
    if (!al || !al->pathwise) return;
    double e[3] = {0.0, 0.0, 0.0}, c[3], t1[3], t2[3];
    double len = 0.0, mu = 0.0, ca = 0.0, cb = 0.0;
    if (!specular) {
        int j = 0;
        if (fabs(n[1]) < fabs(n[j])) j = 1;
        if (fabs(n[2]) < fabs(n[j])) j = 2;
        e[j] = 1.0;
        cross3(e, n, c);
        len = sqrt(dot3(c, c));
        for (int a = 0; a < 3; ++a) t1[a] = c[a] / len;
        cross3(n, t1, t2);
        mu = dot3(o, n);
        ca = dot3(o, t1);
        cb = dot3(o, t2);
    }
    for (int64_t i = 0; i < al->nt; ++i) {
        tangent* q = &al->tg[i];
        const double dn[3] = {q->dx[0] / r, q->dx[1] / r, 0.0};
        if (specular) {
            const double on = dot3(o, n);
            const double don = dot3(q->dO, n) + dot3(o, dn);
            for (int a = 0; a < 3; ++a) q->dO[a] = q->dO[a] - 2.0 * don * n[a] - 2.0 * on * dn[a];
        } else {
            double dc[3], dt1[3], dt2[3], u[3], w[3];
            cross3(e, dn, dc);
            const double p1 = dot3(t1, dc);
            for (int a = 0; a < 3; ++a) dt1[a] = (dc[a] - p1 * t1[a]) / len;
            cross3(dn, t1, u);
            cross3(n, dt1, w);
            for (int a = 0; a < 3; ++a) dt2[a] = u[a] + w[a];
            for (int a = 0; a < 3; ++a) q->dO[a] = mu * dn[a] + ca * dt1[a] + cb * dt2[a];
        }
    }
}

static uint32_t pack_ev(int ev, int64_t bnd, int32_t m)
{
    if (bnd > 255) bnd = 255;
    return ((uint32_t)ev << 28) | ((uint32_t)bnd << 20) | ((uint32_t)m & 0xFFFFFu);
}

static void trace_one(const orc_tables* t, uint64_t seed, uint32_t inst, int64_t pid, double* raw,
                      uint64_t* counts, double* mom, uint32_t* logrow, int32_t stride, double* pts,
                      adj_list* al, double* F_out)
{
    const orc_geom* g = &t->g;
    const orc_problem* pr = &t->pr;
    prt p;
    int64_t src = 0;
    int64_t nlog = 0;
#define LOG(ev, bnd, mode)                                                              \
    do {                                                                                \
        if (logrow) {                                                                   \
            if (nlog + 1 < stride) logrow[1 + nlog] = pack_ev((ev), (bnd), (mode));     \
            ++nlog;                                                                     \
        }                                                                               \
    } while (0)

    counts[ORC_C_PARTICLES] += 1;
    if (emit(t, seed, inst, pid, &p, counts, &src) != 0) {
        counts[ORC_C_ESCAPED] += 1;
        if (logrow) logrow[0] = 0;
        return;
    }
    LOG(p.s > 0 ? ORC_EV_EMIT_POS : ORC_EV_EMIT_NEG, src, p.m);
    const int sa = pr->score_axis;
    double dtr0 = p.dtr;       /* free-flight time drawn for the current flight */
    double F0 = 0.0;           /* flux contribution at the start of the current flight */
    if (al) al->sign = p.s;
    tan_birth(al, t->bin[p.m], t->v[p.m] * p.dtr);
#define CENSORED()                                                                                \
    do {                                                                                          \
        if (!adj_local(al, t, p.m)) adj_push(al, t->bin[p.m], (dtr0 - p.dtr) / t->tau[p.m], F0, 0); \
    } while (0)
    for (;;) {
        if ((int64_t)p.k >= pr->max_events) {
            counts[ORC_C_CAP_END] += 1;
            LOG(ORC_EV_CAP_END, 0, p.m);
            CENSORED();
            break;
        }
        const double v = t->v[p.m];
        const double ds = v * p.dtr;                  /* free-flight distance */
        int hit = 0;
        const double db = next_boundary(g, p.x, p.o, &hit);   /* nearest boundary along the ray */
        enum { EV_RELAX, EV_BND, EV_TIME } ev;
        double d;
        const double dmin = db < ds ? db : ds;
        if (pr->transient && v * (pr->t_max - p.t) <= dmin) {
            ev = EV_TIME;
            d = v * (pr->t_max - p.t);
        } else if (db <= ds) {
            ev = EV_BND;
            d = db;
        } else {
            ev = EV_RELAX;
            d = ds;
        }
        double dt = (ev == EV_RELAX) ? p.dtr : (ev == EV_BND ? d / v : pr->t_max - p.t);
        double t_end = (ev == EV_TIME) ? pr->t_max : p.t + dt;
        double sgn = (double)p.s;
        if (pr->transient) {
            tally_transient(t, p.x, p.o, p.t, t_end, p.m, sgn, raw);
        } else {
            tally_steady(t, p.x, p.o, d, p.m, sgn, raw, pts);
            p.cT += sgn * (d / v);
            p.cq += sgn * (d * p.o[sa]);
        }
        counts[ORC_C_FLIGHTS] += 1;
        for (int a = 0; a < 3; ++a) p.x[a] = p.x[a] + d * p.o[a];
        p.t = t_end;
        if (ev == EV_BND) {
            double r = p.dtr - dt;
            p.dtr = r > 0.0 ? r : 0.0;
        } else {
            p.dtr = 0.0;
        }
        p.k += 1;
        if (ev == EV_TIME) {
            counts[ORC_C_TIMEOUT] += 1;
            LOG(ORC_EV_TIMEOUT, 0, p.m);
            CENSORED();
            break;
        }
        int face_axis = -1, face_side = 0;
        if (ev == EV_BND && hit <= 6) {
            face_axis = FACE_AXIS[hit - 1];
            face_side = FACE_SIDE[hit - 1];
            p.x[face_axis] = face_side ? g->L[face_axis] : 0.0;      /* exactly on the wall */
        }
        if (al && al->pathwise) {                  /* the segment's end, for the tangents */
            const double dl = al->dline + d;       /* straight line since the last tangent update */
            al->dline = 0.0;
            if (ev == EV_RELAX) {
                tan_relax(al, p.o, dl);
            } else if (hit <= 6 && g->face[hit - 1].type == B_PERI) {
                /* a periodic transfer is a translation: the line goes on unchanged */
                al->dline = dl;
            } else {
                double nh[3] = {0.0, 0.0, 0.0};
                if (hit <= 6) {
                    nh[face_axis] = face_side ? -1.0 : 1.0;
                } else {
                    for (int c = 0; c < g->n_cyl; ++c)
                        if (g->cyl[c].id == hit) {
                            nh[0] = (p.x[0] - g->cyl[c].cx) / g->cyl[c].r;
                            nh[1] = (p.x[1] - g->cyl[c].cy) / g->cyl[c].r;
                        }
                }
                tan_hit(al, p.o, dl, nh);
            }
        }
        int escaped = 0;
        for (int a = 0; a < 3; ++a)
            if (!g->unbounded[a] && (p.x[a] < -1e-9 * g->L[a] || p.x[a] > g->L[a] + 1e-9 * g->L[a])) escaped = 1;
        if (escaped) {
            counts[ORC_C_ESCAPED] += 1;
            LOG(ORC_EV_ESCAPE, 0, p.m);
            CENSORED();
            break;
        }
        if (ev == EV_RELAX && p.nx2) {
            /* two-phonon (impurity) scattering (section 3.5.1): the same phonon takes a new
               isotropic direction and a new two-phonon clock; the three-phonon clock keeps
               running (case ii of section 3.3) */
            uint32_t R[8];
            p.j += 1;
            orc_record(seed, inst, pid, 2u + p.j, R);
            orc_dir_iso(unif(R, 4), unif(R, 6), p.o);
            set_clocks(&p, draw_t2(t, seed, inst, pid, p.j, p.m), p.lead);
            counts[ORC_C_TWO] += 1;
            LOG(ORC_EV_TWO, 0, p.m);
            continue;
        }
        if (ev == EV_RELAX) {
            /* three-phonon relaxation (section 3.5.2): new frequency from the post-scattering
               distribution, isotropic direction, sign kept; termination after N_scat^max */
            p.nrel += 1;
            counts[ORC_C_RELAX] += 1;
            if (adj_local(al, t, p.m))                                         /* the flight that ended */
                adj_push_local(al, t->bin[p.m], (double)p.s * (t->v[p.m] * dtr0) * p.o[sa],
                               dtr0 / t->tau[p.m] - 1.0, p.cq);
            else
                adj_push(al, t->bin[p.m], dtr0 / t->tau[p.m] - 1.0, F0, 0);
            if (pr->n_scat_max > 0 && p.nrel >= pr->n_scat_max) {
                counts[ORC_C_NSCAT_END] += 1;
                LOG(ORC_EV_NSCAT_END, 0, p.m);
                break;
            }
            uint32_t R[8];
            p.j += 1;
            orc_record(seed, inst, pid, 2u + p.j, R);
            p.m = (int32_t)orc_cdf_pick(t->thr_rel, t->M, t->last_rel, key64(R, 0));
            orc_dir_iso(unif(R, 4), unif(R, 6), p.o);
            p.dtr = -t->tau[p.m] * log(1.0 - unif(R, 2));
            if (t->two) set_clocks(&p, draw_t2(t, seed, inst, pid, p.j, p.m), p.dtr);   /* both resampled */
            LOG(ORC_EV_RELAX, 0, p.m);
            adj_push(al, t->bin[p.m], -1.0, p.cq, 1);                        /* the draw of the new row */
            tan_birth(al, t->bin[p.m], t->v[p.m] * p.dtr);
            dtr0 = p.dtr;
            F0 = p.cq;
            continue;
        }
        /* boundary interaction (sections 3.5.3-3.5.5) */
        int type;
        double spec = 0.0, spec_wc = 0.0;
        int32_t spec_tab = 0;
        const orc_cyl* cy = NULL;
        const orc_wall* wl = NULL;
        if (hit <= 6) {
            type = g->face[hit - 1].type;
            spec = g->face[hit - 1].data[0];
            spec_wc = g->face[hit - 1].data[1];
            spec_tab = g->face[hit - 1].spec_table;
        } else {
            for (int c = 0; c < g->n_cyl; ++c)
                if (g->cyl[c].id == hit) cy = &g->cyl[c];
            for (int k = 0; k < g->n_wall; ++k)
                if (g->wall[k].id == hit) wl = &g->wall[k];
            type = cy ? cy->type : wl->type;
            spec = cy ? cy->spec : wl->spec;
            spec_wc = cy ? cy->spec_wc : wl->spec_wc;
            spec_tab = cy ? cy->spec_table : wl->spec_table;
        }
        /* section 3.5.3: the specularity may depend on the phonon: the boundary's per-row table
           gives it for the phonon's row, or below the boundary's cutoff frequency the reflection
           is specular */
        if (type == B_ADIA && spec_tab > 0) spec = t->spec_tab[(int64_t)(spec_tab - 1) * t->M + p.m];
        if (type == B_ADIA && spec_wc > 0.0 && t->omega[p.m] < spec_wc) spec = 1.0;
        if (type == B_ISO) {
            counts[ORC_C_ABSORBED] += 1;
            LOG(ORC_EV_ABSORB, hit, p.m);
            CENSORED();
            break;
        }
        if (type == B_PERI) {
            /* linearized periodic condition (Eq. periodic_lin_final): reinsert unchanged */
            p.x[face_axis] = face_side ? 0.0 : g->L[face_axis];
            counts[ORC_C_PERIODIC] += 1;
            LOG(ORC_EV_PERIODIC, hit, p.m);
            continue;
        }
        uint32_t R[8];
        int have_R = 0;
        int specular;
        if (spec >= 1.0) {
            specular = 1;
        } else if (spec <= 0.0) {
            specular = 0;
        } else {
            p.j += 1;
            orc_record(seed, inst, pid, 2u + p.j, R);
            have_R = 1;
            specular = key64(R, 0) < (uint64_t)(spec * TWO64);
        }
        double n[3] = {0.0, 0.0, 0.0};            /* inward normal at the hit point */
        if (cy) {
            n[0] = (p.x[0] - cy->cx) / cy->r;
            n[1] = (p.x[1] - cy->cy) / cy->r;
        } else if (wl) {
            n[0] = wl->nx;
            n[1] = wl->ny;
        } else {
            n[face_axis] = face_side ? -1.0 : 1.0;
        }
        if (specular) {
            if (cy) tan_cyl(al, p.o, n, cy->r, 1);
            else if (!wl) tan_plane(al, face_axis, 1);
            if (cy || wl) {                           /* Eq. specular: k' = k - 2 (k.n) n */
                double k2 = 2.0 * (p.o[0] * n[0] + p.o[1] * n[1] + p.o[2] * n[2]);
                for (int a = 0; a < 3; ++a) p.o[a] = p.o[a] - k2 * n[a];
            } else {
                p.o[face_axis] = -p.o[face_axis];
            }
            counts[ORC_C_SPECULAR] += 1;
            LOG(ORC_EV_SPECULAR, hit, p.m);
        } else {
            if (!have_R) {
                p.j += 1;
                orc_record(seed, inst, pid, 2u + p.j, R);
            }
            orc_dir_cos(unif(R, 4), unif(R, 6), n, p.o);
            if (cy) tan_cyl(al, p.o, n, cy->r, 0);
            else if (!wl) tan_plane(al, face_axis, 0);
            counts[ORC_C_DIFFUSE] += 1;
            LOG(ORC_EV_DIFFUSE, hit, p.m);
        }
    }
#undef LOG
#undef CENSORED
    if (F_out) *F_out = p.cq;
    if (!pr->transient) {
        mom[0] += p.cT;
        mom[1] += p.cT * p.cT;
        mom[2] += p.cq;
        mom[3] += p.cq * p.cq;
    }
    if (logrow) logrow[0] = (uint32_t)nlog;
}

int orc_trace(const orc_tables* t, uint64_t seed, uint32_t instance, int64_t first_pid, int64_t n,
              double* raw, uint64_t* counts, double* moments, uint32_t* log, int64_t n_log, int32_t log_stride)
{
    if (!t || n < 0 || first_pid < 0 || (n_log > 0 && (!log || log_stride < 2))) return E_INVAL;
    int cap = 2;
    for (int a = 0; a < 3; ++a) cap += t->det.n[a];
    double* pts = (double*)malloc(sizeof(double) * cap);
    if (!pts) return E_NOMEM;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t* row = (i < n_log) ? log + i * (int64_t)log_stride : NULL;
        trace_one(t, seed, instance, first_pid + i, raw, counts, moments, row, log_stride, pts, NULL, NULL);
    }
    free(pts);
    return E_OK;
}

int orc_adjoint(const orc_tables* t, uint64_t seed, uint32_t instance, int64_t first_pid, int64_t n,
                int32_t kind, double lambda_split, double* sparse, double* dense, double* F_out, double* pp_out,
                int64_t* n_bad)
{
    if (!t || n < 0 || first_pid < 0 || t->pr.transient || kind < 0 || kind > 2) return E_INVAL;
    if (t->two) return E_INVAL;     /* the estimators differentiate the one-clock flight law */
    if (t->g.n_wall > 0) return E_INVAL;   /* their tangents know planes of the box and cylinders */
    int cap = 2;
    for (int a = 0; a < 3; ++a) cap += t->det.n[a];
    double* pts = (double*)malloc(sizeof(double) * cap);
    double* raw = (double*)calloc((size_t)(t->n_cells * t->n_cols * 4), sizeof(double));
    if (!pts || !raw) { free(pts); free(raw); return E_NOMEM; }
    uint64_t counts[ORC_N_COUNTS] = {0};
    double mom[ORC_N_MOMENTS] = {0};
    adj_list al;
    memset(&al, 0, sizeof(al));
    al.pathwise = kind == 1;
    al.local = kind == 2;
    al.lambda_split = lambda_split;
    const int sa = t->pr.score_axis;
    for (int64_t i = 0; i < n; ++i) {
        al.n = 0;
        al.nt = 0;
        al.dline = 0.0;
        double F = 0.0;
        trace_one(t, seed, instance, first_pid + i, raw, counts, mom, NULL, 0, pts, &al, &F);
        if (al.failed) break;
        for (int64_t e = 0; e < al.n; ++e) {
            const double after = F - al.ev[e].F_before;
            sparse[al.ev[e].bin] += al.ev[e].c0 + al.ev[e].g * after;
            if (al.ev[e].dense) *dense += after;
        }
        for (int64_t e = 0; e < al.nt; ++e) {
            const double c = (double)al.sign * al.tg[e].dx[sa];
            if (!isfinite(c)) {             /* left out and counted */
                if (n_bad) *n_bad += 1;
                continue;
            }
            sparse[al.tg[e].bin] += c;
            if (pp_out) pp_out[i * t->n_bins + al.tg[e].bin] += c;
        }
        if (F_out) F_out[i] = F;
    }
    int failed = al.failed;
    free(al.ev);
    free(al.tg);
    free(pts);
    free(raw);
    return failed ? E_NOMEM : E_OK;
}
