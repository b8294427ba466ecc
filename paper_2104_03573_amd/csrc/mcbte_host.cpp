// Host side of the C ABI (include/mcbte.h): validation, the FP64 table build, device upload,
// launch configuration and the finalization of the tallies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "mcbte.h"
#include "mcbte_dev.h"

namespace mcbte {
hipError_t launch_emit(const DevTab* d_tab, int precision, uint64_t seed, uint32_t inst, int64_t first_pid, int64_t n,
                       void* state, int64_t cap, hipStream_t s);
hipError_t launch_trace(const LaunchArgs& a, int mode, int precision, int tally_kind, int ft, int block, int grid, size_t lds,
                        hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, hipStream_t s);
hipError_t static_queue(int dev, unsigned char** out);
int64_t static_queue_bytes();
hipError_t launch_batch_setup(const BatchSetupArgs& args, unsigned char* q, hipStream_t s);
int trace_occupancy(int mode, int precision, int tally_kind, int ft, int block, size_t lds);
}  // namespace mcbte

using namespace mcbte;

namespace {

const double kHbar = 1.054571817e-34;   // J s (CODATA 2018)
const double kBoltzmann = 1.380649e-23; // J/K (exact, SI 2019)
const double kPi = 3.141592653589793;
const double kTwo64 = 18446744073709551616.0;

// boundary id - 1 -> axis, side (1: the face at L, 0: the face at 0)
const int kFaceAxis[6] = {1, 0, 1, 0, 2, 2};
const int kFaceSide[6] = {0, 1, 1, 0, 0, 1};

// event class of an adiabatic surface of specularity d, as the trajectories of precision R see d
template <typename R>
uint32_t surf_class(double d)
{
    const R r = (R)d;
    return (r > R(0) && r < R(1)) ? SURF_PARTIAL : (r >= R(1) ? SURF_SPECULAR : SURF_DIFFUSE);
}

// volume of a tetrahedron (vertices at v[0..2], v[3..5], v[6..8], v[9..11]): |triple product of the
// edges from vertex 0| / 6
double tetra_volume(const double* v)
{
    double a[3], b[3], c[3];
    for (int i = 0; i < 3; ++i) {
        a[i] = v[3 + i] - v[i];
        b[i] = v[6 + i] - v[i];
        c[i] = v[9 + i] - v[i];
    }
    const double cx = b[1] * c[2] - b[2] * c[1], cy = b[2] * c[0] - b[0] * c[2], cz = b[0] * c[1] - b[1] * c[0];
    return std::fabs(a[0] * cx + a[1] * cy + a[2] * cz) / 6.0;
}

// cumulative distribution as 64-bit thresholds; returns the last positive-weight index (-1 if none)
int64_t build_thresholds(const std::vector<double>& w, std::vector<uint64_t>& thr)
{
    const size_t n = w.size();
    thr.assign(n, 0);
    double total = 0.0;
    int64_t last = -1;
    for (size_t i = 0; i < n; ++i) {
        total += w[i];
        if (w[i] > 0.0) last = (int64_t)i;
    }
    if (last < 0) return -1;
    double running = 0.0;
    for (size_t i = 0; i < n; ++i) {
        running += w[i];
        const double F = running / total;
        thr[i] = F >= 1.0 ? UINT64_MAX : (uint64_t)(F * kTwo64);
    }
    return last;
}

// d e_eq / dT of one mode: k_B (x/2)^2 / sinh^2(x/2) with x = hbar omega / (k_B T)
double bose_einstein_dedT(double omega, double T)
{
    const double x = (kHbar * omega) / (kBoltzmann * T);
    const double h = 0.5 * x;
    const double sh = std::sinh(h);
    return (kBoltzmann * (h * h)) / (sh * sh);
}

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct mcbte_tables {
    int32_t device = -1;
    mcbte_info info{};
    mcbte_problem prob{};
    mcbte_geometry geom{};
    mcbte_detectors det{};
    // host tables
    std::vector<double> C, v, tau, tau2, src_E, ic_edges, ic_dT, t_meas;   // tau2: two-phonon clock (0: none)
    std::vector<double> heat_t, heat_P;   // external heat source: interval edges and power densities
    std::vector<double> heat_tet;         // its tetrahedra: vertex 0 and the three edges from it
    std::vector<uint64_t> thr_tet;        // a tetrahedron by volume
    int64_t last_tet = 0;
    bool two = false;      // some row has a two-phonon clock
    bool spec_w = false;   // some boundary has a specular cutoff frequency
    bool walls = false;    // internal line walls
    bool ext_film = false; // a film whose walls reflect some phonons specularly: the FP32 film paths for
                           // specular and partly specular walls live in the kernels with the extended code
    std::vector<double> omega;
    std::vector<uint64_t> thr_ic, thr_wall, thr_rel, thr_src;
    std::vector<int32_t> src_kind, src_ref, src_sign, bin_of;
    std::vector<double> P_bin;   // relaxation probability mass per frequency bin
    std::vector<uint64_t> prio_thr;   // pore lattice: first-flight keys started first (per mode)
    std::vector<double> spec_d;       // per-row specularity tables the boundaries read (table-major)
    std::vector<uint64_t> spec_thr;   // their thresholds and classes
    std::vector<uint8_t> spec_cls;
    DevTab host_view{};   // device pointers once uploaded
    void* d_mem = nullptr;
    DevTab* d_tab = nullptr;
    int n_cu = 0;
    int max_lds = 0;
};

namespace {

// The deviational energy per particle's normalisation of raw sums (Eq. tally definitions):
// T = e / (C_tot V_cell) * sum s*t, q = e / V_cell * sum s*dx, with e = E_tot / n and V_cell the
// detector cell (the solid volume for an unbinned tally).  Writes n_cells * n_cols * 4 values
// when out is given.
void normalize_raw(const mcbte_tables* t, const double* raw, double n, double* out, double* e_out, double* Vc_out)
{
    const mcbte_info& inf = t->info;
    const double e = inf.E_tot / n;
    double Vc = 1.0;
    bool binned = false;
    for (int a = 0; a < 3; ++a) {
        if (t->det.n[a] > 0) {
            binned = true;
            Vc *= (t->det.hi[a] - t->det.lo[a]) / (double)t->det.n[a];
        } else if (!t->geom.unbounded[a]) {
            Vc *= t->geom.L[a];
        }
    }
    if (!binned) Vc = inf.V_solid;
    if (e_out) *e_out = e;
    if (Vc_out) *Vc_out = Vc;
    if (!out) return;
    const int64_t n_raw = inf.n_cells * inf.n_cols * 4;
    const double sT = e / (inf.C_tot * Vc), sq = e / Vc;
    for (int64_t i = 0; i < n_raw; i += 4) {
        out[i] = sT * raw[i];
        out[i + 1] = sq * raw[i + 1];
        out[i + 2] = sq * raw[i + 2];
        out[i + 3] = sq * raw[i + 3];
    }
}

}  // namespace

extern "C" {

const char* mcbte_strerror(int status)
{
    switch (status) {
    case MCBTE_OK: return "ok";
    case MCBTE_EINVAL: return "invalid argument";
    case MCBTE_ENOMEM: return "out of memory";
    case MCBTE_EHIP: return "HIP runtime error";
    case MCBTE_ENODEV: return "tables were built without a device";
    case MCBTE_ETABLE: return "a distribution or the source list has zero total weight";
    case MCBTE_EGEOM: return "invalid geometry";
    case MCBTE_ESIZE: return "caller buffer too small";
    case MCBTE_ERANGE: return "a sensitivity term was not finite (pathwise tangents grew without bound)";
    case MCBTE_ELIMIT: return "more instances than the allocation-free batched trace holds (MCBTE_STATIC_MAX_INSTANCES)";
    default: return "unknown status";
    }
}

void mcbte_free_tables(mcbte_tables* t)
{
    if (!t) return;
    if (t->d_mem) {
        DeviceGuard g(t->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(t->d_mem);
    }
    delete t;
}

int mcbte_build_tables(const mcbte_mode* modes, int32_t M, const mcbte_geometry* geometry,
                       const mcbte_detectors* detectors, const mcbte_problem* problem, int32_t device,
                       mcbte_tables** out)
{
    if (!out) return MCBTE_EINVAL;
    *out = nullptr;
    if (!modes || !geometry || !detectors || !problem || M < 1 || device < -1) return MCBTE_EINVAL;
    const mcbte_geometry& g = *geometry;
    const mcbte_detectors& dt = *detectors;
    const mcbte_problem& pr = *problem;
    if (pr.N < 1 || !(pr.T_lin > 0.0) || (pr.format != 1 && pr.format != 2)) return MCBTE_EINVAL;
    if (pr.score_axis < 0 || pr.score_axis > 2 || pr.max_events < 1 || pr.max_events > 0x3FFFFFF0LL) return MCBTE_EINVAL;
    if (pr.n_scat_max < 0) return MCBTE_EINVAL;
    const int32_t NT = pr.n_spec_tables;
    if (NT < 0 || (NT > 0 && !pr.spec_table)) return MCBTE_EINVAL;
    for (int64_t i = 0; i < (int64_t)NT * M; ++i)
        if (!(pr.spec_table[i] >= 0.0 && pr.spec_table[i] <= 1.0)) return MCBTE_EINVAL;
    // a boundary's per-row specularity table: a known number, adiabatic, its own d and cutoff 0
    auto bad_tab = [&](int32_t k, bool adiabatic, double d, double wc) {
        return k < 0 || k > NT || (k > 0 && (!adiabatic || d != 0.0 || wc != 0.0));
    };
    // geometry
    for (int a = 0; a < 3; ++a)
        if (!g.unbounded[a] && !(g.L[a] > 0.0)) return MCBTE_EGEOM;
    for (int i = 0; i < 6; ++i) {
        if (g.unbounded[kFaceAxis[i]]) continue;
        const int ty = g.face[i].type;
        if (ty != MCBTE_ISOTHERMAL && ty != MCBTE_ADIABATIC && ty != MCBTE_PERIODIC) return MCBTE_EGEOM;
        if (ty == MCBTE_ADIABATIC && !(g.face[i].data[0] >= 0.0 && g.face[i].data[0] <= 1.0)) return MCBTE_EGEOM;
        if (ty == MCBTE_ADIABATIC && !(g.face[i].data[1] >= 0.0 && std::isfinite(g.face[i].data[1]))) return MCBTE_EGEOM;
        if (bad_tab(g.face[i].spec_table, ty == MCBTE_ADIABATIC, ty == MCBTE_ADIABATIC ? g.face[i].data[0] : 0.0,
                    ty == MCBTE_ADIABATIC ? g.face[i].data[1] : 0.0))
            return MCBTE_EGEOM;
    }
    for (int a = 0; a < 3; ++a) {
        if (g.unbounded[a]) continue;
        int lo = -1, hi = -1;
        for (int i = 0; i < 6; ++i)
            if (kFaceAxis[i] == a) (kFaceSide[i] ? hi : lo) = i;
        const bool plo = g.face[lo].type == MCBTE_PERIODIC, phi = g.face[hi].type == MCBTE_PERIODIC;
        if (plo != phi) return MCBTE_EGEOM;
        if (plo) {   // the translation must carry each face onto its partner
            for (int b = 0; b < 3; ++b) {
                const double want_lo = (b == a) ? g.L[a] : 0.0;
                if (std::fabs(g.face[lo].data[b] - want_lo) > 1e-9 * g.L[a] ||
                    std::fabs(g.face[hi].data[b] + want_lo) > 1e-9 * g.L[a])
                    return MCBTE_EGEOM;
            }
        }
    }
    if (g.n_pores < 0 || g.n_pores > MCBTE_MAX_PORES) return MCBTE_EGEOM;
    for (int c = 0; c < g.n_pores; ++c) {
        const mcbte_pore& p = g.pore[c];
        if (g.unbounded[0] || g.unbounded[1] || !(p.r > 0.0) || p.type != MCBTE_ADIABATIC) return MCBTE_EGEOM;
        if (!(p.specularity >= 0.0 && p.specularity <= 1.0)) return MCBTE_EGEOM;
        if (!(p.spec_omega >= 0.0 && std::isfinite(p.spec_omega))) return MCBTE_EGEOM;
        if (p.reserved != 0 || bad_tab(p.spec_table, true, p.specularity, p.spec_omega)) return MCBTE_EGEOM;
        if (p.cx - p.r < 0.0 || p.cx + p.r > g.L[0] || p.cy - p.r < 0.0 || p.cy + p.r > g.L[1]) return MCBTE_EGEOM;
        if (p.id < 7 || p.id > 255 || (c > 0 && p.id <= g.pore[c - 1].id)) return MCBTE_EGEOM;
    }
    if (g.n_walls < 0 || g.n_walls > MCBTE_MAX_WALLS) return MCBTE_EGEOM;
    for (int k = 0; k < g.n_walls; ++k) {
        const mcbte_wall& w = g.wall[k];
        const int prev = k > 0 ? g.wall[k - 1].id : (g.n_pores > 0 ? g.pore[g.n_pores - 1].id : 6);
        if (g.unbounded[0] || g.unbounded[1] || (w.type != MCBTE_ADIABATIC && w.type != MCBTE_ISOTHERMAL) ||
            w.id <= prev || w.id > 255)
            return MCBTE_EGEOM;
        if (w.type == MCBTE_ADIABATIC && !(w.data >= 0.0 && w.data <= 1.0)) return MCBTE_EGEOM;
        if (w.type == MCBTE_ISOTHERMAL && !(w.data > 0.0 && std::isfinite(w.data))) return MCBTE_EGEOM;
        if (!(w.spec_omega >= 0.0 && std::isfinite(w.spec_omega))) return MCBTE_EGEOM;
        if (w.reserved != 0 || bad_tab(w.spec_table, w.type == MCBTE_ADIABATIC, w.type == MCBTE_ADIABATIC ? w.data : 0.0,
                                       w.spec_omega))
            return MCBTE_EGEOM;
        const double pts[4] = {w.x1, w.y1, w.x2, w.y2};
        for (int q = 0; q < 4; ++q)
            if (!(pts[q] >= 0.0 && pts[q] <= g.L[q & 1])) return MCBTE_EGEOM;
        if (w.x1 == w.x2 && w.y1 == w.y2) return MCBTE_EGEOM;
        const double nn = std::sqrt(w.nx * w.nx + w.ny * w.ny);
        if (!(std::fabs(nn - 1.0) <= 1e-9)) return MCBTE_EGEOM;
    }
    if (g.n_walls > 0 && !(g.volume > 0.0)) return MCBTE_EINVAL;   // the solid volume must be given
    // detectors
    for (int a = 0; a < 3; ++a)
        if (dt.n[a] < 0 || (dt.n[a] > 0 && !(dt.hi[a] > dt.lo[a]))) return MCBTE_EINVAL;
    if (dt.mask < 1 || dt.mask > 15) return MCBTE_EINVAL;
    // run
    if (pr.transient) {
        if (!(pr.t_max > 0.0) || pr.n_times < 1 || !pr.t_meas) return MCBTE_EINVAL;
        for (int k = 0; k < pr.n_times; ++k)
            if (!(pr.t_meas[k] >= 0.0) || (k > 0 && !(pr.t_meas[k] >= pr.t_meas[k - 1]))) return MCBTE_EINVAL;
    } else if (pr.n_ic > 0) {
        return MCBTE_EINVAL;
    }
    // external heat source: transient, ascending edges in [0, t_max], a cuboid inside the box and the solid
    if (pr.n_heat < 0 || pr.n_heat_tet < 0 || (pr.n_heat == 0 && pr.n_heat_tet != 0)) return MCBTE_EINVAL;
    if (pr.n_heat > 0) {
        if (!pr.transient || !pr.heat_t || !pr.heat_P || g.n_walls > 0) return MCBTE_EINVAL;
        if (!(pr.heat_t[0] >= 0.0) || !(pr.heat_t[pr.n_heat] <= pr.t_max)) return MCBTE_EINVAL;
        for (int k = 0; k < pr.n_heat; ++k)
            if (!(pr.heat_t[k + 1] > pr.heat_t[k]) || !std::isfinite(pr.heat_P[k])) return MCBTE_EINVAL;
        for (int a = 0; a < 3; ++a)
            if (!g.unbounded[a] && !(pr.heat_lo[a] >= 0.0 && pr.heat_hi[a] > pr.heat_lo[a] && pr.heat_hi[a] <= g.L[a]))
                return MCBTE_EINVAL;
        for (int c = 0; c < g.n_pores; ++c) {   // the pore's disc keeps off the region's rectangle
            const double dx = std::max({pr.heat_lo[0] - g.pore[c].cx, 0.0, g.pore[c].cx - pr.heat_hi[0]});
            const double dy = std::max({pr.heat_lo[1] - g.pore[c].cy, 0.0, g.pore[c].cy - pr.heat_hi[1]});
            if (dx * dx + dy * dy < g.pore[c].r * g.pore[c].r) return MCBTE_EINVAL;
        }
        // tetrahedra: inside the box, positive volume, x-y bounding rectangle clear of the pores
        if (pr.n_heat_tet > 0 && !pr.heat_tet) return MCBTE_EINVAL;
        for (int k = 0; k < pr.n_heat_tet; ++k) {
            const double* v = pr.heat_tet + 12 * (int64_t)k;
            double lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                lo[a] = hi[a] = v[a];
                for (int q = 0; q < 4; ++q) {
                    const double x = v[3 * q + a];
                    if (!std::isfinite(x) || (!g.unbounded[a] && !(x >= 0.0 && x <= g.L[a]))) return MCBTE_EINVAL;
                    lo[a] = std::min(lo[a], x);
                    hi[a] = std::max(hi[a], x);
                }
            }
            if (!(tetra_volume(v) > 0.0)) return MCBTE_EINVAL;
            for (int c = 0; c < g.n_pores; ++c) {
                const double dx = std::max({lo[0] - g.pore[c].cx, 0.0, g.pore[c].cx - hi[0]});
                const double dy = std::max({lo[1] - g.pore[c].cy, 0.0, g.pore[c].cy - hi[1]});
                if (dx * dx + dy * dy < g.pore[c].r * g.pore[c].r) return MCBTE_EINVAL;
            }
        }
    }
    if (pr.n_ic < 0 || (pr.n_ic > 0 && (!pr.ic_edges || !pr.ic_dT || pr.ic_axis < 0 || pr.ic_axis > 2 || g.n_pores > 0 ||
                                        g.n_walls > 0)))
        return MCBTE_EINVAL;

    mcbte_tables* t = new (std::nothrow) mcbte_tables();
    if (!t) return MCBTE_ENOMEM;
    t->device = device;
    t->prob = pr;
    t->prob.t_meas = nullptr;
    t->prob.ic_edges = nullptr;
    t->prob.heat_t = nullptr;
    t->prob.heat_P = nullptr;
    t->prob.heat_tet = nullptr;
    t->prob.ic_dT = nullptr;
    t->prob.spec_table = nullptr;
    t->geom = g;
    t->det = dt;

    // per-mode heat capacity (first format: DOS x delta-omega x de/dT at T_lin)
    t->C.resize(M);
    t->v.resize(M);
    t->tau.resize(M);
    t->tau2.resize(M);
    t->omega.resize(M);
    for (int m = 0; m < M; ++m) {
        const mcbte_mode& r = modes[m];
        if (!(r.v > 0.0) || !(r.tau > 0.0)) { delete t; return MCBTE_EINVAL; }
        if (!(r.tau_imp >= 0.0) || !std::isfinite(r.tau_imp)) { delete t; return MCBTE_EINVAL; }
        t->v[m] = r.v;
        t->tau[m] = r.tau;
        t->tau2[m] = r.tau_imp;
        if (r.tau_imp > 0.0) t->two = true;
        t->omega[m] = r.omega;
        if (pr.format == 1) {
            if (!(r.dos >= 0.0) || !(r.domega >= 0.0) || !(r.omega > 0.0)) { delete t; return MCBTE_EINVAL; }
            t->C[m] = (r.dos * r.domega) * bose_einstein_dedT(r.omega, pr.T_lin);
        } else {
            if (!(r.C >= 0.0)) { delete t; return MCBTE_EINVAL; }
            t->C[m] = r.C;
        }
    }
    double C_tot = 0.0, Wv = 0.0, kb = 0.0;
    for (int m = 0; m < M; ++m) {
        C_tot += t->C[m];
        Wv += t->C[m] * t->v[m];
        // with a two-phonon clock both processes relax the heat-carrying part: the rates add
        const double tau_eff = t->tau2[m] > 0.0 ? 1.0 / (1.0 / t->tau[m] + 1.0 / t->tau2[m]) : t->tau[m];
        kb += ((t->C[m] * t->v[m]) * t->v[m]) * tau_eff;
    }
    if (!(C_tot > 0.0)) { delete t; return MCBTE_ETABLE; }
    std::vector<double> w(M);
    for (int m = 0; m < M; ++m) w[m] = t->C[m];
    const int64_t last_ic = build_thresholds(w, t->thr_ic);
    for (int m = 0; m < M; ++m) w[m] = t->C[m] * t->v[m];
    const int64_t last_wall = build_thresholds(w, t->thr_wall);
    for (int m = 0; m < M; ++m) w[m] = t->C[m] / t->tau[m];
    const int64_t last_rel = build_thresholds(w, t->thr_rel);
    if (last_ic < 0 || last_wall < 0 || last_rel < 0) { delete t; return MCBTE_ETABLE; }
    // frequency bins: the parameters of the sensitivities dkappa / dln tau_i
    int32_t n_bins = 0;
    t->bin_of.resize(M);
    for (int m = 0; m < M; ++m) {
        if (modes[m].bin < 0 || modes[m].bin >= (1 << 20)) { delete t; return MCBTE_EINVAL; }
        t->bin_of[m] = modes[m].bin;
        n_bins = std::max(n_bins, modes[m].bin + 1);
    }
    t->P_bin.assign(n_bins, 0.0);
    {
        double Wr = 0.0;
        for (int m = 0; m < M; ++m) Wr += t->C[m] / t->tau[m];
        for (int m = 0; m < M; ++m) t->P_bin[t->bin_of[m]] += (t->C[m] / t->tau[m]) / Wr;
    }

    auto extent = [&](int a) { return g.unbounded[a] ? 1.0 : g.L[a]; };
    double V = g.volume;
    if (!(V > 0.0)) {
        V = (extent(0) * extent(1)) * extent(2);
        for (int c = 0; c < g.n_pores; ++c) V = V - (kPi * (g.pore[c].r * g.pore[c].r)) * extent(2);
    }
    const double gnorm = std::sqrt((g.gradT[0] * g.gradT[0] + g.gradT[1] * g.gradT[1]) + g.gradT[2] * g.gradT[2]);

    if (pr.transient) t->t_meas.assign(pr.t_meas, pr.t_meas + pr.n_times);
    if (pr.n_ic > 0) {
        t->ic_edges.assign(pr.ic_edges, pr.ic_edges + pr.n_ic + 1);
        t->ic_dT.assign(pr.ic_dT, pr.ic_dT + pr.n_ic);
        for (int c = 0; c < pr.n_ic; ++c)
            if (!(t->ic_edges[c + 1] > t->ic_edges[c])) { delete t; return MCBTE_EINVAL; }
    }
    // sources: isothermal faces by id, the gradient source, initial-condition cells
    for (int i = 0; i < 6; ++i) {
        const int a = kFaceAxis[i];
        if (g.unbounded[a] || g.face[i].type != MCBTE_ISOTHERMAL) continue;
        const double dT = g.face[i].data[0] - pr.T_lin;
        if (dT == 0.0) continue;
        const int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
        const double area = extent(b) * extent(c);
        double E = ((area * std::fabs(dT)) * Wv) / 4.0;     // A |T_b - T_lin| sum C v / 4
        if (pr.transient) E = E * pr.t_max;
        t->src_kind.push_back(SRC_WALL);
        t->src_ref.push_back(i + 1);
        t->src_sign.push_back(dT > 0.0 ? 1 : -1);
        t->src_E.push_back(E);
    }
    // isothermal line walls by id: area = segment length x thickness
    for (int k = 0; k < g.n_walls; ++k) {
        const mcbte_wall& w = g.wall[k];
        if (w.type != MCBTE_ISOTHERMAL) continue;
        const double dT = w.data - pr.T_lin;
        if (dT == 0.0) continue;
        const double ex = w.x2 - w.x1, ey = w.y2 - w.y1;
        const double area = std::sqrt(ex * ex + ey * ey) * extent(2);
        double E = ((area * std::fabs(dT)) * Wv) / 4.0;
        if (pr.transient) E = E * pr.t_max;
        t->src_kind.push_back(SRC_IWALL);
        t->src_ref.push_back(k);
        t->src_sign.push_back(dT > 0.0 ? 1 : -1);
        t->src_E.push_back(E);
    }
    if (gnorm > 0.0) {
        double E = ((V * gnorm) * Wv) / 2.0;                // V |grad T| sum C v / 2
        if (pr.transient) E = E * pr.t_max;
        t->src_kind.push_back(SRC_GRAD);
        t->src_ref.push_back(0);
        t->src_sign.push_back(0);
        t->src_E.push_back(E);
    }
    for (int c = 0; c < pr.n_ic; ++c) {
        const int a = pr.ic_axis;
        const int b = (a == 0) ? 1 : 0, cc = (a == 2) ? 1 : 2;
        const double Vc = ((t->ic_edges[c + 1] - t->ic_edges[c]) * extent(b)) * extent(cc);
        const double E = (C_tot * std::fabs(t->ic_dT[c])) * Vc; // C_tot |dT_c| V_c
        t->src_kind.push_back(SRC_IC);
        t->src_ref.push_back(c);
        t->src_sign.push_back(t->ic_dT[c] > 0.0 ? 1 : -1);
        t->src_E.push_back(E);
    }
    // the external heat source, one source per time interval: |P_k| V_heat (t_k+1 - t_k)
    if (pr.n_heat > 0) {
        t->heat_t.assign(pr.heat_t, pr.heat_t + pr.n_heat + 1);
        t->heat_P.assign(pr.heat_P, pr.heat_P + pr.n_heat);
        double Vh = 1.0;
        for (int a = 0; a < 3; ++a) Vh *= g.unbounded[a] ? 1.0 : pr.heat_hi[a] - pr.heat_lo[a];
        if (pr.n_heat_tet > 0) {   // the union of the tetrahedra: one drawn by volume
            const int nt = pr.n_heat_tet;
            std::vector<double> vol((size_t)nt);
            t->heat_tet.assign(12 * (size_t)nt, 0.0);
            Vh = 0.0;
            for (int k = 0; k < nt; ++k) {
                const double* v = pr.heat_tet + 12 * (int64_t)k;
                double* o = t->heat_tet.data() + 12 * (size_t)k;
                for (int a = 0; a < 3; ++a) {
                    o[a] = v[a];
                    for (int q = 1; q < 4; ++q) o[3 * q + a] = v[3 * q + a] - v[a];
                }
                vol[(size_t)k] = tetra_volume(v);
                Vh += vol[(size_t)k];
            }
            t->last_tet = build_thresholds(vol, t->thr_tet);
        }
        for (int k = 0; k < pr.n_heat; ++k) {
            if (t->heat_P[k] == 0.0) continue;
            t->src_kind.push_back(SRC_HEAT);
            t->src_ref.push_back(k);
            t->src_sign.push_back(t->heat_P[k] > 0.0 ? 1 : -1);
            t->src_E.push_back((std::fabs(t->heat_P[k]) * Vh) * (t->heat_t[k + 1] - t->heat_t[k]));
        }
    }
    const int S = (int)t->src_E.size();
    if (S == 0) { delete t; return MCBTE_ETABLE; }
    double E_tot = 0.0;
    for (int s = 0; s < S; ++s) E_tot += t->src_E[s];
    const int64_t last_src = build_thresholds(t->src_E, t->thr_src);
    if (last_src < 0) { delete t; return MCBTE_ETABLE; }

    int64_t n_cells = 1;
    for (int a = 0; a < 3; ++a) n_cells *= dt.n[a] > 0 ? dt.n[a] : 1;
    const int64_t n_cols = pr.transient ? pr.n_times : M;

    mcbte_info& inf = t->info;
    inf.C_tot = C_tot;
    inf.sum_Cv = Wv;
    inf.E_tot = E_tot;
    inf.e_eff = E_tot / (double)pr.N;
    inf.V_solid = V;
    inf.kappa_bulk = kb / 3.0;
    inf.n_modes = M;
    inf.n_sources = S;
    inf.n_cells = n_cells;
    inf.n_cols = n_cols;
    inf.tally_bytes = MCBTE_TALLY_HEADER_BYTES + n_cells * n_cols * 4 * (int64_t)sizeof(double);
    inf.n_bins = n_bins;
    inf.adj_doubles = (int64_t)n_bins + 3;
    inf.device = device;

    // device view
    DevTab& h = t->host_view;
    std::memset(&h, 0, sizeof(h));
    h.M = M;
    h.S = S;
    h.transient = pr.transient ? 1 : 0;
    h.n_scat_max = pr.n_scat_max;
    h.score_axis = pr.score_axis;
    h.n_times = pr.transient ? pr.n_times : 0;
    h.ic_axis = pr.ic_axis;
    h.n_ic = pr.n_ic;
    bool binned = false;
    for (int a = 0; a < 3; ++a) binned = binned || dt.n[a] > 0;
    h.tally_kind = pr.transient ? TALLY_TRANSIENT : (binned ? TALLY_STEADY_GRID : TALLY_STEADY_ONE);
    // film-like problems (one bounded axis with fully diffuse faces, no pores, steady, one detector
    // cell): a particle with a long free path bounces between the two walls many times in a row,
    // which the FP32 kernel evaluates 64 bounces at a time with the whole wave
    h.coop_axis = -1;
    h.fold_axis = -1;
    h.coop_min_path = 0.0;
    {
        int nb = 0, axis = -1;
        for (int a = 0; a < 3; ++a)
            if (!g.unbounded[a]) { ++nb; axis = a; }
        if (nb == 1 && g.n_pores == 0 && g.n_walls == 0 && !pr.transient && h.tally_kind == TALLY_STEADY_ONE) {
            // (with a specular cutoff or a per-row table, the same one on both walls: a phonon's
            // class is then the same at every bounce of a chain, and the kernel only starts chains
            // of diffuse ones)
            bool diffuse = true;
            double wc = -1.0;
            int32_t tab = -1;
            for (int i = 0; i < 6; ++i) {
                if (kFaceAxis[i] != axis) continue;
                if (!(g.face[i].type == MCBTE_ADIABATIC && g.face[i].data[0] == 0.0)) diffuse = false;
                if (wc >= 0.0 && g.face[i].data[1] != wc) diffuse = false;
                if (tab >= 0 && g.face[i].spec_table != tab) diffuse = false;
                wc = g.face[i].data[1];
                tab = g.face[i].spec_table;
            }
            if (diffuse) {
                h.coop_axis = axis;
                h.coop_min_path = 16.0 * g.L[axis];
            }
            // both walls adiabatic with the same specularity rule: a phonon the walls reflect
            // specularly crosses the film wall to wall until its free path runs out
            bool same = true;
            const mcbte_face* first = nullptr;
            for (int i = 0; i < 6; ++i) {
                if (kFaceAxis[i] != axis) continue;
                const mcbte_face& f = g.face[i];
                if (f.type != MCBTE_ADIABATIC) same = false;
                if (first && (f.data[0] != first->data[0] || f.data[1] != first->data[1] ||
                              f.spec_table != first->spec_table))
                    same = false;
                first = &f;
            }
            if (same) {
                h.fold_axis = axis;
                h.coop_min_path = 16.0 * g.L[axis];
                for (int i = 0; i < 6; ++i)
                    if (kFaceAxis[i] == axis && (g.face[i].data[0] > 0.0 || g.face[i].data[1] > 0.0 || g.face[i].spec_table > 0))
                        t->ext_film = true;
            }
        }
    }
    // a lattice of pores: x and y periodic, z periodic or unbounded, one pore lying inside the cell,
    // no line walls, steady, one detector cell.  A free path of more than 64 cell widths ahead is
    // walked from pore to pore by the wave in the FP32 form (long enough that the wave's work on one
    // particle pays; the shorter ones leave the wave to its other lanes)
    h.lattice = 0;
    h.lat_min_path = 0.0;
    {
        bool per = g.n_pores == 1 && g.n_walls == 0 && !pr.transient && h.tally_kind == TALLY_STEADY_ONE &&
                   !g.unbounded[0] && !g.unbounded[1];
        for (int i = 0; i < 6 && per; ++i)
            if (!g.unbounded[kFaceAxis[i]] && g.face[i].type != MCBTE_PERIODIC) per = false;
        if (per) {
            const mcbte_pore& q = g.pore[0];
            per = q.cx - q.r > 0.0 && q.cx + q.r < g.L[0] && q.cy - q.r > 0.0 && q.cy + q.r < g.L[1];
        }
        if (per) {
            h.lattice = 1;
            h.lat_min_path = 64.0 * std::max(g.L[0], g.L[1]);
        }
    }
    // ... and there, particles whose first free path exceeds 1000 cell widths are started first (so
    // that their walks run beside the rest instead of after it): a particle qualifies when the top
    // 53 bits of its free-flight key (u = that x 2^-53, flight -lambda ln(1 - u)) reach
    // floor(2^53 (1 - exp(-P / lambda_m))) + 1 for its mode, an integer test both the list and the
    // trace make alike
    if (h.lattice) {
        const double P = 1000.0 * std::max(g.L[0], g.L[1]);
        t->prio_thr.assign((size_t)M, (uint64_t)1 << 53);
        for (int m = 0; m < M; ++m) {
            const double lam = t->v[(size_t)m] * t->tau[(size_t)m];
            if (!(lam > 0.0)) continue;
            const double q = -std::expm1(-P / lam);          // probability mass below the cut
            if (q < 1.0) t->prio_thr[(size_t)m] = (uint64_t)std::floor(q * 0x1p53) + 1;
        }
        t->info.tally_bytes = ((t->info.tally_bytes + 255) & ~int64_t(255)) + 8 * (int64_t)MCBTE_PRIO_CAP;
    }
    h.max_events = pr.max_events;
    h.n_bins = n_bins;
    h.two = t->two ? 1 : 0;
    h.t_max = pr.transient ? pr.t_max : 0.0;
    h.last_ic = last_ic;
    h.last_wall = last_wall;
    h.last_rel = last_rel;
    h.last_src = last_src;
    for (int a = 0; a < 3; ++a) {
        const bool on = pr.n_heat > 0 && !g.unbounded[a];
        h.heat_lo[a] = on ? pr.heat_lo[a] : 0.0;
        h.heat_w[a] = on ? pr.heat_hi[a] - pr.heat_lo[a] : 1.0;
        h.heat_lo32[a] = (float)h.heat_lo[a];
        h.heat_w32[a] = (float)h.heat_w[a];
    }
    DevGeom& dg = h.g;
    // per-row specularity: a boundary with a table of the problem reads it; a boundary with a cutoff
    // frequency reads the table of its special case (1 below the cutoff, d above it); equal tables
    // are stored once.  Returns 1 + the stored table, 0 for a constant d.
    auto spec_tab = [&](int32_t user, double d, double wc) -> int32_t {
        if (user <= 0 && !(wc > 0.0)) return 0;
        std::vector<double> row((size_t)M);
        for (int m = 0; m < M; ++m)
            row[(size_t)m] = user > 0 ? pr.spec_table[(int64_t)(user - 1) * M + m] : (t->omega[(size_t)m] < wc ? 1.0 : d);
        const size_t n_tab = t->spec_d.size() / (size_t)M;
        for (size_t k = 0; k < n_tab; ++k)
            if (std::equal(row.begin(), row.end(), t->spec_d.begin() + (ptrdiff_t)(k * (size_t)M))) return (int32_t)k + 1;
        t->spec_d.insert(t->spec_d.end(), row.begin(), row.end());
        t->spec_w = true;
        return (int32_t)n_tab + 1;
    };
    for (int a = 0; a < 3; ++a) {
        dg.L[a] = g.unbounded[a] ? 1.0 : g.L[a];
        dg.L32[a] = (float)dg.L[a];
        dg.unb[a] = g.unbounded[a] ? 1 : 0;
        dg.ngrad[a] = gnorm > 0.0 ? -g.gradT[a] / gnorm : 0.0;
        dg.ngrad32[a] = (float)dg.ngrad[a];
    }
    for (int i = 0; i < 6; ++i) {
        dg.face_type[i] = g.unbounded[kFaceAxis[i]] ? 0 : g.face[i].type;
        const double d = g.face[i].type == MCBTE_ADIABATIC ? g.face[i].data[0] : 0.0;
        dg.face_spec[i] = d;
        dg.face_thr[i] = (d > 0.0 && d < 1.0) ? (uint64_t)(d * kTwo64) : 0;
        dg.face_code[0] |= ((uint32_t)dg.face_type[i] | surf_class<float>(d) << 2) << (4 * i);
        dg.face_code[1] |= ((uint32_t)dg.face_type[i] | surf_class<double>(d) << 2) << (4 * i);
        dg.face_tab[i] = dg.face_type[i] == MCBTE_ADIABATIC ? spec_tab(g.face[i].spec_table, d, g.face[i].data[1]) : 0;
    }
    for (int a = 0; a < 3; ++a) dg.unb_mask |= (uint32_t)dg.unb[a] << a;
    dg.n_pores = g.n_pores;
    for (int c = 0; c < g.n_pores; ++c) {
        const mcbte_pore& p = g.pore[c];
        dg.pore_cx[c] = p.cx;
        dg.pore_cy[c] = p.cy;
        dg.pore_r[c] = p.r;
        dg.pore_cx32[c] = (float)p.cx;
        dg.pore_cy32[c] = (float)p.cy;
        dg.pore_r32[c] = (float)p.r;
        dg.pore_spec[c] = p.specularity;
        dg.pore_thr[c] = (p.specularity > 0.0 && p.specularity < 1.0) ? (uint64_t)(p.specularity * kTwo64) : 0;
        dg.pore_id[c] = p.id;
        dg.pore32[c] = DevPore32{(float)p.cx, (float)p.cy, (float)p.r, p.id};
        dg.pore64[c] = DevPore64{p.cx, p.cy, p.r, p.id, 0};
        dg.pore_cls[0] |= surf_class<float>(p.specularity) << (2 * c);
        dg.pore_cls[1] |= surf_class<double>(p.specularity) << (2 * c);
        dg.pore_tab[c] = spec_tab(p.spec_table, p.specularity, p.spec_omega);
    }
    dg.n_walls = g.n_walls;
    for (int k = 0; k < g.n_walls; ++k) {
        const mcbte_wall& w = g.wall[k];
        const double nn = std::sqrt(w.nx * w.nx + w.ny * w.ny);
        dg.wall_x1[k] = w.x1;
        dg.wall_y1[k] = w.y1;
        dg.wall_x2[k] = w.x2;
        dg.wall_y2[k] = w.y2;
        dg.wall_nx[k] = w.nx / nn;
        dg.wall_ny[k] = w.ny / nn;
        const double v6[6] = {w.x1, w.y1, w.x2, w.y2, dg.wall_nx[k], dg.wall_ny[k]};
        for (int q = 0; q < 6; ++q) dg.wall32[k][q] = (float)v6[q];
        dg.wall_id[k] = w.id;
        dg.wall_type[k] = w.type;
        const double d = w.type == MCBTE_ADIABATIC ? w.data : 0.0;
        dg.wall_cls[0] |= surf_class<float>(d) << (2 * k);
        dg.wall_cls[1] |= surf_class<double>(d) << (2 * k);
        dg.wall_thr[k] = (d > 0.0 && d < 1.0) ? (uint64_t)(d * kTwo64) : 0;
        dg.wall_tab[k] = w.type == MCBTE_ADIABATIC ? spec_tab(w.spec_table, d, w.spec_omega) : 0;
        dg.wall_loop_end[k] = -1;
    }
    // closed loops of walls: runs of walls each starting where the previous one ends, the last
    // ending where the first starts
    for (int k = 0; k < g.n_walls;) {
        int j = k;
        while (j + 1 < g.n_walls && g.wall[j + 1].x1 == g.wall[j].x2 && g.wall[j + 1].y1 == g.wall[j].y2) ++j;
        if (g.wall[j].x2 == g.wall[k].x1 && g.wall[j].y2 == g.wall[k].y1) dg.wall_loop_end[k] = j;
        k = j + 1;
    }
    if (g.n_walls > 0) t->walls = true;
    h.spec_w = t->spec_w ? 1 : 0;
    t->spec_thr.assign(t->spec_d.size(), 0);
    t->spec_cls.assign(t->spec_d.size(), 0);
    for (size_t i = 0; i < t->spec_d.size(); ++i) {
        const double d = t->spec_d[i];
        t->spec_thr[i] = (d > 0.0 && d < 1.0) ? (uint64_t)(d * kTwo64) : 0;
        t->spec_cls[i] = (uint8_t)(surf_class<float>(d) | surf_class<double>(d) << 2);
    }
    DevDet& dd = h.det;
    int nc = 0;
    for (int q = 0; q < 4; ++q) {
        dd.slot[q] = -1;
        dd.comp[q] = 0;
    }
    for (int q = 0; q < 4; ++q)
        if (dt.mask & (1 << q)) { dd.slot[q] = nc; dd.comp[nc] = q; ++nc; }
    dd.ncomp = nc;
    dd.mask = dt.mask;
    dd.n_cols = (int32_t)n_cols;
    dd.n_cells = n_cells;
    for (int a = 0; a < 3; ++a) {
        dd.n[a] = dt.n[a];
        dd.lo[a] = dt.lo[a];
        dd.hi[a] = dt.hi[a];
        dd.w[a] = dt.n[a] > 0 ? (dt.hi[a] - dt.lo[a]) / (double)dt.n[a] : 1.0;
        dd.lo32[a] = (float)dt.lo[a];
        dd.hi32[a] = (float)dt.hi[a];
        dd.inv_w32[a] = (float)(1.0 / dd.w[a]);
    }

    if (device >= 0) {
        DeviceGuard guard(device);
        if (!guard.ok) { delete t; return MCBTE_EHIP; }
        if (hipDeviceGetAttribute(&t->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
            hipDeviceGetAttribute(&t->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) {
            delete t;
            return MCBTE_EHIP;
        }
        int optin = 0;   // the LDS a kernel may use after raising its dynamic-LDS limit
        if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, device) == hipSuccess &&
            optin > t->max_lds)
            t->max_lds = optin;
        // one allocation, 256-byte aligned pieces
        std::vector<std::pair<const void*, size_t>> parts;
        auto add = [&](const void* src, size_t bytes) { parts.emplace_back(src, bytes); };
        std::vector<float> v32(M), tau32(M), tau2_32(M), tm32(t->t_meas.size());
        for (int m = 0; m < M; ++m) {
            v32[m] = (float)t->v[m];
            tau32[m] = (float)t->tau[m];
            tau2_32[m] = (float)t->tau2[m];
        }
        for (size_t k = 0; k < t->t_meas.size(); ++k) tm32[k] = (float)t->t_meas[k];
        add(nullptr, sizeof(DevTab));
        add(t->v.data(), 8 * (size_t)M);
        add(t->tau.data(), 8 * (size_t)M);
        add(v32.data(), 4 * (size_t)M);
        add(tau32.data(), 4 * (size_t)M);
        add(t->thr_ic.data(), 8 * (size_t)M);
        add(t->thr_wall.data(), 8 * (size_t)M);
        add(t->thr_rel.data(), 8 * (size_t)M);
        add(t->thr_src.data(), 8 * (size_t)S);
        add(t->src_kind.data(), 4 * (size_t)S);
        add(t->src_ref.data(), 4 * (size_t)S);
        add(t->src_sign.data(), 4 * (size_t)S);
        add(t->ic_edges.data(), 8 * t->ic_edges.size());
        add(t->t_meas.data(), 8 * t->t_meas.size());
        add(tm32.data(), 4 * tm32.size());
        add(t->bin_of.data(), 4 * (size_t)M);
        // guide of the relaxation draw: entry b is the number of thresholds <= b 2^52 and the last
        // entry is M, so that the draw for a key K with top 12 bits b lies between entries b and
        // b + 1 (the threshold search then only runs between them; a launch stages every
        // 2^(12 - bits)-th entry, a guide of the key's top bits); tables of more than 65535 rows
        // search the whole table
        const int n_guide = (1 << MCBTE_GUIDE_BITS) + 1;
        auto make_guide = [&](const std::vector<uint64_t>& thr) {
            std::vector<uint16_t> gd(n_guide, 0u);
            if (M <= 65535) {
                for (int b = 0; b < n_guide - 1; ++b)
                    gd[b] = (uint16_t)(std::upper_bound(thr.begin(), thr.end(), (uint64_t)b << (64 - MCBTE_GUIDE_BITS)) -
                                       thr.begin());
                gd[n_guide - 1] = (uint16_t)M;
            }
            return gd;
        };
        const std::vector<uint16_t> guide = make_guide(t->thr_rel);
        add(guide.data(), 2 * (size_t)n_guide);
        add(t->tau2.data(), 8 * (size_t)M);
        add(tau2_32.data(), 4 * (size_t)M);
        add(t->omega.data(), 8 * (size_t)M);
        add(t->prio_thr.data(), 8 * t->prio_thr.size());
        add(t->spec_thr.data(), 8 * t->spec_thr.size());
        add(t->spec_cls.data(), t->spec_cls.size());
        add(t->heat_t.data(), 8 * t->heat_t.size());
        std::vector<float> tet32(t->heat_tet.size());
        for (size_t i = 0; i < tet32.size(); ++i) tet32[i] = (float)t->heat_tet[i];
        add(t->heat_tet.data(), 8 * t->heat_tet.size());
        add(tet32.data(), 4 * tet32.size());
        add(t->thr_tet.data(), 8 * t->thr_tet.size());
        // the emission draws' guides (the same form as the relaxation draw's)
        const std::vector<uint16_t> wall_guide = make_guide(t->thr_wall), ic_guide = make_guide(t->thr_ic);
        add(wall_guide.data(), 2 * (size_t)n_guide);
        add(ic_guide.data(), 2 * (size_t)n_guide);
        // the measurement times' guide (snapshot ranges of transient segments)
        std::vector<uint16_t> tm_guide;
        const bool tm_guided = pr.transient && !t->t_meas.empty() && t->t_meas.size() <= 65535;
        if (tm_guided) {
            tm_guide.resize(257);
            for (int b = 0; b < 256; ++b)
                tm_guide[b] = (uint16_t)(std::lower_bound(t->t_meas.begin(), t->t_meas.end(), b * (pr.t_max / 256.0)) -
                                         t->t_meas.begin());
            tm_guide[256] = (uint16_t)t->t_meas.size();
        }
        add(tm_guide.data(), 2 * tm_guide.size());
        size_t total = 0;
        std::vector<size_t> off;
        for (auto& p : parts) {
            off.push_back(total);
            total += (p.second + 255) & ~size_t(255);
        }
        if (hipMalloc(&t->d_mem, total + 256) != hipSuccess) {
            t->d_mem = nullptr;
            delete t;
            return MCBTE_ENOMEM;
        }
        unsigned char* base = (unsigned char*)t->d_mem;
        auto dptr = [&](int i) { return (void*)(base + off[i]); };
        h.v64 = (const double*)dptr(1);
        h.tau64 = (const double*)dptr(2);
        h.v32 = (const float*)dptr(3);
        h.tau32 = (const float*)dptr(4);
        h.thr_ic = (const uint64_t*)dptr(5);
        h.thr_wall = (const uint64_t*)dptr(6);
        h.thr_rel = (const uint64_t*)dptr(7);
        h.thr_src = (const uint64_t*)dptr(8);
        h.src_kind = (const int32_t*)dptr(9);
        h.src_ref = (const int32_t*)dptr(10);
        h.src_sign = (const int32_t*)dptr(11);
        h.ic_edges = (const double*)dptr(12);
        h.t_meas64 = (const double*)dptr(13);
        h.t_meas32 = (const float*)dptr(14);
        h.bin_of = (const int32_t*)dptr(15);
        h.rel_guide = M <= 65535 ? (const uint16_t*)dptr(16) : nullptr;
        h.tau2_64 = (const double*)dptr(17);
        h.tau2_32 = (const float*)dptr(18);
        h.omega64 = (const double*)dptr(19);
        h.prio_thr = t->prio_thr.empty() ? nullptr : (const uint64_t*)dptr(20);
        h.prio_list_off = t->prio_thr.empty() ? 0 : t->info.tally_bytes - 8 * (int64_t)MCBTE_PRIO_CAP;
        h.spec_thr = t->spec_thr.empty() ? nullptr : (const uint64_t*)dptr(21);
        h.spec_cls = t->spec_cls.empty() ? nullptr : (const uint8_t*)dptr(22);
        h.heat_t = t->heat_t.empty() ? nullptr : (const double*)dptr(23);
        h.n_heat_tet = (int32_t)(t->heat_tet.size() / 12);
        h.heat_tet64 = h.n_heat_tet ? (const double*)dptr(24) : nullptr;
        h.heat_tet32 = h.n_heat_tet ? (const float*)dptr(25) : nullptr;
        h.thr_tet = h.n_heat_tet ? (const uint64_t*)dptr(26) : nullptr;
        h.last_tet = t->last_tet;
        h.wall_guide = M <= 65535 ? (const uint16_t*)dptr(27) : nullptr;
        h.ic_guide = M <= 65535 ? (const uint16_t*)dptr(28) : nullptr;
        h.tm_guide = tm_guided ? (const uint16_t*)dptr(29) : nullptr;
        h.tm_gs64 = tm_guided ? 256.0 / pr.t_max : 0.0;
        h.tm_gs32 = (float)h.tm_gs64;
        parts[0].first = &h;
        for (size_t i = 0; i < parts.size(); ++i) {
            if (parts[i].second == 0) continue;
            if (hipMemcpy(dptr((int)i), parts[i].first, parts[i].second, hipMemcpyHostToDevice) != hipSuccess) {
                mcbte_free_tables(t);
                return MCBTE_EHIP;
            }
        }
        t->d_tab = (DevTab*)dptr(0);
    }
    *out = t;
    return MCBTE_OK;
}

int mcbte_table_info(const mcbte_tables* t, mcbte_info* info)
{
    if (!t || !info) return MCBTE_EINVAL;
    *info = t->info;
    return MCBTE_OK;
}

int mcbte_table_export(const mcbte_tables* t, int32_t which, void* out, int64_t n)
{
    if (!t || !out) return MCBTE_EINVAL;
    auto put = [&](const void* src, int64_t count, size_t elem) {
        if (n < count) return MCBTE_ESIZE;
        std::memcpy(out, src, (size_t)count * elem);
        return MCBTE_OK;
    };
    const int64_t M = t->info.n_modes, S = t->info.n_sources;
    switch (which) {
    case 0: return put(t->C.data(), M, 8);
    case 1: return put(t->thr_ic.data(), M, 8);
    case 2: return put(t->thr_wall.data(), M, 8);
    case 3: return put(t->thr_rel.data(), M, 8);
    case 4: return put(t->src_E.data(), S, 8);
    case 5: return put(t->thr_src.data(), S, 8);
    case 6: return put(t->src_sign.data(), S, 4);
    default: return MCBTE_EINVAL;
    }
}

int64_t mcbte_state_bytes(int32_t precision, int64_t cap)
{
    if ((precision != 32 && precision != 64) || cap < 0) return MCBTE_EINVAL;
    const int64_t rb = precision / 8;
    const int64_t fb = (cap * rb + 255) & ~int64_t(255);
    const int64_t ib = (cap * 4 + 255) & ~int64_t(255);
    return 9 * fb + 7 * ib;
}

int mcbte_emit(const mcbte_tables* t, const mcbte_run* run, int64_t first_pid, int64_t n, void* state,
               int64_t capacity, void* stream)
{
    if (!t || !run || n < 0 || first_pid < 0 || capacity < n || (n > 0 && !state)) return MCBTE_EINVAL;
    if (run->precision != 32 && run->precision != 64) return MCBTE_EINVAL;
    if (t->device < 0 || !t->d_tab) return MCBTE_ENODEV;
    DeviceGuard g(t->device);
    if (!g.ok) return MCBTE_EHIP;
    const hipError_t e = launch_emit(t->d_tab, run->precision, run->seed, run->instance, first_pid, n, state, capacity,
                                     (hipStream_t)stream);
    return e == hipSuccess ? MCBTE_OK : MCBTE_EHIP;
}

namespace {

struct LaunchPlan {
    int block, grid, refill;
    int tally_lds;
    int guide_bits;              // relaxation guide staged in LDS (0: none)
    int64_t lds_tab;
    int64_t lds_tmeas;           // offset of the staged measurement times (0: none)
    size_t lds;
};

int plan_launch(const mcbte_tables* const* ts, int n_inst, const mcbte_run* run, int mode, int ft, LaunchPlan& lp)
{
    const mcbte_tables* t0 = ts[0];
    const int prec = run->precision;
    const int rb = prec / 8;
    int64_t lds_rows = 0, lds_tally = 0;
    bool guided = true;
    for (int i = 0; i < n_inst; ++i) {
        const int64_t M = ts[i]->info.n_modes;
        lds_rows = std::max<int64_t>(lds_rows, ((M * 8 + 15) & ~int64_t(15)) + 2 * ((M * rb + 15) & ~int64_t(15)));
        lds_tally = std::max<int64_t>(lds_tally, ts[i]->info.n_cells * ts[i]->info.n_cols *
                                                     (int64_t)ts[i]->host_view.det.ncomp * 8);
        guided = guided && ts[i]->info.n_modes <= 65535;
    }
    const int min_bits = guided ? MCBTE_GUIDE_MIN_BITS : 0;
    if (lds_rows + guide_lds_bytes(min_bits) > MCBTE_LDS_TABLE_BYTES ||
        lds_rows + guide_lds_bytes(min_bits) > t0->max_lds)
        return MCBTE_EINVAL;
    const int max_block = (ft & FT_WIDE) ? 1024 : 256;
    lp.block = run->block > 0 ? run->block : max_block;
    if (lp.block % 64 != 0 || lp.block > max_block) return MCBTE_EINVAL;
    lp.refill = run->refill > 0 ? run->refill : 4;
    // the LDS layout for a guide of `bits`: tables, guide, tallies, measurement times
    auto layout = [&](int bits) -> bool {
        const int64_t lds_tab = lds_rows + guide_lds_bytes(bits);
        lp.guide_bits = bits;
        lp.lds_tab = lds_tab;
        if (ft & FT_WIDE) {             // wide workgroups: the FP32 tally fills the LDS, tables stay in HBM
            lp.guide_bits = 0;        // wide workgroups: the FP32 tally fills the LDS, tables stay in HBM
            lp.lds_tab = 0;
            lp.tally_lds = 1;
            lp.lds = (size_t)(lds_tally / 2);
            if ((int64_t)lp.lds > t0->max_lds) return false;
        } else if (mode >= 2 && mode <= 4) {   // sensitivity replay: the per-bin sums take the place of the tallies
            const int64_t bins = 8 * t0->info.n_bins;
            if (lds_tab + bins > t0->max_lds) return false;
            lp.tally_lds = 0;
            lp.lds = (size_t)(lds_tab + bins);
        } else {
            lp.tally_lds = (lds_tally <= MCBTE_LDS_TALLY_BYTES && lds_tab + lds_tally <= t0->max_lds) ? 1 : 0;
            lp.lds = (size_t)(lds_tab + (lp.tally_lds ? lds_tally : 0));
        }
        // a solo transient trace also stages its measurement times after the tally where they fit
        lp.lds_tmeas = 0;
        if (mode == 0 && n_inst == 1 && t0->host_view.tally_kind == TALLY_TRANSIENT) {
            const int64_t off = ((int64_t)lp.lds + 15) & ~int64_t(15);
            const int64_t end = off + (int64_t)t0->host_view.n_times * rb;
            if (off > 0 && end <= t0->max_lds) {
                lp.lds_tmeas = off;
                lp.lds = (size_t)end;
            }
        }
        return true;
    };
    if (!layout(min_bits)) return MCBTE_EINVAL;
    // the finest guide that leaves as many workgroups per compute unit as the coarsest (a finer
    // guide shortens the relaxation draw's search, which otherwise idles most lanes of a wave
    // while a few search the crowded stretches of the table)
    if (guided && !(ft & FT_WIDE)) {
        const LaunchPlan coarse = lp;
        const int occ0 = trace_occupancy(mode, prec, t0->host_view.tally_kind, ft, lp.block, lp.lds);
        bool found = false;
        for (int bits = MCBTE_GUIDE_BITS; bits > min_bits && !found; --bits) {
            const bool same_tally = layout(bits) && lp.tally_lds == coarse.tally_lds &&
                                    (lp.lds_tmeas > 0) == (coarse.lds_tmeas > 0);
            found = same_tally && trace_occupancy(mode, prec, t0->host_view.tally_kind, ft, lp.block, lp.lds) >= occ0;
        }
        if (!found) lp = coarse;
    }
    if (run->grid > 0) {
        lp.grid = run->grid;
    } else {
        const int occ = trace_occupancy(mode, prec, t0->host_view.tally_kind, ft, lp.block, lp.lds);
        lp.grid = std::max(1, occ) * std::max(1, t0->n_cu);
    }
    return MCBTE_OK;
}

}  // namespace

int mcbte_trace(const mcbte_tables* t, const mcbte_run* run, int64_t first_pid, int64_t n, const void* state,
                void* tally, void* stream)
{
    if (!t || !run || !tally || n < 0 || first_pid < 0) return MCBTE_EINVAL;
    if (run->precision != 32 && run->precision != 64) return MCBTE_EINVAL;
    if ((run->flags & ~MCBTE_RUN_SEGMENTS) != 0 || run->reserved != 0) return MCBTE_EINVAL;
    if (run->event_log && (run->log_stride < 2 || run->n_log < 0)) return MCBTE_EINVAL;
    if (t->device < 0 || !t->d_tab) return MCBTE_ENODEV;
    if (n == 0) return MCBTE_OK;
    DeviceGuard g(t->device);
    if (!g.ok) return MCBTE_EHIP;
    LaunchPlan lp;
    // the plain kernel has neither a state buffer nor an event log compiled in; an FP32 trace whose
    // FP64 tally is too large for the LDS copy but whose FP32 tally fits runs wide workgroups
    // (FP32 steady traces from pre-emitted states have a kernel without the event log compiled in)
    int ft = (state || run->event_log) ? (FT_STATE | FT_LOG) : 0;
    if (state && !run->event_log && run->precision == 32 && t->host_view.tally_kind == TALLY_STEADY_ONE) ft = FT_STATE;
    if (ft == 0 && run->precision == 32) {
        const int64_t t64 = t->info.n_cells * t->info.n_cols * (int64_t)t->host_view.det.ncomp * 8;
        const int64_t M = t->info.n_modes;
        const int64_t tab = ((M * 8 + 15) & ~int64_t(15)) + 2 * ((M * 4 + 15) & ~int64_t(15)) +
                            guide_lds_bytes(M <= 65535 ? MCBTE_GUIDE_MIN_BITS : 0);
        const bool fits64 = t64 <= MCBTE_LDS_TALLY_BYTES && tab + t64 <= t->max_lds;
        if (!fits64 && t64 / 2 <= t->max_lds) ft = FT_WIDE;
    }
    // FP64 film-like problems: the kernel with the exact cooperative bouncing
    if (run->precision == 64 && t->host_view.coop_axis >= 0) ft |= FT_COOP;
    if (!t->two && !t->spec_w && !t->walls && !t->ext_film) ft |= FT_PLAIN;   // the kernel without the extended physics
    // FP32 pore lattices: long free paths walked from pore to pore by the wave
    if (run->precision == 32 && t->host_view.lattice && !(ft & (FT_STATE | FT_LOG | FT_WIDE)) &&
        !(run->flags & MCBTE_RUN_SEGMENTS))
        ft |= FT_LATTICE;
    const int rc = plan_launch(&t, 1, run, 0, ft, lp);
    if (rc != MCBTE_OK) return rc;
    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.tabs = t->d_tab;
    a.n_inst = 1;
    a.refill = lp.refill;
    a.seed = run->seed;
    a.inst0 = run->instance;
    a.log_stride = run->event_log ? run->log_stride : 2;
    a.first_pid = first_pid;
    a.n = n;
    a.state = state;
    a.capacity = n;
    a.tally = (unsigned char*)tally;
    a.event_log = run->event_log;
    a.n_log = run->event_log ? run->n_log : 0;
    a.tally_lds = lp.tally_lds;
    a.lds_tab_bytes = (int32_t)lp.lds_tab;
    a.guide_bits = lp.guide_bits;
    a.lds_tmeas = (int32_t)lp.lds_tmeas;
    a.particle_F = run->particle_F;
    const hipError_t e = launch_trace(a, 0, run->precision, t->host_view.tally_kind, ft, lp.block, lp.grid, lp.lds,
                                      (hipStream_t)stream);
    return e == hipSuccess ? MCBTE_OK : MCBTE_EHIP;
}

int64_t mcbte_batch_queue_bytes(int32_t n_inst)
{
    if (n_inst < 1) return MCBTE_EINVAL;
    auto al = [](int64_t b) { return (b + 255) / 256 * 256; };
    const int64_t n = n_inst;
    // queue counter | tally pointers | particle counts | chunk starts | instance ids | tables
    return 256 + al(8 * n) + al(8 * n) + al(8 * (n + 1)) + al(4 * n) + al((int64_t)sizeof(DevTab) * n);
}

int mcbte_trace_batch(const mcbte_tables* const* ts, int32_t n_inst, const int64_t* n_particles,
                      const uint32_t* instance_ids, void* const* tallies, const mcbte_run* run, void* queue,
                      void* stream)
{
    if (!ts || n_inst < 1 || !n_particles || !instance_ids || !tallies || !run || !queue) return MCBTE_EINVAL;
    if (run->precision != 32 && run->precision != 64) return MCBTE_EINVAL;
    if ((run->flags & ~MCBTE_RUN_SEGMENTS) != 0 || run->reserved != 0) return MCBTE_EINVAL;
    if (run->event_log) return MCBTE_EINVAL;
    const mcbte_tables* t0 = ts[0];
    if (!t0 || t0->device < 0) return MCBTE_ENODEV;
    for (int i = 0; i < n_inst; ++i) {
        if (!ts[i] || !tallies[i] || n_particles[i] < 0) return MCBTE_EINVAL;
        if (ts[i]->device != t0->device || !ts[i]->d_tab) return MCBTE_ENODEV;
        if (ts[i]->host_view.tally_kind != t0->host_view.tally_kind) return MCBTE_EINVAL;
    }
    DeviceGuard g(t0->device);
    if (!g.ok) return MCBTE_EHIP;
    LaunchPlan lp;
    if (run->particle_F) return MCBTE_EINVAL;
    // the batched kernel without the extended physics unless some instance needs it
    int ft = FT_PLAIN;
    for (int i = 0; i < n_inst; ++i)
        if (ts[i]->two || ts[i]->spec_w || ts[i]->walls || ts[i]->ext_film) ft = 0;
    int rc = plan_launch(ts, n_inst, run, 1, ft, lp);
    if (rc != MCBTE_OK) return rc;
    // chunking: items of chunk_size particles, instance-major
    const int64_t chunk = 8192;
    std::vector<int64_t> cstart(n_inst + 1, 0);
    for (int i = 0; i < n_inst; ++i) cstart[i + 1] = cstart[i] + (n_particles[i] + chunk - 1) / chunk;
    // pack the small device-side arrays into the caller's queue buffer (one host->device copy)
    const int64_t qbytes = mcbte_batch_queue_bytes(n_inst);
    std::vector<unsigned char> host((size_t)qbytes, 0);
    size_t off = 256;
    auto place = [&](const void* src, size_t bytes) {
        const size_t at = off;
        std::memcpy(host.data() + at, src, bytes);
        off = (off + bytes + 255) & ~size_t(255);
        return at;
    };
    std::vector<unsigned char*> tp(n_inst);
    for (int i = 0; i < n_inst; ++i) tp[i] = (unsigned char*)tallies[i];
    const size_t o_tp = place(tp.data(), 8 * (size_t)n_inst);
    const size_t o_n = place(n_particles, 8 * (size_t)n_inst);
    const size_t o_cs = place(cstart.data(), 8 * (size_t)(n_inst + 1));
    const size_t o_id = place(instance_ids, 4 * (size_t)n_inst);
    std::vector<DevTab> tabs(n_inst);
    for (int i = 0; i < n_inst; ++i) tabs[i] = ts[i]->host_view;
    const size_t o_tab = place(tabs.data(), sizeof(DevTab) * (size_t)n_inst);
    if ((int64_t)off > qbytes) return MCBTE_ESIZE;
    unsigned char* qd = (unsigned char*)queue;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(qd, host.data(), (size_t)off, hipMemcpyHostToDevice, s) != hipSuccess) return MCBTE_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return MCBTE_EHIP;   // `host` is a local buffer
    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.tabs = (const DevTab*)(qd + o_tab);
    a.n_inst = n_inst;
    a.refill = lp.refill;
    a.seed = run->seed;
    a.inst_ids = (const uint32_t*)(qd + o_id);
    a.log_stride = 2;
    a.tallies = (unsigned char* const*)(qd + o_tp);
    a.inst_n = (const int64_t*)(qd + o_n);
    a.chunk_start = (const int64_t*)(qd + o_cs);
    a.chunk_size = chunk;
    a.queue = (unsigned long long*)qd;
    a.n_chunks = cstart[n_inst];
    a.tally_lds = lp.tally_lds;
    a.lds_tab_bytes = (int32_t)lp.lds_tab;
    a.guide_bits = lp.guide_bits;
    const hipError_t e = launch_trace(a, 1, run->precision, t0->host_view.tally_kind, ft, lp.block, lp.grid, lp.lds, s);
    return e == hipSuccess ? MCBTE_OK : MCBTE_EHIP;
}

static_assert(MCBTE_STATIC_MAX_INSTANCES == MCBTE_STATIC_INSTANCES, "static batch capacity");

int mcbte_trace_batch_static(const mcbte_tables* const* ts, int32_t n_inst, const int64_t* n_particles,
                             const uint32_t* instance_ids, void* const* tallies, const mcbte_run* run, void* stream)
{
    if (!ts || n_inst < 1 || !n_particles || !instance_ids || !tallies || !run) return MCBTE_EINVAL;
    if (n_inst > MCBTE_STATIC_MAX_INSTANCES) return MCBTE_ELIMIT;
    if (run->precision != 32 && run->precision != 64) return MCBTE_EINVAL;
    if ((run->flags & ~MCBTE_RUN_SEGMENTS) != 0 || run->reserved != 0) return MCBTE_EINVAL;
    if (run->event_log || run->particle_F) return MCBTE_EINVAL;
    const mcbte_tables* t0 = ts[0];
    if (!t0 || t0->device < 0) return MCBTE_ENODEV;
    for (int i = 0; i < n_inst; ++i) {
        if (!ts[i] || !tallies[i] || n_particles[i] < 0) return MCBTE_EINVAL;
        if (ts[i]->device != t0->device || !ts[i]->d_tab) return MCBTE_ENODEV;
        if (ts[i]->host_view.tally_kind != t0->host_view.tally_kind) return MCBTE_EINVAL;
    }
    DeviceGuard g(t0->device);
    if (!g.ok) return MCBTE_EHIP;
    unsigned char* q = nullptr;                  // this device's static work queue
    if (static_queue(t0->device, &q) != hipSuccess) return MCBTE_EHIP;
    if (queue_layout(n_inst).end > static_queue_bytes()) return MCBTE_ELIMIT;
    int ft = FT_PLAIN;
    for (int i = 0; i < n_inst; ++i)
        if (ts[i]->two || ts[i]->spec_w || ts[i]->walls || ts[i]->ext_film) ft = 0;
    LaunchPlan lp;
    int rc = plan_launch(ts, n_inst, run, 1, ft, lp);
    if (rc != MCBTE_OK) return rc;
    // the work table travels as the setup kernel's arguments (no host staging, no copy, no sync)
    const int64_t chunk = 8192;
    BatchSetupArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.n_inst = n_inst;
    sa.cstart[0] = 0;
    for (int i = 0; i < n_inst; ++i) {
        sa.tab[i] = ts[i]->d_tab;
        sa.tally[i] = (unsigned char*)tallies[i];
        sa.n[i] = n_particles[i];
        sa.id[i] = instance_ids[i];
        sa.cstart[i + 1] = sa.cstart[i] + (n_particles[i] + chunk - 1) / chunk;
    }
    hipStream_t s = (hipStream_t)stream;
    if (launch_batch_setup(sa, q, s) != hipSuccess) return MCBTE_EHIP;
    const QueueLayout L = queue_layout(n_inst);
    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.tabs = (const DevTab*)(q + L.o_tab);
    a.n_inst = n_inst;
    a.refill = lp.refill;
    a.seed = run->seed;
    a.inst_ids = (const uint32_t*)(q + L.o_id);
    a.log_stride = 2;
    a.tallies = (unsigned char* const*)(q + L.o_tp);
    a.inst_n = (const int64_t*)(q + L.o_n);
    a.chunk_start = (const int64_t*)(q + L.o_cs);
    a.chunk_size = chunk;
    a.queue = (unsigned long long*)q;
    a.n_chunks = sa.cstart[n_inst];
    a.tally_lds = lp.tally_lds;
    a.lds_tab_bytes = (int32_t)lp.lds_tab;
    a.guide_bits = lp.guide_bits;
    const hipError_t e = launch_trace(a, 1, run->precision, t0->host_view.tally_kind, ft, lp.block, lp.grid, lp.lds, s);
    return e == hipSuccess ? MCBTE_OK : MCBTE_EHIP;
}

int mcbte_autotune(const mcbte_tables* const* ts, int32_t n_inst, const int64_t* n_particles,
                   const uint32_t* instance_ids, void* const* tallies, void* queue, const mcbte_run* base,
                   int64_t n_probe, int32_t reps, mcbte_run* out, double* timings, int32_t n_timings, void* stream)
{
    if (!ts || n_inst < 1 || !n_particles || !tallies || !base || !out || n_probe < 1 || reps < 1) return MCBTE_EINVAL;
    if (base->event_log || base->particle_F) return MCBTE_EINVAL;
    if (n_inst > 1 && (!instance_ids || !queue)) return MCBTE_EINVAL;
    if (timings && n_timings < MCBTE_TUNE_CANDIDATES) return MCBTE_ESIZE;
    if (!ts[0] || ts[0]->device < 0) return MCBTE_ENODEV;
    int64_t total = 0;
    for (int i = 0; i < n_inst; ++i) {
        if (n_particles[i] < 0) return MCBTE_EINVAL;
        total += n_particles[i];
    }
    if (total == 0) return MCBTE_EINVAL;
    // the calibration problem: a prefix (one instance) or every count scaled alike (batched)
    std::vector<int64_t> np((size_t)n_inst);
    const double f = n_probe < total ? (double)n_probe / (double)total : 1.0;
    for (int i = 0; i < n_inst; ++i)
        np[(size_t)i] = n_particles[i] == 0 ? 0 : std::max<int64_t>(1, (int64_t)std::llround((double)n_particles[i] * f));
    DeviceGuard g(ts[0]->device);
    if (!g.ok) return MCBTE_EHIP;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return MCBTE_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MCBTE_EHIP;
    }
    int status = MCBTE_OK;
    int best = -1;
    double best_ms = 0.0;
    static const int kBlocks[6] = {64, 128, 192, 256, 512, 1024};
    for (int c = 0; c < MCBTE_TUNE_CANDIDATES && status == MCBTE_OK; ++c) {
        mcbte_run r = *base;
        r.block = kBlocks[c / 6];
        r.refill = 1 << (c % 6);
        auto go = [&]() {
            return n_inst == 1 ? mcbte_trace(ts[0], &r, 0, np[0], nullptr, tallies[0], stream)
                               : mcbte_trace_batch(ts, n_inst, np.data(), instance_ids, tallies, &r, queue, stream);
        };
        double t_c = INFINITY;
        int rc = go();                                   // warm-up
        if (rc == MCBTE_OK) {
            for (int k = 0; k < reps; ++k) {
                if (hipEventRecord(e0, s) != hipSuccess) { status = MCBTE_EHIP; break; }
                rc = go();
                if (rc != MCBTE_OK) break;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    status = MCBTE_EHIP;
                    break;
                }
                float ms = 0.0f;
                if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { status = MCBTE_EHIP; break; }
                t_c = std::min(t_c, (double)ms);
            }
        }
        if (rc == MCBTE_EHIP) status = MCBTE_EHIP;      // a launch failure ends the search
        if (rc != MCBTE_OK) t_c = INFINITY;              // a shape this problem cannot use
        if (timings) timings[c] = t_c;
        if (t_c < INFINITY && (best < 0 || t_c < best_ms)) {
            best = c;
            best_ms = t_c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != MCBTE_OK) return status;
    if (best < 0) return MCBTE_EINVAL;
    *out = *base;
    out->block = kBlocks[best / 6];
    out->refill = 1 << (best % 6);
    return MCBTE_OK;
}

static_assert(MCBTE_PATH_MAX == MCBTE_PATHWISE_MAX_FLIGHTS, "pathwise capacity");

int mcbte_adjoint(const mcbte_tables* t, const mcbte_run* run, int32_t estimator, double lambda_split,
                  int64_t first_pid, int64_t n, const double* particle_F, double* adj, void* stream)
{
    if (!t || !run || !particle_F || !adj || n < 0 || first_pid < 0) return MCBTE_EINVAL;
    if (run->precision != 32 && run->precision != 64) return MCBTE_EINVAL;
    if ((run->flags & ~MCBTE_RUN_SEGMENTS) != 0 || run->reserved != 0) return MCBTE_EINVAL;
    if (run->event_log) return MCBTE_EINVAL;
    if (estimator != MCBTE_SENS_SCORE && estimator != MCBTE_SENS_PATHWISE && estimator != MCBTE_SENS_LOCAL)
        return MCBTE_EINVAL;
    if (t->two) return MCBTE_EINVAL;       // the estimators differentiate the one-clock flight law
    if (t->spec_w || t->walls) return MCBTE_EINVAL;   // the replays know constant specularities, faces and pores
    if (t->device < 0 || !t->d_tab) return MCBTE_ENODEV;
    if (t->prob.transient) return MCBTE_EINVAL;
    if (estimator == MCBTE_SENS_PATHWISE &&
        (t->prob.n_scat_max < 1 || t->prob.n_scat_max > MCBTE_PATHWISE_MAX_FLIGHTS))
        return MCBTE_EINVAL;
    if (n == 0) return MCBTE_OK;
    DeviceGuard g(t->device);
    if (!g.ok) return MCBTE_EHIP;
    const int mode = estimator == MCBTE_SENS_PATHWISE ? 3 : (estimator == MCBTE_SENS_LOCAL ? 4 : 2);
    // FP64 film-like problems replay with the exact cooperative bouncing, as they trace; FP32 pore
    // lattices with the pore-to-pore walk, as they trace (the pathwise tangents need every segment)
    const bool lat = run->precision == 32 && t->host_view.lattice && !(run->flags & MCBTE_RUN_SEGMENTS);
    if (lat && mode == 3) return MCBTE_EINVAL;
    const int ft = ((run->precision == 64 && t->host_view.coop_axis >= 0) ? FT_COOP : 0) | FT_PLAIN |
                   (lat ? FT_LATTICE : 0);
    LaunchPlan lp;
    const int rc = plan_launch(&t, 1, run, mode, ft, lp);
    if (rc != MCBTE_OK) return rc;
    // the replay keeps its per-bin sums in LDS after the tables
    if ((int64_t)lp.lds < lp.lds_tab + 8 * t->info.n_bins) return MCBTE_EINVAL;
    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.tabs = t->d_tab;
    a.n_inst = 1;
    a.refill = lp.refill;
    a.seed = run->seed;
    a.inst0 = run->instance;
    a.log_stride = 2;
    a.first_pid = first_pid;
    a.n = n;
    a.capacity = n;
    a.lds_tab_bytes = (int32_t)lp.lds_tab;
    a.guide_bits = lp.guide_bits;
    a.particle_F = const_cast<double*>(particle_F);
    a.adj = adj;
    // local form: the split given, else the smallest bounded extent or pore diameter (every mode
    // of the unbounded bulk)
    double split = lambda_split;
    if (!(split > 0.0)) {
        split = INFINITY;
        for (int ax = 0; ax < 3; ++ax)
            if (!t->geom.unbounded[ax]) split = std::min(split, t->geom.L[ax]);
        for (int c = 0; c < t->geom.n_pores; ++c) split = std::min(split, 2.0 * t->geom.pore[c].r);
    }
    a.lambda_split = split;
    hipStream_t s = (hipStream_t)stream;
    // the work counter is the last word of the caller's buffer
    if (launch_zero_u64((unsigned long long*)(adj + t->info.n_bins + 2), s) != hipSuccess) return MCBTE_EHIP;
    const hipError_t e = launch_trace(a, mode, run->precision, t->host_view.tally_kind, ft, lp.block, lp.grid, lp.lds, s);
    return e == hipSuccess ? MCBTE_OK : MCBTE_EHIP;
}

int mcbte_adjoint_finalize(const mcbte_tables* t, const double* adj, int64_t n_particles, double* out, int64_t n_out,
                           void* stream)
{
    if (!t || !adj || !out || n_particles < 1) return MCBTE_EINVAL;
    if (t->device < 0) return MCBTE_ENODEV;
    const int64_t nb = t->info.n_bins;
    if (n_out < nb) return MCBTE_ESIZE;
    const double gs = t->geom.gradT[t->prob.score_axis];
    if (gs == 0.0 || t->prob.transient) return MCBTE_EINVAL;
    DeviceGuard g(t->device);
    if (!g.ok) return MCBTE_EHIP;
    std::vector<double> h((size_t)(nb + 2));
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(h.data(), adj, sizeof(double) * (size_t)(nb + 2), hipMemcpyDeviceToHost, s) != hipSuccess)
        return MCBTE_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return MCBTE_EHIP;
    // same normalisation as kappa: -E_tot / (V_solid gradT_s N) times the summed scores
    const double scale = -t->info.E_tot / (t->info.V_solid * gs * (double)n_particles);
    const double B = h[(size_t)nb];
    for (int64_t i = 0; i < nb; ++i) out[i] = scale * (h[(size_t)i] + t->P_bin[(size_t)i] * B);
    return h[(size_t)nb + 1] != 0.0 ? MCBTE_ERANGE : MCBTE_OK;
}

int mcbte_tally(const mcbte_tables* t, const void* tally, double* host_out, int64_t n_out, mcbte_result* res,
                void* stream)
{
    if (!t || !tally || !res) return MCBTE_EINVAL;
    if (t->device < 0) return MCBTE_ENODEV;
    const int64_t n_raw = t->info.n_cells * t->info.n_cols * 4;
    if (host_out && n_out < n_raw) return MCBTE_ESIZE;
    DeviceGuard g(t->device);
    if (!g.ok) return MCBTE_EHIP;
    std::vector<unsigned char> buf((size_t)t->info.tally_bytes);
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(buf.data(), tally, buf.size(), hipMemcpyDeviceToHost, s) != hipSuccess) return MCBTE_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return MCBTE_EHIP;
    std::memset(res, 0, sizeof(*res));
    std::memcpy(res->counts, buf.data(), sizeof(res->counts));
    std::memcpy(res->moments, buf.data() + 128, sizeof(res->moments));
    const double* raw = (const double*)(buf.data() + MCBTE_TALLY_HEADER_BYTES);
    const double n = (double)res->counts[MCBTE_CNT_PARTICLES];
    if (n <= 0.0) return MCBTE_OK;
    const mcbte_info& inf = t->info;
    normalize_raw(t, raw, n, host_out, &res->e_eff, &res->V_cell);
    if (!t->prob.transient && n > 1.0) {
        const double* m = res->moments;
        const double var_T = std::max(m[1] - m[0] * m[0] / n, 0.0) / (n - 1.0);
        const double var_q = std::max(m[3] - m[2] * m[2] / n, 0.0) / (n - 1.0);
        res->T_mean = inf.E_tot / (inf.C_tot * inf.V_solid) * m[0] / n;
        res->T_mean_sigma = inf.E_tot / (inf.C_tot * inf.V_solid) * std::sqrt(var_T / n);
        res->q_score = inf.E_tot / inf.V_solid * m[2] / n;
        res->q_score_sigma = inf.E_tot / inf.V_solid * std::sqrt(var_q / n);
        const double gs = t->geom.gradT[t->prob.score_axis];
        if (gs != 0.0) {
            res->kappa = -res->q_score / gs;
            res->kappa_sigma = res->q_score_sigma / std::fabs(gs);
            double box = 1.0;
            for (int a = 0; a < 3; ++a) box *= t->geom.unbounded[a] ? 1.0 : t->geom.L[a];
            res->kappa_cell_avg = res->kappa * inf.V_solid / box;
        }
    }
    return MCBTE_OK;
}

}  // extern "C"

namespace {

// Copy a tally buffer to the host and normalise it: T and q per cell and column in
// out[n_cells][n_cols][4]; returns the particles traced (0: none, out all zero).
int64_t finalize_host(const mcbte_tables* t, const void* tally, std::vector<double>& out, hipStream_t s, int& rc)
{
    rc = MCBTE_OK;
    std::vector<unsigned char> buf((size_t)t->info.tally_bytes);
    if (hipMemcpyAsync(buf.data(), tally, buf.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        rc = MCBTE_EHIP;
        return 0;
    }
    uint64_t counts[MCBTE_N_COUNTS];
    std::memcpy(counts, buf.data(), sizeof(counts));
    const int64_t n = (int64_t)counts[MCBTE_CNT_PARTICLES];
    const int64_t n_raw = t->info.n_cells * t->info.n_cols * 4;
    out.assign((size_t)n_raw, 0.0);
    if (n <= 0) return 0;
    normalize_raw(t, (const double*)(buf.data() + MCBTE_TALLY_HEADER_BYTES), (double)n, out.data(), nullptr,
                  nullptr);
    return n;
}

// particle-weighted mean of per-batch values x[b][k] (batch b traced n[b] particles) and its
// batch-mean standard error sqrt(sum_b n_b (x_b - mean)^2 / ((B - 1) N)), B the batches that traced
// particles (a batch without particles weighs nothing; NaN for fewer than two; with no particle at
// all the mean is 0)
void batch_mean(const std::vector<std::vector<double>>& x, const std::vector<int64_t>& n, double* mean, double* sigma,
                int64_t K)
{
    const size_t B = x.size();
    double N = 0.0;
    size_t used = 0;   // batches that traced particles
    for (size_t b = 0; b < B; ++b) {
        N += (double)n[b];
        used += n[b] > 0 ? 1u : 0u;
    }
    for (int64_t k = 0; k < K; ++k) {
        double m = 0.0;
        for (size_t b = 0; b < B; ++b) m += (double)n[b] * x[b][(size_t)k];
        m = N > 0.0 ? m / N : 0.0;
        if (mean) mean[k] = m;
        if (sigma) {
            if (used < 2) {
                sigma[k] = NAN;
            } else {
                double v = 0.0;
                for (size_t b = 0; b < B; ++b) v += (double)n[b] * (x[b][(size_t)k] - m) * (x[b][(size_t)k] - m);
                sigma[k] = std::sqrt(v / ((double)(used - 1) * N));
            }
        }
    }
}

}  // namespace

extern "C" {

int mcbte_tally_batches(const mcbte_tables* t, const void* const* tallies, int32_t n_tallies, double* host_mean,
                        double* host_sigma, int64_t n_out, void* stream)
{
    if (!t || !tallies || n_tallies < 1 || (!host_mean && !host_sigma)) return MCBTE_EINVAL;
    for (int b = 0; b < n_tallies; ++b)
        if (!tallies[b]) return MCBTE_EINVAL;
    const int64_t n_raw = t->info.n_cells * t->info.n_cols * 4;
    if (n_out < n_raw) return MCBTE_ESIZE;
    if (t->device < 0) return MCBTE_ENODEV;
    DeviceGuard g(t->device);
    if (!g.ok) return MCBTE_EHIP;
    std::vector<std::vector<double>> x((size_t)n_tallies);
    std::vector<int64_t> n((size_t)n_tallies);
    for (int b = 0; b < n_tallies; ++b) {
        int rc = MCBTE_OK;
        n[(size_t)b] = finalize_host(t, tallies[b], x[(size_t)b], (hipStream_t)stream, rc);
        if (rc != MCBTE_OK) return rc;
    }
    batch_mean(x, n, host_mean, host_sigma, n_raw);
    return MCBTE_OK;
}

int mcbte_kappa_cumulative(const mcbte_tables* t, const void* const* tallies, int32_t n_tallies, int32_t order,
                           double* keys, double* kappa_cum, double* kappa_cum_sigma, int64_t n_out, void* stream)
{
    if (!t || !tallies || n_tallies < 1 || !kappa_cum) return MCBTE_EINVAL;
    if (order != MCBTE_CUM_MFP && order != MCBTE_CUM_OMEGA) return MCBTE_EINVAL;
    if (t->prob.transient || t->host_view.tally_kind != TALLY_STEADY_ONE) return MCBTE_EINVAL;
    const int sa = t->prob.score_axis;
    const double gs = t->geom.gradT[sa];
    if (gs == 0.0 || !((t->det.mask >> (1 + sa)) & 1)) return MCBTE_EINVAL;
    const int64_t M = t->info.n_modes, NB = t->info.n_bins;
    const int64_t K = order == MCBTE_CUM_MFP ? M : NB;
    if (n_out < K) return MCBTE_ESIZE;
    for (int b = 0; b < n_tallies; ++b)
        if (!tallies[b]) return MCBTE_EINVAL;
    if (t->device < 0) return MCBTE_ENODEV;
    // the order: rows by mean free path v tau, or frequency bins by the lowest angular frequency of
    // their rows (a bin without rows last); ties by index
    std::vector<int64_t> idx((size_t)K);
    std::vector<double> key((size_t)K, INFINITY);
    if (order == MCBTE_CUM_MFP) {
        for (int64_t m = 0; m < M; ++m) {
            // two clocks combine by Matthiessen's rule into the row's relaxation time
            const double tm = t->tau[(size_t)m], t2 = t->tau2[(size_t)m];
            key[(size_t)m] = t->v[(size_t)m] * (t2 > 0.0 ? 1.0 / (1.0 / tm + 1.0 / t2) : tm);
        }
    } else {
        for (int64_t m = 0; m < M; ++m) {
            const int64_t b = t->bin_of[(size_t)m];
            key[(size_t)b] = std::min(key[(size_t)b], t->omega[(size_t)m]);
        }
    }
    for (int64_t k = 0; k < K; ++k) idx[(size_t)k] = k;
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return key[(size_t)a] < key[(size_t)b]; });
    DeviceGuard g(t->device);
    if (!g.ok) return MCBTE_EHIP;
    std::vector<std::vector<double>> cum((size_t)n_tallies, std::vector<double>((size_t)K, 0.0));
    std::vector<int64_t> n((size_t)n_tallies);
    std::vector<double> fin, part((size_t)K);
    for (int b = 0; b < n_tallies; ++b) {
        int rc = MCBTE_OK;
        n[(size_t)b] = finalize_host(t, tallies[b], fin, (hipStream_t)stream, rc);
        if (rc != MCBTE_OK) return rc;
        // each mode's (bin's) kappa, -q_score / gradT_score, then the prefix sums in the order
        std::fill(part.begin(), part.end(), 0.0);
        for (int64_t m = 0; m < M; ++m) {
            const double km = -fin[(size_t)(m * 4 + 1 + sa)] / gs;
            part[(size_t)(order == MCBTE_CUM_MFP ? m : t->bin_of[(size_t)m])] += km;
        }
        double acc = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            acc += part[(size_t)idx[(size_t)k]];
            cum[(size_t)b][(size_t)k] = acc;
        }
    }
    batch_mean(cum, n, kappa_cum, kappa_cum_sigma, K);
    if (keys)
        for (int64_t k = 0; k < K; ++k) keys[k] = key[(size_t)idx[(size_t)k]];
    return MCBTE_OK;
}

}  // extern "C"
