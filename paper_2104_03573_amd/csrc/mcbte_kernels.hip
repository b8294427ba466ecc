// HIP kernels (gfx950) of the deviational phonon Monte Carlo tracer.
//
// One engine, templated on the trajectory precision R (double: FP64 form, bit-for-bit the
// event sequence of the method's steps; float: FP32 form, tables built and tallies summed in
// FP64), drives three kernels:
//   k_emit        one lane per particle, writes the emitted state (section 3.2)
//   k_trace_solo  persistent lanes; a lane whose particle ended is refilled every `refill`
//                 flights from a global counter (wave ballot + prefix popcount, one atomic per
//                 wave); relaxation table, velocities and relaxation times staged in LDS;
//                 tallies privatised in LDS when they fit, then flushed with FP64 atomics.
//                 Where one lane's work would keep a wave waiting, the wave shares it: film
//                 bouncing 64 reflections at a time (coop_bounces, coop_exact), transient
//                 snapshots and sparse waves' detector-grid pieces 64 per pass (snap_wave,
//                 grid_wave); a wave's last lane walks periodic transfers and pore reflections
//                 in a lean loop (lone_chain)
//   k_trace_batch the same lanes over many problem instances: workgroups pull (instance,
//                 particle-chunk) items from a queue, re-stage the tables when the instance
//                 changes and flush that instance's tallies before moving on.
// Nothing here is a dense contraction: the path is bound by plain vector ALU work (Philox,
// transcendentals, divisions), its latency and LDS traffic, not by MFMA or HBM.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "mcbte_dev.h"

namespace mcbte {

// ------------------------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------------------------

// boundary id - 1 -> (axis, side) in the paper's boundary-table order
__device__ __forceinline__ constexpr int face_axis(int i) { return (i == 1 || i == 3) ? 0 : (i == 0 || i == 2) ? 1 : 2; }
__device__ __forceinline__ constexpr int face_side(int i) { return (i == 1 || i == 2 || i == 5) ? 1 : 0; }
// boundary id (index + 1) of the face of axis a on side s (1: at L, 0: at 0)
__device__ __forceinline__ constexpr int face_id(int a, int s) { return a == 0 ? (s ? 2 : 4) : (a == 1 ? (s ? 3 : 1) : (s ? 6 : 5)); }

__host__ __device__ __forceinline__ int64_t align16(int64_t x) { return (x + 15) & ~int64_t(15); }

struct W4 { uint32_t x, y, z, w; };

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64 products
// (v_mad_u64_u32) and two three-way XORs; the key schedule is wave-uniform.  Every stream of a
// launch has the same key (the seed), so the key lives in scalar registers; the empty asm keeps
// its schedule inside each call (two scalar adds a round) instead of twenty round keys held, and
// spilled, across the whole persistent kernel.  (Every lane holds the key, so the first active
// lane's copy is the wave's.)
__device__ __forceinline__ W4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
    k0 = __builtin_amdgcn_readfirstlane(k0);
    k1 = __builtin_amdgcn_readfirstlane(k1);
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return W4{c0, c1, c2, c3};
}

// The random stream of one particle: counter = (block, pid_lo, pid_hi, instance), key = seed.
// Record r is blocks 2r (words W0..W3) and 2r + 1 (W4..W7).
struct Stream {
    uint32_t k0, k1, plo, phi, inst;
    __device__ __forceinline__ W4 block(uint32_t b) const { return philox10(b, plo, phi, inst, k0, k1); }
};

__device__ __forceinline__ uint64_t key64(uint32_t hi, uint32_t lo) { return ((uint64_t)hi << 32) | (uint64_t)lo; }

template <typename R> __device__ __forceinline__ R unif(uint32_t hi, uint32_t lo);
// FP64: 53 bits of the 64-bit key, u in [0, 1 - 2^-53]
template <> __device__ __forceinline__ double unif<double>(uint32_t hi, uint32_t lo)
{
    return (double)(key64(hi, lo) >> 11) * 0x1p-53;
}
// FP32: the top 24 of those 53 bits (common random numbers with the FP64 form)
template <> __device__ __forceinline__ float unif<float>(uint32_t hi, uint32_t)
{
    return (float)(hi >> 8) * 0x1p-24f;
}

// FP64: correctly rounded arithmetic and the device math library (the event sequence of the
// method's spelled-out steps).  FP32: the hardware approximations (v_rcp_f32, v_sqrt_f32,
// v_log_f32, v_sin_f32 / v_cos_f32, about 1 ulp each); the FP32 form is compared with the oracle
// by tolerance, and its discrete choices still come from the same 64-bit keys.
__device__ __forceinline__ double r_log(double x) { return log(x); }
__device__ __forceinline__ float r_log(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
__device__ __forceinline__ double r_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float r_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double r_div(double a, double b) { return a / b; }
__device__ __forceinline__ float r_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ void r_sincos_2pi(double u, double* s, double* c)
{
    const double phi = 6.283185307179586 * u;
    *s = sin(phi);
    *c = cos(phi);
}
// v_sin_f32 / v_cos_f32 take their argument in revolutions: sin(2 pi u) directly, u in [0, 1)
__device__ __forceinline__ void r_sincos_2pi(float u, float* s, float* c)
{
    *s = __builtin_amdgcn_sinf(u);
    *c = __builtin_amdgcn_cosf(u);
}

template <typename R> struct Geo;
template <> struct Geo<double> {
    static __device__ __forceinline__ double L(const DevGeom& g, int a) { return g.L[a]; }
    static __device__ __forceinline__ double cx(const DevGeom& g, int i) { return g.pore_cx[i]; }
    static __device__ __forceinline__ double cy(const DevGeom& g, int i) { return g.pore_cy[i]; }
    static __device__ __forceinline__ double r(const DevGeom& g, int i) { return g.pore_r[i]; }
    static __device__ __forceinline__ double ng(const DevGeom& g, int a) { return g.ngrad[a]; }
    static __device__ __forceinline__ double dlo(const DevDet& d, int a) { return d.lo[a]; }
    static __device__ __forceinline__ double dhi(const DevDet& d, int a) { return d.hi[a]; }
    static __device__ __forceinline__ double dw(const DevDet& d, int a) { return d.w[a]; }
    // cell index of a coordinate, floor((x - lo) / w) exactly as the method's detector binning,
    // from values held in registers: cell_scale is the width
    static __device__ __forceinline__ double cell_scale(const DevDet& d, int a) { return d.w[a]; }
    static __device__ __forceinline__ double cellf_of(double x, double lo, double sc) { return floor((x - lo) / sc); }
    static __device__ __forceinline__ const double* tmeas_ptr(const DevTab& t) { return t.t_meas64; }
    static __device__ __forceinline__ const double* v(const DevTab& t) { return t.v64; }
    static __device__ __forceinline__ const double* tau(const DevTab& t) { return t.tau64; }
    static __device__ __forceinline__ const double* tau2(const DevTab& t) { return t.tau2_64; }
    static __device__ __forceinline__ const DevPore64& pore(const DevGeom& g, int i) { return g.pore64[i]; }
    static __device__ __forceinline__ double heat_lo(const DevTab& t, int a) { return t.heat_lo[a]; }
    static __device__ __forceinline__ double heat_w(const DevTab& t, int a) { return t.heat_w[a]; }
    static __device__ __forceinline__ const double* heat_tet(const DevTab& t) { return t.heat_tet64; }
    static constexpr int prec = 1;
};
template <> struct Geo<float> {
    static __device__ __forceinline__ float L(const DevGeom& g, int a) { return g.L32[a]; }
    static __device__ __forceinline__ float cx(const DevGeom& g, int i) { return g.pore_cx32[i]; }
    static __device__ __forceinline__ float cy(const DevGeom& g, int i) { return g.pore_cy32[i]; }
    static __device__ __forceinline__ float r(const DevGeom& g, int i) { return g.pore_r32[i]; }
    static __device__ __forceinline__ float ng(const DevGeom& g, int a) { return g.ngrad32[a]; }
    static __device__ __forceinline__ float dlo(const DevDet& d, int a) { return d.lo32[a]; }
    static __device__ __forceinline__ float dhi(const DevDet& d, int a) { return d.hi32[a]; }
    static __device__ __forceinline__ float dw(const DevDet& d, int a) { return (float)d.w[a]; }
    // cell index of a coordinate, floor((x - lo) / w), from values held in registers: cell_scale is
    // the inverse width
    static __device__ __forceinline__ float cell_scale(const DevDet& d, int a) { return d.inv_w32[a]; }
    static __device__ __forceinline__ float cellf_of(float x, float lo, float sc) { return floorf((x - lo) * sc); }
    static __device__ __forceinline__ const float* tmeas_ptr(const DevTab& t) { return t.t_meas32; }
    static __device__ __forceinline__ const float* v(const DevTab& t) { return t.v32; }
    static __device__ __forceinline__ const float* tau(const DevTab& t) { return t.tau32; }
    static __device__ __forceinline__ const float* tau2(const DevTab& t) { return t.tau2_32; }
    static __device__ __forceinline__ const DevPore32& pore(const DevGeom& g, int i) { return g.pore32[i]; }
    static __device__ __forceinline__ float heat_lo(const DevTab& t, int a) { return t.heat_lo32[a]; }
    static __device__ __forceinline__ float heat_w(const DevTab& t, int a) { return t.heat_w32[a]; }
    static __device__ __forceinline__ const float* heat_tet(const DevTab& t) { return t.heat_tet32; }
    static constexpr int prec = 0;
};

// first index j with K < thr[j] (thresholds non-decreasing), else `last`: a fixed number of
// halving steps, so all lanes of a wave run the same instructions
__device__ __forceinline__ int cdf_pick(const uint64_t* thr, int n, int64_t last, uint64_t K)
{
    int lo = 0;
    int step = 1;
    while (step * 2 <= n) step *= 2;
    for (; step > 0; step >>= 1) {
        const int probe = lo + step;
        if (probe <= n && thr[probe - 1] <= K) lo = probe;
    }
    return lo < n ? lo : (int)last;
}

// the same choice as cdf_pick for a non-decreasing table, searching only between the bounds the
// guide gives for the key's top 64 - shift bits (guide[b] = count(thr <= b 2^shift), b <= 2^(64 - shift));
// a guide as fine as the table's spread keeps the search at a step or two for every lane
__device__ __forceinline__ int cdf_pick_guided(const uint64_t* thr, const uint16_t* guide, int shift, int n,
                                               int64_t last, uint64_t K)
{
    const uint32_t b = (uint32_t)(K >> shift);
    int lo = guide[b], hi = guide[b + 1];                        // count(thr <= K) lies in [lo, hi]
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (thr[mid] <= K) lo = mid + 1;
        else hi = mid;
    }
    return lo < n ? lo : (int)last;
}

// an emission row draw: guided where the table has a guide (global memory), the same choice
__device__ __forceinline__ int cdf_pick_rows(const uint64_t* thr, const uint16_t* guide, int n, int64_t last, uint64_t K)
{
    return guide ? cdf_pick_guided(thr, guide, 64 - MCBTE_GUIDE_BITS, n, last, K) : cdf_pick(thr, n, last, K);
}

template <typename R> struct Part {
    R x[3], o[3];
    R t, dtr;            // time, time left until the next scattering event
    R lead;              // two clocks: how much later the other one fires (+inf: never); the sign
                         // bit set means the next scattering is the two-phonon one
    int32_t m, s, nrel;  // mode row, sign, three-phonon relaxations so far
    uint32_t k, j;       // segments so far, random-number-drawing events so far
    uint32_t kc;         // pore lattice: k after the last wave walk (no new walk before a segment)
    int32_t src;         // source element (event log only)
    double cT, cq;       // per-particle contributions (variance estimate); cq is the flux score F
    R dtr0;              // free-flight time drawn for the current flight (sensitivity replay)
    double F0;           // flux score at the start of the current flight (sensitivity replay)
    int32_t tk;          // transient tallies: first measurement time not before t (-1: not yet known)
    // the last segment's scores left to the whole wave after the step: transient snapshots (start,
    // direction, start time, speed; first measurement index, count) or, in a sparse wave, the
    // detector-grid pieces (start, direction, length, speed; mode, pending flag)
    R sx[3], so[3], st0, svm;
    int32_t sk0, sn;
};

// cosine-weighted direction about the unit normal n (Eq. wall_dir), frame t1 = e_j x n / |.|
// with j the first axis of smallest |n_j|, t2 = n x t1
template <typename R>
__device__ __forceinline__ void dir_about(R mu, R a, R b, const R n[3], R o[3])
{
    if (n[2] == R(0) && n[0] != R(0) && n[1] != R(0)) {
        // a normal in the x-y plane with both components nonzero (a pore's, a line wall's): the
        // frame below takes j = 2, so t1 = (-n1, n0, 0) / |n|, t2 = (0, 0, n0 t1_1 - n1 t1_0); the
        // same roundings without the products and sums that are exact zeros (only the sign of an
        // exactly zero component can differ)
        const R len = r_sqrt(n[1] * n[1] + n[0] * n[0]);
        const R t10 = r_div(-n[1], len), t11 = r_div(n[0], len);
        const R t22 = n[0] * t11 - n[1] * t10;
        o[0] = mu * n[0] + a * t10;
        o[1] = mu * n[1] + a * t11;
        o[2] = b * t22;
        return;
    }
    int j = 0;
    R m0 = fabs(n[0]);
    if (fabs(n[1]) < m0) { j = 1; m0 = fabs(n[1]); }
    if (fabs(n[2]) < m0) j = 2;
    const R e0 = j == 0 ? R(1) : R(0), e1 = j == 1 ? R(1) : R(0), e2 = j == 2 ? R(1) : R(0);
    R c0 = e1 * n[2] - e2 * n[1];
    R c1 = e2 * n[0] - e0 * n[2];
    R c2 = e0 * n[1] - e1 * n[0];
    const R len = r_sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    const R t10 = r_div(c0, len), t11 = r_div(c1, len), t12 = r_div(c2, len);
    const R t20 = n[1] * t12 - n[2] * t11;
    const R t21 = n[2] * t10 - n[0] * t12;
    const R t22 = n[0] * t11 - n[1] * t10;
    o[0] = mu * n[0] + a * t10 + b * t20;
    o[1] = mu * n[1] + a * t11 + b * t21;
    o[2] = mu * n[2] + a * t12 + b * t22;
}

template <typename R>
__device__ __forceinline__ void dir_cos(R u1, R u2, const R n[3], R o[3])
{
    const R mu = r_sqrt(u1);
    const R st = r_sqrt(R(1) - u1);
    R sn, cs;
    r_sincos_2pi(u2, &sn, &cs);
    dir_about(mu, st * cs, st * sn, n, o);
}

template <typename R>
__device__ __forceinline__ void dir_iso(R u1, R u2, R o[3])
{
    const R mu = R(1) - R(2) * u1;
    const R s2 = (R(1) - mu) * (R(1) + mu);
    const R st = r_sqrt(s2 > R(0) ? s2 : R(0));
    R sn, cs;
    r_sincos_2pi(u2, &sn, &cs);
    o[0] = st * cs;
    o[1] = st * sn;
    o[2] = mu;
}

// ------------------------------------------------------------------------------------------
// the two clocks of section 3.3: a two-phonon and a three-phonon time to scattering, each from
// Eq. time_to_scat, running down together with the particle's time; the earlier one is kept in
// dtr and the other's lead over it in lead (sign bit set: the two-phonon clock is the earlier);
// a tie goes to the three-phonon clock.  An event that redraws the two-phonon time leaves the
// three-phonon time in dtr and lead = NaN; the draw is made at the start of the next step
// (resolve_clocks), where few other values are live.
// ------------------------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ void set_clocks(Part<R>& p, R t2, R t3)
{
    const bool two_first = t2 < t3;
    p.dtr = two_first ? t2 : t3;
    p.lead = two_first ? -(t3 - t2) : t2 - t3;
}

// the two-phonon time of row m drawn at the j-th drawing event (j = 0: emission), from words
// W0W1 of record 0x60000000 + j; +inf for a row without the process
template <typename R>
__device__ __forceinline__ R draw_t2(const DevTab& T, const Stream& st, uint32_t j, int m)
{
    const R tau2 = Geo<R>::tau2(T)[m];
    if (!(tau2 > R(0))) return R(1) / R(0);
    const W4 q = st.block(2u * (0x60000000u + j));
    return -tau2 * r_log(R(1) - unif<R>(q.x, q.y));
}

// internal line wall k in the trajectories' precision: segment ends and unit normal
template <typename R> struct WallR { R x1, y1, x2, y2, nx, ny; };
template <typename R>
__device__ __forceinline__ WallR<R> wall_of(const DevGeom& g, int k)
{
    if constexpr (std::is_same<R, double>::value)
        return WallR<R>{g.wall_x1[k], g.wall_y1[k], g.wall_x2[k], g.wall_y2[k], g.wall_nx[k], g.wall_ny[k]};
    else
        return WallR<R>{g.wall32[k][0], g.wall32[k][1], g.wall32[k][2], g.wall32[k][3], g.wall32[k][4], g.wall32[k][5]};
}

// inside a closed loop of walls (crossing number, half-open edges): outside the solid
template <typename R>
__device__ __forceinline__ bool inside_wall_loops(const DevGeom& g, R px, R py)
{
    bool inside = false;
    for (int k = 0; k < g.n_walls; ++k) {
        const int j = g.wall_loop_end[k];
        if (j < 0) continue;
        bool in = false;
        for (int e = k; e <= j; ++e) {
            const WallR<R> w = wall_of<R>(g, e);
            if ((w.y1 > py) != (w.y2 > py) && px < w.x1 + (py - w.y1) * (w.x2 - w.x1) / (w.y2 - w.y1)) in = !in;
        }
        inside = inside || in;
    }
    return inside;
}

template <typename R>
__device__ __forceinline__ void resolve_clocks(const DevTab& T, const Stream& st, Part<R>& p)
{
    if (isnan(p.lead)) set_clocks(p, draw_t2<R>(T, st, p.j, p.m), p.dtr);
}

// ------------------------------------------------------------------------------------------
// emission (section 3.2)
// ------------------------------------------------------------------------------------------

// kf (optional): the top 53 bits of the first free flight's key (the scheduling test of pore lattices)
template <typename R>
__device__ __forceinline__ void emit_particle(const DevTab& T, const Stream& st, Part<R>& p, uint32_t& rejections,
                                              uint64_t* kf = nullptr)
{
    const DevGeom& g = T.g;
    const W4 r0a = st.block(0), r0b = st.block(1), r1a = st.block(2), r1b = st.block(3);
    const int src = cdf_pick(T.thr_src, T.S, T.last_src, key64(r0a.x, r0a.y));
    const int kind = T.src_kind[src];
    R up[3] = {unif<R>(r1a.z, r1a.w), unif<R>(r1b.x, r1b.y), unif<R>(r1b.z, r1b.w)};
    const R ud1 = unif<R>(r0b.x, r0b.y), ud2 = unif<R>(r0b.z, r0b.w);
    W4 r2a = {0u, 0u, 0u, 0u};
    if (kind == SRC_GRAD || (T.transient && kind != SRC_IC)) r2a = st.block(4);
    p.src = src;
    p.nrel = 0;
    p.k = 0;
    p.j = 0;
    p.cT = 0.0;
    p.cq = 0.0;
    if (kind == SRC_WALL) {
        const int fid = T.src_ref[src] - 1;
        const int a = face_axis(fid), side = face_side(fid);
        const int b = (a == 0) ? 1 : 0;
        R n[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const R L = Geo<R>::L(g, ax);
            const R u = (ax == b) ? up[0] : up[1];
            p.x[ax] = (ax == a) ? (side ? L : R(0)) : (g.unb[ax] ? R(0) : u * L);
            n[ax] = (ax == a) ? (side ? R(-1) : R(1)) : R(0);
        }
        dir_cos(ud1, ud2, n, p.o);
        p.s = T.src_sign[src];
        p.m = cdf_pick_rows(T.thr_wall, T.wall_guide, T.M, T.last_wall, key64(r1a.x, r1a.y));
    } else if (kind == SRC_IWALL) {
        // a point of the isothermal line wall (along the segment, through the thickness),
        // directions cosine-weighted about its normal
        const WallR<R> w = wall_of<R>(g, T.src_ref[src]);
        p.x[0] = w.x1 + up[0] * (w.x2 - w.x1);
        p.x[1] = w.y1 + up[0] * (w.y2 - w.y1);
        p.x[2] = g.unb[2] ? R(0) : up[1] * Geo<R>::L(g, 2);
        const R n[3] = {w.nx, w.ny, R(0)};
        dir_cos(ud1, ud2, n, p.o);
        p.s = T.src_sign[src];
        p.m = cdf_pick_rows(T.thr_wall, T.wall_guide, T.M, T.last_wall, key64(r1a.x, r1a.y));
    } else if (kind == SRC_GRAD) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) p.x[ax] = g.unb[ax] ? R(0) : up[ax] * Geo<R>::L(g, ax);
        // positions outside the solid (inside pores or closed loops of walls) are redrawn
        for (uint32_t attempt = 1; g.n_pores > 0 || g.n_walls > 0; ++attempt) {
            bool inside = false;
            for (int c = 0; c < g.n_pores; ++c) {
                const R dx = p.x[0] - Geo<R>::cx(g, c), dy = p.x[1] - Geo<R>::cy(g, c);
                const R r = Geo<R>::r(g, c);
                if (dx * dx + dy * dy < r * r) inside = true;
            }
            if (g.n_walls > 0 && inside_wall_loops<R>(g, p.x[0], p.x[1])) inside = true;
            if (!inside || attempt > 4096) break;
            ++rejections;
            const uint32_t blk = 2u * (0x40000000u + attempt);
            const W4 qa = st.block(blk), qb = st.block(blk + 1u);
            const R ua[3] = {unif<R>(qa.z, qa.w), unif<R>(qb.x, qb.y), unif<R>(qb.z, qb.w)};
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) p.x[ax] = g.unb[ax] ? R(0) : ua[ax] * Geo<R>::L(g, ax);
        }
        const R n[3] = {Geo<R>::ng(g, 0), Geo<R>::ng(g, 1), Geo<R>::ng(g, 2)};
        dir_cos(ud1, ud2, n, p.o);
        p.s = (r2a.x >> 31) ? -1 : 1;     // both signs equally likely; a negative particle travels reversed
        if (p.s < 0) {
            p.o[0] = -p.o[0];
            p.o[1] = -p.o[1];
            p.o[2] = -p.o[2];
        }
        p.m = cdf_pick_rows(T.thr_wall, T.wall_guide, T.M, T.last_wall, key64(r1a.x, r1a.y));
    } else if (kind == SRC_HEAT) {
        // the external heat source: a point of its cuboid, or of one of its tetrahedra (drawn by
        // volume; the point by folding the unit cube onto the tetrahedron), an isotropic
        // direction, the row drawn by heat capacity (as for the initial condition)
        if (T.n_heat_tet > 0) {
            const W4 r2b = st.block(5);
            const int k = cdf_pick(T.thr_tet, T.n_heat_tet, T.last_tet, key64(r2b.x, r2b.y));
            R b0 = up[0], b1 = up[1], b2 = up[2];
            if (b0 + b1 > R(1)) {              // the cube's halves across b0 + b1 = 1 onto each other
                b0 = R(1) - b0;
                b1 = R(1) - b1;
            }
            if (b1 + b2 > R(1)) {              // then the prism's parts onto the tetrahedron
                const R w = b2;
                b2 = R(1) - b0 - b1;
                b1 = R(1) - w;
            } else if (b0 + b1 + b2 > R(1)) {
                const R w = b2;
                b2 = b0 + b1 + b2 - R(1);
                b0 = R(1) - b1 - w;
            }
            const R* v = Geo<R>::heat_tet(T) + 12 * k;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) p.x[ax] = ((v[ax] + b0 * v[3 + ax]) + b1 * v[6 + ax]) + b2 * v[9 + ax];
        } else {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
                p.x[ax] = g.unb[ax] ? R(0) : Geo<R>::heat_lo(T, ax) + up[ax] * Geo<R>::heat_w(T, ax);
        }
        dir_iso(ud1, ud2, p.o);
        p.s = T.src_sign[src];
        p.m = cdf_pick_rows(T.thr_ic, T.ic_guide, T.M, T.last_ic, key64(r1a.x, r1a.y));
    } else {
        const int c = T.src_ref[src];
        const int ia = T.ic_axis;
        const R e0 = (R)T.ic_edges[c];
        const R width = (R)(T.ic_edges[c + 1] - T.ic_edges[c]);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax)
            p.x[ax] = (ax == ia) ? e0 + up[ax] * width : (g.unb[ax] ? R(0) : up[ax] * Geo<R>::L(g, ax));
        dir_iso(ud1, ud2, p.o);
        p.s = T.src_sign[src];
        p.m = cdf_pick_rows(T.thr_ic, T.ic_guide, T.M, T.last_ic, key64(r1a.x, r1a.y));
    }
    if (kind == SRC_HEAT) {   // a time uniform in the source's interval
        const int k = T.src_ref[src];
        p.t = (R)T.heat_t[k] + unif<R>(r2a.z, r2a.w) * (R)(T.heat_t[k + 1] - T.heat_t[k]);
    } else {
        p.t = (T.transient && kind != SRC_IC) ? unif<R>(r2a.z, r2a.w) * (R)T.t_max : R(0);
    }
    const R tau = Geo<R>::tau(T)[p.m];
    p.dtr = -tau * r_log(R(1) - unif<R>(r0a.z, r0a.w));
    if (kf) *kf = key64(r0a.z, r0a.w) >> 11;
    p.lead = T.two ? R(NAN) : R(0);     // two clocks: the two-phonon time is still to be drawn
    p.dtr0 = p.dtr;
    p.F0 = 0.0;
}

// ------------------------------------------------------------------------------------------
// tallies
// ------------------------------------------------------------------------------------------

struct TallyCtx {
    double* lds;     // compact per-workgroup copy (ncomp components per cell-column) or NULL
    double* glob;    // raw sums in the tally buffer, 4 components per cell-column
    float* lds32;    // compact per-workgroup FP32 copy (wide workgroups) or NULL
};

__device__ __forceinline__ void tadd(const TallyCtx& tc, const DevDet& D, int64_t cc, int q, double val)
{
    if (tc.lds32) atomicAdd(tc.lds32 + cc * D.ncomp + D.slot[q], (float)val);
    else if (tc.lds) atomicAdd(tc.lds + cc * D.ncomp + D.slot[q], val);
    else if (tc.glob) atomicAdd(tc.glob + cc * 4 + q, val);
}

__device__ __forceinline__ void tadd_c(const TallyCtx& tc, int ncomp, uint32_t slots, int64_t cc, int q, double val)
{
    const int slot = (int)((slots >> (8 * q)) & 0xFFu);
    if (tc.lds32) atomicAdd(tc.lds32 + cc * ncomp + slot, (float)val);
    else if (tc.lds) atomicAdd(tc.lds + cc * ncomp + slot, val);
    else if (tc.glob) atomicAdd(tc.glob + cc * 4 + q, val);
}

template <typename R>
__device__ __forceinline__ void add4_c(const TallyCtx& tc, int mask, int ncomp, uint32_t slots, int64_t cc, R sg,
                                       R l, R vm, const R o[3])
{
    if (mask & 1) tadd_c(tc, ncomp, slots, cc, 0, (double)(sg * r_div(l, vm)));
    if (mask & 2) tadd_c(tc, ncomp, slots, cc, 1, (double)(sg * (l * o[0])));
    if (mask & 4) tadd_c(tc, ncomp, slots, cc, 2, (double)(sg * (l * o[1])));
    if (mask & 8) tadd_c(tc, ncomp, slots, cc, 3, (double)(sg * (l * o[2])));
}

// steady track-length estimator (Eqs. temp_steady, flux_x_steady) for the segment x0 + s o,
// s in [0, d]: the pieces between consecutive detector-cell planes, each scored in the cell of
// its midpoint; the plane parameters (lo + j w - x0) / o are the same numbers the method's
// sorted-crossing description produces, visited in increasing order per axis
template <typename R>
__device__ __forceinline__ void tally_grid(const DevTab& T, const TallyCtx& tc, const R x0[3], const R o[3], R d,
                                           int m, R sg, R vm)
{
    const DevDet& D = T.det;
    if (!(d > R(0))) return;
    // the detector grid, read once per segment
    int gn[3];
    R glo[3], ghi[3], gw[3], gsc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        gn[a] = D.n[a];
        glo[a] = Geo<R>::dlo(D, a);
        ghi[a] = Geo<R>::dhi(D, a);
        gw[a] = Geo<R>::dw(D, a);
        gsc[a] = Geo<R>::cell_scale(D, a);
    }
    const int mask = D.mask, ncomp = D.ncomp, n_cols = D.n_cols;
    uint32_t slots = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) slots |= ((uint32_t)D.slot[q] & 0xFFu) << (8 * q);
    R s_lo = R(0), s_hi = d;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (gn[a] <= 0) continue;
        const R lo = glo[a], hi = ghi[a];
        if (o[a] == R(0)) {
            if (x0[a] < lo || x0[a] > hi) return;
        } else {
            R s1 = r_div(lo - x0[a], o[a]);
            R s2 = r_div(hi - x0[a], o[a]);
            if (s1 > s2) { const R tt = s1; s1 = s2; s2 = tt; }
            if (s1 > s_lo) s_lo = s1;
            if (s2 < s_hi) s_hi = s2;
        }
    }
    if (!(s_hi > s_lo)) return;
    const R INF = R(1) / R(0);
    int jn[3];
    R sn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        jn[a] = 0;
        sn[a] = INF;
        const int n = gn[a];
        if (n <= 1 || o[a] == R(0)) continue;
        const R lo = glo[a], w = gw[a];
        const int dir = o[a] > R(0) ? 1 : -1;
        // entry cell (clamped: a segment may start exactly on the outer faces of the grid), then
        // the plane ahead of it, corrected so that j is the first plane (in travel order) whose
        // parameter exceeds s_lo
        const R xs = x0[a] + o[a] * s_lo;
        int ic = (int)floor((double)((xs - lo) / w));
        ic = ic < 0 ? 0 : (ic > n - 1 ? n - 1 : ic);
        int j = ic + (dir > 0 ? 1 : 0);
        for (int it = 0; it < 4; ++it) {
            const int jb = j - dir;
            if (jb >= 1 && jb <= n - 1 && r_div(lo + (R)jb * w - x0[a], o[a]) > s_lo) j = jb;
            else break;
        }
        for (int it = 0; it < 4; ++it) {
            if (j >= 1 && j <= n - 1 && !(r_div(lo + (R)j * w - x0[a], o[a]) > s_lo)) j += dir;
            else break;
        }
        jn[a] = j;
        if (j >= 1 && j <= n - 1) sn[a] = r_div(lo + (R)j * w - x0[a], o[a]);
    }
    R s_cur = s_lo;
    for (int guard = 0; guard < 1 << 20; ++guard) {
        R s_n = s_hi;
        if (sn[0] < s_n) s_n = sn[0];
        if (sn[1] < s_n) s_n = sn[1];
        if (sn[2] < s_n) s_n = sn[2];
        const R l = s_n - s_cur;
        if (l > R(0)) {
            const R mid = R(0.5) * (s_cur + s_n);
            int64_t cell = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int n = gn[a] > 0 ? gn[a] : 1;
                int64_t ci = 0;
                if (gn[a] > 0) {
                    const R xa = x0[a] + o[a] * mid;
                    const R f = Geo<R>::cellf_of(xa, glo[a], gsc[a]);
                    ci = (int64_t)f;
                    ci = ci < 0 ? 0 : (ci > n - 1 ? n - 1 : ci);
                }
                cell = cell * n + ci;
            }
            add4_c(tc, mask, ncomp, slots, cell * n_cols + m, sg, l, vm, o);
        }
        if (!(s_n < s_hi)) break;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (sn[a] == s_n) {
                const int dir = o[a] > R(0) ? 1 : -1;
                jn[a] += dir;
                const int j = jn[a];
                sn[a] = (j >= 1 && j <= gn[a] - 1) ? r_div(glo[a] + (R)j * gw[a] - x0[a], o[a]) : INF;
            }
        }
        s_cur = s_n;
    }
}

// Transient snapshot estimator (Eq. sampling): a particle alive at measurement time t_k scores
// s (and s v Omega) into the detector cell holding x(t_k).  A segment [t0, t1) holds the times
// t_k with t0 <= t_k < t1; the step only records them (snap_pend) and the whole wave then scores
// the records of all its lanes together (snap_wave), 64 snapshots per pass however they are
// spread over the lanes (a per-lane loop ran at 9 % lane efficiency: few lanes have many).
// bounds of count(t_k < t) from the measurement-time guide gd: one bucket of slack on each side
// covers the rounding of t's bucket and of the times' copies in the trajectories' precision
template <typename R>
__device__ __forceinline__ void tm_bounds(const uint16_t* gd, R gs, R t, int& lo, int& hi)
{
    int b = (int)(t * gs);
    b = b < 0 ? 0 : (b > 255 ? 255 : b);
    lo = gd[b > 0 ? b - 1 : 0];
    hi = gd[b + 2 < 256 ? b + 2 : 256];
}

template <typename R>
__device__ __forceinline__ void snap_pend(const R* tmeas, int nt, const uint16_t* gd, R gs, Part<R>& p, R t1, R vm)
{
    // first k with t_k >= t0: found once per particle, then carried from segment to segment (a
    // particle's time only grows, and each segment starts where the previous one ended)
    int k0 = p.tk;
    if (k0 < 0) {
        int hi = nt;
        k0 = 0;
        if (gd) tm_bounds<R>(gd, gs, p.t, k0, hi);
        while (k0 < hi) {
            const int mid = (k0 + hi) >> 1;
            if (tmeas[mid] < p.t) k0 = mid + 1;
            else hi = mid;
        }
    }
    int k1 = k0;                     // first k >= k0 with t_k >= t1
    if (k1 < nt && tmeas[k1] < t1) {
        int hi = nt;
        ++k1;
        if (gd) {
            int lo;
            tm_bounds<R>(gd, gs, t1, lo, hi);
            k1 = k1 > lo ? k1 : lo;
        }
        while (k1 < hi) {
            const int mid = (k1 + hi) >> 1;
            if (tmeas[mid] < t1) k1 = mid + 1;
            else hi = mid;
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        p.sx[a] = p.x[a];
        p.so[a] = p.o[a];
    }
    p.st0 = p.t;
    p.svm = vm;
    p.sk0 = k0;
    p.sn = k1 - k0;
    p.tk = k1;
}

template <typename R>
__device__ __forceinline__ R lane_r(R v, int src) { return __shfl(v, src, 64); }

// Wave-wide scans by DPP (all 64 lanes active): within each row of 16 lanes the partial results
// move right by 1, 2, 4 and 8 lanes, then the last lane of a row is broadcast into the next rows
// (row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3).  Register-to-register moves,
// with none of the LDS round trip a cross-lane shuffle takes.
__device__ __forceinline__ int dpp_incl_sum(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return v;
}

// the OR of every lane's v (in every lane)
__device__ __forceinline__ uint32_t dpp_or_all(uint32_t v)
{
    int x = (int)v;
    x |= __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);
    x |= __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);
    x |= __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);
    x |= __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);
    x |= __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);
    x |= __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);
    return (uint32_t)__builtin_amdgcn_readlane(x, 63);
}

// the minimum of every lane's v (in every lane; all 64 lanes active), the same DPP pattern; v
// non-negative or +inf, whose order is that of their bit patterns as unsigned integers (the
// unsigned minimum's identity, all ones, fills the lanes a shift leaves without a source, so each
// step is one v_min_u32 with its DPP operand)
__device__ __forceinline__ float dpp_min_nonneg(float v)
{
    uint32_t x = (uint32_t)__float_as_int(v);
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x111, 0xF, 0xF, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x112, 0xF, 0xF, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x114, 0xF, 0xF, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x118, 0xF, 0xF, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x142, 0xA, 0xF, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x143, 0xC, 0xF, false));
    return __int_as_float(__builtin_amdgcn_readlane((int)x, 63));
}

// the position of the set bit of L that has r set bits below it (L holds more than r)
__device__ __forceinline__ int nth_set_bit(unsigned long long L, int r)
{
    int pos = 0;                     // the largest pos with popcount(L below pos) <= r
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if (__popcll(L & ((1ull << (pos + step)) - 1ull)) <= r) pos += step;
    return pos;
}

// the detector layout snapshot scoring reads (launch-uniform)
template <typename R>
struct SnapDet {
    int gn[3];
    R glo[3], ghi[3], gsc[3];
    int mask, ncomp, n_cols;
    uint32_t slots;
    __device__ __forceinline__ explicit SnapDet(const DevDet& D)
    {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            gn[a] = D.n[a];
            glo[a] = Geo<R>::dlo(D, a);
            ghi[a] = Geo<R>::dhi(D, a);
            gsc[a] = Geo<R>::cell_scale(D, a);
        }
        mask = D.mask;
        ncomp = D.ncomp;
        n_cols = D.n_cols;
        slots = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) slots |= ((uint32_t)D.slot[q] & 0xFFu) << (8 * q);
    }
};

// one snapshot: the particle of sign sg that left x0 along o at t0 with speed vm, at measurement
// time k, scores sg and sg vm Omega into the cell holding its position then
template <typename R>
__device__ __forceinline__ void snap_score(const SnapDet<R>& G, const TallyCtx& tc, const R* tmeas, const R x0[3],
                                           const R o[3], R t0, R vm, R sg, int k)
{
    const R dist = vm * (tmeas[k] - t0);
    int64_t cell = 0;
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int n = G.gn[a] > 0 ? G.gn[a] : 1;
        int64_t ci = 0;
        if (G.gn[a] > 0) {
            const R xa = x0[a] + o[a] * dist;
            if (xa < G.glo[a] || xa > G.ghi[a]) inside = false;
            const R f = Geo<R>::cellf_of(xa, G.glo[a], G.gsc[a]);
            ci = (int64_t)f;
            ci = ci < 0 ? 0 : (ci > n - 1 ? n - 1 : ci);
        }
        cell = cell * n + ci;
    }
    if (inside) {
        const int64_t cc = cell * G.n_cols + k;
        if (G.mask & 1) tadd_c(tc, G.ncomp, G.slots, cc, 0, (double)sg);
        if (G.mask & 2) tadd_c(tc, G.ncomp, G.slots, cc, 1, (double)(sg * (vm * o[0])));
        if (G.mask & 4) tadd_c(tc, G.ncomp, G.slots, cc, 2, (double)(sg * (vm * o[1])));
        if (G.mask & 8) tadd_c(tc, G.ncomp, G.slots, cc, 3, (double)(sg * (vm * o[2])));
    }
}

template <typename R>
__device__ __forceinline__ void snap_wave(const DevTab& T, const TallyCtx& tc, const R* tmeas, Part<R>& p)
{
    if (__ballot(p.sn > 0) == 0ull) return;
    const int lane = threadIdx.x & 63;
    const SnapDet<R> G(T.det);
    // every lane scores the first snapshot of its segment itself (most segments hold at most one)
    if (p.sn > 0) snap_score<R>(G, tc, tmeas, p.sx, p.so, p.st0, p.svm, (R)p.s, p.sk0);
    // the rest, 64 per pass however they are spread over the lanes
    const int rest = p.sn > 0 ? p.sn - 1 : 0;
    const unsigned long long L = __ballot(rest > 0);   // the lanes holding more snapshots
    if (L != 0ull) {
        const int S = dpp_incl_sum(rest);   // inclusive prefix sum of the lanes' remaining counts
        const int total = __builtin_amdgcn_readlane(S, 63);
        const int kb = (p.sk0 + 1) - (S - rest);   // measurement index of snapshot g of this lane: kb + g
        const R sv = p.s < 0 ? -p.svm : p.svm;
        for (int base = 0; base < total; base += 64) {
            const int g = base + lane;
            // the lane whose records hold snapshot g: among the lanes with snapshots (L), the one
            // after the rank(g) = #{i in L : S_i <= g} whose ranges end at or before g.  Ranges
            // ending in this pass's window (1 <= S_i - base <= 63) are distinct bits of W; those
            // ending before it are counted by one ballot.
            const int e = S - base;
            const bool ends_in = ((L >> lane) & 1ull) && e >= 1 && e <= 63;
            const uint32_t wlo = dpp_or_all(ends_in && e < 32 ? 1u << e : 0u);
            const uint32_t whi = dpp_or_all(ends_in && e >= 32 ? 1u << (e - 32) : 0u);
            const unsigned long long W = ((unsigned long long)whi << 32) | wlo;
            const int c0 = __popcll(__ballot(((L >> lane) & 1ull) && e <= 0));
            const unsigned long long upto = lane == 63 ? ~0ull : (2ull << lane) - 1ull;
            const int rank = c0 + __popcll(W & upto);
            const int own = rank < __popcll(L) ? nth_set_bit(L, rank) : 63;
            const int k = __shfl(kb, own, 64) + g;
            // the owner's segment: positions along the binned axes, direction components those
            // axes and the scored flux components need, start time, speed with the particle's sign
            R x0[3] = {R(0), R(0), R(0)}, o[3] = {R(0), R(0), R(0)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (G.gn[a] > 0) x0[a] = lane_r<R>(p.sx[a], own);
                if (G.gn[a] > 0 || (G.mask & (2 << a))) o[a] = lane_r<R>(p.so[a], own);
            }
            const R t0 = lane_r<R>(p.st0, own), svm = lane_r<R>(sv, own);
            if (g < total) snap_score<R>(G, tc, tmeas, x0, o, t0, fabs(svm), copysign(R(1), svm), k);
        }
    }
    p.sn = 0;
}

// ------------------------------------------------------------------------------------------
// one flight (sections 3.3 and 3.5)
// ------------------------------------------------------------------------------------------

enum : uint32_t {
    EV_EMIT_POS = 0, EV_RELAX = 1, EV_SPECULAR = 2, EV_DIFFUSE = 3, EV_PERIODIC = 4, EV_ABSORB = 5,
    EV_TIMEOUT = 6, EV_NSCAT = 7, EV_CAP = 8, EV_EMIT_NEG = 9, EV_ESCAPE = 10, EV_TWO = 11
};

struct LaneCounts {
    static constexpr int N = 13;   // the counters up to the two-phonon events (MCBTE_CNT_*)
    uint32_t c[N];
};

struct LogRow {
    uint32_t* row;   // NULL: not logged
    int32_t n;
    int32_t stride;
    __device__ __forceinline__ void put(uint32_t ev, int bnd, int m)
    {
        if (row) {
            const uint32_t b = (uint32_t)(bnd > 255 ? 255 : bnd);
            if (n + 1 < stride) row[1 + n] = (ev << 28) | (b << 20) | ((uint32_t)m & 0xFFFFFu);
            ++n;
        }
    }
};

// likelihood-ratio bookkeeping of the sensitivity replay (dkappa / dln tau per frequency bin):
// a flight ended by a relaxation scores T/tau - 1, one cut short T/tau, a relaxation draw -1 for
// the drawn row's bin (plus P_i for every bin, summed into `dense`); each score multiplies the
// part of the particle's flux score F that follows it
struct AdjCtx {
    double* bins;            // LDS, n_bins sums
    double F_total;          // this particle's F from the forward trace
    double dense;            // per-lane sum of (F_total - F) over relaxation draws
    uint32_t bad;            // pathwise terms that were not finite
    double split;            // local pathwise form: modes with v tau <= split
    __device__ __forceinline__ void add(int bin, double g, double after) { atomicAdd(bins + bin, g * after); }
};

// Local pathwise form (AK = 3), for a mode whose mean free path v tau is at most the split: a
// flight's own flux depends on tau only through its length L = v tau E and changes by s L Omega_a
// (Omega the direction of its last segment) if it ended in a relaxation, by nothing if it was cut
// short; what follows it keeps the likelihood ratio (T/tau - 1) (F_total - F at the flight's end).
// Longer modes take the likelihood-ratio form of AK = 1.
template <int AK>
__device__ __forceinline__ bool local_form(const DevTab& T, int m, const AdjCtx& adj)
{
    return AK == 3 && T.v64[m] * T.tau64[m] <= adj.split;
}

template <typename R>
struct Tabs {
    const uint64_t* thr_rel;   // LDS
    const R* v;                // LDS
    const R* tau;              // LDS
    const uint16_t* guide;     // bounds of the relaxation draw (LDS when staged), or NULL (search the whole table)
    const R* tmeas;            // measurement times (transient tallies): LDS where staged, else the table block
    int gshift;                // key bits below the guide's index
};

// The launch-uniform values the flight loop reads, loaded once before it so that they stay in
// registers instead of being fetched from the table block at every segment.
// the reflection class of a phonon of row m at a boundary that reads per-row table tab (1-based),
// as the trajectories of precision R see its specularity
template <typename R>
__device__ __forceinline__ uint32_t tab_class(const DevTab& T, int tab, int m)
{
    const uint32_t c = T.spec_cls[(int64_t)(tab - 1) * T.M + m];
    return std::is_same<R, float>::value ? (c & 3u) : ((c >> 2) & 3u);
}

template <typename R>
struct Hot {
    R L[3];
    R t_max;
    R coop_min;          // remaining free path above which a film-wall bounce turns cooperative
    R lat_min;           // pore lattice: remaining free path above which the wave walks the particle
    uint32_t unb;        // bit a: axis a has no faces
    uint32_t face;       // 4 bits per face id - 1: type | class << 2
    uint32_t pcls;       // 2 bits per pore: class
    uint32_t det_slot;   // 8 bits per tally component: compact slot
    int32_t det_mask, det_ncomp;
    int32_t n_pores, max_events, n_scat_max, M, last_rel, transient, score_axis, coop_axis;
    int32_t fold_axis;   // film axis whose specular crossings run at once (FP32 trace), -1: off
    R p0cx, p0cy, p0r;   // the first pore (most geometries have at most one)
    int32_t p0id;
    int32_t grid_axis;   // the one detector axis with more than one cell, if only one has (else -1)
};

// fold: the launch may run a specular phonon's film crossings at once (not when it records each
// particle's flux score for a replay, which steps them one at a time)
template <typename R>
__device__ __forceinline__ Hot<R> load_hot(const DevTab& T, bool fold = false)
{
    const DevGeom& g = T.g;
    Hot<R> h;
#pragma unroll
    for (int a = 0; a < 3; ++a) h.L[a] = Geo<R>::L(g, a);
    h.t_max = (R)T.t_max;
    h.coop_min = (R)T.coop_min_path;
    h.lat_min = (R)T.lat_min_path;
    h.unb = g.unb_mask;
    h.face = g.face_code[Geo<R>::prec];
    h.pcls = g.pore_cls[Geo<R>::prec];
    uint32_t slots = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) slots |= ((uint32_t)T.det.slot[q] & 0xFFu) << (8 * q);
    h.det_slot = slots;
    h.det_mask = T.det.mask;
    h.det_ncomp = T.det.ncomp;
    h.n_pores = g.n_pores;
    h.max_events = (int32_t)T.max_events;
    h.n_scat_max = T.n_scat_max;
    h.M = T.M;
    h.last_rel = (int32_t)T.last_rel;
    h.transient = T.transient;
    h.score_axis = T.score_axis;
    h.coop_axis = T.coop_axis;
    h.fold_axis = (fold && std::is_same<R, float>::value) ? T.fold_axis : -1;
    const auto P0 = Geo<R>::pore(g, 0);
    h.p0cx = P0.cx;
    h.p0cy = P0.cy;
    h.p0r = P0.r;
    h.p0id = P0.id;
    int na = 0, ax = -1;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (T.det.n[a] > 1) { ++na; ax = a; }
    h.grid_axis = na == 1 ? ax : -1;
    return h;
}

// Pathwise sensitivity state of one particle (replay form).  A free flight of mode m covers
// the distance L = v_m tau_m E with E fixed by its random numbers, so dL / dln tau_m = L.  With the
// sequence of events held fixed, stretching a flight shifts what follows it, linearly.  At the
// start of a flight every earlier stretch has become a pure position shift (the relaxation that
// began the flight drew a direction that does not depend on where it happened), so the flight
// is described by its response g: how its position, direction and remaining distance (gx, go, gb)
// follow a position shift at the flight's start.  g is updated at each boundary hit and
// reflection (three columns, whatever the number of stored shifts); at the relaxation that ends
// the flight it becomes the 3x3 map J = gx + o gb^T + d go, applied to every stored shift, and
// the flight's own stretch joins them as L o.  The flux score F = s (x_end - x_start)_a changes by
// s (gx tx)_a for each stored shift tx.
template <typename R>
struct PathCtx {
    R gx[3][3], go[3][3], gb[3];      // [component][column]
    R tx[MCBTE_PATH_MAX][3];          // stored shifts, one per finished flight
    int tbin[MCBTE_PATH_MAX];         // frequency bin of each
    int nt;
    R dline;                          // straight distance since the last update (a periodic
                                      // transfer is a translation: the line goes on unchanged)

    __device__ __forceinline__ void begin_flight()
    {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                gx[i][c] = i == c ? R(1) : R(0);
                go[i][c] = R(0);
            }
            gb[i] = R(0);
        }
        dline = R(0);
    }
    // the segment x -> x + d o ended on a surface with unit normal n: the hit point stays on the
    // surface, n . (dx + dd o + d dO) = 0, and the flight has dd less distance left
    __device__ __forceinline__ void hit(const R o[3], R d, const R n[3])
    {
        const R on = o[0] * n[0] + o[1] * n[1] + o[2] * n[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R nx = n[0] * gx[0][c] + n[1] * gx[1][c] + n[2] * gx[2][c];
            const R no = n[0] * go[0][c] + n[1] * go[1][c] + n[2] * go[2][c];
            const R dd = -r_div(nx + d * no, on);
#pragma unroll
            for (int i = 0; i < 3; ++i) gx[i][c] = gx[i][c] + dd * o[i] + d * go[i][c];
            gb[c] = gb[c] - dd;
        }
    }
    // the segment x -> x + d o ended in a relaxation: fold the flight into the stored shifts and
    // store the flight's own stretch L o (its bin `bin`)
    __device__ __forceinline__ void end_flight(const R o[3], R d, R L, int bin)
    {
        R J[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) J[i][c] = gx[i][c] + o[i] * gb[c] + d * go[i][c];
#pragma unroll
        for (int q = 0; q < MCBTE_PATH_MAX; ++q) {
            if (q < nt) {
                const R a0 = tx[q][0], a1 = tx[q][1], a2 = tx[q][2];
#pragma unroll
                for (int i = 0; i < 3; ++i) tx[q][i] = J[i][0] * a0 + J[i][1] * a1 + J[i][2] * a2;
            } else if (q == nt) {
#pragma unroll
                for (int i = 0; i < 3; ++i) tx[q][i] = L * o[i];
                tbin[q] = bin;
            }
        }
        if (nt < MCBTE_PATH_MAX) ++nt;
        begin_flight();
    }
    // reflection off a plane normal to axis fa: specular negates that direction component,
    // diffuse draws a direction that does not depend on the hit point
    __device__ __forceinline__ void plane(int fa, bool specular)
    {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) go[i][c] = specular ? (i == fa ? -go[i][c] : go[i][c]) : R(0);
    }
    // specular reflection off a cylinder of radius r (o before the reflection): the normal turns
    // with the hit point, dn = (dx_h)_xy / r, and o' = o - 2 (o.n) n
    __device__ __forceinline__ void cyl_specular(const R o[3], const R n[3], R r)
    {
        const R on = o[0] * n[0] + o[1] * n[1] + o[2] * n[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R dn0 = r_div(gx[0][c], r), dn1 = r_div(gx[1][c], r);
            const R don = (go[0][c] * n[0] + go[1][c] * n[1] + go[2][c] * n[2]) + (o[0] * dn0 + o[1] * dn1);
            go[0][c] = go[0][c] - R(2) * don * n[0] - R(2) * on * dn0;
            go[1][c] = go[1][c] - R(2) * don * n[1] - R(2) * on * dn1;
            go[2][c] = go[2][c] - R(2) * don * n[2];
        }
    }
    // diffuse reflection off a cylinder (o after the reflection): o = mu n + a t1 + b t2 with the
    // drawn (mu, a, b) and the frame of dir_about, t1 = e_j x n / |e_j x n|, t2 = n x t1
    __device__ __forceinline__ void cyl_diffuse(const R o[3], const R n[3], R r)
    {
        int j = 0;
        R m0 = fabs(n[0]);
        if (fabs(n[1]) < m0) { j = 1; m0 = fabs(n[1]); }
        if (fabs(n[2]) < m0) j = 2;
        const R e0 = j == 0 ? R(1) : R(0), e1 = j == 1 ? R(1) : R(0), e2 = j == 2 ? R(1) : R(0);
        const R c0 = e1 * n[2] - e2 * n[1], c1 = e2 * n[0] - e0 * n[2], c2 = e0 * n[1] - e1 * n[0];
        const R len = r_sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        const R t1[3] = {r_div(c0, len), r_div(c1, len), r_div(c2, len)};
        const R t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
        const R mu = o[0] * n[0] + o[1] * n[1] + o[2] * n[2];
        const R ca = o[0] * t1[0] + o[1] * t1[1] + o[2] * t1[2];
        const R cb = o[0] * t2[0] + o[1] * t2[1] + o[2] * t2[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R dn[3] = {r_div(gx[0][c], r), r_div(gx[1][c], r), R(0)};
            const R dc[3] = {e1 * dn[2] - e2 * dn[1], e2 * dn[0] - e0 * dn[2], e0 * dn[1] - e1 * dn[0]};
            const R p1 = t1[0] * dc[0] + t1[1] * dc[1] + t1[2] * dc[2];
            R dt1[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) dt1[i] = r_div(dc[i] - p1 * t1[i], len);
            const R dt2[3] = {(dn[1] * t1[2] - dn[2] * t1[1]) + (n[1] * dt1[2] - n[2] * dt1[1]),
                              (dn[2] * t1[0] - dn[0] * t1[2]) + (n[2] * dt1[0] - n[0] * dt1[2]),
                              (dn[0] * t1[1] - dn[1] * t1[0]) + (n[0] * dt1[1] - n[1] * dt1[0])};
#pragma unroll
            for (int i = 0; i < 3; ++i) go[i][c] = mu * dn[i] + ca * dt1[i] + cb * dt2[i];
        }
    }
    // the particle has ended: add s (gx tx)_a of every stored shift to its bin; a term that is not
    // finite (tangents grown without bound) is counted in `bad` instead
    __device__ __forceinline__ void flush(double* bins, int s, int a, uint32_t& bad)
    {
        const R r0 = a == 0 ? gx[0][0] : (a == 1 ? gx[1][0] : gx[2][0]);
        const R r1 = a == 0 ? gx[0][1] : (a == 1 ? gx[1][1] : gx[2][1]);
        const R r2 = a == 0 ? gx[0][2] : (a == 1 ? gx[1][2] : gx[2][2]);
#pragma unroll
        for (int q = 0; q < MCBTE_PATH_MAX; ++q) {
            if (q < nt) {
                const double c = (double)((R)s * (r0 * tx[q][0] + r1 * tx[q][1] + r2 * tx[q][2]));
                if (isfinite(c)) atomicAdd(bins + tbin[q], c);
                else ++bad;
            }
        }
    }
};

// Detector-grid scores of the pending segments of a sparse wave, for grids with one axis of more
// than one cell: the pieces of a segment lie between consecutive planes of that axis, each piece's
// bounds are the plane parameters tally_grid computes one after another, so the wave evaluates 64
// pieces per pass whichever lanes they belong to (a lone lane's flight across a 50-cell slab is
// one pass instead of 50 steps).  Same pieces, lengths, cells and values as tally_grid.
template <typename R>
__device__ __forceinline__ void grid_wave(const DevTab& T, const Hot<R>& H, const TallyCtx& tc, Part<R>& p)
{
    if (__ballot(p.sn > 0) == 0ull) return;
    const int lane = threadIdx.x & 63;
    const DevDet& D = T.det;
    int gn[3];
    R glo[3], ghi[3], gw[3], gsc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        gn[a] = D.n[a];
        glo[a] = Geo<R>::dlo(D, a);
        ghi[a] = Geo<R>::dhi(D, a);
        gw[a] = Geo<R>::dw(D, a);
        gsc[a] = Geo<R>::cell_scale(D, a);
    }
    const int mask = D.mask, ncomp = D.ncomp, n_cols = D.n_cols;
    uint32_t slots = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) slots |= ((uint32_t)D.slot[q] & 0xFFu) << (8 * q);
    const int A = H.grid_axis;
    const int nA = A == 0 ? gn[0] : (A == 1 ? gn[1] : gn[2]);
    const R loA = A == 0 ? glo[0] : (A == 1 ? glo[1] : glo[2]);
    const R wA = A == 0 ? gw[0] : (A == 1 ? gw[1] : gw[2]);
    // this lane's segment: the part inside the grid [s_lo, s_hi], its first plane j0 and the
    // number of planes P it crosses (pieces: P + 1)
    R s_lo = R(0), s_hi = R(0);
    int j0 = 0, c = 0;
    if (p.sn > 0) {
        const R d = p.st0;
        bool in = d > R(0);
        s_hi = d;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (gn[a] <= 0) continue;
            if (p.so[a] == R(0)) {
                if (p.sx[a] < glo[a] || p.sx[a] > ghi[a]) in = false;
            } else {
                R s1 = r_div(glo[a] - p.sx[a], p.so[a]);
                R s2 = r_div(ghi[a] - p.sx[a], p.so[a]);
                if (s1 > s2) { const R tt = s1; s1 = s2; s2 = tt; }
                if (s1 > s_lo) s_lo = s1;
                if (s2 < s_hi) s_hi = s2;
            }
        }
        if (in && s_hi > s_lo) {
            const R xA = A == 0 ? p.sx[0] : (A == 1 ? p.sx[1] : p.sx[2]);
            const R oA = A == 0 ? p.so[0] : (A == 1 ? p.so[1] : p.so[2]);
            int P = 0;
            if (oA != R(0)) {
                const int dir = oA > R(0) ? 1 : -1;
                const R xs = xA + oA * s_lo;
                int ic = (int)floor((double)((xs - loA) / wA));
                ic = ic < 0 ? 0 : (ic > nA - 1 ? nA - 1 : ic);
                int j = ic + (dir > 0 ? 1 : 0);
                for (int it = 0; it < 4; ++it) {
                    const int jb = j - dir;
                    if (jb >= 1 && jb <= nA - 1 && r_div(loA + (R)jb * wA - xA, oA) > s_lo) j = jb;
                    else break;
                }
                for (int it = 0; it < 4; ++it) {
                    if (j >= 1 && j <= nA - 1 && !(r_div(loA + (R)j * wA - xA, oA) > s_lo)) j += dir;
                    else break;
                }
                j0 = j;
                const int Rn = (j >= 1 && j <= nA - 1) ? (dir > 0 ? nA - j : j) : 0;
                int lo = 0, hi = Rn;     // first plane of the run not before s_hi
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (r_div(loA + (R)(j0 + mid * dir) * wA - xA, oA) < s_hi) lo = mid + 1;
                    else hi = mid;
                }
                P = lo;
            }
            c = P + 1;
        }
    }
    int S = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(S, off, 64);
        if (lane >= off) S += t;
    }
    const int total = __shfl(S, 63, 64);
    for (int base = 0; base < total; base += 64) {
        const int g = base + lane;
        int own = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
            const int cc = own + step - 1;
            if (__shfl(S, cc < 63 ? cc : 63, 64) <= g) own += step;
        }
        own = own < 63 ? own : 63;
        const int cnt_own = __shfl(c, own, 64);
        const int q = g - (__shfl(S, own, 64) - cnt_own);       // piece index within the segment
        R x0[3], o[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            x0[a] = lane_r<R>(p.sx[a], own);
            o[a] = lane_r<R>(p.so[a], own);
        }
        const R lo_s = lane_r<R>(s_lo, own), hi_s = lane_r<R>(s_hi, own), vm = lane_r<R>(p.svm, own);
        const int jj = __shfl(j0, own, 64), m = __shfl(p.sk0, own, 64);
        const R sg = (R)__shfl(p.s, own, 64);
        if (g < total) {
            const R xA = A == 0 ? x0[0] : (A == 1 ? x0[1] : x0[2]);
            const R oA = A == 0 ? o[0] : (A == 1 ? o[1] : o[2]);
            const int dir = oA > R(0) ? 1 : -1;
            const int P = cnt_own - 1;
            const R s_a = q == 0 ? lo_s : r_div(loA + (R)(jj + (q - 1) * dir) * wA - xA, oA);
            const R s_b = q == P ? hi_s : r_div(loA + (R)(jj + q * dir) * wA - xA, oA);
            const R l = s_b - s_a;
            if (l > R(0)) {
                const R mid = R(0.5) * (s_a + s_b);
                int64_t cell = 0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int n = gn[a] > 0 ? gn[a] : 1;
                    int64_t ci = 0;
                    if (gn[a] > 0) {
                        const R xa = x0[a] + o[a] * mid;
                        const R f = Geo<R>::cellf_of(xa, glo[a], gsc[a]);
                        ci = (int64_t)f;
                        ci = ci < 0 ? 0 : (ci > n - 1 ? n - 1 : ci);
                    }
                    cell = cell * n + ci;
                }
                add4_c(tc, mask, ncomp, slots, cell * n_cols + m, sg, l, vm, o);
            }
        }
    }
    p.sn = 0;
}

// The segments of a lane that is the last one live in its wave, up to its next event that is
// neither a transfer through a periodic face nor a diffuse or specular reflection off the pore
// (these leave the mode and the remaining flight as they were): the faces the ray moves toward
// are fixed while the direction is, so the loop keeps only positions, times, the direction and
// the particle's scores, and the steady tally terms (one mode throughout) are summed here and
// added once.  Every quantity is computed as the one-segment step computes it, so the trajectory is the
// same; the next event (found again by the caller) is left to that step.  Lanes that share a wave
// take one segment per trace-loop pass instead, so that a long chain in one lane does not hold up
// the others.  Returns true if the particle left the box on the way (the caller ends it).
template <typename R>
__device__ __forceinline__ bool lone_chain(const Hot<R>& H, const TallyCtx& tc, const Stream& st, Part<R>& p,
                                           LaneCounts& cnt, R vm, R sg, uint32_t pcls)
{
    if (H.n_pores > 1) return false;
    // pcls: the pore's reflection class for this phonon
    const bool pore_walk = H.n_pores == 1 && pcls != SURF_PARTIAL;
    bool ok[3], up[3], per[3];
    int fid[3];
    R os, qa;
    // the faces the ray moves toward, fixed while the direction is
    auto aim = [&]() {
        bool any = pore_walk;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const R oa = p.o[a];
            up[a] = oa > R(0);
            ok[a] = ((H.unb >> a) & 1u) == 0u && (up[a] | (oa < R(0)));
            fid[a] = face_id(a, up[a] ? 1 : 0);
            per[a] = ((H.face >> (4 * (fid[a] - 1))) & 3u) == 3u;
            any = any | (ok[a] & per[a]);
        }
        const int sa = H.score_axis;
        os = sa == 0 ? p.o[0] : (sa == 1 ? p.o[1] : p.o[2]);
        qa = p.o[0] * p.o[0] + p.o[1] * p.o[1];
        return any;
    };
    if (!aim()) return false;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    uint32_t n = 0;
    bool escaped = false;
    for (;;) {
        if (p.k >= (uint32_t)H.max_events) break;
        const R ds = vm * p.dtr;
        R db = R(1) / R(0);
        int hit = 0, ax = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const R d = r_div(up[a] ? H.L[a] - p.x[a] : R(0) - p.x[a], p.o[a]);
            const bool better = ok[a] & ((d < db) | ((d == db) & (fid[a] < hit)));
            db = better ? d : db;
            hit = better ? fid[a] : hit;
            ax = better ? a : ax;
        }
        bool at_pore = false;
        if (H.n_pores == 1) {
            const R dx = p.x[0] - H.p0cx, dy = p.x[1] - H.p0cy, rr = H.p0r;
            const R qb = dx * p.o[0] + dy * p.o[1];
            const R qc = dx * dx + dy * dy - rr * rr;
            const R disc = qb * qb - qa * qc;
            const R d = (qc < R(0)) ? R(0) : r_div(qc, -qb + r_sqrt(disc >= R(0) ? disc : R(0)));
            at_pore = (qb < R(0)) & (disc >= R(0)) & (d < db);
            db = at_pore ? d : db;
        }
        // a transfer through a periodic face, or a reflection off the pore (diffuse or specular),
        // before the flight ends; anything else is left to the one-segment step
        const bool go = (db <= ds) & (at_pore ? pore_walk : ((hit > 0) & (ax == 0 ? per[0] : (ax == 1 ? per[1] : per[2]))));
        if (!go) break;
        const R d = db;
        const R dt = r_div(d, vm);
        if (d > R(0)) {
            acc[0] += (double)(sg * r_div(d, vm));
            acc[1] += (double)(sg * (d * p.o[0]));
            acc[2] += (double)(sg * (d * p.o[1]));
            acc[3] += (double)(sg * (d * p.o[2]));
        }
        p.cT += (double)(sg * r_div(d, vm));
        p.cq += (double)(sg * (d * os));
        ++cnt.c[1];
#pragma unroll
        for (int a = 0; a < 3; ++a) p.x[a] = p.x[a] + d * p.o[a];
        p.t = p.t + dt;
        const R r = p.dtr - dt;
        p.dtr = r > R(0) ? r : R(0);
        p.k += 1;
        ++n;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const R L = H.L[a];
            if (!at_pore && a == ax) p.x[a] = up[a] ? L : R(0);    // exactly on the face
            if (!((H.unb >> a) & 1u) && (p.x[a] < R(-1e-9) * L || p.x[a] > L + R(1e-9) * L)) escaped = true;
        }
        if (escaped) break;
        if (!at_pore) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (a == ax) p.x[a] = up[a] ? R(0) : H.L[a];   // reinserted at the partner face
            ++cnt.c[5];
            continue;
        }
        // reflection off the pore, as the one-segment step makes it
        const R n0 = r_div(p.x[0] - H.p0cx, H.p0r), n1 = r_div(p.x[1] - H.p0cy, H.p0r);
        if (pcls == SURF_DIFFUSE) {
            p.j += 1;
            const W4 w1 = st.block(2u * (2u + p.j) + 1u);
            const R u1 = unif<R>(w1.x, w1.y), u2 = unif<R>(w1.z, w1.w);
            const R mu = r_sqrt(u1), sth = r_sqrt(R(1) - u1);
            R sn, cs;
            r_sincos_2pi(u2, &sn, &cs);
            const R n[3] = {n0, n1, R(0)};
            dir_about(mu, sth * cs, sth * sn, n, p.o);
            ++cnt.c[4];
        } else {
            const R k2 = R(2) * (p.o[0] * n0 + p.o[1] * n1 + p.o[2] * R(0));
            p.o[0] = p.o[0] - k2 * n0;
            p.o[1] = p.o[1] - k2 * n1;
            p.o[2] = p.o[2] - k2 * R(0);
            ++cnt.c[3];
        }
        aim();
    }
    if (n > 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if ((H.det_mask >> q) & 1) tadd_c(tc, H.det_ncomp, H.det_slot, (int64_t)p.m, q, acc[q]);
    }
    return escaped;
}

// A phonon on a film wall, just reflected specularly, whose walls reflect it specularly: until its
// free path runs out it crosses the film wall to wall, each crossing a chord L / |Omega_a| long
// with the film-axis direction flipped at every wall.  The n complete crossings are run at once:
// the in-plane coordinates and scores advance by n chords along the unchanged in-plane direction,
// the film-axis score by the net displacement between the walls (L for an odd n, else 0), n
// specular reflections and n segments are counted, and the particle is left on the wall it reaches
// with the last partial segment to the one-segment step.  The lengths are taken in FP64 (the
// remaining path is a small difference of large numbers).  The segment cap stays with the step.
template <typename R>
__device__ __forceinline__ void fold_crossings(const Hot<R>& H, const TallyCtx& tc, Part<R>& p, LaneCounts& cnt,
                                               R vm, R sg, int fa)
{
    // (scalars and selects only: a local array indexed at run time would live in scratch memory)
    const R Lf = fa == 0 ? H.L[0] : (fa == 1 ? H.L[1] : H.L[2]);
    const double L = (double)Lf;
    const double o0 = (double)p.o[0], o1 = (double)p.o[1], o2 = (double)p.o[2];
    const double oa = fa == 0 ? o0 : (fa == 1 ? o1 : o2);
    const double chord = L / fabs(oa);
    const double lam = (double)vm * (double)p.dtr;
    double nd = floor(lam / chord);
    const double room = (double)H.max_events - (double)p.k - 1.0;
    nd = nd < room ? nd : room;
    if (!(nd >= 1.0)) return;
    const uint32_t n = (uint32_t)nd;
    const double len = nd * chord;
    const bool odd = (n & 1u) != 0u;
    const double dfa = odd ? (oa > 0.0 ? L : -L) : 0.0;     // net film-axis displacement
    const double q0 = fa == 0 ? dfa : len * o0, q1 = fa == 1 ? dfa : len * o1, q2 = fa == 2 ? dfa : len * o2;
    const double s = (double)sg;
    const double tT = s * (len / (double)vm);
    const int mask = H.det_mask;
    if (mask & 1) tadd_c(tc, H.det_ncomp, H.det_slot, (int64_t)p.m, 0, tT);
    if (mask & 2) tadd_c(tc, H.det_ncomp, H.det_slot, (int64_t)p.m, 1, s * q0);
    if (mask & 4) tadd_c(tc, H.det_ncomp, H.det_slot, (int64_t)p.m, 2, s * q1);
    if (mask & 8) tadd_c(tc, H.det_ncomp, H.det_slot, (int64_t)p.m, 3, s * q2);
    p.cT += tT;
    p.cq += s * (H.score_axis == 0 ? q0 : (H.score_axis == 1 ? q1 : q2));
    const bool at_far = (fa == 0 ? p.x[0] : (fa == 1 ? p.x[1] : p.x[2])) > R(0.5) * Lf;
    const R wall = (at_far != odd) ? Lf : R(0);
    p.x[0] = fa == 0 ? wall : (R)((double)p.x[0] + q0);
    p.x[1] = fa == 1 ? wall : (R)((double)p.x[1] + q1);
    p.x[2] = fa == 2 ? wall : (R)((double)p.x[2] + q2);
    if (odd) {
        p.o[0] = fa == 0 ? -p.o[0] : p.o[0];
        p.o[1] = fa == 1 ? -p.o[1] : p.o[1];
        p.o[2] = fa == 2 ? -p.o[2] : p.o[2];
    }
    p.dtr = (R)((lam - len) / (double)vm);
    p.t = (R)((double)p.t + len / (double)vm);
    p.k += n;
    cnt.c[1] += n;
    cnt.c[3] += n;
}

// Advance particle p by one segment; returns true when the particle has ended.  With `chain`
// set (the lane is the last one of its wave still tracing), the periodic transfers and pore
// reflections ahead of it run first in lone_chain; with `spread` set (a sparse wave), a
// detector-grid segment is left to grid_wave.
// AK: 0 trace, 1 likelihood-ratio replay, 2 pathwise replay, 3 local pathwise replay.
template <typename R, int TK, int AK, int FT>
__device__ __forceinline__ bool flight(const DevTab& T, const Hot<R>& H, const Tabs<R>& tb, const TallyCtx& tc,
                                       const Stream& st, Part<R>& p, LaneCounts& cnt, LogRow& lg, bool& coop,
                                       AdjCtx& adj, PathCtx<R>& pc, bool chain, bool spread = false)
{
    const DevGeom& g = T.g;
    const R vm = tb.v[p.m];
    const R sg = (R)p.s;
    int hit, pore, ev, fa, fs;
    int wall = -1;                       // the line wall hit (-1: none)
    R pcx, pcy, pr;                      // centre and radius of the pore hit
    uint32_t fcode;
    // the extended physics (two-phonon clock, specular cutoff frequencies) is compiled in
    constexpr bool EXT = (FT & FT_PLAIN) == 0;
    if (EXT && T.two) resolve_clocks<R>(T, st, p);
    if constexpr ((FT & FT_LATTICE) != 0) {
        // pore lattice: a long free path ahead is walked from pore to pore by the whole wave
        // (lattice_walk), unless the last walk left the particle where it is
        if (p.kc != p.k && vm * p.dtr > H.lat_min) {
            uint32_t pc0 = H.pcls & 3u;
            if (EXT && T.spec_w && g.pore_tab[0] > 0) pc0 = tab_class<R>(T, g.pore_tab[0], p.m);
            if (pc0 != SURF_PARTIAL) {
                coop = true;
                return false;
            }
        }
    }
    if constexpr (TK == TALLY_STEADY_ONE && AK != 2 && (FT & FT_LOG) == 0) {
        if (chain && !(EXT && g.n_walls > 0)) {   // (the lone-lane walk knows faces and pores)
            uint32_t pc0 = H.pcls & 3u;      // the first pore's reflection class for this phonon
            if (EXT && T.spec_w && H.n_pores == 1 && g.pore_tab[0] > 0) pc0 = tab_class<R>(T, g.pore_tab[0], p.m);
            if (lone_chain<R>(H, tc, st, p, cnt, vm, sg, pc0)) {   // left the box on the way
                ++cnt.c[10];
                if (AK == 1 || (AK == 3 && !local_form<AK>(T, p.m, adj)))
                    adj.add(T.bin_of[p.m], (double)(p.dtr0 - p.dtr) / T.tau64[p.m], adj.F_total - p.F0);
                return true;
            }
        }
    }
    for (;;) {
        if (p.k >= (uint32_t)H.max_events) {
            ++cnt.c[9];
            lg.put(EV_CAP, 0, p.m);
            if (AK == 1 || (AK == 3 && !local_form<AK>(T, p.m, adj)))
                adj.add(T.bin_of[p.m], (double)(p.dtr0 - p.dtr) / T.tau64[p.m], adj.F_total - p.F0);
            if (AK == 2) pc.flush(adj.bins, p.s, H.score_axis, adj.bad);
            return true;
        }
        const R ds = vm * p.dtr;
        // nearest boundary along the ray: faces in id order, then pores; ties keep the lower id
        R db = R(1) / R(0);
        hit = 0;
        pore = -1;
        wall = -1;
        pcx = R(0);
        pcy = R(0);
        pr = R(1);
        // (evaluated without branches: per axis the one face the ray moves toward, then the
        // lexicographic minimum of (distance, id), which is the id-order scan's first minimum)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const R oa = p.o[a];
            const bool up = oa > R(0);
            // (bitwise rather than short-circuit logic: selects, no branches)
            const bool valid = ((H.unb >> a) & 1u) == 0u && (up | (oa < R(0)));
            const R d = r_div(up ? H.L[a] - p.x[a] : R(0) - p.x[a], oa);
            const int id = face_id(a, up ? 1 : 0);
            const bool better = valid & ((d < db) | ((d == db) & (id < hit)));
            db = better ? d : db;
            hit = better ? id : hit;
        }
        for (int c = 0; c < H.n_pores; ++c) {
            R cx = H.p0cx, cy = H.p0cy, rr = H.p0r;
            int id = H.p0id;
            if (c > 0) {
                const auto P = Geo<R>::pore(g, c);
                cx = P.cx;
                cy = P.cy;
                rr = P.r;
                id = P.id;
            }
            const R dx = p.x[0] - cx, dy = p.x[1] - cy;
            const R qa = p.o[0] * p.o[0] + p.o[1] * p.o[1];
            const R qb = dx * p.o[0] + dy * p.o[1];
            const R qc = dx * dx + dy * dy - rr * rr;
            const R disc = qb * qb - qa * qc;
            // the ray meets the circle while approaching its centre: qb < 0, disc >= 0
            const bool meets = (qb < R(0)) & (disc >= R(0));
            const R d = (qc < R(0)) ? R(0) : r_div(qc, -qb + r_sqrt(disc >= R(0) ? disc : R(0)));
            const bool better = meets & (d < db);
            db = better ? d : db;
            hit = better ? id : hit;
            pore = better ? c : pore;
            pcx = better ? cx : pcx;
            pcy = better ? cy : pcy;
            pr = better ? rr : pr;
        }
        if constexpr (EXT) {
            // internal line walls (ids after the pores'), met from the side their normal points
            // to: x + d o = P1 + s (P2 - P1) in the x-y plane, d >= 0, 0 <= s <= 1
            for (int k = 0; k < g.n_walls; ++k) {
                const WallR<R> w = wall_of<R>(g, k);
                const R on = p.o[0] * w.nx + p.o[1] * w.ny;
                const R ex = w.x2 - w.x1, ey = w.y2 - w.y1;
                const R den = p.o[0] * ey - p.o[1] * ex;
                const R wx = w.x1 - p.x[0], wy = w.y1 - p.x[1];
                const R d = r_div(wx * ey - wy * ex, den);
                const R sp = r_div(wx * p.o[1] - wy * p.o[0], den);
                const bool better = (on < R(0)) & (den != R(0)) & (d >= R(0)) & (sp >= R(0)) & (sp <= R(1)) & (d < db);
                db = better ? d : db;
                hit = better ? g.wall_id[k] : hit;
                wall = better ? k : wall;
                pore = better ? -1 : pore;
            }
        }
        // event: the time horizon first, then the boundary (segment (x0, x1]), then relaxation
        const R dmin = db < ds ? db : ds;
        const R tmax = H.t_max;
        R d;
        if (H.transient && vm * (tmax - p.t) <= dmin) { ev = 2; d = vm * (tmax - p.t); }
        else if (db <= ds) { ev = 1; d = db; }
        else { ev = 0; d = ds; }
        const R dt = (ev == 0) ? p.dtr : (ev == 1 ? r_div(d, vm) : tmax - p.t);
        const R t_end = (ev == 2) ? tmax : p.t + dt;
        if (TK == TALLY_TRANSIENT) {
            snap_pend<R>(tb.tmeas, T.n_times, T.tm_guide, std::is_same<R, float>::value ? (R)T.tm_gs32 : (R)T.tm_gs64,
                         p, t_end, vm);
        } else {
            if (TK == TALLY_STEADY_ONE) {
                if (d > R(0)) add4_c(tc, H.det_mask, H.det_ncomp, H.det_slot, (int64_t)p.m, sg, d, vm, p.o);
            } else {
                if (spread && H.grid_axis >= 0) {   // the wave scores the pieces after the step
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        p.sx[a] = p.x[a];
                        p.so[a] = p.o[a];
                    }
                    p.st0 = d;
                    p.svm = vm;
                    p.sk0 = p.m;
                    p.sn = 1;
                } else {
                    tally_grid(T, tc, p.x, p.o, d, p.m, sg, vm);
                }
            }
            const int sa = H.score_axis;
            const R os = sa == 0 ? p.o[0] : (sa == 1 ? p.o[1] : p.o[2]);
            p.cT += (double)(sg * r_div(d, vm));
            p.cq += (double)(sg * (d * os));
        }
        ++cnt.c[1];
#pragma unroll
        for (int a = 0; a < 3; ++a) p.x[a] = p.x[a] + d * p.o[a];
        p.t = t_end;
        if (ev == 1) {
            const R r = p.dtr - dt;
            p.dtr = r > R(0) ? r : R(0);
        } else {
            p.dtr = R(0);
        }
        p.k += 1;
        if (ev == 2) {
            ++cnt.c[7];
            lg.put(EV_TIMEOUT, 0, p.m);
            if (AK == 1 || (AK == 3 && !local_form<AK>(T, p.m, adj)))
                adj.add(T.bin_of[p.m], (double)(p.dtr0 - p.dtr) / T.tau64[p.m], adj.F_total - p.F0);
            if (AK == 2) pc.flush(adj.bins, p.s, H.score_axis, adj.bad);
            return true;
        }
        const bool on_face = (ev == 1) && hit <= 6;
        fa = on_face ? face_axis(hit - 1) : -1;
        fs = on_face ? face_side(hit - 1) : 0;
        bool escaped = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const R L = H.L[a];
            if (a == fa) p.x[a] = fs ? L : R(0);     // exactly on the wall
            if (!(H.unb & (1u << a)) && (p.x[a] < R(-1e-9) * L || p.x[a] > L + R(1e-9) * L)) escaped = true;
        }
        fcode = on_face ? (H.face >> (4 * (hit - 1))) & 15u : 0u;
        const bool periodic = on_face && (fcode & 3u) == 3u;
        if (AK == 2) {   // the segment's end, for the pathwise state
            const R dl = pc.dline + d;
            pc.dline = R(0);
            if (ev == 0) {
                pc.end_flight(p.o, dl, vm * p.dtr0, T.bin_of[p.m]);
            } else if (periodic) {
                pc.dline = dl;
            } else if (ev == 1) {
                R nh[3] = {R(0), R(0), R(0)};
                if (hit <= 6) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) nh[a] = a == fa ? R(1) : R(0);
                } else {
                    nh[0] = r_div(p.x[0] - pcx, pr);
                    nh[1] = r_div(p.x[1] - pcy, pr);
                }
                pc.hit(p.o, dl, nh);
            }
        }
        if (escaped) {
            ++cnt.c[10];
            lg.put(EV_ESCAPE, 0, p.m);
            if (AK == 1 || (AK == 3 && !local_form<AK>(T, p.m, adj)))
                adj.add(T.bin_of[p.m], (double)(p.dtr0 - p.dtr) / T.tau64[p.m], adj.F_total - p.F0);
            if (AK == 2) pc.flush(adj.bins, p.s, H.score_axis, adj.bad);
            return true;
        }
        if (!periodic) break;
        // linearised periodic condition: reinsert unchanged at the partner face
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (a == fa) p.x[a] = fs ? R(0) : H.L[a];
        ++cnt.c[5];
        lg.put(EV_PERIODIC, hit, p.m);
        return false;
    }
    // what the event needs: the free flight's end is a two-phonon scattering when that clock
    // is the earlier one, else a three-phonon relaxation
    bool two_ev = false;
    bool relax = (ev == 0);
    if (EXT && relax && T.two && signbit(p.lead)) {
        relax = false;
        two_ev = true;
    }
    if (relax) {
        p.nrel += 1;
        ++cnt.c[2];
        if (AK == 3 && local_form<AK>(T, p.m, adj)) {
            const int sa = H.score_axis;
            const double os = (double)(sa == 0 ? p.o[0] : (sa == 1 ? p.o[1] : p.o[2]));
            atomicAdd(adj.bins + T.bin_of[p.m], (double)p.s * (T.v64[p.m] * (double)p.dtr0) * os);
            adj.add(T.bin_of[p.m], (double)p.dtr0 / T.tau64[p.m] - 1.0, adj.F_total - p.cq);
        } else if (AK == 1 || AK == 3) {
            adj.add(T.bin_of[p.m], (double)p.dtr0 / T.tau64[p.m] - 1.0, adj.F_total - p.F0);
        }
        if (H.n_scat_max > 0 && p.nrel >= H.n_scat_max) {
            ++cnt.c[8];
            lg.put(EV_NSCAT, 0, p.m);
            if (AK == 2) pc.flush(adj.bins, p.s, H.score_axis, adj.bad);
            return true;
        }
    }
    uint32_t cls = SURF_DIFFUSE;
    int64_t tab_i = -1;                  // the boundary's per-row table entry for this phonon (-1: none)
    if (ev == 1) {
        int btype;
        if (hit <= 6) {
            btype = (int)(fcode & 3u);
            cls = fcode >> 2;
        } else if (EXT && wall >= 0) {
            btype = g.wall_type[wall];
            cls = (g.wall_cls[Geo<R>::prec] >> (2 * wall)) & 3u;
        } else {
            btype = 2;
            cls = (H.pcls >> (2 * pore)) & 3u;
        }
        // specularity per phonon (a cutoff frequency is a table too): the row's class and threshold
        if (EXT && T.spec_w && btype == 2) {
            const int tab = hit <= 6 ? g.face_tab[hit - 1] : (wall >= 0 ? g.wall_tab[wall] : g.pore_tab[pore]);
            if (tab > 0) {
                tab_i = (int64_t)(tab - 1) * H.M + p.m;
                cls = tab_class<R>(T, tab, p.m);
            }
        }
        if (btype == 1) {
            ++cnt.c[6];
            lg.put(EV_ABSORB, hit, p.m);
            if (AK == 1 || (AK == 3 && !local_form<AK>(T, p.m, adj)))
                adj.add(T.bin_of[p.m], (double)(p.dtr0 - p.dtr) / T.tau64[p.m], adj.F_total - p.F0);
            if (AK == 2) pc.flush(adj.bins, p.s, H.score_axis, adj.bad);
            return true;
        }
    }
    // film-like problem: a diffuse reflection off the film wall with a long free path left is
    // handed to the whole wave, which runs the coming bounces 64 at a time (coop_bounces for the
    // FP32 trajectories, which it does not log; coop_exact for the FP64 ones)
    // (FP32 trace: also walls that reflect this phonon partly specularly, the same on both walls)
    constexpr bool COOP = std::is_same<R, float>::value || (FT & FT_COOP) != 0;
    if (COOP && ev == 1 && fa >= 0 && (std::is_same<R, double>::value || !lg.row) && vm * p.dtr > H.coop_min &&
        ((cls == SURF_DIFFUSE && fa == H.coop_axis) ||
         (std::is_same<R, float>::value && EXT && cls == SURF_PARTIAL && fa == H.fold_axis))) {
        if (AK == 2) pc.plane(fa, false);    // the chain starts with a diffuse reflection
        coop = true;
        return false;
    }
    const bool adia = (ev == 1);
    const bool partial = adia && cls == SURF_PARTIAL;
    const bool need_b0 = relax || partial;
    const bool need_rec = need_b0 || two_ev || (adia && cls == SURF_DIFFUSE);
    if (need_rec) p.j += 1;
    const uint32_t blk = 2u * (2u + p.j);
    W4 w0 = {0u, 0u, 0u, 0u};
    if (need_b0) w0 = st.block(blk);
    bool specular = adia && cls == SURF_SPECULAR;
    if (partial)
        specular = key64(w0.x, w0.y) <
                   ((EXT && tab_i >= 0) ? T.spec_thr[tab_i]
                                        : (pore >= 0 ? g.pore_thr[pore] : ((EXT && wall >= 0) ? g.wall_thr[wall] : g.face_thr[hit - 1])));
    const bool diffuse = adia && !specular;
    if (relax || diffuse || two_ev) {
        const W4 w1 = st.block(blk + 1u);
        const R u1 = unif<R>(w1.x, w1.y), u2 = unif<R>(w1.z, w1.w);
        // the new direction's polar cosine mu and sine about its axis: isotropic for a relaxation
        // (axis e_z, mu = 1 - 2 u1), cosine-weighted about the inward normal for a diffuse wall
        // (mu = sqrt(u1)); one azimuth 2 pi u2 serves both (dir_iso and dir_cos, shared by the
        // lanes of a wave that do different ones)
        const R mu_i = R(1) - R(2) * u1;
        const R s2 = (R(1) - mu_i) * (R(1) + mu_i);
        const bool iso = relax || two_ev;
        const R mu = iso ? mu_i : r_sqrt(u1);
        const R sth = r_sqrt(iso ? (s2 > R(0) ? s2 : R(0)) : R(1) - u1);
        R sn, cs;
        r_sincos_2pi(u2, &sn, &cs);
        if (relax) {
            // three-phonon relaxation: frequency from the post-scattering distribution
            // (weights C/tau), isotropic direction, new free flight, sign kept
            p.m = tb.guide ? cdf_pick_guided(tb.thr_rel, tb.guide, tb.gshift, H.M, H.last_rel, key64(w0.x, w0.y))
                           : cdf_pick(tb.thr_rel, H.M, H.last_rel, key64(w0.x, w0.y));
            p.o[0] = sth * cs;
            p.o[1] = sth * sn;
            p.o[2] = mu;
            p.dtr = -tb.tau[p.m] * r_log(R(1) - unif<R>(w0.z, w0.w));
            if (EXT && T.two) p.lead = R(NAN);   // both clocks redrawn: the two-phonon one next step
            lg.put(EV_RELAX, 0, p.m);
            if (AK != 0) {
                adj.add(T.bin_of[p.m], -1.0, adj.F_total - p.cq);
                adj.dense += adj.F_total - p.cq;
            }
            p.dtr0 = p.dtr;
            p.F0 = p.cq;
        } else if (two_ev) {
            // two-phonon scattering (section 3.5.1): the same phonon, a new isotropic direction and
            // a new two-phonon clock; the three-phonon clock runs on (its lead is what is left)
            p.o[0] = sth * cs;
            p.o[1] = sth * sn;
            p.o[2] = mu;
            p.dtr = -p.lead;
            p.lead = R(NAN);
            ++cnt.c[12];
            lg.put(EV_TWO, 0, p.m);
        } else {
            R n[3];
            if (pore >= 0) {
                n[0] = r_div(p.x[0] - pcx, pr);
                n[1] = r_div(p.x[1] - pcy, pr);
                n[2] = R(0);
            } else if (EXT && wall >= 0) {
                const WallR<R> w = wall_of<R>(g, wall);
                n[0] = w.nx;
                n[1] = w.ny;
                n[2] = R(0);
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a) n[a] = (a == fa) ? (fs ? R(-1) : R(1)) : R(0);
            }
            dir_about(mu, sth * cs, sth * sn, n, p.o);
            if (AK == 2) {
                if (pore >= 0) pc.cyl_diffuse(p.o, n, pr);
                else pc.plane(fa, false);
            }
            ++cnt.c[4];
            lg.put(EV_DIFFUSE, hit, p.m);
        }
    } else if (specular) {
        if (pore >= 0) {   // k' = k - 2 (k.n) n
            const R rr = pr;
            const R n0 = r_div(p.x[0] - pcx, rr);
            const R n1 = r_div(p.x[1] - pcy, rr);
            if (AK == 2) {
                const R nn[3] = {n0, n1, R(0)};
                pc.cyl_specular(p.o, nn, rr);
            }
            const R k2 = R(2) * (p.o[0] * n0 + p.o[1] * n1 + p.o[2] * R(0));
            p.o[0] = p.o[0] - k2 * n0;
            p.o[1] = p.o[1] - k2 * n1;
            p.o[2] = p.o[2] - k2 * R(0);
        } else if (EXT && wall >= 0) {
            const WallR<R> w = wall_of<R>(g, wall);
            const R k2 = R(2) * (p.o[0] * w.nx + p.o[1] * w.ny + p.o[2] * R(0));
            p.o[0] = p.o[0] - k2 * w.nx;
            p.o[1] = p.o[1] - k2 * w.ny;
            p.o[2] = p.o[2] - k2 * R(0);
        } else {
            if (AK == 2) pc.plane(fa, true);
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (a == fa) p.o[a] = -p.o[a];
        }
        ++cnt.c[3];
        lg.put(EV_SPECULAR, hit, p.m);
        // a film whose walls reflect this phonon specularly: its next wall-to-wall crossings until
        // the free path runs out, at once (FP32 trace)
        if constexpr (std::is_same<R, float>::value && AK == 0 && EXT) {
            if (fa >= 0 && fa == H.fold_axis && cls == SURF_SPECULAR && !lg.row && vm * p.dtr > H.coop_min)
                fold_crossings(H, tc, p, cnt, vm, sg, fa);
        }
    }
    return false;
}

__device__ __forceinline__ uint32_t wave_rank(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ------------------------------------------------------------------------------------------
// wave-cooperative bouncing in a film (FP32 form)
// ------------------------------------------------------------------------------------------

// The particle of lane `leader` sits on a wall of the film, about to be reflected diffusely or
// partly specularly, with remaining free path lam = v dt_rem.  Its next reflections draw the records
// the sequential loop would draw (record 2 + j + 1 + k for the k-th), and between two reflections
// it crosses the film wall to wall (chord L / |Omega_axis|), so 64 lanes evaluate 64 consecutive
// bounces at once: each lane decides its reflection (partly specular walls: the record's key
// against the threshold both walls share) and draws its direction (a diffuse one) or takes the
// in-plane direction and |Omega_axis| of the last diffuse reflection before it, pointed away from
// its wall (a specular one, which only flips the film-axis component); a prefix sum of the chords
// finds the bounce during which the free path runs out, and the completed segments are scored
// with one reduction.  The particle is handed back at the start of its last (partial) segment; the
// sequential loop then ends that segment with the relaxation.
// PART: partly specular walls are handled (compiled into the kernels with the extended physics)
template <typename R, bool PART>
__device__ __forceinline__ void coop_bounces(const DevTab& T, const Tabs<R>& tb, const TallyCtx& tc, Part<R>& p,
                                             const Stream& st_own, int leader, LaneCounts& cnt)
{
    const int lane = threadIdx.x & 63;
    const int aw = T.fold_axis;
    const R L = Geo<R>::L(T.g, aw);
    const int m = __shfl(p.m, leader, 64);
    const R sg = (R)__shfl(p.s, leader, 64);
    // the owner's random stream
    const Stream st{(uint32_t)__shfl((int)st_own.k0, leader, 64), (uint32_t)__shfl((int)st_own.k1, leader, 64),
                    (uint32_t)__shfl((int)st_own.plo, leader, 64), (uint32_t)__shfl((int)st_own.phi, leader, 64),
                    (uint32_t)__shfl((int)st_own.inst, leader, 64)};
    const R xw = __shfl(aw == 0 ? p.x[0] : (aw == 1 ? p.x[1] : p.x[2]), leader, 64);
    const int side = xw > R(0.5) * L ? 1 : 0;
    const uint32_t j0 = (uint32_t)__shfl((int)p.j, leader, 64);
    // the segment cap: the step caps the particle once its segment count reaches max_events, so at
    // most kcap more crossings complete (each one ends at a wall with the next reflection drawn)
    const uint32_t k0 = (uint32_t)__shfl((int)p.k, leader, 64);
    const uint32_t kcap = k0 < (uint32_t)T.max_events ? (uint32_t)T.max_events - k0 : 0u;
    // the walls' reflection class and partial threshold for this phonon (both walls read the same rule)
    bool partial = false;
    uint64_t thr = 0;
    if constexpr (PART) {
        const int fid = face_id(aw, 0) - 1;
        uint32_t cls = (T.g.face_code[Geo<R>::prec] >> (4 * fid + 2)) & 3u;
        thr = T.g.face_thr[fid];
        if (T.spec_w && T.g.face_tab[fid] > 0) {
            cls = tab_class<R>(T, T.g.face_tab[fid], m);
            thr = T.spec_thr[(int64_t)(T.g.face_tab[fid] - 1) * T.M + m];
        }
        partial = cls == SURF_PARTIAL;
    }
    const R vm = tb.v[m];
    double lam = (double)vm * (double)__shfl(p.dtr, leader, 64);
    const int sa = T.score_axis;
    double aT = 0.0, aQ0 = 0.0, aQ1 = 0.0, aQ2 = 0.0, acq = 0.0;
    R disp0 = R(0), disp1 = R(0), disp2 = R(0);
    uint32_t j = j0;
    uint32_t n_full = 0;       // this lane's completed segments
    uint32_t n_spec = 0, n_diff = 0;   // this lane's reflections
    int kstar = 64;
    R of0 = R(0), of1 = R(0), of2 = R(0);
    double lam_end = 0.0;
    // the direction a specular reflection starts from when no diffuse one precedes it in its chunk
    R c0 = __shfl(p.o[0], leader, 64), c1 = __shfl(p.o[1], leader, 64), c2 = __shfl(p.o[2], leader, 64);
    for (int chunk = 0; chunk < (1 << 24); ++chunk) {
        const int sk = side ^ (lane & 1);            // wall this lane's reflection happens at
        const uint32_t rec = 2u + j + 1u + (uint32_t)lane;
        bool spec = false;
        if (PART && partial) {
            const W4 w0 = st.block(2u * rec);
            spec = key64(w0.x, w0.y) < thr;
        }
        R o[3];
        if (!spec) {
            const W4 w1 = st.block(2u * rec + 1u);
            const R u1 = unif<R>(w1.x, w1.y), u2 = unif<R>(w1.z, w1.w);
            R n[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) n[a] = (a == aw) ? (sk ? R(-1) : R(1)) : R(0);
            dir_cos(u1, u2, n, o);
        }
        if (PART && partial) {
            // a specular lane takes the direction of the last diffuse lane at or before it
            const unsigned long long dm = __ballot(!spec);
            const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
            const unsigned long long below = dm & upto;
            const int src = below ? 63 - __clzll((long long)below) : 0;
            const R t0 = __shfl(o[0], src, 64), t1 = __shfl(o[1], src, 64), t2 = __shfl(o[2], src, 64);
            if (spec) {
                o[0] = below ? t0 : c0;
                o[1] = below ? t1 : c1;
                o[2] = below ? t2 : c2;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    if (a == aw) o[a] = sk ? -fabs(o[a]) : fabs(o[a]);
            }
            c0 = __shfl(o[0], 63, 64);
            c1 = __shfl(o[1], 63, 64);
            c2 = __shfl(o[2], 63, 64);
        }
        const R oz = aw == 0 ? o[0] : (aw == 1 ? o[1] : o[2]);
        const R len = oz != R(0) ? r_div(L, fabs(oz)) : R(1) / R(0);
        R P = len;                                   // inclusive prefix sum of the chords
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const R t = __shfl_up(P, off, 64);
            if (lane >= off) P += t;
        }
        const unsigned long long over = __ballot((double)P > lam || (j - j0) + (uint32_t)lane >= kcap);
        kstar = over ? __ffsll((long long)over) - 1 : 64;
        if (lane <= kstar) {                         // this lane's reflection happens
            n_spec += spec ? 1u : 0u;
            n_diff += spec ? 0u : 1u;
        }
        if (lane < kstar) {
            const R os = sa == 0 ? o[0] : (sa == 1 ? o[1] : o[2]);
            aT += (double)(sg * r_div(len, vm));
            aQ0 += (double)(sg * (len * o[0]));
            aQ1 += (double)(sg * (len * o[1]));
            aQ2 += (double)(sg * (len * o[2]));
            acq += (double)(sg * (len * os));
            disp0 += len * o[0];
            disp1 += len * o[1];
            disp2 += len * o[2];
            n_full += 1;
        }
        if (kstar < 64) {
            const R Pprev = __shfl(P, kstar > 0 ? kstar - 1 : 0, 64);
            lam_end = lam - (kstar > 0 ? (double)Pprev : 0.0);
            of0 = __shfl(o[0], kstar, 64);
            of1 = __shfl(o[1], kstar, 64);
            of2 = __shfl(o[2], kstar, 64);
            j += (uint32_t)kstar + 1u;
            break;
        }
        lam -= (double)__shfl(P, 63, 64);
        j += 64u;
    }
    const uint32_t full = wave_sum<uint32_t>(n_full);
    const uint32_t nspec = wave_sum<uint32_t>(n_spec), ndiff = wave_sum<uint32_t>(n_diff);
    const double sT = wave_sum<double>(aT), s0 = wave_sum<double>(aQ0), s1 = wave_sum<double>(aQ1),
                 s2 = wave_sum<double>(aQ2), scq = wave_sum<double>(acq);
    const R d0 = wave_sum<R>(disp0), d1 = wave_sum<R>(disp1), d2 = wave_sum<R>(disp2);
    if (lane == leader) {
        const DevDet& D = T.det;
        const int mask = D.mask;
        if (full > 0) {
            if (mask & 1) tadd(tc, D, (int64_t)m, 0, sT);
            if (mask & 2) tadd(tc, D, (int64_t)m, 1, s0);
            if (mask & 4) tadd(tc, D, (int64_t)m, 2, s1);
            if (mask & 8) tadd(tc, D, (int64_t)m, 3, s2);
        }
        p.cT += sT;
        p.cq += scq;
        const int side_end = side ^ (kstar & 1);
        p.x[0] = p.x[0] + d0;
        p.x[1] = p.x[1] + d1;
        p.x[2] = p.x[2] + d2;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (a == aw) p.x[a] = side_end ? L : R(0);
        p.o[0] = of0;
        p.o[1] = of1;
        p.o[2] = of2;
        p.dtr = (R)(lam_end / (double)vm);
        p.j = j;
        p.k += full;
        cnt.c[1] += full;              // completed segments
        cnt.c[3] += nspec;             // specular reflections
        cnt.c[4] += ndiff;             // diffuse reflections
    }
}

// value of v in lane k (k the same in every lane)
__device__ __forceinline__ double lane_value(double v, int k)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}

// Exact form of the cooperative bouncing for the FP64 trajectories.  A reflection's direction,
// the chord to the opposite wall, its flight time and its flux terms depend only on the
// reflection's own record and on the wall it starts from, so the lanes evaluate 64 consecutive
// reflections at once, each with the sequential loop's own arithmetic (the chord is the division
// the geometry step makes from the wall coordinate).  Where the walk stops is decided by the
// remaining flight time and the test against it alone: a wave prefix sum settles it whenever every
// test clears its rounding bound, the in-order recursion otherwise.  Then, in a loop with no exit,
// the sequential arithmetic for everything that carries over from one segment to the next
// (remaining time, position, time, the particle's scores) runs over the completed segments in
// order, then segment count and event log; the particle leaves the chain in exactly the state the
// one-segment-at-a-time loop reaches.  The tallies take each lane's terms (their summation order
// is free, as it is for the atomics).
__device__ __forceinline__ void coop_exact(const Hot<double>& H, const Tabs<double>& tb, const TallyCtx& tc,
                                           Part<double>& p, const Stream& st_own, int leader, LaneCounts& cnt,
                                           LogRow& lg)
{
    const int lane = threadIdx.x & 63;
    const int aw = H.coop_axis;
    const double L = aw == 0 ? H.L[0] : (aw == 1 ? H.L[1] : H.L[2]);
    const int m = __shfl(p.m, leader, 64);
    const double sg = (double)__shfl(p.s, leader, 64);
    const Stream st{(uint32_t)__shfl((int)st_own.k0, leader, 64), (uint32_t)__shfl((int)st_own.k1, leader, 64),
                    (uint32_t)__shfl((int)st_own.plo, leader, 64), (uint32_t)__shfl((int)st_own.phi, leader, 64),
                    (uint32_t)__shfl((int)st_own.inst, leader, 64)};
    const double x0 = __shfl(p.x[0], leader, 64), x1 = __shfl(p.x[1], leader, 64), x2 = __shfl(p.x[2], leader, 64);
    const int side0 = (aw == 0 ? x0 : (aw == 1 ? x1 : x2)) > 0.5 * L ? 1 : 0;
    // the in-plane axes b0 < b1 and the particle's coordinates along them (the coordinate along
    // the film axis is the wall's at every reflection)
    const int b0 = aw == 0 ? 1 : 0;
    double y0 = aw == 0 ? x1 : x0, y1 = aw == 2 ? x1 : x2;
    uint32_t j = (uint32_t)__shfl((int)p.j, leader, 64);
    uint32_t pk = (uint32_t)__shfl((int)p.k, leader, 64);
    double D = __shfl(p.dtr, leader, 64);
    double t = __shfl(p.t, leader, 64);
    double cT = __shfl(p.cT, leader, 64);
    double cq = __shfl(p.cq, leader, 64);
    const double vm = tb.v[m];
    const int sa = H.score_axis;
    int id0 = 0, id1 = 0;              // boundary ids of the faces at 0 and at L of the film axis
#pragma unroll
    for (int i = 0; i < 6; ++i)
        if (face_axis(i) == aw) {
            if (face_side(i)) id1 = i + 1;
            else id0 = i + 1;
        }
    double aT = 0.0, aQ0 = 0.0, aQ1 = 0.0, aQ2 = 0.0;
    uint32_t full = 0;
    uint32_t refl = 0;
    int side = side0;                  // wall of the current chunk's first reflection
    double o_end[3] = {0.0, 0.0, 0.0};
    for (int chunk = 0; chunk < (1 << 24); ++chunk) {
        const int sk = side ^ (lane & 1);
        const W4 w1 = st.block(2u * (2u + j + 1u + (uint32_t)lane) + 1u);
        const double u1 = unif<double>(w1.x, w1.y), u2 = unif<double>(w1.z, w1.w);
        double n[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) n[a] = (a == aw) ? (sk ? -1.0 : 1.0) : 0.0;
        double o[3];
        dir_cos(u1, u2, n, o);
        const double oa = aw == 0 ? o[0] : (aw == 1 ? o[1] : o[2]);
        double d = 1.0 / 0.0;
        if (sk ? oa < 0.0 : oa > 0.0) d = sk ? (0.0 - L) / oa : (L - 0.0) / oa;
        const double dt = d / vm;
        const double q0 = d * o[0], q1 = d * o[1], q2 = d * o[2];
        const double qs = sa == 0 ? q0 : (sa == 1 ? q1 : q2);
        const double r0 = aw == 0 ? q1 : q0, r1 = aw == 2 ? q1 : q2;   // in-plane displacements
        // the segment in which the free flight ends (or the event cap stops the walk): decided by
        // the remaining-time recursion D_k = D_(k-1) - dt_(k-1).  Each lane takes the prefix sum of
        // the earlier chords' times (tree order), which differs from the recursion by at most a
        // few hundred ulp of D + prefix; where every test up to the stop clears that by more, the
        // decisions are the recursion's, else the recursion itself is run in order
        const uint32_t cap_left = pk < (uint32_t)H.max_events ? (uint32_t)H.max_events - pk : 0u;
        const bool capped = (uint32_t)lane >= cap_left;
        double P = dt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double tt = __shfl_up(P, off, 64);
            if (lane >= off) P += tt;
        }
        double Pex = __shfl_up(P, 1, 64);
        if (lane == 0) Pex = 0.0;
        const double rhs = vm * (D - Pex);
        const unsigned long long stops = __ballot(capped || !(d <= rhs));
        int kstop = stops ? __ffsll((long long)stops) - 1 : 64;
        const double tol = 0x1p-45 * (vm * (D + Pex) + d);
        if (__ballot(!capped && lane <= kstop && !(fabs(d - rhs) > tol))) {
            kstop = 64;
            double Dk = D;
            for (int k = 0; k < 64; ++k) {
                if (pk + (uint32_t)k >= (uint32_t)H.max_events || !(lane_value(d, k) <= vm * Dk)) {
                    kstop = k;
                    break;
                }
                const double r = Dk - lane_value(dt, k);
                Dk = r > 0.0 ? r : 0.0;
            }
        }
        // the segments completed before it, in order: nothing in them ends the walk (every lane
        // holds the same kstop); the remaining time as the recursion computes it
        kstop = __builtin_amdgcn_readfirstlane(kstop);
        if (sa != aw) {                  // the scored flux is one of the in-plane displacements
            const bool s0 = sa == b0;
            for (int k = 0; k < kstop; ++k) {
                const double dtk = lane_value(dt, k), e0 = lane_value(r0, k), e1 = lane_value(r1, k);
                const double r = D - dtk;
                D = r > 0.0 ? r : 0.0;
                y0 = y0 + e0;
                y1 = y1 + e1;
                t = t + dtk;
                cT += sg * dtk;
                cq += sg * (s0 ? e0 : e1);
            }
        } else {
            for (int k = 0; k < kstop; ++k) {
                const double dtk = lane_value(dt, k);
                const double r = D - dtk;
                D = r > 0.0 ? r : 0.0;
                y0 = y0 + lane_value(r0, k);
                y1 = y1 + lane_value(r1, k);
                t = t + dtk;
                cT += sg * dtk;
                cq += sg * lane_value(qs, k);
            }
        }
        pk += (uint32_t)kstop;
        full += (uint32_t)kstop;
        if (lane < kstop) {              // each lane's own segment, if completed
            aT += sg * dt;
            aQ0 += sg * q0;
            aQ1 += sg * q1;
            aQ2 += sg * q2;
        }
        // every reflection up to the one that stopped the walk drew its record
        const int drawn = kstop < 64 ? kstop + 1 : 64;
        refl += (uint32_t)drawn;
        if (lane == leader && lg.row)
            for (int k = 0; k < drawn; ++k) lg.put(EV_DIFFUSE, (side ^ (k & 1)) ? id1 : id0, m);
        if (kstop < 64) {
            o_end[0] = __shfl(o[0], kstop, 64);
            o_end[1] = __shfl(o[1], kstop, 64);
            o_end[2] = __shfl(o[2], kstop, 64);
            side ^= (kstop & 1);
            j += (uint32_t)kstop + 1u;
            break;
        }
        j += 64u;                                        // 64 reflections: back on the same wall
    }
    const double sT = wave_sum<double>(aT), s0 = wave_sum<double>(aQ0), s1 = wave_sum<double>(aQ1),
                 s2 = wave_sum<double>(aQ2);
    if (lane == leader) {
        if (full > 0) {
            if (H.det_mask & 1) tadd_c(tc, H.det_ncomp, H.det_slot, (int64_t)m, 0, sT);
            if (H.det_mask & 2) tadd_c(tc, H.det_ncomp, H.det_slot, (int64_t)m, 1, s0);
            if (H.det_mask & 4) tadd_c(tc, H.det_ncomp, H.det_slot, (int64_t)m, 2, s1);
            if (H.det_mask & 8) tadd_c(tc, H.det_ncomp, H.det_slot, (int64_t)m, 3, s2);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p.x[a] = (a == aw) ? (side ? L : 0.0) : (a == b0 ? y0 : y1);
            p.o[a] = o_end[a];
        }
        p.t = t;
        p.dtr = D;
        p.j = j;
        p.k = pk;
        p.cT = cT;
        p.cq = cq;
        cnt.c[1] += full;              // completed segments
        cnt.c[4] += refl;              // diffuse reflections
    }
}

// ------------------------------------------------------------------------------------------
// wave-cooperative walk through a periodic lattice of pores (FP32 form)
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ float lane_f(float v, int k)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

// a wave-uniform decision from a condition every active lane evaluates alike
__device__ __forceinline__ bool wave_any(bool c) { return __builtin_amdgcn_ballot_w64(c) != 0ull; }

// A cell periodic in x and y (periodic or without faces in z) holding one z-axis pore tiles an
// infinite square lattice of pores, and a transfer through a periodic face -- the particle
// reinserted unchanged at the partner face (Eq. periodic_lin_final) -- is the same as flying on
// through that lattice.  The particle of lane `leader`, with a free path of many cells ahead, is
// followed by the whole wave from pore to pore in these unfolded coordinates:
//   - the lanes test the pores of a window of 64 cells ahead of the ray (32 x 2, 16 x 4 or 8 x 8
//     along the axis it moves fastest on, by its slope), and the nearest entry into a pore within
//     the free path (a DPP minimum) is the first pore met: a pore lies inside its cell and the
//     cells the ray passes form a staircase in its direction, so any pore met before the ray
//     leaves the window is in it; with none, the walk moves on to the window's far edge;
//   - a pore's discriminant is taken in Lagrange's form, qa r^2 - (dP x o)^2 (dP the pore's offset,
//     o the direction, in the x-y plane), so that a pore many cells away is decided from the cross
//     product's rounding rather than from a difference of squares of its distance;
//   - the transfers on the way are the cell boundaries crossed, counted per axis;
//   - the reflection uses the unit normal at the hit point (the hit point's offset from the axis,
//     normalized) and, for a diffuse one, the record the one-segment step would draw; the
//     records are drawn 64 at a time, one per lane (the polar and azimuthal cosines do not depend
//     on the hit point), and turned into the direction in the cylinder's frame (n, e_z x n, e_z);
//   - the walked segments' scores are the summed length and displacement (one mode, one sign);
//   - once the free path ends before the next pore, the particle is placed at its last face
//     crossing and the one-segment step makes the final segment.
// The events and their counts are the one-segment stepping's; positions and directions differ by
// rounding (a hit point is computed from its pore's centre instead of through the transfers before
// it, and the frame about the normal is written out for the cylinder).
template <int FT>
__device__ void lattice_walk(const DevTab& T, const Hot<float>& H, const Tabs<float>& tb, const TallyCtx& tc,
                             Part<float>& p, const Stream& st_own, int leader, LaneCounts& cnt)
{
    constexpr bool EXT = (FT & FT_PLAIN) == 0;
    const int lane = threadIdx.x & 63;
    leader = __builtin_amdgcn_readfirstlane(leader);
    const int m = __builtin_amdgcn_readlane(p.m, leader);
    const float sg = (float)__builtin_amdgcn_readlane(p.s, leader);
    const Stream st{(uint32_t)__builtin_amdgcn_readlane((int)st_own.k0, leader),
                    (uint32_t)__builtin_amdgcn_readlane((int)st_own.k1, leader),
                    (uint32_t)__builtin_amdgcn_readlane((int)st_own.plo, leader),
                    (uint32_t)__builtin_amdgcn_readlane((int)st_own.phi, leader),
                    (uint32_t)__builtin_amdgcn_readlane((int)st_own.inst, leader)};
    float x0 = lane_f(p.x[0], leader), x1 = lane_f(p.x[1], leader), x2 = lane_f(p.x[2], leader);
    float o0 = lane_f(p.o[0], leader), o1 = lane_f(p.o[1], leader), o2 = lane_f(p.o[2], leader);
    float dtr = lane_f(p.dtr, leader), t = lane_f(p.t, leader);
    uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)p.k, leader);
    uint32_t j = (uint32_t)__builtin_amdgcn_readlane((int)p.j, leader);
    const float vm = tb.v[m];
    // the phonon's reflection class at the pore (diffuse or specular; partly specular pores are not walked)
    uint32_t cls = H.pcls & 3u;
    if (EXT && T.spec_w && T.g.pore_tab[0] > 0) cls = tab_class<float>(T, T.g.pore_tab[0], m);
    const float Wx = H.L[0], Wy = H.L[1], Wz = H.L[2];
    const bool zper = ((H.unb >> 2) & 1u) == 0u;
    const float cx = H.p0cx, cy = H.p0cy, rr = H.p0r;
    const float iWx = r_div(1.0f, Wx), iWy = r_div(1.0f, Wy), iWz = r_div(1.0f, Wz);
    const uint32_t kmax = (uint32_t)H.max_events;
    const int sa = H.score_axis;
    // scores of the walked segments (one mode, one sign): the summed length and the summed
    // displacement, in FP64 (s l / v and s l Omega_a follow at the end)
    double aL = 0.0, aQ0 = 0.0, aQ1 = 0.0, aQ2 = 0.0;
    uint32_t nf = 0, np = 0, nd = 0, ns = 0;   // segments, periodic transfers, diffuse, specular
    // a straight piece of length l along the current direction: clocks and scores
    auto advance_time = [&](float l) {
        const float dt = r_div(l, vm);
        t = t + dt;
        const float rem = dtr - dt;
        dtr = rem > 0.0f ? rem : 0.0f;
        aL += (double)l;
        aQ0 += (double)(l * o0);
        aQ1 += (double)(l * o1);
        aQ2 += (double)(l * o2);
    };
    // this lane's pre-drawn diffuse reflection: (mu, sin theta cos phi, sin theta sin phi) of
    // record 2 + jb + 1 + lane, jb the draws made before the batch
    float dmu = 0.0f, dca = 0.0f, dcb = 0.0f;
    uint32_t used = 64;
    const float r2 = rr * rr;
    // the free path only shrinks along the walk and |o2| <= 1, so no later step's z cells (zcap
    // below) exceed those of the whole free path at the start (a 0.1 % margin covers rounding and
    // the last bits of a unit direction): while k <= k_safe the cap test holds without evaluation
    const double need = (double)(zper ? fminf(vm * dtr * iWz, 1.0e9f) : 0.0f) * 1.001 + 70.0;
    const bool safe_ok = need < (double)kmax;
    const uint32_t k_safe = __builtin_amdgcn_readfirstlane(safe_ok ? (uint32_t)((double)kmax - need) : 0u);
    bool finish = true;          // false: stopped ahead of the segment cap (left to the one-segment step)
    for (int guard = 0; guard < (1 << 24); ++guard) {
        const float D = vm * dtr;
        if (!(safe_ok && k <= k_safe)) {
            // the segment cap: one step below crosses at most 65 cell boundaries in x and y and the z
            // cells within the free path; closer to the cap the one-segment step goes on (and ends it)
            const float zcap = zper ? fminf(D * fabsf(o2) * iWz, 1.0e9f) : 0.0f;
            // (every lane holds the same values, so a ballot is the wave's decision; below 2^24 events
            // of budget the integer is exact in FP32, and one event of margin covers zcap + 68's rounding)
            const uint32_t budget = kmax - k;
            const bool room = budget < (1u << 24) ? zcap + 68.0f <= (float)budget
                                                 : (double)k + 67.0 + (double)zcap <= (double)kmax;
            if (!wave_any(room)) {
                finish = false;
                break;
            }
        }
        const float ax = fabsf(o0), ay = fabsf(o1);
        // the window of cells the lanes test: A cells along x by B along y (A B = 64), counted in
        // the ray's direction from the particle's cell and shaped by its slope (32 x 2, 16 x 4 or
        // 8 x 8 along the axis it moves fastest on), lane (i, j) = (lane mod A, lane / A)
        const bool xmaj = wave_any(ax >= ay);
        const float amaj = xmaj ? ax : ay, amin = xmaj ? ay : ax;
        if (!wave_any(amaj > 0.0f)) break;   // along z: no pore ahead
        const int lgM = wave_any(amin * 32.0f < amaj) ? 5 : (wave_any(amin * 16.0f < 3.0f * amaj) ? 4 : 3);
        const int lgA = xmaj ? lgM : 6 - lgM;
        const int A = 1 << lgA, B = 64 >> lgA;
        const bool sxp = wave_any(o0 >= 0.0f), syp = wave_any(o1 >= 0.0f);
        const float fi = (float)(lane & (A - 1)) * Wx, fj = (float)(lane >> lgA) * Wy;
        const float qa = o0 * o0 + o1 * o1;
        const float iqa = r_div(1.0f, qa), qar2 = qa * r2;
        // the pore of cell (i, j) relative to the particle, and the ray's entry into it: the
        // discriminant in Lagrange's form qa r^2 - (dP x o)^2, which keeps the precision of the
        // cross product for a distant pore (no difference of squares of the distance)
        const float dX = x0 - ((sxp ? fi : -fi) + cx);
        const float dY = x1 - ((syp ? fj : -fj) + cy);
        const float qb = dX * o0 + dY * o1;
        const float cr = dX * o1 - dY * o0;
        const float disc = qar2 - cr * cr;
        const float dd = (-qb - r_sqrt(disc > 0.0f ? disc : 0.0f)) * iqa;
        const float d = dd > 0.0f ? dd : 0.0f;
        const bool met = (qb < 0.0f) & (disc >= 0.0f) & (d <= D);
        const float rxl = dX + d * o0, ryl = dY + d * o1;   // the entry point relative to the pore
        // the first pore met is the nearest entry: a pore lies inside its cell and the cells the
        // ray passes form a staircase in its direction, so every pore it meets before leaving the
        // window is in the window
        const float dm = met ? d : INFINITY;
        const float dh = dpp_min_nonneg(dm);          // +inf: no pore met (a met entry is <= D)
        if (__float_as_uint(dh) == 0x7f800000u) {
            // no pore met in the window: the free path ends in it, or the walk moves on to the
            // window's far edge (the cell boundaries crossed counted per axis, the particle placed
            // on the partner face of the edge it leaves through, as after a transfer)
            const float gx = sxp ? (float)A * Wx - x0 : x0 + (float)(A - 1) * Wx;
            const float gy = syp ? (float)B * Wy - x1 : x1 + (float)(B - 1) * Wy;
            const float sxe = ax > 0.0f ? r_div(gx, ax) : INFINITY;
            const float sye = ay > 0.0f ? r_div(gy, ay) : INFINITY;
            const bool ex = wave_any(sxe <= sye);
            const float s = ex ? sxe : sye;
            if (!wave_any(D > s)) break;   // the free path ends first
            const float X = x0 + s * o0, Y = x1 + s * o1;
            const float kx = ex ? 0.0f : floorf(X * iWx), ky = ex ? floorf(Y * iWy) : 0.0f;
            float z = x2 + s * o2, kz = 0.0f;
            if (zper) kz = floorf(z * iWz);
            const uint32_t nx = (uint32_t)(ex ? A : B) + (uint32_t)fabsf(ex ? ky : kx) + (uint32_t)fabsf(kz);
            advance_time(s);
            if (zper) z = z - kz * Wz;
            x0 = ex ? (sxp ? 0.0f : Wx) : X - kx * Wx;
            x1 = ex ? Y - ky * Wy : (syp ? 0.0f : Wy);
            x2 = zper ? (z < 0.0f ? 0.0f : (z > Wz ? Wz : z)) : z;
            k += nx;
            nf += nx;
            np += nx;
            continue;
        }
        // the hit: the winning lane's cell (the lowest lane among equal entries) and its entry
        // point; the cells crossed on the way
        const int wl = __ffsll((long long)__builtin_amdgcn_ballot_w64(dm == dh)) - 1;
        const int wi = wl & (A - 1), wj = wl >> lgA;
        const float rx = lane_f(rxl, wl), ry = lane_f(ryl, wl);
        float z = x2 + dh * o2, kz = 0.0f;
        if (zper) kz = floorf(z * iWz);
        const uint32_t nx = (uint32_t)wi + (uint32_t)wj + (uint32_t)fabsf(kz);
        advance_time(dh);
        if (zper) z = z - kz * Wz;
        x0 = cx + rx;
        x1 = cy + ry;
        x2 = zper ? (z < 0.0f ? 0.0f : (z > Wz ? Wz : z)) : z;
        k += nx + 1u;
        nf += nx + 1u;
        np += nx;
        // the reflection off the pore about the unit normal at the hit point
        const float inv = __builtin_amdgcn_rsqf(rx * rx + ry * ry);
        const float n0 = rx * inv, n1 = ry * inv;
        if (cls == SURF_DIFFUSE) {
            if (used == 64u) {
                const W4 w1 = st.block(2u * (2u + j + 1u + (uint32_t)lane) + 1u);
                const float u1 = unif<float>(w1.x, w1.y), u2 = unif<float>(w1.z, w1.w);
                dmu = r_sqrt(u1);
                const float sth = r_sqrt(1.0f - u1);
                float sn, cs;
                r_sincos_2pi(u2, &sn, &cs);
                dca = sth * cs;
                dcb = sth * sn;
                used = 0u;
            }
            const float mu = lane_f(dmu, (int)used), ca = lane_f(dca, (int)used), cb = lane_f(dcb, (int)used);
            ++used;
            j += 1u;
            // cosine-weighted about n (Eq. wall_dir) in the frame (n, e_z x n, e_z)
            o0 = mu * n0 - ca * n1;
            o1 = mu * n1 + ca * n0;
            o2 = cb;
            ++nd;
        } else {                                     // Eq. specular: k' = k - 2 (k.n) n
            const float k2 = 2.0f * (o0 * n0 + o1 * n1);
            o0 = o0 - k2 * n0;
            o1 = o1 - k2 * n1;
            ++ns;
        }
    }
    if (finish) {
        // the free path ends before the next pore: the face crossings ahead within it, per axis
        // (distance to the first face g, then one per cell width), and the particle placed at the
        // last of them, on the partner face
        const double D = (double)(vm * dtr);
        const double xs[3] = {x0, x1, x2}, os[3] = {o0, o1, o2}, Ws[3] = {Wx, Wy, Wz};
        double s_last = 0.0;
        int a_last = -1;
        uint32_t ncr[3] = {0u, 0u, 0u};
        for (int a = 0; a < 3; ++a) {
            if ((a == 2 && !zper) || os[a] == 0.0) continue;
            const double ao = fabs(os[a]);
            const double g = os[a] > 0.0 ? Ws[a] - xs[a] : xs[a];
            const double La = D * ao;
            if (!(La >= g)) continue;
            const double n = floor((La - g) / Ws[a]) + 1.0;
            ncr[a] = (uint32_t)n;
            const double sa_ = (g + (n - 1.0) * Ws[a]) / ao;
            if (sa_ > s_last || a_last < 0) {
                s_last = sa_;
                a_last = a;
            }
        }
        const uint32_t nx = ncr[0] + ncr[1] + ncr[2];
        if (nx > 0u && k + nx <= kmax) {
            const float s = (float)s_last;
            double xn[3];
            for (int a = 0; a < 3; ++a) {
                xn[a] = xs[a] + s_last * os[a];
                if (a == 2 && !zper) continue;
                xn[a] = xn[a] - (os[a] > 0.0 ? (double)ncr[a] : -(double)ncr[a]) * Ws[a];
                if (a == a_last) xn[a] = os[a] > 0.0 ? 0.0 : Ws[a];     // reinserted at the partner face
                xn[a] = xn[a] < 0.0 ? 0.0 : (xn[a] > Ws[a] ? Ws[a] : xn[a]);
            }
            advance_time(s);
            x0 = (float)xn[0];
            x1 = (float)xn[1];
            x2 = (float)xn[2];
            k += nx;
            nf += nx;
            np += nx;
        }
    }
    const double aT = (double)sg * aL / (double)vm;
    aQ0 *= (double)sg;
    aQ1 *= (double)sg;
    aQ2 *= (double)sg;
    const double aF = sa == 0 ? aQ0 : (sa == 1 ? aQ1 : aQ2);
    if (lane == leader) {
        if (nf > 0u) {
            if (H.det_mask & 1) tadd_c(tc, H.det_ncomp, H.det_slot, (int64_t)m, 0, aT);
            if (H.det_mask & 2) tadd_c(tc, H.det_ncomp, H.det_slot, (int64_t)m, 1, aQ0);
            if (H.det_mask & 4) tadd_c(tc, H.det_ncomp, H.det_slot, (int64_t)m, 2, aQ1);
            if (H.det_mask & 8) tadd_c(tc, H.det_ncomp, H.det_slot, (int64_t)m, 3, aQ2);
        }
        p.cT += aT;
        p.cq += aF;
        p.x[0] = x0;
        p.x[1] = x1;
        p.x[2] = x2;
        p.o[0] = o0;
        p.o[1] = o1;
        p.o[2] = o2;
        p.t = t;
        p.dtr = dtr;
        p.k = k;
        p.j = j;
        p.kc = k;
        cnt.c[1] += nf;
        cnt.c[3] += ns;
        cnt.c[4] += nd;
        cnt.c[5] += np;
    }
}

// ------------------------------------------------------------------------------------------
// particle state buffer (structure of arrays)
// ------------------------------------------------------------------------------------------

template <typename R>
struct StateView {
    R* f[9];          // x, y, z, ox, oy, oz, t, dtr, then (after the integers) lead
    int32_t* i[7];    // m, s, nrel, k, j, src, rejections
    __device__ __host__ StateView(void* base, int64_t cap)
    {
        unsigned char* b = (unsigned char*)base;
        const int64_t fb = (cap * (int64_t)sizeof(R) + 255) & ~int64_t(255);
        const int64_t ib = (cap * 4 + 255) & ~int64_t(255);
        for (int q = 0; q < 8; ++q) f[q] = (R*)(b + q * fb);
        for (int q = 0; q < 7; ++q) i[q] = (int32_t*)(b + 8 * fb + q * ib);
        f[8] = (R*)(b + 8 * fb + 7 * ib);
    }
    __device__ void store(int64_t s, const Part<R>& p, uint32_t rej) const
    {
        f[0][s] = p.x[0]; f[1][s] = p.x[1]; f[2][s] = p.x[2];
        f[3][s] = p.o[0]; f[4][s] = p.o[1]; f[5][s] = p.o[2];
        f[6][s] = p.t; f[7][s] = p.dtr; f[8][s] = p.lead;
        i[0][s] = p.m; i[1][s] = p.s; i[2][s] = p.nrel; i[3][s] = (int32_t)p.k; i[4][s] = (int32_t)p.j;
        i[5][s] = p.src; i[6][s] = (int32_t)rej;
    }
    __device__ void load(int64_t s, Part<R>& p, uint32_t& rej) const
    {
        p.x[0] = f[0][s]; p.x[1] = f[1][s]; p.x[2] = f[2][s];
        p.o[0] = f[3][s]; p.o[1] = f[4][s]; p.o[2] = f[5][s];
        p.t = f[6][s]; p.dtr = f[7][s]; p.lead = f[8][s];
        p.m = i[0][s]; p.s = i[1][s]; p.nrel = i[2][s]; p.k = (uint32_t)i[3][s]; p.j = (uint32_t)i[4][s];
        p.src = i[5][s];
        rej = (uint32_t)i[6][s];
        p.cT = 0.0;
        p.cq = 0.0;
        p.dtr0 = p.dtr;
        p.F0 = 0.0;
    }
};

template <typename R>
__global__ void __launch_bounds__(256) k_emit(const DevTab* __restrict__ tabs, uint64_t seed, uint32_t inst,
                                             int64_t first_pid, int64_t n, void* state, int64_t cap)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const DevTab& T = tabs[0];
    const uint64_t pid = (uint64_t)(first_pid + i);
    const Stream st{(uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)pid, (uint32_t)(pid >> 32), inst};
    Part<R> p;
    uint32_t rej = 0;
    emit_particle<R>(T, st, p, rej);
    if (T.two) resolve_clocks<R>(T, st, p);
    StateView<R>(state, cap).store(i, p, rej);
}

// ------------------------------------------------------------------------------------------
// persistent trace kernels
// ------------------------------------------------------------------------------------------

// stage the relaxation table, velocities and relaxation times of one instance into LDS, with the
// relaxation guide coarsened to 2^bits + 1 bounds (entry i of the finest guide every 2^(12 - bits))
template <typename R>
__device__ __forceinline__ Tabs<R> stage_tables(const DevTab& T, unsigned char* smem, int bits)
{
    const int M = T.M;
    uint64_t* s_thr = (uint64_t*)smem;
    R* s_v = (R*)(smem + align16((int64_t)M * 8));
    R* s_tau = (R*)(smem + align16((int64_t)M * 8) + align16((int64_t)M * sizeof(R)));
    uint16_t* s_guide = (uint16_t*)(smem + align16((int64_t)M * 8) + 2 * align16((int64_t)M * sizeof(R)));
    const R* gv = Geo<R>::v(T);
    const R* gt = Geo<R>::tau(T);
    for (int i = threadIdx.x; i < M; i += blockDim.x) {
        s_thr[i] = T.thr_rel[i];
        s_v[i] = gv[i];
        s_tau[i] = gt[i];
    }
    const bool guided = T.rel_guide && bits >= MCBTE_GUIDE_MIN_BITS && bits <= MCBTE_GUIDE_BITS;
    if (guided)
        for (int i = threadIdx.x; i <= (1 << bits); i += blockDim.x) s_guide[i] = T.rel_guide[i << (MCBTE_GUIDE_BITS - bits)];
    return Tabs<R>{s_thr, s_v, s_tau, guided ? s_guide : nullptr, Geo<R>::tmeas_ptr(T), 64 - bits};
}

__device__ __forceinline__ int64_t lds_tally_size(const DevTab& T) { return T.det.n_cells * T.det.n_cols * T.det.ncomp; }

// the FP32 copy of a wide workgroup into the FP64 sums
__device__ __forceinline__ void flush_lds_tally32(const DevTab& T, const float* s_tally, double* glob)
{
    const int64_t n = lds_tally_size(T);
    const int nc = T.det.ncomp;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const float v = s_tally[i];
        if (v != 0.0f) {
            const int64_t cc = i / nc;
            atomicAdd(glob + cc * 4 + T.det.comp[i - cc * nc], (double)v);
        }
    }
}

__device__ __forceinline__ void flush_lds_tally(const DevTab& T, double* s_tally, double* glob)
{
    const int64_t n = lds_tally_size(T);
    const int nc = T.det.ncomp;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double v = s_tally[i];
        if (v != 0.0) {
            const int64_t cc = i / nc;
            const int q = T.det.comp[i - cc * nc];
            atomicAdd(glob + cc * 4 + q, v);
        }
        s_tally[i] = 0.0;
    }
}

// per-lane counters and moments -> the tally-buffer header (one atomic per wave and counter)
__device__ __forceinline__ void flush_lane_stats(unsigned char* tally, const LaneCounts& cnt, const double mom[4])
{
    unsigned long long* counts = (unsigned long long*)tally;
    double* moments = (double*)(tally + 128);
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < LaneCounts::N; ++q) {
        const uint32_t s = wave_sum<uint32_t>(cnt.c[q]);
        if (lane == 0 && s) atomicAdd(counts + q, (unsigned long long)s);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double s = wave_sum<double>(mom[q]);
        if (lane == 0 && s != 0.0) atomicAdd(moments + q, s);
    }
}

// returns the emission's rejected position draws; kf as for emit_particle (emitted particles only)
template <typename R, int TK, int FT>
__device__ __forceinline__ uint32_t start_particle(const DevTab& T, const LaunchArgs& a, int64_t pid, uint32_t inst,
                                                   Part<R>& p, Stream& st, LaneCounts& cnt, LogRow& lg,
                                                   uint64_t* kf = nullptr)
{
    st = Stream{(uint32_t)a.seed, (uint32_t)(a.seed >> 32), (uint32_t)(uint64_t)pid, (uint32_t)((uint64_t)pid >> 32),
                inst};
    uint32_t rej = 0;
    if ((FT & FT_STATE) && a.state) StateView<R>((void*)a.state, a.capacity).load(pid - a.first_pid, p, rej);
    else emit_particle<R>(T, st, p, rej, kf);
    p.tk = -1;
    p.sn = 0;
    p.kc = 0xFFFFFFFFu;
    cnt.c[0] += 1;
    cnt.c[11] += rej;
    lg.row = nullptr;
    lg.n = 0;
    lg.stride = a.log_stride;
    if ((FT & FT_LOG) && a.event_log && pid - a.first_pid < a.n_log) {
        lg.row = a.event_log + (pid - a.first_pid) * (int64_t)a.log_stride;
        lg.put(p.s > 0 ? EV_EMIT_POS : EV_EMIT_NEG, p.src, p.m);
    }
    return rej;
}

// Pore lattices: the particles whose first free flight passes the scheduling test (emission's
// source, mode and flight keys, records 0 and 1, against the mode's threshold) are listed, so that
// the trace starts them first.  Their number goes to the tally header; a list longer than the
// room for it turns the scheduling off (the trace then takes every particle in order).
__global__ void __launch_bounds__(256) k_prio_scan(const DevTab* __restrict__ tabs, uint64_t seed, uint32_t inst,
                                                   int64_t first_pid, int64_t n, unsigned char* tally)
{
    const DevTab& T = tabs[0];
    unsigned long long* count = (unsigned long long*)(tally + MCBTE_TALLY_PRIO_COUNT_OFFSET);
    int64_t* list = (int64_t*)(tally + T.prio_list_off);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t pid = (uint64_t)(first_pid + i);
        const Stream st{(uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)pid, (uint32_t)(pid >> 32), inst};
        const W4 r0a = st.block(0), r1a = st.block(2);
        const int src = T.S == 1 ? 0 : cdf_pick(T.thr_src, T.S, T.last_src, key64(r0a.x, r0a.y));
        const int m = T.src_kind[src] == SRC_IC || T.src_kind[src] == SRC_HEAT
                          ? cdf_pick_rows(T.thr_ic, T.ic_guide, T.M, T.last_ic, key64(r1a.x, r1a.y))
                          : cdf_pick_rows(T.thr_wall, T.wall_guide, T.M, T.last_wall, key64(r1a.x, r1a.y));
        if ((key64(r0a.z, r0a.w) >> 11) >= T.prio_thr[m]) {
            const unsigned long long k = atomicAdd(count, 1ull);
            if (k < MCBTE_PRIO_CAP) list[k] = (int64_t)pid;
        }
    }
}

template <typename R>
__device__ __forceinline__ void end_particle(const Part<R>& p, int transient, double mom[4], LogRow& lg)
{
    if (!transient) {
        mom[0] += p.cT;
        mom[1] += p.cT * p.cT;
        mom[2] += p.cq;
        mom[3] += p.cq * p.cq;
    }
    if (lg.row) lg.row[0] = (uint32_t)lg.n;
}

// AK = 0: the forward trace (tallies, counters, moments, optional per-particle flux score F).
// AK = 1 (likelihood ratio), 2 (pathwise) or 3 (local pathwise): the sensitivity replay of the same particles: no
// tallies; the per-bin sums go to LDS and then to a.adj; the work counter lives after the sums.
template <typename R, int TK, int AK, int FT>
// (the plain pore-lattice kernel is held to 128 VGPRs, four waves per SIMD, which it fits without
// spilling; the others keep what their register use allows)
__global__ void __launch_bounds__((FT & FT_WIDE) ? 1024 : 256, (FT & (FT_LATTICE | FT_PLAIN)) == (FT_LATTICE | FT_PLAIN) ? 4 : 1)
k_trace_solo(const DevTab* __restrict__ tabs, LaunchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const DevTab& T = tabs[0];
    const Hot<R> H = load_hot<R>(T, AK == 0 && a.particle_F == nullptr);
    constexpr bool WIDE = (FT & FT_WIDE) != 0;
    Tabs<R> tb = WIDE ? Tabs<R>{T.thr_rel, Geo<R>::v(T), Geo<R>::tau(T), T.rel_guide, Geo<R>::tmeas_ptr(T),
                                64 - MCBTE_GUIDE_BITS}
                      : stage_tables<R>(T, smem, a.guide_bits);
    if (TK == TALLY_TRANSIENT && a.lds_tmeas > 0) {     // the measurement times, where the LDS has room
        R* s_tm = (R*)(smem + a.lds_tmeas);
        for (int i = threadIdx.x; i < T.n_times; i += blockDim.x) s_tm[i] = tb.tmeas[i];
        tb.tmeas = s_tm;
    }
    double* s_tally = (double*)(smem + a.lds_tab_bytes);
    float* s_tally32 = (float*)smem;
    constexpr bool ADJ = AK != 0;
    if (ADJ) {
        for (int i = threadIdx.x; i < T.n_bins; i += blockDim.x) s_tally[i] = 0.0;
    } else if (WIDE) {
        const int64_t n = lds_tally_size(T);
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s_tally32[i] = 0.0f;
    } else if (a.tally_lds) {
        const int64_t n = lds_tally_size(T);
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s_tally[i] = 0.0;
    }
    __syncthreads();
    double* const gsum = (double*)(a.tally + MCBTE_TALLY_HEADER_BYTES);
    const TallyCtx tc = ADJ ? TallyCtx{nullptr, nullptr, nullptr}
                            : (WIDE ? TallyCtx{nullptr, gsum, s_tally32}
                                    : TallyCtx{a.tally_lds ? s_tally : nullptr, gsum, nullptr});
    unsigned long long* counter = ADJ ? (unsigned long long*)(a.adj + T.n_bins + 2)
                                      : (unsigned long long*)(a.tally + MCBTE_TALLY_COUNTER_OFFSET);
    const int lane = threadIdx.x & 63;
    const unsigned long long n = (unsigned long long)a.n;

    Part<R> p;
    p.sn = 0;                          // no pending snapshots (lanes that never hold a particle too)
    p.tk = -1;
    Stream st{(uint32_t)a.seed, (uint32_t)(a.seed >> 32), 0u, 0u, 0u};   // the launch's key in every lane
    LaneCounts cnt;
#pragma unroll
    for (int q = 0; q < LaneCounts::N; ++q) cnt.c[q] = 0;
    double mom[4] = {0.0, 0.0, 0.0, 0.0};
    LogRow lg{nullptr, 0, a.log_stride};
    AdjCtx adj{s_tally, 0.0, 0.0, 0u, a.lambda_split};
    PathCtx<R> pc;
    pc.nt = 0;
    int64_t my_pid = 0;
    bool alive = false;
    bool exhausted = false;        // wave-uniform: the particle counter has run past n, the pool is empty
    bool counter_done = false;     // wave-uniform: the counter has run past n
    unsigned long long pool_next = 0, pool_end = 0;   // the wave's unused ids [pool_next, pool_end)
    unsigned long long seen = 0;   // the counter's value after this wave's last grab
    const unsigned long long n_waves = (unsigned long long)gridDim.x * (blockDim.x / 64);
    int since_refill = 0;
    // pore lattices: the listed particles (long first flights) are taken first, one per refill of a
    // wave, and skipped when the counter reaches them; a list that overflowed is not used
    constexpr bool PRIO = (FT & FT_LATTICE) != 0 && AK == 0;
    unsigned long long* const pnext = (unsigned long long*)(a.tally + MCBTE_TALLY_PRIO_NEXT_OFFSET);
    const int64_t* const plist = PRIO ? (const int64_t*)(a.tally + T.prio_list_off) : nullptr;
    unsigned long long pcount = 0;
    if constexpr (PRIO)
        if (T.prio_thr) pcount = *(volatile const unsigned long long*)(a.tally + MCBTE_TALLY_PRIO_COUNT_OFFSET);
    const bool prio_on = PRIO && T.prio_thr && pcount <= MCBTE_PRIO_CAP;
    bool prio_left = prio_on && pcount > 0;   // wave-uniform
    for (;;) {
        unsigned long long live = __ballot(alive);
        if ((!exhausted || prio_left) && (live == 0ull || since_refill >= a.refill)) {
            since_refill = 0;
            unsigned long long need = __ballot(!alive);
            if constexpr (PRIO) {
                if (need && prio_left) {
                    const int ld = __ffsll((long long)need) - 1;
                    unsigned long long pi = 0;
                    if (lane == ld) pi = atomicAdd(pnext, 1ull);
                    pi = __shfl(pi, ld, 64);
                    if (pi < pcount) {
                        if (lane == ld) {
                            my_pid = plist[pi];
                            start_particle<R, TK, FT>(T, a, my_pid, a.inst0, p, st, cnt, lg);
                            alive = true;
                        }
                        need &= need - 1ull;
                    } else {
                        prio_left = false;
                    }
                }
            }
            if (need && !exhausted) {
                // ids from the wave's pool, topped up from the global counter in chunks of up to 64
                // (half the ids left per wave when the counter was last read, at least what is
                // needed), so that thousands of waves refilling every few steps do not queue on
                // one atomic and no wave hoards ids at the end
                const uint32_t cnt_need = (uint32_t)__popcll(need);
                const unsigned long long avail = pool_end - pool_next;
                unsigned long long fresh = 0;
                if (avail < cnt_need) {
                    const int leader = __ffsll((long long)need) - 1;
                    const unsigned long long short_by = cnt_need - avail;
                    const unsigned long long share = (n > seen ? n - seen : 0ull) / (2ull * n_waves);
                    const unsigned long long chunk = share > 64ull ? 64ull : (share > short_by ? share : short_by);
                    unsigned long long b0 = 0;
                    if (lane == leader) b0 = atomicAdd(counter, chunk);
                    b0 = __shfl(b0, leader, 64);
                    fresh = b0;
                    seen = b0 + chunk;
                    if (b0 + chunk >= n) counter_done = true;
                    pool_end = b0 + chunk < n ? b0 + chunk : (b0 < n ? n : b0);
                }
                const uint32_t rank = wave_rank(need);
                const unsigned long long idx = rank < avail ? pool_next + rank : fresh + (rank - avail);
                pool_next = avail < cnt_need ? fresh + (cnt_need - avail) : pool_next + cnt_need;
                if (pool_next > pool_end) pool_next = pool_end;
                if (counter_done && pool_next >= pool_end) exhausted = true;
                if ((need >> lane) & 1ull) {
                    if (idx < n) {
                        my_pid = a.first_pid + (int64_t)idx;
                        uint64_t kf = 0;
                        const uint32_t rej = start_particle<R, TK, FT>(T, a, my_pid, a.inst0, p, st, cnt, lg,
                                                                       PRIO ? &kf : nullptr);
                        alive = true;
                        if (PRIO && prio_on && kf >= T.prio_thr[p.m]) {   // listed: traced from the list
                            cnt.c[0] -= 1;
                            cnt.c[11] -= rej;
                            alive = false;
                        }
                        if (ADJ) adj.F_total = a.particle_F[idx];
                        if (AK == 2) {
                            pc.nt = 0;
                            pc.begin_flight();
                        }
                    }
                }
            }
            live = __ballot(alive);
        }
        if (live == 0ull) {
            if (exhausted && !prio_left) break;
            continue;
        }
        ++since_refill;
        const bool lone = exhausted && !prio_left && (live & (live - 1ull)) == 0ull;   // one lane left in the wave
        // detector-grid pieces of a sparse wave are scored by the whole wave after the step
        const bool spread = TK == TALLY_STEADY_GRID && !ADJ && __popcll(live) <= 16;
        bool coop = false;
        if (alive) {
            if (flight<R, TK, AK, FT>(T, H, tb, tc, st, p, cnt, lg, coop, adj, pc, lone, spread)) {
                end_particle(p, T.transient, mom, lg);
                if (!ADJ && a.particle_F) a.particle_F[my_pid - a.first_pid] = p.cq;
                alive = false;
            }
        }
        if constexpr (TK == TALLY_STEADY_ONE) {
            for (unsigned long long pend = __ballot(coop); pend; pend &= pend - 1ull) {
                if constexpr ((FT & FT_LATTICE) != 0 && std::is_same<R, float>::value)
                    lattice_walk<FT>(T, H, tb, tc, p, st, __ffsll((long long)pend) - 1, cnt);
                else if constexpr (std::is_same<R, float>::value)
                    coop_bounces<R, (FT & FT_PLAIN) == 0>(T, tb, tc, p, st, __ffsll((long long)pend) - 1, cnt);
                else if constexpr ((FT & FT_COOP) != 0)
                    coop_exact(H, tb, tc, p, st, __ffsll((long long)pend) - 1, cnt, lg);
            }
        }
        if constexpr (TK == TALLY_TRANSIENT) snap_wave<R>(T, tc, tb.tmeas, p);
        if constexpr (TK == TALLY_STEADY_GRID && !ADJ) grid_wave<R>(T, H, tc, p);
    }
    if (ADJ) {
        const double d = wave_sum<double>(adj.dense);
        if (lane == 0 && d != 0.0) atomicAdd(a.adj + T.n_bins, d);
        const double nb = wave_sum<double>((double)adj.bad);
        if (lane == 0 && nb != 0.0) atomicAdd(a.adj + T.n_bins + 1, nb);
        __syncthreads();
        for (int i = threadIdx.x; i < T.n_bins; i += blockDim.x)
            if (s_tally[i] != 0.0) atomicAdd(a.adj + i, s_tally[i]);
        return;
    }
    flush_lane_stats(a.tally, cnt, mom);
    if (WIDE) {
        __syncthreads();
        flush_lds_tally32(T, s_tally32, gsum);
    } else if (a.tally_lds) {
        __syncthreads();
        flush_lds_tally(T, s_tally, gsum);
    }
}

// Batched form: the work items are (instance, chunk of chunk_size particles), numbered
// instance-major; a workgroup takes one item at a time, its lanes refill from the item's
// particle range through an LDS counter, and the workgroup moves on once every lane is idle.
template <typename R, int TK, int FT>
__global__ void __launch_bounds__(256) k_trace_batch(const DevTab* __restrict__ tabs, LaunchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long s_item;
    __shared__ int s_inst;
    __shared__ unsigned long long s_next;       // next particle of the current item
    double* s_tally = (double*)(smem + a.lds_tab_bytes);
    const int lane = threadIdx.x & 63;
    int cur = -1;                                // instance whose tables are staged
    Tabs<R> tb{nullptr, nullptr, nullptr};
    LaneCounts cnt;
    double mom[4];
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned long long it = atomicAdd(a.queue, 1ull);
            s_item = (long long)it;
            int inst = -1;
            if ((long long)it < a.n_chunks) {
                int lo = 0, hi = a.n_inst - 1;      // instance with chunk_start[i] <= it < chunk_start[i+1]
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (a.chunk_start[mid] <= (int64_t)it) lo = mid;
                    else hi = mid - 1;
                }
                inst = lo;
            }
            s_inst = inst;
            s_next = 0ull;
        }
        __syncthreads();
        const long long item = s_item;
        const int inst = s_inst;
        if (cur >= 0 && inst != cur) {          // leaving an instance: flush its tallies
            const DevTab& Tc = tabs[cur];
            if (a.tally_lds) flush_lds_tally(Tc, s_tally, (double*)(a.tallies[cur] + MCBTE_TALLY_HEADER_BYTES));
            flush_lane_stats(a.tallies[cur], cnt, mom);
            __syncthreads();
        }
        if (inst < 0) break;
        const DevTab& T = tabs[inst];
        const Hot<R> H = load_hot<R>(T, true);
        if (inst != cur) {
            tb = stage_tables<R>(T, smem, a.guide_bits);
            if (a.tally_lds) {
                const int64_t n = lds_tally_size(T);
                for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s_tally[i] = 0.0;
            }
#pragma unroll
            for (int q = 0; q < LaneCounts::N; ++q) cnt.c[q] = 0;
            mom[0] = mom[1] = mom[2] = mom[3] = 0.0;
            cur = inst;
            __syncthreads();
        }
        const int64_t first = (item - a.chunk_start[inst]) * a.chunk_size;
        int64_t last = first + a.chunk_size;
        if (last > a.inst_n[inst]) last = a.inst_n[inst];
        const unsigned long long n = (unsigned long long)(last - first);
        const uint32_t inst_id = a.inst_ids[inst];
        const TallyCtx tc{a.tally_lds ? s_tally : nullptr, (double*)(a.tallies[inst] + MCBTE_TALLY_HEADER_BYTES),
                          nullptr};
        Part<R> p;
        p.sn = 0;
        p.tk = -1;
        Stream st{(uint32_t)a.seed, (uint32_t)(a.seed >> 32), 0u, 0u, 0u};
        LogRow lg{nullptr, 0, 2};
        AdjCtx adj{nullptr, 0.0, 0.0, 0u, 0.0};
        PathCtx<R> pc;            // unused by the trace
        pc.nt = 0;
        bool alive = false;
        bool exhausted = false;
        int since_refill = 0;
        for (;;) {
            unsigned long long live = __ballot(alive);
            if (!exhausted && (live == 0ull || since_refill >= a.refill)) {
                since_refill = 0;
                const unsigned long long need = __ballot(!alive);
                if (need) {
                    const uint32_t cnt_need = (uint32_t)__popcll(need);
                    const int leader = __ffsll((long long)need) - 1;
                    unsigned long long base = 0;
                    if (lane == leader) base = atomicAdd(&s_next, (unsigned long long)cnt_need);
                    base = __shfl(base, leader, 64);
                    if (base + cnt_need >= n) exhausted = true;
                    if (!alive) {
                        const unsigned long long idx = base + wave_rank(need);
                        if (idx < n) {
                            const int64_t pid = first + (int64_t)idx;
                            st = Stream{(uint32_t)a.seed, (uint32_t)(a.seed >> 32), (uint32_t)(uint64_t)pid,
                                        (uint32_t)((uint64_t)pid >> 32), inst_id};
                            uint32_t rej = 0;
                            emit_particle<R>(T, st, p, rej);
                            p.tk = -1;
                            p.sn = 0;
                            cnt.c[0] += 1;
                            cnt.c[11] += rej;
                            alive = true;
                        }
                    }
                    live = __ballot(alive);
                }
            }
            if (live == 0ull) {
                if (exhausted) break;
                continue;
            }
            ++since_refill;
            bool coop = false;
            if (alive) {
                // (no lone-lane chains here: their registers would cost the film sweeps, for which
                // this kernel exists, an occupancy step)
                if (flight<R, TK, 0, FT>(T, H, tb, tc, st, p, cnt, lg, coop, adj, pc, false)) {
                    end_particle(p, T.transient, mom, lg);
                    alive = false;
                }
            }
            if constexpr (TK == TALLY_STEADY_ONE) {
                for (unsigned long long pend = __ballot(coop); pend; pend &= pend - 1ull) {
                    if constexpr (std::is_same<R, float>::value)
                        coop_bounces<R, (FT & FT_PLAIN) == 0>(T, tb, tc, p, st, __ffsll((long long)pend) - 1, cnt);
                }
            }
            if constexpr (TK == TALLY_TRANSIENT) snap_wave<R>(T, tc, tb.tmeas, p);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------
// launchers (called from the host side of the library)
// ------------------------------------------------------------------------------------------

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }
__global__ void k_zero_u64_n(unsigned long long* p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

template <typename R>
static hipError_t emit_t(const DevTab* d_tab, uint64_t seed, uint32_t inst, int64_t first_pid, int64_t n, void* state,
                         int64_t cap, hipStream_t s)
{
    const int block = 256;
    const int64_t grid = (n + block - 1) / block;
    hipLaunchKernelGGL(k_emit<R>, dim3((unsigned)grid), dim3(block), 0, s, d_tab, seed, inst, first_pid, n, state, cap);
    return hipGetLastError();
}

hipError_t launch_emit(const DevTab* d_tab, int precision, uint64_t seed, uint32_t inst, int64_t first_pid, int64_t n,
                       void* state, int64_t cap, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    return precision == 64 ? emit_t<double>(d_tab, seed, inst, first_pid, n, state, cap, s)
                           : emit_t<float>(d_tab, seed, inst, first_pid, n, state, cap, s);
}

// raise the dynamic-LDS limit of a kernel once per (kernel, size)
static void ensure_lds_limit(const void* fn, size_t lds)
{
    static std::mutex mu;
    static std::map<const void*, size_t> done;
    std::lock_guard<std::mutex> lock(mu);
    auto it = done.find(fn);
    if (it != done.end() && it->second >= lds) return;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess) done[fn] = lds;
}

// the kernel of a launch: mode 0 trace, 1 batched trace, 2 likelihood-ratio replay, 3 pathwise
// replay, 4 local pathwise replay; ft the optional features (FT_STATE | FT_LOG: a state buffer and/or an event log;
// FT_WIDE: FP32 trace with the tally in LDS in FP32; FT_PLAIN: no table has a two-phonon clock or a
// specular cutoff, the kernels without that code; FT_LATTICE: FP32 steady trace or likelihood-ratio /
// local replay of a pore lattice, walked pore to pore by the wave).  The replays refuse tables with the
// extended physics and are built without it.  NULL: no such kernel.
template <typename R, int TK, int PLAIN>
static const void* pick_solo(int mode, int ft)
{
    if constexpr (std::is_same<R, double>::value && TK == TALLY_STEADY_ONE) {
        if (ft & FT_COOP) {
            if (mode == 2) return (const void*)k_trace_solo<R, TK, 1, FT_COOP | FT_PLAIN>;
            if (mode == 3) return (const void*)k_trace_solo<R, TK, 2, FT_COOP | FT_PLAIN>;
            if (mode == 4) return (const void*)k_trace_solo<R, TK, 3, FT_COOP | FT_PLAIN>;
            if (ft & (FT_STATE | FT_LOG)) return (const void*)k_trace_solo<R, TK, 0, FT_STATE | FT_LOG | FT_COOP | PLAIN>;
            return (const void*)k_trace_solo<R, TK, 0, FT_COOP | PLAIN>;
        }
    }
    if constexpr (std::is_same<R, float>::value && TK == TALLY_STEADY_ONE) {
        // pre-emitted states without an event log: refills load states instead of emitting
        if (mode == 0 && (ft & FT_STATE) && !(ft & FT_LOG)) return (const void*)k_trace_solo<R, TK, 0, FT_STATE | PLAIN>;
        if (ft & FT_LATTICE) {   // (never with a state buffer or an event log)
            if (mode == 2) return (const void*)k_trace_solo<R, TK, 1, FT_LATTICE | FT_PLAIN>;
            if (mode == 4) return (const void*)k_trace_solo<R, TK, 3, FT_LATTICE | FT_PLAIN>;
            if (mode == 0) return (const void*)k_trace_solo<R, TK, 0, FT_LATTICE | PLAIN>;
            return nullptr;
        }
    }
    if (mode == 2) return (const void*)k_trace_solo<R, TK, 1, FT_PLAIN>;
    if (mode == 3) return (const void*)k_trace_solo<R, TK, 2, FT_PLAIN>;
    if (mode == 4) return (const void*)k_trace_solo<R, TK, 3, FT_PLAIN>;
    if (ft & (FT_STATE | FT_LOG)) return (const void*)k_trace_solo<R, TK, 0, FT_STATE | FT_LOG | PLAIN>;
    if constexpr (std::is_same<R, float>::value) {
        if (ft & FT_WIDE) return (const void*)k_trace_solo<R, TK, 0, FT_WIDE | PLAIN>;
    }
    return (const void*)k_trace_solo<R, TK, 0, PLAIN>;
}

template <typename R, int TK>
static const void* pick_kernel(int mode, int ft)
{
    if (mode == 1)
        return (ft & FT_PLAIN) ? (const void*)k_trace_batch<R, TK, FT_PLAIN> : (const void*)k_trace_batch<R, TK, 0>;
    return (ft & FT_PLAIN) ? pick_solo<R, TK, FT_PLAIN>(mode, ft) : pick_solo<R, TK, 0>(mode, ft);
}

static const void* kernel_for(int mode, int precision, int tally_kind, int ft)
{
    if (precision == 64) {
        switch (tally_kind) {
        case TALLY_STEADY_ONE: return pick_kernel<double, TALLY_STEADY_ONE>(mode, ft);
        case TALLY_STEADY_GRID: return pick_kernel<double, TALLY_STEADY_GRID>(mode, ft);
        default: return pick_kernel<double, TALLY_TRANSIENT>(mode, ft);
        }
    }
    switch (tally_kind) {
    case TALLY_STEADY_ONE: return pick_kernel<float, TALLY_STEADY_ONE>(mode, ft);
    case TALLY_STEADY_GRID: return pick_kernel<float, TALLY_STEADY_GRID>(mode, ft);
    default: return pick_kernel<float, TALLY_TRANSIENT>(mode, ft);
    }
}

hipError_t launch_trace(const LaunchArgs& a, int mode, int precision, int tally_kind, int ft, int block, int grid,
                        size_t lds, hipStream_t s)
{
    const void* fn = kernel_for(mode, precision, tally_kind, ft);
    if (!fn) return hipErrorInvalidDeviceFunction;
    ensure_lds_limit(fn, lds);
    if (mode == 0 && (ft & FT_LATTICE)) {
        // the work counter, the scheduling list's length and its next entry (tally header), then
        // the list of the particles to start first
        hipLaunchKernelGGL(k_zero_u64_n, dim3(1), dim3(64), 0, s,
                           (unsigned long long*)(a.tally + MCBTE_TALLY_COUNTER_OFFSET), 3);
        const int64_t blocks = std::min<int64_t>(4096, (a.n + 255) / 256);
        if (blocks > 0)
            hipLaunchKernelGGL(k_prio_scan, dim3((unsigned)blocks), dim3(256), 0, s, a.tabs, a.seed, a.inst0,
                               a.first_pid, a.n, a.tally);
    } else if (mode == 0) {   // the work counter of a solo trace lives in the tally header
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s,
                           (unsigned long long*)(a.tally + MCBTE_TALLY_COUNTER_OFFSET));
    }
    const DevTab* tabs = a.tabs;
    LaunchArgs args = a;
    void* kargs[] = {(void*)&tabs, (void*)&args};
    const hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(block), kargs, lds, s);
    return e != hipSuccess ? e : hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// allocation-free batched trace: the work queue in a static device array
// ------------------------------------------------------------------------------------------

// The work queue of mcbte_trace_batch_static, for at most MCBTE_STATIC_INSTANCES instances; each
// device holds its own copy until the process ends, and every call on a device shares it.
static constexpr int64_t kStaticQueueBytes =
    256 + 2 * ((8 * MCBTE_STATIC_INSTANCES + 255) / 256 * 256) + (8 * (MCBTE_STATIC_INSTANCES + 1) + 255) / 256 * 256 +
    (4 * MCBTE_STATIC_INSTANCES + 255) / 256 * 256 + ((int64_t)sizeof(DevTab) * MCBTE_STATIC_INSTANCES + 255) / 256 * 256;
static __device__ __align__(256) unsigned char scratch[kStaticQueueBytes];

int64_t static_queue_bytes() { return kStaticQueueBytes; }

// The device address of `scratch` on device `dev` (which must be current), looked up once per device
// (in host code the array's name stands for no device address).
hipError_t static_queue(int dev, unsigned char** out)
{
    static std::mutex mu;
    static std::map<int, unsigned char*> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
        it = addr.emplace(dev, (unsigned char*)ptr).first;
    }
    *out = it->second;
    return hipSuccess;
}

// Fill the work queue in q (the layout of queue_layout) from the setup arguments: the counter page
// cleared, the per-instance arrays written, each instance's tables copied from its device copy.
__global__ void __launch_bounds__(256) k_batch_setup(BatchSetupArgs args, unsigned char* q)
{
    const QueueLayout L = queue_layout(args.n_inst);
    const int n = args.n_inst;
    for (int i = threadIdx.x; i < 32; i += blockDim.x) ((unsigned long long*)q)[i] = 0ull;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        ((unsigned char**)(q + L.o_tp))[i] = args.tally[i];
        ((int64_t*)(q + L.o_n))[i] = args.n[i];
        ((uint32_t*)(q + L.o_id))[i] = args.id[i];
    }
    for (int i = threadIdx.x; i <= n; i += blockDim.x) ((int64_t*)(q + L.o_cs))[i] = args.cstart[i];
    constexpr int W = (int)(sizeof(DevTab) / 8);
    static_assert(sizeof(DevTab) % 8 == 0, "DevTab copied in 8-byte words");
    for (int w = threadIdx.x; w < n * W; w += blockDim.x) {
        const int inst = w / W, k = w - inst * W;
        ((uint64_t*)(q + L.o_tab))[w] = ((const uint64_t*)args.tab[inst])[k];
    }
}

hipError_t launch_batch_setup(const BatchSetupArgs& args, unsigned char* q, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_setup, dim3(1), dim3(256), 0, s, args, q);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, p);
    return hipGetLastError();
}

// occupancy of the trace kernel (workgroups per compute unit) for a block size and LDS size,
// cached per (kernel, block, LDS)
int trace_occupancy(int mode, int precision, int tally_kind, int ft, int block, size_t lds)
{
    const void* fn = kernel_for(mode, precision, tally_kind, ft);
    if (!fn) return 1;
    static std::mutex mu;
    static std::map<std::tuple<const void*, int, size_t>, int> cache;
    const auto key = std::make_tuple(fn, block, lds);
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    ensure_lds_limit(fn, lds);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, lds) != hipSuccess || nb < 1) nb = 1;
    std::lock_guard<std::mutex> lock(mu);
    cache[key] = nb;
    return nb;
}

}  // namespace mcbte
