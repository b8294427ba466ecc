// Device-side view of one table set, shared by the host builder (mcbte_host.cpp) and the
// kernels (mcbte_kernels.hip).  Library-internal: not part of the C ABI.
#pragma once
#include <stdint.h>

#define MCBTE_DEV_MAX_PORES 8
#define MCBTE_DEV_MAX_WALLS 16
#define MCBTE_LDS_TABLE_BYTES (48 * 1024)   // mode tables staged in LDS (thresholds + v + tau)
#define MCBTE_LDS_TALLY_BYTES (40 * 1024)   // per-workgroup tally privatisation budget
#define MCBTE_GUIDE_BITS 12                  // finest guide of the relaxation draw: 2^12 + 1 bounds
#define MCBTE_GUIDE_MIN_BITS 8               // coarsest guide staged in LDS
// LDS bytes of a guide of 2^bits + 1 uint16 bounds (0 bits: no guide)
__host__ __device__ inline int64_t guide_lds_bytes(int bits) { return bits > 0 ? (((int64_t(1) << bits) + 1) * 2 + 15) & ~int64_t(15) : 0; }
#define MCBTE_TALLY_HEADER_BYTES 256
#define MCBTE_TALLY_COUNTER_OFFSET 192
// pore lattices: particles whose first free path is long enough to be walked for a while are
// listed before the trace and started first; the list's length and the next entry to take live in
// the tally header, the list after the raw sums
#define MCBTE_TALLY_PRIO_COUNT_OFFSET 200
#define MCBTE_TALLY_PRIO_NEXT_OFFSET 208
#define MCBTE_PRIO_CAP 4096
#define MCBTE_PATH_MAX 16                    // flights per particle the pathwise replay holds

namespace mcbte {

// SRC_IWALL: isothermal line wall; SRC_HEAT: one time interval of the external heat source
enum SourceKind : int32_t { SRC_WALL = 0, SRC_GRAD = 1, SRC_IC = 2, SRC_IWALL = 3, SRC_HEAT = 4 };
enum TallyKind : int32_t { TALLY_STEADY_ONE = 0, TALLY_STEADY_GRID = 1, TALLY_TRANSIENT = 2 };

// optional features of the trace kernels, compiled in only where used: particles loaded from a
// state buffer written by k_emit, the per-particle event log, (FP32 trace) wide workgroups
// whose whole LDS holds an FP32 copy of a tally too large for the FP64 one, the mode tables
// being read from global memory instead, and (FP64 film-like problems) the exact cooperative
// bouncing, whose registers the other FP64 problems need not reserve
// FT_PLAIN: no table uses the two-phonon clock or a specular cutoff frequency (kernels without that code)
// FT_LATTICE: (FP32 steady trace of a cell periodic in x and y, one pore, no line walls) a particle
// with a long free path is followed from pore to pore by its whole wave (lattice_walk)
enum : int { FT_STATE = 1, FT_LOG = 2, FT_WIDE = 4, FT_COOP = 8, FT_PLAIN = 16, FT_LATTICE = 32 };

// Geometry in the form the flight loop reads it (uniform across a launch; scalar loads).
struct DevPore32 { float cx, cy, r; int32_t id; };
struct DevPore64 { double cx, cy, r; int32_t id, pad; };

// class of an adiabatic surface for the event choice: 0 diffuse (d <= 0), 1 specular (d >= 1),
// 2 partly specular (0 < d < 1, decided by a key against the surface's threshold); each
// precision classifies its own rounding of d
enum : uint32_t { SURF_DIFFUSE = 0, SURF_SPECULAR = 1, SURF_PARTIAL = 2 };

struct DevGeom {
    double L[3];
    int32_t unb[3];              // axis without faces
    int32_t n_pores;
    int32_t face_type[6];        // by boundary id - 1
    int32_t pad0;
    double face_spec[6];         // adiabatic specularity
    uint64_t face_thr[6];        // floor(d 2^64) for 0 < d < 1
    double pore_cx[MCBTE_DEV_MAX_PORES], pore_cy[MCBTE_DEV_MAX_PORES], pore_r[MCBTE_DEV_MAX_PORES];
    double pore_spec[MCBTE_DEV_MAX_PORES];
    uint64_t pore_thr[MCBTE_DEV_MAX_PORES];
    int32_t pore_id[MCBTE_DEV_MAX_PORES];
    double ngrad[3];             // -gradT / |gradT| (0 if no gradient)
    // single-precision copies for the FP32 trajectories
    float L32[3];
    float pore_cx32[MCBTE_DEV_MAX_PORES], pore_cy32[MCBTE_DEV_MAX_PORES], pore_r32[MCBTE_DEV_MAX_PORES];
    float ngrad32[3];
    // compact forms for the flight loop, read into registers once per launch: axis mask, and per
    // precision ([0] FP32, [1] FP64) 4 bits per face id - 1 (type | class << 2) and 2 bits per
    // pore (class); the pores again as one record each
    uint32_t unb_mask;
    uint32_t face_code[2];
    uint32_t pore_cls[2];
    DevPore32 pore32[MCBTE_DEV_MAX_PORES];
    DevPore64 pore64[MCBTE_DEV_MAX_PORES];
    // specularity per phonon: 1 + the per-row table a boundary reads its class and threshold from
    // (0: the boundary's own constant d)
    int32_t face_tab[6];
    int32_t pore_tab[MCBTE_DEV_MAX_PORES];
    // internal line walls: segment, unit normal (FP64 and FP32), id, 2 bits of class per wall and
    // precision, partial-specularity threshold, per-row table, and the closed loops (loop_end[k] = last
    // wall of the loop that wall k starts, -1 otherwise)
    int32_t n_walls;
    int32_t pad_w;
    double wall_x1[MCBTE_DEV_MAX_WALLS], wall_y1[MCBTE_DEV_MAX_WALLS];
    double wall_x2[MCBTE_DEV_MAX_WALLS], wall_y2[MCBTE_DEV_MAX_WALLS];
    double wall_nx[MCBTE_DEV_MAX_WALLS], wall_ny[MCBTE_DEV_MAX_WALLS];
    float wall32[MCBTE_DEV_MAX_WALLS][6];
    int32_t wall_id[MCBTE_DEV_MAX_WALLS];
    int32_t wall_type[MCBTE_DEV_MAX_WALLS];
    int32_t wall_loop_end[MCBTE_DEV_MAX_WALLS];
    uint32_t wall_cls[2];
    uint64_t wall_thr[MCBTE_DEV_MAX_WALLS];
    int32_t wall_tab[MCBTE_DEV_MAX_WALLS];
};

struct DevDet {
    double lo[3], hi[3], w[3];   // w = (hi - lo) / n on binned axes
    float lo32[3], hi32[3], inv_w32[3];
    int32_t n[3];
    int32_t mask;
    int32_t ncomp;               // number of components in the mask
    int32_t slot[4];             // compact LDS slot of each component, -1 if masked out
    int32_t comp[4];             // component of each compact slot
    int32_t n_cols;
    int64_t n_cells;
};

struct DevTab {
    int32_t M, S;
    int32_t transient, n_scat_max;
    int32_t score_axis, n_times;
    int32_t ic_axis, n_ic;
    int32_t tally_kind;          // TallyKind
    int32_t coop_axis;           // film axis for wave-cooperative diffuse bouncing (FP32), -1: off
    int32_t fold_axis;           // film axis whose two walls reflect every phonon alike, -1: off (the
                                 // FP32 trace then runs a specular phonon's wall-to-wall crossings at once)
    int32_t pad_f;
    double coop_min_path;        // remaining free path (m) above which a wall bounce turns cooperative
    double lat_min_path;         // pore lattice: remaining free path (m) above which the wave walks the
                                 // particle from pore to pore (0: the geometry is not such a lattice)
    int64_t max_events;
    double t_max;
    int64_t last_ic, last_wall, last_rel, last_src;
    // device arrays (inside the table allocation)
    const double* v64;
    const double* tau64;
    const float* v32;
    const float* tau32;
    const uint64_t* thr_ic;
    const uint64_t* thr_wall;
    const uint64_t* thr_rel;
    const uint64_t* thr_src;
    const int32_t* src_kind;
    const int32_t* src_ref;
    const int32_t* src_sign;
    const double* ic_edges;
    const double* heat_t;        // external heat source: interval edges (n_heat + 1), or NULL
    // its tetrahedra (region built from them): vertex 0 and the edges to vertices 1-3, 12 values
    // each, FP64 and FP32, and the choice of one by volume
    const double* heat_tet64;
    const float* heat_tet32;
    const uint64_t* thr_tet;
    int64_t last_tet;
    // emission row draws: guides of thr_wall and thr_ic in the form of rel_guide, or NULL
    const uint16_t* wall_guide;
    const uint16_t* ic_guide;
    // measurement times: entry b = count(t_k < b t_max / 256) for b < 256, entry 256 = n_times (a
    // time t lies in bucket floor(t 256 / t_max)); NULL: not transient or more than 65535 times
    const uint16_t* tm_guide;
    double tm_gs64;              // 256 / t_max
    float tm_gs32;
    int32_t pad_tg;
    int32_t n_heat_tet;
    int32_t pad_t;
    const double* t_meas64;
    const float* t_meas32;
    const int32_t* bin_of;       // frequency bin of each mode (sensitivity parameters)
    const uint16_t* rel_guide;   // relaxation draw: entry b = count(thr_rel <= b 2^52), b <= 2^12 (the last
                                 // entry is M), or NULL (tables of more than 65535 rows)
    const double* tau2_64;       // two-phonon relaxation time of each row (0: no such process)
    const float* tau2_32;
    const double* omega64;       // angular frequency of each row
    // per-row specularity tables (table k, row m at k * M + m): threshold floor(d 2^64) for a partly
    // specular row, class (bits 0-1 as FP32 trajectories see d, bits 2-3 as FP64 ones do)
    const uint64_t* spec_thr;
    const uint8_t* spec_cls;
    const uint64_t* prio_thr;    // pore lattice: a particle is started first when the top 53 bits of its first
                                 // free-flight key reach prio_thr[mode] (NULL: no such scheduling)
    int64_t prio_list_off;       // byte offset of the list of those particles in the tally buffer
    int32_t n_bins;
    int32_t two;                 // some row has a two-phonon clock
    int32_t spec_w;              // some boundary's specularity depends on the phonon (a per-row table)
    int32_t lattice;             // the cell tiles a lattice of pores (lat_min_path > 0)
    // external heat source region: corner and widths per axis (0 and 1 m along an unbounded axis)
    double heat_lo[3], heat_w[3];
    float heat_lo32[3], heat_w32[3];
    DevGeom g;
    DevDet det;
};

// launch description shared by the solo and batched trace kernels
struct LaunchArgs {
    const DevTab* tabs;          // device array, one per instance
    int32_t n_inst;
    int32_t refill;
    uint64_t seed;
    const uint32_t* inst_ids;    // device array (batched) or NULL (solo: inst0)
    uint32_t inst0;
    int32_t log_stride;
    int64_t first_pid;
    int64_t n;                   // solo: particle count
    const void* state;           // solo: pre-emitted states or NULL
    int64_t capacity;
    unsigned char* tally;        // solo: tally buffer
    uint32_t* event_log;
    int64_t n_log;
    // batched: per-instance tallies and particle counts plus the chunk table
    unsigned char* const* tallies;
    const int64_t* inst_n;
    const int64_t* chunk_start;  // prefix sum of chunks per instance (n_inst + 1)
    int64_t chunk_size;
    unsigned long long* queue;   // [0]: next chunk
    int64_t n_chunks;
    int32_t tally_lds;           // tallies privatised in LDS
    int32_t lds_tab_bytes;       // offset of the tally region in dynamic LDS
    int32_t lds_tmeas;           // offset of the staged measurement times in dynamic LDS (0: not staged)
    int32_t guide_bits;          // bits of the relaxation guide staged in LDS (0: the whole table is searched)
    // sensitivity replay
    double* particle_F;          // per-particle flux score (written by the trace, read by the replay)
    double* adj;                 // n_bins sums, the relaxation-draw sum B, then a work counter
    double lambda_split;         // local pathwise replay: modes with v tau <= this take that form
};

// Work-queue layout of the batched trace (in the caller's queue buffer, or in the library's static
// scratch for the allocation-free entry point): counter page, per-instance tally pointers, particle
// counts, chunk starts (n + 1), Philox instance ids, tables; every piece 256-byte aligned.
struct QueueLayout {
    int64_t o_tp, o_n, o_cs, o_id, o_tab, end;
};
__host__ __device__ inline int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }
__host__ __device__ inline QueueLayout queue_layout(int64_t n_inst)
{
    QueueLayout q;
    q.o_tp = 256;
    q.o_n = q.o_tp + align256(8 * n_inst);
    q.o_cs = q.o_n + align256(8 * n_inst);
    q.o_id = q.o_cs + align256(8 * (n_inst + 1));
    q.o_tab = q.o_id + align256(4 * n_inst);
    q.end = q.o_tab + align256((int64_t)sizeof(DevTab) * n_inst);
    return q;
}

// the allocation-free batched trace: at most this many instances (its per-instance data travel as
// the setup kernel's arguments, and its work queue lives in a static device array of this size)
#define MCBTE_STATIC_INSTANCES 64
struct BatchSetupArgs {
    int32_t n_inst;
    int32_t pad;
    const DevTab* tab[MCBTE_STATIC_INSTANCES];    // device copies of the instances' tables
    unsigned char* tally[MCBTE_STATIC_INSTANCES];
    int64_t n[MCBTE_STATIC_INSTANCES];
    int64_t cstart[MCBTE_STATIC_INSTANCES + 1];
    uint32_t id[MCBTE_STATIC_INSTANCES];
};

}  // namespace mcbte
