// lj_internal.h -- internal structures and launchers of the gfx950 LJ library.
//
// Every kernel works on a batch of independent systems (a single system is a
// batch of one).  System s owns records [atom0, atom0 + n) of the caller's
// concatenated position/velocity/force arrays and is described on the device
// by an lj_sys record.
//
// Data layout in HBM:
//   positions  caller's array: records of double4 (x, y, z, pad) or SoA 3 x N
//   cells      count[ncell], cell_start[ncell + 1] over the concatenated cell
//              grids (system s owns cells [cell0, cell0 + ncell_s)), cid[N]
//              (cell of atom), order[N] (cell-sorted rank -> atom), spos[N]
//              (cell-sorted double4 (x, y, z, w) whose w holds the atom index
//              as the bits of a 64-bit integer) plus LJ_SPOS_PAD unused
//              records.  The ranks of system s are [atom0, atom0 + n).
//   list       wavefront-sliced rows: a slice is C = 64 / G rows served by one
//              wavefront with G lanes per row; rows are the atoms in cell
//              order.  System s owns slices [slice0, slice0 + nslices), a
//              multiple of 4G (whole 256-row blocks), so that every
//              wavefront, 4-slice force block and 256-row block belongs to one
//              system; row r of the system is rank atom0 + r - slice0 * C.
//              Entry k of row c of slice t (local index t - slice0) is taken
//              at step s = k / G by lane p = c * G + k % G and sits at
//                col[col0 + t_local * (cap / G) * 64 + (s / 4) * 256 + p * 4 + s % 4]
//              so each lane loads its indices of 4 consecutive steps with one
//              16-byte load (1 KiB per wavefront).  cap is a multiple of 4 G.
//              row_atom, row_len per row; slice_iters[t] = the slice's longest
//              row in G-wide steps; slots past a row's length (up to its
//              slice's length rounded up to 4 steps) hold the row's own atom
//              so every gather stays in bounds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lj.h"

#define LJ_WAVE 64
#define LJ_BLOCK 256
#define LJ_WAVES_PER_BLOCK (LJ_BLOCK / LJ_WAVE)
#define LJ_NXCD 8
// Records past the end of the cell-sorted positions, so that a list-build lane
// may load a whole batch of candidates past the end of its range (the extra
// records are never used).
#define LJ_SPOS_PAD 8

// One system of a batch (device and host copies).
struct lj_sys {
    // atoms
    int64_t atom0, n;
    // cells
    int64_t cell0, ncell;
    int32_t nc[3];
    int32_t reach[3];      // cells within rs + delta of a point lie within +-reach
    int32_t full[3];       // 1: fewer than 2 reach + 2 cells -> the dimension is scanned whole
    int32_t pad0;
    double box[3], half_box[3], inv_box[3], inv_cs[3], cs[3];
    float cs2f[3];         // cell side^2 (FP32, culling only)
    float rsd2f;           // (rs + delta)^2, inflated (culling only)
    float r2lo, r2hi;      // FP32 pair test: r^2 below r2lo is a pair and at or above
                           // r2hi is not, whatever the FP64 test gives; in between
                           // the FP64 test decides
    double rs, rc_list, skin, rs2;
    // list
    int64_t slice0, nslices, col0;
    int32_t cap;           // slots per row, a multiple of the lanes per row
    int32_t pad1;
};

// Force constants of one system.
struct lj_fconst {
    double rc2, sig2, c4, c24, c48;       // rc^2, sigma^2, 4 eps, 24 eps, 48 eps
    double vc;                            // energy subtracted per interacting pair: V(rc),
                                          // or V(rc) + rc Fc when force-shifted
    double fcut;                          // force-shifted: Fc = -V'(rc); else 0
    int32_t fshift, pad0;                 // 1: force-shifted truncation
    float sig2f, c4f, c24f, c48f, fcutf;
    // Mixed precision: positions as 32-bit fixed point, x = u * L / 2^32
    double qinv[3];        // 2^32 / L per dimension (quantisation)
    double qs[3];          // L / 2^32 per dimension: one fixed-point unit (exact)
    // An r^2 of fixed-point displacements below rc2lo interacts and at or
    // above rc2hi does not, whatever the test on the unquantised positions
    // gives; in between that test decides
    double rc2lo, rc2hi;
};

// Device status words of a context.
struct lj_dev_status {
    int32_t flags;                 // LJ_DEV_* bits raised by kernels
    int32_t pad0;
    unsigned long long pad1;
};
#define LJ_DEV_BAD_POSITION 1
#define LJ_DEV_ROW_OVERFLOW 2
#define LJ_DEV_STALE 4          // an integrator step found an atom moved more than skin/2
                                // since the list was built (fixed rebuild cadence)
#define LJ_DEV_RESTORED 8       // an integrator run stopped and restored its last good step
// errors after which force and integrator kernels leave their outputs as they were
#define LJ_DEV_ERRORS (LJ_DEV_BAD_POSITION | LJ_DEV_ROW_OVERFLOW)

// Row statistics of one system of a list, written by its latest build.
struct lj_list_stats {
    int32_t max_row;               // longest row (before clamping to the capacity)
    int32_t pad;
    unsigned long long entries;    // entries stored
    unsigned long long tests;      // candidate pairs tested by the build
};

struct lj_prof_rec {
    int phase;
    hipEvent_t a, b;
};

struct lj_ctx {
    int device;
    hipStream_t stream;
    lj_dev_status* st;             // device
    double* partials;              // device, per-block E/W/count partials
    int64_t partials_cap;          // in blocks
    double* scratch;               // the device's static partials (lj_forces_noalloc)
    bool prof_on;
    std::vector<lj_prof_rec> prof;
    int32_t tune[LJ_TUNE_N];       // tuning knobs (lj_tune_set)
    int cus;                       // compute units of the device
};

// Records HIP events around a launch on the context's stream while the
// profiler is on.
struct lj_prof_scope {
    lj_ctx* ctx;
    int idx;
    lj_prof_scope(lj_ctx* c, int phase);
    ~lj_prof_scope();
};

struct lj_cells {
    int nsys;
    int64_t n;                     // atoms over all systems
    int64_t ncell;                 // cells over all systems
    std::vector<lj_sys> hsys;      // cell fields valid
    lj_sys* dsys;                  // device copy
    int32_t* atom_sys;             // device, system of each atom (NULL for one system)
    int32_t* count;                // ncell
    int32_t* cell_start;           // ncell + 1
    int32_t* cid;                  // n
    int32_t* slot;                 // n: slot of each atom in its cell (arbitrary order)
    int32_t* order_tmp;            // n (unsorted within cells)
    int32_t* order;                // n
    double4* spos;                 // n + LJ_SPOS_PAD
    float4* spos32;                // n + LJ_SPOS_PAD: the same rounded to FP32 (x, y, z,
                                   // atom index bits)
    int32_t* block_sums;           // scan workspace
    bool counts_dirty;             // count[] may be non-zero (a build was interrupted)
};

struct lj_list {
    int device;                    // device of the context that built it
    hipStream_t stream;            // stream of its latest build or update
    int nsys;
    int64_t n;
    int kind;
    int lanes;                     // G
    int build_lanes;               // GB: lanes per row in the build, fixed at creation
    int64_t nslices, ncol;
    std::vector<lj_sys> hsys;      // all fields valid
    lj_sys* dsys;                  // device copy
    int32_t* slice_sys;            // nslices: system of each slice
    int32_t* row_atom;             // nslices * C
    int32_t* row_len;              // nslices * C
    int32_t* slice_iters;          // nslices
    int4* slice_stats;             // nslices: longest row before clamping, entries,
                                   // candidates tested, unused
    int32_t* col;                  // ncol
    lj_list_stats* stats;          // device, nsys
    bool stats_stale;              // stats predate the latest build
    lj_fconst* fc;                 // device, nsys: force constants of the last lj_forces*
    std::vector<lj_fconst> hfc;    // host copy of fc
    bool fc_valid;
    lj_cells* cells;               // owned cell structure for in-place rebuilds (lazy)
    double* acc;                   // half list: spread force accumulator, zero between calls
    int32_t* hwin;                 // half list: each force block's window of rank chunks
                                   // (count, then up to LJ_HWIN_MAX chunk offsets)
    uint4* q32;                    // mixed precision: fixed-point positions (one record per
                                   // row, lazy)
    double2* xy;                   // FP64 forces gather from this copy of the positions, one
    double* zz;                    // per row: (x, y) 16-byte records and z
};

// ---------------------------------------------------------------- errors
lj_status lj_fail(lj_status st, const std::string& msg);
lj_status lj_hip_fail(hipError_t e, const char* what);
#define LJ_HIP(call)                                            \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return lj_hip_fail(e_, #call);    \
    } while (0)

// ------------------------------------------------------ position layouts
// Kernels are built for two forms: AoS records whose first three doubles are
// (x, y, z) -- LJ_AOS4 (32-byte records) and LJ_AOS8 (64-byte records whose
// second half the caller uses, e.g. for velocities) -- and LJ_SOA.  The AoS
// record stride is passed as a shift.
inline int lj_tmpl_layout(int layout) { return layout == LJ_SOA ? LJ_SOA : LJ_AOS4; }
inline uint32_t lj_qshift(int layout) { return layout == LJ_AOS8 ? 6u : 5u; }

// -------------------------------------------------------------- launchers
// cells (lj_cells.hip).  gate: device word; when not NULL the kernels do
// nothing unless it is non-zero (a rebuild decided on the device).
lj_status lj_launch_cells(lj_ctx* ctx, const double* pos, int layout, lj_cells* c,
                          const int32_t* gate = nullptr);
int64_t lj_scan_workspace(int64_t m);
// neighbor list (lj_neigh.hip): rebuild every system of l from cells c; the
// per-system statistics (longest row, entries) follow at once with `stats`,
// else when they are next asked for (lj_launch_list_stats)
lj_status lj_launch_neighbors(lj_ctx* ctx, const lj_cells* c, lj_list* l, bool stats,
                              const int32_t* gate = nullptr);
lj_status lj_launch_list_stats(hipStream_t s, lj_list* l);
// lanes per row the list build of a new list uses (tuning knob, <= lanes)
int lj_build_lanes(const lj_ctx* ctx, int lanes);
// forces (lj_force.hip): per-system energy, virial, pair count
int64_t lj_force_blocks(int64_t nslices);

// Half lists: a force block sums the j contributions of its entries in LDS
// for the partners in its window, the set of chunks of LJ_HWIN_CHUNK
// consecutive ranks its entries name (at most LJ_HWIN_MAX chunks: those of
// the lowest offsets when a block names more), and adds each window record
// to the global accumulator once; partners outside the window are added
// directly.  A chunk is named by its offset from the chunk of the block's
// first row, taken modulo the system's chunks into (-nch/2, nch/2], and
// looked up in a table of LJ_HWIN_TABLE offsets.
#define LJ_HWIN_SHIFT 4
#define LJ_HWIN_CHUNK (1 << LJ_HWIN_SHIFT)
#define LJ_HWIN_MAX 96
#define LJ_HWIN_TABLE 16384
#define LJ_HWIN_REC (1 + LJ_HWIN_MAX)   // int32 per block in lj_list::hwin
__device__ __forceinline__ int lj_hwin_offset(int rel, int c0, int nch) {
    int off = (rel >> LJ_HWIN_SHIFT) - c0;
    off += off > nch / 2 ? -nch : (off <= -((nch + 1) / 2) ? nch : 0);
    return off;
}
// Window of the half list's force blocks, after each build (gated like it).
lj_status lj_launch_half_windows(lj_ctx* ctx, lj_list* l, const int32_t* gate);
// Reduction levels of the force kernel's block partials: the number of
// first-level spans per system (1: a single level), and the partial records
// (double4) the context must hold for list l.
int lj_force_split(const lj_list* l);
int64_t lj_force_partials(const lj_list* l);
// lj_forces_noalloc: block partials in a static device array of
// LJ_SCRATCH_RECORDS double4 records (4 MiB) per GPU; its device address
// on `device` (resolved once per device, then cached).
#define LJ_SCRATCH_RECORDS (1 << 17)
#define LJ_MAX_DEVICES 64
lj_status lj_scratch_partials(int device, double** ptr);
// Momentum update folded into the force pass (the impulse form of Alg. 1),
// full lists only: once a row's force F is summed, its atom's velocity is
// kicked in place.
//   LJ_KICK_SYNC : v += F dt/2 (the kick that ends a velocity-Verlet step)
//   LJ_KICK_LEAP : v += F dt/2 twice, each rounded as a separate kick: the
//                  kick that ends this step and the one that opens the next
//                  (the next drift then only moves the atoms)
// Either way the kinetic energy of the synchronised velocity (after the
// first kick) joins the block partials.
#define LJ_KICK_NONE 0
#define LJ_KICK_SYNC 1
#define LJ_KICK_LEAP 2

// LJ_MIXED needs the list's fixed-point position buffer (lj_list_ensure_q32,
// called before any launch that a graph may capture).
struct lj_force_opts {
    double* partials = nullptr;   // block partials (double4 records); NULL: the context's
    int64_t partials_cap = 0;     // their capacity in records
    int trunc = LJ_TRUNC_SHIFT;   // must match the constants in fc
    int kick = 0;                 // LJ_KICK_* (lj_force_loop.h), full lists only
    double* vel = nullptr;        // kicked velocities, layout of the positions
    double hdt = 0.0;             // dt / 2
    bool write_f = true;          // with a kick: also store the forces
    double* kinetic = nullptr;    // with a kick: per-system kinetic energy
};
lj_status lj_launch_forces(lj_ctx* ctx, const double* pos, int layout, int precision,
                           const lj_list* l, const lj_fconst* fc, double* force, double* energy,
                           double* virial, int64_t* npairs,
                           const lj_force_opts& o = lj_force_opts());
// host and device: one coordinate in the mixed kernel's fixed point,
// rint(x 2^32 / L) mod 2^32
__host__ __device__ __forceinline__ uint32_t lj_fix32(double x, double inv_unit) {
    return (uint32_t)(uint64_t)(int64_t)rint(x * inv_unit);
}
lj_status lj_list_ensure_q32(lj_list* l);
// integrator (lj_nve.hip)
lj_status lj_nve_make(lj_ctx* ctx, double* pos, double* vel, double* force, int32_t layout,
                      const lj_fconst* hfc, int32_t precision, int32_t trunc, lj_list* list,
                      double dt, int32_t rebuild_every, double* log, int64_t log_rows,
                      lj_nve** out);
lj_status lj_nve_start(lj_nve* s);
lj_status lj_nve_advance(lj_nve* s, int32_t nsteps, int32_t use_graph);
void lj_nve_release(lj_nve* s);
// steps completed since lj_nve_start, read from the device (synchronous)
lj_status lj_nve_device_steps(lj_nve* s, int64_t* steps);
lj_status lj_list_ensure_cells(lj_ctx* ctx, lj_list* l);
// exclusive scan of m int32 values into out[0..m] (out[m] = total); with
// clear_in the input is zeroed as it is read
lj_status lj_launch_scan(hipStream_t s, int32_t* in, int32_t* out, int64_t m, int32_t* work,
                         bool clear_in, const int32_t* gate = nullptr);
lj_status lj_launch_zero(hipStream_t s, void* p, int64_t bytes);
// host: force constants of one system with box lengths box[3]
lj_fconst lj_make_fconst(double eps, double sigma, double rc, const double box[3], int trunc);

// ------------------------------------------------------- device helpers
// Offset of entry k of a row from its slot base (the slice's first slot plus
// 4 c G for row c of the slice; layout above).
__host__ __device__ __forceinline__ uint32_t lj_slot(uint32_t base, uint32_t k, int G) {
    const uint32_t s = k / (uint32_t)G;
    return base + (s >> 2) * 256u + (k % (uint32_t)G) * 4u + (s & 3u);
}
// Logical block index that gives each XCD a contiguous range of blocks
// (the dispatcher deals consecutive workgroups round-robin to the 8 XCDs,
// each of which has its own L2).  A bijection on [0, nb).
__device__ __forceinline__ int64_t lj_xcd_block(int64_t b, int64_t nb) {
    const int64_t x = b % LJ_NXCD, l = b / LJ_NXCD;
    const int64_t per = nb / LJ_NXCD, rem = nb % LJ_NXCD;
    return x * per + (x < rem ? x : rem) + l;
}

// Cell coordinate of a coordinate value: floor(x * nc / L) clamped to the grid.
__device__ __forceinline__ int lj_cell_coord(double x, double inv_cs, int nc) {
    int k = (int)(x * inv_cs);
    k = k < 0 ? 0 : k;
    return k >= nc ? nc - 1 : k;
}
