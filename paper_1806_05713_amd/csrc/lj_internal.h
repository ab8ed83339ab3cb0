// lj_internal.h -- internal structures and launchers of the gfx950 LJ library.
//
// Data layout in HBM (per system):
//   positions     caller's array: n x double4 (x, y, z, pad) or SoA 3 x n
//   cells         count[ncell], cell_start[ncell + 1], cid[n] (cell of atom),
//                 order[n] (cell-sorted rank -> atom), spos[n] (cell-sorted
//                 double4 (x, y, z, atom index as a double))
//   list          wavefront-sliced rows: rows are the atoms in cell order; a
//                 wavefront of 64 lanes serves C = 64 / G rows with G lanes
//                 each; entry k of row c of slice s is stored at
//                   col[(s * (cap / G) + k / G) * 64 + c * G + k % G]
//                 so that one 64-lane load fetches 256 contiguous bytes.
//                 row_atom[r], row_len[r] per row, slice_iters[s] = the
//                 longest row of the slice in G-wide steps.  Slots past a
//                 row's length (up to its slice's length) hold the row's own
//                 atom so that every gather stays in bounds.
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

// Device status words of a context.
struct lj_dev_status {
    int32_t flags;                 // LJ_DEV_* bits raised by kernels
    int32_t pad0;
    unsigned long long pad1;
    unsigned int done_blocks;      // arrival counter of the last-block reductions
    unsigned int pad;
};

// Row statistics of a list, written by its latest build on the device.
struct lj_list_stats {
    int32_t max_row;               // longest row (before clamping to the capacity)
    int32_t pad;
    unsigned long long entries;    // entries stored
};
#define LJ_DEV_BAD_POSITION 1
#define LJ_DEV_ROW_OVERFLOW 2
#define LJ_DEV_CELL_OVERFLOW 4

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
    bool prof_on;
    std::vector<lj_prof_rec> prof;
    int32_t tune[LJ_TUNE_N];       // tuning knobs (lj_tune_set)
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
    int64_t n;
    int nc[3];
    double cs[3];
    double box[3];
    int64_t ncell;
    int32_t* count;      // ncell
    int32_t* cell_start; // ncell + 1
    int32_t* cid;        // n
    int32_t* order_tmp;  // n (unsorted within cells)
    int32_t* order;      // n
    double4* spos;       // n
    int32_t* block_sums; // scan workspace
    bool counts_dirty;   // count[] may be non-zero (a build was interrupted)
};

struct lj_list {
    int64_t n;
    int kind;
    int lanes;         // G
    int cap;           // multiple of G
    int max_row;
    int64_t entries;
    int64_t nslices;
    double rc, skin, box[3];
    int nc[3];
    int32_t* row_atom;     // nslices * C
    int32_t* row_len;      // nslices * C
    int32_t* slice_iters;  // nslices
    int32_t* slice_stats;  // 2 * nslices: longest row before clamping, entries
    int32_t* col;          // nslices * (cap / G) * 64
    lj_list_stats* stats;  // device
    lj_cells* cells;       // owned cell structure for in-place rebuilds (lazy)
};

// ---------------------------------------------------------------- errors
lj_status lj_fail(lj_status st, const std::string& msg);
lj_status lj_hip_fail(hipError_t e, const char* what);
#define LJ_HIP(call)                                            \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return lj_hip_fail(e_, #call);    \
    } while (0)

// -------------------------------------------------------------- launchers
// cells (lj_cells.hip)
lj_status lj_launch_cells(lj_ctx* ctx, const double* pos, int layout, lj_cells* c);
int64_t lj_scan_workspace(int64_t m);
// neighbor list (lj_neigh.hip)
lj_status lj_launch_neighbors(lj_ctx* ctx, const lj_cells* c, lj_list* l, double rs);
int64_t lj_force_blocks(int64_t nslices);
// forces (lj_force.hip)
struct lj_force_params {
    double box[3];
    double eps, sigma, rc;
    int layout, precision;
};
lj_status lj_launch_forces(lj_ctx* ctx, const double* pos, const lj_list* l,
                           const lj_force_params& p, double* force, double* energy,
                           double* virial, int64_t* npairs);
// integrator (lj_nve.hip)
lj_status lj_nve_make(lj_ctx* ctx, double* pos, double* vel, double* force, int64_t n,
                      int32_t layout, const double box[3], double eps, double sigma, double rc,
                      int32_t precision, lj_list* list, double dt, int32_t rebuild_every,
                      double* log, int64_t log_rows, lj_nve** out);
lj_status lj_nve_start(lj_nve* s);
lj_status lj_nve_advance(lj_nve* s, int32_t nsteps, int32_t use_graph);
void lj_nve_release(lj_nve* s);
int64_t lj_nve_step_count(const lj_nve* s);
lj_status lj_list_ensure_cells(lj_ctx* ctx, lj_list* l);
// exclusive scan of m int32 values into out[0..m] (out[m] = total)
lj_status lj_launch_scan(hipStream_t s, const int32_t* in, int32_t* out, int64_t m,
                         int32_t* work);
lj_status lj_launch_zero(hipStream_t s, void* p, int64_t bytes);

// ------------------------------------------------------- device helpers
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
