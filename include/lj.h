/*
 * lj.h -- C ABI of the MI355X (gfx950) Lennard-Jones Verlet-list library.
 *
 * The library computes the truncated 12-6 Lennard-Jones forces, potential
 * energy and virial of a periodic system over a Verlet neighbor list, and
 * builds that list with a cell (linked-list) search.  The method is the one
 * studied by Watanabe & Nakagawa, "SIMD Vectorization for the Lennard-Jones
 * Potential with AVX2 and AVX-512 instructions":
 *   - V(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6], truncated at rc and shifted
 *     by a constant so that V(rc) = 0 (Sec. III.A, Eq. 1);
 *   - the Verlet list registers every pair closer than the search length
 *     rs = rc + skin, built in O(N) with cells, so that it can be reused while
 *     atoms move less than skin/2; pairs beyond rc are masked at force time
 *     (Sec. III.B);
 *   - the list is grouped by i atom ("SortedList", built by a counting sort)
 *     so that the i data stays in registers over its row (Sec. III.C, Alg. 3);
 *   - positions may be stored as padded array-of-structures (x, y, z, pad:
 *     one 32-byte record per atom) or structure-of-arrays (Sec. III, Fig. 1;
 *     Sec. IV.A, Fig. 6).
 *
 * Conventions for every call:
 *   - Every call returns lj_status; nothing throws or aborts across the ABI.
 *     On an error the outputs are left untouched and lj_last_error() returns
 *     a text for the calling thread.
 *   - Device pointers are HIP device memory on the context's device.  The
 *     caller owns them (typically torch tensors); the library never frees
 *     them.  Host pointers are ordinary host memory.
 *   - Positions: `pos` with `layout`
 *       LJ_AOS4: n x 4 doubles, record i = (x_i, y_i, z_i, pad), 32-byte aligned;
 *       LJ_SOA : 3 x n doubles, x block then y block then z block;
 *       LJ_AOS8: n x 8 doubles, record i = (x_i, y_i, z_i, pad, 4 doubles of the
 *                caller), 32-byte aligned, n <= 2^26.
 *     Coordinates must be finite and lie in [0, box[d]).
 *   - Forces are returned in the same layout as the positions (the pad of
 *     an LJ_AOS4 record is written as 0; LJ_AOS8 positions give LJ_AOS4
 *     forces).
 *   - box: host array of 3 box lengths of the periodic, orthorhombic box.
 *     Every box[d] must be >= 2 (rc + skin) so that the nearest image of a
 *     pair within the search length is unique (LJ_E_BOX otherwise).
 *   - Displacement of a pair: t = q_j - q_i per dimension, brought to the
 *     nearest image; a pair is listed iff |t|^2 < (rc + skin)^2 and
 *     interacts iff |t|^2 < rc^2 (strict).  The list build evaluates |t|^2 as
 *     (tx*tx + ty*ty) + tz*tz with every operation rounded on its own, so the
 *     set of listed pairs is exactly that of this definition.
 *   - Work is enqueued on the context's HIP stream and is asynchronous unless
 *     a call says otherwise.  A context must be used by one host thread at a
 *     time; two calls that overlap on one context race.
 *   - Errors found on the device (a bad coordinate, a list row over its
 *     capacity) are recorded in the context and reported by the next lj_sync.
 *     Until then every force and integrator launch of the context leaves its
 *     outputs untouched.
 */
#ifndef LJ_H
#define LJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(LJ_BUILD)
#define LJ_API __attribute__((visibility("default")))
#else
#define LJ_API
#endif

/* Largest atom count of one call (all systems of a batch together): kernels
 * address 32-byte records with 32-bit byte offsets. */
#define LJ_MAX_ATOMS (1LL << 27)

typedef enum {
    LJ_OK = 0,
    LJ_E_INVALID = -1,   /* NULL pointer, n < 1, n > LJ_MAX_ATOMS, rc <= 0, skin < 0,
                            eps/sigma <= 0, non-finite parameter, unknown enum value */
    LJ_E_BOX = -2,       /* some box[d] < 2 (rc + skin) */
    LJ_E_POSITION = -3,  /* a coordinate is non-finite or outside [0, box[d]) */
    LJ_E_CAPACITY = -4,  /* a fixed capacity was exceeded (see the call) */
    LJ_E_STALE = -5,     /* the list does not match the positions or parameters */
    LJ_E_NOMEM = -6,     /* device or host allocation failed */
    LJ_E_HIP = -7,       /* a HIP runtime call failed */
    LJ_E_NODEVICE = -8   /* no usable gfx950 device */
} lj_status;

/* list kinds */
#define LJ_LIST_HALF 0   /* each unordered pair once; forces use Newton's third law
                            and scatter to j with atomic adds (Alg. 3) */
#define LJ_LIST_FULL 1   /* each pair in both rows; no atomics, every row owns its sum */
/* precisions */
#define LJ_FP64 0        /* every operation in FP64 */
#define LJ_MIXED 1       /* positions read as 32-bit fixed point in the box (the
                            displacement is off by at most L / 2^32 per component);
                            r^2 in FP64 and the cutoff test exact (the same pairs as
                            LJ_FP64); the pair terms ((sigma/r)^2, ^6, the force
                            factor and pair energy) in FP32; per-atom force, energy
                            and virial accumulated in FP64.  The quantisation adds a
                            relative force error of about 13 (L / 2^32) / r: ~1e-7
                            for L ~ 100 sigma, near 1e-5 for L ~ 3,000 sigma (use
                            LJ_FP64 for such boxes).  Needs n x 16 bytes more device
                            memory per list (allocated on first use) */
/* position / force layouts */
#define LJ_AOS4 0
#define LJ_SOA 1
#define LJ_AOS8 2        /* positions only: n records of 8 doubles (x, y, z, pad, u0, u1, u2,
                            pad), 32-byte aligned, of which the library reads the first
                            three: the packed (q, p) records of Sec. V.F (in the integrator
                            the second half holds the velocity).  Forces for LJ_AOS8
                            positions are LJ_AOS4 records.  At most 2^26 atoms */
/* truncation of the potential at rc (Sec. III.A) */
#define LJ_TRUNC_SHIFT 0         /* V(r) - V(rc) for r < rc: the potential is shifted by a
                                    constant; the force is that of V and jumps to 0 at rc */
#define LJ_TRUNC_FORCE_SHIFT 1   /* V(r) - V(rc) + (r - rc) Fc, Fc = -V'(rc): force
                                    F(r) - Fc along the pair; force and energy both vanish
                                    at rc (the remedy for energy conservation) */

typedef struct lj_ctx lj_ctx;
typedef struct lj_cells lj_cells;
typedef struct lj_list lj_list;

/* Description of a built list (lj_list_info). */
typedef struct {
    int64_t n;            /* atoms (rows) */
    int32_t kind;         /* LJ_LIST_HALF or LJ_LIST_FULL */
    int32_t lanes;        /* lanes of a 64-wide wavefront that share one row */
    int32_t cap;          /* entries reserved per row */
    int32_t max_row;      /* longest row */
    int64_t entries;      /* stored (i, j) entries: pairs (half) or 2 x pairs (full) */
    int64_t slots;        /* entries including the padding of each wavefront slice */
    double rc, skin;      /* cutoff and skin the list was built for */
    double box[3];        /* box it was built in (system 0 of a batch) */
    int32_t nc[3];        /* cells per dimension used by the search (system 0) */
    int32_t nsys;         /* systems in the list (1 unless built as a batch) */
    int32_t pad;
    int64_t tests;        /* candidate pairs the latest build tested (distance tests) */
} lj_list_desc;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  `stream` is a hipStream_t (NULL =
 * the null stream); it is not owned.  Fails with LJ_E_NODEVICE if the device
 * is missing or is not gfx950. */
LJ_API lj_status lj_create(int device, void* stream, lj_ctx** out);
LJ_API lj_status lj_destroy(lj_ctx* ctx);
/* Point the context at another stream (not owned). */
LJ_API lj_status lj_set_stream(lj_ctx* ctx, void* stream);
/* Wait for the context's stream and report device-side errors raised by
 * asynchronous calls since the last check (LJ_E_POSITION, LJ_E_CAPACITY, and
 * LJ_E_STALE for an integrator step at a fixed rebuild cadence whose atoms
 * had moved more than skin/2 since the list was built); each error is
 * reported once and cleared. */
LJ_API lj_status lj_sync(lj_ctx* ctx);

/* ------------------------------------------------------------------ cells */

/* Bin the atoms into a grid of cells of side >= min_cell per dimension
 * (cells per dimension nc[d] = the largest count whose side is >= min_cell)
 * and sort them by cell with a stable counting sort: atoms of a cell are
 * contiguous and in ascending index (the linked-list method of Sec. III.B and
 * the counting sort of Sec. III.C, in array form).  Synchronous: positions
 * are validated and LJ_E_POSITION is returned for a bad coordinate.  *cells
 * is owned by the library until lj_cells_free. */
LJ_API lj_status lj_build_cells(lj_ctx* ctx, const double* pos, int64_t n, int32_t layout,
                         const double box[3], double min_cell, lj_cells** cells);
/* Grid shape and atom count of a cell structure. */
LJ_API lj_status lj_cells_info(const lj_cells* cells, int32_t nc[3], int64_t* n);
/* Copy the cell structure to the host: cell_start (ncell + 1 entries, atoms
 * of cell c are order[cell_start[c] .. cell_start[c+1])), order (n entries),
 * cell ids are (cz * nc[1] + cy) * nc[0] + cx.  Either pointer may be NULL.
 * Synchronous. */
LJ_API lj_status lj_cells_export(lj_ctx* ctx, const lj_cells* cells, int32_t* cell_start,
                          int32_t* order);
LJ_API lj_status lj_cells_free(lj_cells* cells);

/* --------------------------------------------------------------- the list */

/* Build the Verlet list of pairs closer than rs = rc + skin (Sec. III.B).
 * kind: LJ_LIST_HALF or LJ_LIST_FULL.  lanes: lanes of a wavefront that share
 * one row in the force kernel (1, 2, 4, 8, 16, 32 or 64; 0 = the library's
 * tuned choice); the list is laid out for that width.  cells: a structure
 * from lj_build_cells on the same positions with cells of side >= rs, or NULL
 * to build one internally.  Synchronous (one device-to-host read of the
 * longest row; the per-row capacity grows and the build repeats if it was
 * too small).  *list is owned by the library until lj_list_free.
 * Rows follow the cell order of the atoms; in a half list the pair (a, b)
 * sits in exactly one of the two rows, chosen so that every row holds about
 * half of its atom's neighbors. */
LJ_API lj_status lj_build_neighbors(lj_ctx* ctx, const double* pos, int64_t n, int32_t layout,
                             const double box[3], double rc, double skin, int32_t kind,
                             int32_t lanes, const lj_cells* cells, lj_list** list);
/* Rebuild the list in place for new positions of the same atoms (same n,
 * box, rc, skin, kind and lanes): the cells are binned and sorted again and
 * the rows refilled, reusing the list's buffers.  Asynchronous and free of
 * host synchronisation and allocation (safe inside HIP graph capture after the
 * list's first update).  A coordinate outside the box or a row longer than the
 * list's capacity is recorded on the device and reported by the next lj_sync
 * (LJ_E_POSITION, LJ_E_CAPACITY); after LJ_E_CAPACITY the list's contents are
 * incomplete and it must be built again with lj_build_neighbors. */
LJ_API lj_status lj_update_neighbors(lj_ctx* ctx, const double* pos, int64_t n, int32_t layout,
                                     const double box[3], lj_list* list);
/* Describe the list.  Synchronous: reads the row statistics of the latest
 * build or update from the device. */
LJ_API lj_status lj_list_info(const lj_list* list, lj_list_desc* out);
/* Copy the list's entries to the host as (i, j) atom-index pairs: ij[2k],
 * ij[2k+1] for k < *npairs.  cap: capacity of ij in pairs; if it is too small
 * *npairs receives the required count and LJ_E_CAPACITY is returned.
 * Synchronous. */
LJ_API lj_status lj_list_pairs(lj_ctx* ctx, const lj_list* list, int64_t cap, int32_t* ij,
                        int64_t* npairs);
LJ_API lj_status lj_list_free(lj_list* list);

/* Read-only device view of a list's layout, for kernels of the caller that
 * consume the list directly.  Rows are the atoms in cell order, grouped in
 * slices of C = 64 / lanes rows.  Entry k of row c of slice s is taken at
 * step t = k / lanes by lane p = c * lanes + k % lanes of a wavefront, and
 * sits at
 *   col[s * (cap / lanes) * 64 + (t / 4) * 256 + p * 4 + t % 4]
 * for k < row_len[s * C + c] (each lane finds its indices of 4 consecutive
 * steps in 16 contiguous bytes; cap is a multiple of 4 lanes).  Entries are
 * cell-sorted ranks: row r is the atom of rank r, row_atom[r] (for a row
 * r < n), so the atom of entry j is row_atom[j].  Slots past a row's length,
 * up to slice_iters[s] rounded up to a multiple of 4 steps, hold the row's
 * own rank.  The pointers stay valid until the list is rebuilt or freed. */
typedef struct {
    const int32_t* col;
    const int32_t* row_atom;     /* nslices * C */
    const int32_t* row_len;      /* nslices * C */
    const int32_t* slice_iters;  /* nslices */
    int64_t nslices;
    int32_t lanes, cap;
} lj_list_view;
LJ_API lj_status lj_list_device_view(const lj_list* list, lj_list_view* out);

/* ----------------------------------------------------------------- forces */

/* Forces, potential energy and virial of the truncated, shifted LJ potential
 * over the list (Alg. 1 inside the sorted-list loop of Alg. 3, returning the
 * force rather than the impulse).  For every listed pair with r^2 < rc^2:
 *   fs = 24 eps (sigma/r)^6 [2 (sigma/r)^6 - 1] / r^2,  F_j += fs t,  F_i -= fs t,
 *   energy += 4 eps (sigma/r)^6 [(sigma/r)^6 - 1] - V(rc),  virial += fs r^2.
 * force: device, n records in `layout`.  energy, virial: device, 1 double
 * each.  npairs: device int64 receiving the number of interacting pairs, or
 * NULL.  precision: LJ_FP64 or LJ_MIXED.  The list must have been built for
 * the same n, layout, box and rc (LJ_E_STALE otherwise), and is valid while
 * no atom has moved more than skin/2 since the build (not checked here).
 * trunc: LJ_TRUNC_SHIFT (the above) or LJ_TRUNC_FORCE_SHIFT (fs - Fc / r in
 * place of fs, and (r - rc) Fc added to each pair's energy).
 * Asynchronous; energy, virial and npairs are reduced on the device in a
 * fixed order, so a full list gives bitwise-reproducible results.  While an
 * error is pending on the context (see lj_sync) nothing is written. */
LJ_API lj_status lj_forces(lj_ctx* ctx, const double* pos, int64_t n, int32_t layout,
                    const double box[3], double eps, double sigma, double rc,
                    const lj_list* list, int32_t precision, int32_t trunc, double* force,
                    double* energy, double* virial, int64_t* npairs);

/* lj_forces for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, results and kernels, but the per-block energy/virial
 * partials live in a static device array of the library (131,072 records of
 * 32 bytes, 4 MiB, on each GPU it runs on, held until the process ends)
 * instead of the context's buffer, and the call allocates nothing.
 * LJ_E_CAPACITY if the list needs more partials than that (about 4M atoms
 * at 8 lanes per row); LJ_E_INVALID for LJ_MIXED before the list's
 * fixed-point buffer exists (lj_forces creates it on its first mixed call).
 * Every call on one GPU shares that array: calls that overlap on a GPU (two
 * streams or contexts) race and must be ordered by the caller.  The first
 * call with new eps, sigma, rc or truncation uploads them (synchronously);
 * with the profiler on, timing events are created. */
LJ_API lj_status lj_forces_noalloc(lj_ctx* ctx, const double* pos, int64_t n, int32_t layout,
                                   const double box[3], double eps, double sigma, double rc,
                                   const lj_list* list, int32_t precision, int32_t trunc,
                                   double* force, double* energy, double* virial,
                                   int64_t* npairs);

/* ----------------------------------------------------------------- batches */

/* Many independent systems of uneven size handled by every launch together
 * (one launch per phase covers all systems).  System s owns the records
 * [off_s, off_s + n[s]) of the caller's concatenated arrays, off_s = n[0] +
 * ... + n[s-1], in the layout given (an LJ_SOA array is 3 x N for the total
 * N).  Host arrays: n[nsys], box[3 * nsys], rc[nsys], eps[nsys], sigma[nsys].
 * Each system has its own periodic box, cutoff and cells; the skin, list kind
 * and lanes are shared.  The list's pairs (lj_list_pairs) carry record
 * indices of the concatenated arrays; pairs never join two systems. */
LJ_API lj_status lj_build_neighbors_batch(lj_ctx* ctx, const double* pos, int32_t layout,
                                          int32_t nsys, const int64_t* n, const double* box,
                                          const double* rc, double skin, int32_t kind,
                                          int32_t lanes, lj_list** list);
/* Forces over a batch list.  energy, virial: device arrays of nsys doubles;
 * npairs: device array of nsys int64 or NULL. */
LJ_API lj_status lj_forces_batch(lj_ctx* ctx, const double* pos, int32_t layout,
                                 const lj_list* list, const double* eps, const double* sigma,
                                 const double* rc, int32_t precision, int32_t trunc,
                                 double* force, double* energy, double* virial,
                                 int64_t* npairs);
/* Row statistics of system s of a list (synchronous). */
LJ_API lj_status lj_list_sys_info(const lj_list* list, int32_t s, int64_t* n, int32_t* max_row,
                                  int64_t* entries, int32_t* cap);

/* -------------------------------------------------------------- integrator */

/* Velocity-Verlet NVE integration at unit mass around the force path.  One
 * step, as in the oracle:
 *   v += F dt/2;  x += v dt, wrapped to x - L floor(x/L) (a result equal to L
 *   becomes 0), and each atom's displacement since the last list build grows
 *   by v dt;  the list is rebuilt in place at the new positions
 *   (lj_update_neighbors)
 *     rebuild_every > 0: when step % rebuild_every == 0 (a fixed cadence; a
 *       step between builds at which some atom has moved more than skin/2
 *       since the build is reported as LJ_E_STALE by lj_sync, the list may
 *       then miss pairs);
 *     rebuild_every = 0: when some atom's displacement since the last build
 *       exceeds skin/2 (|d|^2 = (dx*dx + dy*dy) + dz*dz > (skin/2)^2), the
 *       first step at which a pair beyond rs at the build could have come
 *       within rc (Sec. III.B: the list stays exact); decided on the device;
 *   F = F(x) (lj_forces, in the integrator's precision and truncation);
 *   v += F dt/2.
 * With a full list and a fixed cadence, the kick that ends a step is folded
 * into the force pass (the momentum update of Alg. 1), and inside a rebuild
 * cycle so is the kick that opens the next step, each rounded as a separate
 * kick (the trajectory is the same bit for bit).
 * All state stays on the device and the integrator itself is FP64 whatever
 * the force precision.  The caller's arrays are bound at creation (so that a
 * captured HIP graph can replay them): pos, vel and force are device arrays
 * of n records in `layout`; with LJ_AOS8, pos holds the packed (x, y, z, pad,
 * vx, vy, vz, pad) records, vel must be pos + 4 and force is LJ_AOS4.  log
 * is a device array of log_rows x 6 doubles that receives, for step s (row s,
 * when s < log_rows): potential energy, kinetic energy (sum of v^2/2),
 * virial, the largest displacement of any atom since the last list build
 * (0 at a step that rebuilt), the number of interacting pairs, and 1 if the
 * list was rebuilt at that step (row 0: 1).  The list must belong to the same
 * context and stay alive while the integrator is used.  *out is owned by the
 * library until lj_nve_free. */
typedef struct lj_nve lj_nve;
LJ_API lj_status lj_nve_create(lj_ctx* ctx, double* pos, double* vel, double* force, int64_t n,
                               int32_t layout, const double box[3], double eps, double sigma,
                               double rc, int32_t precision, int32_t trunc, lj_list* list,
                               double dt, int32_t rebuild_every, double* log, int64_t log_rows,
                               lj_nve** out);
/* The integrator of a batch list: eps, sigma, rc are host arrays of nsys
 * values; the log holds log_rows x nsys x 6 doubles (row, system, quantity).
 * With rebuild_every = 0 every system is rebuilt at a step at which any
 * system needs it. */
LJ_API lj_status lj_nve_create_batch(lj_ctx* ctx, double* pos, double* vel, double* force,
                                     int32_t layout, const double* eps, const double* sigma,
                                     const double* rc, int32_t precision, int32_t trunc,
                                     lj_list* list, double dt, int32_t rebuild_every,
                                     double* log, int64_t log_rows, lj_nve** out);
/* Step 0: forces at the current positions and log row 0; resets the step
 * count and the displacement record.  Asynchronous. */
LJ_API lj_status lj_nve_init(lj_nve* nve);
/* Advance nsteps steps.  use_graph != 0: whole rebuild cycles (rebuild_every
 * steps ending with a rebuild; 10 steps when rebuild_every = 0) are captured
 * once into a HIP graph and replayed; the remaining steps run as ordinary
 * launches.  The arithmetic is the same as taking the steps one call at a
 * time, bit for bit, and vel holds the synchronised velocities when the run
 * ends.  Requires the context's stream to be a created stream (not the null
 * stream) when use_graph != 0.  Asynchronous.  If a list rebuild meets a bad
 * coordinate or a row over the list's capacity, the run stops at its last
 * good step: pos, vel and force are restored to that step's values, the
 * later steps (and their log rows) are skipped, lj_sync reports the error
 * and lj_nve_steps the last good step.  The list must then be built again
 * (lj_build_neighbors) for a new integrator. */
LJ_API lj_status lj_nve_run(lj_nve* nve, int32_t nsteps, int32_t use_graph);
/* Steps completed since lj_nve_init.  Synchronous (reads the device's step
 * counter: after an error, the last good step). */
LJ_API lj_status lj_nve_steps(const lj_nve* nve, int64_t* steps);
LJ_API lj_status lj_nve_free(lj_nve* nve);

/* ------------------------------------------------------------------ tuning */

/* Launch-shape knobs of a context, set by the autotuner (or by hand).  They
 * change only speed, never results: every setting computes the same list
 * (as a set) and the same forces.  0 selects the library's default. */
#define LJ_TUNE_BUILD_LANES 0   /* lanes per row in the list-build kernel: 64 (the
                                   whole wavefront builds one row at a time, the
                                   default) or 1, 2 or 4 (groups of lanes build
                                   rows side by side, at most the list's lanes).
                                   Fixed for a list when it is created. */
#define LJ_TUNE_FORCE_BATCH 1   /* list entries each lane has in flight in the force
                                   kernel: 4 or 8 (2 is accepted and runs as 4);
                                   default 4 */
#define LJ_TUNE_CELL_DIV 2      /* lists built without caller cells use cells of side
                                   (rc + skin) / k in y and z and half that in x,
                                   k = 1, 2, 3 or 4; default 2 */
#define LJ_TUNE_KICK 3          /* integrators created afterwards: 1 folds the kicks into
                                   the force pass where it can (full list, fixed cadence;
                                   the default), 2 keeps them in separate kernels.  The
                                   trajectory is the same bit for bit */
#define LJ_TUNE_N 4
/* Set knob `knob` to `value` (LJ_E_INVALID for an unknown knob or value). */
LJ_API lj_status lj_tune_set(lj_ctx* ctx, int32_t knob, int32_t value);
/* Current value of a knob (0 = default). */
LJ_API lj_status lj_tune_get(const lj_ctx* ctx, int32_t knob, int32_t* value);

/* ---------------------------------------------------------------- profiling */

/* Phases timed by the profiler (HIP events recorded on the context's stream
 * around each launch). */
#define LJ_PROF_CELLS 0   /* binning, prefix sum, scatter, per-cell sort */
#define LJ_PROF_NEIGH 1   /* the list-build kernel */
#define LJ_PROF_FORCE 2   /* the force kernel */
#define LJ_PROF_OTHER 3   /* energy/virial reduction, half-list force write-out, zero fills */
#define LJ_PROF_INTEGRATE 4  /* NVE: drift, kick (fused or alone), log row */
#define LJ_PROF_N 5
/* Start recording (drops anything recorded before). */
LJ_API lj_status lj_profile_begin(lj_ctx* ctx);
/* Stop recording, wait for the stream and return, per phase, the summed
 * device time in milliseconds and the number of launches (arrays of
 * LJ_PROF_N entries, host).  At most 65,536 launches are recorded. */
LJ_API lj_status lj_profile_end(lj_ctx* ctx, double* ms, int64_t* launches);

/* Text of the last error on the calling thread ("" if none). */
LJ_API const char* lj_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LJ_H */
