/*
 * ljref.h -- CPU oracle for the truncated Lennard-Jones force over a Verlet list.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, scalar, obviously
 * correct FP64 reference that the GPU library is checked against.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no source, header, table or helper with the GPU library.
 *
 * What it computes (the paper: Watanabe & Nakagawa, "SIMD Vectorization for
 * the Lennard-Jones Potential with AVX2 and AVX-512 instructions"):
 *   - V(r) = 4 eps [ (sigma/r)^12 - (sigma/r)^6 ]                (Sec. III.A, Eq. 1)
 *     truncated at rc and shifted by a constant so that V(rc) = 0 (Sec. III.A);
 *   - the Verlet pair list with search length rs = rc + skin > rc, built with
 *     the linked-list cell method in O(N) and grouped by i with a counting
 *     sort into SortedList[i]                                    (Sec. III.B, III.C);
 *   - the force loop over the sorted list: i data held once per row, j data
 *     gathered, pairs beyond rc skipped, Newton's third law applied to j
 *     (Sec. III.C, Alg. 3, with the pair arithmetic of Alg. 1 returning the
 *     force rather than the impulse, and with +f on j, -f on i).
 *
 * Conventions shared by every function:
 *   pos   : host array, n x 3 doubles, row-major (x, y, z per atom), each
 *           coordinate in [0, box[d]).
 *   box   : 3 doubles, periodic box lengths; every box[d] must be >= 2 rs
 *           so that the minimum image is unique.
 *   Displacement t = q_j - q_i per dimension, then t -= L if t > L/2,
 *   t += L if t < -L/2; r2 = (tx*tx + ty*ty) + tz*tz, every operation
 *   rounded separately (built with -ffp-contract=off).
 *   A pair is listed iff r2 < rs*rs and interacts iff r2 < rc*rc (strict).
 *   Lists are CSR: row_ptr[n+1] (int64), col[] (int32), rows ascending in i,
 *   columns ascending in j; the half list holds each unordered pair once
 *   with i < j.
 * Return value: 0 on success, negative LJREF_E_* on error (outputs untouched).
 */
#ifndef LJREF_H
#define LJREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LJREF_OK 0
#define LJREF_E_INVALID (-1)
#define LJREF_E_BOX (-2)
#define LJREF_E_CAPACITY (-4)
#define LJREF_E_NOMEM (-6)

/* Truncation of the potential at rc (Sec. III.A), the `trunc` argument:
 *   LJREF_TRUNC_SHIFT        V(r) - V(rc) for r < rc: the paper's simple
 *                            truncation; the force is that of V and jumps to
 *                            zero at rc;
 *   LJREF_TRUNC_FORCE_SHIFT  V(r) - V(rc) + (r - rc) Fc with Fc = -V'(rc):
 *                            the force F(r) - Fc and the energy both vanish
 *                            at rc (the truncation Sec. III.A recommends for
 *                            energy conservation). */
#define LJREF_TRUNC_SHIFT 0
#define LJREF_TRUNC_FORCE_SHIFT 1

/* Half pair list by the definition: every i < j with r2 < rs^2, O(N^2).
 * cap: capacity of col; on overflow returns LJREF_E_CAPACITY with *npairs set
 * to the required size. */
int ljref_brute_pairs(int64_t n, const double* pos, const double* box, double rs,
                      int64_t cap, int64_t* row_ptr, int32_t* col, int64_t* npairs);

/* The same half list through the linked-list cell method (cells of side
 * >= rs, 27-cell stencil with repeated cells removed when a dimension has
 * fewer than 3 cells), then a counting sort of the pairs by i. */
int ljref_cell_pairs(int64_t n, const double* pos, const double* box, double rs,
                     int64_t cap, int64_t* row_ptr, int32_t* col, int64_t* npairs);

/* Forces, potential energy and virial over a half list (row_ptr, col).
 * force: n x 3 output.  energy = sum over listed pairs with r < rc of the
 * truncated pair energy; virial = sum of r . F_pair = fs * r2; n_in = number
 * of those pairs.  Energy and virial use compensated (Neumaier) summation. */
int ljref_forces(int64_t n, const double* pos, const double* box, double eps, double sigma,
                 double rc, int trunc, const int64_t* row_ptr, const int32_t* col,
                 double* force, double* energy, double* virial, int64_t* n_in);

/* The full list of a half list: every pair in both of its rows, rows and
 * columns ascending.  frow_ptr has n + 1 entries, fcol 2 row_ptr[n]. */
int ljref_full_pairs(int64_t n, const int64_t* row_ptr, const int32_t* col, int64_t* frow_ptr,
                     int32_t* fcol);

/* The same forces, energy and virial over a full list: each row sums its own
 * force and no j is updated, so the rows are independent and run under
 * OpenMP; the result does not depend on the thread count (row energies and
 * virials are compensated sums added afterwards in row order).  Every pair is
 * seen twice: energy, virial and n_in are halved. */
int ljref_forces_full(int64_t n, const double* pos, const double* box, double eps, double sigma,
                      double rc, int trunc, const int64_t* row_ptr, const int32_t* col,
                      double* force, double* energy, double* virial, int64_t* n_in);

/* Threads of the OpenMP loops (nthreads > 0 sets the count); returns the
 * count in effect.  Results never depend on it. */
int ljref_set_threads(int nthreads);

/* Per-atom quantities for a sample of atoms, found one by one with a cell
 * search (no list): for each sampled atom i,
 *   f[3s..3s+2]  force on i from every j with r < rc,
 *   e[s]         half of the sum of the truncated pair energies over those j,
 *   w[s]         half of the sum of fs * r2 over those j,
 *   nrs[s]       number of j with r < rs (the full-list row length),
 *   rows[s*rowcap ..] the j of that row ascending (if rows != NULL; the row is
 *                cut at rowcap entries, nrs still counts them all).
 * The sampled atoms are independent (OpenMP; same result on any thread count). */
int ljref_sample(int64_t n, const double* pos, const double* box, double eps, double sigma,
                 double rc, int trunc, double rs, int64_t ns, const int64_t* idx, double* f,
                 double* e, double* w, int64_t* nrs, int32_t* rows, int64_t rowcap);

/* Velocity Verlet at unit mass for nsteps steps of dt:
 *   v += F dt/2;  x += v dt (then wrap x - L floor(x/L), a result equal to L
 *   mapped to 0), and the displacement since the last build grows by v dt;
 *   rebuild the half list at the new x
 *     rebuild_every > 0: when step % rebuild_every == 0 (a fixed cadence);
 *     rebuild_every = 0: when some atom's displacement since the last build
 *       exceeds skin/2 (|d|^2 = (dx*dx + dy*dy) + dz*dz > (skin/2)^2), the
 *       first step at which a pair beyond rs at the build could have come
 *       within rc (Sec. III.B);
 *   after a rebuild the displacements restart from 0;  F = F(x);  v += F dt/2.
 * The list is built once before the first step.  log has (nsteps+1) rows of 6
 * doubles: potential energy, kinetic energy, virial, the largest displacement
 * of any atom since the last list build at the force evaluation, the number
 * of interacting pairs, and 1 if the list was built at that step (row 0: 1).
 * pos and vel are updated in place; force (n x 3) receives the last forces. */
int ljref_nve(int64_t n, double* pos, double* vel, const double* box, double eps,
              double sigma, double rc, int trunc, double skin, double dt, int32_t nsteps,
              int32_t rebuild_every, double* log, double* force);

#ifdef __cplusplus
}
#endif
#endif
