/*
 * ljref.c -- CPU oracle (test infrastructure only; see ljref.h).
 *
 * Plain scalar FP64, one function per step of the method, in the order and
 * notation of the paper (Sec. III).  Built with -O2 -ffp-contract=off so that
 * every product and sum is rounded on its own.  Nothing here is tuned: the
 * only parallelism is an OpenMP loop over rows in the O(N^2) brute force,
 * which writes each row independently (same result with any thread count).
 */
#include "ljref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- geometry */

/* Minimum-image component of q_j - q_i in a periodic box of side L (Sec. II:
 * a cubic periodic box; L >= 2 rs makes the nearest image unique). */
static double min_image(double t, double L) {
    if (t > 0.5 * L)
        t -= L;
    else if (t < -0.5 * L)
        t += L;
    return t;
}

/* r = q_j - q_i (minimum image) and r^2 = r . r (Alg. 1, first two lines). */
static double displacement(const double* qi, const double* qj, const double* box, double t[3]) {
    t[0] = min_image(qj[0] - qi[0], box[0]);
    t[1] = min_image(qj[1] - qi[1], box[1]);
    t[2] = min_image(qj[2] - qi[2], box[2]);
    return (t[0] * t[0] + t[1] * t[1]) + t[2] * t[2];
}

static int check_args(int64_t n, const double* pos, const double* box, double rs) {
    if (n < 1 || pos == NULL || box == NULL || !(rs > 0.0) || !isfinite(rs)) return LJREF_E_INVALID;
    for (int d = 0; d < 3; ++d) {
        if (!(box[d] > 0.0) || !isfinite(box[d])) return LJREF_E_INVALID;
        if (box[d] < 2.0 * rs) return LJREF_E_BOX;
    }
    return LJREF_OK;
}

/* Compensated (Neumaier) accumulation, so that the reference energy and
 * virial are accurate to about one rounding of the final value. */
typedef struct { double s, c; } ksum;
static void ksum_add(ksum* k, double x) {
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x))
        k->c += (k->s - t) + x;
    else
        k->c += (x - t) + k->s;
    k->s = t;
}
static double ksum_get(const ksum* k) { return k->s + k->c; }

/* --------------------------------------------------- the list by definition */

int ljref_brute_pairs(int64_t n, const double* pos, const double* box, double rs, int64_t cap,
                      int64_t* row_ptr, int32_t* col, int64_t* npairs) {
    int st = check_args(n, pos, box, rs);
    if (st) return st;
    if (row_ptr == NULL || npairs == NULL || cap < 0) return LJREF_E_INVALID;
    const double rs2 = rs * rs;
    int64_t* cnt = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    if (!cnt) return LJREF_E_NOMEM;
    /* pass 1: how many j > i lie within rs of each i */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double t[3];
        int64_t c = 0;
        for (int64_t j = i + 1; j < n; ++j)
            if (displacement(pos + 3 * i, pos + 3 * j, box, t) < rs2) ++c;
        cnt[i] = c;
    }
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) total += cnt[i];
    *npairs = total;
    if (total > cap || (total > 0 && col == NULL)) {
        free(cnt);
        return LJREF_E_CAPACITY;
    }
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
    /* pass 2: the same test again, writing j in ascending order */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double t[3];
        int64_t k = row_ptr[i];
        for (int64_t j = i + 1; j < n; ++j)
            if (displacement(pos + 3 * i, pos + 3 * j, box, t) < rs2) col[k++] = (int32_t)j;
    }
    free(cnt);
    return LJREF_OK;
}

/* ------------------------------------------------- linked-list cell method */

typedef struct {
    int nc[3];
    double cs[3];
    int64_t ncell;
    int64_t* head; /* first atom of each cell, -1 if empty */
    int64_t* next; /* next atom in the same cell, -1 at the end */
} cell_grid;

/* Cells of side cs = L/nc >= rs (with a relative margin of 1e-12 so that a
 * coordinate rounded onto a cell face cannot hide a pair). */
static int grid_build(cell_grid* g, int64_t n, const double* pos, const double* box, double rs) {
    g->ncell = 1;
    for (int d = 0; d < 3; ++d) {
        int nc = (int)floor(box[d] / rs);
        while (nc > 1 && box[d] / nc < rs * (1.0 + 1e-12)) --nc;
        if (nc < 1) nc = 1;
        g->nc[d] = nc;
        g->cs[d] = box[d] / nc;
        g->ncell *= nc;
    }
    g->head = (int64_t*)malloc((size_t)g->ncell * sizeof(int64_t));
    g->next = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!g->head || !g->next) {
        free(g->head);
        free(g->next);
        return LJREF_E_NOMEM;
    }
    for (int64_t c = 0; c < g->ncell; ++c) g->head[c] = -1;
    /* insert atoms in descending order so that each cell's chain runs in
     * ascending atom index */
    for (int64_t i = n - 1; i >= 0; --i) {
        int64_t c = 0;
        for (int d = 2; d >= 0; --d) {
            int k = (int)(pos[3 * i + d] / g->cs[d]);
            if (k < 0) k = 0;
            if (k >= g->nc[d]) k = g->nc[d] - 1;
            c = c * g->nc[d] + k;
        }
        g->next[i] = g->head[c];
        g->head[c] = i;
    }
    return LJREF_OK;
}

static void grid_free(cell_grid* g) {
    free(g->head);
    free(g->next);
}

/* The distinct cells among the 27 around the cell of a point (a dimension
 * with fewer than 3 cells repeats cells; each is kept once).  Returns count. */
static int grid_stencil(const cell_grid* g, const double* q, int64_t out[27]) {
    int c[3];
    for (int d = 0; d < 3; ++d) {
        int k = (int)(q[d] / g->cs[d]);
        if (k < 0) k = 0;
        if (k >= g->nc[d]) k = g->nc[d] - 1;
        c[d] = k;
    }
    int m = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int x = (c[0] + dx + g->nc[0]) % g->nc[0];
                int y = (c[1] + dy + g->nc[1]) % g->nc[1];
                int z = (c[2] + dz + g->nc[2]) % g->nc[2];
                int64_t id = ((int64_t)z * g->nc[1] + y) * g->nc[0] + x;
                int seen = 0;
                for (int k = 0; k < m; ++k)
                    if (out[k] == id) seen = 1;
                if (!seen) out[m++] = id;
            }
    return m;
}

int ljref_cell_pairs(int64_t n, const double* pos, const double* box, double rs, int64_t cap,
                     int64_t* row_ptr, int32_t* col, int64_t* npairs) {
    int st = check_args(n, pos, box, rs);
    if (st) return st;
    if (row_ptr == NULL || npairs == NULL || cap < 0) return LJREF_E_INVALID;
    const double rs2 = rs * rs;
    cell_grid g;
    st = grid_build(&g, n, pos, box, rs);
    if (st) return st;

    /* Pair list (i, j) with i < j (Fig. 3a), in the order the cell search finds them. */
    int64_t pcap = 1024, np = 0;
    int32_t* pi = (int32_t*)malloc((size_t)pcap * sizeof(int32_t));
    int32_t* pj = (int32_t*)malloc((size_t)pcap * sizeof(int32_t));
    if (!pi || !pj) {
        free(pi);
        free(pj);
        grid_free(&g);
        return LJREF_E_NOMEM;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t st_cells[27];
        int m = grid_stencil(&g, pos + 3 * i, st_cells);
        for (int k = 0; k < m; ++k) {
            for (int64_t j = g.head[st_cells[k]]; j >= 0; j = g.next[j]) {
                if (j <= i) continue;
                double t[3];
                if (displacement(pos + 3 * i, pos + 3 * j, box, t) < rs2) {
                    if (np == pcap) {
                        pcap *= 2;
                        int32_t* a = (int32_t*)realloc(pi, (size_t)pcap * sizeof(int32_t));
                        if (a) pi = a;
                        int32_t* b = (int32_t*)realloc(pj, (size_t)pcap * sizeof(int32_t));
                        if (b) pj = b;
                        if (!a || !b) {
                            free(pi);
                            free(pj);
                            grid_free(&g);
                            return LJREF_E_NOMEM;
                        }
                    }
                    pi[np] = (int32_t)i;
                    pj[np] = (int32_t)j;
                    ++np;
                }
            }
        }
    }
    grid_free(&g);
    *npairs = np;
    if (np > cap || (np > 0 && col == NULL)) {
        free(pi);
        free(pj);
        return LJREF_E_CAPACITY;
    }
    /* Counting sort by i (Sec. III.C): histogram, prefix sum, scatter. */
    for (int64_t i = 0; i <= n; ++i) row_ptr[i] = 0;
    for (int64_t p = 0; p < np; ++p) row_ptr[pi[p] + 1]++;
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
    int64_t* fill = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!fill) {
        free(pi);
        free(pj);
        return LJREF_E_NOMEM;
    }
    memcpy(fill, row_ptr, (size_t)n * sizeof(int64_t));
    for (int64_t p = 0; p < np; ++p) col[fill[pi[p]]++] = pj[p];
    free(fill);
    free(pi);
    free(pj);
    /* Within a row, ascending j (insertion sort; rows are short). */
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t a = row_ptr[i] + 1; a < row_ptr[i + 1]; ++a) {
            int32_t v = col[a];
            int64_t b = a - 1;
            while (b >= row_ptr[i] && col[b] > v) {
                col[b + 1] = col[b];
                --b;
            }
            col[b + 1] = v;
        }
    }
    return LJREF_OK;
}

/* ------------------------------------------------------------------ forces */

/* Constant added to V so that the truncated potential vanishes at rc
 * (Sec. III.A): Vc = V(rc). */
static double lj_shift(double eps, double sigma, double rc) {
    double s2 = (sigma * sigma) / (rc * rc);
    double s6 = s2 * s2 * s2;
    return 4.0 * eps * s6 * (s6 - 1.0);
}

/* Magnitude of the pair force at rc, Fc = -V'(rc) = 24 eps (sigma/rc)^6
 * [2 (sigma/rc)^6 - 1] / rc: what the force-shifted truncation subtracts. */
static double lj_force_at(double eps, double sigma, double rc) {
    double s2 = (sigma * sigma) / (rc * rc);
    double s6 = s2 * s2 * s2;
    return 24.0 * eps * s6 * (2.0 * s6 - 1.0) / rc;
}

/* Parameters of the truncated potential. */
typedef struct {
    double eps, sig2, rc, rc2, vc, fc;
    int trunc;
} lj_par;

static int make_par(lj_par* p, double eps, double sigma, double rc, int trunc) {
    if (!(eps > 0.0) || !(sigma > 0.0) || !isfinite(eps) || !isfinite(sigma) || !(rc > 0.0) ||
        !isfinite(rc))
        return LJREF_E_INVALID;
    if (trunc != LJREF_TRUNC_SHIFT && trunc != LJREF_TRUNC_FORCE_SHIFT) return LJREF_E_INVALID;
    p->eps = eps;
    p->sig2 = sigma * sigma;
    p->rc = rc;
    p->rc2 = rc * rc;
    p->vc = lj_shift(eps, sigma, rc);
    p->fc = lj_force_at(eps, sigma, rc);
    p->trunc = trunc;
    return LJREF_OK;
}

/* Alg. 1 for one pair at squared distance r2 < rc^2, with sigma and eps kept
 * general: fs = -(dV/dr)/r, so that the force on j is +fs t and on i -fs t
 * (t points from i to j), and e, the pair's truncated energy.
 *   simple truncation (the paper's, Sec. III.A): V(r) - V(rc), force unchanged;
 *   force-shifted truncation (the remedy Sec. III.A recommends, in which the
 *   force also vanishes at rc): V(r) - V(rc) + (r - rc) Fc, force F(r) - Fc. */
static void pair_terms(const lj_par* p, double r2, double* fs, double* e) {
    const double sr2 = p->sig2 / r2;
    const double sr6 = sr2 * sr2 * sr2;
    double f = 24.0 * p->eps * sr6 * (2.0 * sr6 - 1.0) / r2;
    double v = 4.0 * p->eps * sr6 * (sr6 - 1.0) - p->vc;
    if (p->trunc == LJREF_TRUNC_FORCE_SHIFT) {
        const double r = sqrt(r2);
        f = f - p->fc / r;
        v = v + (r - p->rc) * p->fc;
    }
    *fs = f;
    *e = v;
}

int ljref_forces(int64_t n, const double* pos, const double* box, double eps, double sigma,
                 double rc, int trunc, const int64_t* row_ptr, const int32_t* col, double* force,
                 double* energy, double* virial, int64_t* n_in) {
    int st = check_args(n, pos, box, rc);
    if (st) return st;
    if (row_ptr == NULL || force == NULL || energy == NULL || virial == NULL || n_in == NULL)
        return LJREF_E_INVALID;
    lj_par par;
    if ((st = make_par(&par, eps, sigma, rc, trunc))) return st;
    for (int64_t k = 0; k < 3 * n; ++k) force[k] = 0.0;
    ksum E = {0.0, 0.0}, W = {0.0, 0.0};
    int64_t count = 0;
    /* Alg. 3: the i data is loaded once per row, the j data per entry, and
     * Newton's third law updates j in place; pairs listed within rs but
     * beyond rc are skipped. */
    for (int64_t i = 0; i < n; ++i) {
        const double* qi = pos + 3 * i;
        double fi[3] = {0.0, 0.0, 0.0};
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const int32_t j = col[k];
            double t[3];
            const double r2 = displacement(qi, pos + 3 * (int64_t)j, box, t);
            if (!(r2 < par.rc2)) continue;
            double fs, e;
            pair_terms(&par, r2, &fs, &e);
            /* t points from i to j: the force on j is +fs t, on i it is -fs t. */
            fi[0] -= fs * t[0];
            fi[1] -= fs * t[1];
            fi[2] -= fs * t[2];
            force[3 * (int64_t)j + 0] += fs * t[0];
            force[3 * (int64_t)j + 1] += fs * t[1];
            force[3 * (int64_t)j + 2] += fs * t[2];
            ksum_add(&E, e);
            ksum_add(&W, fs * r2);
            ++count;
        }
        force[3 * i + 0] += fi[0];
        force[3 * i + 1] += fi[1];
        force[3 * i + 2] += fi[2];
    }
    *energy = ksum_get(&E);
    *virial = ksum_get(&W);
    *n_in = count;
    return LJREF_OK;
}

/* ---------------------------------------------------------- the full list */

int ljref_full_pairs(int64_t n, const int64_t* row_ptr, const int32_t* col, int64_t* frow_ptr,
                     int32_t* fcol) {
    if (n < 1 || !row_ptr || !frow_ptr || (row_ptr[n] > 0 && (!col || !fcol)))
        return LJREF_E_INVALID;
    /* row lengths of the full list: each half-list pair (i, j) adds one entry
     * to row i and one to row j */
    for (int64_t i = 0; i <= n; ++i) frow_ptr[i] = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            frow_ptr[i + 1]++;
            frow_ptr[(int64_t)col[k] + 1]++;
        }
    for (int64_t i = 0; i < n; ++i) frow_ptr[i + 1] += frow_ptr[i];
    int64_t* fill = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!fill) return LJREF_E_NOMEM;
    memcpy(fill, frow_ptr, (size_t)n * sizeof(int64_t));
    /* in ascending i: row j receives its partners i < j in ascending order,
     * then row i its own j > i in ascending order -- every row ends sorted */
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) fcol[fill[col[k]]++] = (int32_t)i;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) fcol[fill[i]++] = col[k];
    free(fill);
    /* the two passes above interleave within a row only if a row held j < i,
     * which a half list does not; sort anyway so the order is the stated one */
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t a = frow_ptr[i] + 1; a < frow_ptr[i + 1]; ++a) {
            int32_t v = fcol[a];
            int64_t b = a - 1;
            while (b >= frow_ptr[i] && fcol[b] > v) {
                fcol[b + 1] = fcol[b];
                --b;
            }
            fcol[b + 1] = v;
        }
    }
    return LJREF_OK;
}

int ljref_forces_full(int64_t n, const double* pos, const double* box, double eps, double sigma,
                      double rc, int trunc, const int64_t* row_ptr, const int32_t* col,
                      double* force, double* energy, double* virial, int64_t* n_in) {
    int st = check_args(n, pos, box, rc);
    if (st) return st;
    if (row_ptr == NULL || force == NULL || energy == NULL || virial == NULL || n_in == NULL)
        return LJREF_E_INVALID;
    lj_par par;
    if ((st = make_par(&par, eps, sigma, rc, trunc))) return st;
    double* erow = (double*)malloc((size_t)n * sizeof(double));
    double* wrow = (double*)malloc((size_t)n * sizeof(double));
    int64_t* crow = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!erow || !wrow || !crow) {
        free(erow);
        free(wrow);
        free(crow);
        return LJREF_E_NOMEM;
    }
    /* Every row owns its force: F_i = -sum_j fs t (no scatter to j), so rows
     * are independent and the loop over them may run on any number of
     * threads with the same result.  Each row's energy and virial are its
     * own compensated sums, added afterwards in row order. */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        const double* qi = pos + 3 * i;
        double fi[3] = {0.0, 0.0, 0.0};
        ksum E = {0.0, 0.0}, W = {0.0, 0.0};
        int64_t c = 0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            double t[3];
            const double r2 = displacement(qi, pos + 3 * (int64_t)col[k], box, t);
            if (!(r2 < par.rc2)) continue;
            double fs, e;
            pair_terms(&par, r2, &fs, &e);
            fi[0] -= fs * t[0];
            fi[1] -= fs * t[1];
            fi[2] -= fs * t[2];
            ksum_add(&E, e);
            ksum_add(&W, fs * r2);
            ++c;
        }
        force[3 * i + 0] = fi[0];
        force[3 * i + 1] = fi[1];
        force[3 * i + 2] = fi[2];
        erow[i] = ksum_get(&E);
        wrow[i] = ksum_get(&W);
        crow[i] = c;
    }
    /* every pair is visited from both of its rows */
    ksum E = {0.0, 0.0}, W = {0.0, 0.0};
    int64_t count = 0;
    for (int64_t i = 0; i < n; ++i) {
        ksum_add(&E, erow[i]);
        ksum_add(&W, wrow[i]);
        count += crow[i];
    }
    *energy = 0.5 * ksum_get(&E);
    *virial = 0.5 * ksum_get(&W);
    *n_in = count / 2;
    free(erow);
    free(wrow);
    free(crow);
    return LJREF_OK;
}

int ljref_set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* ------------------------------------------------------------ per-atom sample */

int ljref_sample(int64_t n, const double* pos, const double* box, double eps, double sigma,
                 double rc, int trunc, double rs, int64_t ns, const int64_t* idx, double* f,
                 double* e, double* w, int64_t* nrs, int32_t* rows, int64_t rowcap) {
    int st = check_args(n, pos, box, rs);
    if (st) return st;
    if (!(rc > 0.0) || rc > rs || ns < 0 || (ns > 0 && (!idx || !f || !e || !w || !nrs)))
        return LJREF_E_INVALID;
    lj_par par;
    if ((st = make_par(&par, eps, sigma, rc, trunc))) return st;
    for (int64_t s = 0; s < ns; ++s)
        if (idx[s] < 0 || idx[s] >= n) return LJREF_E_INVALID;
    cell_grid g;
    st = grid_build(&g, n, pos, box, rs);
    if (st) return st;
    const double rs2 = rs * rs;
    /* Each sampled atom is found and summed on its own (the grid is only
     * read), so the loop may run on any number of threads with the same result. */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < ns; ++s) {
        const int64_t i = idx[s];
        const double* qi = pos + 3 * i;
        double fi[3] = {0.0, 0.0, 0.0};
        ksum E = {0.0, 0.0}, W = {0.0, 0.0};
        int64_t m = 0;
        int32_t* row = rows ? rows + s * rowcap : NULL;
        int64_t cells[27];
        int nc = grid_stencil(&g, qi, cells);
        for (int k = 0; k < nc; ++k) {
            for (int64_t j = g.head[cells[k]]; j >= 0; j = g.next[j]) {
                if (j == i) continue;
                double t[3];
                const double r2 = displacement(qi, pos + 3 * j, box, t);
                if (r2 < rs2) {
                    if (row && m < rowcap) row[m] = (int32_t)j;
                    ++m;
                }
                if (!(r2 < par.rc2)) continue;
                double fs, ep;
                pair_terms(&par, r2, &fs, &ep);
                fi[0] -= fs * t[0];
                fi[1] -= fs * t[1];
                fi[2] -= fs * t[2];
                ksum_add(&E, ep);
                ksum_add(&W, fs * r2);
            }
        }
        if (row) { /* ascending j */
            int64_t len = m < rowcap ? m : rowcap;
            for (int64_t a = 1; a < len; ++a) {
                int32_t v = row[a];
                int64_t b = a - 1;
                while (b >= 0 && row[b] > v) {
                    row[b + 1] = row[b];
                    --b;
                }
                row[b + 1] = v;
            }
        }
        f[3 * s + 0] = fi[0];
        f[3 * s + 1] = fi[1];
        f[3 * s + 2] = fi[2];
        e[s] = 0.5 * ksum_get(&E);
        w[s] = 0.5 * ksum_get(&W);
        nrs[s] = m;
    }
    grid_free(&g);
    return LJREF_OK;
}

/* --------------------------------------------------------------------- NVE */

static int build_list(int64_t n, const double* pos, const double* box, double rs,
                      int64_t* row_ptr, int32_t** col, int64_t* cap) {
    int64_t np = 0;
    int st = ljref_cell_pairs(n, pos, box, rs, *cap, row_ptr, *col, &np);
    if (st == LJREF_E_CAPACITY) {
        free(*col);
        *cap = np + np / 8 + 16;
        *col = (int32_t*)malloc((size_t)(*cap) * sizeof(int32_t));
        if (!*col) return LJREF_E_NOMEM;
        st = ljref_cell_pairs(n, pos, box, rs, *cap, row_ptr, *col, &np);
    }
    return st;
}

int ljref_nve(int64_t n, double* pos, double* vel, const double* box, double eps, double sigma,
              double rc, int trunc, double skin, double dt, int32_t nsteps,
              int32_t rebuild_every, double* log, double* force) {
    const double rs = rc + skin;
    int st = check_args(n, pos, box, rs);
    if (st) return st;
    if (!vel || !log || !force || nsteps < 0 || rebuild_every < 0 || !(skin >= 0.0) ||
        !isfinite(dt))
        return LJREF_E_INVALID;
    /* Sec. III.B: the list stays valid while no pair has closed in by more
     * than the margin rs - rc = skin, which holds while every atom has moved
     * less than skin/2 since the build.  The displacement-triggered mode
     * rebuilds at the first step whose largest displacement exceeds that. */
    const double half_skin2 = (0.5 * skin) * (0.5 * skin);
    int64_t* row_ptr = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    double* disp = (double*)calloc((size_t)(3 * n), sizeof(double));
    int64_t cap = 64 * n + 1024;
    int32_t* col = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    if (!row_ptr || !disp || !col) {
        free(row_ptr);
        free(disp);
        free(col);
        return LJREF_E_NOMEM;
    }
    st = build_list(n, pos, box, rs, row_ptr, &col, &cap);
    double pe = 0.0, vir = 0.0;
    int64_t nin = 0;
    if (!st)
        st = ljref_forces(n, pos, box, eps, sigma, rc, trunc, row_ptr, col, force, &pe, &vir,
                          &nin);
    for (int32_t step = 0; !st && step <= nsteps; ++step) {
        int rebuilt = step == 0;
        if (step > 0) {
            for (int64_t k = 0; k < 3 * n; ++k) vel[k] += 0.5 * dt * force[k];
            double dmax = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                for (int d = 0; d < 3; ++d) {
                    const double dx = dt * vel[3 * i + d];
                    double x = pos[3 * i + d] + dx;
                    disp[3 * i + d] += dx;
                    x = x - box[d] * floor(x / box[d]);
                    if (x >= box[d]) x = 0.0;
                    pos[3 * i + d] = x;
                }
                const double* u = disp + 3 * i;
                const double d2 = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
                if (d2 > dmax) dmax = d2;
            }
            rebuilt = rebuild_every > 0 ? step % rebuild_every == 0 : dmax > half_skin2;
            if (rebuilt) {
                st = build_list(n, pos, box, rs, row_ptr, &col, &cap);
                if (st) break;
                for (int64_t k = 0; k < 3 * n; ++k) disp[k] = 0.0;
            }
            st = ljref_forces(n, pos, box, eps, sigma, rc, trunc, row_ptr, col, force, &pe, &vir,
                              &nin);
            if (st) break;
            for (int64_t k = 0; k < 3 * n; ++k) vel[k] += 0.5 * dt * force[k];
        }
        ksum K = {0.0, 0.0};
        double dmax = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const double* v = vel + 3 * i;
            ksum_add(&K, 0.5 * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]));
            const double* u = disp + 3 * i;
            const double d2 = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
            if (d2 > dmax) dmax = d2;
        }
        log[6 * step + 0] = pe;
        log[6 * step + 1] = ksum_get(&K);
        log[6 * step + 2] = vir;
        log[6 * step + 3] = sqrt(dmax);
        log[6 * step + 4] = (double)nin;
        log[6 * step + 5] = (double)rebuilt;
    }
    free(row_ptr);
    free(disp);
    free(col);
    return st;
}
