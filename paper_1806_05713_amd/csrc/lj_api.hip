// lj_api.hip -- the C ABI of include/lj.h: argument checks, ownership of
// device buffers, capacity management, and the launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "lj_internal.h"

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

lj_status lj_fail(lj_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

lj_status lj_hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? LJ_E_NOMEM : LJ_E_HIP;
}

extern "C" const char* lj_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------- profiler

static const size_t kMaxProf = 65536;

lj_prof_scope::lj_prof_scope(lj_ctx* c, int phase) : ctx(c), idx(-1) {
    if (!ctx || !ctx->prof_on || ctx->prof.size() >= kMaxProf) return;
    lj_prof_rec r;
    r.phase = phase;
    if (hipEventCreate(&r.a) != hipSuccess) return;
    if (hipEventCreate(&r.b) != hipSuccess) {
        (void)hipEventDestroy(r.a);
        return;
    }
    if (hipEventRecord(r.a, ctx->stream) != hipSuccess) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
        return;
    }
    ctx->prof.push_back(r);
    idx = (int)ctx->prof.size() - 1;
}

lj_prof_scope::~lj_prof_scope() {
    if (idx >= 0) (void)hipEventRecord(ctx->prof[idx].b, ctx->stream);
}

static void prof_clear(lj_ctx* ctx) {
    for (auto& r : ctx->prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    ctx->prof.clear();
}

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

template <typename T>
lj_status dmalloc(T** p, int64_t count) {
    *p = nullptr;
    if (count <= 0) count = 1;
    hipError_t e = hipMalloc((void**)p, (size_t)count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return lj_hip_fail(e, "hipMalloc");
    }
    return LJ_OK;
}

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

lj_status check_box(const double* box, double rs) {
    if (!box) return lj_fail(LJ_E_INVALID, "box is NULL");
    for (int d = 0; d < 3; ++d) {
        if (!finite_pos(box[d])) return lj_fail(LJ_E_INVALID, "box lengths must be finite and > 0");
        if (box[d] < 2.0 * rs) {
            char buf[160];
            snprintf(buf, sizeof buf, "box[%d] = %.17g is shorter than 2 (rc + skin) = %.17g", d,
                     box[d], 2.0 * rs);
            return lj_fail(LJ_E_BOX, buf);
        }
    }
    return LJ_OK;
}

lj_status check_common(lj_ctx* ctx, const double* pos, int64_t n, int32_t layout) {
    if (!ctx) return lj_fail(LJ_E_INVALID, "context is NULL");
    if (!pos) return lj_fail(LJ_E_INVALID, "positions are NULL");
    if (n < 1) return lj_fail(LJ_E_INVALID, "n must be >= 1");
    if (n > (int64_t)INT32_MAX / 2) return lj_fail(LJ_E_INVALID, "n exceeds the 32-bit index range");
    if (layout != LJ_AOS4 && layout != LJ_SOA) return lj_fail(LJ_E_INVALID, "unknown layout");
    if (layout == LJ_AOS4 && ((uintptr_t)pos & 31u))
        return lj_fail(LJ_E_INVALID, "LJ_AOS4 positions must be 32-byte aligned");
    return LJ_OK;
}

// Largest cell count per dimension whose cell side is >= min_cell, with a
// relative margin of 1e-12 so that a coordinate rounded onto a cell face
// cannot put a pair closer than min_cell two cells apart.
int cells_for(double L, double min_cell) {
    double q = floor(L / min_cell);
    int nc = q > 1e6 ? 1000000 : (int)q;
    while (nc > 1 && L / nc < min_cell * (1.0 + 1e-12)) --nc;
    return nc < 1 ? 1 : nc;
}

lj_status read_status(lj_ctx* ctx, lj_dev_status* h) {
    LJ_HIP(hipMemcpyAsync(h, ctx->st, sizeof(*h), hipMemcpyDeviceToHost, ctx->stream));
    LJ_HIP(hipStreamSynchronize(ctx->stream));
    return LJ_OK;
}

lj_status reset_status(lj_ctx* ctx) {
    // flags only; the reduction arrival counter keeps its own state
    return lj_launch_zero(ctx->stream, ctx->st, offsetof(lj_dev_status, done_blocks));
}

void cells_release(lj_cells* c) {
    if (!c) return;
    dfree(c->count);
    dfree(c->cell_start);
    dfree(c->cid);
    dfree(c->order_tmp);
    dfree(c->order);
    dfree(c->spos);
    dfree(c->block_sums);
    delete c;
}

void list_release(lj_list* l) {
    if (!l) return;
    dfree(l->row_atom);
    dfree(l->row_len);
    dfree(l->slice_iters);
    dfree(l->slice_stats);
    dfree(l->col);
    dfree(l->stats);
    cells_release(l->cells);
    delete l;
}

lj_status alloc_cells(int64_t n, const double* box, double min_cell, lj_cells** out) {
    lj_cells* c = new (std::nothrow) lj_cells();
    if (!c) return lj_fail(LJ_E_NOMEM, "host allocation");
    c->n = n;
    c->ncell = 1;
    c->counts_dirty = true;   // fresh allocation: cleared by the first build
    for (int d = 0; d < 3; ++d) {
        c->box[d] = box[d];
        c->nc[d] = cells_for(box[d], min_cell);
        c->cs[d] = box[d] / c->nc[d];
        c->ncell *= c->nc[d];
    }
    if (c->ncell > (int64_t)16 * 1024 * 1024) {
        delete c;
        return lj_fail(LJ_E_CAPACITY, "more than 16.7M cells: raise min_cell");
    }
    lj_status st;
    if ((st = dmalloc(&c->count, c->ncell)) || (st = dmalloc(&c->cell_start, c->ncell + 1)) ||
        (st = dmalloc(&c->cid, n)) || (st = dmalloc(&c->order_tmp, n)) ||
        (st = dmalloc(&c->order, n)) || (st = dmalloc(&c->spos, n)) ||
        (st = dmalloc(&c->block_sums, lj_scan_workspace(c->ncell)))) {
        cells_release(c);
        return st;
    }
    *out = c;
    return LJ_OK;
}

// Bin and sort, then wait and report a bad coordinate.
lj_status fill_cells_sync(lj_ctx* ctx, const double* pos, int32_t layout, lj_cells* c) {
    lj_status st;
    if ((st = reset_status(ctx)) || (st = lj_launch_cells(ctx, pos, layout, c))) return st;
    lj_dev_status h;
    if ((st = read_status(ctx, &h))) return st;
    if (h.flags & LJ_DEV_BAD_POSITION)
        return lj_fail(LJ_E_POSITION, "a coordinate is non-finite or outside [0, box)");
    return LJ_OK;
}

lj_status read_stats(const lj_list* l, hipStream_t s, lj_list_stats* h) {
    LJ_HIP(hipMemcpyAsync(h, l->stats, sizeof(*h), hipMemcpyDeviceToHost, s));
    LJ_HIP(hipStreamSynchronize(s));
    return LJ_OK;
}

int default_lanes(int kind) { return kind == LJ_LIST_FULL ? 8 : 8; }

// Side of the cells the library bins into for its own list builds: the search
// length over k (default k = 2: each row then visits about 2.7x fewer
// candidates than with a 27-cell stencil of side rs), with a small relative
// margin so that rounding cannot push the reach of rs + delta to one more cell.
double internal_min_cell(const lj_ctx* ctx, double rs) {
    int k = ctx->tune[LJ_TUNE_CELL_DIV];
    if (k < 1 || k > 4) k = 2;
    return rs / k * (1.0 + 1e-11);
}

}  // namespace

// ----------------------------------------------------------------- context

extern "C" lj_status lj_create(int device, void* stream, lj_ctx** out) {
    if (!out) return lj_fail(LJ_E_INVALID, "out is NULL");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
        return lj_fail(LJ_E_NODEVICE, "no HIP device");
    if (device < 0 || device >= count) return lj_fail(LJ_E_NODEVICE, "device index out of range");
    hipDeviceProp_t prop;
    LJ_HIP(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return lj_fail(LJ_E_NODEVICE, std::string("device is ") + prop.gcnArchName +
                                          ", this library is built for gfx950");
    DeviceGuard guard(device);
    lj_ctx* ctx = new (std::nothrow) lj_ctx();
    if (!ctx) return lj_fail(LJ_E_NOMEM, "host allocation");
    ctx->device = device;
    ctx->stream = (hipStream_t)stream;
    ctx->prof_on = false;
    for (int k = 0; k < LJ_TUNE_N; ++k) ctx->tune[k] = 0;
    lj_status st = dmalloc(&ctx->st, 1);
    if (st) {
        delete ctx;
        return st;
    }
    ctx->partials_cap = 4096;
    if ((st = dmalloc(&ctx->partials, 4 * ctx->partials_cap))) {
        dfree(ctx->st);
        delete ctx;
        return st;
    }
    hipError_t e = hipMemsetAsync(ctx->st, 0, sizeof(lj_dev_status), ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        dfree(ctx->st);
        dfree(ctx->partials);
        delete ctx;
        return lj_hip_fail(e, "context init");
    }
    *out = ctx;
    return LJ_OK;
}

extern "C" lj_status lj_destroy(lj_ctx* ctx) {
    if (!ctx) return LJ_OK;
    DeviceGuard guard(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    prof_clear(ctx);
    dfree(ctx->st);
    dfree(ctx->partials);
    delete ctx;
    return LJ_OK;
}

extern "C" lj_status lj_set_stream(lj_ctx* ctx, void* stream) {
    if (!ctx) return lj_fail(LJ_E_INVALID, "context is NULL");
    ctx->stream = (hipStream_t)stream;
    return LJ_OK;
}

extern "C" lj_status lj_sync(lj_ctx* ctx) {
    if (!ctx) return lj_fail(LJ_E_INVALID, "context is NULL");
    DeviceGuard guard(ctx->device);
    lj_dev_status h;
    lj_status st = read_status(ctx, &h);
    if (st) return st;
    if (h.flags) {   // report once: clear the flags
        if ((st = reset_status(ctx))) return st;
        LJ_HIP(hipStreamSynchronize(ctx->stream));
    }
    if (h.flags & LJ_DEV_BAD_POSITION)
        return lj_fail(LJ_E_POSITION, "a coordinate is non-finite or outside [0, box)");
    if (h.flags & (LJ_DEV_ROW_OVERFLOW | LJ_DEV_CELL_OVERFLOW))
        return lj_fail(LJ_E_CAPACITY, "a list row exceeded its capacity");
    return LJ_OK;
}

// ------------------------------------------------------------------- cells

extern "C" lj_status lj_build_cells(lj_ctx* ctx, const double* pos, int64_t n, int32_t layout,
                                    const double box[3], double min_cell, lj_cells** cells) {
    lj_status st = check_common(ctx, pos, n, layout);
    if (st) return st;
    if (!cells) return lj_fail(LJ_E_INVALID, "cells is NULL");
    if (!finite_pos(min_cell)) return lj_fail(LJ_E_INVALID, "min_cell must be finite and > 0");
    if (!box) return lj_fail(LJ_E_INVALID, "box is NULL");
    for (int d = 0; d < 3; ++d)
        if (!finite_pos(box[d])) return lj_fail(LJ_E_INVALID, "box lengths must be finite and > 0");
    DeviceGuard guard(ctx->device);
    lj_cells* c = nullptr;
    if ((st = alloc_cells(n, box, min_cell, &c))) return st;
    if ((st = fill_cells_sync(ctx, pos, layout, c))) {
        cells_release(c);
        return st;
    }
    *cells = c;
    return LJ_OK;
}

extern "C" lj_status lj_cells_info(const lj_cells* c, int32_t nc[3], int64_t* n) {
    if (!c) return lj_fail(LJ_E_INVALID, "cells is NULL");
    if (nc)
        for (int d = 0; d < 3; ++d) nc[d] = c->nc[d];
    if (n) *n = c->n;
    return LJ_OK;
}

extern "C" lj_status lj_cells_export(lj_ctx* ctx, const lj_cells* c, int32_t* cell_start,
                                     int32_t* order) {
    if (!ctx || !c) return lj_fail(LJ_E_INVALID, "context or cells is NULL");
    DeviceGuard guard(ctx->device);
    if (cell_start)
        LJ_HIP(hipMemcpyAsync(cell_start, c->cell_start, (size_t)(c->ncell + 1) * sizeof(int32_t),
                              hipMemcpyDeviceToHost, ctx->stream));
    if (order)
        LJ_HIP(hipMemcpyAsync(order, c->order, (size_t)c->n * sizeof(int32_t),
                              hipMemcpyDeviceToHost, ctx->stream));
    LJ_HIP(hipStreamSynchronize(ctx->stream));
    return LJ_OK;
}

extern "C" lj_status lj_cells_free(lj_cells* c) {
    cells_release(c);
    return LJ_OK;
}

// -------------------------------------------------------------------- list

extern "C" lj_status lj_build_neighbors(lj_ctx* ctx, const double* pos, int64_t n,
                                        int32_t layout, const double box[3], double rc,
                                        double skin, int32_t kind, int32_t lanes,
                                        const lj_cells* cells, lj_list** list) {
    lj_status st = check_common(ctx, pos, n, layout);
    if (st) return st;
    if (!list) return lj_fail(LJ_E_INVALID, "list is NULL");
    if (!finite_pos(rc)) return lj_fail(LJ_E_INVALID, "rc must be finite and > 0");
    if (!(skin >= 0.0) || !isfinite(skin)) return lj_fail(LJ_E_INVALID, "skin must be finite and >= 0");
    if (kind != LJ_LIST_HALF && kind != LJ_LIST_FULL) return lj_fail(LJ_E_INVALID, "unknown list kind");
    if (lanes == 0) lanes = default_lanes(kind);
    if (lanes < 1 || lanes > 64 || (lanes & (lanes - 1)))
        return lj_fail(LJ_E_INVALID, "lanes must be 1, 2, 4, 8, 16, 32 or 64");
    const double rs = rc + skin;
    if ((st = check_box(box, rs))) return st;
    DeviceGuard guard(ctx->device);

    if (cells) {
        if (cells->n != n) return lj_fail(LJ_E_STALE, "cells were built for another atom count");
        for (int d = 0; d < 3; ++d) {
            if (cells->box[d] != box[d]) return lj_fail(LJ_E_STALE, "cells were built for another box");
            if (cells->nc[d] > 1 && cells->cs[d] * 16.0 < rs)
                return lj_fail(LJ_E_INVALID, "cells are smaller than (rc + skin) / 16");
        }
    }
    lj_list* l = new (std::nothrow) lj_list();
    if (!l) return lj_fail(LJ_E_NOMEM, "host allocation");
    l->n = n;
    l->kind = kind;
    l->lanes = lanes;
    l->rc = rc;
    l->skin = skin;
    for (int d = 0; d < 3; ++d) l->box[d] = box[d];
    const lj_cells* c = cells;
    if (!c) {
        if ((st = alloc_cells(n, box, internal_min_cell(ctx, rs), &l->cells)) ||
            (st = fill_cells_sync(ctx, pos, layout, l->cells))) {
            list_release(l);
            return st;
        }
        c = l->cells;
    }
    for (int d = 0; d < 3; ++d) l->nc[d] = c->nc[d];
    const int C = LJ_WAVE / lanes;
    // whole wavefronts of the build (up to 16 slices each, when it uses fewer
    // lanes per row than the layout); trailing slices stay empty
    l->nslices = ((n + C - 1) / C + 15) / 16 * 16;
    // First guess of the row capacity: 1.25 x the neighbors within rs of an
    // atom at the mean density, plus a margin; grown on overflow.
    const double vol = box[0] * box[1] * box[2];
    double expect = 4.18879020478639 * rs * rs * rs * (double)n / vol;   // (4/3) pi rs^3 rho
    if (kind == LJ_LIST_HALF) expect *= 0.5;
    int64_t cap = (int64_t)(1.25 * expect + 32.0);
    if (cap > n) cap = n;
    const int64_t slice_rows = l->nslices * C;
    if ((st = dmalloc(&l->row_atom, slice_rows)) || (st = dmalloc(&l->row_len, slice_rows)) ||
        (st = dmalloc(&l->slice_iters, l->nslices)) ||
        (st = dmalloc(&l->slice_stats, 2 * l->nslices)) || (st = dmalloc(&l->stats, 1))) {
        list_release(l);
        return st;
    }
    for (int attempt = 0; attempt < 3; ++attempt) {
        cap = ((cap + lanes - 1) / lanes) * lanes;
        if (cap < lanes) cap = lanes;
        if (l->nslices * cap * C > ((int64_t)1 << 40)) {
            st = lj_fail(LJ_E_CAPACITY, "list would exceed 2^40 slots");
            break;
        }
        l->cap = (int)cap;
        dfree(l->col);
        l->col = nullptr;
        if ((st = dmalloc(&l->col, l->nslices * (cap / lanes) * LJ_WAVE))) break;
        lj_list_stats h;
        if ((st = lj_launch_neighbors(ctx, c, l, rs)) || (st = read_stats(l, ctx->stream, &h)))
            break;
        l->max_row = h.max_row;
        l->entries = (int64_t)h.entries;
        if (h.max_row <= cap) {
            st = LJ_OK;
            break;
        }
        cap = (int64_t)h.max_row + h.max_row / 16 + lanes;
        st = lj_fail(LJ_E_CAPACITY, "row capacity still too small after regrowth");
    }
    if (st) {
        list_release(l);
        return st;
    }
    // the force kernel's block partials must fit in the context
    const int64_t blocks = lj_force_blocks(l->nslices);
    if (blocks > ctx->partials_cap) {
        double* p = nullptr;
        if ((st = dmalloc(&p, 4 * blocks))) {
            list_release(l);
            return st;
        }
        (void)hipStreamSynchronize(ctx->stream);
        dfree(ctx->partials);
        ctx->partials = p;
        ctx->partials_cap = blocks;
    }
    *list = l;
    return LJ_OK;
}

lj_status lj_list_ensure_cells(lj_ctx* ctx, lj_list* l) {
    if (l->cells) return LJ_OK;
    return alloc_cells(l->n, l->box, internal_min_cell(ctx, l->rc + l->skin), &l->cells);
}

extern "C" lj_status lj_update_neighbors(lj_ctx* ctx, const double* pos, int64_t n,
                                         int32_t layout, const double box[3], lj_list* l) {
    lj_status st = check_common(ctx, pos, n, layout);
    if (st) return st;
    if (!l) return lj_fail(LJ_E_INVALID, "list is NULL");
    if (!box) return lj_fail(LJ_E_INVALID, "box is NULL");
    if (l->n != n) return lj_fail(LJ_E_STALE, "list was built for another atom count");
    for (int d = 0; d < 3; ++d)
        if (l->box[d] != box[d]) return lj_fail(LJ_E_STALE, "list was built for another box");
    DeviceGuard guard(ctx->device);
    if ((st = lj_list_ensure_cells(ctx, l))) return st;   // lists built on caller cells
    if ((st = lj_launch_cells(ctx, pos, layout, l->cells))) return st;
    return lj_launch_neighbors(ctx, l->cells, l, l->rc + l->skin);
}

extern "C" lj_status lj_list_info(const lj_list* l, lj_list_desc* out) {
    if (!l || !out) return lj_fail(LJ_E_INVALID, "list or out is NULL");
    lj_list_stats h;
    // the list may have been rebuilt on any stream of its context: wait for the device
    LJ_HIP(hipDeviceSynchronize());
    LJ_HIP(hipMemcpy(&h, l->stats, sizeof(h), hipMemcpyDeviceToHost));
    out->n = l->n;
    out->kind = l->kind;
    out->lanes = l->lanes;
    out->cap = l->cap;
    out->max_row = h.max_row;
    out->entries = (int64_t)h.entries;
    out->slots = l->nslices * (int64_t)(l->cap / l->lanes) * LJ_WAVE;
    out->rc = l->rc;
    out->skin = l->skin;
    for (int d = 0; d < 3; ++d) {
        out->box[d] = l->box[d];
        out->nc[d] = l->nc[d];
    }
    return LJ_OK;
}

extern "C" lj_status lj_list_pairs(lj_ctx* ctx, const lj_list* l, int64_t cap, int32_t* ij,
                                   int64_t* npairs) {
    if (!ctx || !l || !npairs) return lj_fail(LJ_E_INVALID, "context, list or npairs is NULL");
    DeviceGuard guard(ctx->device);
    const int G = l->lanes, C = LJ_WAVE / G, S = l->cap / G;
    const int64_t rows = l->nslices * C;
    const int64_t slots = l->nslices * (int64_t)S * LJ_WAVE;
    int32_t* ra = (int32_t*)malloc((size_t)rows * sizeof(int32_t));
    int32_t* rl = (int32_t*)malloc((size_t)rows * sizeof(int32_t));
    int32_t* col = (int32_t*)malloc((size_t)slots * sizeof(int32_t));
    lj_status st = LJ_OK;
    if (!ra || !rl || !col) {
        st = lj_fail(LJ_E_NOMEM, "host allocation");
    } else {
        hipError_t e = hipMemcpyAsync(ra, l->row_atom, rows * sizeof(int32_t),
                                      hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(rl, l->row_len, rows * sizeof(int32_t), hipMemcpyDeviceToHost,
                               ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(col, l->col, slots * sizeof(int32_t), hipMemcpyDeviceToHost,
                               ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            st = lj_hip_fail(e, "list copy");
        } else {
            int64_t total = 0;
            for (int64_t r = 0; r < l->n; ++r) total += rl[r];
            *npairs = total;
            if (cap < total || (!ij && total > 0)) {
                st = lj_fail(LJ_E_CAPACITY, "ij is too small for the list");
            } else {
                int64_t k = 0;
                for (int64_t r = 0; r < l->n; ++r) {
                    const int64_t s = r / C, c = r % C;
                    for (int e2 = 0; e2 < rl[r]; ++e2) {
                        const int64_t at = (s * S + e2 / G) * LJ_WAVE + c * G + (e2 % G);
                        ij[2 * k] = ra[r];
                        ij[2 * k + 1] = col[at];
                        ++k;
                    }
                }
            }
        }
    }
    free(ra);
    free(rl);
    free(col);
    return st;
}

extern "C" lj_status lj_list_device_view(const lj_list* l, lj_list_view* out) {
    if (!l || !out) return lj_fail(LJ_E_INVALID, "list or out is NULL");
    out->col = l->col;
    out->row_atom = l->row_atom;
    out->row_len = l->row_len;
    out->slice_iters = l->slice_iters;
    out->nslices = l->nslices;
    out->lanes = l->lanes;
    out->cap = l->cap;
    return LJ_OK;
}

extern "C" lj_status lj_list_free(lj_list* l) {
    list_release(l);
    return LJ_OK;
}

// -------------------------------------------------------------- integrator

extern "C" lj_status lj_nve_create(lj_ctx* ctx, double* pos, double* vel, double* force,
                                   int64_t n, int32_t layout, const double box[3], double eps,
                                   double sigma, double rc, int32_t precision, lj_list* list,
                                   double dt, int32_t rebuild_every, double* log,
                                   int64_t log_rows, lj_nve** out) {
    lj_status st = check_common(ctx, pos, n, layout);
    if (st) return st;
    if (!vel || !force || !list || !out || !box)
        return lj_fail(LJ_E_INVALID, "vel, force, list, box or out is NULL");
    if (layout == LJ_AOS4 && (((uintptr_t)vel & 31u) || ((uintptr_t)force & 31u)))
        return lj_fail(LJ_E_INVALID, "LJ_AOS4 arrays must be 32-byte aligned");
    if (!finite_pos(eps) || !finite_pos(sigma) || !finite_pos(rc) || !finite_pos(dt))
        return lj_fail(LJ_E_INVALID, "eps, sigma, rc and dt must be finite and > 0");
    if (precision != LJ_FP64 && precision != LJ_MIXED)
        return lj_fail(LJ_E_INVALID, "unknown precision");
    if (rebuild_every < 1) return lj_fail(LJ_E_INVALID, "rebuild_every must be >= 1");
    if (log_rows < 0 || (log_rows > 0 && !log)) return lj_fail(LJ_E_INVALID, "log is NULL");
    if (list->n != n) return lj_fail(LJ_E_STALE, "list was built for another atom count");
    for (int d = 0; d < 3; ++d)
        if (list->box[d] != box[d]) return lj_fail(LJ_E_STALE, "list was built for another box");
    if (rc > list->rc) return lj_fail(LJ_E_STALE, "rc is larger than the list's cutoff");
    DeviceGuard guard(ctx->device);
    if ((st = lj_list_ensure_cells(ctx, list))) return st;
    return lj_nve_make(ctx, pos, vel, force, n, layout, box, eps, sigma, rc, precision, list, dt,
                       rebuild_every, log, log_rows, out);
}

extern "C" lj_status lj_nve_init(lj_nve* nve) {
    if (!nve) return lj_fail(LJ_E_INVALID, "integrator is NULL");
    return lj_nve_start(nve);
}

extern "C" lj_status lj_nve_run(lj_nve* nve, int32_t nsteps, int32_t use_graph) {
    if (!nve) return lj_fail(LJ_E_INVALID, "integrator is NULL");
    if (nsteps < 0) return lj_fail(LJ_E_INVALID, "nsteps must be >= 0");
    return lj_nve_advance(nve, nsteps, use_graph);
}

extern "C" lj_status lj_nve_steps(const lj_nve* nve, int64_t* steps) {
    if (!nve || !steps) return lj_fail(LJ_E_INVALID, "integrator or steps is NULL");
    *steps = lj_nve_step_count(nve);
    return LJ_OK;
}

extern "C" lj_status lj_nve_free(lj_nve* nve) {
    lj_nve_release(nve);
    return LJ_OK;
}

// ------------------------------------------------------------------ tuning

extern "C" lj_status lj_tune_set(lj_ctx* ctx, int32_t knob, int32_t value) {
    if (!ctx) return lj_fail(LJ_E_INVALID, "context is NULL");
    bool ok = false;
    switch (knob) {
        case LJ_TUNE_BUILD_LANES: ok = value == 0 || value == 1 || value == 2 || value == 4; break;
        case LJ_TUNE_FORCE_BATCH: ok = value == 0 || value == 2 || value == 4 || value == 8; break;
        case LJ_TUNE_CELL_DIV: ok = value >= 0 && value <= 4; break;
        default: return lj_fail(LJ_E_INVALID, "unknown tuning knob");
    }
    if (!ok) return lj_fail(LJ_E_INVALID, "value not allowed for this knob");
    ctx->tune[knob] = value;
    return LJ_OK;
}

extern "C" lj_status lj_tune_get(const lj_ctx* ctx, int32_t knob, int32_t* value) {
    if (!ctx || !value) return lj_fail(LJ_E_INVALID, "context or value is NULL");
    if (knob < 0 || knob >= LJ_TUNE_N) return lj_fail(LJ_E_INVALID, "unknown tuning knob");
    *value = ctx->tune[knob];
    return LJ_OK;
}

// --------------------------------------------------------------- profiling

extern "C" lj_status lj_profile_begin(lj_ctx* ctx) {
    if (!ctx) return lj_fail(LJ_E_INVALID, "context is NULL");
    DeviceGuard guard(ctx->device);
    prof_clear(ctx);
    ctx->prof_on = true;
    return LJ_OK;
}

extern "C" lj_status lj_profile_end(lj_ctx* ctx, double* ms, int64_t* launches) {
    if (!ctx || !ms || !launches) return lj_fail(LJ_E_INVALID, "context, ms or launches is NULL");
    DeviceGuard guard(ctx->device);
    ctx->prof_on = false;
    for (int k = 0; k < LJ_PROF_N; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        prof_clear(ctx);
        return lj_hip_fail(e, "profile sync");
    }
    for (auto& r : ctx->prof) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess && r.phase >= 0 && r.phase < LJ_PROF_N) {
            ms[r.phase] += t;
            launches[r.phase] += 1;
        }
    }
    prof_clear(ctx);
    return LJ_OK;
}

// ------------------------------------------------------------------ forces

extern "C" lj_status lj_forces(lj_ctx* ctx, const double* pos, int64_t n, int32_t layout,
                               const double box[3], double eps, double sigma, double rc,
                               const lj_list* list, int32_t precision, double* force,
                               double* energy, double* virial, int64_t* npairs) {
    lj_status st = check_common(ctx, pos, n, layout);
    if (st) return st;
    if (!list || !force || !energy || !virial)
        return lj_fail(LJ_E_INVALID, "list, force, energy or virial is NULL");
    if (layout == LJ_AOS4 && ((uintptr_t)force & 31u))
        return lj_fail(LJ_E_INVALID, "LJ_AOS4 forces must be 32-byte aligned");
    if (!finite_pos(eps) || !finite_pos(sigma) || !finite_pos(rc))
        return lj_fail(LJ_E_INVALID, "eps, sigma and rc must be finite and > 0");
    if (precision != LJ_FP64 && precision != LJ_MIXED)
        return lj_fail(LJ_E_INVALID, "unknown precision");
    if (!box) return lj_fail(LJ_E_INVALID, "box is NULL");
    if (list->n != n) return lj_fail(LJ_E_STALE, "list was built for another atom count");
    for (int d = 0; d < 3; ++d)
        if (list->box[d] != box[d]) return lj_fail(LJ_E_STALE, "list was built for another box");
    if (rc > list->rc) return lj_fail(LJ_E_STALE, "rc is larger than the list's cutoff");
    DeviceGuard guard(ctx->device);
    lj_force_params p;
    for (int d = 0; d < 3; ++d) p.box[d] = box[d];
    p.eps = eps;
    p.sigma = sigma;
    p.rc = rc;
    p.layout = layout;
    p.precision = precision;
    return lj_launch_forces(ctx, pos, list, p, force, energy, virial, npairs);
}
