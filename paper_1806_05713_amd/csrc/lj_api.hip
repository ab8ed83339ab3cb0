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
    if (n > LJ_MAX_ATOMS)
        return lj_fail(LJ_E_INVALID, "n exceeds LJ_MAX_ATOMS (2^27 atoms per call)");
    if (layout != LJ_AOS4 && layout != LJ_SOA && layout != LJ_AOS8)
        return lj_fail(LJ_E_INVALID, "unknown layout");
    if (layout != LJ_SOA && ((uintptr_t)pos & 31u))
        return lj_fail(LJ_E_INVALID, "AoS positions must be 32-byte aligned");
    if (layout == LJ_AOS8 && n > LJ_MAX_ATOMS / 2)
        return lj_fail(LJ_E_INVALID, "LJ_AOS8 holds at most 2^26 atoms per call");
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
    return lj_launch_zero(ctx->stream, ctx->st, sizeof(lj_dev_status));
}

void cells_release(lj_cells* c) {
    if (!c) return;
    dfree(c->dsys);
    dfree(c->atom_sys);
    dfree(c->count);
    dfree(c->cell_start);
    dfree(c->cid);
    dfree(c->slot);
    dfree(c->order_tmp);
    dfree(c->order);
    dfree(c->spos);
    dfree(c->spos32);
    dfree(c->block_sums);
    delete c;
}

void list_release(lj_list* l) {
    if (!l) return;
    dfree(l->dsys);
    dfree(l->slice_sys);
    dfree(l->row_atom);
    dfree(l->row_len);
    dfree(l->slice_iters);
    dfree(l->slice_stats);
    dfree(l->acc);
    dfree(l->hwin);
    dfree(l->q32);
    dfree(l->xy);
    dfree(l->zz);
    dfree(l->col);
    dfree(l->stats);
    dfree(l->fc);
    cells_release(l->cells);
    delete l;
}

template <typename T>
lj_status upload(T* dst, const T* src, int64_t count, hipStream_t s) {
    LJ_HIP(hipMemcpyAsync(dst, src, (size_t)count * sizeof(T), hipMemcpyHostToDevice, s));
    LJ_HIP(hipStreamSynchronize(s));
    return LJ_OK;
}

// Cell grid of one system: the largest cell count per dimension whose side
// is >= min_cell.
void sys_cells(lj_sys& sy, const double* box, const double* min_cell) {
    sy.ncell = 1;
    for (int d = 0; d < 3; ++d) {
        sy.box[d] = box[d];
        sy.half_box[d] = 0.5 * box[d];
        sy.inv_box[d] = 1.0 / box[d];
        sy.nc[d] = cells_for(box[d], min_cell[d]);
        sy.cs[d] = box[d] / sy.nc[d];
        sy.inv_cs[d] = (double)sy.nc[d] / box[d];
        sy.ncell *= sy.nc[d];
    }
}

// Cells for nsys systems with n[s] atoms each; cells of side >= min_cell[3 s + d]
// in dimension d.
lj_status alloc_cells(int nsys, const int64_t* n, const double* box, const double* min_cell,
                      hipStream_t stream, lj_cells** out) {
    lj_cells* c = new (std::nothrow) lj_cells();
    if (!c) return lj_fail(LJ_E_NOMEM, "host allocation");
    c->nsys = nsys;
    c->counts_dirty = true;   // fresh allocation: cleared by the first build
    c->hsys.assign(nsys, lj_sys());
    int64_t atoms = 0, cells = 0;
    for (int s = 0; s < nsys; ++s) {
        lj_sys& sy = c->hsys[s];
        sy.atom0 = atoms;
        sy.n = n[s];
        sy.cell0 = cells;
        sys_cells(sy, box + 3 * s, min_cell + 3 * s);
        atoms += n[s];
        cells += sy.ncell;
    }
    c->n = atoms;
    c->ncell = cells;
    if (cells > (int64_t)16 * 1024 * 1024) {
        delete c;
        return lj_fail(LJ_E_CAPACITY, "more than 16.7M cells: raise the cell size");
    }
    lj_status st;
    if ((st = dmalloc(&c->dsys, nsys)) || (st = dmalloc(&c->count, cells)) ||
        (st = dmalloc(&c->cell_start, cells + 1)) || (st = dmalloc(&c->cid, atoms)) || (st = dmalloc(&c->slot, atoms)) ||
        (st = dmalloc(&c->order_tmp, atoms)) || (st = dmalloc(&c->order, atoms)) ||
        (st = dmalloc(&c->spos, atoms + LJ_SPOS_PAD)) ||
        (st = dmalloc(&c->spos32, atoms + LJ_SPOS_PAD)) ||
        (st = dmalloc(&c->block_sums, lj_scan_workspace(cells)))) {
        cells_release(c);
        return st;
    }
    if (nsys > 1) {
        std::vector<int32_t> as((size_t)atoms);
        for (int s = 0; s < nsys; ++s)
            for (int64_t i = 0; i < n[s]; ++i) as[(size_t)(c->hsys[s].atom0 + i)] = s;
        if ((st = dmalloc(&c->atom_sys, atoms)) || (st = upload(c->atom_sys, as.data(), atoms, stream))) {
            cells_release(c);
            return st;
        }
    }
    if ((st = upload(c->dsys, c->hsys.data(), nsys, stream))) {
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
    if (h.flags & LJ_DEV_BAD_POSITION) {
        (void)reset_status(ctx);
        return lj_fail(LJ_E_POSITION, "a coordinate is non-finite or outside [0, box)");
    }
    return LJ_OK;
}

int default_lanes(int kind) { return kind == LJ_LIST_FULL ? 8 : 8; }

// Sides of the cells the library bins into for its own list builds: the
// search length over k in y and z (default k = 2: each row then visits about
// 2.7x fewer candidates than with a 27-cell stencil of side rs), with a small
// relative margin so that rounding cannot push the reach of rs + delta to one
// more cell.
// Cells are twice as fine along x, the dimension the per-row chords trim at
// cell granularity: about 14% fewer candidates than cubic cells of rs / 2.
void internal_min_cell(const lj_ctx* ctx, double rs, double* mc) {
    int k = ctx->tune[LJ_TUNE_CELL_DIV];
    if (k < 1 || k > 4) k = 2;
    const double side = rs / k * (1.0 + 1e-11);
    mc[0] = 0.5 * side;
    mc[1] = side;
    mc[2] = side;
}

// List fields of a system derived from its cell grid and search length.
void sys_list(lj_sys& sy, double rc, double skin) {
    sy.rc_list = rc;
    sy.skin = skin;
    sy.rs = rc + skin;
    sy.rs2 = sy.rs * sy.rs;
    // delta: a few roundings of the largest coordinate, so that the cell range
    // of a point never misses a cell holding a pair with r < rs
    double L = sy.box[0] > sy.box[1] ? sy.box[0] : sy.box[1];
    L = L > sy.box[2] ? L : sy.box[2];
    const double delta = 16.0 * 2.220446049250313e-16 * (L + sy.rs);
    const double rsd = sy.rs + delta;
    // FP32 culling: inflated by a relative 1e-5, far above the FP32 rounding of
    // the cell-relative quantities it is computed from
    sy.rsd2f = (float)(rsd * rsd * (1.0 + 1e-5));
    // Band of the FP32 pair test.  Coordinates in [0, L) rounded to FP32 are
    // off by at most u L (u = 2^-24); a difference t of two of them, its
    // rounding and an FP32 image shift of +-L leave each component of the
    // separation off by e <= 4 u L + u |t|; then for r <= rx = 1.001 rs
    //   |r2_fp32 - r^2| <= 2 sqrt(3) r e + 3 e^2 + 3.01 u r^2,
    // and the FP64 r^2 is within a few 2^-53 (L rx + rx^2) of r^2.  Beyond rx
    // both tests reject (r^2 - rs^2 > 0.002 rs^2 far exceeds either bound),
    // so outside twice the bound the FP32 test decides exactly as the FP64
    // test does.
    {
        const double u = 5.9604644775390625e-08, u64 = 1.1102230246251565e-16;
        const double rx = 1.001 * sy.rs;
        const double e = 4.0 * u * L + u * rx;
        const double b32 = 2.0 * 1.7320508075688772 * rx * e + 3.0 * e * e + 3.01 * u * rx * rx;
        const double b64 = 16.0 * u64 * (L * rx + rx * rx);
        const double band = 2.0 * (b32 + b64);
        const float lo = (float)(sy.rs2 - band), hi = (float)(sy.rs2 + band);
        // round outward
        sy.r2lo = (double)lo > sy.rs2 - band ? nextafterf(lo, 0.0f) : lo;
        sy.r2hi = (double)hi < sy.rs2 + band ? nextafterf(hi, 3.0e38f) : hi;
    }
    for (int d = 0; d < 3; ++d) {
        sy.cs2f[d] = (float)(sy.cs[d] * sy.cs[d]);
        sy.reach[d] = (int)ceil(rsd / sy.cs[d]);
        sy.full[d] = (sy.nc[d] < 2 * sy.reach[d] + 2) ? 1 : 0;
    }
}

// Slice ranges and slot offsets of every system for the current capacities.
void layout_slices(lj_list* l) {
    const int G = l->lanes, C = LJ_WAVE / G;
    int64_t slices = 0, slots = 0;
    for (lj_sys& sy : l->hsys) {
        sy.slice0 = slices;
        // whole 256-row blocks per system (a multiple of 4G slices)
        const int64_t align = 4 * G;
        sy.nslices = ((sy.n + C - 1) / C + align - 1) / align * align;
        sy.col0 = slots;
        slices += sy.nslices;
        slots += sy.nslices * (int64_t)(sy.cap / G) * LJ_WAVE;
    }
    l->nslices = slices;
    l->ncol = slots;
}

// Allocate the row and slice arrays of a list and fill slice_sys.
lj_status alloc_rows(lj_list* l, hipStream_t stream) {
    const int C = LJ_WAVE / l->lanes;
    const int64_t rows = l->nslices * C;
    lj_status st;
    if ((st = dmalloc(&l->slice_sys, l->nslices)) || (st = dmalloc(&l->row_atom, rows)) ||
        (st = dmalloc(&l->row_len, rows)) || (st = dmalloc(&l->slice_iters, l->nslices)) ||
        (st = dmalloc(&l->slice_stats, l->nslices)) || (st = dmalloc(&l->stats, l->nsys)) ||
        (st = dmalloc(&l->dsys, l->nsys)) || (st = dmalloc(&l->fc, l->nsys)) ||
        (st = dmalloc(&l->xy, rows)) || (st = dmalloc(&l->zz, rows)))
        return st;
    if (l->kind == LJ_LIST_HALF) {
        // the half list's spread force accumulator, zero between force calls
        const int64_t words = 3 * 16 * ((l->n + 15) / 16);
        if ((st = dmalloc(&l->hwin, lj_force_blocks(l->nslices) * LJ_HWIN_REC)) ||
            (st = dmalloc(&l->acc, words)) ||
            (st = lj_launch_zero(stream, l->acc, words * (int64_t)sizeof(double))))
            return st;
    }
    std::vector<int32_t> ss((size_t)l->nslices);
    for (int s = 0; s < l->nsys; ++s)
        for (int64_t t = 0; t < l->hsys[s].nslices; ++t) ss[(size_t)(l->hsys[s].slice0 + t)] = s;
    return upload(l->slice_sys, ss.data(), l->nslices, stream);
}

// The whole build: cells (given or own), then rows, growing each system's
// capacity until every row fits.
lj_status build_list(lj_ctx* ctx, const double* pos, int32_t layout, int nsys, const int64_t* n,
                     const double* box, const double* rc, double skin, int32_t kind,
                     int32_t lanes, const lj_cells* cells, lj_list** out) {
    lj_list* l = new (std::nothrow) lj_list();
    if (!l) return lj_fail(LJ_E_NOMEM, "host allocation");
    l->nsys = nsys;
    l->kind = kind;
    l->lanes = lanes;
    l->build_lanes = lj_build_lanes(ctx, lanes);
    l->device = ctx->device;
    l->stream = ctx->stream;
    l->fc_valid = false;
    lj_status st;
    const lj_cells* c = cells;
    if (!c) {
        std::vector<double> mc((size_t)3 * nsys);
        for (int s = 0; s < nsys; ++s) internal_min_cell(ctx, rc[s] + skin, &mc[(size_t)(3 * s)]);
        if ((st = alloc_cells(nsys, n, box, mc.data(), ctx->stream, &l->cells)) ||
            (st = fill_cells_sync(ctx, pos, layout, l->cells))) {
            list_release(l);
            return st;
        }
        c = l->cells;
    }
    l->n = c->n;
    l->hsys = c->hsys;
    for (int s = 0; s < nsys; ++s) {
        lj_sys& sy = l->hsys[(size_t)s];
        sys_list(sy, rc[s], skin);
        if (sy.reach[0] > 32 || sy.reach[1] > 32 || sy.reach[2] > 32) {
            list_release(l);
            return lj_fail(LJ_E_INVALID, "cells are smaller than (rc + skin) / 32");
        }
        // first guess of the row capacity: 1.25 x the neighbors within rs of
        // an atom at the mean density, plus a margin; grown on overflow
        const double vol = sy.box[0] * sy.box[1] * sy.box[2];
        double expect = 4.18879020478639 * sy.rs * sy.rs * sy.rs * (double)sy.n / vol;
        if (kind == LJ_LIST_HALF) expect *= 0.5;
        int64_t cap = (int64_t)(1.25 * expect + 32.0);
        if (cap > sy.n) cap = sy.n;
        // whole groups of 4 steps of the lanes of a row
        cap = ((cap + 4 * lanes - 1) / (4 * lanes)) * (4 * lanes);
        sy.cap = (int32_t)(cap < 4 * lanes ? 4 * lanes : cap);
    }
    layout_slices(l);
    if ((st = alloc_rows(l, ctx->stream))) {
        list_release(l);
        return st;
    }
    std::vector<lj_list_stats> hs((size_t)nsys);
    for (int attempt = 0; attempt < 3; ++attempt) {
        if (l->ncol > ((int64_t)1 << 31) - 1) {
            st = lj_fail(LJ_E_CAPACITY, "list would exceed 2^31 slots");
            break;
        }
        dfree(l->col);
        l->col = nullptr;
        if ((st = dmalloc(&l->col, l->ncol)) || (st = upload(l->dsys, l->hsys.data(), nsys, ctx->stream)))
            break;
        if ((st = lj_launch_neighbors(ctx, c, l, true))) break;
        LJ_HIP(hipMemcpyAsync(hs.data(), l->stats, (size_t)nsys * sizeof(lj_list_stats),
                              hipMemcpyDeviceToHost, ctx->stream));
        LJ_HIP(hipStreamSynchronize(ctx->stream));
        bool grown = false;
        for (int s = 0; s < nsys; ++s) {
            lj_sys& sy = l->hsys[(size_t)s];
            if (hs[(size_t)s].max_row > sy.cap) {
                int64_t cap = (int64_t)hs[(size_t)s].max_row + hs[(size_t)s].max_row / 16 + lanes;
                cap = ((cap + 4 * lanes - 1) / (4 * lanes)) * (4 * lanes);
                sy.cap = (int32_t)cap;
                grown = true;
            }
        }
        if (!grown) {
            st = LJ_OK;
            break;
        }
        (void)reset_status(ctx);   // drop the overflow flag of the discarded build
        layout_slices(l);
        st = lj_fail(LJ_E_CAPACITY, "row capacity still too small after regrowth");
    }
    if (st) {
        list_release(l);
        return st;
    }
    // the force kernel's block partials must fit in the context
    const int64_t blocks = lj_force_partials(l);
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
    *out = l;
    return LJ_OK;
}

// Force constants for the list's systems; uploaded when they change.
lj_status set_fconst(lj_ctx* ctx, lj_list* l, const double* eps, const double* sigma,
                     const double* rc, int trunc) {
    std::vector<lj_fconst> f((size_t)l->nsys);
    for (int s = 0; s < l->nsys; ++s)
        f[(size_t)s] = lj_make_fconst(eps[s], sigma[s], rc[s], l->hsys[(size_t)s].box, trunc);
    if (l->fc_valid && memcmp(f.data(), l->hfc.data(), f.size() * sizeof(lj_fconst)) == 0)
        return LJ_OK;
    l->hfc = f;
    lj_status st = upload(l->fc, l->hfc.data(), l->nsys, ctx->stream);
    if (st) return st;
    l->fc_valid = true;
    return LJ_OK;
}

lj_status check_trunc(int32_t trunc) {
    if (trunc != LJ_TRUNC_SHIFT && trunc != LJ_TRUNC_FORCE_SHIFT)
        return lj_fail(LJ_E_INVALID, "unknown truncation");
    return LJ_OK;
}

// Forces are written as 32-byte records for AoS positions of either stride.
lj_status check_force_out(int32_t layout, const double* force) {
    if (layout != LJ_SOA && ((uintptr_t)force & 31u))
        return lj_fail(LJ_E_INVALID, "AoS forces must be 32-byte aligned");
    return LJ_OK;
}

lj_status check_params(int nsys, const double* eps, const double* sigma, const double* rc,
                       const lj_list* l) {
    for (int s = 0; s < nsys; ++s) {
        if (!finite_pos(eps[s]) || !finite_pos(sigma[s]) || !finite_pos(rc[s]))
            return lj_fail(LJ_E_INVALID, "eps, sigma and rc must be finite and > 0");
        if (rc[s] > l->hsys[(size_t)s].rc_list)
            return lj_fail(LJ_E_STALE, "rc is larger than the list's cutoff");
    }
    return LJ_OK;
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
    ctx->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    for (int k = 0; k < LJ_TUNE_N; ++k) ctx->tune[k] = 0;
    lj_status st = dmalloc(&ctx->st, 1);
    if (st) {
        delete ctx;
        return st;
    }
    ctx->partials_cap = 4096;
    if ((st = dmalloc(&ctx->partials, 4 * ctx->partials_cap)) ||
        (st = lj_scratch_partials(device, &ctx->scratch))) {
        dfree(ctx->st);
        dfree(ctx->partials);
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
    if (h.flags & LJ_DEV_ROW_OVERFLOW)
        return lj_fail(LJ_E_CAPACITY, (h.flags & LJ_DEV_RESTORED)
                                          ? "a list row exceeded its capacity (the integrator "
                                            "stopped at its last good step)"
                                          : "a list row exceeded its capacity");
    if (h.flags & LJ_DEV_STALE)
        return lj_fail(LJ_E_STALE, "an integrator step at a fixed rebuild cadence found an atom "
                                   "moved more than skin/2 since the list was built");
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
    const double mc[3] = {min_cell, min_cell, min_cell};
    if ((st = alloc_cells(1, &n, box, mc, ctx->stream, &c))) return st;
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
        for (int d = 0; d < 3; ++d) nc[d] = c->hsys[0].nc[d];
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
    if ((st = check_box(box, rc + skin))) return st;
    if (cells) {
        if (cells->nsys != 1 || cells->n != n)
            return lj_fail(LJ_E_STALE, "cells were built for another atom count");
        for (int d = 0; d < 3; ++d)
            if (cells->hsys[0].box[d] != box[d])
                return lj_fail(LJ_E_STALE, "cells were built for another box");
    }
    DeviceGuard guard(ctx->device);
    return build_list(ctx, pos, layout, 1, &n, box, &rc, skin, kind, lanes, cells, list);
}

extern "C" lj_status lj_build_neighbors_batch(lj_ctx* ctx, const double* pos, int32_t layout,
                                              int32_t nsys, const int64_t* n, const double* box,
                                              const double* rc, double skin, int32_t kind,
                                              int32_t lanes, lj_list** list) {
    if (!ctx || !pos || !n || !box || !rc || !list)
        return lj_fail(LJ_E_INVALID, "NULL argument");
    if (nsys < 1) return lj_fail(LJ_E_INVALID, "nsys must be >= 1");
    int64_t total = 0;
    for (int s = 0; s < nsys; ++s) {
        if (n[s] < 1) return lj_fail(LJ_E_INVALID, "every system needs at least one atom");
        if (!finite_pos(rc[s])) return lj_fail(LJ_E_INVALID, "rc must be finite and > 0");
        total += n[s];
    }
    lj_status st = check_common(ctx, pos, total, layout);
    if (st) return st;
    if (!(skin >= 0.0) || !isfinite(skin)) return lj_fail(LJ_E_INVALID, "skin must be finite and >= 0");
    if (kind != LJ_LIST_HALF && kind != LJ_LIST_FULL) return lj_fail(LJ_E_INVALID, "unknown list kind");
    if (lanes == 0) lanes = default_lanes(kind);
    if (lanes < 1 || lanes > 64 || (lanes & (lanes - 1)))
        return lj_fail(LJ_E_INVALID, "lanes must be 1, 2, 4, 8, 16, 32 or 64");
    for (int s = 0; s < nsys; ++s)
        if ((st = check_box(box + 3 * s, rc[s] + skin))) return st;
    DeviceGuard guard(ctx->device);
    return build_list(ctx, pos, layout, nsys, n, box, rc, skin, kind, lanes, nullptr, list);
}

// The mixed kernel's fixed-point copy of the positions: allocated on first
// use, outside any graph capture.
lj_status lj_list_ensure_q32(lj_list* l) {
    if (l->q32) return LJ_OK;
    return dmalloc(&l->q32, l->nslices * (LJ_WAVE / l->lanes));
}

lj_status lj_list_ensure_cells(lj_ctx* ctx, lj_list* l) {
    if (l->cells) return LJ_OK;
    std::vector<int64_t> n((size_t)l->nsys);
    std::vector<double> box((size_t)3 * l->nsys), mc((size_t)3 * l->nsys);
    for (int s = 0; s < l->nsys; ++s) {
        const lj_sys& sy = l->hsys[(size_t)s];
        n[(size_t)s] = sy.n;
        for (int d = 0; d < 3; ++d) box[(size_t)(3 * s + d)] = sy.box[d];
        internal_min_cell(ctx, sy.rs, &mc[(size_t)(3 * s)]);
    }
    lj_status st = alloc_cells(l->nsys, n.data(), box.data(), mc.data(), ctx->stream, &l->cells);
    if (st) return st;
    // the list's own cells may have another grid than the caller's: adopt it
    for (int s = 0; s < l->nsys; ++s) {
        lj_sys& sy = l->hsys[(size_t)s];
        const lj_sys& cs = l->cells->hsys[(size_t)s];
        sy.cell0 = cs.cell0;
        sy.ncell = cs.ncell;
        for (int d = 0; d < 3; ++d) {
            sy.nc[d] = cs.nc[d];
            sy.cs[d] = cs.cs[d];
            sy.inv_cs[d] = cs.inv_cs[d];
        }
        sys_list(sy, sy.rc_list, sy.skin);
    }
    return upload(l->dsys, l->hsys.data(), l->nsys, ctx->stream);
}

extern "C" lj_status lj_update_neighbors(lj_ctx* ctx, const double* pos, int64_t n,
                                         int32_t layout, const double box[3], lj_list* l) {
    lj_status st = check_common(ctx, pos, n, layout);
    if (st) return st;
    if (!l) return lj_fail(LJ_E_INVALID, "list is NULL");
    if (l->n != n) return lj_fail(LJ_E_STALE, "list was built for another atom count");
    if (l->nsys == 1) {
        if (!box) return lj_fail(LJ_E_INVALID, "box is NULL");
        for (int d = 0; d < 3; ++d)
            if (l->hsys[0].box[d] != box[d]) return lj_fail(LJ_E_STALE, "list was built for another box");
    }
    DeviceGuard guard(ctx->device);
    if ((st = lj_list_ensure_cells(ctx, l))) return st;   // lists built on caller cells
    l->stream = ctx->stream;
    if ((st = lj_launch_cells(ctx, pos, layout, l->cells))) return st;
    return lj_launch_neighbors(ctx, l->cells, l, false);
}

// Statistics of the list's latest build, summed on the device first if the
// build did not do it; ordered on the stream of the list's latest build.
lj_status read_list_stats(const lj_list* cl, lj_list_stats* out) {
    lj_list* l = const_cast<lj_list*>(cl);
    DeviceGuard guard(l->device);
    if (l->stats_stale) {
        lj_status st = lj_launch_list_stats(l->stream, l);
        if (st) return st;
    }
    LJ_HIP(hipMemcpyAsync(out, l->stats, (size_t)l->nsys * sizeof(lj_list_stats),
                          hipMemcpyDeviceToHost, l->stream));
    LJ_HIP(hipStreamSynchronize(l->stream));
    return LJ_OK;
}

extern "C" lj_status lj_list_info(const lj_list* l, lj_list_desc* out) {
    if (!l || !out) return lj_fail(LJ_E_INVALID, "list or out is NULL");
    std::vector<lj_list_stats> h((size_t)l->nsys);
    lj_status st = read_list_stats(l, h.data());
    if (st) return st;
    out->n = l->n;
    out->kind = l->kind;
    out->lanes = l->lanes;
    out->cap = 0;
    out->max_row = 0;
    out->entries = 0;
    out->tests = 0;
    for (int s = 0; s < l->nsys; ++s) {
        out->cap = out->cap > l->hsys[(size_t)s].cap ? out->cap : l->hsys[(size_t)s].cap;
        out->max_row = out->max_row > h[(size_t)s].max_row ? out->max_row : h[(size_t)s].max_row;
        out->entries += (int64_t)h[(size_t)s].entries;
        out->tests += (int64_t)h[(size_t)s].tests;
    }
    out->pad = 0;
    out->slots = l->ncol;
    out->rc = l->hsys[0].rc_list;
    out->skin = l->hsys[0].skin;
    for (int d = 0; d < 3; ++d) {
        out->box[d] = l->hsys[0].box[d];
        out->nc[d] = l->hsys[0].nc[d];
    }
    out->nsys = l->nsys;
    return LJ_OK;
}

extern "C" lj_status lj_list_sys_info(const lj_list* l, int32_t s, int64_t* n, int32_t* max_row,
                                      int64_t* entries, int32_t* cap) {
    if (!l) return lj_fail(LJ_E_INVALID, "list is NULL");
    if (s < 0 || s >= l->nsys) return lj_fail(LJ_E_INVALID, "system index out of range");
    std::vector<lj_list_stats> hs((size_t)l->nsys);
    lj_status st = read_list_stats(l, hs.data());
    if (st) return st;
    const lj_list_stats& h = hs[(size_t)s];
    if (n) *n = l->hsys[(size_t)s].n;
    if (max_row) *max_row = h.max_row;
    if (entries) *entries = (int64_t)h.entries;
    if (cap) *cap = l->hsys[(size_t)s].cap;
    return LJ_OK;
}

extern "C" lj_status lj_list_pairs(lj_ctx* ctx, const lj_list* l, int64_t cap, int32_t* ij,
                                   int64_t* npairs) {
    if (!ctx || !l || !npairs) return lj_fail(LJ_E_INVALID, "context, list or npairs is NULL");
    DeviceGuard guard(ctx->device);
    const int G = l->lanes, C = LJ_WAVE / G;
    const int64_t rows = l->nslices * C;
    std::vector<int32_t> ra((size_t)rows), rl((size_t)rows), col((size_t)l->ncol);
    LJ_HIP(hipMemcpyAsync(ra.data(), l->row_atom, rows * sizeof(int32_t), hipMemcpyDeviceToHost,
                          ctx->stream));
    LJ_HIP(hipMemcpyAsync(rl.data(), l->row_len, rows * sizeof(int32_t), hipMemcpyDeviceToHost,
                          ctx->stream));
    LJ_HIP(hipMemcpyAsync(col.data(), l->col, l->ncol * sizeof(int32_t), hipMemcpyDeviceToHost,
                          ctx->stream));
    LJ_HIP(hipStreamSynchronize(ctx->stream));
    int64_t total = 0;
    for (const lj_sys& sy : l->hsys)
        for (int64_t r = 0; r < sy.n; ++r) total += rl[(size_t)(sy.slice0 * C + r)];
    *npairs = total;
    if (cap < total || (!ij && total > 0))
        return lj_fail(LJ_E_CAPACITY, "ij is too small for the list");
    int64_t k = 0;
    for (const lj_sys& sy : l->hsys) {
        const int S = sy.cap / G;
        for (int64_t r = 0; r < sy.n; ++r) {
            const int64_t R = sy.slice0 * C + r;
            const int64_t t = r / C, c = r % C;
            const uint32_t base = (uint32_t)(t * S * LJ_WAVE + c * G * 4);
            for (int e = 0; e < rl[(size_t)R]; ++e) {
                const int64_t at = sy.col0 + lj_slot(base, (uint32_t)e, G);
                ij[2 * k] = ra[(size_t)R];
                // entries are cell-sorted ranks: the atom of rank j is that of row j
                ij[2 * k + 1] = ra[(size_t)(sy.slice0 * C + (col[(size_t)at] - sy.atom0))];
                ++k;
            }
        }
    }
    return LJ_OK;
}

extern "C" lj_status lj_list_device_view(const lj_list* l, lj_list_view* out) {
    if (!l || !out) return lj_fail(LJ_E_INVALID, "list or out is NULL");
    if (l->nsys != 1) return lj_fail(LJ_E_INVALID, "the device view describes single-system lists");
    out->col = l->col;
    out->row_atom = l->row_atom;
    out->row_len = l->row_len;
    out->slice_iters = l->slice_iters;
    out->nslices = l->nslices;
    out->lanes = l->lanes;
    out->cap = l->hsys[0].cap;
    return LJ_OK;
}

extern "C" lj_status lj_list_free(lj_list* l) {
    list_release(l);
    return LJ_OK;
}

// ------------------------------------------------------------------ forces

extern "C" lj_status lj_forces(lj_ctx* ctx, const double* pos, int64_t n, int32_t layout,
                               const double box[3], double eps, double sigma, double rc,
                               const lj_list* list, int32_t precision, int32_t trunc,
                               double* force, double* energy, double* virial, int64_t* npairs) {
    lj_status st = check_common(ctx, pos, n, layout);
    if (st) return st;
    if (!list || !force || !energy || !virial)
        return lj_fail(LJ_E_INVALID, "list, force, energy or virial is NULL");
    if ((st = check_force_out(layout, force)) || (st = check_trunc(trunc))) return st;
    if (precision != LJ_FP64 && precision != LJ_MIXED)
        return lj_fail(LJ_E_INVALID, "unknown precision");
    if (!box) return lj_fail(LJ_E_INVALID, "box is NULL");
    if (list->nsys != 1) return lj_fail(LJ_E_INVALID, "a batch list needs lj_forces_batch");
    if (list->n != n) return lj_fail(LJ_E_STALE, "list was built for another atom count");
    for (int d = 0; d < 3; ++d)
        if (list->hsys[0].box[d] != box[d]) return lj_fail(LJ_E_STALE, "list was built for another box");
    if ((st = check_params(1, &eps, &sigma, &rc, list))) return st;
    DeviceGuard guard(ctx->device);
    lj_list* l = const_cast<lj_list*>(list);
    if ((st = set_fconst(ctx, l, &eps, &sigma, &rc, trunc))) return st;
    if (precision == LJ_MIXED && (st = lj_list_ensure_q32(l))) return st;
    lj_force_opts o;
    o.trunc = trunc;
    return lj_launch_forces(ctx, pos, layout, precision, l, l->fc, force, energy, virial, npairs,
                            o);
}

extern "C" lj_status lj_forces_noalloc(lj_ctx* ctx, const double* pos, int64_t n,
                                       int32_t layout, const double box[3], double eps,
                                       double sigma, double rc, const lj_list* list,
                                       int32_t precision, int32_t trunc, double* force,
                                       double* energy, double* virial, int64_t* npairs) {
    lj_status st = check_common(ctx, pos, n, layout);
    if (st) return st;
    if (!list || !force || !energy || !virial)
        return lj_fail(LJ_E_INVALID, "list, force, energy or virial is NULL");
    if ((st = check_force_out(layout, force)) || (st = check_trunc(trunc))) return st;
    if (precision != LJ_FP64 && precision != LJ_MIXED)
        return lj_fail(LJ_E_INVALID, "unknown precision");
    if (!box) return lj_fail(LJ_E_INVALID, "box is NULL");
    if (list->nsys != 1) return lj_fail(LJ_E_INVALID, "a batch list needs lj_forces_batch");
    if (list->n != n) return lj_fail(LJ_E_STALE, "list was built for another atom count");
    for (int d = 0; d < 3; ++d)
        if (list->hsys[0].box[d] != box[d]) return lj_fail(LJ_E_STALE, "list was built for another box");
    if ((st = check_params(1, &eps, &sigma, &rc, list))) return st;
    if (lj_force_partials(list) > LJ_SCRATCH_RECORDS)
        return lj_fail(LJ_E_CAPACITY, "the list needs more block partials than the static "
                                      "scratch holds (131,072 records: about 4M atoms at 8 "
                                      "lanes per row); use lj_forces");
    if (precision == LJ_MIXED && !list->q32)
        return lj_fail(LJ_E_INVALID, "mixed precision needs the list's fixed-point buffer, "
                                     "which lj_forces allocates on its first mixed call");
    DeviceGuard guard(ctx->device);
    lj_list* l = const_cast<lj_list*>(list);
    if ((st = set_fconst(ctx, l, &eps, &sigma, &rc, trunc))) return st;
    lj_force_opts o;
    o.trunc = trunc;
    o.partials = ctx->scratch;
    o.partials_cap = LJ_SCRATCH_RECORDS;
    return lj_launch_forces(ctx, pos, layout, precision, l, l->fc, force, energy, virial, npairs,
                            o);
}

extern "C" lj_status lj_forces_batch(lj_ctx* ctx, const double* pos, int32_t layout,
                                     const lj_list* list, const double* eps, const double* sigma,
                                     const double* rc, int32_t precision, int32_t trunc,
                                     double* force, double* energy, double* virial,
                                     int64_t* npairs) {
    if (!list || !eps || !sigma || !rc || !force || !energy || !virial)
        return lj_fail(LJ_E_INVALID, "NULL argument");
    lj_status st = check_common(ctx, pos, list->n, layout);
    if (st) return st;
    if ((st = check_force_out(layout, force)) || (st = check_trunc(trunc))) return st;
    if (precision != LJ_FP64 && precision != LJ_MIXED)
        return lj_fail(LJ_E_INVALID, "unknown precision");
    if ((st = check_params(list->nsys, eps, sigma, rc, list))) return st;
    DeviceGuard guard(ctx->device);
    lj_list* l = const_cast<lj_list*>(list);
    if ((st = set_fconst(ctx, l, eps, sigma, rc, trunc))) return st;
    if (precision == LJ_MIXED && (st = lj_list_ensure_q32(l))) return st;
    lj_force_opts o;
    o.trunc = trunc;
    return lj_launch_forces(ctx, pos, layout, precision, l, l->fc, force, energy, virial, npairs,
                            o);
}

// -------------------------------------------------------------- integrator

static lj_status nve_create(lj_ctx* ctx, double* pos, double* vel, double* force, int32_t layout,
                            const double* eps, const double* sigma, const double* rc,
                            int32_t precision, int32_t trunc, lj_list* list, double dt,
                            int32_t rebuild_every, double* log, int64_t log_rows, lj_nve** out) {
    lj_status st = check_common(ctx, pos, list ? list->n : 0, layout);
    if (st) return st;
    if (!vel || !force || !list || !out)
        return lj_fail(LJ_E_INVALID, "vel, force, list or out is NULL");
    if (layout == LJ_AOS4 && ((uintptr_t)vel & 31u))
        return lj_fail(LJ_E_INVALID, "LJ_AOS4 velocities must be 32-byte aligned");
    if (layout == LJ_AOS8 && vel != pos + 4)
        return lj_fail(LJ_E_INVALID, "with LJ_AOS8 records vel must be pos + 4");
    if ((st = check_force_out(layout, force)) || (st = check_trunc(trunc))) return st;
    if (!finite_pos(dt)) return lj_fail(LJ_E_INVALID, "dt must be finite and > 0");
    if (precision != LJ_FP64 && precision != LJ_MIXED)
        return lj_fail(LJ_E_INVALID, "unknown precision");
    if (rebuild_every < 0) return lj_fail(LJ_E_INVALID, "rebuild_every must be >= 0");
    if (log_rows < 0 || (log_rows > 0 && !log)) return lj_fail(LJ_E_INVALID, "log is NULL");
    if ((st = check_params(list->nsys, eps, sigma, rc, list))) return st;
    DeviceGuard guard(ctx->device);
    if ((st = lj_list_ensure_cells(ctx, list))) return st;
    if (precision == LJ_MIXED && (st = lj_list_ensure_q32(list))) return st;
    list->stream = ctx->stream;   // the integrator rebuilds it there
    std::vector<lj_fconst> f((size_t)list->nsys);
    for (int s = 0; s < list->nsys; ++s)
        f[(size_t)s] = lj_make_fconst(eps[s], sigma[s], rc[s], list->hsys[(size_t)s].box, trunc);
    return lj_nve_make(ctx, pos, vel, force, layout, f.data(), precision, trunc, list, dt,
                       rebuild_every, log, log_rows, out);
}

extern "C" lj_status lj_nve_create(lj_ctx* ctx, double* pos, double* vel, double* force,
                                   int64_t n, int32_t layout, const double box[3], double eps,
                                   double sigma, double rc, int32_t precision, int32_t trunc,
                                   lj_list* list, double dt, int32_t rebuild_every, double* log,
                                   int64_t log_rows, lj_nve** out) {
    if (!list || !box) return lj_fail(LJ_E_INVALID, "list or box is NULL");
    if (list->nsys != 1) return lj_fail(LJ_E_INVALID, "a batch list needs lj_nve_create_batch");
    if (list->n != n) return lj_fail(LJ_E_STALE, "list was built for another atom count");
    for (int d = 0; d < 3; ++d)
        if (list->hsys[0].box[d] != box[d]) return lj_fail(LJ_E_STALE, "list was built for another box");
    return nve_create(ctx, pos, vel, force, layout, &eps, &sigma, &rc, precision, trunc, list, dt,
                      rebuild_every, log, log_rows, out);
}

extern "C" lj_status lj_nve_create_batch(lj_ctx* ctx, double* pos, double* vel, double* force,
                                         int32_t layout, const double* eps, const double* sigma,
                                         const double* rc, int32_t precision, int32_t trunc,
                                         lj_list* list, double dt, int32_t rebuild_every,
                                         double* log, int64_t log_rows, lj_nve** out) {
    if (!list || !eps || !sigma || !rc) return lj_fail(LJ_E_INVALID, "NULL argument");
    return nve_create(ctx, pos, vel, force, layout, eps, sigma, rc, precision, trunc, list, dt,
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
    return lj_nve_device_steps(const_cast<lj_nve*>(nve), steps);
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
        case LJ_TUNE_BUILD_LANES:
            ok = value == 0 || value == 1 || value == 2 || value == 4 || value == 64;
            break;
        case LJ_TUNE_FORCE_BATCH: ok = value == 0 || value == 2 || value == 4 || value == 8; break;
        case LJ_TUNE_CELL_DIV: ok = value >= 0 && value <= 4; break;
        case LJ_TUNE_KICK: ok = value >= 0 && value <= 2; break;
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
