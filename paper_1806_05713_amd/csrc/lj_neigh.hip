// lj_neigh.hip -- Verlet list build (Sec. III.B: every pair closer than the
// search length rs = rc + skin, found through the cells; Sec. III.C: grouped
// by i so each row is that atom's SortedList).
//
// One wavefront builds one slice of C = 64 / G rows, G lanes per row.  Rows
// are the atoms in cell order, so the C rows of a slice share (almost always)
// one cell and hence one stencil.  For each of the (up to) 9 (dy, dz) cell
// rows of the stencil the three x-neighbor cells are one or two contiguous
// ranges of the cell-sorted atoms; the G lanes of a row stride through them.
// Accepted neighbors are appended with a wavefront ballot and a prefix count
// within the lane group, straight into the row's sliced slots: a single pass,
// no count-then-fill.
//
// Exactness: the displacement is t = q_j - q_i followed by the nearest-image
// correction, and r^2 = (tx*tx + ty*ty) + tz*tz with each operation rounded
// on its own (no FMA contraction).  When a dimension has >= 3 cells the image
// is known from the stencil offset and applied as one addition of -L, 0 or
// +L -- the same rounded value as the compare-and-subtract form, since a
// pair reached through a different image has |t| >= L/2 >= rs and is
// rejected either way.  With < 3 cells the compare form is used directly.
#include "lj_internal.h"

namespace {

struct NeighArgs {
    int64_t n;
    int64_t nslices;
    int nc[3];
    double box[3];
    double half_box[3];
    double inv_cs[3];
    double rs2;
    int cap;
    const int32_t* cell_start;
    const double4* spos;
    int32_t* row_atom;
    int32_t* row_len;
    int32_t* slice_iters;
    int32_t* col;
    lj_dev_status* st;
    lj_list_stats* stats;
};

__device__ __forceinline__ double r2_rounded(double x, double y, double z) {
#pragma clang fp contract(off)
    return (x * x + y * y) + z * z;
}

// Nearest image by comparison against L/2 (used when a dimension has < 3 cells).
__device__ __forceinline__ double nearest(double t, double L, double hL) {
    const double a = t - L, b = t + L;
    return t > hL ? a : (t < -hL ? b : t);
}

template <int G>
__device__ __forceinline__ int64_t slot(int64_t slice, int S, int c, int k) {
    return ((slice * S + k / G) * LJ_WAVE) + c * G + (k % G);
}

template <int G, bool HALF>
__global__ __launch_bounds__(LJ_BLOCK) void k_neigh(NeighArgs a) {
    constexpr int C = LJ_WAVE / G;
    const int lane = threadIdx.x & (LJ_WAVE - 1);
    const int64_t slice =
        lj_xcd_block(blockIdx.x, gridDim.x) * LJ_WAVES_PER_BLOCK + (threadIdx.x >> 6);
    if (slice >= a.nslices) return;   // whole wavefront leaves together
    const int c = lane / G, g = lane % G;
    const int64_t r = slice * C + c;
    const bool row_ok = r < a.n;
    const double4 qi = a.spos[row_ok ? r : 0];
    const int32_t self = (int32_t)qi.w;
    const int S = a.cap / G;

    const int cx = lj_cell_coord(qi.x, a.inv_cs[0], a.nc[0]);
    const int cy = lj_cell_coord(qi.y, a.inv_cs[1], a.nc[1]);
    const int cz = lj_cell_coord(qi.z, a.inv_cs[2], a.nc[2]);
    const int nx = a.nc[0], ny = a.nc[1], nz = a.nc[2];
    const bool sx = nx >= 3, sy = ny >= 3, sz = nz >= 3;

    // x-ranges of the stencil: cells [xa0, xa1) with no shift, plus [xb0, xb1)
    // shifted by shb (only when the stencil wraps in x).
    int xa0, xa1, xb0 = 0, xb1 = 0;
    double shb = 0.0;
    if (!sx) {
        xa0 = 0;
        xa1 = nx;
    } else if (cx == 0) {
        xa0 = 0;
        xa1 = 2;
        xb0 = nx - 1;
        xb1 = nx;
        shb = -a.box[0];
    } else if (cx == nx - 1) {
        xa0 = nx - 2;
        xa1 = nx;
        xb0 = 0;
        xb1 = 1;
        shb = a.box[0];
    } else {
        xa0 = cx - 1;
        xa1 = cx + 2;
    }

    int cnt = 0;
    const int kz_n = sz ? 3 : nz, ky_n = sy ? 3 : ny;
    for (int kz = 0; kz < kz_n; ++kz) {
        int zz;
        double shz = 0.0;
        if (sz) {
            zz = cz + kz - 1;
            if (zz < 0) {
                zz += nz;
                shz = -a.box[2];
            } else if (zz >= nz) {
                zz -= nz;
                shz = a.box[2];
            }
        } else {
            zz = kz;
        }
        for (int ky = 0; ky < ky_n; ++ky) {
            int yy;
            double shy = 0.0;
            if (sy) {
                yy = cy + ky - 1;
                if (yy < 0) {
                    yy += ny;
                    shy = -a.box[1];
                } else if (yy >= ny) {
                    yy -= ny;
                    shy = a.box[1];
                }
            } else {
                yy = ky;
            }
            const int64_t rowbase = ((int64_t)zz * ny + yy) * nx;
            const int a0 = a.cell_start[rowbase + xa0], a1 = a.cell_start[rowbase + xa1];
            int b0 = 0, b1 = 0;
            if (xb1 > xb0) {
                b0 = a.cell_start[rowbase + xb0];
                b1 = a.cell_start[rowbase + xb1];
            }
            const int ma = a1 - a0;
            const int m = row_ok ? ma + (b1 - b0) : 0;
            for (int base = 0; __any(base < m); base += G) {
                const int f = base + g;
                bool pass = false;
                int32_t jv = 0;
                if (f < m) {
                    const bool in_a = f < ma;
                    const int64_t s = in_a ? (int64_t)(a0 + f) : (int64_t)(b0 + f - ma);
                    const double4 qj = a.spos[s];
                    double tx = qj.x - qi.x, ty = qj.y - qi.y, tz = qj.z - qi.z;
                    if (sx) {
                        tx = tx + (in_a ? 0.0 : shb);
                    } else {
                        tx = nearest(tx, a.box[0], a.half_box[0]);
                    }
                    ty = sy ? ty + shy : nearest(ty, a.box[1], a.half_box[1]);
                    tz = sz ? tz + shz : nearest(tz, a.box[2], a.half_box[2]);
                    const double r2 = r2_rounded(tx, ty, tz);
                    bool own = true;
                    if (HALF) own = ((s > r) != (((s + r) & 1) != 0));
                    pass = (s != r) && own && (r2 < a.rs2);
                    jv = (int32_t)qj.w;
                }
                const uint64_t ball = __ballot(pass);
                uint64_t gm;
                if (G == LJ_WAVE)
                    gm = ball;
                else
                    gm = (ball >> (c * G)) & ((1ull << (G & 63)) - 1ull);
                const int k = cnt + __popcll(gm & ((1ull << g) - 1ull));
                if (pass && k < a.cap) a.col[slot<G>(slice, S, c, k)] = jv;
                cnt += __popcll(gm);
            }
        }
    }

    const int len = cnt < a.cap ? cnt : a.cap;
    // longest row and total of the slice
    int mx = len, over = cnt, tot = (g == 0) ? len : 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        mx = max(mx, __shfl_xor(mx, d, LJ_WAVE));
        over = max(over, __shfl_xor(over, d, LJ_WAVE));
        tot += __shfl_xor(tot, d, LJ_WAVE);
    }
    const int iters = (mx + G - 1) / G;
    // pad the row up to the slice length with the row's own atom
    for (int k = len + g; k < iters * G; k += G) a.col[slot<G>(slice, S, c, k)] = self;
    if (g == 0) {
        a.row_atom[r] = row_ok ? self : 0;
        a.row_len[r] = row_ok ? len : 0;
    }
    if (lane == 0) {
        a.slice_iters[slice] = iters;
        atomicMax(&a.stats->max_row, over);
        atomicAdd(&a.stats->entries, (unsigned long long)tot);
        if (over > a.cap) atomicOr(&a.st->flags, LJ_DEV_ROW_OVERFLOW);
    }
}

template <int G>
lj_status launch_g(lj_ctx* ctx, const NeighArgs& a, bool half) {
    const int64_t blocks = (a.nslices + LJ_WAVES_PER_BLOCK - 1) / LJ_WAVES_PER_BLOCK;
    if (half)
        hipLaunchKernelGGL((k_neigh<G, true>), dim3((unsigned)blocks), dim3(LJ_BLOCK), 0,
                           ctx->stream, a);
    else
        hipLaunchKernelGGL((k_neigh<G, false>), dim3((unsigned)blocks), dim3(LJ_BLOCK), 0,
                           ctx->stream, a);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}

}  // namespace

lj_status lj_launch_neighbors(lj_ctx* ctx, const lj_cells* c, lj_list* l, double rs) {
    NeighArgs a;
    a.n = l->n;
    a.nslices = l->nslices;
    for (int d = 0; d < 3; ++d) {
        a.nc[d] = c->nc[d];
        a.box[d] = c->box[d];
        a.half_box[d] = 0.5 * c->box[d];
        a.inv_cs[d] = (double)c->nc[d] / c->box[d];
    }
    a.rs2 = rs * rs;
    a.cap = l->cap;
    a.cell_start = c->cell_start;
    a.spos = c->spos;
    a.row_atom = l->row_atom;
    a.row_len = l->row_len;
    a.slice_iters = l->slice_iters;
    a.col = l->col;
    a.st = ctx->st;
    a.stats = l->stats;
    lj_status st = lj_launch_zero(ctx->stream, l->stats, sizeof(lj_list_stats));
    if (st) return st;
    lj_prof_scope prof(ctx, LJ_PROF_NEIGH);
    const bool half = l->kind == LJ_LIST_HALF;
    switch (l->lanes) {
        case 1: return launch_g<1>(ctx, a, half);
        case 2: return launch_g<2>(ctx, a, half);
        case 4: return launch_g<4>(ctx, a, half);
        case 8: return launch_g<8>(ctx, a, half);
        case 16: return launch_g<16>(ctx, a, half);
        case 32: return launch_g<32>(ctx, a, half);
        case 64: return launch_g<64>(ctx, a, half);
        default: return lj_fail(LJ_E_INVALID, "lanes must be 1, 2, 4, 8, 16, 32 or 64");
    }
}
