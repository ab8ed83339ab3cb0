// lj_neigh.hip -- Verlet list build (Sec. III.B: every pair closer than the
// search length rs = rc + skin, found through the cells; Sec. III.C: grouped
// by i so each row is that atom's SortedList).
//
// Work mapping.  Rows are the atoms in cell order.  A wavefront builds
// 64 / GB consecutive rows with GB lanes per row (GB <= G, the lanes per row
// of the list layout), and appends straight into the wavefront-sliced slots of
// the layout: a single pass, no count-then-fill.
//
// Candidate cells.  Cells have side >= rs/2 by default, so a neighbor lies
// within R = 2 cells per dimension.  Each row visits only the (y, z) cell rows
// within rs of its atom and, in each, only the x cells covering the chord
// [x - w, x + w], w = sqrt(rs^2 - d_yz^2): about 2.7x fewer candidates than a
// 27-cell stencil of side rs.  This culling only decides which candidates are
// tested; it runs in FP32 on cell-relative coordinates with margins that make
// it conservative.  The x cells of a cell row are one contiguous range of the
// cell-sorted atoms, split in two where it wraps around the box.
//
// Exactness of the pair test.  t = q_j - q_i is formed in FP64 and brought to
// the nearest image, and r^2 = (tx*tx + ty*ty) + tz*tz with every operation
// rounded on its own (no FMA contraction); the pair is kept iff r^2 < rs^2.
// When a dimension has at least 2R + 2 cells the image is known from the cell
// offset and applied as one addition of -L, 0 or +L, which rounds exactly as
// the compare-and-subtract form does, because a pair reached through another
// image has |t| >= L/2 >= rs and is rejected either way.  A dimension with
// fewer cells is scanned whole with the compare form.
#include "lj_internal.h"

namespace {

struct NeighArgs {
    int64_t n;
    int64_t nslices;
    int nc[3];
    int reach[3];          // R: cells within rs + delta of a point lie within +-R
    int full[3];           // 1: the dimension has < 2R + 2 cells -> scan all of them
    double box[3];
    double half_box[3];
    double inv_cs[3];
    float cs2f[3];         // cell side^2 (FP32, culling only)
    float rsd2f;           // (rs + delta)^2, inflated (culling only)
    double rs2;
    int cap;
    const int32_t* cell_start;
    const double4* spos;
    int32_t* row_atom;
    int32_t* row_len;
    int32_t* slice_iters;
    int32_t* slice_stats;  // 2 per slice: longest row before clamping, entries stored
    int32_t* col;
};

__device__ __forceinline__ double r2_rounded(double x, double y, double z) {
#pragma clang fp contract(off)
    return (x * x + y * y) + z * z;
}

// Nearest image by comparison against L/2 (used when a dimension is scanned whole).
__device__ __forceinline__ double nearest(double t, double L, double hL) {
    const double a = t - L, b = t + L;
    return t > hL ? a : (t < -hL ? b : t);
}

// Gap, in cells, between a point at fraction f in [0, 1) of its cell and the
// cell at offset o (0 for the point's own cell).
__device__ __forceinline__ float cell_gap(int o, float f) {
    return o > 0 ? (float)o - f : (o < 0 ? f - (float)(o + 1) : 0.0f);
}

template <int G, int GB, bool HALF, bool ANYFULL>
__global__ __launch_bounds__(LJ_BLOCK) void k_neigh(NeighArgs a) {
    constexpr int CB = LJ_WAVE / GB;   // rows per wavefront in the build
    constexpr int C = LJ_WAVE / G;     // rows per slice of the layout
    constexpr int SL = C * GB;         // lanes of the wavefront that hold one slice
    const int lane = threadIdx.x & (LJ_WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(
        (int)lj_xcd_block(blockIdx.x, gridDim.x) * LJ_WAVES_PER_BLOCK + (threadIdx.x >> 6));
    const int64_t row0 = (int64_t)wv * CB;
    if (row0 >= a.nslices * C) return;   // whole wavefront leaves together
    const int cb = lane / GB, g = lane % GB;
    const int64_t r = row0 + cb;
    const int r32 = (int)r;
    const bool row_ok = r < a.n;
    const int64_t slice = r / C;
    const int c = (int)(r % C);
    const int S = a.cap / G;
    const int64_t slot0 = slice * (int64_t)S * LJ_WAVE + c * G;
    int32_t* __restrict__ col = a.col;

    const double4 qi = a.spos[row_ok ? r : 0];
    const int32_t self = (int32_t)qi.w;
    const int nx = a.nc[0], ny = a.nc[1], nz = a.nc[2];
    // cell of the atom and its fractional position in the cell (FP32, culling only)
    const int cx = lj_cell_coord(qi.x, a.inv_cs[0], nx);
    const int cy = lj_cell_coord(qi.y, a.inv_cs[1], ny);
    const int cz = lj_cell_coord(qi.z, a.inv_cs[2], nz);
    const float fx = (float)(qi.x * a.inv_cs[0] - cx);
    const float fy = (float)(qi.y * a.inv_cs[1] - cy);
    const float fz = (float)(qi.z * a.inv_cs[2] - cz);

    const bool fullx = ANYFULL && a.full[0], fully = ANYFULL && a.full[1],
               fullz = ANYFULL && a.full[2];
    const int Rx = a.reach[0], Ry = fully ? 0 : a.reach[1], Rz = fullz ? 0 : a.reach[2];
    const int ky_n = fully ? ny : 2 * Ry + 1, kz_n = fullz ? nz : 2 * Rz + 1;

    // the ballot bits of this row's GB lanes
    const uint64_t grp = (GB == LJ_WAVE) ? ~0ull : (((1ull << (GB & 63)) - 1ull) << (cb * GB));
    const uint32_t grp_lo = (uint32_t)grp, grp_hi = (uint32_t)(grp >> 32);
    int cnt = 0;

    // test candidates s0 .. s0+m-1 (cell-sorted ranks); x shifted by shx if shifted_x
    auto test = [&](int s, double shx, double shy, double shz, bool shifted_x, int32_t& jv) {
        const double4 qj = *reinterpret_cast<const double4*>(
            reinterpret_cast<const char*>(a.spos) + (uint32_t)s * 32u);
        double tx = qj.x - qi.x, ty = qj.y - qi.y, tz = qj.z - qi.z;
        if (ANYFULL) {
            tx = fullx ? nearest(tx, a.box[0], a.half_box[0]) : (shifted_x ? tx + shx : tx);
            ty = fully ? nearest(ty, a.box[1], a.half_box[1]) : ty + shy;
            tz = fullz ? nearest(tz, a.box[2], a.half_box[2]) : tz + shz;
        } else {
            if (shifted_x) tx = tx + shx;
            ty = ty + shy;
            tz = tz + shz;
        }
        const double r2 = r2_rounded(tx, ty, tz);
        bool own = true;
        if (HALF) own = ((s > r32) != (((s + r32) & 1) != 0));
        jv = (int32_t)qj.w;
        // bitwise: no short-circuit branch around the loads
        return (s != r32) & own & (r2 < a.rs2);
    };
    auto put = [&](uint32_t k, int32_t jv) {
        col[slot0 + (int64_t)(k / (uint32_t)G) * LJ_WAVE + (k % (uint32_t)G)] = jv;
    };
    auto scan = [&](int s0, int m, double shx, double shy, double shz, bool shifted_x) {
        if (GB == 1) {
            // one lane per row: each lane appends to its own row, no ballot
            int f = 0;
            for (; f + 1 < m; f += 2) {
                int32_t j0, j1;
                const bool p0 = test(s0 + f, shx, shy, shz, shifted_x, j0);
                const bool p1 = test(s0 + f + 1, shx, shy, shz, shifted_x, j1);
                if (p0) {
                    if (cnt < a.cap) put((uint32_t)cnt, j0);
                    ++cnt;
                }
                if (p1) {
                    if (cnt < a.cap) put((uint32_t)cnt, j1);
                    ++cnt;
                }
            }
            if (f < m) {
                int32_t j0;
                if (test(s0 + f, shx, shy, shz, shifted_x, j0)) {
                    if (cnt < a.cap) put((uint32_t)cnt, j0);
                    ++cnt;
                }
            }
        } else {
            for (int base = 0; __any(base < m); base += GB) {
                const int f = base + g;
                bool pass = false;
                int32_t jv = 0;
                if (f < m) pass = test(s0 + f, shx, shy, shz, shifted_x, jv);
                const uint64_t ball = __ballot(pass);
                const uint32_t blo = (uint32_t)ball & grp_lo,
                               bhi = (uint32_t)(ball >> 32) & grp_hi;
                const int k = cnt + (int)__builtin_amdgcn_mbcnt_hi(
                                        bhi, __builtin_amdgcn_mbcnt_lo(blo, 0u));
                if (pass && k < a.cap) put((uint32_t)k, jv);
                cnt += __builtin_popcount(blo) + __builtin_popcount(bhi);
            }
        }
    };

    for (int kz = 0; kz < kz_n; ++kz) {
        int wz;
        double shz = 0.0;
        float gz = 0.0f;
        if (fullz) {
            wz = kz;
        } else {
            const int oz = kz - Rz;
            gz = cell_gap(oz, fz);
            wz = cz + oz;
            if (wz < 0) {
                wz += nz;
                shz = -a.box[2];
            } else if (wz >= nz) {
                wz -= nz;
                shz = a.box[2];
            }
        }
        for (int ky = 0; ky < ky_n; ++ky) {
            int wy;
            double shy = 0.0;
            float gy = 0.0f;
            if (fully) {
                wy = ky;
            } else {
                const int oy = ky - Ry;
                gy = cell_gap(oy, fy);
                wy = cy + oy;
                if (wy < 0) {
                    wy += ny;
                    shy = -a.box[1];
                } else if (wy >= ny) {
                    wy -= ny;
                    shy = a.box[1];
                }
            }
            // squared distance from the atom to this cell row (FP32, conservative)
            const float d2 = fmaf(gy * gy, a.cs2f[1], gz * gz * a.cs2f[2]);
            int xa0 = 0, xa1 = 0, xb0 = 0, xb1 = 0;
            double shb = 0.0;
            if (row_ok && d2 < a.rsd2f) {
                if (fullx) {
                    xa1 = nx;
                } else {
                    // chord half-width in cells, inflated
                    const float wcell =
                        __builtin_amdgcn_sqrtf((a.rsd2f - d2) / a.cs2f[0]) * 1.00001f + 1e-5f;
                    int u0 = cx + (int)floorf(fx - wcell);
                    int u1 = cx + (int)floorf(fx + wcell);
                    u0 = max(u0, cx - Rx);
                    u1 = min(u1, cx + Rx);
                    if (u0 < 0) {           // [u0, -1] wraps to the top with -L
                        xb0 = u0 + nx;
                        xb1 = nx;
                        shb = -a.box[0];
                        xa1 = u1 + 1;
                    } else if (u1 >= nx) {  // [nx, u1] wraps to the bottom with +L
                        xa0 = u0;
                        xa1 = nx;
                        xb1 = u1 - nx + 1;
                        shb = a.box[0];
                    } else {
                        xa0 = u0;
                        xa1 = u1 + 1;
                    }
                }
            }
            const int rowbase = (wz * ny + wy) * nx;
            int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
            if (xa1 > xa0) {
                a0 = a.cell_start[rowbase + xa0];
                a1 = a.cell_start[rowbase + xa1];
            }
            if (xb1 > xb0) {
                b0 = a.cell_start[rowbase + xb0];
                b1 = a.cell_start[rowbase + xb1];
            }
            scan(a0, a1 - a0, 0.0, shy, shz, false);
            scan(b0, b1 - b0, shb, shy, shz, true);
        }
    }

    const int len = cnt < a.cap ? cnt : a.cap;
    // longest row and entries of each slice (its SL lanes; no atomics)
    int mx = len, over = cnt, tot = (g == 0) ? len : 0;
#pragma unroll
    for (int d = SL / 2; d >= 1; d >>= 1) {
        mx = max(mx, __shfl_xor(mx, d, LJ_WAVE));
        over = max(over, __shfl_xor(over, d, LJ_WAVE));
        tot += __shfl_xor(tot, d, LJ_WAVE);
    }
    const int iters = (mx + G - 1) / G;
    // pad the row up to the slice length with the row's own atom
    for (int k = len + g; k < iters * G; k += GB) put((uint32_t)k, self);
    if (g == 0) {
        a.row_atom[r] = row_ok ? self : 0;
        a.row_len[r] = row_ok ? len : 0;
    }
    if ((lane % SL) == 0) {
        a.slice_iters[slice] = iters;
        a.slice_stats[2 * slice] = over;
        a.slice_stats[2 * slice + 1] = tot;
    }
}

// One block: longest row and total entries over all slices, and the overflow
// flag of the context when a row did not fit.
__global__ __launch_bounds__(1024) void k_list_stats(const int32_t* __restrict__ slice_stats,
                                                     int64_t nslices, int cap,
                                                     lj_list_stats* stats, lj_dev_status* st) {
    __shared__ int smax[16];
    __shared__ unsigned long long ssum[16];
    int mx = 0;
    unsigned long long tot = 0;
    for (int64_t k = threadIdx.x; k < nslices; k += 1024) {
        mx = max(mx, slice_stats[2 * k]);
        tot += (unsigned long long)slice_stats[2 * k + 1];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        mx = max(mx, __shfl_xor(mx, d, LJ_WAVE));
        tot += __shfl_xor(tot, d, LJ_WAVE);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        smax[wave] = mx;
        ssum[wave] = tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = 0;
        tot = 0;
        for (int w = 0; w < 16; ++w) {
            mx = max(mx, smax[w]);
            tot += ssum[w];
        }
        stats->max_row = mx;
        stats->entries = tot;
        if (mx > cap) atomicOr(&st->flags, LJ_DEV_ROW_OVERFLOW);
    }
}

template <int G, int GB>
lj_status launch_g(lj_ctx* ctx, const NeighArgs& a, bool half, bool anyfull) {
    constexpr int CB = LJ_WAVE / GB;
    const int64_t rows = a.nslices * (LJ_WAVE / G);
    const int64_t waves = (rows + CB - 1) / CB;
    const int64_t blocks = (waves + LJ_WAVES_PER_BLOCK - 1) / LJ_WAVES_PER_BLOCK;
    dim3 grid((unsigned)blocks), block(LJ_BLOCK);
    lj_prof_scope prof(ctx, LJ_PROF_NEIGH);
    if (half) {
        if (anyfull)
            hipLaunchKernelGGL((k_neigh<G, GB, true, true>), grid, block, 0, ctx->stream, a);
        else
            hipLaunchKernelGGL((k_neigh<G, GB, true, false>), grid, block, 0, ctx->stream, a);
    } else {
        if (anyfull)
            hipLaunchKernelGGL((k_neigh<G, GB, false, true>), grid, block, 0, ctx->stream, a);
        else
            hipLaunchKernelGGL((k_neigh<G, GB, false, false>), grid, block, 0, ctx->stream, a);
    }
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}

}  // namespace

lj_status lj_launch_neighbors(lj_ctx* ctx, const lj_cells* c, lj_list* l, double rs) {
    NeighArgs a;
    a.n = l->n;
    a.nslices = l->nslices;
    // delta: a few roundings of the largest coordinate, so that the cell range
    // of a point never misses a cell holding a pair with r < rs
    double L = c->box[0] > c->box[1] ? c->box[0] : c->box[1];
    L = L > c->box[2] ? L : c->box[2];
    const double delta = 16.0 * 2.220446049250313e-16 * (L + rs);
    const double rsd = rs + delta;
    // FP32 culling: inflate by a relative 1e-5 (far above the FP32 rounding of
    // the cell-relative quantities it is computed from)
    a.rsd2f = (float)(rsd * rsd * (1.0 + 1e-5));
    bool anyfull = false;
    for (int d = 0; d < 3; ++d) {
        a.nc[d] = c->nc[d];
        a.box[d] = c->box[d];
        a.half_box[d] = 0.5 * c->box[d];
        a.inv_cs[d] = (double)c->nc[d] / c->box[d];
        a.cs2f[d] = (float)(c->cs[d] * c->cs[d]);
        a.reach[d] = (int)ceil(rsd / c->cs[d]);
        a.full[d] = (c->nc[d] < 2 * a.reach[d] + 2) ? 1 : 0;
        anyfull = anyfull || a.full[d];
    }
    a.rs2 = rs * rs;
    a.cap = l->cap;
    a.cell_start = c->cell_start;
    a.spos = c->spos;
    a.row_atom = l->row_atom;
    a.row_len = l->row_len;
    a.slice_iters = l->slice_iters;
    a.slice_stats = l->slice_stats;
    a.col = l->col;
    const bool half = l->kind == LJ_LIST_HALF;
    // lanes per row in the build: tuned value, at most the layout's
    int gb = ctx->tune[LJ_TUNE_BUILD_LANES];
    if (gb != 1 && gb != 2 && gb != 4) gb = 1;
    if (gb > l->lanes) gb = l->lanes;
    lj_status st;
#define LJ_GB(G)                                                     \
    (gb == 1 ? launch_g<G, 1>(ctx, a, half, anyfull)                 \
             : gb == 2 ? launch_g<G, (G >= 2 ? 2 : 1)>(ctx, a, half, anyfull) \
                       : launch_g<G, (G >= 4 ? 4 : (G >= 2 ? 2 : 1))>(ctx, a, half, anyfull))
    switch (l->lanes) {
        case 1: st = launch_g<1, 1>(ctx, a, half, anyfull); break;
        case 2: st = LJ_GB(2); break;
        case 4: st = LJ_GB(4); break;
        case 8: st = LJ_GB(8); break;
        case 16: st = LJ_GB(16); break;
        case 32: st = LJ_GB(32); break;
        case 64: st = LJ_GB(64); break;
        default: return lj_fail(LJ_E_INVALID, "lanes must be 1, 2, 4, 8, 16, 32 or 64");
    }
#undef LJ_GB
    if (st) return st;
    lj_prof_scope prof(ctx, LJ_PROF_OTHER);
    hipLaunchKernelGGL(k_list_stats, dim3(1), dim3(1024), 0, ctx->stream,
                       (const int32_t*)l->slice_stats, l->nslices, l->cap, l->stats, ctx->st);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}
