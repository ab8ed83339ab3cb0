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
    int64_t nslices;       // over all systems
    const lj_sys* sys;
    const int32_t* slice_sys;
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
    // the wavefront's rows belong to one system (systems own whole 256-row blocks)
    const int sid = __builtin_amdgcn_readfirstlane(a.slice_sys[row0 / C]);
    const lj_sys& sy = a.sys[sid];
    const int cb = lane / GB, g = lane % GB;
    const int64_t R = row0 + cb;                 // row of the list
    const int64_t lr = R - sy.slice0 * C;        // row within the system
    const bool row_ok = lr < sy.n;
    const int64_t rank = sy.atom0 + (row_ok ? lr : 0);
    const int r32 = (int)rank;
    const int64_t slice = R / C;
    const int c = (int)(R % C);
    const int S = sy.cap / G;
    const int cap = sy.cap;
    const double rs2 = sy.rs2;
    const int64_t slot0 = sy.col0 + (slice - sy.slice0) * (int64_t)S * LJ_WAVE + c * G;
    int32_t* __restrict__ col = a.col;
    const int32_t* __restrict__ cell_start = a.cell_start + sy.cell0;

    const double4 qi = a.spos[rank];
    const int32_t self = (int32_t)qi.w;
    const int nx = sy.nc[0], ny = sy.nc[1], nz = sy.nc[2];
    // cell of the atom and its fractional position in the cell (FP32, culling only)
    const int cx = lj_cell_coord(qi.x, sy.inv_cs[0], nx);
    const int cy = lj_cell_coord(qi.y, sy.inv_cs[1], ny);
    const int cz = lj_cell_coord(qi.z, sy.inv_cs[2], nz);
    const float fx = (float)(qi.x * sy.inv_cs[0] - cx);
    const float fy = (float)(qi.y * sy.inv_cs[1] - cy);
    const float fz = (float)(qi.z * sy.inv_cs[2] - cz);

    const bool fullx = ANYFULL && sy.full[0], fully = ANYFULL && sy.full[1],
               fullz = ANYFULL && sy.full[2];
    const int Rx = sy.reach[0], Ry = fully ? 0 : sy.reach[1], Rz = fullz ? 0 : sy.reach[2];
    const int ky_n = fully ? ny : 2 * Ry + 1, kz_n = fullz ? nz : 2 * Rz + 1;
    const float rsd2f = sy.rsd2f;

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
            tx = fullx ? nearest(tx, sy.box[0], sy.half_box[0]) : (shifted_x ? tx + shx : tx);
            ty = fully ? nearest(ty, sy.box[1], sy.half_box[1]) : ty + shy;
            tz = fullz ? nearest(tz, sy.box[2], sy.half_box[2]) : tz + shz;
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
        return (s != r32) & own & (r2 < rs2);
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
                    if (cnt < cap) put((uint32_t)cnt, j0);
                    ++cnt;
                }
                if (p1) {
                    if (cnt < cap) put((uint32_t)cnt, j1);
                    ++cnt;
                }
            }
            if (f < m) {
                int32_t j0;
                if (test(s0 + f, shx, shy, shz, shifted_x, j0)) {
                    if (cnt < cap) put((uint32_t)cnt, j0);
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
                if (pass && k < cap) put((uint32_t)k, jv);
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
                shz = -sy.box[2];
            } else if (wz >= nz) {
                wz -= nz;
                shz = sy.box[2];
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
                    shy = -sy.box[1];
                } else if (wy >= ny) {
                    wy -= ny;
                    shy = sy.box[1];
                }
            }
            // squared distance from the atom to this cell row (FP32, conservative)
            const float d2 = fmaf(gy * gy, sy.cs2f[1], gz * gz * sy.cs2f[2]);
            int xa0 = 0, xa1 = 0, xb0 = 0, xb1 = 0;
            double shb = 0.0;
            if (row_ok && d2 < rsd2f) {
                if (fullx) {
                    xa1 = nx;
                } else {
                    // chord half-width in cells, inflated
                    const float wcell =
                        __builtin_amdgcn_sqrtf((rsd2f - d2) / sy.cs2f[0]) * 1.00001f + 1e-5f;
                    int u0 = cx + (int)floorf(fx - wcell);
                    int u1 = cx + (int)floorf(fx + wcell);
                    u0 = max(u0, cx - Rx);
                    u1 = min(u1, cx + Rx);
                    if (u0 < 0) {           // [u0, -1] wraps to the top with -L
                        xb0 = u0 + nx;
                        xb1 = nx;
                        shb = -sy.box[0];
                        xa1 = u1 + 1;
                    } else if (u1 >= nx) {  // [nx, u1] wraps to the bottom with +L
                        xa0 = u0;
                        xa1 = nx;
                        xb1 = u1 - nx + 1;
                        shb = sy.box[0];
                    } else {
                        xa0 = u0;
                        xa1 = u1 + 1;
                    }
                }
            }
            const int rowbase = (wz * ny + wy) * nx;
            int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
            if (xa1 > xa0) {
                a0 = cell_start[rowbase + xa0];
                a1 = cell_start[rowbase + xa1];
            }
            if (xb1 > xb0) {
                b0 = cell_start[rowbase + xb0];
                b1 = cell_start[rowbase + xb1];
            }
            scan(a0, a1 - a0, 0.0, shy, shz, false);
            scan(b0, b1 - b0, shb, shy, shz, true);
        }
    }

    const int len = cnt < cap ? cnt : cap;
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
        a.row_atom[R] = row_ok ? self : 0;
        a.row_len[R] = row_ok ? len : 0;
    }
    if ((lane % SL) == 0) {
        a.slice_iters[slice] = iters;
        a.slice_stats[2 * slice] = over;
        a.slice_stats[2 * slice + 1] = tot;
    }
}

// One block per system: longest row and entries over the system's slices, in
// a fixed order, and the overflow flag of the context when a row did not fit.
__global__ __launch_bounds__(1024) void k_list_stats(const int32_t* __restrict__ slice_stats,
                                                     const lj_sys* sys, lj_list_stats* stats,
                                                     lj_dev_status* st) {
    __shared__ int smax[16];
    __shared__ unsigned long long ssum[16];
    const lj_sys& sy = sys[blockIdx.x];
    int mx = 0;
    unsigned long long tot = 0;
    for (int64_t k = sy.slice0 + threadIdx.x; k < sy.slice0 + sy.nslices; k += 1024) {
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
        stats[blockIdx.x].max_row = mx;
        stats[blockIdx.x].entries = tot;
        if (mx > sy.cap) atomicOr(&st->flags, LJ_DEV_ROW_OVERFLOW);
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

lj_status lj_launch_neighbors(lj_ctx* ctx, const lj_cells* c, lj_list* l) {
    NeighArgs a;
    a.nslices = l->nslices;
    a.sys = l->dsys;
    a.slice_sys = l->slice_sys;
    a.cell_start = c->cell_start;
    a.spos = c->spos;
    a.row_atom = l->row_atom;
    a.row_len = l->row_len;
    a.slice_iters = l->slice_iters;
    a.slice_stats = l->slice_stats;
    a.col = l->col;
    bool anyfull = false;
    for (const lj_sys& sy : l->hsys) anyfull = anyfull || sy.full[0] || sy.full[1] || sy.full[2];
    const bool half = l->kind == LJ_LIST_HALF;
    // lanes per row in the build: tuned value, at most the layout's
    int gb = ctx->tune[LJ_TUNE_BUILD_LANES];
    if (gb != 1 && gb != 2 && gb != 4) gb = 4;
    if (gb > l->lanes) gb = l->lanes;
    lj_status st;
#define LJ_GB(G)                                                              \
    (gb == 1 ? launch_g<G, 1>(ctx, a, half, anyfull)                          \
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
    hipLaunchKernelGGL(k_list_stats, dim3((unsigned)l->nsys), dim3(1024), 0, ctx->stream,
                       (const int32_t*)l->slice_stats, (const lj_sys*)l->dsys, l->stats, ctx->st);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}
