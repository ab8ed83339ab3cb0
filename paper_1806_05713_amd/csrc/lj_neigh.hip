// lj_neigh.hip -- Verlet list build (Sec. III.B: every pair closer than the
// search length rs = rc + skin, found through the cells; Sec. III.C: grouped
// by i so each row is that atom's SortedList).
//
// Work mapping.  Rows are the atoms in cell order.  A wavefront builds
// 64 / GB consecutive rows with GB lanes per row (GB <= G, the lanes per row
// of the list layout), and appends straight into the wavefront-sliced slots of
// the layout: a single pass, no count-then-fill.  With one lane per row
// (GB = 1) each lane walks its own candidate range with NB candidate records
// in flight at once (the range may be overrun by up to NB - 1 records, which
// the cell-sorted position array is padded for; those lanes are masked); with
// GB > 1 the lanes of a row test consecutive candidates and append in order
// with a ballot.
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
#include <type_traits>

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
    int4* slice_stats;     // per slice: longest row before clamping, entries stored,
                           // candidates tested, unused
    int32_t* col;
    lj_dev_status* st;     // a row that overflows its capacity raises a flag here
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

// Value of lane q of each group of GB consecutive lanes, for every lane of the
// group (GB <= 4: one quad permutation of the data-parallel primitives).
template <int GB, int Q>
__device__ __forceinline__ int group_bcast(int v) {
    if constexpr (GB == 1) {
        return v;
    } else if constexpr (GB == 2) {
        return __builtin_amdgcn_mov_dpp(v, Q | (Q << 2) | ((2 + Q) << 4) | ((2 + Q) << 6), 0xF,
                                        0xF, true);
    } else {
        return __builtin_amdgcn_mov_dpp(v, Q * 0x55, 0xF, 0xF, true);
    }
}
template <int GB, int Q>
__device__ __forceinline__ double group_bcast(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = group_bcast<GB, Q>((int)(b & 0xffffffffll)),
              hi = group_bcast<GB, Q>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int G, int GB, bool HALF, bool ANYFULL>
__global__ __launch_bounds__(LJ_BLOCK) void k_neigh(NeighArgs a) {
    constexpr int CB = LJ_WAVE / GB;   // rows per wavefront in the build
    constexpr int C = LJ_WAVE / G;     // rows per slice of the layout
    constexpr int SL = C * GB;         // lanes of the wavefront that hold one slice
    constexpr int NB = LJ_SPOS_PAD;    // candidates in flight per lane when GB = 1
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
    // the wavefront's slots start at its first slice; a lane's row at lane_slot
    const int64_t slice_first = row0 / C;
    int32_t* __restrict__ wcol =
        a.col + sy.col0 + (slice_first - sy.slice0) * (int64_t)S * LJ_WAVE;
    const uint32_t lane_slot =
        (uint32_t)((slice - slice_first) * (int64_t)S * LJ_WAVE) + (uint32_t)(c * G);
    const int32_t* __restrict__ cell_start = a.cell_start + sy.cell0;
    const char* __restrict__ spos_b = reinterpret_cast<const char*>(a.spos);

    const double4 qi = a.spos[rank];
    const int32_t self = (int32_t)__double_as_longlong(qi.w);
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
    const float inv_cs2x = 1.0f / sy.cs2f[0];

    // the ballot bits of this row's GB lanes
    const uint64_t grp = (GB == LJ_WAVE) ? ~0ull : (((1ull << (GB & 63)) - 1ull) << (cb * GB));
    const uint32_t grp_lo = (uint32_t)grp, grp_hi = (uint32_t)(grp >> 32);
    int cnt = 0;
    int tests = 0;   // candidates this row tested

    // pair test of candidate rank s with record qj; x shifted by shx if shifted_x
    auto test_q = [&](const double4& qj, int s, double shx, double shy, double shz,
                      bool shifted_x, int32_t& jv) {
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
        jv = (int32_t)__double_as_longlong(qj.w);
        // bitwise: no short-circuit branch around the loads; the candidate is
        // the row's own atom iff its index is
        return (jv != self) & own & (r2 < rs2);
    };
    auto test = [&](int s, double shx, double shy, double shz, bool shifted_x, int32_t& jv) {
        const double4 qj = *reinterpret_cast<const double4*>(spos_b + (uint32_t)s * 32u);
        return test_q(qj, s, shx, shy, shz, shifted_x, jv);
    };
    // entry k of the row: one store through the wavefront's base with a
    // 32-bit offset
    auto put = [&](uint32_t k, int32_t jv) {
        wcol[lane_slot + (k / (uint32_t)G) * (uint32_t)LJ_WAVE + (k % (uint32_t)G)] = jv;
    };
    auto scan = [&](int s0, int m, double shx, double shy, double shz, bool shifted_x) {
        if (GB == 1) {
            // one lane per row: each lane appends to its own row, no ballot;
            // NB records in flight, loaded before any is tested
            for (int f = 0; f < m; f += NB) {
                const char* p = spos_b + (uint32_t)(s0 + f) * 32u;
                double4 q[NB];
#pragma unroll
                for (int u = 0; u < NB; ++u) q[u] = *reinterpret_cast<const double4*>(p + 32 * u);
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    int32_t jv;
                    const bool pass =
                        (f + u < m) & test_q(q[u], s0 + f + u, shx, shy, shz, shifted_x, jv);
                    if (pass) {
                        if (cnt < cap) put((uint32_t)cnt, jv);
                        ++cnt;
                    }
                }
            }
        } else {
            // the row's GB lanes test consecutive candidates; a lane past the
            // end re-tests the last one (masked), so the test never branches
            const int last = m > 0 ? m - 1 : 0;
            for (int base = 0; __any(base < m); base += GB) {
                const int f = base + g;
                int32_t jv;
                const bool pass =
                    (f < m) & test(s0 + min(f, last), shx, shy, shz, shifted_x, jv);
                const uint64_t ball = __builtin_amdgcn_ballot_w64(pass);
                const uint32_t blo = (uint32_t)ball & grp_lo,
                               bhi = (uint32_t)(ball >> 32) & grp_hi;
                const int k = cnt + (int)__builtin_amdgcn_mbcnt_hi(
                                        bhi, __builtin_amdgcn_mbcnt_lo(blo, 0u));
                if (pass & (k < cap)) put((uint32_t)k, jv);
                cnt += __builtin_popcount(blo) + __builtin_popcount(bhi);
            }
        }
    };

    // Candidate ranges of (y, z) cell-row combination cc: segment A (cell
    // rank range [a0, a1), x not shifted) and segment B ([b0, b1), x shifted
    // by shb), with the y and z image shifts.
    struct Seg {
        int a0, a1, b0, b1;
        double shy, shz, shb;
    };
    auto segment = [&](int cc) {
        Seg sg = {0, 0, 0, 0, 0.0, 0.0, 0.0};
        const int kz = cc / ky_n, ky = cc - kz * ky_n;
        int wz, wy;
        float gz = 0.0f, gy = 0.0f;
        if (fullz) {
            wz = kz;
        } else {
            const int oz = kz - Rz;
            gz = cell_gap(oz, fz);
            wz = cz + oz;
            if (wz < 0) {
                wz += nz;
                sg.shz = -sy.box[2];
            } else if (wz >= nz) {
                wz -= nz;
                sg.shz = sy.box[2];
            }
        }
        if (fully) {
            wy = ky;
        } else {
            const int oy = ky - Ry;
            gy = cell_gap(oy, fy);
            wy = cy + oy;
            if (wy < 0) {
                wy += ny;
                sg.shy = -sy.box[1];
            } else if (wy >= ny) {
                wy -= ny;
                sg.shy = sy.box[1];
            }
        }
        // squared distance from the atom to this cell row (FP32, conservative)
        const float d2 = fmaf(gy * gy, sy.cs2f[1], gz * gz * sy.cs2f[2]);
        int xa0 = 0, xa1 = 0, xb0 = 0, xb1 = 0;
        if (row_ok && cc < ky_n * kz_n && d2 < rsd2f) {
            if (fullx) {
                xa1 = nx;
            } else {
                // chord half-width in cells, inflated (far above the rounding
                // of the FP32 quantities it comes from)
                const float wcell =
                    __builtin_amdgcn_sqrtf((rsd2f - d2) * inv_cs2x) * 1.00001f + 1e-5f;
                int u0 = cx + (int)floorf(fx - wcell);
                int u1 = cx + (int)floorf(fx + wcell);
                u0 = max(u0, cx - Rx);
                u1 = min(u1, cx + Rx);
                if (u0 < 0) {           // [u0, -1] wraps to the top with -L
                    xb0 = u0 + nx;
                    xb1 = nx;
                    sg.shb = -sy.box[0];
                    xa1 = u1 + 1;
                } else if (u1 >= nx) {  // [nx, u1] wraps to the bottom with +L
                    xa0 = u0;
                    xa1 = nx;
                    xb1 = u1 - nx + 1;
                    sg.shb = sy.box[0];
                } else {
                    xa0 = u0;
                    xa1 = u1 + 1;
                }
            }
        }
        const int rowbase = (wz * ny + wy) * nx;
        if (xa1 > xa0) {
            sg.a0 = cell_start[rowbase + xa0];
            sg.a1 = cell_start[rowbase + xa1];
        }
        if (xb1 > xb0) {
            sg.b0 = cell_start[rowbase + xb0];
            sg.b1 = cell_start[rowbase + xb1];
        }
        return sg;
    };
    // the row's member q computed combination c0 + q for the whole row
    auto scan_member = [&](const Seg& mine, auto qc) {
        constexpr int Q = decltype(qc)::value;
        const int a0 = group_bcast<GB, Q>(mine.a0), a1 = group_bcast<GB, Q>(mine.a1);
        const int b0 = group_bcast<GB, Q>(mine.b0), b1 = group_bcast<GB, Q>(mine.b1);
        const double shy = group_bcast<GB, Q>(mine.shy), shz = group_bcast<GB, Q>(mine.shz);
        const double shb = group_bcast<GB, Q>(mine.shb);
        tests += (a1 - a0) + (b1 - b0);
        scan(a0, a1 - a0, 0.0, shy, shz, false);
        scan(b0, b1 - b0, shb, shy, shz, true);
    };

    // The (y, z) cell-row combinations, GB at a time: lane g of a row works
    // out combination c0 + g, then the row scans the GB combinations in order.
    const int ncombo = ky_n * kz_n;
    for (int c0 = 0; c0 < ncombo; c0 += GB) {
        const Seg mine = segment(c0 + g);
        scan_member(mine, std::integral_constant<int, 0>());
        if constexpr (GB > 1) {
            if (c0 + 1 < ncombo) scan_member(mine, std::integral_constant<int, 1>());
        }
        if constexpr (GB > 2) {
            if (c0 + 2 < ncombo) scan_member(mine, std::integral_constant<int, 2>());
            if (c0 + 3 < ncombo) scan_member(mine, std::integral_constant<int, 3>());
        }
    }

    const int len = cnt < cap ? cnt : cap;
    // longest row and entries of each slice (its SL lanes; no atomics)
    int mx = len, over = cnt, tot = (g == 0) ? len : 0, ntest = (g == 0) ? tests : 0;
#pragma unroll
    for (int d = SL / 2; d >= 1; d >>= 1) {
        mx = max(mx, __shfl_xor(mx, d, LJ_WAVE));
        over = max(over, __shfl_xor(over, d, LJ_WAVE));
        tot += __shfl_xor(tot, d, LJ_WAVE);
        ntest += __shfl_xor(ntest, d, LJ_WAVE);
    }
    const int iters = (mx + G - 1) / G;
    // pad the row up to the slice length with the row's own atom
    for (int k = len + g; k < iters * G; k += GB) put((uint32_t)k, self);
    if (g == 0) {
        a.row_atom[R] = row_ok ? self : 0;
        a.row_len[R] = row_ok ? len : 0;
        if (cnt > cap) atomicOr(&a.st->flags, LJ_DEV_ROW_OVERFLOW);   // rare: no contention
    }
    if ((lane % SL) == 0) {
        a.slice_iters[slice] = iters;
        a.slice_stats[slice] = make_int4(over, tot, ntest, 0);
    }
}

// One block per system: longest row and entries over the system's slices, in
// a fixed order (the list build itself raises the overflow flag).
__global__ __launch_bounds__(1024) void k_list_stats(const int4* __restrict__ slice_stats,
                                                     const lj_sys* sys, lj_list_stats* stats) {
    __shared__ int smax[16];
    __shared__ unsigned long long ssum[16], stest[16];
    const lj_sys& sy = sys[blockIdx.x];
    int mx = 0;
    unsigned long long tot = 0, tst = 0;
    // four slices per thread and pass, loaded before they are combined
    const int64_t end = sy.slice0 + sy.nslices;
    for (int64_t k0 = sy.slice0 + threadIdx.x; k0 < end; k0 += 4 * 1024) {
        int4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t k = k0 + u * 1024;
            v[u] = k < end ? slice_stats[k] : make_int4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            mx = max(mx, v[u].x);
            tot += (unsigned long long)v[u].y;
            tst += (unsigned long long)v[u].z;
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        mx = max(mx, __shfl_xor(mx, d, LJ_WAVE));
        tot += __shfl_xor(tot, d, LJ_WAVE);
        tst += __shfl_xor(tst, d, LJ_WAVE);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        smax[wave] = mx;
        ssum[wave] = tot;
        stest[wave] = tst;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = 0;
        tot = 0;
        tst = 0;
        for (int w = 0; w < 16; ++w) {
            mx = max(mx, smax[w]);
            tot += ssum[w];
            tst += stest[w];
        }
        stats[blockIdx.x].max_row = mx;
        stats[blockIdx.x].entries = tot;
        stats[blockIdx.x].tests = tst;
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

int lj_build_lanes(const lj_ctx* ctx, int lanes) {
    // tuned value (default 4), at most the layout's lanes per row
    int gb = ctx->tune[LJ_TUNE_BUILD_LANES];
    if (gb != 1 && gb != 2 && gb != 4) gb = 4;
    return gb > lanes ? lanes : gb;
}

lj_status lj_launch_neighbors(lj_ctx* ctx, const lj_cells* c, lj_list* l, bool stats) {
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
    a.st = ctx->st;
    bool anyfull = false;
    for (const lj_sys& sy : l->hsys) anyfull = anyfull || sy.full[0] || sy.full[1] || sy.full[2];
    const bool half = l->kind == LJ_LIST_HALF;
    const int gb = l->build_lanes;
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
    if (!stats) {
        l->stats_stale = true;
        return LJ_OK;
    }
    lj_prof_scope prof(ctx, LJ_PROF_OTHER);
    return lj_launch_list_stats(ctx->stream, l);
}

lj_status lj_launch_list_stats(hipStream_t s, lj_list* l) {
    hipLaunchKernelGGL(k_list_stats, dim3((unsigned)l->nsys), dim3(1024), 0, s,
                       (const int4*)l->slice_stats, (const lj_sys*)l->dsys, l->stats);
    LJ_HIP(hipGetLastError());
    l->stats_stale = false;
    return LJ_OK;
}
