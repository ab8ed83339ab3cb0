// lj_neigh.hip -- Verlet list build (Sec. III.B: every pair closer than the
// search length rs = rc + skin, found through the cells; Sec. III.C: grouped
// by i so each row is that atom's SortedList).
//
// Work mapping.  Rows are the atoms in cell order, and every entry goes
// straight into the wavefront-sliced slots of the layout: a single pass, no
// count-then-fill.  Two kernels, chosen by the build-lanes knob:
//   k_neigh_rows (the default): a wavefront builds its rows one at a time,
//     all 64 lanes walking the row's candidates laid end to end (described
//     where it is defined);
//   k_neigh: a wavefront builds 64 / GB consecutive rows side by side with
//     GB lanes per row (GB <= G, the lanes per row of the layout).  With one
//     lane per row (GB = 1) each lane walks its own candidate range with NB
//     candidate records in flight at once (the range may be overrun by up to
//     NB - 1 records, which the cell-sorted position array is padded for;
//     those lanes are masked); with GB > 1 the lanes of a row test
//     consecutive candidates and append in order with a ballot.
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
// (k_neigh_rows decides most candidates with an FP32 test whose outcome is
// provably this one, and the rest with this test.)
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
    const float4* spos32;  // the same rounded to FP32 (x, y, z, atom index bits)
    int32_t* row_atom;
    int32_t* row_len;
    int32_t* slice_iters;
    int4* slice_stats;     // per slice: longest row before clamping, entries stored,
                           // candidates tested, and 1 if a row has entries across a
                           // periodic face (the force kernel then takes nearest images)
    int32_t* col;
    lj_dev_status* st;     // a row that overflows its capacity raises a flag here
    const int32_t* gate;   // when not NULL, build only if *gate != 0 (decided on the device)
};

__device__ __forceinline__ bool gated_off(const int32_t* gate) {
    return gate && __builtin_nontemporal_load(gate) == 0;
}

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
    // (o - f for o > 0, f - (o + 1) for o < 0, 0 for o = 0; f in [0, 1])
    const float of = (float)o;
    return fmaxf(of - f, 0.0f) + fmaxf(f - of - 1.0f, 0.0f);
}

// Which (y, z) cell rows a row visits: R cells either side, or the whole
// dimension when it has too few cells for the image to follow from the offset;
// with the system's grid and culling constants, read once per wavefront.
struct Stencil {
    int ky_n, kz_n, ncombo;
    int Rx, Ry, Rz;
    bool fullx, fully, fullz;
    int nx, ny, nz;
    float inv_kyn;               // 1 / ky_n, for the combination's (y, z) offsets
    float cs2y, cs2z, rsd2f, inv_cs2x;
    double inv_cs[3], box[3];
};

template <bool ANYFULL>
__device__ __forceinline__ Stencil make_stencil(const lj_sys& sy) {
    Stencil s;
    s.fullx = ANYFULL && sy.full[0];
    s.fully = ANYFULL && sy.full[1];
    s.fullz = ANYFULL && sy.full[2];
    s.Rx = sy.reach[0];
    s.Ry = s.fully ? 0 : sy.reach[1];
    s.Rz = s.fullz ? 0 : sy.reach[2];
    s.nx = sy.nc[0];
    s.ny = sy.nc[1];
    s.nz = sy.nc[2];
    s.ky_n = s.fully ? s.ny : 2 * s.Ry + 1;
    s.kz_n = s.fullz ? s.nz : 2 * s.Rz + 1;
    s.ncombo = s.ky_n * s.kz_n;
    s.inv_kyn = 1.0f / (float)s.ky_n;
    s.cs2y = sy.cs2f[1];
    s.cs2z = sy.cs2f[2];
    s.rsd2f = sy.rsd2f;
    s.inv_cs2x = 1.0f / sy.cs2f[0];
    for (int d = 0; d < 3; ++d) {
        s.inv_cs[d] = sy.inv_cs[d];
        s.box[d] = sy.box[d];
    }
    return s;
}

// Cell of a row's atom and its fractional position in the cell (FP32,
// culling only); ok = false for the padding rows past the system's atoms.
struct RowGeo {
    int cx, cy, cz;
    float fx, fy, fz;
    bool ok;
};

__device__ __forceinline__ RowGeo row_geo(const Stencil& st, const double4& q, bool ok) {
    RowGeo g;
    g.cx = lj_cell_coord(q.x, st.inv_cs[0], st.nx);
    g.cy = lj_cell_coord(q.y, st.inv_cs[1], st.ny);
    g.cz = lj_cell_coord(q.z, st.inv_cs[2], st.nz);
    g.fx = (float)(q.x * st.inv_cs[0] - g.cx);
    g.fy = (float)(q.y * st.inv_cs[1] - g.cy);
    g.fz = (float)(q.z * st.inv_cs[2] - g.cz);
    g.ok = ok;
    return g;
}

// Candidate ranges of (y, z) cell-row combination cc of a row: segment A
// (cell rank range [a0, a1), x not shifted) and segment B ([b0, b1), x
// shifted by shb), with the y and z image shifts.  The image of each range is
// also given as a code dx + 3 dy + 9 dz, digit 0 for none, 1 for -L, 2 for +L:
// `code` for A, code + codeb for B.  Written with selects rather than
// branches: every lane of a wavefront runs the same instructions.
struct Seg {
    int a0, a1, b0, b1;
    double shy, shz, shb;
    int code, codeb;
};

__device__ __forceinline__ Seg cell_row_segment(const Stencil& st,
                                                const int32_t* __restrict__ cell_start,
                                                const RowGeo& g, int cc) {
    Seg sg;
    // (y, z) offsets of the combination: the FP32 quotient is within one of
    // the exact one for any realistic count (< 2^22), and corrected
    int kz = (int)(((float)cc + 0.5f) * st.inv_kyn);
    int ky = cc - kz * st.ky_n;
    kz = ky < 0 ? kz - 1 : (ky >= st.ky_n ? kz + 1 : kz);
    ky = cc - kz * st.ky_n;
    int wz = kz, wy = ky;
    float gz = 0.0f, gy = 0.0f;
    int code = 0;
    double shz = 0.0, shy = 0.0;
    if (!st.fullz) {
        const int oz = kz - st.Rz;
        gz = cell_gap(oz, g.fz);
        wz = g.cz + oz;
        const bool lo = wz < 0, hi = wz >= st.nz;
        wz += lo ? st.nz : (hi ? -st.nz : 0);
        code += lo ? 9 : (hi ? 18 : 0);
        shz = lo ? -st.box[2] : (hi ? st.box[2] : 0.0);
    }
    if (!st.fully) {
        const int oy = ky - st.Ry;
        gy = cell_gap(oy, g.fy);
        wy = g.cy + oy;
        const bool lo = wy < 0, hi = wy >= st.ny;
        wy += lo ? st.ny : (hi ? -st.ny : 0);
        code += lo ? 3 : (hi ? 6 : 0);
        shy = lo ? -st.box[1] : (hi ? st.box[1] : 0.0);
    }
    // squared distance from the atom to this cell row (FP32, conservative)
    const float d2 = fmaf(gy * gy, st.cs2y, gz * gz * st.cs2z);
    const bool visit = g.ok && cc < st.ncombo && d2 < st.rsd2f;
    int xa0 = 0, xa1 = st.nx, xb0 = 0, xb1 = 0, codeb = 0;
    double shb = 0.0;
    if (!st.fullx) {
        // chord half-width in cells, inflated (far above the rounding of the
        // FP32 quantities it comes from)
        const float wcell =
            __builtin_amdgcn_sqrtf(fmaxf(st.rsd2f - d2, 0.0f) * st.inv_cs2x) * 1.00001f + 1e-5f;
        const int u0 = max(g.cx + (int)floorf(g.fx - wcell), g.cx - st.Rx);
        const int u1 = min(g.cx + (int)floorf(g.fx + wcell), g.cx + st.Rx);
        const bool lo = u0 < 0, hi = u1 >= st.nx;
        // [u0, -1] wraps to the top with -L; [nx, u1] to the bottom with +L
        xa0 = lo ? 0 : u0;
        xa1 = hi ? st.nx : u1 + 1;
        xb0 = lo ? u0 + st.nx : 0;
        xb1 = lo ? st.nx : (hi ? u1 - st.nx + 1 : 0);
        codeb = lo ? 1 : (hi ? 2 : 0);
        shb = lo ? -st.box[0] : (hi ? st.box[0] : 0.0);
    }
    // a wavefront past the last combination may hold out-of-grid rows: clamp
    // the row it would read (its ranges are empty anyway)
    const int rowbase = visit ? (wz * st.ny + wy) * st.nx : 0;
    const bool va = visit && xa1 > xa0, vb = visit && xb1 > xb0;
    // both loads issued together (a row's whole cell range is in the grid)
    const int a0 = cell_start[rowbase + (va ? xa0 : 0)];
    const int a1 = cell_start[rowbase + (va ? xa1 : 0)];
    sg.a0 = a0;
    sg.a1 = va ? a1 : a0;
    sg.b0 = 0;
    sg.b1 = 0;
    if (vb) {
        sg.b0 = cell_start[rowbase + xb0];
        sg.b1 = cell_start[rowbase + xb1];
    }
    sg.shy = shy;
    sg.shz = shz;
    sg.shb = shb;
    sg.code = code;
    sg.codeb = codeb;
    return sg;
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
    if (gated_off(a.gate)) return;
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
        (uint32_t)((slice - slice_first) * (int64_t)S * LJ_WAVE) + (uint32_t)(c * G * 4);
    const int32_t* __restrict__ cell_start = a.cell_start + sy.cell0;
    const char* __restrict__ spos_b = reinterpret_cast<const char*>(a.spos);

    const double4 qi = a.spos[rank];
    const int32_t self_atom = (int32_t)__double_as_longlong(qi.w);
    const int32_t self = r32;   // entries are cell-sorted ranks; the row's own rank pads it
    const Stencil stn = make_stencil<ANYFULL>(sy);
    const RowGeo geo = row_geo(stn, qi, row_ok);
    const bool fullx = stn.fullx, fully = stn.fully, fullz = stn.fullz;

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
        jv = s;
        // bitwise: no short-circuit branch around the loads; the candidate is
        // the row's own atom iff its rank is
        return (jv != self) & own & (r2 < rs2);
    };
    auto test = [&](int s, double shx, double shy, double shz, bool shifted_x, int32_t& jv) {
        const double4 qj = *reinterpret_cast<const double4*>(spos_b + (uint32_t)s * 32u);
        return test_q(qj, s, shx, shy, shz, shifted_x, jv);
    };
    // entry k of the row: one store through the wavefront's base with a
    // 32-bit offset
    auto put = [&](uint32_t k, int32_t jv) { wcol[lj_slot(lane_slot, k, G)] = jv; };
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
    const int ncombo = stn.ncombo;
    for (int c0 = 0; c0 < ncombo; c0 += GB) {
        const Seg mine = cell_row_segment(stn, cell_start, geo, c0 + g);
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
    // pad the row with the row's own atom up to the slice length rounded to
    // whole groups of 4 steps (the force kernel loads a lane's indices 4 steps
    // at a time)
    for (int k = len + g; k < ((iters + 3) & ~3) * G; k += GB) put((uint32_t)k, self);
    if (g == 0) {
        a.row_atom[R] = row_ok ? self_atom : 0;
        a.row_len[R] = row_ok ? len : 0;
        if (cnt > cap) atomicOr(&a.st->flags, LJ_DEV_ROW_OVERFLOW);   // rare: no contention
    }
    if ((lane % SL) == 0) {
        a.slice_iters[slice] = iters;
        a.slice_stats[slice] = make_int4(over, tot, ntest, 1);   // images not tracked here
    }
}

// ------------------------------------------------------------ row walk
// A wavefront builds RW consecutive rows one at a time, all 64 lanes on one
// row.  The row's candidate ranges (the nonempty segments of its cell rows, in
// combination order) are laid end to end into one stream of T candidates, and
// the wavefront walks the stream 64 at a time: lane l of tile t takes stream
// position 64 t + l.  Only the last tile of a row has idle lanes, where the
// per-segment walk above idles the lanes of every short segment.
//
// Set-up, two rows at once (one per half-wavefront, a cell-row combination
// per lane): prefix sums of the ranges' counts and lengths give each range its
// table entry and its start in the stream; each tile records the entry that
// holds its position 0 and a bit for every range that starts inside it, so a
// lane finds its range with one masked bit count.  A row with more ranges or
// tiles than the table holds walks its segments one at a time instead.
//
// Pair test.  Unless one of its system's dimensions is scanned whole, each
// candidate is first tested on its 16-byte FP32 record (one load instead of
// two for the 32-byte FP64 record): r^2 below the system's r2lo is a pair and
// r^2 at or above r2hi is not, bounds set from the FP32 rounding error (see
// sys_list) so that these decisions are the FP64 test's; the few candidates
// in between are tested again in FP64.
//
// Entries are appended to a copy of the row in LDS and written out when the
// row is done, 16 bytes per lane, so that a row costs one or two store
// instructions rather than one per tile.  Candidate records are read through a
// buffer resource spanning the system's atoms: an offset outside it reads zeros
// and cannot fault.
constexpr int RT_MAXE = 64;   // table entries (nonempty ranges) per row
constexpr int RT_NT = 16;     // tiles of 64 stream positions per row
constexpr int RT_RB = 512;    // entries of a row staged in LDS (the rest go straight out)

// Tile map record: bit p - 1 of `starts` is set when a range starts at tile
// position p; `first` is the entry holding tile position 0.
struct TileMap {
    unsigned long long starts;
    int first, pad;
};

struct RowTable {
    int2 ent[2][RT_MAXE];                  // first rank (system-relative) - stream start, image code
    TileMap tile[2][RT_NT];
    int4 row[RT_RB / 4];                   // the row being built, entries 0 .. RT_RB - 1
};

// Inclusive prefix sum within each 32-lane half of the wavefront (all lanes
// active): shifts within rows of 16 lanes, then row 1 and 3 add the last
// lane of row 0 and 2.
__device__ __forceinline__ int half_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    return v;
}

// Orders the wavefront's LDS accesses before and after this point.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Mask of the lanes below `rem` (none for rem <= 0, all for rem >= 64).
__device__ __forceinline__ uint64_t lanes_below(int rem) {
    return rem >= LJ_WAVE ? ~0ull : (rem <= 0 ? 0ull : ((1ull << rem) - 1ull));
}

__device__ __forceinline__ double dword_pair(unsigned int lo, unsigned int hi) {
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// At least 7 wavefronts per SIMD (up to 72 VGPRs): at 8 (64 VGPRs) the set-up
// spills to scratch, which costs more than the eighth wavefront gains.
// RWMIN: at least this many rows per wavefront (8 or 16; whole slices in any
// case).  Large systems take 16: half the blocks, which matters when a
// launch gated off by the displacement rule still dispatches every block.
template <int G, bool HALF, bool ANYFULL, int RWMIN>
__global__ __launch_bounds__(LJ_BLOCK, 7) void k_neigh_rows(NeighArgs a) {
    if (gated_off(a.gate)) return;
    constexpr int C = LJ_WAVE / G;          // rows per slice of the layout
    constexpr int RW = C > RWMIN ? C : RWMIN;   // rows per wavefront: whole slices
    __shared__ RowTable tables[LJ_WAVES_PER_BLOCK];
    __shared__ double4 shift[27];     // image shift of each code (the block's system)
    __shared__ float4 shift32[27];    // the same rounded to FP32
    RowTable& tb = tables[threadIdx.x >> 6];
    const int lane = threadIdx.x & (LJ_WAVE - 1);
    const int hw = lane >> 5, hl = lane & 31;
    const int64_t blk = lj_xcd_block(blockIdx.x, gridDim.x);
    const int wv = __builtin_amdgcn_readfirstlane(
        (int)blk * LJ_WAVES_PER_BLOCK + (threadIdx.x >> 6));
    // a block's rows belong to one system (systems own whole 256-row blocks)
    {
        const int64_t brow = blk * LJ_WAVES_PER_BLOCK * RW;
        if (brow < a.nslices * C && threadIdx.x < 27) {
            const lj_sys& sb = a.sys[a.slice_sys[brow / C]];
            const int dx = threadIdx.x % 3, dy = (threadIdx.x / 3) % 3, dz = threadIdx.x / 9;
            auto img = [](int d, double L) { return d == 1 ? -L : (d == 2 ? L : 0.0); };
            const double sx = img(dx, sb.box[0]), sy_ = img(dy, sb.box[1]), sz = img(dz, sb.box[2]);
            shift[threadIdx.x] = make_double4(sx, sy_, sz, 0.0);
            shift32[threadIdx.x] = make_float4((float)sx, (float)sy_, (float)sz, 0.0f);
        }
        __syncthreads();
    }
    const int64_t row0 = (int64_t)wv * RW;
    if (row0 >= a.nslices * C) return;   // whole wavefront leaves together
    const int sid = __builtin_amdgcn_readfirstlane(a.slice_sys[row0 / C]);
    const lj_sys& sy = a.sys[sid];
    // the system's constants as values: the list stores in the loops below
    // would otherwise make the compiler read them again from memory
    const int S = sy.cap / G;
    const int cap = sy.cap;
    const double rs2 = sy.rs2;
    const int64_t nsys = sy.n;
    const double hbx = sy.half_box[0], hby = sy.half_box[1], hbz = sy.half_box[2];
    const int64_t slice_first = row0 / C;
    const int64_t lr0 = row0 - sy.slice0 * C;   // first row within the system
    int32_t* __restrict__ wcol =
        a.col + sy.col0 + (slice_first - sy.slice0) * (int64_t)S * LJ_WAVE;
    const int32_t* __restrict__ cell_start = a.cell_start + sy.cell0;
    const int atom0 = (int)sy.atom0;
    const double4* __restrict__ spos = a.spos + atom0;
    const uint64_t nbytes = (uint64_t)nsys * 32u;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)spos, (short)0, (int)(nbytes > 0xffffffffull ? 0xffffffffull : nbytes),
        0x00020000);
    const __amdgpu_buffer_rsrc_t rsrc32 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(a.spos32 + atom0), (short)0, (int)(nbytes / 2u), 0x00020000);
    const float r2lo = sy.r2lo, r2hi = sy.r2hi;
    const Stencil stn = make_stencil<ANYFULL>(sy);

    // entry k of the row whose slots start at `slot`
    auto put = [&](uint32_t slot, uint32_t k, int32_t v) { wcol[lj_slot(slot, k, G)] = v; };
    auto row_slot = [&](int rr) {
        return (uint32_t)((rr / C) * S * LJ_WAVE + (rr % C) * G * 4);
    };

    int keep_len = 0, keep_self = 0, keep_atom = 0;   // lane r: row r of the wavefront
    int sl_mx = 0, sl_over = 0, sl_tot = 0, sl_tests = 0;
    bool sl_img = false;

    // the atoms of all the wavefront's rows (one load) and their cell
    // geometry, one lane per row, kept in LDS
    __shared__ double4 row_q[LJ_WAVES_PER_BLOCK][RW];
    __shared__ RowGeo row_g[LJ_WAVES_PER_BLOCK][RW];
    double4* rq = row_q[threadIdx.x >> 6];
    RowGeo* rg = row_g[threadIdx.x >> 6];
    if (lane < RW) {
        const int64_t lr = lr0 + lane;
        const double4 q = spos[lr < nsys ? (int)lr : 0];
        rq[lane] = q;
        rg[lane] = row_geo(stn, q, lr < nsys);
    }

    for (int p = 0; p < RW; p += 2) {
        // ---- set-up: the table of row p + hw
        wave_lds_sync();
        const RowGeo geo = rg[p + hw];
        if (hl < RT_NT) tb.tile[hw][hl].starts = 0ull;
        wave_lds_sync();
        int ebase = 0, fbase = 0;
        bool img = false;
        for (int cb = 0; cb < stn.ncombo; cb += 32) {
            const Seg sg = cell_row_segment(stn, cell_start, geo, cb + hl);
            const int mA = sg.a1 - sg.a0, mB = sg.b1 - sg.b0;
            const int nA = mA > 0 ? 1 : 0, nB = mB > 0 ? 1 : 0;
            const int ei = half_scan(nA + nB), fi = half_scan(mA + mB);
            int e = ebase + ei - (nA + nB), f = fbase + fi - (mA + mB);
            auto add_range = [&](int s0, int m, int code) {
                if (e < RT_MAXE) tb.ent[hw][e] = make_int2(s0 - atom0 - f, code);
                const int t0 = f >> 6, p0 = f & 63;
                if (p0 != 0 && t0 < RT_NT) atomicOr(&tb.tile[hw][t0].starts, 1ull << (p0 - 1));
                const int t1 = (f + m - 1) >> 6;
                for (int t = (f + 63) >> 6; t <= t1 && t < RT_NT; ++t) tb.tile[hw][t].first = e;
                ++e;
                f += m;
            };
            if (nA) add_range(sg.a0, mA, sg.code);
            if (nB) add_range(sg.b0, mB, sg.code + sg.codeb);
            img = img || (nA && sg.code != 0) || nB;
            ebase += __shfl(ei, (lane & 32) | 31, LJ_WAVE);
            fbase += __shfl(fi, (lane & 32) | 31, LJ_WAVE);
        }
        const uint64_t img_ball = __builtin_amdgcn_ballot_w64(img);
        wave_lds_sync();

        // ---- walk rows p and p + 1
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            const int rr = p + h;
            const int T = __builtin_amdgcn_readlane(fbase, 32 * h);
            const int E = __builtin_amdgcn_readlane(ebase, 32 * h);
            const bool row_img = ((img_ball >> (32 * h)) & 0xffffffffull) != 0;
            const int64_t lrh = lr0 + rr;
            const bool okh = lrh < nsys;
            const int rh = okh ? (int)lrh : 0;
            const double4 qi = rq[rr];
            const int32_t self_atom = (int32_t)__double_as_longlong(qi.w);
            const int32_t self = atom0 + rh;   // entries are ranks; the row's own pads it
            const uint32_t slot = row_slot(rr);
            int cnt = 0;

            // candidate srel (system-relative rank): its record, then the
            // test and the append
            struct Rec {
                double x, y, z;
                int32_t j;
            };
            auto fetch = [&](int srel) {
                const uint32_t off = (uint32_t)srel << 5;
                const auto v0 = __builtin_amdgcn_raw_buffer_load_b128(rsrc, off, 0, 0);
                const auto v1 = __builtin_amdgcn_raw_buffer_load_b128(rsrc, off + 16u, 0, 0);
                return Rec{dword_pair(v0[0], v0[1]), dword_pair(v0[2], v0[3]),
                           dword_pair(v1[0], v1[1]), (int32_t)v1[2]};
            };
            // the lanes of `pass` append their candidate j in lane order
            const int lim = cap < RT_RB ? cap : RT_RB;   // appends that need no check
            auto append = [&](uint64_t pass, int32_t j) {
                const int k = (int)__builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(pass >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)pass, (uint32_t)cnt));
                const int npass = (int)__builtin_popcountll(pass);
                if (cnt + npass <= lim) {
                    if (__builtin_amdgcn_inverse_ballot_w64(pass))
                        reinterpret_cast<int*>(tb.row)[k] = j;
                } else if (__builtin_amdgcn_inverse_ballot_w64(pass) && k < cap) {
                    if (k < RT_RB)
                        reinterpret_cast<int*>(tb.row)[k] = j;
                    else
                        put(slot, (uint32_t)k, j);
                }
                cnt += npass;
            };
            auto test_append = [&](const Rec& q, int srel, uint64_t valid, double shx, double shy,
                                   double shz, auto img_c) {
                constexpr bool IMG = decltype(img_c)::value;
                double tx = q.x - qi.x, ty = q.y - qi.y, tz = q.z - qi.z;
                if (ANYFULL) {
                    tx = stn.fullx ? nearest(tx, stn.box[0], hbx) : (IMG ? tx + shx : tx);
                    ty = stn.fully ? nearest(ty, stn.box[1], hby) : (IMG ? ty + shy : ty);
                    tz = stn.fullz ? nearest(tz, stn.box[2], hbz) : (IMG ? tz + shz : tz);
                } else if (IMG) {
                    tx = tx + shx;
                    ty = ty + shy;
                    tz = tz + shz;
                }
                const double r2 = r2_rounded(tx, ty, tz);
                uint64_t pass = __builtin_amdgcn_ballot_w64(r2 < rs2) & valid &
                                __builtin_amdgcn_ballot_w64(srel != rh);
                if (HALF) pass &= __builtin_amdgcn_ballot_w64((srel > rh) !=
                                                              (((srel + rh) & 1) != 0));
                append(pass, atom0 + srel);
            };
            // table entry of the lane's stream position in tile t
            auto entry = [&](int t) {
                const TileMap tm = tb.tile[h][t];
                const int k = (int)__builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(tm.starts >> 32),
                    __builtin_amdgcn_mbcnt_lo((uint32_t)tm.starts, (uint32_t)tm.first));
                return tb.ent[h][k];
            };
            // software-pipelined: the entry of tile t + 1 is looked up while
            // the records of tile t are in flight
            auto walk = [&](auto img_c) {
                const int nt = (T + 63) >> 6;
                int2 en = nt > 0 ? entry(0) : make_int2(0, 0);
                for (int t = 0; t < nt; ++t) {
                    const int pos = (t << 6) + lane;
                    const int srel = en.x + pos;
                    const Rec q = fetch(srel);
                    double shx = 0.0, shy = 0.0, shz = 0.0;
                    if constexpr (decltype(img_c)::value) {
                        const double4 sh = shift[en.y];
                        shx = sh.x;
                        shy = sh.y;
                        shz = sh.z;
                    }
                    if (t + 1 < nt) en = entry(t + 1);
                    test_append(q, srel, lanes_below(T - (t << 6)), shx, shy, shz, img_c);
                }
            };
            // the same with the FP32 test first (no dimension scanned whole);
            // conditions are kept as 64-bit lane masks
            const float qxf = (float)qi.x, qyf = (float)qi.y, qzf = (float)qi.z;
            auto walk32 = [&](auto img_c) {
                constexpr bool IMG = decltype(img_c)::value;
                const int nt = (T + 63) >> 6;
                int2 en = nt > 0 ? entry(0) : make_int2(0, 0);
                for (int t = 0; t < nt; ++t) {
                    const int pos = (t << 6) + lane;
                    const int srel = en.x + pos;
                    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc32, (uint32_t)srel << 4,
                                                                         0, 0);
                    const int code = en.y;
                    if (t + 1 < nt) en = entry(t + 1);
                    float tx = __uint_as_float(v[0]) - qxf, ty = __uint_as_float(v[1]) - qyf,
                          tz = __uint_as_float(v[2]) - qzf;
                    if constexpr (IMG) {
                        const float4 sh = shift32[code];
                        tx = tx + sh.x;
                        ty = ty + sh.y;
                        tz = tz + sh.z;
                    }
                    // fused: fewer roundings than the bound of sys_list allows for
                    const float r2f = fmaf(tz, tz, fmaf(ty, ty, tx * tx));
                    const uint64_t valid = lanes_below(T - (t << 6));
                    const uint64_t in = __builtin_amdgcn_ballot_w64(r2f < r2lo) & valid;
                    const uint64_t amb = __builtin_amdgcn_ballot_w64(r2f < r2hi) & valid & ~in;
                    uint64_t exact = 0;
                    if (amb != 0) {
                        // rare: the FP64 test for the candidates in the band
                        bool ex = false;
                        if (__builtin_amdgcn_inverse_ballot_w64(amb)) {
                            const Rec q = fetch(srel);
                            double ex_ = q.x - qi.x, ey = q.y - qi.y, ez = q.z - qi.z;
                            if constexpr (IMG) {
                                const double4 sh = shift[code];
                                ex_ = ex_ + sh.x;
                                ey = ey + sh.y;
                                ez = ez + sh.z;
                            }
                            ex = r2_rounded(ex_, ey, ez) < rs2;
                        }
                        exact = __builtin_amdgcn_ballot_w64(ex) & amb;
                    }
                    uint64_t pass = (in | exact) & __builtin_amdgcn_ballot_w64(srel != rh);
                    if (HALF) pass &= __builtin_amdgcn_ballot_w64((srel > rh) !=
                                                                  (((srel + rh) & 1) != 0));
                    append(pass, atom0 + srel);
                }
            };
            if (T <= RT_NT * LJ_WAVE && E <= RT_MAXE) {
                if (ANYFULL && (stn.fullx || stn.fully || stn.fullz)) {
                    if (row_img)
                        walk(std::true_type());
                    else
                        walk(std::false_type());
                } else {
                    if (row_img)
                        walk32(std::true_type());
                    else
                        walk32(std::false_type());
                }
            } else {
                // a long row: its segments one at a time, 64 candidates per pass
                const RowGeo g1 = rg[rr];
                for (int cc = 0; cc < stn.ncombo; ++cc) {
                    const Seg sg = cell_row_segment(stn, cell_start, g1, cc);
                    const int mA = sg.a1 - sg.a0, mB = sg.b1 - sg.b0;
                    for (int o = 0; o < mA; o += LJ_WAVE) {
                        const int srel = sg.a0 - atom0 + o + lane;
                        test_append(fetch(srel), srel, lanes_below(mA - o), 0.0, sg.shy, sg.shz,
                                    std::true_type());
                    }
                    for (int o = 0; o < mB; o += LJ_WAVE) {
                        const int srel = sg.b0 - atom0 + o + lane;
                        test_append(fetch(srel), srel, lanes_below(mB - o), sg.shb, sg.shy, sg.shz,
                                    std::true_type());
                    }
                }
            }

            const int len = cnt < cap ? cnt : cap;
            // write out the staged entries, one per lane and pass (64
            // consecutive entries of a row fill whole 128-byte runs of the
            // layout), the last group of G completed with the row's own atom
            {
                wave_lds_sync();
                const int fl = len <= RT_RB ? (len + G - 1) / G * G : RT_RB;
                const int* rowb = reinterpret_cast<const int*>(tb.row);
                for (int k = lane; k < fl; k += LJ_WAVE)
                    put(slot, (uint32_t)k, k < len ? rowb[k] : self);
                wave_lds_sync();
            }
            if (lane == rr) {
                keep_len = len;
                keep_self = self;
                keep_atom = okh ? self_atom : 0;
            }
            if (cnt > cap && lane == 0) atomicOr(&a.st->flags, LJ_DEV_ROW_OVERFLOW);
            sl_mx = max(sl_mx, len);
            sl_over = max(sl_over, cnt);
            sl_tot += len;
            sl_tests += T;
            // a dimension scanned whole takes nearest images in the walk
            sl_img = sl_img || row_img || (ANYFULL && (stn.fullx || stn.fully || stn.fullz));
            if ((rr + 1) % C == 0) {
                // the slice is complete: pad its rows with their own atom
                const int iters = (sl_mx + G - 1) / G;
                const int padded = ((iters + 3) & ~3) * G;   // whole groups of 4 steps
                for (int j = rr + 1 - C; j <= rr; ++j) {
                    const int lj = __builtin_amdgcn_readlane(keep_len, j);
                    const int sj = __builtin_amdgcn_readlane(keep_self, j);
                    const uint32_t sl = row_slot(j);
                    // written so far: the staged entries rounded up to G
                    const int from = lj <= RT_RB ? (lj + G - 1) / G * G : lj;
                    for (int k = from + lane; k < padded; k += LJ_WAVE) put(sl, (uint32_t)k, sj);
                }
                if (lane == 0) {
                    const int64_t slice = slice_first + rr / C;
                    a.slice_iters[slice] = iters;
                    a.slice_stats[slice] = make_int4(sl_over, sl_tot, sl_tests, sl_img ? 1 : 0);
                }
                sl_mx = sl_over = sl_tot = sl_tests = 0;
                sl_img = false;
            }
        }
    }
    if (lane < RW) {
        a.row_atom[row0 + lane] = keep_atom;
        a.row_len[row0 + lane] = keep_len;
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

template <int G, int RWMIN>
lj_status launch_rows_rw(lj_ctx* ctx, const NeighArgs& a, bool half, bool anyfull) {
    constexpr int C = LJ_WAVE / G;
    constexpr int RW = C > RWMIN ? C : RWMIN;
    const int64_t rows = a.nslices * C;
    const int64_t waves = (rows + RW - 1) / RW;
    const int64_t blocks = (waves + LJ_WAVES_PER_BLOCK - 1) / LJ_WAVES_PER_BLOCK;
    dim3 grid((unsigned)blocks), block(LJ_BLOCK);
    lj_prof_scope prof(ctx, LJ_PROF_NEIGH);
    if (half) {
        if (anyfull)
            hipLaunchKernelGGL((k_neigh_rows<G, true, true, RWMIN>), grid, block, 0, ctx->stream, a);
        else
            hipLaunchKernelGGL((k_neigh_rows<G, true, false, RWMIN>), grid, block, 0, ctx->stream, a);
    } else {
        if (anyfull)
            hipLaunchKernelGGL((k_neigh_rows<G, false, true, RWMIN>), grid, block, 0, ctx->stream, a);
        else
            hipLaunchKernelGGL((k_neigh_rows<G, false, false, RWMIN>), grid, block, 0, ctx->stream,
                               a);
    }
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}

// 16 rows per wavefront once the list has rows for more than four rounds of
// resident blocks at 16 (7 wavefronts per SIMD), else 8.
template <int G>
lj_status launch_rows(lj_ctx* ctx, const NeighArgs& a, bool half, bool anyfull) {
    const int64_t rows = a.nslices * (LJ_WAVE / G);
    const int64_t resident_rows16 = (int64_t)ctx->cus * 4 * 7 * 16;
    if (rows >= 4 * resident_rows16) return launch_rows_rw<G, 16>(ctx, a, half, anyfull);
    return launch_rows_rw<G, 8>(ctx, a, half, anyfull);
}

}  // namespace

int lj_build_lanes(const lj_ctx* ctx, int lanes) {
    // tuned value; default: the whole wavefront on one row (any layout).
    // 1, 2 or 4 lanes per row are at most the layout's lanes per row.
    int gb = ctx->tune[LJ_TUNE_BUILD_LANES];
    if (gb != 1 && gb != 2 && gb != 4) return LJ_WAVE;
    return gb > lanes ? lanes : gb;
}

lj_status lj_launch_neighbors(lj_ctx* ctx, const lj_cells* c, lj_list* l, bool stats,
                              const int32_t* gate) {
    NeighArgs a;
    a.gate = gate;
    a.nslices = l->nslices;
    a.sys = l->dsys;
    a.slice_sys = l->slice_sys;
    a.cell_start = c->cell_start;
    a.spos = c->spos;
    a.spos32 = c->spos32;
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
    (gb == LJ_WAVE ? launch_rows<G>(ctx, a, half, anyfull)                    \
     : gb == 1 ? launch_g<G, 1>(ctx, a, half, anyfull)                        \
             : gb == 2 ? launch_g<G, (G >= 2 ? 2 : 1)>(ctx, a, half, anyfull) \
                       : launch_g<G, (G >= 4 ? 4 : (G >= 2 ? 2 : 1))>(ctx, a, half, anyfull))
    switch (l->lanes) {
        case 1: st = gb == LJ_WAVE ? launch_rows<1>(ctx, a, half, anyfull)
                           : launch_g<1, 1>(ctx, a, half, anyfull);
                break;
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
    if ((st = lj_launch_half_windows(ctx, l, gate))) return st;
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
