// lj_force_loop.h -- the force loop over one slice of the wavefront-sliced
// Verlet list (Alg. 1 inside the sorted-list loop of Alg. 3): the body of the
// force kernel, kept apart from its launch and reductions so that another
// kernel can evaluate the forces of a slice with the same arithmetic.
// Device code only; included by HIP sources.
#pragma once

#include <type_traits>

#include "lj_internal.h"

namespace ljf {

typedef int v4i __attribute__((ext_vector_type(4)));

struct ForceArgs {
    const double* pos;
    double* force;
    int64_t n;               // atoms over all systems (SoA stride)
    int64_t nslices;
    const lj_sys* sys;
    const lj_fconst* fc;
    const int32_t* slice_sys;
    const int32_t* row_atom;
    const int32_t* row_len;
    const int32_t* slice_iters;
    const int4* slice_stats;  // per slice, .w: 1 if a row has entries across a periodic face
    const int32_t* col;
    double* partials;        // 4 doubles per (logical) block
    double* acc;             // half list: spread force accumulator (3 x 16 n16 doubles),
                             // by rank
    const int32_t* hwin;     // half list: the force blocks' windows
    int64_t n16;
    uint4* q32;              // mixed: fixed-point positions (x, y, z as fractions of the
                             // box), one per row
    const double2* xy;       // FP64: the positions, one per row, split into (x, y)
    const double* zz;        // records and z: one 16-byte and one 8-byte gather
                             // (the row of rank j of a system is j + slice0 C - atom0)
    const int32_t* halt;     // device status flags: the kernel does nothing once an
                             // error flag is raised (NULL: never)
    uint32_t qshift;         // AoS record stride as a shift: 5 (32-byte records) or 6
                             // (64-byte position-velocity records)
    int32_t kick;            // LJ_KICK_*
    double* vel;             // kicked velocities (layout and stride of the positions)
    double hdt;              // dt / 2
    int32_t write_f;         // with a kick: also store the forces
};

__device__ __forceinline__ double r2_rounded(double x, double y, double z) {
#pragma clang fp contract(off)
    return (x * x + y * y) + z * z;
}

// Half list: the Newton's-third-law scatter goes into an accumulator with
// one block per component, so that the three atomics of a pair do not queue
// on one cache line.
__device__ __forceinline__ void acc_add(double* __restrict__ acc, int64_t n16, int64_t i,
                                        double x, double y, double z) {
    unsafeAtomicAdd(acc + i, x);
    unsafeAtomicAdd(acc + 16 * n16 + i, y);
    unsafeAtomicAdd(acc + 32 * n16 + i, z);
}

// Forces: 32-byte records (x, y, z, 0) for AoS positions of either stride, or SoA.
template <int LAYOUT>
__device__ __forceinline__ void store_f(double* __restrict__ f, int64_t n, int64_t i, double x,
                                        double y, double z) {
    if (LAYOUT == LJ_AOS4) {
        reinterpret_cast<double4*>(f)[i] = make_double4(x, y, z, 0.0);
    } else {
        f[i] = x;
        f[n + i] = y;
        f[2 * n + i] = z;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, LJ_WAVE);
    return v;
}

// 1/x as v_rcp_f64 refined by one Newton step y <- y + y (1 - x y), which
// squares the relative error: measured on gfx950 over x in [0.25, 35]
// (the r^2 of the pairs), v_rcp_f64 is within 4.6e-8 of the correctly
// rounded 1/x and one step within 2.2e-15 (mean 1e-16), far inside the
// 1e-10 force and 1e-12 energy tolerances of the FP64 path.
__device__ __forceinline__ double recip(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}

// m ? x : x with its high word cleared, which is +0 or a subnormal below
// 2^-1022 whatever x was (inf and NaN included): its square underflows to an
// exact zero, so every term built from its square or higher powers is an
// exact zero (one 32-bit select in place of two).
__device__ __forceinline__ double keep_or_tiny(bool m, double x) {
    const long long b = __double_as_longlong(x);
    const unsigned hi = m ? (unsigned)((unsigned long long)b >> 32) : 0u;
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) |
                                            ((unsigned long long)b & 0xffffffffull)));
}

// x, y, z of record j: AoS records of 1 << qshift bytes (the position is the
// first three doubles) addressed with a 32-bit byte offset from a uniform
// base, or SoA.
template <int LAYOUT>
__device__ __forceinline__ void gather_q(const double* __restrict__ pos, int64_t n,
                                         uint32_t qshift, int j, double& x, double& y,
                                         double& z) {
    if (LAYOUT == LJ_AOS4) {
        // one dwordx4 + one dwordx2 load
        const double4* q = reinterpret_cast<const double4*>(
            reinterpret_cast<const char*>(pos) + ((uint32_t)j << qshift));
        x = q->x;
        y = q->y;
        z = q->z;
    } else {
        const uint32_t o = (uint32_t)j * 8u;
        x = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(pos) + o);
        y = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(pos + n) + o);
        z = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(pos + 2 * n) + o);
    }
}

// The kick of one row atom i with its summed force (fx, fy, fz): returns the
// kinetic energy of the synchronised velocity.  Every product and sum is
// rounded on its own, as in the integrator's separate kick and drift kernels,
// so both forms give the same velocities bit for bit.
template <int LAYOUT>
__device__ __forceinline__ double kick_row(const ForceArgs& a, int64_t i, double fx, double fy,
                                           double fz) {
#pragma clang fp contract(off)
    double vx, vy, vz, vw = 0.0;
    double4* rec = nullptr;
    if (LAYOUT == LJ_AOS4) {
        rec = reinterpret_cast<double4*>(reinterpret_cast<char*>(a.vel) + (i << a.qshift));
        const double4 v = *rec;
        vx = v.x;
        vy = v.y;
        vz = v.z;
        vw = v.w;
    } else {
        vx = a.vel[i];
        vy = a.vel[a.n + i];
        vz = a.vel[2 * a.n + i];
    }
    const double h = a.hdt;
    vx = vx + h * fx;
    vy = vy + h * fy;
    vz = vz + h * fz;
    const double ke = 0.5 * ((vx * vx + vy * vy) + vz * vz);
    if (a.kick == LJ_KICK_LEAP) {
        vx = vx + h * fx;
        vy = vy + h * fy;
        vz = vz + h * fz;
    }
    if (LAYOUT == LJ_AOS4) {
        *rec = make_double4(vx, vy, vz, vw);
    } else {
        a.vel[i] = vx;
        a.vel[a.n + i] = vy;
        a.vel[2 * a.n + i] = vz;
    }
    return ke;
}

// Loads are issued U entries (U / 4 groups of 4 steps) at a time, and the
// indices of the entries two batches ahead are requested before the current
// ones are computed, so each wavefront keeps up to 2U gathers and U / 2 index
// loads in flight (the load/compute overlap that software pipelining gives a
// CPU core).
// The forces of one slice of system sid, computed by the calling wavefront
// (C = 64 / G rows, G lanes per row); returns the lane's shares of the
// energy, the virial, the pair count and (with a kick) the kinetic energy,
// for the caller to sum in a fixed order.  FS: the force-shifted truncation
// (Sec. III.A), in which each interacting pair's force loses Fc = -V'(rc)
// along the pair and its energy gains (r - rc) Fc, so that both vanish at rc.
template <int G, bool HALF, int LAYOUT, int PREC, int U, bool FS>
__device__ __forceinline__ void slice_forces(const ForceArgs& a, int slice, int sid,
                                             double& e_out, double& w_out, double& c_out,
                                             double& k_out, const signed char* htab,
                                             double* hacc, int hc0) {
    constexpr int C = LJ_WAVE / G;
    const int lane = threadIdx.x & (LJ_WAVE - 1);
    const lj_sys& sy = a.sys[sid];
    const lj_fconst& fc = a.fc[sid];
    const int iters = __builtin_amdgcn_readfirstlane(a.slice_iters[slice]);
    const int c = lane / G, g = lane % G;
    const int64_t r = (int64_t)slice * C + c;
    const int i = a.row_atom[r];        // the row's atom (forces, velocities)
    const int lim = a.row_len[r] - g;   // entry it*G + g is inside the row iff it*G < lim
    const int64_t lr = r - sy.slice0 * C;
    const bool row_ok = lr < sy.n;
    // its cell-sorted rank (entries, gathered copies and the half list's
    // accumulator are indexed by rank)
    const int ri = (int)(sy.atom0 + (row_ok ? lr : 0));
    const double bx = sy.box[0], by = sy.box[1], bz = sy.box[2];
    const double ibx = sy.inv_box[0], iby = sy.inv_box[1], ibz = sy.inv_box[2];
    const double rc2 = fc.rc2;
    double qx, qy, qz;
    // the copies' records of this system, indexed by rank (a uniform offset)
    const int64_t rows_off = sy.slice0 * C - sy.atom0;
    const double2* __restrict__ xys = a.xy + rows_off;
    const double* __restrict__ zzs = a.zz + rows_off;
    const uint4* __restrict__ q32s = a.q32 + rows_off;
    if constexpr (PREC == LJ_FP64) {
        const double2 q = xys[ri];
        qx = q.x;
        qy = q.y;
        qz = zzs[ri];
    } else {
        gather_q<LAYOUT>(a.pos, a.n, a.qshift, i, qx, qy, qz);
    }

    const char* colbase = reinterpret_cast<const char*>(
        a.col + sy.col0 + (int64_t)(slice - sy.slice0) * (sy.cap / G) * LJ_WAVE);
    const uint32_t lane_off = (uint32_t)lane * 16u;
    double fx = 0.0, fy = 0.0, fz = 0.0, sA = 0.0, sB = 0.0, sR = 0.0;
    int cnt = 0;       // the lane's pairs outside the loop (the mixed kernels' band pass)
    int wcnt = 0;      // the wavefront's pairs in the loop (wave-uniform)

    // The lane's indices of steps 4 q .. 4 q + 3: one 16-byte load from the
    // slice's group q, clamped into the slice so that every index load is
    // unconditional (no branch for the compiler to wait behind).
    constexpr int NQ = U / 4;                 // groups of 4 steps per batch
    const int lastq = iters > 0 ? (iters - 1) >> 2 : 0;
    auto group_at = [&](int q) -> v4i {
        const int k = q < lastq ? q : lastq;
        return __builtin_nontemporal_load(
            reinterpret_cast<const v4i*>(colbase + (uint32_t)(k * LJ_WAVE * 16) + lane_off));
    };
    // the lane's index of step `it` alone (the rare exact pass of the mixed kernel)
    auto idx_at = [&](int it) -> int {
        return *reinterpret_cast<const int*>(colbase + (uint32_t)((it >> 2) * LJ_WAVE * 16) +
                                             lane_off + (uint32_t)(it & 3) * 4u);
    };
    // the force constants as values, read once
    const double sig2 = fc.sig2, c24 = fc.c24, c48 = fc.c48;
    const float sig2f = fc.sig2f, c24f = fc.c24f, c48f = fc.c48f;
    const double fcut = fc.fcut;
    const float fcutf = fc.fcutf;
    const double qs0 = fc.qs[0], qs1 = fc.qs[1], qs2 = fc.qs[2];
    const double rc2lo = fc.rc2lo, rc2hi = fc.rc2hi;
    // mixed: the row atom's fixed-point record; whether the lane met an entry
    // whose r^2 lies in the quantisation band of rc^2 (decided after the loop)
    uint4 qi4 = make_uint4(0u, 0u, 0u, 0u);
    if constexpr (PREC != LJ_FP64) qi4 = q32s[ri];
    bool had_amb = false;
    // FP64: the terms in powers of 1/r^2, sigma^6 and sigma^12 folded into
    // the constants: fs = (1/r^8) (48 eps sigma^12 / r^6 - 24 eps sigma^6),
    // and the energy sums over 1/r^6 and 1/r^12 scaled after the loop
    const double sig6 = sig2 * sig2 * sig2;
    const double sig12 = sig6 * sig6;
    const double k48 = c48 * sig12, k24 = c24 * sig6;
    // pair terms of an interacting entry from its r^2 (mixed: FP32 terms);
    // sr6d: the term whose sum and sum of squares give the energy and virial
    // (FP64: 1/r^6, mixed: (sigma/r)^6, zero if masked); rr: the pair's
    // distance r for the force-shifted energy (0 if masked)
    auto pair_terms = [&](double r2, bool m, double& fs, double& sr6d, double& rr) {
        if constexpr (PREC == LJ_FP64) {
            double ir2, rd = 0.0;
            if constexpr (FS) {
                // 1/r from v_rsq_f64 and one Newton step, then r and 1/r^2
                // from it (measured on gfx950 over r^2 in [0.25, 35]: within
                // 4.2e-15 and 8.4e-15 of the correctly rounded values; the
                // library square root would cost some 20 instructions more)
                const double y = __builtin_amdgcn_rsq(r2);
                const double ri = fma(0.5 * y, fma(-r2 * y, y, 1.0), y);
                ir2 = keep_or_tiny(m, ri * ri);
                rd = m ? r2 * ri : 0.0;
            } else {
                ir2 = keep_or_tiny(m, recip(r2));
            }
            const double ir4 = ir2 * ir2;
            const double ir6 = ir4 * ir2;
            const double ir8 = ir4 * ir4;
            fs = ir8 * fma(k48, ir6, -k24);
            sr6d = ir6;
            if constexpr (FS) {
                fs = fma(-fcut * rd, ir2, fs);     // fs - Fc / r
                rr = rd;
            }
        } else {
            const float ir2 = m ? __builtin_amdgcn_rcpf((float)r2) : 0.0f;
            const float sr2 = sig2f * ir2;
            const float sr6 = sr2 * sr2 * sr2;
            float fsf = ir2 * (sr6 * fmaf(c48f, sr6, -c24f));
            if constexpr (FS) {
                const float rf = m ? __builtin_amdgcn_sqrtf((float)r2) : 0.0f;
                fsf = fmaf(-fcutf * rf, ir2, fsf);
                rr = (double)rf;
            }
            fs = (double)fsf;
            sr6d = (double)sr6;
        }
    };
    // half lists: the j share of a pair (rank j) goes to the block's window in
    // LDS when j's chunk is in it, else straight to the accumulator
    const int hnch = (int)((sy.n + LJ_HWIN_CHUNK - 1) >> LJ_HWIN_SHIFT);
    // (the window slot of rank j, or -1: looked up as soon as j is known, so
    // that the LDS read overlaps the pair arithmetic)
    auto j_slot = [&](int j) -> int {
        const int ti = lj_hwin_offset(j - (int)sy.atom0, hc0, hnch) + LJ_HWIN_TABLE / 2;
        return (ti >= 0 && ti < LJ_HWIN_TABLE) ? (int)htab[ti] : -1;
    };
    auto j_put = [&](int j, int slot, double x, double y, double z) {
        const int rel = j - (int)sy.atom0;
        if (slot >= 0) {
            // (workgroup scope: LDS atomics, kept apart from the global ones)
            double* p = hacc + slot * LJ_HWIN_CHUNK + (rel & (LJ_HWIN_CHUNK - 1));
            __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(p + LJ_HWIN_MAX * LJ_HWIN_CHUNK, y, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(p + 2 * LJ_HWIN_MAX * LJ_HWIN_CHUNK, z, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            acc_add(a.acc, a.n16, j, x, y, z);
        }
    };
    auto j_add = [&](int j, double x, double y, double z) { j_put(j, j_slot(j), x, y, z); };
    auto fixed_disp = [&](const uint4& qj, double& tx, double& ty, double& tz) {
        // nearest-image displacement from the wrapping fixed-point
        // difference: an exact integer times an exact unit, one rounding
        tx = (double)(int32_t)(qj.x - qi4.x) * qs0;
        ty = (double)(int32_t)(qj.y - qi4.y) * qs1;
        tz = (double)(int32_t)(qj.z - qi4.z) * qs2;
    };
    // The nearest-image correction is needed only by slices whose rows reach
    // across a periodic face (the list build records which): the others run
    // the loop without it.
    const bool img =
        PREC == LJ_FP64 && __builtin_amdgcn_readfirstlane(a.slice_stats[slice].w) != 0;
    auto run = [&](auto img_c) {
        constexpr bool IMG = decltype(img_c)::value;
        // Index groups in two sets used alternately (even and odd batches): a
        // batch's set is refilled with the indices two batches ahead as soon as
        // its gathers are issued (the list streams from HBM), and no register
        // copies make the refill wait.
        v4i ja[NQ], jb[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            ja[q] = group_at(q);
            jb[q] = group_at(NQ + q);
        }
        // one batch of U entries starting at step it0, its indices in jq
        auto batch = [&](v4i* jq, int it0) {
            // a batch's loads stay in their place (not hoisted into the previous
            // batch's arithmetic, which would hold more registers and order its
            // gathers behind the index refill)
            __builtin_amdgcn_sched_barrier(0);
            double px[U], py[U], pz[U];
            uint4 qv[U];
            int jn[U];
#pragma unroll
            for (int u = 0; u < U; ++u) jn[u] = jq[u >> 2][u & 3];
            if constexpr (PREC == LJ_FP64) {
                // the (x, y) record and z of each entry: 24 bytes over 16- and
                // 8-byte records (the 8 entries a row takes per step span about
                // half the cache lines of 32-byte records)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double2 q = *reinterpret_cast<const double2*>(
                        reinterpret_cast<const char*>(xys) + (uint32_t)jn[u] * 16u);
                    px[u] = q.x;
                    py[u] = q.y;
                    pz[u] = *reinterpret_cast<const double*>(
                        reinterpret_cast<const char*>(zzs) + (uint32_t)jn[u] * 8u);
                }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) qv[u] = q32s[jn[u]];
            }
            int jc[U], js[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                jc[u] = jn[u];
                if constexpr (HALF) js[u] = j_slot(jn[u]);
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) jq[q] = group_at((it0 + 2 * U) / 4 + q);
            // keep the next indices' loads issued here, ahead of the arithmetic
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // (a step at or past iters is past every row's length as well)
                const bool valid = (it0 + u) * G < lim;
                double tx, ty, tz, fs, sr6d, rr = 0.0;
                bool in, m;
                if constexpr (PREC == LJ_FP64) {
                    tx = px[u] - qx;
                    ty = py[u] - qy;
                    tz = pz[u] - qz;
                    if constexpr (IMG) {
                        tx = fma(-rint(tx * ibx), bx, tx);
                        ty = fma(-rint(ty * iby), by, ty);
                        tz = fma(-rint(tz * ibz), bz, tz);
                    }
                    const double r2 = r2_rounded(tx, ty, tz);
                    in = r2 < rc2;
                    m = valid && in;
                    pair_terms(r2, m, fs, sr6d, rr);
                } else {
                    fixed_disp(qv[u], tx, ty, tz);
                    const double r2 = r2_rounded(tx, ty, tz);
                    in = r2 < rc2lo;
                    m = valid && in;
                    had_amb = had_amb || (valid && !(r2 < rc2lo) && (r2 < rc2hi));
                    pair_terms(r2, m, fs, sr6d, rr);
                }
                // energy and virial from two sums: sum (sigma/r)^12 and sum (sigma/r)^6
                // (and sum r for the force-shifted truncation)
                sA = fma(sr6d, sr6d, sA);
                sB += sr6d;
                if constexpr (FS) sR += rr;
                // (two ballots of plain compares: lane masks the compares already wrote)
                wcnt += __builtin_popcountll(__builtin_amdgcn_ballot_w64(in) &
                                             __builtin_amdgcn_ballot_w64(valid));
                fx = fma(-fs, tx, fx);
                fy = fma(-fs, ty, fy);
                fz = fma(-fs, tz, fz);
                if constexpr (HALF) {
                    if (m) j_put(jc[u], js[u], fs * tx, fs * ty, fs * tz);
                }
            }
        };
        // whole pairs of batches, then an odd last batch: the loop's back edge
        // always comes from the second batch, so its head waits only for the
        // first set's indices (requested two batches earlier)
        const int nbatch = (iters + U - 1) / U;
        int it0 = 0;
        for (int p = 0; p < (nbatch >> 1); ++p, it0 += 2 * U) {
            batch(ja, it0);
            batch(jb, it0 + U);
        }
        if (nbatch & 1) batch(ja, it0);
    };
    // (the mixed kernels' fixed-point differences wrap by themselves)
    if constexpr (PREC == LJ_FP64) {
        if (img)
            run(std::true_type());
        else
            run(std::false_type());
    } else {
        run(std::false_type());
    }
    if constexpr (PREC != LJ_FP64) {
        // rare: entries whose fixed-point r^2 fell within the band around rc^2,
        // decided on the unquantised positions as in the FP64 kernel
        if (__builtin_amdgcn_ballot_w64(had_amb) != 0 && had_amb) {
            for (int it = 0; it < iters && it * G < lim; ++it) {
                const int j = idx_at(it);
                double tx, ty, tz;
                fixed_disp(q32s[j], tx, ty, tz);
                const double r2 = r2_rounded(tx, ty, tz);
                if (r2 < rc2lo || !(r2 < rc2hi)) continue;
                // the atom of rank j: the row of that rank
                const int aj = a.row_atom[sy.slice0 * C + (j - sy.atom0)];
                double ex, ey, ez;
                gather_q<LAYOUT>(a.pos, a.n, a.qshift, aj, ex, ey, ez);
                ex = ex - qx;
                ey = ey - qy;
                ez = ez - qz;
                ex = fma(-rint(ex * ibx), bx, ex);
                ey = fma(-rint(ey * iby), by, ey);
                ez = fma(-rint(ez * ibz), bz, ez);
                if (!(r2_rounded(ex, ey, ez) < rc2)) continue;
                double fs, sr6d, rr = 0.0;
                pair_terms(r2, true, fs, sr6d, rr);
                sA = fma(sr6d, sr6d, sA);
                sB += sr6d;
                if constexpr (FS) sR += rr;
                cnt += 1;
                fx = fma(-fs, tx, fx);
                fy = fma(-fs, ty, fy);
                fz = fma(-fs, tz, fz);
                if (HALF) j_add(j, fs * tx, fs * ty, fs * tz);
            }
        }
    }
    // sum the row over its G lanes
#pragma unroll
    for (int d = G / 2; d >= 1; d >>= 1) {
        fx += __shfl_xor(fx, d, LJ_WAVE);
        fy += __shfl_xor(fy, d, LJ_WAVE);
        fz += __shfl_xor(fz, d, LJ_WAVE);
    }
    double ke = 0.0;
    if (g == 0 && row_ok) {
        if (HALF) {
            j_add(ri, fx, fy, fz);
        } else if (a.kick == LJ_KICK_NONE) {
            store_f<LAYOUT>(a.force, a.n, i, fx, fy, fz);
        } else {
            ke = kick_row<LAYOUT>(a, i, fx, fy, fz);
            if (a.write_f) store_f<LAYOUT>(a.force, a.n, i, fx, fy, fz);
        }
    }
    // per lane: 4 eps (A - B) [+ Fc sum r] and 24 eps (2A - B) [- Fc sum r],
    // A and B the sums of (sigma/r)^12 and (sigma/r)^6
    if constexpr (PREC == LJ_FP64) {
        sA *= sig12;
        sB *= sig6;
    }
    e_out = fc.c4 * (sA - sB);
    w_out = fc.c24 * (2.0 * sA - sB);
    if constexpr (FS) {
        e_out = fma(fcut, sR, e_out);
        w_out = fma(-fcut, sR, w_out);
    }
    c_out = (double)(cnt + (lane == 0 ? wcnt : 0));
    k_out = ke;
}

}  // namespace ljf
