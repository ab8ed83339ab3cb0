// lj_force.hip -- LJ forces, energy and virial over the wavefront-sliced
// Verlet list (Alg. 1 inside the sorted-list loop of Alg. 3).
//
// One wavefront serves one slice: C = 64 / G rows, G lanes per row.  As in
// Alg. 3 the i atom's position and force stay in registers for the whole row;
// each lane walks every G-th entry of its row:
//   j      = col[slot]                 one coalesced 256-byte load per wavefront
//   q_j    = pos[j]                    gather (double4: one 32-byte record)
//   t      = q_j - q_i, nearest image  t -= L * rint(t / L)
//   r^2    = (tx*tx + ty*ty) + tz*tz   rounded as in the list build, so the
//                                      cutoff test selects exactly the pairs
//                                      r^2 < rc^2 of the definition
//   mask   = entry inside the row  and  r^2 < rc^2   (the masks of Fig. 8 and
//            of the remainder-loop elimination of Alg. 4: no remainder loop)
//   fs     = 24 eps (sigma/r)^6 [2 (sigma/r)^6 - 1] / r^2 (0 where masked)
//   F_i   -= fs t;  half list: F_j += fs t by atomic add (Newton's third law)
//   A     += (sigma/r)^12, B += (sigma/r)^6, count += mask, so that
//            E = 4 eps (A - B) - count V(rc) and W = sum fs r^2 = 24 eps (2A - B)
// Mixed precision (LJ_MIXED) gathers 16-byte fixed-point records instead
// (k_quantize writes them): t is the wrapping integer difference times the
// unit L / 2^32, r^2 stays FP64, and the few entries whose r^2 falls within
// the quantisation band around rc^2 are decided on the FP64 positions after
// the main loop; the pair terms are FP32.
// The row's force is summed over its G lanes with cross-lane shuffles.
// Energy, virial and the pair count are summed per block in a fixed order,
// and one block per system sums the block partials in a fixed order (in two
// levels when a system has more than 4096 blocks) and writes
// E = scale * (sum - count * V(rc)), W = scale * sum, count * scale, with
// scale = 1/2 for a full list (every pair is visited twice).
#include <math.h>

#include <algorithm>

#include "lj_internal.h"

namespace {

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
    const int32_t* col;
    double* partials;        // 4 doubles per (logical) block
    double* acc;             // half list: spread force accumulator (3 x 16 n16 doubles)
    int64_t n16;
    uint4* q32;              // mixed: fixed-point positions (x, y, z as fractions of the box)
};

__device__ __forceinline__ double r2_rounded(double x, double y, double z) {
#pragma clang fp contract(off)
    return (x * x + y * y) + z * z;
}

template <int LAYOUT>
__device__ __forceinline__ void load_q(const double* __restrict__ pos, int64_t n, int64_t i,
                                       double& x, double& y, double& z) {
    if (LAYOUT == LJ_AOS4) {
        const double4 q = reinterpret_cast<const double4*>(pos)[i];
        x = q.x;
        y = q.y;
        z = q.z;
    } else {
        x = pos[i];
        y = pos[n + i];
        z = pos[2 * n + i];
    }
}

template <int LAYOUT>
__device__ __forceinline__ void add_f(double* __restrict__ f, int64_t n, int64_t i, double x,
                                      double y, double z) {
    if (LAYOUT == LJ_AOS4) {
        unsafeAtomicAdd(f + 4 * i + 0, x);
        unsafeAtomicAdd(f + 4 * i + 1, y);
        unsafeAtomicAdd(f + 4 * i + 2, z);
    } else {
        unsafeAtomicAdd(f + i, x);
        unsafeAtomicAdd(f + n + i, y);
        unsafeAtomicAdd(f + 2 * n + i, z);
    }
}

// Half list: the Newton's-third-law scatter goes into an accumulator with
// one block per component, so that the three atomics of a pair do not queue
// on one cache line.
__device__ __forceinline__ int64_t spread_at(int64_t i, int64_t n16) { return i; }
__device__ __forceinline__ void acc_add(double* __restrict__ acc, int64_t n16, int64_t i,
                                        double x, double y, double z) {
    const int64_t s = spread_at(i, n16);
    unsafeAtomicAdd(acc + s, x);
    unsafeAtomicAdd(acc + 16 * n16 + s, y);
    unsafeAtomicAdd(acc + 32 * n16 + s, z);
}

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

// Block partials (E, W, count) -> partials[4 * block], summed in a fixed
// order.  No atomics: a device-scope atomic must stay coherent across the
// eight per-XCD L2 caches and is resolved beyond them, so thousands of blocks
// hitting one counter serialise.
__device__ void block_partials(const ForceArgs& a, int64_t blk, double e, double w, double cnt) {
    __shared__ double red[LJ_WAVES_PER_BLOCK][3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    e = wave_sum(e);
    w = wave_sum(w);
    cnt = wave_sum(cnt);
    if (lane == 0) {
        red[wave][0] = e;
        red[wave][1] = w;
        red[wave][2] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double be = 0.0, bw = 0.0, bc = 0.0;
        for (int k = 0; k < LJ_WAVES_PER_BLOCK; ++k) {
            be += red[k][0];
            bw += red[k][1];
            bc += red[k][2];
        }
        double* p = a.partials + 4 * blk;
        p[0] = be;
        p[1] = bw;
        p[2] = bc;
    }
}

// Fixed-order block sum of partial records [b0, b1): thread t adds records
// t, t + 1024, ... (four loads in flight per pass), then the waves' sums are
// added in wave order.  The result is valid in thread 0.
__device__ double3 span_sum(const double4* __restrict__ p, int64_t b0, int64_t b1) {
    __shared__ double red[16][3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double se = 0.0, sw = 0.0, sc = 0.0;
    for (int64_t bb = b0 + threadIdx.x; bb < b1; bb += 4 * 1024) {
        double4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t b = bb + u * 1024;
            v[u] = b < b1 ? p[b] : make_double4(0.0, 0.0, 0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            se += v[u].x;
            sw += v[u].y;
            sc += v[u].z;
        }
    }
    se = wave_sum(se);
    sw = wave_sum(sw);
    sc = wave_sum(sc);
    if (lane == 0) {
        red[wave][0] = se;
        red[wave][1] = sw;
        red[wave][2] = sc;
    }
    __syncthreads();
    double3 t = make_double3(0.0, 0.0, 0.0);
    if (threadIdx.x == 0) {
        for (int k = 0; k < 16; ++k) {
            t.x += red[k][0];
            t.y += red[k][1];
            t.z += red[k][2];
        }
    }
    return t;
}

// First level for systems with many blocks: block (s, k), k < split, sums
// the k-th of split equal contiguous spans of system s's block partials.
__global__ __launch_bounds__(1024) void k_force_reduce_split(const double4* __restrict__ partials,
                                                             const lj_sys* sys, int split,
                                                             double4* __restrict__ out) {
    const int s = blockIdx.x / split, k = blockIdx.x % split;
    const lj_sys& sy = sys[s];
    const int64_t b0 = sy.slice0 / LJ_WAVES_PER_BLOCK;
    const int64_t b1 = (sy.slice0 + sy.nslices) / LJ_WAVES_PER_BLOCK;
    const int64_t span = (b1 - b0 + split - 1) / split;
    const int64_t lo = b0 + k * span < b1 ? b0 + k * span : b1;
    const int64_t hi = lo + span < b1 ? lo + span : b1;
    const double3 t = span_sum(partials, lo, hi);
    if (threadIdx.x == 0) out[blockIdx.x] = make_double4(t.x, t.y, t.z, 0.0);
}

// One block per system: the fixed-order sum of its block partials (split = 1)
// or of its split first-level sums; writes the system's energy, virial and
// pair count.
__global__ __launch_bounds__(1024) void k_force_reduce(const double4* __restrict__ partials,
                                                       const lj_sys* sys, int split,
                                                       const lj_fconst* fc, double scale,
                                                       double* energy, double* virial,
                                                       int64_t* npairs) {
    const int s = blockIdx.x;
    const lj_sys& sy = sys[s];
    int64_t b0 = (int64_t)s * split, b1 = b0 + split;
    if (split == 1) {
        b0 = sy.slice0 / LJ_WAVES_PER_BLOCK;
        b1 = (sy.slice0 + sy.nslices) / LJ_WAVES_PER_BLOCK;
    }
    const double3 t = span_sum(partials, b0, b1);
    if (threadIdx.x == 0) {
        energy[s] = scale * (t.x - t.z * fc[s].vc);
        virial[s] = scale * t.y;
        if (npairs) npairs[s] = (int64_t)(scale * t.z + 0.5);
    }
}

// 1/x as v_rcp_f64 refined by two Newton steps y <- y (2 - x y) (each step
// squares the relative error, which v_rcp_f64 already bounds far below 2^-20).
__device__ __forceinline__ double recip(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

template <int LAYOUT>
__device__ __forceinline__ void gather_q(const double* __restrict__ pos, int64_t n, int j,
                                         double& x, double& y, double& z) {
    if (LAYOUT == LJ_AOS4) {
        // 32-bit byte offset from a uniform base: one dwordx4 + one dwordx2 load
        const double4* q = reinterpret_cast<const double4*>(
            reinterpret_cast<const char*>(pos) + (uint32_t)j * 32u);
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

// Mixed precision: each coordinate as a 32-bit fraction of its box length,
// u = rint(x 2^32 / L) mod 2^32.  A wrapping 32-bit difference u_j - u_i is
// then the nearest-image displacement in units of L / 2^32 (1.2e-8 at
// L = 50.8), exact up to the two roundings of u: one 16-byte record per
// entry instead of 32, and no image arithmetic.  r^2 is formed in FP64 from
// it; the pair terms are FP32.  One thread per row of the
// list; the thread of a system's k-th row converts its k-th atom.
template <int LAYOUT>
__global__ __launch_bounds__(LJ_BLOCK) void k_quantize(const double* __restrict__ pos, int64_t n,
                                                       const lj_sys* sys,
                                                       const int32_t* slice_sys, int C,
                                                       const lj_fconst* fc,
                                                       uint4* __restrict__ q32) {
    const int64_t r = blockIdx.x * (int64_t)LJ_BLOCK + threadIdx.x;
    const int sid = __builtin_amdgcn_readfirstlane(
        slice_sys[(blockIdx.x * (int64_t)LJ_BLOCK) / C]);
    const lj_sys& sy = sys[sid];
    const int64_t t = r - sy.slice0 * C;
    if (t >= sy.n) return;
    const int64_t i = sy.atom0 + t;
    double x, y, z;
    if (LAYOUT == LJ_AOS4) {
        const double4 q = reinterpret_cast<const double4*>(pos)[i];
        x = q.x;
        y = q.y;
        z = q.z;
    } else {
        x = pos[i];
        y = pos[n + i];
        z = pos[2 * n + i];
    }
    const lj_fconst& f = fc[sid];
    q32[i] = make_uint4(lj_fix32(x, f.qinv[0]), lj_fix32(y, f.qinv[1]), lj_fix32(z, f.qinv[2]), 0u);
}

// Loads are issued U entries at a time, and the indices of the next U
// entries are requested before the current ones are computed, so each
// wavefront keeps up to 3U gathers and U index loads in flight (the
// load/compute overlap that software pipelining gives a CPU core).
template <int G, bool HALF, int LAYOUT, int PREC, int U>
__global__ __launch_bounds__(LJ_BLOCK) void k_force(ForceArgs a) {
    constexpr int C = LJ_WAVE / G;
    const int lane = threadIdx.x & (LJ_WAVE - 1);
    const int64_t blk = lj_xcd_block(blockIdx.x, gridDim.x);
    const int slice = __builtin_amdgcn_readfirstlane(
        (int)blk * LJ_WAVES_PER_BLOCK + (threadIdx.x >> 6));
    // a block's four slices belong to one system (systems own whole 256-row blocks)
    const int sid = __builtin_amdgcn_readfirstlane(a.slice_sys[blk * LJ_WAVES_PER_BLOCK]);
    const lj_sys& sy = a.sys[sid];
    const lj_fconst& fc = a.fc[sid];
    const int iters = __builtin_amdgcn_readfirstlane(a.slice_iters[slice]);
    const int c = lane / G, g = lane % G;
    const int64_t r = (int64_t)slice * C + c;
    const int i = a.row_atom[r];
    const int lim = a.row_len[r] - g;   // entry it*G + g is inside the row iff it*G < lim
    const bool row_ok = (r - sy.slice0 * C) < sy.n;
    const double bx = sy.box[0], by = sy.box[1], bz = sy.box[2];
    const double ibx = sy.inv_box[0], iby = sy.inv_box[1], ibz = sy.inv_box[2];
    const double rc2 = fc.rc2;
    double qx, qy, qz;
    gather_q<LAYOUT>(a.pos, a.n, i, qx, qy, qz);

    const char* colbase = reinterpret_cast<const char*>(
        a.col + sy.col0 + (int64_t)(slice - sy.slice0) * (sy.cap / G) * LJ_WAVE);
    const uint32_t lane_off = (uint32_t)lane * 4u;
    double fx = 0.0, fy = 0.0, fz = 0.0, sA = 0.0, sB = 0.0;
    int cnt = 0;

    // slot of step `it`, clamped into the slice so that every index load is
    // unconditional (no branch for the compiler to wait behind)
    const int last = iters > 0 ? iters - 1 : 0;
    auto idx_at = [&](int it) -> int {
        const int k = it < last ? it : last;
        return __builtin_nontemporal_load(
            reinterpret_cast<const int*>(colbase + (uint32_t)(k * LJ_WAVE * 4) + lane_off));
    };
    int jn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) jn[u] = idx_at(u);
    // the force constants as values, read once
    const double sig2 = fc.sig2, c24 = fc.c24, c48 = fc.c48;
    const float sig2f = fc.sig2f, c24f = fc.c24f, c48f = fc.c48f;
    const double qs0 = fc.qs[0], qs1 = fc.qs[1], qs2 = fc.qs[2];
    const double rc2lo = fc.rc2lo, rc2hi = fc.rc2hi;
    // mixed: the row atom's fixed-point record; whether the lane met an entry
    // whose r^2 lies in the quantisation band of rc^2 (decided after the loop)
    uint4 qi4 = make_uint4(0u, 0u, 0u, 0u);
    if constexpr (PREC != LJ_FP64) qi4 = a.q32[i];
    bool had_amb = false;
    // pair terms of an interacting entry from its r^2 (mixed: FP32 terms)
    auto pair_terms = [&](double r2, bool m, double& fs, double& sr6d) {
        if constexpr (PREC == LJ_FP64) {
            const double ir2 = m ? recip(r2) : 0.0;
            const double sr2 = sig2 * ir2;
            const double sr6 = sr2 * sr2 * sr2;
            fs = ir2 * (sr6 * fma(c48, sr6, -c24));
            sr6d = sr6;
        } else {
            const float ir2 = m ? __builtin_amdgcn_rcpf((float)r2) : 0.0f;
            const float sr2 = sig2f * ir2;
            const float sr6 = sr2 * sr2 * sr2;
            fs = (double)(ir2 * (sr6 * fmaf(c48f, sr6, -c24f)));
            sr6d = (double)sr6;
        }
    };
    auto fixed_disp = [&](const uint4& qj, double& tx, double& ty, double& tz) {
        // nearest-image displacement from the wrapping fixed-point
        // difference: an exact integer times an exact unit, one rounding
        tx = (double)(int32_t)(qj.x - qi4.x) * qs0;
        ty = (double)(int32_t)(qj.y - qi4.y) * qs1;
        tz = (double)(int32_t)(qj.z - qi4.z) * qs2;
    };
    for (int it0 = 0; it0 < iters; it0 += U) {
        double px[U], py[U], pz[U];
        uint4 qv[U];
        if constexpr (PREC == LJ_FP64) {
#pragma unroll
            for (int u = 0; u < U; ++u) gather_q<LAYOUT>(a.pos, a.n, jn[u], px[u], py[u], pz[u]);
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) qv[u] = a.q32[jn[u]];
        }
        int jc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) jc[u] = jn[u];
#pragma unroll
        for (int u = 0; u < U; ++u) jn[u] = idx_at(it0 + U + u);
        // keep the next indices' loads issued here, ahead of the arithmetic
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool valid = (it0 + u < iters) && ((it0 + u) * G < lim);
            double tx, ty, tz, fs, sr6d;
            bool m;
            if constexpr (PREC == LJ_FP64) {
                tx = px[u] - qx;
                ty = py[u] - qy;
                tz = pz[u] - qz;
                tx = fma(-rint(tx * ibx), bx, tx);
                ty = fma(-rint(ty * iby), by, ty);
                tz = fma(-rint(tz * ibz), bz, tz);
                const double r2 = r2_rounded(tx, ty, tz);
                m = valid && (r2 < rc2);
                pair_terms(r2, m, fs, sr6d);
            } else {
                fixed_disp(qv[u], tx, ty, tz);
                const double r2 = r2_rounded(tx, ty, tz);
                m = valid && (r2 < rc2lo);
                had_amb = had_amb || (valid && !(r2 < rc2lo) && (r2 < rc2hi));
                pair_terms(r2, m, fs, sr6d);
            }
            // energy and virial from two sums: sum (sigma/r)^12 and sum (sigma/r)^6
            sA = fma(sr6d, sr6d, sA);
            sB += sr6d;
            cnt += m ? 1 : 0;
            fx = fma(-fs, tx, fx);
            fy = fma(-fs, ty, fy);
            fz = fma(-fs, tz, fz);
            if (HALF && m) acc_add(a.acc, a.n16, jc[u], fs * tx, fs * ty, fs * tz);
        }
    }
    if constexpr (PREC != LJ_FP64) {
        // rare: entries whose fixed-point r^2 fell within the band around rc^2,
        // decided on the unquantised positions as in the FP64 kernel
        if (__builtin_amdgcn_ballot_w64(had_amb) != 0 && had_amb) {
            for (int it = 0; it < iters && it * G < lim; ++it) {
                const int j = idx_at(it);
                double tx, ty, tz;
                fixed_disp(a.q32[j], tx, ty, tz);
                const double r2 = r2_rounded(tx, ty, tz);
                if (r2 < rc2lo || !(r2 < rc2hi)) continue;
                double ex, ey, ez;
                gather_q<LAYOUT>(a.pos, a.n, j, ex, ey, ez);
                ex = ex - qx;
                ey = ey - qy;
                ez = ez - qz;
                ex = fma(-rint(ex * ibx), bx, ex);
                ey = fma(-rint(ey * iby), by, ey);
                ez = fma(-rint(ez * ibz), bz, ez);
                if (!(r2_rounded(ex, ey, ez) < rc2)) continue;
                double fs, sr6d;
                pair_terms(r2, true, fs, sr6d);
                sA = fma(sr6d, sr6d, sA);
                sB += sr6d;
                cnt += 1;
                fx = fma(-fs, tx, fx);
                fy = fma(-fs, ty, fy);
                fz = fma(-fs, tz, fz);
                if (HALF) acc_add(a.acc, a.n16, j, fs * tx, fs * ty, fs * tz);
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
    if (g == 0 && row_ok) {
        if (HALF)
            acc_add(a.acc, a.n16, i, fx, fy, fz);
        else
            store_f<LAYOUT>(a.force, a.n, i, fx, fy, fz);
    }
    // per lane: 4 eps (A - B) and 24 eps (2A - B)
    block_partials(a, blk, fc.c4 * (sA - sB), fc.c24 * (2.0 * sA - sB), (double)cnt);
}

// Half list: the forces from the spread accumulator, which is cleared for
// the next evaluation.
template <int LAYOUT>
__global__ __launch_bounds__(LJ_BLOCK) void k_acc_out(double* __restrict__ acc, int64_t n16,
                                                      int64_t n, double* __restrict__ f) {
    const int64_t i = blockIdx.x * (int64_t)LJ_BLOCK + threadIdx.x;
    if (i >= n) return;
    const int64_t s = spread_at(i, n16);
    const double x = acc[s], y = acc[16 * n16 + s], z = acc[32 * n16 + s];
    acc[s] = 0.0;
    acc[16 * n16 + s] = 0.0;
    acc[32 * n16 + s] = 0.0;
    store_f<LAYOUT>(f, n, i, x, y, z);
}

template <int G, int U>
lj_status launch_g(lj_ctx* ctx, const ForceArgs& a, bool half, int layout, int prec,
                   int64_t blocks) {
    dim3 grid((unsigned)blocks), block(LJ_BLOCK);
    hipStream_t s = ctx->stream;
#define LJ_K(H, L, P) hipLaunchKernelGGL((k_force<G, H, L, P, U>), grid, block, 0, s, a)
    if (half) {
        if (layout == LJ_AOS4) {
            if (prec == LJ_FP64) LJ_K(true, LJ_AOS4, LJ_FP64); else LJ_K(true, LJ_AOS4, LJ_MIXED);
        } else {
            if (prec == LJ_FP64) LJ_K(true, LJ_SOA, LJ_FP64); else LJ_K(true, LJ_SOA, LJ_MIXED);
        }
    } else {
        if (layout == LJ_AOS4) {
            if (prec == LJ_FP64) LJ_K(false, LJ_AOS4, LJ_FP64); else LJ_K(false, LJ_AOS4, LJ_MIXED);
        } else {
            if (prec == LJ_FP64) LJ_K(false, LJ_SOA, LJ_FP64); else LJ_K(false, LJ_SOA, LJ_MIXED);
        }
    }
#undef LJ_K
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}

}  // namespace

int64_t lj_force_blocks(int64_t nslices) {
    return (nslices + LJ_WAVES_PER_BLOCK - 1) / LJ_WAVES_PER_BLOCK;
}

// One 1024-thread block reads at most this many block partials of a system
// per reduction level: a single block streams only about 0.1 TB/s, so a
// 4M-atom system's 125k partials take two levels.
static const int64_t kReduceSpan = 4096;

int lj_force_split(const lj_list* l) {
    int64_t most = 0;
    for (const lj_sys& sy : l->hsys) most = std::max(most, sy.nslices / LJ_WAVES_PER_BLOCK);
    return (int)std::max<int64_t>(1, (most + kReduceSpan - 1) / kReduceSpan);
}

int64_t lj_force_partials(const lj_list* l) {
    const int split = lj_force_split(l);
    return lj_force_blocks(l->nslices) + (split > 1 ? (int64_t)l->nsys * split : 0);
}

lj_fconst lj_make_fconst(double eps, double sigma, double rc, const double box[3]) {
    lj_fconst f = {};
    f.rc2 = rc * rc;
    f.sig2 = sigma * sigma;
    f.c4 = 4.0 * eps;
    f.c24 = 24.0 * eps;
    f.c48 = 48.0 * eps;
    const double s2 = f.sig2 / f.rc2;
    const double s6 = s2 * s2 * s2;
    f.vc = 4.0 * eps * s6 * (s6 - 1.0);
    f.sig2f = (float)f.sig2;
    f.c4f = (float)f.c4;
    f.c24f = (float)f.c24;
    f.c48f = (float)f.c48;
    // Fixed point for the mixed kernel, and the band around rc^2 in which its
    // r^2 defers to the test on the unquantised positions.  A displacement
    // component from the fixed-point records is off by at most one unit
    // s = L / 2^32 (two roundings of half a unit; the product by the exact
    // unit adds one FP64 rounding): e <= 1.0001 s.  Its r^2 then differs from
    // that of the unquantised positions by at most 2 sqrt(3) r e + 3 e^2 for r
    // up to 1.001 rc (beyond that both tests reject); the band is twice that
    // bound plus a margin for the FP64 roundings of either r^2.
    const double two32 = 4294967296.0;
    double smax = 0.0;
    for (int d = 0; d < 3; ++d) {
        f.qinv[d] = two32 / box[d];
        f.qs[d] = box[d] / two32;
        smax = std::max(smax, f.qs[d]);
    }
    const double rx = 1.001 * rc, e = 1.0001 * smax;
    const double band = 2.0 * (2.0 * sqrt(3.0) * rx * e + 3.0 * e * e) + 1e-12 * f.rc2;
    f.rc2lo = f.rc2 - band;
    f.rc2hi = f.rc2 + band;
    return f;
}

lj_status lj_launch_forces(lj_ctx* ctx, const double* pos, int layout, int precision,
                           const lj_list* l, const lj_fconst* fc, double* force, double* energy,
                           double* virial, int64_t* npairs, bool quantized) {
    const int64_t blocks = lj_force_blocks(l->nslices);
    if (lj_force_partials(l) > ctx->partials_cap)
        return lj_fail(LJ_E_INVALID, "context partials too small");
    const bool half = l->kind == LJ_LIST_HALF;
    if (half && !l->acc) return lj_fail(LJ_E_INVALID, "half list without its force accumulator");
    ForceArgs a;
    a.pos = pos;
    a.force = force;
    a.n = l->n;
    a.nslices = l->nslices;
    a.sys = l->dsys;
    a.fc = fc;
    a.slice_sys = l->slice_sys;
    a.row_atom = l->row_atom;
    a.row_len = l->row_len;
    a.slice_iters = l->slice_iters;
    a.col = l->col;
    a.partials = ctx->partials;
    a.acc = l->acc;
    a.q32 = l->q32;
    a.n16 = (l->n + 15) / 16;
    if (precision != LJ_FP64 && !l->q32)
        return lj_fail(LJ_E_INVALID, "mixed precision without the list's fixed-point buffer");
    lj_status st;
    {
        lj_prof_scope prof(ctx, LJ_PROF_FORCE);
        if (precision != LJ_FP64 && !quantized) {
            const dim3 qgrid((unsigned)(l->nslices * (LJ_WAVE / l->lanes) / LJ_BLOCK));
            if (layout == LJ_AOS4)
                hipLaunchKernelGGL(k_quantize<LJ_AOS4>, qgrid, dim3(LJ_BLOCK), 0, ctx->stream,
                                   pos, l->n, (const lj_sys*)l->dsys, (const int32_t*)l->slice_sys,
                                   LJ_WAVE / l->lanes, fc, l->q32);
            else
                hipLaunchKernelGGL(k_quantize<LJ_SOA>, qgrid, dim3(LJ_BLOCK), 0, ctx->stream,
                                   pos, l->n, (const lj_sys*)l->dsys, (const int32_t*)l->slice_sys,
                                   LJ_WAVE / l->lanes, fc, l->q32);
            LJ_HIP(hipGetLastError());
        }
        // entries in flight per lane: tuned value
        const int u = ctx->tune[LJ_TUNE_FORCE_BATCH];
#define LJ_U(G)                                                                      \
    (u == 2 ? launch_g<G, 2>(ctx, a, half, layout, precision, blocks)                \
            : u == 8 ? launch_g<G, 8>(ctx, a, half, layout, precision, blocks)       \
                     : launch_g<G, 4>(ctx, a, half, layout, precision, blocks))
        switch (l->lanes) {
            case 1: st = LJ_U(1); break;
            case 2: st = LJ_U(2); break;
            case 4: st = LJ_U(4); break;
            case 8: st = LJ_U(8); break;
            case 16: st = LJ_U(16); break;
            case 32: st = LJ_U(32); break;
            case 64: st = LJ_U(64); break;
            default: return lj_fail(LJ_E_INVALID, "lanes must be 1, 2, 4, 8, 16, 32 or 64");
        }
#undef LJ_U
    }
    if (st) return st;
    lj_prof_scope prof(ctx, LJ_PROF_OTHER);
    if (half) {
        const dim3 grid((unsigned)((l->n + LJ_BLOCK - 1) / LJ_BLOCK)), block(LJ_BLOCK);
        if (layout == LJ_AOS4)
            hipLaunchKernelGGL(k_acc_out<LJ_AOS4>, grid, block, 0, ctx->stream, l->acc, a.n16,
                               l->n, force);
        else
            hipLaunchKernelGGL(k_acc_out<LJ_SOA>, grid, block, 0, ctx->stream, l->acc, a.n16,
                               l->n, force);
        LJ_HIP(hipGetLastError());
    }
    const int split = lj_force_split(l);
    const double4* first = reinterpret_cast<const double4*>(ctx->partials);
    if (split > 1) {
        double4* second = reinterpret_cast<double4*>(ctx->partials) + blocks;
        hipLaunchKernelGGL(k_force_reduce_split, dim3((unsigned)(l->nsys * split)), dim3(1024), 0,
                           ctx->stream, first, (const lj_sys*)l->dsys, split, second);
        LJ_HIP(hipGetLastError());
        first = second;
    }
    hipLaunchKernelGGL(k_force_reduce, dim3((unsigned)l->nsys), dim3(1024), 0, ctx->stream, first,
                       (const lj_sys*)l->dsys, split, fc, half ? 1.0 : 0.5, energy, virial,
                       npairs);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}
