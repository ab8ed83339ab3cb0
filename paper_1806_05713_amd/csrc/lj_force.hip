// lj_force.hip -- LJ forces, energy and virial over the wavefront-sliced
// Verlet list (Alg. 1 inside the sorted-list loop of Alg. 3).
//
// One wavefront serves one slice: C = 64 / G rows, G lanes per row.  As in
// Alg. 3 the i atom's position and force stay in registers for the whole row;
// each lane walks every G-th entry of its row:
//   j      = col[slot]                 the cell-sorted rank of the neighbour; a
//                                      lane loads its indices of 4 steps at once
//                                      (1 KiB per wavefront)
//   q_j    = xy[j], z[j]               gathers from the positions copied into
//                                      rank order (16 + 8 bytes) before the kernel
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
// (k_gather_copy writes them): t is the wrapping integer difference times the
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
#include <mutex>

#include "lj_force_loop.h"
#include "lj_internal.h"

namespace {

using namespace ljf;

// Block partials (E, W, count, kinetic energy) -> partials[4 * block],
// summed in a fixed order.  No atomics: a device-scope atomic must stay
// coherent across the eight per-XCD L2 caches and is resolved beyond them, so
// thousands of blocks hitting one counter serialise.
__device__ void block_partials(const ForceArgs& a, int64_t blk, double e, double w, double cnt,
                               double ke) {
    __shared__ double red[LJ_WAVES_PER_BLOCK][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    e = wave_sum(e);
    w = wave_sum(w);
    cnt = wave_sum(cnt);
    ke = wave_sum(ke);
    if (lane == 0) {
        red[wave][0] = e;
        red[wave][1] = w;
        red[wave][2] = cnt;
        red[wave][3] = ke;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double be = 0.0, bw = 0.0, bc = 0.0, bk = 0.0;
        for (int k = 0; k < LJ_WAVES_PER_BLOCK; ++k) {
            be += red[k][0];
            bw += red[k][1];
            bc += red[k][2];
            bk += red[k][3];
        }
        reinterpret_cast<double4*>(a.partials)[blk] = make_double4(be, bw, bc, bk);
    }
}

// True once a kernel has raised an error flag on the device (a bad coordinate
// or an overflowing list row): later force, reduction and integrator kernels
// of the stream then leave every output as it was.
__device__ __forceinline__ bool halted(const int32_t* flags) {
    return flags && (__builtin_nontemporal_load(flags) & LJ_DEV_ERRORS) != 0;
}

// Fixed-order block sum of partial records [b0, b1): thread t adds records
// t, t + 1024, ... (four loads in flight per pass), then the waves' sums are
// added in wave order.  The result is valid in thread 0.
__device__ double4 span_sum(const double4* __restrict__ p, int64_t b0, int64_t b1) {
    __shared__ double red[16][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double se = 0.0, sw = 0.0, sc = 0.0, sk = 0.0;
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
            sk += v[u].w;
        }
    }
    se = wave_sum(se);
    sw = wave_sum(sw);
    sc = wave_sum(sc);
    sk = wave_sum(sk);
    if (lane == 0) {
        red[wave][0] = se;
        red[wave][1] = sw;
        red[wave][2] = sc;
        red[wave][3] = sk;
    }
    __syncthreads();
    double4 t = make_double4(0.0, 0.0, 0.0, 0.0);
    if (threadIdx.x == 0) {
        for (int k = 0; k < 16; ++k) {
            t.x += red[k][0];
            t.y += red[k][1];
            t.z += red[k][2];
            t.w += red[k][3];
        }
    }
    return t;
}

// First level for systems with many blocks: block (s, k), k < split, sums
// the k-th of split equal contiguous spans of system s's block partials.
__global__ __launch_bounds__(1024) void k_force_reduce_split(const double4* __restrict__ partials,
                                                             const lj_sys* sys, int split,
                                                             const int32_t* flags,
                                                             double4* __restrict__ out) {
    if (halted(flags)) return;
    const int s = blockIdx.x / split, k = blockIdx.x % split;
    const lj_sys& sy = sys[s];
    const int64_t b0 = sy.slice0 / LJ_WAVES_PER_BLOCK;
    const int64_t b1 = (sy.slice0 + sy.nslices) / LJ_WAVES_PER_BLOCK;
    const int64_t span = (b1 - b0 + split - 1) / split;
    const int64_t lo = b0 + k * span < b1 ? b0 + k * span : b1;
    const int64_t hi = lo + span < b1 ? lo + span : b1;
    const double4 t = span_sum(partials, lo, hi);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// One block per system: the fixed-order sum of its block partials (split = 1)
// or of its split first-level sums; writes the system's energy, virial and
// pair count, and (when `kinetic` is not NULL) the kinetic energy of a
// kicking force pass.
__global__ __launch_bounds__(1024) void k_force_reduce(const double4* __restrict__ partials,
                                                       const lj_sys* sys, int split,
                                                       const lj_fconst* fc, double scale,
                                                       const int32_t* flags, double* energy,
                                                       double* virial, int64_t* npairs,
                                                       double* kinetic) {
    if (halted(flags)) return;
    const int s = blockIdx.x;
    const lj_sys& sy = sys[s];
    int64_t b0 = (int64_t)s * split, b1 = b0 + split;
    if (split == 1) {
        b0 = sy.slice0 / LJ_WAVES_PER_BLOCK;
        b1 = (sy.slice0 + sy.nslices) / LJ_WAVES_PER_BLOCK;
    }
    const double4 t = span_sum(partials, b0, b1);
    if (threadIdx.x == 0) {
        energy[s] = scale * (t.x - t.z * fc[s].vc);
        virial[s] = scale * t.y;
        if (npairs) npairs[s] = (int64_t)(scale * t.z + 0.5);
        if (kinetic) kinetic[s] = t.w;
    }
}

// The copies the force kernel gathers from, one record per row of the list
// (rows are in cell-sorted rank order, so the rows' neighbours sit close
// together in memory whatever the caller's atom order; a system's rank j is
// its row j + slice0 C - atom0, a per-system offset the force kernel adds to
// its base pointers): the thread of row r reads the position of the row's
// atom and writes record r.  Rows past a system's atoms hold atom 0 and are
// never gathered, so every thread stores and none waits for the system's
// descriptor.
//   FP64: (x, y) 16-byte records and z;
//   mixed: each coordinate as a 32-bit fraction of its box length,
//     u = rint(x 2^32 / L) mod 2^32.  A wrapping 32-bit difference u_j - u_i
//     is then the nearest-image displacement in units of L / 2^32 (1.2e-8 at
//     L = 50.8), exact up to the two roundings of u: one 16-byte record per
//     entry instead of 24, and no image arithmetic.  r^2 is formed in FP64
//     from it; the pair terms are FP32.
template <int LAYOUT, int PREC>
__global__ __launch_bounds__(LJ_BLOCK) void k_gather_copy(const double* __restrict__ pos,
                                                          int64_t n, uint32_t qshift,
                                                          const int32_t* slice_sys, int C,
                                                          const int32_t* __restrict__ row_atom,
                                                          const lj_fconst* fc,
                                                          double2* __restrict__ xy,
                                                          double* __restrict__ zz,
                                                          uint4* __restrict__ q32) {
    const int64_t r = blockIdx.x * (int64_t)LJ_BLOCK + threadIdx.x;
    const int64_t i = row_atom[r];
    double x, y, z;
    if (LAYOUT == LJ_AOS4) {
        const double4 q = *reinterpret_cast<const double4*>(
            reinterpret_cast<const char*>(pos) + (i << qshift));
        x = q.x;
        y = q.y;
        z = q.z;
    } else {
        x = pos[i];
        y = pos[n + i];
        z = pos[2 * n + i];
    }
    if (PREC == LJ_FP64) {
        xy[r] = make_double2(x, y);
        zz[r] = z;
    } else {
        const int sid = __builtin_amdgcn_readfirstlane(
            slice_sys[(blockIdx.x * (int64_t)LJ_BLOCK) / C]);
        const lj_fconst& f = fc[sid];
        q32[r] = make_uint4(lj_fix32(x, f.qinv[0]), lj_fix32(y, f.qinv[1]),
                               lj_fix32(z, f.qinv[2]), 0u);
    }
}

// Wavefronts per SIMD the compiler must fit (1: no constraint).  The plain
// full-list loop (4 entries per batch) fits in 80 registers without spilling,
// which lets 6 wavefronts share a SIMD instead of 5 (4% faster in FP64, 6% in
// mixed precision at 131k atoms); the force-shifted loop fits 5 in 96 (4
// unbounded).  The half-list and 8-entry forms would spill at such bounds.
template <bool HALF, int U, bool FS>
constexpr int force_waves() {
    return (HALF || U != 4) ? 1 : (FS ? 5 : 6);
}

// One wavefront per slice; a block's four slices belong to one system
// (systems own whole 256-row blocks).
template <int G, bool HALF, int LAYOUT, int PREC, int U, bool FS>
__global__ __launch_bounds__(LJ_BLOCK)
__attribute__((amdgpu_waves_per_eu(force_waves<HALF, U, FS>()))) void k_force(ForceArgs a) {
    if (halted(a.halt)) return;
    const int64_t blk = lj_xcd_block(blockIdx.x, gridDim.x);
    const int slice = __builtin_amdgcn_readfirstlane(
        (int)blk * LJ_WAVES_PER_BLOCK + (threadIdx.x >> 6));
    const int sid = __builtin_amdgcn_readfirstlane(a.slice_sys[blk * LJ_WAVES_PER_BLOCK]);
    double e, w, c, k;
    if constexpr (HALF) {
        // the block's window (its chunk table and LDS sums), then the
        // slices, then the window's sums added to the accumulator once
        __shared__ int4 htab4[LJ_HWIN_TABLE / 16];
        __shared__ double hacc[3 * LJ_HWIN_MAX * LJ_HWIN_CHUNK];
        __shared__ int hoff[LJ_HWIN_MAX];
        signed char* htab = reinterpret_cast<signed char*>(htab4);
        constexpr int C = LJ_WAVE / G;
        constexpr int HS = LJ_HWIN_MAX * LJ_HWIN_CHUNK;
        const lj_sys& sy = a.sys[sid];
        const int c0 = (int)((blk * LJ_WAVES_PER_BLOCK * C - sy.slice0 * C) >> LJ_HWIN_SHIFT);
        const int nch = (int)((sy.n + LJ_HWIN_CHUNK - 1) >> LJ_HWIN_SHIFT);
        for (int t = threadIdx.x; t < LJ_HWIN_TABLE / 16; t += LJ_BLOCK)
            htab4[t] = make_int4(-1, -1, -1, -1);
        for (int t = threadIdx.x; t < 3 * HS; t += LJ_BLOCK) hacc[t] = 0.0;
        const int32_t* rec = a.hwin + blk * LJ_HWIN_REC;
        const int cnt = __builtin_amdgcn_readfirstlane(rec[0]);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const int off = rec[1 + threadIdx.x];
            hoff[threadIdx.x] = off;
            htab[off + LJ_HWIN_TABLE / 2] = (signed char)threadIdx.x;
        }
        __syncthreads();
        slice_forces<G, HALF, LAYOUT, PREC, U, FS>(a, slice, sid, e, w, c, k, htab, hacc, c0);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt * LJ_HWIN_CHUNK; t += LJ_BLOCK) {
            int ch = c0 + hoff[t >> LJ_HWIN_SHIFT];
            ch += ch < 0 ? nch : (ch >= nch ? -nch : 0);
            const int64_t rel = (int64_t)ch * LJ_HWIN_CHUNK + (t & (LJ_HWIN_CHUNK - 1));
            const double x = hacc[t], y = hacc[HS + t], z = hacc[2 * HS + t];
            if (rel < sy.n && (x != 0.0 || y != 0.0 || z != 0.0))
                acc_add(a.acc, a.n16, sy.atom0 + rel, x, y, z);
        }
    } else {
        slice_forces<G, HALF, LAYOUT, PREC, U, FS>(a, slice, sid, e, w, c, k, nullptr, nullptr,
                                                   0);
    }
    block_partials(a, blk, e, w, c, k);
}

// The window of each half-list force block (one thread block per force
// block): the chunks of LJ_HWIN_CHUNK ranks named by any slot of its slices
// (entries and the rows' own padding), marked in an LDS table of offsets,
// then numbered in offset order; the first LJ_HWIN_MAX are the window.
__global__ __launch_bounds__(LJ_BLOCK) void k_half_windows(const int32_t* __restrict__ col,
                                                           const lj_sys* sys,
                                                           const int32_t* slice_sys,
                                                           const int32_t* slice_iters, int C,
                                                           int G, int32_t* __restrict__ hwin,
                                                           const int32_t* gate) {
    if (gate && __builtin_nontemporal_load(gate) == 0) return;
    __shared__ int4 mark4[LJ_HWIN_TABLE / 16];
    __shared__ int wsum[LJ_WAVES_PER_BLOCK];
    unsigned char* mark = reinterpret_cast<unsigned char*>(mark4);
    const int tid = threadIdx.x, lane = tid & (LJ_WAVE - 1), wave = tid >> 6;
    for (int k = tid; k < LJ_HWIN_TABLE / 16; k += LJ_BLOCK) mark4[k] = make_int4(0, 0, 0, 0);
    const int64_t blk = blockIdx.x;
    const int64_t slice0 = blk * LJ_WAVES_PER_BLOCK;
    const int sid = __builtin_amdgcn_readfirstlane(slice_sys[slice0]);
    const lj_sys& sy = sys[sid];
    const int c0 = (int)((slice0 * C - sy.slice0 * C) >> LJ_HWIN_SHIFT);
    const int nch = (int)((sy.n + LJ_HWIN_CHUNK - 1) >> LJ_HWIN_SHIFT);
    __syncthreads();
    for (int w = 0; w < LJ_WAVES_PER_BLOCK; ++w) {
        const int64_t t = slice0 + w;
        const int64_t nslots = (int64_t)((slice_iters[t] + 3) & ~3) * LJ_WAVE;
        const int32_t* base = col + sy.col0 + (t - sy.slice0) * (int64_t)(sy.cap / G) * LJ_WAVE;
        for (int64_t k = tid; k < nslots; k += LJ_BLOCK) {
            const int ti = lj_hwin_offset(base[k] - (int)sy.atom0, c0, nch) + LJ_HWIN_TABLE / 2;
            if (ti >= 0 && ti < LJ_HWIN_TABLE) mark[ti] = 1;
        }
    }
    __syncthreads();
    // number the marked offsets in order: thread t owns table bytes
    // [t * 64, t * 64 + 64), a block-wide exclusive sum gives its first number
    // (bytes are 0 or 1, so a 32-bit word's count is its bytes' sum)
    constexpr int PER = LJ_HWIN_TABLE / LJ_BLOCK;
    constexpr int PER4 = PER / 16;
    int4 wv[PER4];
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < PER4; ++q) {
        wv[q] = mark4[tid * PER4 + q];
        cnt += (int)(((unsigned)wv[q].x * 0x01010101u) >> 24) +
               (int)(((unsigned)wv[q].y * 0x01010101u) >> 24) +
               (int)(((unsigned)wv[q].z * 0x01010101u) >> 24) +
               (int)(((unsigned)wv[q].w * 0x01010101u) >> 24);
    }
    int incl = cnt;
    for (int d = 1; d < LJ_WAVE; d <<= 1) {
        const int v = __shfl_up(incl, d, LJ_WAVE);
        if (lane >= d) incl += v;
    }
    if (lane == LJ_WAVE - 1) wsum[wave] = incl;
    __syncthreads();
    int before = incl - cnt, total = 0;
    for (int w = 0; w < LJ_WAVES_PER_BLOCK; ++w) {
        if (w < wave) before += wsum[w];
        total += wsum[w];
    }
    int32_t* rec = hwin + blk * LJ_HWIN_REC;
#pragma unroll
    for (int q = 0; q < PER4; ++q) {
        const unsigned wq[4] = {(unsigned)wv[q].x, (unsigned)wv[q].y, (unsigned)wv[q].z,
                                (unsigned)wv[q].w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            for (unsigned bits = wq[c]; bits != 0u; bits &= bits - 1u) {
                const int byte = __builtin_ctz(bits) >> 3;   // the lowest marked byte
                if (before < LJ_HWIN_MAX)
                    rec[1 + before] = tid * PER + q * 16 + c * 4 + byte - LJ_HWIN_TABLE / 2;
                ++before;
            }
        }
    }
    if (tid == 0) rec[0] = total < LJ_HWIN_MAX ? total : LJ_HWIN_MAX;
}

// Half list: the forces from the accumulator (by rank), which is cleared for
// the next evaluation.  One thread per row of the list: the thread of a
// system's k-th row takes rank k and stores the force of that row's atom.
template <int LAYOUT>
__global__ __launch_bounds__(LJ_BLOCK) void k_acc_out(double* __restrict__ acc, int64_t n16,
                                                      int64_t n, const lj_sys* sys,
                                                      const int32_t* slice_sys, int C,
                                                      const int32_t* __restrict__ row_atom,
                                                      const int32_t* flags,
                                                      double* __restrict__ f) {
    if (halted(flags)) return;
    const int64_t r = blockIdx.x * (int64_t)LJ_BLOCK + threadIdx.x;
    const int sid = __builtin_amdgcn_readfirstlane(
        slice_sys[(blockIdx.x * (int64_t)LJ_BLOCK) / C]);
    const lj_sys& sy = sys[sid];
    const int64_t t = r - sy.slice0 * C;
    if (t >= sy.n) return;
    const int64_t k = sy.atom0 + t;
    const double x = acc[k], y = acc[16 * n16 + k], z = acc[32 * n16 + k];
    acc[k] = 0.0;
    acc[16 * n16 + k] = 0.0;
    acc[32 * n16 + k] = 0.0;
    store_f<LAYOUT>(f, n, row_atom[r], x, y, z);
}

template <int G, int U, bool FS>
lj_status launch_g(lj_ctx* ctx, const ForceArgs& a, bool half, int layout, int prec,
                   int64_t blocks) {
    dim3 grid((unsigned)blocks), block(LJ_BLOCK);
    hipStream_t s = ctx->stream;
#define LJ_K(H, L, P) hipLaunchKernelGGL((k_force<G, H, L, P, U, FS>), grid, block, 0, s, a)
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

// Entries in flight per lane (tuning knob: 4 or 8; 2 runs as 4, since a
// lane's indices come 4 steps at a time); the force-shifted truncation is
// built for 4 only (the knob changes speed, never results).
template <int G>
lj_status launch_u(lj_ctx* ctx, const ForceArgs& a, bool half, int layout, int prec,
                   int64_t blocks, bool fs) {
    if (fs) return launch_g<G, 4, true>(ctx, a, half, layout, prec, blocks);
    if (ctx->tune[LJ_TUNE_FORCE_BATCH] == 8)
        return launch_g<G, 8, false>(ctx, a, half, layout, prec, blocks);
    return launch_g<G, 4, false>(ctx, a, half, layout, prec, blocks);
}

}  // namespace

// Block partials of lj_forces_noalloc: device memory of the library itself,
// one copy per GPU (each device holds its own instance of a __device__
// array), so that the call allocates nothing.  Host code must not pass the
// array's name to a kernel (in host code it is a stand-in, not a device
// address): the address is resolved once per device with
// hipGetSymbolAddress.  Every force launch writes every record it later
// reads, so nothing has to be cleared between calls.
static __device__ __align__(256) double4 scratch[LJ_SCRATCH_RECORDS];

lj_status lj_scratch_partials(int device, double** ptr) {
    static std::mutex mu;
    static double* addr[LJ_MAX_DEVICES] = {};
    if (device < 0 || device >= LJ_MAX_DEVICES)
        return lj_fail(LJ_E_INVALID, "device index beyond the library's table");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int prev = -1;
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        hipError_t e = hipSetDevice(device);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
        if (e != hipSuccess) return lj_hip_fail(e, "hipGetSymbolAddress(scratch)");
        addr[device] = static_cast<double*>(p);
    }
    *ptr = addr[device];
    return LJ_OK;
}

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

lj_status lj_launch_half_windows(lj_ctx* ctx, lj_list* l, const int32_t* gate) {
    if (l->kind != LJ_LIST_HALF || !l->hwin) return LJ_OK;
    lj_prof_scope prof(ctx, LJ_PROF_NEIGH);
    hipLaunchKernelGGL(k_half_windows, dim3((unsigned)lj_force_blocks(l->nslices)),
                       dim3(LJ_BLOCK), 0, ctx->stream, (const int32_t*)l->col,
                       (const lj_sys*)l->dsys, (const int32_t*)l->slice_sys,
                       (const int32_t*)l->slice_iters, LJ_WAVE / l->lanes, l->lanes, l->hwin,
                       gate);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}

lj_fconst lj_make_fconst(double eps, double sigma, double rc, const double box[3], int trunc) {
    lj_fconst f = {};
    f.rc2 = rc * rc;
    f.sig2 = sigma * sigma;
    f.c4 = 4.0 * eps;
    f.c24 = 24.0 * eps;
    f.c48 = 48.0 * eps;
    const double s2 = f.sig2 / f.rc2;
    const double s6 = s2 * s2 * s2;
    // V(rc), and Fc = -V'(rc) = 24 eps (sigma/rc)^6 [2 (sigma/rc)^6 - 1] / rc.
    // Per interacting pair the reduction subtracts vc from the energy: V(rc)
    // for the simple truncation, V(rc) + rc Fc for the force-shifted one,
    // whose pair energy V(r) - V(rc) + (r - rc) Fc also adds Fc r (summed in
    // the kernel).
    const double v_rc = 4.0 * eps * s6 * (s6 - 1.0);
    const double f_rc = 24.0 * eps * s6 * (2.0 * s6 - 1.0) / rc;
    f.fshift = trunc == LJ_TRUNC_FORCE_SHIFT ? 1 : 0;
    f.fcut = f.fshift ? f_rc : 0.0;
    f.vc = f.fshift ? v_rc + rc * f_rc : v_rc;
    f.sig2f = (float)f.sig2;
    f.c4f = (float)f.c4;
    f.c24f = (float)f.c24;
    f.c48f = (float)f.c48;
    f.fcutf = (float)f.fcut;
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
                           double* virial, int64_t* npairs, const lj_force_opts& o) {
    const int64_t blocks = lj_force_blocks(l->nslices);
    double* partials = o.partials ? o.partials : ctx->partials;
    const int64_t cap = o.partials ? o.partials_cap : ctx->partials_cap;
    if (lj_force_partials(l) > cap) return lj_fail(LJ_E_INVALID, "block partials too small");
    const bool half = l->kind == LJ_LIST_HALF;
    if (half && !l->acc) return lj_fail(LJ_E_INVALID, "half list without its force accumulator");
    if (half && o.kick != LJ_KICK_NONE)
        return lj_fail(LJ_E_INVALID, "a kick needs whole rows: full lists only");
    const int tl = lj_tmpl_layout(layout);
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
    a.slice_stats = l->slice_stats;
    a.col = l->col;
    a.partials = partials;
    a.acc = l->acc;
    a.hwin = l->hwin;
    a.q32 = l->q32;
    a.xy = l->xy;
    a.zz = l->zz;
    a.n16 = (l->n + 15) / 16;
    a.halt = &ctx->st->flags;
    a.qshift = lj_qshift(layout);
    a.kick = o.kick;
    a.vel = o.vel;
    a.hdt = o.hdt;
    a.write_f = o.write_f ? 1 : 0;
    if (precision != LJ_FP64 && !l->q32)
        return lj_fail(LJ_E_INVALID, "mixed precision without the list's fixed-point buffer");
    const bool fs = o.trunc == LJ_TRUNC_FORCE_SHIFT;
    lj_status st;
    {
        lj_prof_scope prof(ctx, LJ_PROF_OTHER);
        // the rank-ordered copy of the positions the kernel gathers from
        {
            const int C = LJ_WAVE / l->lanes;
            const dim3 qgrid((unsigned)(l->nslices * C / LJ_BLOCK));
#define LJ_COPY(L, P)                                                                      \
    hipLaunchKernelGGL((k_gather_copy<L, P>), qgrid, dim3(LJ_BLOCK), 0, ctx->stream, pos, \
                       l->n, a.qshift, (const int32_t*)l->slice_sys, C,                    \
                       (const int32_t*)l->row_atom, fc, l->xy, l->zz, l->q32)
            if (tl == LJ_AOS4) {
                if (precision == LJ_FP64) LJ_COPY(LJ_AOS4, LJ_FP64); else LJ_COPY(LJ_AOS4, LJ_MIXED);
            } else {
                if (precision == LJ_FP64) LJ_COPY(LJ_SOA, LJ_FP64); else LJ_COPY(LJ_SOA, LJ_MIXED);
            }
#undef LJ_COPY
            LJ_HIP(hipGetLastError());
        }
    }
    {
        lj_prof_scope prof(ctx, LJ_PROF_FORCE);
        switch (l->lanes) {
            case 1: st = launch_u<1>(ctx, a, half, tl, precision, blocks, fs); break;
            case 2: st = launch_u<2>(ctx, a, half, tl, precision, blocks, fs); break;
            case 4: st = launch_u<4>(ctx, a, half, tl, precision, blocks, fs); break;
            case 8: st = launch_u<8>(ctx, a, half, tl, precision, blocks, fs); break;
            case 16: st = launch_u<16>(ctx, a, half, tl, precision, blocks, fs); break;
            case 32: st = launch_u<32>(ctx, a, half, tl, precision, blocks, fs); break;
            case 64: st = launch_u<64>(ctx, a, half, tl, precision, blocks, fs); break;
            default: return lj_fail(LJ_E_INVALID, "lanes must be 1, 2, 4, 8, 16, 32 or 64");
        }
    }
    if (st) return st;
    lj_prof_scope prof(ctx, LJ_PROF_OTHER);
    const int32_t* flags = &ctx->st->flags;
    if (half) {
        const int C = LJ_WAVE / l->lanes;
        const dim3 grid((unsigned)(l->nslices * C / LJ_BLOCK)), block(LJ_BLOCK);
        if (tl == LJ_AOS4)
            hipLaunchKernelGGL(k_acc_out<LJ_AOS4>, grid, block, 0, ctx->stream, l->acc, a.n16,
                               l->n, (const lj_sys*)l->dsys, (const int32_t*)l->slice_sys, C,
                               (const int32_t*)l->row_atom, flags, force);
        else
            hipLaunchKernelGGL(k_acc_out<LJ_SOA>, grid, block, 0, ctx->stream, l->acc, a.n16,
                               l->n, (const lj_sys*)l->dsys, (const int32_t*)l->slice_sys, C,
                               (const int32_t*)l->row_atom, flags, force);
        LJ_HIP(hipGetLastError());
    }
    const int split = lj_force_split(l);
    const double4* first = reinterpret_cast<const double4*>(partials);
    if (split > 1) {
        double4* second = reinterpret_cast<double4*>(partials) + blocks;
        hipLaunchKernelGGL(k_force_reduce_split, dim3((unsigned)(l->nsys * split)), dim3(1024), 0,
                           ctx->stream, first, (const lj_sys*)l->dsys, split, flags, second);
        LJ_HIP(hipGetLastError());
        first = second;
    }
    hipLaunchKernelGGL(k_force_reduce, dim3((unsigned)l->nsys), dim3(1024), 0, ctx->stream, first,
                       (const lj_sys*)l->dsys, split, fc, half ? 1.0 : 0.5, flags, energy, virial,
                       npairs, o.kick != LJ_KICK_NONE ? o.kinetic : nullptr);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}
