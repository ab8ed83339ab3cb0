// lj_cells.hip -- cell binning and counting sort (the linked-list cell method
// of Sec. III.B in array form, grouped with the counting sort of Sec. III.C).
//
//   k_bin        validate each position, compute its cell, and take a slot of
//                the cell with an atomic increment of its count
//   scan         exclusive prefix sum of the counts -> cell_start; the counts
//                are cleared as they are read, ready for the next build
//   k_place      atom i goes to cell_start[cell] + slot (order within a cell
//                is whatever the atomics gave)
//   k_rank       one thread per atom ranks it among its cell's atoms by index,
//                so the final order is the stable counting-sort order, and
//                writes the cell-sorted double4 copy (x, y, z, atom index)
// All kernels are streaming passes over n atoms or ncell cells (a few MB per
// call at 131k atoms).
#include "lj_internal.h"

namespace {

__global__ void k_zero(uint32_t* __restrict__ p, int64_t words) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride) p[i] = 0u;
}

// When `gate` is not NULL a kernel does nothing unless *gate != 0 (a rebuild
// decided on the device).
__device__ __forceinline__ bool gated_off(const int32_t* gate) {
    return gate && __builtin_nontemporal_load(gate) == 0;
}

// Position of atom i: AoS records of 32 (LJ_AOS4) or 64 (LJ_AOS8) bytes, or SoA.
__device__ __forceinline__ void load_xyz(const double* __restrict__ pos, int64_t n, int layout,
                                         int64_t i, double& x, double& y, double& z) {
    if (layout != LJ_SOA) {
        const double4 q = reinterpret_cast<const double4*>(pos)[layout == LJ_AOS8 ? 2 * i : i];
        x = q.x;
        y = q.y;
        z = q.z;
    } else {
        x = pos[i];
        y = pos[n + i];
        z = pos[2 * n + i];
    }
}

struct BinArgs {
    const double* pos;
    int64_t n;                 // atoms over all systems
    int layout;
    const lj_sys* sys;
    const int32_t* atom_sys;   // system of each atom, or NULL for a single system
    int32_t* cid;
    int32_t* slot;
    int32_t* count;
    lj_dev_status* st;
    const int32_t* gate;
};

__global__ __launch_bounds__(LJ_BLOCK) void k_bin(BinArgs a) {
    if (gated_off(a.gate)) return;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const lj_sys& sy = a.sys[a.atom_sys ? a.atom_sys[i] : 0];
    double x, y, z;
    load_xyz(a.pos, a.n, a.layout, i, x, y, z);
    const bool ok = isfinite(x) && isfinite(y) && isfinite(z) && x >= 0.0 && y >= 0.0 &&
                    z >= 0.0 && x < sy.box[0] && y < sy.box[1] && z < sy.box[2];
    int64_t c = sy.cell0;
    if (ok) {
        const int cx = lj_cell_coord(x, sy.inv_cs[0], sy.nc[0]);
        const int cy = lj_cell_coord(y, sy.inv_cs[1], sy.nc[1]);
        const int cz = lj_cell_coord(z, sy.inv_cs[2], sy.nc[2]);
        c += ((int64_t)cz * sy.nc[1] + cy) * sy.nc[0] + cx;
    } else {
        atomicOr(&a.st->flags, LJ_DEV_BAD_POSITION);
    }
    a.cid[i] = (int32_t)c;
    a.slot[i] = atomicAdd(&a.count[c], 1);
}

// Each atom goes to its slot of its cell's range.
__global__ __launch_bounds__(LJ_BLOCK) void k_place(int64_t n, const int32_t* __restrict__ cid,
                                                    const int32_t* __restrict__ slot,
                                                    const int32_t* __restrict__ cell_start,
                                                    int32_t* __restrict__ order_tmp,
                                                    const int32_t* gate) {
    if (gated_off(gate)) return;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    order_tmp[cell_start[cid[i]] + slot[i]] = (int32_t)i;
}

// One thread per position p of the cell-grouped order: the atom there is
// ranked among its cell's atoms by index (the number with a smaller index),
// which puts every cell in index order.  Writes order[], spos[] and spos32[].
__global__ __launch_bounds__(LJ_BLOCK) void k_rank(int64_t n, const int32_t* __restrict__ cid,
                                                   const int32_t* __restrict__ cell_start,
                                                   const int32_t* __restrict__ order_tmp,
                                                   const double* __restrict__ pos, int layout,
                                                   int32_t* __restrict__ order,
                                                   double4* __restrict__ spos,
                                                   float4* __restrict__ spos32,
                                                   const int32_t* gate) {
    if (gated_off(gate)) return;
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int v = order_tmp[p];
    const int c = cid[v];
    const int s0 = cell_start[c], s1 = cell_start[c + 1];
    int rank = 0;
    for (int q = s0; q < s1; ++q) rank += (order_tmp[q] < v) ? 1 : 0;
    double x, y, z;
    load_xyz(pos, n, layout, v, x, y, z);
    order[s0 + rank] = v;
    spos[s0 + rank] = make_double4(x, y, z, __longlong_as_double((long long)v));
    spos32[s0 + rank] = make_float4((float)x, (float)y, (float)z, __int_as_float(v));
}

// ------------------------------------------------------------------ scan
// Large arrays, two passes over tiles of SCAN_ITEMS x LJ_BLOCK values: the
// sum of every tile, then each tile adds up the sums of the tiles before it
// and scans itself.  Thread t of a tile holds the 4 contiguous values
// [4 t, 4 t + 4), loaded and stored as one 16-byte vector (the whole tile is
// one contiguous run per wavefront).
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_ITEMS * LJ_BLOCK;   // 1024

__device__ __forceinline__ int wave_isum(int x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// Sum over the block (every thread gets it).
__device__ __forceinline__ int block_sum(int v, int* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_isum(v);
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    int t = 0;
    for (int w = 0; w < LJ_WAVES_PER_BLOCK; ++w) t += lds[w];
    __syncthreads();
    return t;
}

__device__ __forceinline__ int block_exclusive_scan(int v, int* lds, int& total) {
    // wave inclusive scan
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < LJ_WAVES_PER_BLOCK; ++w) {
        if (w < wave) off += lds[w];
        tot += lds[w];
    }
    __syncthreads();
    total = tot;
    return off + x - v;
}

// Values [4 i, 4 i + 4) of the array (zeros past its end m).
__device__ __forceinline__ int4 load4(const int32_t* __restrict__ in, int64_t i4, int64_t m) {
    const int64_t i = 4 * i4;
    if (i + 4 <= m) return reinterpret_cast<const int4*>(in)[i4];
    return make_int4(i < m ? in[i] : 0, i + 1 < m ? in[i + 1] : 0, i + 2 < m ? in[i + 2] : 0, 0);
}

__global__ __launch_bounds__(LJ_BLOCK) void k_scan_reduce(const int32_t* __restrict__ in,
                                                          int64_t m,
                                                          int32_t* __restrict__ tile_sums,
                                                          const int32_t* gate) {
    if (gated_off(gate)) return;
    __shared__ int lds[LJ_WAVES_PER_BLOCK];
    const int4 v = load4(in, blockIdx.x * (int64_t)LJ_BLOCK + threadIdx.x, m);
    const int s = block_sum(v.x + v.y + v.z + v.w, lds);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = s;
}

__global__ __launch_bounds__(LJ_BLOCK) void k_scan_tiles(int32_t* __restrict__ in,
                                                         int32_t* __restrict__ out, int64_t m,
                                                         const int32_t* __restrict__ tile_sums,
                                                         int clear_in, const int32_t* gate) {
    if (gated_off(gate)) return;
    __shared__ int lds[LJ_WAVES_PER_BLOCK];
    // offset of this tile: the sums of the tiles before it
    int before = 0;
    for (int t = threadIdx.x; t < (int)blockIdx.x; t += LJ_BLOCK) before += tile_sums[t];
    before = block_sum(before, lds);
    const int64_t i4 = blockIdx.x * (int64_t)LJ_BLOCK + threadIdx.x, i = 4 * i4;
    const int4 v = load4(in, i4, m);
    if (clear_in) {
        if (i + 4 <= m) {
            reinterpret_cast<int4*>(in)[i4] = make_int4(0, 0, 0, 0);
        } else {
            for (int64_t k = i; k < m; ++k) in[k] = 0;
        }
    }
    int total;
    const int run = before + block_exclusive_scan(v.x + v.y + v.z + v.w, lds, total);
    const int4 o = make_int4(run, run + v.x, run + v.x + v.y, run + v.x + v.y + v.z);
    if (i + 4 <= m) {
        reinterpret_cast<int4*>(out)[i4] = o;
    } else {
        if (i < m) out[i] = o.x;
        if (i + 1 < m) out[i + 1] = o.y;
        if (i + 2 < m) out[i + 2] = o.z;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[m] = before + total;
}

// Small arrays: one block.  The array is loaded with coalesced loads (all of
// a thread's loads in flight at once) into LDS, padded by one word per 32 so
// that thread t can then scan its contiguous chunk [32 t, 32 t + 32) without
// bank conflicts; a block scan of the chunk totals gives each chunk its
// offset, and the result goes back out coalesced.
constexpr int SCAN1_THREADS = 1024;
constexpr int SCAN1_PER = 32;
constexpr int64_t SCAN1_MAX = (int64_t)SCAN1_THREADS * SCAN1_PER;
__device__ __forceinline__ int scan1_pad(int i) { return i + (i >> 5); }
__global__ __launch_bounds__(SCAN1_THREADS) void k_scan_single(int32_t* __restrict__ in,
                                                               int32_t* __restrict__ out,
                                                               int64_t m, int clear_in,
                                                               const int32_t* gate) {
    if (gated_off(gate)) return;
    __shared__ int buf[SCAN1_MAX + SCAN1_MAX / 32];
    __shared__ int lds[SCAN1_THREADS / 64];
    const int t = threadIdx.x;
    {
        int v[SCAN1_PER];
#pragma unroll
        for (int k = 0; k < SCAN1_PER; ++k) {
            const int idx = k * SCAN1_THREADS + t;
            v[k] = idx < m ? in[idx] : 0;
        }
#pragma unroll
        for (int k = 0; k < SCAN1_PER; ++k) buf[scan1_pad(k * SCAN1_THREADS + t)] = v[k];
        if (clear_in) {
#pragma unroll
            for (int k = 0; k < SCAN1_PER; ++k) {
                const int idx = k * SCAN1_THREADS + t;
                if (idx < m) in[idx] = 0;
            }
        }
    }
    __syncthreads();
    const int c0 = scan1_pad(t * SCAN1_PER);   // the chunk is contiguous in LDS
    int v[SCAN1_PER];
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN1_PER; ++k) {
        v[k] = buf[c0 + k];
        s += v[k];
    }
    const int lane = t & 63, wave = t >> 6;
    int x = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < SCAN1_THREADS / 64; ++w) {
        if (w < wave) off += lds[w];
        tot += lds[w];
    }
    int run = off + x - s;
#pragma unroll
    for (int k = 0; k < SCAN1_PER; ++k) {
        buf[c0 + k] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCAN1_PER; ++k) {
        const int idx = k * SCAN1_THREADS + t;
        if (idx < m) out[idx] = buf[scan1_pad(idx)];
    }
    if (t == 0) out[m] = tot;
}


inline unsigned grid_for(int64_t n, int per_block) {
    return (unsigned)((n + per_block - 1) / per_block);
}

}  // namespace

int64_t lj_scan_workspace(int64_t m) { return (m + SCAN_TILE - 1) / SCAN_TILE + 1; }

lj_status lj_launch_zero(hipStream_t s, void* p, int64_t bytes) {
    if (bytes <= 0) return LJ_OK;
    const int64_t words = (bytes + 3) / 4;
    int64_t blocks = (words + LJ_BLOCK - 1) / LJ_BLOCK;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(LJ_BLOCK), 0, s, (uint32_t*)p, words);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}

lj_status lj_launch_scan(hipStream_t s, int32_t* in, int32_t* out, int64_t m, int32_t* work,
                         bool clear_in, const int32_t* gate) {
    const int64_t nt = (m + SCAN_TILE - 1) / SCAN_TILE;
    if (nt > 16 * SCAN_TILE) return lj_fail(LJ_E_CAPACITY, "scan: more than 16.7M elements");
    if (m == 0) return lj_launch_zero(s, out, sizeof(int32_t));
    if (m <= SCAN1_MAX) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(SCAN1_THREADS), 0, s, in, out, m,
                           clear_in ? 1 : 0, gate);
        LJ_HIP(hipGetLastError());
        return LJ_OK;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nt), dim3(LJ_BLOCK), 0, s,
                       (const int32_t*)in, m, work, gate);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(LJ_BLOCK), 0, s, in, out, m,
                       (const int32_t*)work, clear_in ? 1 : 0, gate);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}

lj_status lj_launch_cells(lj_ctx* ctx, const double* pos, int layout, lj_cells* c,
                          const int32_t* gate) {
    hipStream_t s = ctx->stream;
    lj_prof_scope prof(ctx, LJ_PROF_CELLS);
    lj_status st;
    // The per-cell counts are zero between builds: the scan clears them as it
    // reads them.  Clear them here only after an interrupted build.
    if (c->counts_dirty) {
        if ((st = lj_launch_zero(s, c->count, c->ncell * (int64_t)sizeof(int32_t)))) return st;
    }
    c->counts_dirty = true;
    BinArgs a;
    a.pos = pos;
    a.n = c->n;
    a.layout = layout;
    a.sys = c->dsys;
    a.atom_sys = c->atom_sys;
    a.cid = c->cid;
    a.slot = c->slot;
    a.count = c->count;
    a.st = ctx->st;
    a.gate = gate;
    hipLaunchKernelGGL(k_bin, dim3(grid_for(c->n, LJ_BLOCK)), dim3(LJ_BLOCK), 0, s, a);
    LJ_HIP(hipGetLastError());
    st = lj_launch_scan(s, c->count, c->cell_start, c->ncell, c->block_sums, true, gate);
    if (st) return st;
    c->counts_dirty = false;
    hipLaunchKernelGGL(k_place, dim3(grid_for(c->n, LJ_BLOCK)), dim3(LJ_BLOCK), 0, s, c->n,
                       (const int32_t*)c->cid, (const int32_t*)c->slot,
                       (const int32_t*)c->cell_start, c->order_tmp, gate);
    LJ_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_rank, dim3(grid_for(c->n, LJ_BLOCK)), dim3(LJ_BLOCK), 0, s, c->n,
                       (const int32_t*)c->cid, (const int32_t*)c->cell_start,
                       (const int32_t*)c->order_tmp, pos, layout, c->order, c->spos,
                       c->spos32, gate);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}
