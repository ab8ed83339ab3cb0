// lj_cells.hip -- cell binning and counting sort (the linked-list cell method
// of Sec. III.B in array form, grouped with the counting sort of Sec. III.C).
//
//   k_bin        validate each position, compute its cell, count atoms per cell
//   scan         exclusive prefix sum of the counts -> cell_start
//   k_scatter    place each atom in its cell's range (order within a cell is
//                whatever the atomics give)
//   k_cell_sort  one wavefront per cell ranks the cell's atoms by index, so
//                the final order is the stable counting-sort order, and writes
//                the cell-sorted double4 copy (x, y, z, atom index)
// All kernels are streaming passes over n atoms or ncell cells (HBM bound,
// a few MB per call at 131k atoms).
#include "lj_internal.h"

namespace {

__global__ void k_zero(uint32_t* __restrict__ p, int64_t words) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride) p[i] = 0u;
}

__device__ __forceinline__ void load_xyz(const double* __restrict__ pos, int64_t n, int layout,
                                         int64_t i, double& x, double& y, double& z) {
    if (layout == LJ_AOS4) {
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

struct BinArgs {
    const double* pos;
    int64_t n;                 // atoms over all systems
    int layout;
    const lj_sys* sys;
    const int32_t* atom_sys;   // system of each atom, or NULL for a single system
    int32_t* cid;
    int32_t* count;
    lj_dev_status* st;
};

__global__ __launch_bounds__(LJ_BLOCK) void k_bin(BinArgs a) {
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
    atomicAdd(&a.count[c], 1);
}

// Each atom takes a slot of its cell by counting the cell down from the top.
__global__ __launch_bounds__(LJ_BLOCK) void k_scatter(int64_t n, const int32_t* __restrict__ cid,
                                                      const int32_t* __restrict__ cell_start,
                                                      int32_t* __restrict__ count,
                                                      int32_t* __restrict__ order_tmp) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cid[i];
    const int k = atomicSub(&count[c], 1) - 1;
    order_tmp[cell_start[c] + k] = (int32_t)i;
}

// One wavefront per cell: the rank of an atom within its cell is the number
// of the cell's atoms with a smaller index.  Writes order[] and spos[].
__global__ __launch_bounds__(LJ_BLOCK) void k_cell_sort(
    int64_t ncell, int64_t n, const int32_t* __restrict__ cell_start,
    const int32_t* __restrict__ order_tmp, const double* __restrict__ pos, int layout,
    int32_t* __restrict__ order, double4* __restrict__ spos) {
    const int lane = threadIdx.x & (LJ_WAVE - 1);
    const int64_t cell = blockIdx.x * (int64_t)LJ_WAVES_PER_BLOCK + (threadIdx.x >> 6);
    if (cell >= ncell) return;
    const int s0 = cell_start[cell], s1 = cell_start[cell + 1];
    const int m = s1 - s0;
    for (int a = lane; a - lane < m; a += LJ_WAVE) {
        const int v = a < m ? order_tmp[s0 + a] : INT32_MAX;
        int rank = 0;
        if (m <= LJ_WAVE) {
            for (int b = 0; b < m; ++b) rank += (__shfl(v, b, LJ_WAVE) < v) ? 1 : 0;
        } else {
            for (int b = 0; b < m; ++b) rank += (order_tmp[s0 + b] < v) ? 1 : 0;
        }
        if (a < m) {
            double x, y, z;
            load_xyz(pos, n, layout, v, x, y, z);
            order[s0 + rank] = v;
            spos[s0 + rank] = make_double4(x, y, z, __longlong_as_double((long long)v));
        }
    }
}

// ------------------------------------------------------------------ scan
// Three-phase exclusive scan: per-block scan of SCAN_ITEMS x LJ_BLOCK values
// with block totals, scan of the totals (one block), add back.
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_ITEMS * LJ_BLOCK;   // 4096

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

__global__ __launch_bounds__(LJ_BLOCK) void k_scan_tile(const int32_t* __restrict__ in,
                                                        int32_t* __restrict__ out, int64_t m,
                                                        int32_t* __restrict__ tile_sums) {
    __shared__ int lds[LJ_WAVES_PER_BLOCK];
    const int64_t base = blockIdx.x * (int64_t)SCAN_TILE + threadIdx.x * (int64_t)SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = (base + k < m) ? in[base + k] : 0;
        s += v[k];
    }
    int total;
    int run = block_exclusive_scan(s, lds, total);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < m) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// Scans up to SCAN_TILE tile sums in place (exclusive) and writes the total.
__global__ __launch_bounds__(LJ_BLOCK) void k_scan_sums(int32_t* __restrict__ sums, int64_t nt,
                                                        int32_t* __restrict__ out_total) {
    __shared__ int lds[LJ_WAVES_PER_BLOCK];
    const int64_t base = threadIdx.x * (int64_t)SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = (base + k < nt) ? sums[base + k] : 0;
        s += v[k];
    }
    int total;
    int run = block_exclusive_scan(s, lds, total);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < nt) sums[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) *out_total = total;
}

// Small arrays: one block stages the whole array in LDS with coalesced loads,
// each thread scans a contiguous chunk there, and the result is written back
// coalesced.
constexpr int SCAN1_THREADS = 1024;
constexpr int64_t SCAN1_MAX = 32768;   // 128 KB of LDS
__global__ __launch_bounds__(SCAN1_THREADS) void k_scan_single(const int32_t* __restrict__ in,
                                                               int32_t* __restrict__ out,
                                                               int64_t m) {
    __shared__ int buf[SCAN1_MAX];
    __shared__ int lds[SCAN1_THREADS / 64];
    for (int64_t k = threadIdx.x; k < m; k += SCAN1_THREADS) buf[k] = in[k];
    __syncthreads();
    const int per = (int)((m + SCAN1_THREADS - 1) / SCAN1_THREADS);
    const int b0 = threadIdx.x * per;
    int s = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < m) s += buf[b0 + k];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
    for (int k = 0; k < per; ++k)
        if (b0 + k < m) {
            const int v = buf[b0 + k];
            buf[b0 + k] = run;
            run += v;
        }
    __syncthreads();
    for (int64_t k = threadIdx.x; k < m; k += SCAN1_THREADS) out[k] = buf[k];
    if (threadIdx.x == 0) out[m] = tot;
}

__global__ __launch_bounds__(LJ_BLOCK) void k_scan_add(int32_t* __restrict__ out, int64_t m,
                                                       const int32_t* __restrict__ sums) {
    const int add = sums[blockIdx.x];
    const int64_t base = blockIdx.x * (int64_t)SCAN_TILE;
    for (int k = threadIdx.x; k < SCAN_TILE; k += LJ_BLOCK)
        if (base + k < m) out[base + k] += add;
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

lj_status lj_launch_scan(hipStream_t s, const int32_t* in, int32_t* out, int64_t m,
                         int32_t* work) {
    const int64_t nt = (m + SCAN_TILE - 1) / SCAN_TILE;
    if (nt > SCAN_TILE) return lj_fail(LJ_E_CAPACITY, "scan: more than 16.7M elements");
    if (m == 0) return lj_launch_zero(s, out, sizeof(int32_t));
    if (m <= SCAN1_MAX) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(SCAN1_THREADS), 0, s, in, out, m);
        LJ_HIP(hipGetLastError());
        return LJ_OK;
    }
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nt), dim3(LJ_BLOCK), 0, s, in, out, m, work);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(LJ_BLOCK), 0, s, work, nt, out + m);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nt), dim3(LJ_BLOCK), 0, s, out, m,
                       (const int32_t*)work);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}

lj_status lj_launch_cells(lj_ctx* ctx, const double* pos, int layout, lj_cells* c) {
    hipStream_t s = ctx->stream;
    lj_prof_scope prof(ctx, LJ_PROF_CELLS);
    lj_status st;
    // The per-cell counts are zero between builds: the scatter counts each
    // cell back down to zero.  Clear them only after an interrupted build.
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
    a.count = c->count;
    a.st = ctx->st;
    hipLaunchKernelGGL(k_bin, dim3(grid_for(c->n, LJ_BLOCK)), dim3(LJ_BLOCK), 0, s, a);
    LJ_HIP(hipGetLastError());
    st = lj_launch_scan(s, c->count, c->cell_start, c->ncell, c->block_sums);
    if (st) return st;
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(c->n, LJ_BLOCK)), dim3(LJ_BLOCK), 0, s, c->n,
                       (const int32_t*)c->cid, (const int32_t*)c->cell_start, c->count,
                       c->order_tmp);
    LJ_HIP(hipGetLastError());
    c->counts_dirty = false;
    hipLaunchKernelGGL(k_cell_sort, dim3(grid_for(c->ncell, LJ_WAVES_PER_BLOCK)), dim3(LJ_BLOCK),
                       0, s, c->ncell, c->n, (const int32_t*)c->cell_start,
                       (const int32_t*)c->order_tmp, pos, layout, c->order, c->spos);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}
