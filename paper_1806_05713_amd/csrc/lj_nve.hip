// lj_nve.hip -- velocity-Verlet NVE integration around the force path, for a
// batch of independent systems (a single system is a batch of one).
//
// Per step (unit mass):
//   drift   : v += F dt/2; dx = v dt; x += dx, wrapped into [0, L);
//             disp += dx, or disp = 0 at a rebuild step
//   [rebuild: cells + list in place]
//   forces  : F, per-system potential energy, virial, pair count
//   kick    : v += F dt/2; per-block partial sums of v^2/2 and max |disp|^2
//   k_log   : one block per system sums its partials in a fixed order and
//             writes the system's log row (PE, KE, W, max displacement, pairs)
// Within a run of consecutive steps the kick that ends step k and the drift
// that opens step k + 1 use the same force, so one kernel (k_kick_drift) does
// both and streams each atom once; the velocity between the two half kicks
// is rounded to FP64 as if it had been stored, so the trajectory is the same
// bit for bit however a run is cut into launches.  Only a run's last step
// ends with a kick of its own (k_kick).
// The per-atom kernels take one thread per row of the list (256-row blocks,
// each inside one system), so every block knows its system and box, but the
// thread of a system's k-th row handles the system's k-th atom in memory
// order, not the row's atom: the arrays stream instead of being gathered.
// In a mixed-precision run the drift also writes the force kernel's
// fixed-point positions, so the forces that follow need no conversion pass.
// Every product and sum is rounded on its own, as in the oracle's
// integrator.  Bytes per atom (AoS4): drift 208 (reads vel, force, pos 32
// each and disp 24; writes vel, pos, disp), kick 120 (reads vel, force,
// disp; writes vel); the fused kernel moves the same 208 as the drift alone,
// 224 in a mixed run (the 16-byte fixed-point record).
#include <math.h>

#include <algorithm>

#include "lj_internal.h"

struct lj_nve {
    lj_ctx* ctx;
    lj_list* list;
    double *pos, *vel, *force, *log;
    int64_t log_rows;
    int layout, precision, rebuild_every, nsys;
    double dt;
    lj_fconst* fc;         // device, nsys
    double* disp;          // n x 3: displacement since the last build
    double* partials;      // 2 per row block: kinetic energy, max |disp|^2
    double* pe_w;          // nsys potential energies, then nsys virials
    int64_t* npairs;       // per system
    int64_t* dstep;        // device step counter: log row of the current step
    int64_t steps;         // host step counter
    int64_t rblocks;       // 256-row blocks of the list
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipStream_t cap_stream;
};

namespace {

// Three components of one atom's record; w is AoS4's fourth double, kept as read.
struct Rec {
    double v[3];
    double w;
};

template <int LAYOUT>
__device__ __forceinline__ Rec load_rec(const double* a, int64_t n, int64_t i) {
    Rec o;
    if constexpr (LAYOUT == LJ_AOS4) {
        const double4 q = reinterpret_cast<const double4*>(a)[i];
        o.v[0] = q.x;
        o.v[1] = q.y;
        o.v[2] = q.z;
        o.w = q.w;
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) o.v[d] = a[(int64_t)d * n + i];
        o.w = 0.0;
    }
    return o;
}

template <int LAYOUT>
__device__ __forceinline__ void store_rec(double* a, int64_t n, int64_t i, const Rec& o) {
    if constexpr (LAYOUT == LJ_AOS4) {
        reinterpret_cast<double4*>(a)[i] = make_double4(o.v[0], o.v[1], o.v[2], o.w);
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) a[(int64_t)d * n + i] = o.v[d];
    }
}

struct RowArgs {
    double* pos;
    double* vel;
    const double* force;
    double* disp;
    int64_t n;             // atoms over all systems (SoA stride)
    const lj_sys* sys;
    const int32_t* slice_sys;
    int C;                 // rows per slice
    double* partials;
    int64_t* dstep;
    uint4* q32;            // mixed precision: fixed-point copy written by the drift (or NULL)
    const lj_fconst* fc;   // per system: the fixed-point unit
};

// Half kick, drift and displacement update of one atom (record index i).
template <int LAYOUT>
__device__ __forceinline__ void drift_atom(const RowArgs& a, const lj_sys& sy, int64_t i, Rec& v,
                                           const Rec& f, double hdt, double dt, int reset) {
#pragma clang fp contract(off)
    Rec x = load_rec<LAYOUT>(a.pos, a.n, i);
    double* u = a.disp + 3 * i;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double L = sy.box[d];
        v.v[d] = v.v[d] + hdt * f.v[d];
        const double dx = dt * v.v[d];
        double xd = x.v[d] + dx;
        xd = xd - L * floor(xd / L);
        if (xd >= L) xd = 0.0;
        x.v[d] = xd;
        u[d] = reset ? 0.0 : u[d] + dx;
    }
    store_rec<LAYOUT>(a.vel, a.n, i, v);
    store_rec<LAYOUT>(a.pos, a.n, i, x);
    if (a.q32) {
        const double* inv = a.fc[&sy - a.sys].qinv;   // sy is an element of a.sys
        a.q32[i] = make_uint4(lj_fix32(x.v[0], inv[0]), lj_fix32(x.v[1], inv[1]),
                              lj_fix32(x.v[2], inv[2]), 0u);
    }
}

// Half kick of one atom; returns its kinetic energy and |disp|^2.
__device__ __forceinline__ void kick_atom(const RowArgs& a, int64_t i, Rec& v, const Rec& f,
                                          double hdt, double& ke, double& d2) {
#pragma clang fp contract(off)
#pragma unroll
    for (int d = 0; d < 3; ++d) v.v[d] = v.v[d] + hdt * f.v[d];
    ke = 0.5 * ((v.v[0] * v.v[0] + v.v[1] * v.v[1]) + v.v[2] * v.v[2]);
    const double* u = a.disp + 3 * i;
    d2 = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
}

// Block partials of the kinetic energy (fixed-order sum) and of max |disp|^2.
__device__ __forceinline__ void block_partials(const RowArgs& a, double ke, double d2) {
    __shared__ double red[LJ_WAVES_PER_BLOCK][2];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        ke += __shfl_xor(ke, d, LJ_WAVE);
        d2 = fmax(d2, __shfl_xor(d2, d, LJ_WAVE));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[wave][0] = ke;
        red[wave][1] = d2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double k = 0.0, m = 0.0;
        for (int w = 0; w < LJ_WAVES_PER_BLOCK; ++w) {
            k += red[w][0];
            m = fmax(m, red[w][1]);
        }
        a.partials[2 * blockIdx.x] = k;
        a.partials[2 * blockIdx.x + 1] = m;
    }
}

// Thread r of the list's row space handles atom atom0 + (r - first row of
// its system): the system's atoms in memory order, so every array streams.
// A negative result means the thread has no atom.
__device__ __forceinline__ int64_t row_to_atom(const RowArgs& a, const lj_sys*& sy) {
    const int64_t r = blockIdx.x * (int64_t)LJ_BLOCK + threadIdx.x;
    const int sid = __builtin_amdgcn_readfirstlane(
        a.slice_sys[(blockIdx.x * (int64_t)LJ_BLOCK) / a.C]);
    sy = a.sys + sid;
    const int64_t t = r - sy->slice0 * a.C;
    return t < sy->n ? sy->atom0 + t : -1;
}

// Opens a step: half kick with the current force, drift; bumps the step counter.
template <int LAYOUT>
__global__ __launch_bounds__(LJ_BLOCK) void k_drift(RowArgs a, double hdt, double dt, int reset) {
    const lj_sys* sy;
    const int64_t i = row_to_atom(a, sy);
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.dstep += 1;
    if (i < 0) return;
    Rec v = load_rec<LAYOUT>(a.vel, a.n, i);
    const Rec f = load_rec<LAYOUT>(a.force, a.n, i);
    drift_atom<LAYOUT>(a, *sy, i, v, f, hdt, dt, reset);
}

// Ends a step: half kick with the new force; kinetic energy and displacement
// partials for the step's log row.
template <int LAYOUT>
__global__ __launch_bounds__(LJ_BLOCK) void k_kick(RowArgs a, double hdt) {
    const lj_sys* sy;
    const int64_t i = row_to_atom(a, sy);
    double ke = 0.0, d2 = 0.0;
    if (i >= 0) {
        Rec v = load_rec<LAYOUT>(a.vel, a.n, i);
        const Rec f = load_rec<LAYOUT>(a.force, a.n, i);
        kick_atom(a, i, v, f, hdt, ke, d2);
        store_rec<LAYOUT>(a.vel, a.n, i, v);
    }
    block_partials(a, ke, d2);
}

// Ends step k and opens step k + 1: the kick's partials are those of step k
// (its displacement is read before the drift updates it).
template <int LAYOUT>
__global__ __launch_bounds__(LJ_BLOCK) void k_kick_drift(RowArgs a, double hdt, double dt,
                                                         int reset) {
    const lj_sys* sy;
    const int64_t i = row_to_atom(a, sy);
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.dstep += 1;
    double ke = 0.0, d2 = 0.0;
    if (i >= 0) {
        Rec v = load_rec<LAYOUT>(a.vel, a.n, i);
        const Rec f = load_rec<LAYOUT>(a.force, a.n, i);
        kick_atom(a, i, v, f, hdt, ke, d2);
        drift_atom<LAYOUT>(a, *sy, i, v, f, hdt, dt, reset);
    }
    block_partials(a, ke, d2);
}

// One block per system: fixed-order sums of its row blocks' partials, then
// the system's log row for step *dstep + back (back = -1 after the fused
// kernel has opened the next step).
__global__ __launch_bounds__(1024) void k_log(const double* __restrict__ partials,
                                              const lj_sys* sys, int C, const double* pe_w,
                                              const int64_t* npairs, const int64_t* dstep,
                                              int back, double* log, int64_t log_rows,
                                              int nsys) {
    __shared__ double red[16][2];
    const int s = blockIdx.x;
    const lj_sys& sy = sys[s];
    const int64_t b0 = sy.slice0 * C / LJ_BLOCK, b1 = (sy.slice0 + sy.nslices) * C / LJ_BLOCK;
    double ke = 0.0, d2 = 0.0;
    // four partials per thread and pass, loaded before they are added (the
    // order of the sums is fixed by the thread and the pass)
    for (int64_t bb = b0 + threadIdx.x; bb < b1; bb += 4 * 1024) {
        double2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t b = bb + u * 1024;
            v[u] = b < b1 ? reinterpret_cast<const double2*>(partials)[b] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ke += v[u].x;
            d2 = fmax(d2, v[u].y);
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        ke += __shfl_xor(ke, d, LJ_WAVE);
        d2 = fmax(d2, __shfl_xor(d2, d, LJ_WAVE));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[wave][0] = ke;
        red[wave][1] = d2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double k = 0.0, m = 0.0;
        for (int w = 0; w < 16; ++w) {
            k += red[w][0];
            m = fmax(m, red[w][1]);
        }
        const int64_t row = *dstep + back;
        if (row >= 0 && row < log_rows) {
            double* out = log + 5 * (row * nsys + s);
            out[0] = pe_w[s];
            out[1] = k;
            out[2] = pe_w[nsys + s];
            out[3] = sqrt(m);
            out[4] = (double)npairs[s];
        }
    }
}

__global__ void k_set_step(int64_t* dstep, int64_t v) { *dstep = v; }

RowArgs row_args(lj_nve* s) {
    RowArgs a;
    a.pos = s->pos;
    a.vel = s->vel;
    a.force = s->force;
    a.disp = s->disp;
    a.n = s->list->n;
    a.sys = s->list->dsys;
    a.slice_sys = s->list->slice_sys;
    a.C = LJ_WAVE / s->list->lanes;
    a.partials = s->partials;
    a.dstep = s->dstep;
    a.q32 = s->precision != LJ_FP64 ? s->list->q32 : nullptr;
    a.fc = s->fc;
    return a;
}

// after a drift the mixed kernel's fixed-point copy is already current
lj_status forces(lj_nve* s, bool after_drift) {
    return lj_launch_forces(s->ctx, s->pos, s->layout, s->precision, s->list, s->fc, s->force,
                            s->pe_w, s->pe_w + s->nsys, s->npairs, after_drift);
}

lj_status log_row(lj_nve* s, int back) {
    lj_prof_scope prof(s->ctx, LJ_PROF_INTEGRATE);
    hipLaunchKernelGGL(k_log, dim3((unsigned)s->nsys), dim3(1024), 0, s->ctx->stream,
                       (const double*)s->partials, (const lj_sys*)s->list->dsys,
                       LJ_WAVE / s->list->lanes, (const double*)s->pe_w,
                       (const int64_t*)s->npairs, (const int64_t*)s->dstep, back, s->log,
                       s->log_rows, s->nsys);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}

// Steps first + 1 .. first + count as one chain: drift, then per step
// [rebuild] and forces, with the kick that ends a step fused into the drift
// that opens the next; the chain ends with a kick of its own.  Every step's
// log row is written before the next step's forces replace its energies.
template <int LAYOUT>
lj_status enqueue_chain(lj_nve* s, int64_t first, int64_t count) {
    lj_ctx* ctx = s->ctx;
    const dim3 grid((unsigned)s->rblocks), block(LJ_BLOCK);
    const RowArgs a = row_args(s);
    const double hdt = 0.5 * s->dt, dt = s->dt;
    lj_status st;
    for (int64_t k = 1; k <= count; ++k) {
        const bool rebuild = (first + k) % s->rebuild_every == 0;
        if (k == 1) {
            lj_prof_scope prof(ctx, LJ_PROF_INTEGRATE);
            hipLaunchKernelGGL(k_drift<LAYOUT>, grid, block, 0, ctx->stream, a, hdt, dt,
                               rebuild ? 1 : 0);
            LJ_HIP(hipGetLastError());
        } else {
            {
                lj_prof_scope prof(ctx, LJ_PROF_INTEGRATE);
                hipLaunchKernelGGL(k_kick_drift<LAYOUT>, grid, block, 0, ctx->stream, a, hdt, dt,
                                   rebuild ? 1 : 0);
                LJ_HIP(hipGetLastError());
            }
            if ((st = log_row(s, -1))) return st;
        }
        if (rebuild) {
            lj_list* l = s->list;
            if ((st = lj_launch_cells(ctx, s->pos, s->layout, l->cells))) return st;
            if ((st = lj_launch_neighbors(ctx, l->cells, l, false))) return st;
        }
        if ((st = forces(s, true))) return st;
    }
    {
        lj_prof_scope prof(ctx, LJ_PROF_INTEGRATE);
        hipLaunchKernelGGL(k_kick<LAYOUT>, grid, block, 0, ctx->stream, a, hdt);
        LJ_HIP(hipGetLastError());
    }
    return log_row(s, 0);
}

lj_status chain(lj_nve* s, int64_t first, int64_t count) {
    if (count <= 0) return LJ_OK;
    return s->layout == LJ_AOS4 ? enqueue_chain<LJ_AOS4>(s, first, count)
                                : enqueue_chain<LJ_SOA>(s, first, count);
}

void release(lj_nve* s) {
    if (!s) return;
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    if (s->fc) (void)hipFree(s->fc);
    if (s->disp) (void)hipFree(s->disp);
    if (s->partials) (void)hipFree(s->partials);
    if (s->pe_w) (void)hipFree(s->pe_w);
    if (s->npairs) (void)hipFree(s->npairs);
    if (s->dstep) (void)hipFree(s->dstep);
    delete s;
}

lj_status capture_cycle(lj_nve* s) {
    lj_ctx* ctx = s->ctx;
    if (!s->cap_stream) LJ_HIP(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    // the capture stream must see everything already queued on the context's stream
    hipEvent_t ev;
    LJ_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, ctx->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s->cap_stream, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return lj_hip_fail(e, "capture stream ordering");
    hipStream_t saved = ctx->stream;
    const bool prof = ctx->prof_on;
    ctx->prof_on = false;
    ctx->stream = s->cap_stream;
    lj_status st = LJ_OK;
    e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        st = lj_hip_fail(e, "hipStreamBeginCapture");
    } else {
        st = chain(s, 0, s->rebuild_every);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s->cap_stream, &g);
        if (!st && e != hipSuccess) st = lj_hip_fail(e, "hipStreamEndCapture");
        if (!st) {
            s->graph = g;
            e = hipGraphInstantiate(&s->exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) st = lj_hip_fail(e, "hipGraphInstantiate");
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    ctx->stream = saved;
    ctx->prof_on = prof;
    return st;
}

}  // namespace

lj_status lj_nve_make(lj_ctx* ctx, double* pos, double* vel, double* force, int32_t layout,
                      const lj_fconst* hfc, int32_t precision, lj_list* list, double dt,
                      int32_t rebuild_every, double* log, int64_t log_rows, lj_nve** out) {
    lj_nve* s = new (std::nothrow) lj_nve();
    if (!s) return lj_fail(LJ_E_NOMEM, "host allocation");
    s->ctx = ctx;
    s->list = list;
    s->pos = pos;
    s->vel = vel;
    s->force = force;
    s->log = log;
    s->log_rows = log_rows;
    s->layout = layout;
    s->precision = precision;
    s->rebuild_every = rebuild_every;
    s->nsys = list->nsys;
    s->dt = dt;
    s->rblocks = list->nslices * (LJ_WAVE / list->lanes) / LJ_BLOCK;
    const int64_t n = list->n;
    hipError_t e = hipMalloc((void**)&s->disp, (size_t)n * 3 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&s->fc, (size_t)s->nsys * sizeof(lj_fconst));
    if (e == hipSuccess)
        e = hipMalloc((void**)&s->partials, (size_t)s->rblocks * 2 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&s->pe_w, (size_t)s->nsys * 2 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&s->npairs, (size_t)s->nsys * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc((void**)&s->dstep, sizeof(int64_t));
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->fc, hfc, (size_t)s->nsys * sizeof(lj_fconst), hipMemcpyHostToDevice,
                           ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        release(s);
        return lj_hip_fail(e, "integrator allocation");
    }
    *out = s;
    return LJ_OK;
}

lj_status lj_nve_start(lj_nve* s) {
    lj_ctx* ctx = s->ctx;
    lj_status st;
    if ((st = lj_launch_zero(ctx->stream, s->disp, s->list->n * 3 * (int64_t)sizeof(double))))
        return st;
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, ctx->stream, s->dstep, (int64_t)0);
    if ((st = forces(s, false))) return st;
    // kinetic energy of the initial velocities: a kick of zero length
    const dim3 grid((unsigned)s->rblocks), block(LJ_BLOCK);
    if (s->layout == LJ_AOS4)
        hipLaunchKernelGGL(k_kick<LJ_AOS4>, grid, block, 0, ctx->stream, row_args(s), 0.0);
    else
        hipLaunchKernelGGL(k_kick<LJ_SOA>, grid, block, 0, ctx->stream, row_args(s), 0.0);
    LJ_HIP(hipGetLastError());
    if ((st = log_row(s, 0))) return st;
    s->steps = 0;
    return LJ_OK;
}

lj_status lj_nve_advance(lj_nve* s, int32_t nsteps, int32_t use_graph) {
    lj_status st;
    const int64_t k = s->rebuild_every;
    int64_t left = nsteps;
    while (left > 0) {
        if (use_graph && s->steps % k == 0 && left >= k) {
            // a whole rebuild cycle: replay the captured graph
            if (!s->exec && (st = capture_cycle(s))) return st;
            LJ_HIP(hipGraphLaunch(s->exec, s->ctx->stream));
            s->steps += k;
            left -= k;
            continue;
        }
        // eagerly: with graphs, up to the next cycle boundary; without, all of it
        int64_t count = left;
        if (use_graph) count = std::min(left, k - s->steps % k);
        if ((st = chain(s, s->steps, count))) return st;
        s->steps += count;
        left -= count;
    }
    return LJ_OK;
}

void lj_nve_release(lj_nve* s) { release(s); }

int64_t lj_nve_step_count(const lj_nve* s) { return s->steps; }
