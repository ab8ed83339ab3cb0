// lj_nve.hip -- velocity-Verlet NVE integration around the force path.
//
// Per step (unit mass):
//   k_drift : v += F dt/2; dx = v dt; x += dx, wrapped into [0, L);
//             disp += dx, or disp = 0 at a rebuild step
//   [rebuild: cells + list in place]
//   forces  : F, potential energy, virial, pair count (lj_launch_forces)
//   k_kick  : v += F dt/2; per-block partial sums of v^2/2 and max |disp|^2
//   k_log   : one block sums the partials in a fixed order and writes the
//             step's log row (PE, KE, W, max displacement, pairs)
// Every product and sum is rounded on its own, as in the oracle's integrator.
// Streaming kernels: about 100 bytes per atom per step, HBM bound.
#include <math.h>

#include "lj_internal.h"

struct lj_nve {
    lj_ctx* ctx;
    lj_list* list;
    double *pos, *vel, *force, *log;
    int64_t n, log_rows;
    int layout, precision, rebuild_every;
    double dt, box[3];
    lj_force_params fp;
    double* disp;          // n x 3: displacement since the last build
    double* partials;      // 2 per block: kinetic energy, max |disp|^2
    double* scratch;       // potential energy, virial
    int64_t* npairs;       // device
    int64_t* dstep;        // device step counter (row of the next log entry - 1)
    int64_t steps;         // host step counter
    int64_t blocks;
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipStream_t cap_stream;
};

namespace {

template <int LAYOUT>
__device__ __forceinline__ double* comp(double* a, int64_t n, int64_t i, int d) {
    return LAYOUT == LJ_AOS4 ? a + 4 * i + d : a + (int64_t)d * n + i;
}

template <int LAYOUT>
__global__ __launch_bounds__(LJ_BLOCK) void k_drift(double* __restrict__ pos,
                                                    double* __restrict__ vel,
                                                    const double* __restrict__ force,
                                                    double* __restrict__ disp, int64_t n,
                                                    double hdt, double dt, double Lx, double Ly,
                                                    double Lz, int reset) {
#pragma clang fp contract(off)
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double L[3] = {Lx, Ly, Lz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double* pv = comp<LAYOUT>(vel, n, i, d);
        double* px = comp<LAYOUT>(pos, n, i, d);
        const double f = *comp<LAYOUT>(const_cast<double*>(force), n, i, d);
        const double v = *pv + hdt * f;
        const double dx = dt * v;
        double x = *px + dx;
        x = x - L[d] * floor(x / L[d]);
        if (x >= L[d]) x = 0.0;
        *pv = v;
        *px = x;
        disp[3 * i + d] = reset ? 0.0 : disp[3 * i + d] + dx;
    }
}

template <int LAYOUT>
__global__ __launch_bounds__(LJ_BLOCK) void k_kick(double* __restrict__ vel,
                                                   const double* __restrict__ force,
                                                   const double* __restrict__ disp, int64_t n,
                                                   double hdt, double* __restrict__ partials) {
#pragma clang fp contract(off)
    __shared__ double red[LJ_WAVES_PER_BLOCK][2];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double ke = 0.0, d2 = 0.0;
    if (i < n) {
        double v[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double* pv = comp<LAYOUT>(vel, n, i, d);
            v[d] = *pv + hdt * *comp<LAYOUT>(const_cast<double*>(force), n, i, d);
            *pv = v[d];
        }
        ke = 0.5 * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
        const double* u = disp + 3 * i;
        d2 = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
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
        for (int w = 0; w < LJ_WAVES_PER_BLOCK; ++w) {
            k += red[w][0];
            m = fmax(m, red[w][1]);
        }
        partials[2 * blockIdx.x] = k;
        partials[2 * blockIdx.x + 1] = m;
    }
}

// One block: fixed-order sums of the partials, then the log row of the step.
// first != 0: step 0 (row 0, counter reset); else row = counter + 1.
__global__ __launch_bounds__(1024) void k_log(const double* __restrict__ partials,
                                              int64_t nblocks, const double* pe_w,
                                              const int64_t* npairs, int64_t* dstep,
                                              double* log, int64_t log_rows, int first) {
    __shared__ double red[16][2];
    double ke = 0.0, d2 = 0.0;
    for (int64_t b = threadIdx.x; b < nblocks; b += 1024) {
        ke += partials[2 * b];
        d2 = fmax(d2, partials[2 * b + 1]);
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
        const int64_t row = first ? 0 : *dstep + 1;
        *dstep = row;
        if (row < log_rows) {
            double* r = log + 5 * row;
            r[0] = pe_w[0];
            r[1] = k;
            r[2] = pe_w[1];
            r[3] = sqrt(m);
            r[4] = (double)*npairs;
        }
    }
}

template <int LAYOUT>
lj_status enqueue_step(lj_nve* s, bool rebuild) {
    lj_ctx* ctx = s->ctx;
    const dim3 grid((unsigned)s->blocks), block(LJ_BLOCK);
    hipLaunchKernelGGL(k_drift<LAYOUT>, grid, block, 0, ctx->stream, s->pos, s->vel,
                       (const double*)s->force, s->disp, s->n, 0.5 * s->dt, s->dt, s->box[0],
                       s->box[1], s->box[2], rebuild ? 1 : 0);
    LJ_HIP(hipGetLastError());
    lj_status st;
    if (rebuild) {
        lj_list* l = s->list;
        if ((st = lj_launch_cells(ctx, s->pos, s->layout, l->cells))) return st;
        if ((st = lj_launch_neighbors(ctx, l->cells, l, l->rc + l->skin))) return st;
    }
    if ((st = lj_launch_forces(ctx, s->pos, s->list, s->fp, s->force, s->scratch,
                               s->scratch + 1, s->npairs)))
        return st;
    hipLaunchKernelGGL(k_kick<LAYOUT>, grid, block, 0, ctx->stream, s->vel,
                       (const double*)s->force, (const double*)s->disp, s->n, 0.5 * s->dt,
                       s->partials);
    hipLaunchKernelGGL(k_log, dim3(1), dim3(1024), 0, ctx->stream, (const double*)s->partials,
                       s->blocks, (const double*)s->scratch, (const int64_t*)s->npairs, s->dstep,
                       s->log, s->log_rows, 0);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}

lj_status step(lj_nve* s, bool rebuild) {
    return s->layout == LJ_AOS4 ? enqueue_step<LJ_AOS4>(s, rebuild)
                                : enqueue_step<LJ_SOA>(s, rebuild);
}

void release(lj_nve* s) {
    if (!s) return;
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    if (s->disp) (void)hipFree(s->disp);
    if (s->partials) (void)hipFree(s->partials);
    if (s->scratch) (void)hipFree(s->scratch);
    if (s->npairs) (void)hipFree(s->npairs);
    if (s->dstep) (void)hipFree(s->dstep);
    delete s;
}

}  // namespace

lj_status lj_nve_make(lj_ctx* ctx, double* pos, double* vel, double* force, int64_t n,
                      int32_t layout, const double box[3], double eps, double sigma, double rc,
                      int32_t precision, lj_list* list, double dt, int32_t rebuild_every,
                      double* log, int64_t log_rows, lj_nve** out) {
    lj_nve* s = new (std::nothrow) lj_nve();
    if (!s) return lj_fail(LJ_E_NOMEM, "host allocation");
    s->ctx = ctx;
    s->list = list;
    s->pos = pos;
    s->vel = vel;
    s->force = force;
    s->log = log;
    s->n = n;
    s->log_rows = log_rows;
    s->layout = layout;
    s->precision = precision;
    s->rebuild_every = rebuild_every;
    s->dt = dt;
    for (int d = 0; d < 3; ++d) {
        s->box[d] = box[d];
        s->fp.box[d] = box[d];
    }
    s->fp.eps = eps;
    s->fp.sigma = sigma;
    s->fp.rc = rc;
    s->fp.layout = layout;
    s->fp.precision = precision;
    s->blocks = (n + LJ_BLOCK - 1) / LJ_BLOCK;
    hipError_t e = hipMalloc((void**)&s->disp, (size_t)n * 3 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&s->partials, (size_t)s->blocks * 2 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&s->scratch, 2 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&s->npairs, sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc((void**)&s->dstep, sizeof(int64_t));
    if (e != hipSuccess) {
        release(s);
        return lj_hip_fail(e, "hipMalloc");
    }
    *out = s;
    return LJ_OK;
}

lj_status lj_nve_start(lj_nve* s) {
    lj_ctx* ctx = s->ctx;
    lj_status st;
    if ((st = lj_launch_zero(ctx->stream, s->disp, s->n * 3 * (int64_t)sizeof(double)))) return st;
    if ((st = lj_launch_forces(ctx, s->pos, s->list, s->fp, s->force, s->scratch, s->scratch + 1,
                               s->npairs)))
        return st;
    // kinetic energy of the initial velocities: a kick of zero length
    const dim3 grid((unsigned)s->blocks), block(LJ_BLOCK);
    if (s->layout == LJ_AOS4)
        hipLaunchKernelGGL(k_kick<LJ_AOS4>, grid, block, 0, ctx->stream, s->vel,
                           (const double*)s->force, (const double*)s->disp, s->n, 0.0,
                           s->partials);
    else
        hipLaunchKernelGGL(k_kick<LJ_SOA>, grid, block, 0, ctx->stream, s->vel,
                           (const double*)s->force, (const double*)s->disp, s->n, 0.0,
                           s->partials);
    hipLaunchKernelGGL(k_log, dim3(1), dim3(1024), 0, ctx->stream, (const double*)s->partials,
                       s->blocks, (const double*)s->scratch, (const int64_t*)s->npairs, s->dstep,
                       s->log, s->log_rows, 1);
    LJ_HIP(hipGetLastError());
    s->steps = 0;
    return LJ_OK;
}

static lj_status capture_cycle(lj_nve* s) {
    lj_ctx* ctx = s->ctx;
    if (!s->cap_stream) LJ_HIP(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    hipStream_t saved = ctx->stream;
    const bool prof = ctx->prof_on;
    ctx->prof_on = false;
    ctx->stream = s->cap_stream;
    lj_status st = LJ_OK;
    hipError_t e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        st = lj_hip_fail(e, "hipStreamBeginCapture");
    } else {
        for (int k = 1; k <= s->rebuild_every && !st; ++k) st = step(s, k == s->rebuild_every);
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
        const int64_t next = s->steps + 1;
        if ((st = step(s, next % k == 0))) return st;
        s->steps = next;
        --left;
    }
    return LJ_OK;
}

void lj_nve_release(lj_nve* s) { release(s); }

int64_t lj_nve_step_count(const lj_nve* s) { return s->steps; }
