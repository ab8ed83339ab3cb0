// lj_nve.hip -- velocity-Verlet NVE integration around the force path, for a
// batch of independent systems (a single system is a batch of one).
//
// Per step k (unit mass):
//   drift    : v += F dt/2; dx = v dt; x += dx, wrapped into [0, L);
//              disp += dx (from 0 after a rebuild); per-block max |disp|^2
//   k_trigger: per system, the largest |disp|^2; with the displacement rule
//              (rebuild_every = 0) a device word decides the rebuild of this
//              step; with a fixed cadence a step between builds whose atoms
//              moved more than skin/2 raises the stale flag
//   [rebuild : cells + list in place, its kernels gated by that word]
//   forces   : F, per-system potential energy, virial, pair count
//   kick     : v += F dt/2; kinetic energy
//   k_log    : the system's log row (PE, KE, W, max displacement, pairs,
//              rebuilt)
// Two ways to place the kicks, with the same arithmetic (each kick rounded on
// its own) and so the same trajectory bit for bit:
//   separate (half lists, and the displacement rule): the kick that ends
//     step k and the drift that opens step k + 1 are one streaming kernel
//     (k_drift in its kick-and-drift mode); a chain of steps ends with a
//     kick of its own (k_kick);
//   folded into the force pass (full lists at a fixed cadence; the momentum
//     update of Alg. 1): the force kernel kicks each row's atom as soon as
//     its force is summed, twice inside a rebuild cycle (ending this step and
//     opening the next: the next drift only moves the atoms) and once before
//     a rebuild step and at the end of a chain (a synchronised velocity and a
//     stored force, which a rebuild step may have to restore).
// Rebuild steps are guarded: their drift first copies the step's starting
// positions and (synchronised) velocities aside, and if the rebuild meets a
// bad coordinate or an overflowing row, k_restore puts them back; from then
// on every force and integrator kernel of the context does nothing, so the
// run stops at its last good step (pos, vel, force of that step).
// The per-atom kernels take one thread per row of the list (256-row blocks,
// each inside one system), but the thread of a system's k-th row handles the
// system's k-th atom in memory order: the arrays stream instead of being
// gathered.  Every product and sum is rounded on its
// own, as in the oracle's integrator.  Bytes per atom (AoS4): kick-drift 208
// (reads vel, force, pos 32 each and disp 24; writes vel, pos, disp), drift
// alone 144 (no force, no velocity written), kick 88; a guarded drift writes
// 64 more; a folded kick adds 64 to the force pass (velocity read and
// written) and saves its 32-byte force store inside a cycle.  The force pass
// starts with its rank-ordered copy of the positions (56 bytes per atom).
#include <math.h>

#include <algorithm>

#include "lj_internal.h"

struct lj_nve {
    lj_ctx* ctx;
    lj_list* list;
    double *pos, *vel, *force, *log;
    int64_t log_rows;
    int layout, precision, trunc, rebuild_every, nsys;
    bool folded;           // kicks folded into the force pass
    double dt, half_skin2;
    lj_fconst* fc;         // device, nsys
    double* disp;          // n x 3: displacement since the last build
    double* kpart;         // per row block: kinetic energy (separate kicks)
    double* dpart;         // per row block: max |disp|^2 after the drift
    double* fpart;         // the force kernel's block partials (double4 records)
    int64_t fpart_cap;
    double* sysv;          // per system: PE, W, KE (force pass), max |disp|^2
    int64_t* npairs;       // per system
    int32_t* gate;         // 2 words: rebuild decided at even / odd steps
    int64_t* dstep;        // device step counter: log row of the current step
    double *bpos, *bvel;   // the starting state of a guarded step
    int32_t* armed;        // 1 while the current step's starting state is held in bpos/bvel
    int64_t steps;         // host step counter
    int64_t rblocks;       // 256-row blocks of the list
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipStream_t cap_stream;
};

namespace {

// Three components of one atom's record; w is the record's fourth double, kept as read.
struct Rec {
    double v[3];
    double w;
};

struct RowArgs {
    double* pos;
    double* vel;
    const double* force;
    double* disp;
    int64_t n;             // atoms over all systems (SoA stride)
    int rec;               // AoS: doubles per position/velocity record (4 or 8)
    const lj_sys* sys;
    const int32_t* slice_sys;
    int C;                 // rows per slice
    double* kpart;
    double* dpart;
    int64_t* dstep;
    int32_t* flags;        // the context's device status flags
    int32_t* gate;
    const lj_fconst* fc;   // per system: the fixed-point unit
    double* bpos;
    double* bvel;
    int32_t* armed;
};

template <int LAYOUT>
__device__ __forceinline__ Rec load_rec(const double* a, int64_t n, int rec, int64_t i) {
    Rec o;
    if constexpr (LAYOUT == LJ_AOS4) {
        const double4 q = *reinterpret_cast<const double4*>(a + i * rec);
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
__device__ __forceinline__ void store_rec(double* a, int64_t n, int rec, int64_t i, const Rec& o) {
    if constexpr (LAYOUT == LJ_AOS4) {
        *reinterpret_cast<double4*>(a + i * rec) = make_double4(o.v[0], o.v[1], o.v[2], o.w);
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) a[(int64_t)d * n + i] = o.v[d];
    }
}

__device__ __forceinline__ bool halted(const int32_t* flags) {
    return (__builtin_nontemporal_load(flags) & LJ_DEV_ERRORS) != 0;
}

// Kinds of drift kernel: what the velocity in memory is when the step opens.
enum { DRIFT_KICK = 0,        // synchronised: kick it with the stored force, then drift
       DRIFT_ONLY = 1 };      // already kicked by the force pass: drift only

// Drift of one atom (record index i) with velocity v (already kicked), and
// its displacement since the last build: from 0 when `reset`.
template <int LAYOUT>
__device__ __forceinline__ double drift_atom(const RowArgs& a, const lj_sys& sy, int64_t i,
                                             const Rec& v, double dt, bool reset) {
#pragma clang fp contract(off)
    Rec x = load_rec<LAYOUT>(a.pos, a.n, a.rec, i);
    double* u = a.disp + 3 * i;
    double un[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double L = sy.box[d];
        const double dx = dt * v.v[d];
        double xd = x.v[d] + dx;
        xd = xd - L * floor(xd / L);
        if (xd >= L) xd = 0.0;
        x.v[d] = xd;
        un[d] = (reset ? 0.0 : u[d]) + dx;
        u[d] = un[d];
    }
    store_rec<LAYOUT>(a.pos, a.n, a.rec, i, x);
    return (un[0] * un[0] + un[1] * un[1]) + un[2] * un[2];
}

// Half kick of one atom; returns its kinetic energy.
__device__ __forceinline__ double kick_atom(Rec& v, const Rec& f, double hdt) {
#pragma clang fp contract(off)
#pragma unroll
    for (int d = 0; d < 3; ++d) v.v[d] = v.v[d] + hdt * f.v[d];
    return 0.5 * ((v.v[0] * v.v[0] + v.v[1] * v.v[1]) + v.v[2] * v.v[2]);
}

// Fixed-order block sum (or max) of one value per thread; thread 0 stores it.
__device__ __forceinline__ void block_store(double v, bool is_max, double* out) {
    __shared__ double red[LJ_WAVES_PER_BLOCK];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const double o = __shfl_xor(v, d, LJ_WAVE);
        v = is_max ? fmax(v, o) : v + o;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < LJ_WAVES_PER_BLOCK; ++w) t = is_max ? fmax(t, red[w]) : t + red[w];
        *out = t;
    }
    __syncthreads();
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

// Opens step k (`parity` = k mod 2).  end_kick: first end step k - 1 with its
// kick (kinetic-energy partials for its log row).  mode: DRIFT_KICK or
// DRIFT_ONLY.  reset: the displacement restarts (a rebuild at step k - 1):
// 1 yes, 0 no, -1 as the device decided at step k - 1.  guard: copy the
// step's starting positions and velocities aside first.
template <int LAYOUT>
__global__ __launch_bounds__(LJ_BLOCK) void k_drift(RowArgs a, double hdt, double dt, int mode,
                                                    int end_kick, int reset, int guard,
                                                    int parity) {
    if (halted(a.flags)) {
        // an error is pending from before this step: nothing to restore
        if (blockIdx.x == 0 && threadIdx.x == 0) *a.armed = 0;
        return;
    }
    const lj_sys* sy;
    const int64_t i = row_to_atom(a, sy);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *a.dstep += 1;
        a.gate[parity] = 0;
        *a.armed = guard;
    }
    const bool rs = reset < 0 ? a.gate[parity ^ 1] != 0 : reset != 0;
    double ke = 0.0, d2 = 0.0;
    if (i >= 0) {
        Rec v = load_rec<LAYOUT>(a.vel, a.n, a.rec, i);
        Rec f;
        if (mode == DRIFT_KICK) {
            f = load_rec<LAYOUT == LJ_SOA ? LJ_SOA : LJ_AOS4>(a.force, a.n, 4, i);
            if (end_kick) ke = kick_atom(v, f, hdt);
        }
        if (guard) {
            store_rec<LAYOUT>(a.bvel, a.n, a.rec, i, v);
            store_rec<LAYOUT>(a.bpos, a.n, a.rec, i, load_rec<LAYOUT>(a.pos, a.n, a.rec, i));
        }
        if (mode == DRIFT_KICK) {
            (void)kick_atom(v, f, hdt);
            store_rec<LAYOUT>(a.vel, a.n, a.rec, i, v);
        }
        d2 = drift_atom<LAYOUT>(a, *sy, i, v, dt, rs);
    }
    if (end_kick) block_store(ke, false, a.kpart + blockIdx.x);
    block_store(d2, true, a.dpart + blockIdx.x);
}

// Ends a chain of steps: half kick with the new force; kinetic-energy partials.
template <int LAYOUT>
__global__ __launch_bounds__(LJ_BLOCK) void k_kick(RowArgs a, double hdt) {
    if (halted(a.flags)) return;
    const lj_sys* sy;
    const int64_t i = row_to_atom(a, sy);
    double ke = 0.0;
    if (i >= 0) {
        Rec v = load_rec<LAYOUT>(a.vel, a.n, a.rec, i);
        const Rec f = load_rec<LAYOUT == LJ_SOA ? LJ_SOA : LJ_AOS4>(a.force, a.n, 4, i);
        ke = kick_atom(v, f, hdt);
        store_rec<LAYOUT>(a.vel, a.n, a.rec, i, v);
    }
    block_store(ke, false, a.kpart + blockIdx.x);
}

// After the rebuild of a guarded step: if it met a bad coordinate or an
// overflowing row (and the step's drift ran, so its starting state is held
// aside), put back the starting positions and velocities and step the device
// counter back to the last good step.  Atoms in memory order, grid-stride.
template <int LAYOUT>
__global__ __launch_bounds__(LJ_BLOCK) void k_restore(RowArgs a) {
    if (!halted(a.flags) || __builtin_nontemporal_load(a.armed) == 0) return;
    for (int64_t i = blockIdx.x * (int64_t)LJ_BLOCK + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * LJ_BLOCK) {
        store_rec<LAYOUT>(a.pos, a.n, a.rec, i, load_rec<LAYOUT>(a.bpos, a.n, a.rec, i));
        store_rec<LAYOUT>(a.vel, a.n, a.rec, i, load_rec<LAYOUT>(a.bvel, a.n, a.rec, i));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *a.dstep -= 1;
        atomicOr(a.flags, LJ_DEV_RESTORED);
    }
}

// Fixed-order sum (or max) over the row-block partials [b0, b1) by one
// 1024-thread block (four loads in flight per thread and pass); valid in
// thread 0.
__device__ double span_reduce(const double* __restrict__ p, int64_t b0, int64_t b1, bool is_max) {
    __shared__ double red[16];
    double v = 0.0;
    for (int64_t bb = b0 + threadIdx.x; bb < b1; bb += 4 * 1024) {
        double x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t b = bb + u * 1024;
            x[u] = b < b1 ? p[b] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) v = is_max ? fmax(v, x[u]) : v + x[u];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const double o = __shfl_xor(v, d, LJ_WAVE);
        v = is_max ? fmax(v, o) : v + o;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < 16; ++w) t = is_max ? fmax(t, red[w]) : t + red[w];
    return t;
}

// One block per system after the drift of step k: the system's largest
// |disp|^2 (kept for the log); mode 1 (displacement rule): a system beyond
// (skin/2)^2 makes step k rebuild every system; mode 2 (fixed cadence, no
// rebuild at this step): such a system raises the stale flag.
__global__ __launch_bounds__(1024) void k_trigger(const double* __restrict__ dpart,
                                                  const lj_sys* sys, int C, double half_skin2,
                                                  int mode, int parity, int32_t* flags,
                                                  int32_t* gate, double* sysv, int nsys) {
    if (halted(flags)) return;
    const int s = blockIdx.x;
    const lj_sys& sy = sys[s];
    const int64_t b0 = sy.slice0 * C / LJ_BLOCK, b1 = (sy.slice0 + sy.nslices) * C / LJ_BLOCK;
    const double m = span_reduce(dpart, b0, b1, true);
    if (threadIdx.x == 0) {
        sysv[3 * nsys + s] = m;
        if (m > half_skin2) {
            if (mode == 1) atomicOr(gate + parity, 1);
            if (mode == 2) atomicOr(flags, LJ_DEV_STALE);
        }
    }
}

// One block per system: the log row of step *dstep + back (back = -1 after
// a drift has opened the next step).  Kinetic energy from the force pass
// (sysv) or from the kick partials; the displacement from k_trigger, 0 at a
// step that rebuilt.  rebuilt: 1, 0, or -1 as the device decided
// (gate[parity]).
__global__ __launch_bounds__(1024) void k_log(const double* __restrict__ kpart, int ke_folded,
                                              const lj_sys* sys, int C, const double* sysv,
                                              const int64_t* npairs, const int64_t* dstep,
                                              int back, const int32_t* flags,
                                              const int32_t* gate, int rebuilt, int parity,
                                              double* log, int64_t log_rows, int nsys) {
    if (halted(flags)) return;
    const int s = blockIdx.x;
    const lj_sys& sy = sys[s];
    double k = 0.0;
    if (!ke_folded) {
        const int64_t b0 = sy.slice0 * C / LJ_BLOCK, b1 = (sy.slice0 + sy.nslices) * C / LJ_BLOCK;
        k = span_reduce(kpart, b0, b1, false);
    }
    if (threadIdx.x == 0) {
        if (ke_folded) k = sysv[2 * nsys + s];
        const bool rb = rebuilt < 0 ? gate[parity] != 0 : rebuilt != 0;
        const int64_t row = *dstep + back;
        if (row >= 0 && row < log_rows) {
            double* out = log + 6 * (row * nsys + s);
            out[0] = sysv[s];
            out[1] = k;
            out[2] = sysv[nsys + s];
            out[3] = rb ? 0.0 : sqrt(sysv[3 * nsys + s]);
            out[4] = (double)npairs[s];
            out[5] = rb ? 1.0 : 0.0;
        }
    }
}

__global__ void k_set_state(int64_t* dstep, int32_t* gate, int32_t* armed) {
    *dstep = 0;
    gate[0] = 0;
    gate[1] = 0;
    *armed = 0;
}

int tmpl(const lj_nve* s) { return lj_tmpl_layout(s->layout); }

RowArgs row_args(lj_nve* s) {
    RowArgs a;
    a.pos = s->pos;
    a.vel = s->vel;
    a.force = s->force;
    a.disp = s->disp;
    a.n = s->list->n;
    a.rec = s->layout == LJ_AOS8 ? 8 : 4;
    a.sys = s->list->dsys;
    a.slice_sys = s->list->slice_sys;
    a.C = LJ_WAVE / s->list->lanes;
    a.kpart = s->kpart;
    a.dpart = s->dpart;
    a.dstep = s->dstep;
    a.flags = &s->ctx->st->flags;
    a.gate = s->gate;
    a.fc = s->fc;
    a.bpos = s->bpos;
    a.bvel = s->layout == LJ_AOS8 ? s->bpos + 4 : s->bvel;
    a.armed = s->armed;
    return a;
}

// The force pass of a step: kick = LJ_KICK_* (folded kicks write the
// kinetic energy next to the potential energy).
lj_status forces(lj_nve* s, int kick) {
    lj_force_opts o;
    o.partials = s->fpart;
    o.partials_cap = s->fpart_cap;
    o.trunc = s->trunc;
    o.kick = kick;
    o.vel = s->vel;
    o.hdt = 0.5 * s->dt;
    o.write_f = kick != LJ_KICK_LEAP;
    o.kinetic = s->sysv + 2 * s->nsys;
    return lj_launch_forces(s->ctx, s->pos, s->layout, s->precision, s->list, s->fc, s->force,
                            s->sysv, s->sysv + s->nsys, s->npairs, o);
}

lj_status log_row(lj_nve* s, bool ke_folded, int back, int rebuilt, int parity) {
    lj_prof_scope prof(s->ctx, LJ_PROF_INTEGRATE);
    hipLaunchKernelGGL(k_log, dim3((unsigned)s->nsys), dim3(1024), 0, s->ctx->stream,
                       (const double*)s->kpart, ke_folded ? 1 : 0, (const lj_sys*)s->list->dsys,
                       LJ_WAVE / s->list->lanes, (const double*)s->sysv,
                       (const int64_t*)s->npairs, (const int64_t*)s->dstep, back,
                       (const int32_t*)&s->ctx->st->flags, (const int32_t*)s->gate, rebuilt,
                       parity, s->log, s->log_rows, s->nsys);
    LJ_HIP(hipGetLastError());
    return LJ_OK;
}

// Steps first + 1 .. first + count as one chain (the chain starts and ends
// with synchronised velocities and stored forces).
template <int LAYOUT>
lj_status enqueue_chain(lj_nve* s, int64_t first, int64_t count) {
    lj_ctx* ctx = s->ctx;
    const dim3 grid((unsigned)s->rblocks), block(LJ_BLOCK);
    const RowArgs a = row_args(s);
    const double hdt = 0.5 * s->dt, dt = s->dt;
    const int every = s->rebuild_every;
    const bool trig = every == 0;
    const int C = LJ_WAVE / s->list->lanes;
    lj_status st;
    bool leapt = false;        // the velocity in memory was kicked ahead by the force pass
    for (int64_t k = 1; k <= count; ++k) {
        const int64_t step = first + k;
        const int parity = (int)(step & 1);
        const bool rebuild = trig || step % every == 0;   // trig: decided on the device
        const bool rebuilt_before = !trig && (step - 1) % every == 0;
        {
            lj_prof_scope prof(ctx, LJ_PROF_INTEGRATE);
            const int mode = leapt ? DRIFT_ONLY : DRIFT_KICK;
            const int end_kick = (!s->folded && k > 1) ? 1 : 0;
            const int reset = trig ? -1 : (rebuilt_before ? 1 : 0);
            hipLaunchKernelGGL(k_drift<LAYOUT>, grid, block, 0, ctx->stream, a, hdt, dt, mode,
                               end_kick, reset, rebuild ? 1 : 0, parity);
            LJ_HIP(hipGetLastError());
        }
        if (!s->folded && k > 1) {
            // the log row of the previous step, whose kick the drift just took
            if ((st = log_row(s, false, -1, trig ? -1 : (rebuilt_before ? 1 : 0), parity ^ 1)))
                return st;
        }
        {
            lj_prof_scope prof(ctx, LJ_PROF_INTEGRATE);
            hipLaunchKernelGGL(k_trigger, dim3((unsigned)s->nsys), dim3(1024), 0, ctx->stream,
                               (const double*)s->dpart, (const lj_sys*)s->list->dsys, C,
                               s->half_skin2, trig ? 1 : (rebuild ? 0 : 2), parity,
                               &ctx->st->flags, s->gate, s->sysv, s->nsys);
            LJ_HIP(hipGetLastError());
        }
        if (rebuild) {
            lj_list* l = s->list;
            const int32_t* gate = trig ? s->gate + parity : nullptr;
            if ((st = lj_launch_cells(ctx, s->pos, s->layout, l->cells, gate))) return st;
            if ((st = lj_launch_neighbors(ctx, l->cells, l, false, gate))) return st;
            lj_prof_scope prof(ctx, LJ_PROF_INTEGRATE);
            const dim3 rgrid((unsigned)std::min<int64_t>(s->rblocks, 1024));
            hipLaunchKernelGGL(k_restore<LAYOUT>, rgrid, block, 0, ctx->stream, a);
            LJ_HIP(hipGetLastError());
        }
        if (s->folded) {
            // kick twice unless the next step may rebuild or the chain ends here
            const bool next_guarded = (step + 1) % every == 0;
            const int kick = (k == count || next_guarded) ? LJ_KICK_SYNC : LJ_KICK_LEAP;
            if ((st = forces(s, kick))) return st;
            leapt = kick == LJ_KICK_LEAP;
            if ((st = log_row(s, true, 0, rebuild ? 1 : 0, parity))) return st;
        } else {
            if ((st = forces(s, LJ_KICK_NONE))) return st;
        }
    }
    if (!s->folded) {
        {
            lj_prof_scope prof(ctx, LJ_PROF_INTEGRATE);
            hipLaunchKernelGGL(k_kick<LAYOUT>, grid, block, 0, ctx->stream, a, hdt);
            LJ_HIP(hipGetLastError());
        }
        const int64_t last = first + count;
        const int rb = trig ? -1 : (last % every == 0 ? 1 : 0);
        if ((st = log_row(s, false, 0, rb, (int)(last & 1)))) return st;
    }
    return LJ_OK;
}

lj_status chain(lj_nve* s, int64_t first, int64_t count) {
    if (count <= 0) return LJ_OK;
    return tmpl(s) == LJ_AOS4 ? enqueue_chain<LJ_AOS4>(s, first, count)
                              : enqueue_chain<LJ_SOA>(s, first, count);
}

void release(lj_nve* s) {
    if (!s) return;
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    void* bufs[] = {s->fc, s->disp, s->kpart, s->dpart, s->fpart, s->sysv, s->npairs,
                    s->gate, s->dstep, s->bpos, s->bvel, s->armed};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    delete s;
}

// Steps of one captured cycle: a rebuild cycle at a fixed cadence, else 10.
int64_t cycle_len(const lj_nve* s) { return s->rebuild_every > 0 ? s->rebuild_every : 10; }

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
        st = chain(s, 0, cycle_len(s));
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

template <typename T>
hipError_t alloc(T** p, int64_t count) {
    return hipMalloc((void**)p, (size_t)std::max<int64_t>(count, 1) * sizeof(T));
}

}  // namespace

lj_status lj_nve_make(lj_ctx* ctx, double* pos, double* vel, double* force, int32_t layout,
                      const lj_fconst* hfc, int32_t precision, int32_t trunc, lj_list* list,
                      double dt, int32_t rebuild_every, double* log, int64_t log_rows,
                      lj_nve** out) {
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
    s->trunc = trunc;
    s->rebuild_every = rebuild_every;
    s->folded = list->kind == LJ_LIST_FULL && rebuild_every > 0 && ctx->tune[LJ_TUNE_KICK] != 2;
    s->nsys = list->nsys;
    s->dt = dt;
    s->half_skin2 = 0.25 * list->hsys[0].skin * list->hsys[0].skin;
    s->rblocks = list->nslices * (LJ_WAVE / list->lanes) / LJ_BLOCK;
    s->fpart_cap = lj_force_partials(list);
    const int64_t n = list->n;
    const int64_t rec = layout == LJ_AOS8 ? 8 : (layout == LJ_AOS4 ? 4 : 3);
    hipError_t e = alloc(&s->disp, n * 3);
    if (e == hipSuccess) e = alloc(&s->fc, s->nsys);
    if (e == hipSuccess) e = alloc(&s->kpart, s->rblocks);
    if (e == hipSuccess) e = alloc(&s->dpart, s->rblocks);
    if (e == hipSuccess) e = alloc(&s->fpart, 4 * s->fpart_cap);
    if (e == hipSuccess) e = alloc(&s->sysv, 4 * (int64_t)s->nsys);
    if (e == hipSuccess) e = alloc(&s->npairs, s->nsys);
    if (e == hipSuccess) e = alloc(&s->gate, 2);
    if (e == hipSuccess) e = alloc(&s->dstep, 1);
    if (e == hipSuccess) e = alloc(&s->armed, 1);
    if (e == hipSuccess) e = alloc(&s->bpos, n * rec);
    if (e == hipSuccess && layout != LJ_AOS8) e = alloc(&s->bvel, n * rec);
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
    if ((st = lj_launch_zero(ctx->stream, s->sysv, 4 * (int64_t)s->nsys * sizeof(double))))
        return st;
    hipLaunchKernelGGL(k_set_state, dim3(1), dim3(1), 0, ctx->stream, s->dstep, s->gate,
                       s->armed);
    LJ_HIP(hipGetLastError());
    if ((st = forces(s, LJ_KICK_NONE))) return st;
    // kinetic energy of the initial velocities: a kick of zero length
    const dim3 grid((unsigned)s->rblocks), block(LJ_BLOCK);
    if (tmpl(s) == LJ_AOS4)
        hipLaunchKernelGGL(k_kick<LJ_AOS4>, grid, block, 0, ctx->stream, row_args(s), 0.0);
    else
        hipLaunchKernelGGL(k_kick<LJ_SOA>, grid, block, 0, ctx->stream, row_args(s), 0.0);
    LJ_HIP(hipGetLastError());
    if ((st = log_row(s, false, 0, 1, 0))) return st;
    s->steps = 0;
    return LJ_OK;
}

lj_status lj_nve_advance(lj_nve* s, int32_t nsteps, int32_t use_graph) {
    lj_status st;
    const int64_t k = cycle_len(s);
    int64_t left = nsteps;
    while (left > 0) {
        if (use_graph && s->steps % k == 0 && left >= k) {
            // a whole cycle: replay the captured graph
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

lj_status lj_nve_device_steps(lj_nve* s, int64_t* steps) {
    LJ_HIP(hipMemcpyAsync(steps, s->dstep, sizeof(int64_t), hipMemcpyDeviceToHost,
                          s->ctx->stream));
    LJ_HIP(hipStreamSynchronize(s->ctx->stream));
    return LJ_OK;
}

void lj_nve_release(lj_nve* s) { release(s); }
