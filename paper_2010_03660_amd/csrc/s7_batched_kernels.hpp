// Batched form: many independent BiCGStab systems of uneven size in one
// persistent launch.  The paper motivates this (section VIII-B) with many
// compact problems solved together, and with the four solves per timestep of
// its application (Algorithm 2).
//
// Execution model (no grid barrier, no fence):
// * A work item is (system, phase, chunk), where a chunk is `chunk_cells`
//   consecutive cells of one system.  The phases of an iteration are P1, P2
//   and P3, the three-pass schedule of the single-system path: P2 forms
//   q = r - alpha s on the fly, and P3 forms it again.
//   Around the iteration a job also runs, on the device, its epilogue and
//   its refinement steps: X (x += scale d), R (the FP64 residual) and I (the
//   next inner right-hand side), so a job needs the host only to start.
// * Each system owns a 64-bit claim word, (phase sequence << 32) | next chunk;
//   the low three bits of the sequence name the phase.
//   A workgroup claims a chunk with one atomic add, which tells it both the
//   chunk and the phase it belongs to.  Claims past the last chunk are
//   ignored.
// * A workgroup publishes its chunk's partial sums, then counts itself done.
//   The workgroup completing a phase sums that system's partials in unit
//   order (one partial per 1024 cells, summed by one wavefront), runs the
//   scalar step of Algorithm 1 on a private copy of the state, stores it, and
//   opens the next phase by storing the next sequence into the claim word.
//   The sum order is fixed per system, so a system's iterates depend neither
//   on the rest of the batch, nor on scheduling, nor on the chunk size.
// * Everything one workgroup hands to another inside the launch goes through
//   device-scope (coherent) loads and stores: the Krylov vectors, partials,
//   state and control words.  Each XCD's L2 is private and not coherent with
//   the others.  Release fences would restore coherence only by writing back
//   a whole L2 per hand-off, at tens of nanoseconds each, serialized.
// * Every wait is bounded.  A workgroup that finds no work spins with
//   s_sleep.  After `spin_limit` fruitless tries it records an error and
//   leaves, and the launch always drains.
// * Each system names its operator: OP_7PT, the 3D 7-point stencil, or
//   OP_9PT, the 2D 9-point stencil of section IV.  One launch may hold
//   systems of both.
// Included by the solver translation unit (s7_single.hip) only.
#pragma once

#include <hip/hip_runtime.h>

#include "s7_device.hpp"
#include "s7_stencil9_device.hpp"

namespace s7 {

// ---------------------------------------------------------------- coherent access
template <class T>
struct Bits;
template <>
struct Bits<float> {
    using U = uint32_t;
};
template <>
struct Bits<bf16> {
    using U = uint16_t;
};
template <>
struct Bits<f16> {
    using U = uint16_t;
};
template <>
struct Bits<double> {
    using U = uint64_t;
};

template <class T>
__device__ __forceinline__ T cload(const T* p) {
    using U = typename Bits<T>::U;
    const U u = __hip_atomic_load(gbl(reinterpret_cast<U*>(const_cast<T*>(p))), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(T, u);
}
template <class T>
__device__ __forceinline__ void cstore(T* p, T v) {
    using U = typename Bits<T>::U;
    __hip_atomic_store(gbl(reinterpret_cast<U*>(p)), __builtin_bit_cast(U, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double cload_d(const double* p) { return fetch_published(p); }
__device__ __forceinline__ void cstore_d(double* p, double v) { publish(p, v); }
__device__ __forceinline__ int32_t cload_i(const int32_t* p) {
    return __hip_atomic_load(gbl(const_cast<int32_t*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void cstore_i(int32_t* p, int32_t v) {
    __hip_atomic_store(gbl(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ Nbr<T> cload_nbr(const T* v, const Cell& c) {
    const T* p = v + c.idx;
    return Nbr<T>{cload(p), cload(p + c.dw), cload(p + c.de), cload(p + c.ds),
                  cload(p + c.dn), cload(p + c.db), cload(p + c.dt)};
}

// The State copied between memory and an LDS copy with coherent accesses, one
// 4-byte word per thread of the workgroup, so that a copy costs one round trip
// to memory rather than one per word.  Called by every thread.
constexpr int kStateWords = (int)(sizeof(State) / 4);
static_assert(sizeof(State) % 4 == 0 && kStateWords <= kThreads, "State is copied one word per thread");
// state_fetch loads this thread's word; state_put stores it into the LDS copy
// (the load may still be in flight between the two).
__device__ __forceinline__ uint32_t state_fetch(const State* src) {
    const int w = (int)threadIdx.x;
    return w < kStateWords ? __hip_atomic_load(gbl(const_cast<uint32_t*>(reinterpret_cast<const uint32_t*>(src) + w)),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                           : 0u;
}
__device__ __forceinline__ void state_put(uint32_t word, State& dst) {
    const int w = (int)threadIdx.x;
    if (w < kStateWords) reinterpret_cast<uint32_t*>(&dst)[w] = word;
    __syncthreads();
}
// Each thread waits until its word has reached memory.
__device__ __forceinline__ void state_store(State* dst, const State& src) {
    const int w = (int)threadIdx.x;
    if (w < kStateWords) {
        __hip_atomic_store(gbl(reinterpret_cast<uint32_t*>(dst) + w), reinterpret_cast<const uint32_t*>(&src)[w],
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_stores();
    }
}

// ---------------------------------------------------------------- tables
// One system of a batch.  The view is stored with FP32 element pointers and
// re-typed by `tag` (TypeTag of the storage type); the pointer members are
// identical in every instantiation.  Red.part holds kMaxDots sums per unit of
// kUnitCells cells.
struct BCtl;

enum OpKind : int { OP_7PT = 0, OP_9PT = 1 };

struct BSys {
    SysView<float> S;
    BCtl* ctl;   // the system's control words (in its own workspace slice)
    int nchunk;
    int tag;
    int budget;  // iterations this system may run in the launch
    int chunk;   // cells per work item (a multiple of kUnitCells)
    int op;      // OpKind of the system
    int pad;
    Coef7 cf;    // the caller's FP32 coefficients (residual passes)
    const double* b;
    double* x;
    // OP_9PT: the caller's coefficients 7 and 8 (nw, ne), and the working
    // copies of coefficients 7 and 8 (the first seven are in S)
    const float* cf9[2];
    const float* wk9[2];
};

// Phases of a job.  An iteration is P1, P2, P3.  Around the inner
// iteration: S (an FP32 job's start: r0 = b - A x0), X (x += scale d), R (FP64
// residual b - A x) and, for refinement, I (next inner right-hand side
// r = r0 = p = d / scale).  A refinement job starts at R.  A phase sequence
// number is (count << 3) | kind.
enum PhaseKind : int { K_P1 = 0, K_P2 = 1, K_P3 = 2, K_X = 3, K_R = 4, K_I = 5, K_S = 6, K_FINAL = 7 };
constexpr int kND[7] = {1, 5, 2, 0, 3, 1, 3};  // sums of each phase
__host__ __device__ inline uint32_t seq_next(uint32_t seq, int kind) {
    return (((seq >> 3) + 1u) << 3) | (uint32_t)kind;
}

template <class T>
__device__ __forceinline__ SysView<T> as_view(const SysView<float>& v) {
    SysView<T> o;
    o.m = v.m;
    o.n = v.n;
    o.unit = v.unit;
    for (int a = 0; a < 7; ++a) o.c[a] = reinterpret_cast<const T*>(v.c[a]);
    o.r = reinterpret_cast<T*>(v.r);
    o.rhat = reinterpret_cast<T*>(v.rhat);
    o.p = reinterpret_cast<T*>(v.p);
    o.s = reinterpret_cast<T*>(v.s);
    o.y = reinterpret_cast<T*>(v.y);
    o.q = reinterpret_cast<T*>(v.q);
    o.d = v.d;
    o.st = v.st;
    o.red = v.red;
    o.cell_blocks = v.cell_blocks;
    o.stream_blocks = v.stream_blocks;
    o.pair_blocks = v.pair_blocks;
    return o;
}

struct BCtl {
    unsigned long long claim;  // (phase sequence << 32) | next chunk
    uint32_t done_cnt;         // chunks finished in the current phase
    int32_t budget;            // iterations this launch may still run
    int32_t active;            // 1 while the system takes part in this launch
    int32_t pad;
};

// Restarts a system's phase sequence at phase `kind`.
__global__ void k_ctl_reset(BCtl* ctl, int kind) {
    if (threadIdx.x == 0) {
        ctl->claim = (unsigned long long)kind << 32;
        ctl->done_cnt = 0u;
        ctl->budget = 0;
        ctl->active = 0;
    }
}

// One new job of a batch (a table of these is filled by the host).  The
// start kernel writes its working-precision coefficient copies and sets its
// State and control words; its first phase then runs in the persistent
// launch.  Coefficient copies are read there with plain loads, so they must be
// written by an earlier kernel, not by a phase of the same launch.
struct JobStart {
    Coef7 cf;        // the caller's FP32 coefficients
    const float* cf9[2];  // OP_9PT: the caller's coefficients 7 and 8
    void* coef_dst;  // first working-precision copy; copies are `span` elements apart
    size_t span;
    Mesh m;
    int n, jacobi, tag, first;  // first: the first phase (K_S, or K_R for refinement)
    State* st;
    uint32_t* cnt;
    BCtl* ctl;
    double rtol, inner_tol;
    int inner_cap, outer_cap, max_total, ir, op;
};

template <class T>
__device__ void start_coef_copies(const JobStart& J, int i0, int step) {
    const int first = J.jacobi ? 1 : 0;
    T* dst0 = reinterpret_cast<T*>(J.coef_dst);
    for (int i = i0; i < J.n; i += step) {
        const Cell c = cell_at(i, J.m, J.n);
        const bool in[7] = {true, c.dw != 0, c.de != 0, c.ds != 0, c.dn != 0, c.db != 0, c.dt != 0};
        const float dg = J.cf.c[0][i];
#pragma unroll
        for (int a = 0; a < 7; ++a) {
            if (a < first) continue;
            float v = in[a] ? J.cf.c[a][i] : 0.0f;
            if (J.jacobi) v = v / dg;
            dst0[(size_t)(a - first) * J.span + i] = from_f32<T>(v);
        }
    }
}

// The same for the 2D 9-point operator: c[a] / diag for a = 1..8 with Jacobi
// scaling, else all nine; outward links (axis or corner) zeroed.
template <class T>
__device__ void start_coef_copies9(const JobStart& J, int i0, int step) {
    const int first = J.jacobi ? 1 : 0;
    T* dst0 = reinterpret_cast<T*>(J.coef_dst);
    const Coef9 src = coef9_of(J.cf, J.cf9);
    for (int i = i0; i < J.n; i += step) {
        const Cell c = cell_at(i, J.m, J.n);
        bool in[9];
        inside9(c, in);
        const float dg = src.c[0][i];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            if (a < first) continue;
            float v = in[a] ? src.c[a][i] : 0.0f;
            if (J.jacobi) v = v / dg;
            dst0[(size_t)(a - first) * J.span + i] = from_f32<T>(v);
        }
    }
}

// Starts every new job of a step in one launch: blockIdx.y is the job.
// Working-precision coefficient copies: c[a] / diag for a = 1..6 with Jacobi
// scaling (unit diagonal), else all seven; outward links on the boundary faces
// are zeroed, so the iteration never needs face tests.
__global__ __launch_bounds__(kThreads) void k_jobs_start(const JobStart* jobs) {
    const JobStart& J = jobs[blockIdx.y];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        State st{};
        st.ir = J.ir;
        st.rtol_o = J.rtol;
        st.inner_tol = J.inner_tol;
        st.inner_cap = J.inner_cap;
        st.outer_cap = J.outer_cap;
        st.max_total = J.max_total;
        st.rel = INFINITY;
        st.ostatus = ST_NOT_CONVERGED;
        st.oreason = RS_NONE;
        *J.st = st;
        *J.cnt = 0u;
        J.ctl->claim = (unsigned long long)J.first << 32;
        J.ctl->done_cnt = 0u;
        J.ctl->budget = 0;
        J.ctl->active = 0;
    }
    const int i0 = (int)(blockIdx.x * kThreads + threadIdx.x), step = (int)gridDim.x * kThreads;
    if (J.op == OP_9PT) {
        if (J.tag == 0) start_coef_copies9<float>(J, i0, step);
        else if (J.tag == 1) start_coef_copies9<bf16>(J, i0, step);
        else start_coef_copies9<f16>(J, i0, step);
    } else if (J.tag == 0) {
        start_coef_copies<float>(J, i0, step);
    } else if (J.tag == 1) {
        start_coef_copies<bf16>(J, i0, step);
    } else {
        start_coef_copies<f16>(J, i0, step);
    }
}

struct BGlobal {
    int32_t active;       // systems still active in this launch
    int32_t error;        // 1: a workgroup gave up waiting
    long long t0;         // wall clock at the arm step
    long long slice;      // wall-clock ticks after which systems park (0: no limit)
};

// ---------------------------------------------------------------- chunk work
// Partial sums are kept per unit of kUnitCells consecutive cells of a system
// (the last unit may be shorter): one wavefront sums a unit's products, lane l
// taking the unit's cells (or x-adjacent pairs) l, l + 64, l + 128, ... in that
// order, then the fixed DPP sequence of wave_reduce, and lane 63 publishes the
// unit's sums to part[unit].  The phase's completer adds the units' sums in
// unit order.  A system's sums therefore depend only on the system: not on
// how many cells a work item (chunk) covers, nor on which workgroup took it,
// so the host may size the chunks by load.  A chunk is a whole number of unit
// groups (kUnitGroup cells, one unit per wavefront of the workgroup), except
// at the end of a system.
constexpr int kUnitCells = 1024;
constexpr int kUnitGroup = kWaves * kUnitCells;
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x / kWave); }

// The end of a unit: its ND sums reduced over the wavefront, published by lane
// 63 (sums j with bit j of MAXMASK set are maxima).  All 64 lanes take part.
template <int ND, unsigned MAXMASK>
__device__ __forceinline__ void unit_done(const double (&acc)[kMaxDots], double* part, int unit) {
    if constexpr (ND > 0) {
        double v[ND];
#pragma unroll
        for (int j = 0; j < ND; ++j) v[j] = acc[j];
        wave_reduce<ND, MAXMASK>(v);
        if (lane_id() == kWave - 1) {
#pragma unroll
            for (int j = 0; j < ND; ++j) publish(&part[(size_t)unit * kMaxDots + j], v[j]);
        }
    }
}

// The units of chunk [c0, c1): wavefront w takes units w, w + kWaves, ...
// f(u0, u1, acc) sums one unit's cells [u0, u1) into acc.
template <int ND, unsigned MAXMASK, class F>
__device__ __forceinline__ void over_units(int c0, int c1, double* part, F&& f) {
    for (int u0 = c0 + wave_id() * kUnitCells; u0 < c1; u0 += kUnitGroup) {
        double acc[kMaxDots] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        f(u0, min(c1, u0 + kUnitCells), acc);
        unit_done<ND, MAXMASK>(acc, part, u0 / kUnitCells);
    }
}

// P1 of a unit on single cells, kU per lane and step: lane l takes cells
// base + 64 u + l for u < kU.  All loads of a step are issued before any store.
constexpr int kU = 4;
template <class T, bool UNIT>
__device__ void chunk_p1_b(const SysView<T>& S, int c0, int c1, double (&acc)[kMaxDots]) {
    for (int base = c0; base < c1; base += kU * kWave) {
        Cell cl[kU];
        Nbr<T> pv[kU];
        Coefs<T, UNIT> k[kU];
        T rh[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int g = base + u * kWave + lane_id();
            cl[u] = cell_at(g < c1 ? g : S.n, S.m, S.n);
            cl[u].own = g < c1;
            pv[u] = cload_nbr(S.p, cl[u]);
            k[u] = load_coefs<T, UNIT>(S.c, cl[u].idx);
            rh[u] = cload(S.rhat + cl[u].idx);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const T sv = from_f32<T>(apply7<float, T, UNIT, false>(k[u], nbr_f32(pv[u]), cl[u]));
            if (cl[u].own) {
                cstore(S.s + cl[u].idx, sv);
                acc[0] = fma((double)to_f32(rh[u]), (double)to_f32(sv), acc[0]);
            }
        }
    }
}

// Coherent loads and stores of two adjacent elements (8 bytes FP32, 4 bytes
// 16-bit; the first element's index is even).
__device__ __forceinline__ F2 cload2(const float* p) {
    const uint64_t u = __hip_atomic_load(gbl(reinterpret_cast<uint64_t*>(const_cast<float*>(p))),
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return F2{__uint_as_float((uint32_t)u), __uint_as_float((uint32_t)(u >> 32))};
}
template <class T>
__device__ __forceinline__ F2 cload2(const T* p) {
    const uint32_t u = __hip_atomic_load(gbl(reinterpret_cast<uint32_t*>(const_cast<T*>(p))), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return split16(u, p);
}
__device__ __forceinline__ void cstore2(float* p, float a, float b) {
    const uint64_t u = (uint64_t)__float_as_uint(a) | ((uint64_t)__float_as_uint(b) << 32);
    __hip_atomic_store(gbl(reinterpret_cast<uint64_t*>(p)), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void cstore2(T* p, T a, T b) {
    using U = typename Bits<T>::U;
    const uint32_t u = (uint32_t)__builtin_bit_cast(U, a) | ((uint32_t)__builtin_bit_cast(U, b) << 16);
    __hip_atomic_store(gbl(reinterpret_cast<uint32_t*>(p)), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void cload_nbr2(const T* v, const Cell& c, Nbr<float>& v0, Nbr<float>& v1) {
    const T* p = v + c.idx;
    const F2 ce = cload2(p), s = cload2(p + c.ds), nn = cload2(p + c.dn), b = cload2(p + c.db),
             t = cload2(p + c.dt);
    const float w = to_f32(cload(p + c.dw)), e = to_f32(cload(p + c.de));
    v0 = Nbr<float>{ce.a, w, ce.b, s.a, nn.a, b.a, t.a};
    v1 = Nbr<float>{ce.b, ce.a, e, s.b, nn.b, b.b, t.b};
}

// P1 of a unit on x-adjacent cell pairs (systems with an even nx): lane l
// takes pairs base/2 + 64 u + l for u < kUP.
constexpr int kUP = 2;
template <class T, bool UNIT>
__device__ void chunk_p1_pairs(const SysView<T>& S, int c0, int c1, double (&acc)[kMaxDots]) {
    for (int base = c0; base < c1; base += 2 * kUP * kWave) {
        Cell cl[kUP];
        Nbr<float> p0[kUP], p1[kUP];
        Coefs<float, UNIT> k0[kUP], k1[kUP];
        F2 rh[kUP];
#pragma unroll
        for (int u = 0; u < kUP; ++u) {
            const int gp = base / 2 + u * kWave + lane_id();
            const bool in = 2 * gp < c1;
            cl[u] = cell2_at(in ? gp : S.n / 2 - 1, S.m, S.n);
            cl[u].own = in;
            cload_nbr2(S.p, cl[u], p0[u], p1[u]);
            load_coefs2_nt<T, UNIT>(S.c, cl[u].idx, k0[u], k1[u]);
            rh[u] = cload2(S.rhat + cl[u].idx);
        }
#pragma unroll
        for (int u = 0; u < kUP; ++u) {
            const T s0 = from_f32<T>(apply7<float, float, UNIT, false>(k0[u], p0[u], cl[u]));
            const T s1 = from_f32<T>(apply7<float, float, UNIT, false>(k1[u], p1[u], cl[u]));
            if (cl[u].own) {
                cstore2(S.s + cl[u].idx, s0, s1);
                acc[0] = fma((double)rh[u].b, (double)to_f32(s1), fma((double)rh[u].a, (double)to_f32(s0), acc[0]));
            }
        }
    }
}

// P2 of the three-phase iteration: q = r - alpha s formed in FP32 at the cell
// and its six neighbours, y = A q stored; sums (q,y), (y,y), (q,q), (r0,q),
// (r0,y).  Two cells per lane and step.
__device__ __forceinline__ Nbr<float> q_of(const Nbr<float>& r, const Nbr<float>& s, float alpha) {
    return Nbr<float>{fmaT(-alpha, s.c, r.c), fmaT(-alpha, s.w, r.w), fmaT(-alpha, s.e, r.e),
                      fmaT(-alpha, s.s, r.s), fmaT(-alpha, s.n, r.n), fmaT(-alpha, s.b, r.b),
                      fmaT(-alpha, s.t, r.t)};
}
__device__ __forceinline__ void acc_p2f(double (&acc)[kMaxDots], double q, double y, double h) {
    acc[0] = fma(q, y, acc[0]);
    acc[1] = fma(y, y, acc[1]);
    acc[2] = fma(q, q, acc[2]);
    acc[3] = fma(h, q, acc[3]);
    acc[4] = fma(h, y, acc[4]);
}
constexpr int kUF = 2;
template <class T, bool UNIT>
__device__ void chunk_p2f_b(const SysView<T>& S, int c0, int c1, float alpha, double (&acc)[kMaxDots]) {
    for (int base = c0; base < c1; base += kUF * kWave) {
        Cell cl[kUF];
        Nbr<T> rv[kUF], sv[kUF];
        Coefs<T, UNIT> k[kUF];
        T rh[kUF];
#pragma unroll
        for (int u = 0; u < kUF; ++u) {
            const int g = base + u * kWave + lane_id();
            cl[u] = cell_at(g < c1 ? g : S.n, S.m, S.n);
            cl[u].own = g < c1;
            rv[u] = cload_nbr(S.r, cl[u]);
            sv[u] = cload_nbr(S.s, cl[u]);
            k[u] = load_coefs<T, UNIT>(S.c, cl[u].idx);
            rh[u] = cload(S.rhat + cl[u].idx);
        }
#pragma unroll
        for (int u = 0; u < kUF; ++u) {
            const Nbr<float> q = q_of(nbr_f32(rv[u]), nbr_f32(sv[u]), alpha);
            const T yt = from_f32<T>(apply7<float, T, UNIT, false>(k[u], q, cl[u]));
            if (cl[u].own) {
                cstore(S.y + cl[u].idx, yt);
                acc_p2f(acc, (double)q.c, (double)to_f32(yt), (double)to_f32(rh[u]));
            }
        }
    }
}

// The same on x-adjacent cell pairs (systems with an even nx).
template <class T, bool UNIT>
__device__ void chunk_p2f_pairs(const SysView<T>& S, int c0, int c1, float alpha, double (&acc)[kMaxDots]) {
    for (int base = c0; base < c1; base += 2 * kWave) {
        const int gp = base / 2 + lane_id();
        const bool in = 2 * gp < c1;
        Cell cl = cell2_at(in ? gp : S.n / 2 - 1, S.m, S.n);
        cl.own = in;
        Nbr<float> r0, r1, s0, s1;
        cload_nbr2(S.r, cl, r0, r1);
        cload_nbr2(S.s, cl, s0, s1);
        Coefs<float, UNIT> k0, k1;
        load_coefs2_nt<T, UNIT>(S.c, cl.idx, k0, k1);
        const F2 rh = cload2(S.rhat + cl.idx);
        const Nbr<float> q0 = q_of(r0, s0, alpha), q1 = q_of(r1, s1, alpha);
        const T y0 = from_f32<T>(apply7<float, float, UNIT, false>(k0, q0, cl));
        const T y1 = from_f32<T>(apply7<float, float, UNIT, false>(k1, q1, cl));
        if (in) {
            cstore2(S.y + cl.idx, y0, y1);
            acc_p2f(acc, (double)q0.c, (double)to_f32(y0), (double)rh.a);
            acc_p2f(acc, (double)q1.c, (double)to_f32(y1), (double)rh.b);
        }
    }
}

// ---------------------------------------------------------------- staged chunk work
// The paired P1 and P2 of a chunk with the stencil operand staged in LDS, for
// systems with an even nx of at most kStageMaxNx.  The chunk is taken one unit
// group (kStageTile cells) at a time; each group is staged with one row either
// side (P2: q = r - alpha s formed once per cell), then wavefront w sums unit w
// of the group: its pairs read the centre and the x and y neighbours from LDS
// and the z neighbours with coherent loads.  Staging uses 16-byte loads that
// bypass the XCD's L2 (volatile, system scope): the values were written by
// other workgroups of the launch.  Lane l visits the unit's pairs l, l + 64, ...
// as the unstaged pair functions do, so the sums are the same bit for bit.
constexpr int kStageTile = kUnitGroup;
constexpr int kStageMaxNx = 1024;
constexpr int kStageLds = kStageTile + 2 * kStageMaxNx + 24;  // one row and cell either side, 8-aligned

typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));
template <class T>
__device__ __forceinline__ void stage_coherent(const T* v, const T* w, float alpha, bool q, int lo, int cnt,
                                               int n, float* sm) {
    constexpr int W = kVec<T>;
    for (int e = (int)threadIdx.x; e < cnt / W; e += kThreads) {
        const int g = lo + W * e;
        float a[W], b[W];
        if (g >= 0 && g + W <= n) {
            if constexpr (sizeof(T) == 4) {
                const f32x4 x = *(volatile __attribute__((address_space(1))) f32x4*)gbl(
                    reinterpret_cast<f32x4*>(const_cast<T*>(v + g)));
                a[0] = x.x, a[1] = x.y, a[2] = x.z, a[3] = x.w;
                if (q) {
                    const f32x4 y = *(volatile __attribute__((address_space(1))) f32x4*)gbl(
                        reinterpret_cast<f32x4*>(const_cast<T*>(w + g)));
                    b[0] = y.x, b[1] = y.y, b[2] = y.z, b[3] = y.w;
                }
            } else {
                const u16x8_t x = *(volatile __attribute__((address_space(1))) u16x8_t*)gbl(
                    reinterpret_cast<u16x8_t*>(const_cast<T*>(v + g)));
#pragma unroll
                for (int j = 0; j < W; ++j) a[j] = to_f32(__builtin_bit_cast(T, (uint16_t)x[j]));
                if (q) {
                    const u16x8_t y = *(volatile __attribute__((address_space(1))) u16x8_t*)gbl(
                        reinterpret_cast<u16x8_t*>(const_cast<T*>(w + g)));
#pragma unroll
                    for (int j = 0; j < W; ++j) b[j] = to_f32(__builtin_bit_cast(T, (uint16_t)y[j]));
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const bool in = g + j >= 0 && g + j < n;
                a[j] = in ? to_f32(cload(v + g + j)) : 0.0f;
                b[j] = (q && in) ? to_f32(cload(w + g + j)) : 0.0f;
            }
        }
#pragma unroll
        for (int j = 0; j < W; ++j) sm[W * e + j] = q ? fmaT(-alpha, b[j], a[j]) : a[j];
    }
}

template <class T, bool UNIT, bool P2>
__device__ void chunk_staged(const SysView<T>& S, int c0, int c1, float alpha, float* sm, double* part) {
    const int nx = S.m.nx;
    for (int t0 = c0; t0 < c1; t0 += kStageTile) {
        const int t1 = min(c1, t0 + kStageTile);
        const int lo = (t0 - nx) >> 3 << 3, hi = (t1 + nx + 7) >> 3 << 3;
        __syncthreads();  // the previous group's reads of sm are over
        stage_coherent<T>(P2 ? S.r : S.p, S.s, alpha, P2, lo, hi - lo, S.n, sm);
        __syncthreads();
        const int u0 = t0 + wave_id() * kUnitCells;
        if (u0 >= t1) continue;  // the same for the whole wavefront
        const int u1 = min(t1, u0 + kUnitCells);
        double acc[kMaxDots] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        // kSP pairs per lane and step, all their loads issued before any store;
        // a lane past the unit's end works on the unit's first pair and keeps
        // nothing
        constexpr int kSP = 2;
        for (int u = 0; u < kUnitCells / (2 * kWave); u += kSP) {
            int idx[kSP];
            bool own[kSP];
            Nbr<float> v0[kSP], v1[kSP];
            Coefs<float, UNIT> k0[kSP], k1[kSP];
            F2 rh[kSP];
#pragma unroll
            for (int w = 0; w < kSP; ++w) {
                const int i = u0 + 2 * ((u + w) * kWave + lane_id());
                own[w] = i < u1;
                idx[w] = own[w] ? i : u0;
                int db, dt;
                z_offsets(idx[w], S.m, db, dt);
                F2 vb, vt;
                if (P2) {
                    const F2 rb = cload2(S.r + idx[w] + db), sb = cload2(S.s + idx[w] + db);
                    const F2 rt = cload2(S.r + idx[w] + dt), st = cload2(S.s + idx[w] + dt);
                    vb = F2{fmaT(-alpha, sb.a, rb.a), fmaT(-alpha, sb.b, rb.b)};
                    vt = F2{fmaT(-alpha, st.a, rt.a), fmaT(-alpha, st.b, rt.b)};
                } else {
                    vb = cload2(S.p + idx[w] + db);
                    vt = cload2(S.p + idx[w] + dt);
                }
                lds_nbr2(sm, idx[w] - lo, nx, vb, vt, v0[w], v1[w]);
                load_coefs2_nt<T, UNIT>(S.c, idx[w], k0[w], k1[w]);
                rh[w] = cload2(S.rhat + idx[w]);
            }
#pragma unroll
            for (int w = 0; w < kSP; ++w) {
                const Cell none{};
                const T o0 = from_f32<T>(apply7<float, float, UNIT, false>(k0[w], v0[w], none));
                const T o1 = from_f32<T>(apply7<float, float, UNIT, false>(k1[w], v1[w], none));
                if (!own[w]) continue;
                if (P2) {
                    cstore2(S.y + idx[w], o0, o1);
                    acc_p2f(acc, (double)v0[w].c, (double)to_f32(o0), (double)rh[w].a);
                    acc_p2f(acc, (double)v1[w].c, (double)to_f32(o1), (double)rh[w].b);
                } else {
                    cstore2(S.s + idx[w], o0, o1);
                    acc[0] = fma((double)rh[w].b, (double)to_f32(o1),
                                 fma((double)rh[w].a, (double)to_f32(o0), acc[0]));
                }
            }
        }
        unit_done<P2 ? 5 : 1, 0u>(acc, part, u0 / kUnitCells);
    }
}

// P3.  QR (three-phase iteration): q = r - alpha s is formed from the old r
// and s instead of being read.
template <class T, bool QR>
__device__ void chunk_p3_b(const SysView<T>& S, int c0, int c1, float alpha, float omega,
                           float beta, double (&acc)[kMaxDots]) {
    // pairs of cells (c0 is even), then a last odd cell if c1 is odd; lane l
    // takes pairs l, l + 64, ... in that order, two per step with all loads of
    // the step issued before any store (a second pair past the end is the
    // first one again and keeps nothing)
    const int c1e = c0 + ((c1 - c0) & ~1);
    for (int i0 = c0 + 2 * lane_id(); i0 < c1e; i0 += 4 * kWave) {
        const int i1 = i0 + 2 * kWave;
        const bool own1 = i1 < c1e;
        const int ii[2] = {i0, own1 ? i1 : i0};
        F2 d2[2], p2[2], s2[2], y2[2], h2[2], q2[2];
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const int i = ii[w];
            d2[w] = cload2(S.d + i), p2[w] = cload2(S.p + i), s2[w] = cload2(S.s + i);
            y2[w] = cload2(S.y + i), h2[w] = cload2(S.rhat + i);
            q2[w] = cload2((QR ? S.r : S.q) + i);
        }
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            if (w == 1 && !own1) break;
            const int i = ii[w];
            F2 q = q2[w];
            if (QR) {
                q.a = fmaT(-alpha, s2[w].a, q.a);
                q.b = fmaT(-alpha, s2[w].b, q.b);
            }
            float da = d2[w].a, db = d2[w].b;
            T ra, pa, rb, pb;
            p3_math<T>(alpha, omega, beta, p2[w].a, s2[w].a, y2[w].a, q.a, da, ra, pa);
            p3_math<T>(alpha, omega, beta, p2[w].b, s2[w].b, y2[w].b, q.b, db, rb, pb);
            cstore2(S.d + i, da, db);
            cstore2(S.r + i, ra, rb);
            cstore2(S.p + i, pa, pb);
            const double xa = (double)to_f32(ra), xb = (double)to_f32(rb);
            acc[0] = fma((double)h2[w].b, xb, fma((double)h2[w].a, xa, acc[0]));
            acc[1] = fma(xb, xb, fma(xa, xa, acc[1]));
        }
    }
    for (int i = c1e + lane_id(); i < c1; i += kWave) {
        float dv = cload(S.d + i);
        T rn, pn;
        const float sv = to_f32(cload(S.s + i));
        const float qv = QR ? fmaT(-alpha, sv, to_f32(cload(S.r + i))) : to_f32(cload(S.q + i));
        p3_math<T>(alpha, omega, beta, to_f32(cload(S.p + i)), sv, to_f32(cload(S.y + i)), qv, dv, rn, pn);
        cstore(S.d + i, dv);
        cstore(S.r + i, rn);
        cstore(S.p + i, pn);
        const double rd = (double)to_f32(rn);
        acc[0] = fma((double)to_f32(cload(S.rhat + i)), rd, acc[0]);
        acc[1] = fma(rd, rd, acc[1]);
    }
}

// X: x += scale d in FP64 (x = 0 when zero is set).
__device__ void chunk_x_b(const SysView<float>& S, double* x, int c0, int c1, double scale, bool zero) {
    for (int i = c0 + lane_id(); i < c1; i += kWave)
        cstore(x + i, zero ? 0.0 : fma(scale, (double)cload(S.d + i), cload(x + i)));
}

// R: r = b - A x in FP64 with the caller's coefficients; r_s = r / diag with
// Jacobi scaling.  write_d: d = fl32(r_s), the next inner right-hand side.
// Sums: ||b||^2, ||r||^2, max |fl32(r_s)|.
__device__ void chunk_r_b(const SysView<float>& S, const Coef7& cf, const double* b, const double* x,
                          int c0, int c1, bool write_d, double (&acc)[kMaxDots]) {
    for (int g = c0 + lane_id(); g < c1; g += kWave) {
        const Cell c = cell_at(g, S.m, S.n);
        const double* px = x + c.idx;
        const Nbr<double> xv{cload(px), cload(px + c.dw), cload(px + c.de), cload(px + c.ds),
                             cload(px + c.dn), cload(px + c.db), cload(px + c.dt)};
        const Coefs<float, false> k = load_coefs<float, false>(cf.c, c.idx);
        const double bi = *gbl(b + c.idx);
        const double r0 = bi - apply7<double, float, false, true>(k, xv, c);
        const double rs = S.unit ? r0 / (double)k.a[0] : r0;
        const float rf = (float)rs;
        if (write_d) cstore(S.d + c.idx, rf);
        acc[0] = fma(bi, bi, acc[0]);
        acc[1] = fma(r0, r0, acc[1]);
        acc[2] = fmax(acc[2], (double)fabsf(rf));
    }
}

// S (FP32 jobs): r0 = b - A x0 in FP64 with the caller's coefficients,
// Jacobi-scaled, rounded to FP32 into r, r0 and p; d = 0.  Sums: ||b_s||^2,
// (r,r) of the rounded r, ||b||^2 unscaled.
__device__ void chunk_s_b(const SysView<float>& S, const Coef7& cf, const double* b, const double* x,
                          int c0, int c1, double (&acc)[kMaxDots]) {
    for (int g = c0 + lane_id(); g < c1; g += kWave) {
        const Cell c = cell_at(g, S.m, S.n);
        const double* px = x + c.idx;
        const Nbr<double> xv{cload(px), cload(px + c.dw), cload(px + c.de), cload(px + c.ds),
                             cload(px + c.dn), cload(px + c.db), cload(px + c.dt)};
        const Coefs<float, false> k = load_coefs<float, false>(cf.c, c.idx);
        const double bi = *gbl(b + c.idx);
        double r0 = bi - apply7<double, float, false, true>(k, xv, c), bs = bi;
        if (S.unit) {
            const double dg = (double)k.a[0];
            r0 = r0 / dg;
            bs = bs / dg;
        }
        const float rf = (float)r0;
        cstore(S.r + c.idx, rf);
        cstore(S.rhat + c.idx, rf);
        cstore(S.p + c.idx, rf);
        cstore(S.d + c.idx, 0.0f);
        acc[0] = fma(bs, bs, acc[0]);
        acc[1] = fma((double)rf, (double)rf, acc[1]);
        acc[2] = fma(bi, bi, acc[2]);
    }
}

// I: r = r0 = p = fl_T(d * inv_scale), d = 0; sum (r, r).
template <class T>
__device__ void chunk_i_b(const SysView<T>& S, int c0, int c1, float inv_scale, double (&acc)[kMaxDots]) {
    for (int i = c0 + lane_id(); i < c1; i += kWave) {
        const T rt = from_f32<T>(cload(S.d + i) * inv_scale);
        cstore(S.r + i, rt);
        cstore(S.rhat + i, rt);
        cstore(S.p + i, rt);
        cstore(S.d + i, 0.0f);
        const double v = (double)to_f32(rt);
        acc[0] = fma(v, v, acc[0]);
    }
}

// The iteration phases (and I) of chunk [c0, c1) of a 7-point system, with
// each unit's sums published to part.
template <class T>
__device__ __forceinline__ void run_chunk(const SysView<float>& raw, int phase, int c0, int c1,
                                          float alpha, float omega, float beta, float inv_scale,
                                          float* sm, double* part) {
    const SysView<T> S = as_view<T>(raw);
    if (phase == K_I) {
        over_units<1, 0u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kMaxDots]) {
            chunk_i_b<T>(S, u0, u1, inv_scale, acc);
        });
    } else if (phase == K_P1) {
        if (S.pair_blocks > 0 && S.m.nx <= kStageMaxNx) {
            if (S.unit) chunk_staged<T, true, false>(S, c0, c1, 0.0f, sm, part);
            else chunk_staged<T, false, false>(S, c0, c1, 0.0f, sm, part);
        } else {
            over_units<1, 0u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kMaxDots]) {
                if (S.pair_blocks > 0) {
                    if (S.unit) chunk_p1_pairs<T, true>(S, u0, u1, acc);
                    else chunk_p1_pairs<T, false>(S, u0, u1, acc);
                } else if (S.unit) {
                    chunk_p1_b<T, true>(S, u0, u1, acc);
                } else {
                    chunk_p1_b<T, false>(S, u0, u1, acc);
                }
            });
        }
    } else if (phase == K_P2) {
        if (S.pair_blocks > 0 && S.m.nx <= kStageMaxNx) {
            if (S.unit) chunk_staged<T, true, true>(S, c0, c1, alpha, sm, part);
            else chunk_staged<T, false, true>(S, c0, c1, alpha, sm, part);
        } else {
            over_units<5, 0u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kMaxDots]) {
                if (S.pair_blocks > 0) {
                    if (S.unit) chunk_p2f_pairs<T, true>(S, u0, u1, alpha, acc);
                    else chunk_p2f_pairs<T, false>(S, u0, u1, alpha, acc);
                } else if (S.unit) {
                    chunk_p2f_b<T, true>(S, u0, u1, alpha, acc);
                } else {
                    chunk_p2f_b<T, false>(S, u0, u1, alpha, acc);
                }
            });
        }
    } else {
        over_units<2, 0u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kMaxDots]) {
            chunk_p3_b<T, true>(S, u0, u1, alpha, omega, beta, acc);
        });
    }
}

// ---------------------------------------------------------------- 2D 9-point chunk work
// The nine values of a vector at a cell (order diag, w, e, s, n, sw, se, nw,
// ne), coherent loads; working vectors widened to FP32.
template <class T>
__device__ __forceinline__ void cload9f(const T* v, const Cell& c, float (&x)[9]) {
    int o[9];
    offsets9(c, o);
    const T* p = v + c.idx;
#pragma unroll
    for (int a = 0; a < 9; ++a) x[a] = to_f32(cload(p + o[a]));
}
__device__ __forceinline__ void cload9d(const double* v, const Cell& c, double (&x)[9]) {
    int o[9];
    offsets9(c, o);
    const double* p = v + c.idx;
#pragma unroll
    for (int a = 0; a < 9; ++a) x[a] = cload(p + o[a]);
}

// The working copies of a 9-point system: the first seven in the view, the
// last two beside it.
template <class T>
__device__ __forceinline__ Coef9T<T> work9(const SysView<T>& S, const float* const (&extra)[2]) {
    Coef9T<T> k;
#pragma unroll
    for (int a = 0; a < 7; ++a) k.c[a] = S.c[a];
    k.c[7] = reinterpret_cast<const T*>(extra[0]);
    k.c[8] = reinterpret_cast<const T*>(extra[1]);
    return k;
}

// P1 of a unit: s = A p, rounded to T; (r0, s).  Two cells per lane and step,
// lane l taking cells base + 64 u + l; all loads of a step before any store.
constexpr int kU9 = 2;
template <class T, bool UNIT>
__device__ void chunk_p1_b9(const SysView<T>& S, const Coef9T<T>& k, int c0, int c1, double (&acc)[kMaxDots]) {
    for (int base = c0; base < c1; base += kU9 * kWave) {
        Cell cl[kU9];
        float pv[kU9][9];
        T rh[kU9];
#pragma unroll
        for (int u = 0; u < kU9; ++u) {
            const int g = base + u * kWave + lane_id();
            cl[u] = cell_at(g < c1 ? g : S.n, S.m, S.n);
            cl[u].own = g < c1;
            cload9f(S.p, cl[u], pv[u]);
            rh[u] = cload(S.rhat + cl[u].idx);
        }
#pragma unroll
        for (int u = 0; u < kU9; ++u) {
            const T sv = from_f32<T>(apply9_work<T, UNIT>(k, cl[u].idx, pv[u]));
            if (cl[u].own) {
                cstore(S.s + cl[u].idx, sv);
                acc[0] = fma((double)to_f32(rh[u]), (double)to_f32(sv), acc[0]);
            }
        }
    }
}

// P2: q = r - alpha s formed in FP32 at the cell and its eight neighbours,
// y = A q stored; sums (q,y), (y,y), (q,q), (r0,q), (r0,y).
template <class T, bool UNIT>
__device__ void chunk_p2f_b9(const SysView<T>& S, const Coef9T<T>& k, int c0, int c1, float alpha,
                             double (&acc)[kMaxDots]) {
    for (int base = c0; base < c1; base += kU9 * kWave) {
        Cell cl[kU9];
        float q[kU9][9];
        T rh[kU9];
#pragma unroll
        for (int u = 0; u < kU9; ++u) {
            const int g = base + u * kWave + lane_id();
            cl[u] = cell_at(g < c1 ? g : S.n, S.m, S.n);
            cl[u].own = g < c1;
            float rv[9], sv[9];
            cload9f(S.r, cl[u], rv);
            cload9f(S.s, cl[u], sv);
#pragma unroll
            for (int a = 0; a < 9; ++a) q[u][a] = fmaT(-alpha, sv[a], rv[a]);
            rh[u] = cload(S.rhat + cl[u].idx);
        }
#pragma unroll
        for (int u = 0; u < kU9; ++u) {
            const T yt = from_f32<T>(apply9_work<T, UNIT>(k, cl[u].idx, q[u]));
            if (cl[u].own) {
                cstore(S.y + cl[u].idx, yt);
                acc_p2f(acc, (double)q[u][0], (double)to_f32(yt), (double)to_f32(rh[u]));
            }
        }
    }
}

// R: r = b - A x in FP64 with the caller's coefficients (outward links
// masked); the rest as for the 7-point operator.
__device__ void chunk_r_b9(const SysView<float>& S, const Coef9& cf, const double* b, const double* x,
                           int c0, int c1, bool write_d, double (&acc)[kMaxDots]) {
    for (int g = c0 + lane_id(); g < c1; g += kWave) {
        const Cell c = cell_at(g, S.m, S.n);
        double xv[9];
        cload9d(x, c, xv);
        const double bi = *gbl(b + c.idx);
        const double r0 = bi - apply9_masked<double>(cf, c, xv);
        const double rs = S.unit ? r0 / (double)*gbl(cf.c[0] + c.idx) : r0;
        const float rf = (float)rs;
        if (write_d) cstore(S.d + c.idx, rf);
        acc[0] = fma(bi, bi, acc[0]);
        acc[1] = fma(r0, r0, acc[1]);
        acc[2] = fmax(acc[2], (double)fabsf(rf));
    }
}

// S (FP32 jobs): r0 = b - A x0, as for the 7-point operator.
__device__ void chunk_s_b9(const SysView<float>& S, const Coef9& cf, const double* b, const double* x,
                           int c0, int c1, double (&acc)[kMaxDots]) {
    for (int g = c0 + lane_id(); g < c1; g += kWave) {
        const Cell c = cell_at(g, S.m, S.n);
        double xv[9];
        cload9d(x, c, xv);
        const double bi = *gbl(b + c.idx);
        double r0 = bi - apply9_masked<double>(cf, c, xv), bs = bi;
        if (S.unit) {
            const double dg = (double)*gbl(cf.c[0] + c.idx);
            r0 = r0 / dg;
            bs = bs / dg;
        }
        const float rf = (float)r0;
        cstore(S.r + c.idx, rf);
        cstore(S.rhat + c.idx, rf);
        cstore(S.p + c.idx, rf);
        cstore(S.d + c.idx, 0.0f);
        acc[0] = fma(bs, bs, acc[0]);
        acc[1] = fma((double)rf, (double)rf, acc[1]);
        acc[2] = fma(bi, bi, acc[2]);
    }
}

// The 9-point P1 and P2 of a chunk with the operand staged in LDS (systems with
// nx of at most kStageMaxNx): each unit group is staged with one row and one
// cell either side, and all nine points of a cell are read from LDS.  Lane l
// of wavefront w visits the cells l, l + 64, ... of unit w of the group, as
// the unstaged functions do, so the sums are the same bit for bit.
template <class T, bool UNIT, bool P2>
__device__ void chunk_staged9(const SysView<T>& S, const Coef9T<T>& k, int c0, int c1, float alpha, float* sm,
                              double* part) {
    const int nx = S.m.nx;
    for (int t0 = c0; t0 < c1; t0 += kStageTile) {
        const int t1 = min(c1, t0 + kStageTile);
        const int lo = (t0 - nx - 1) >> 3 << 3, hi = (t1 + nx + 1 + 7) >> 3 << 3;
        __syncthreads();
        stage_coherent<T>(P2 ? S.r : S.p, S.s, alpha, P2, lo, hi - lo, S.n, sm);
        __syncthreads();
        const int u0 = t0 + wave_id() * kUnitCells;
        if (u0 >= t1) continue;  // the same for the whole wavefront
        const int u1 = min(t1, u0 + kUnitCells);
        double acc[kMaxDots] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        // four cells per lane and step, their coefficient and r0 loads issued
        // before any store; a lane past the unit's end works on the unit's
        // first cell and keeps nothing
        constexpr int kSC = 4;
        for (int u = 0; u < kUnitCells / kWave; u += kSC) {
            int idx[kSC];
            bool own[kSC];
            float kc[kSC][9];
            T rh[kSC];
#pragma unroll
            for (int w = 0; w < kSC; ++w) {
                const int i = u0 + (u + w) * kWave + lane_id();
                own[w] = i < u1;
                idx[w] = own[w] ? i : u0;
                kc[w][0] = UNIT ? 1.0f : to_f32(ld_nt(k.c[0] + idx[w]));
#pragma unroll
                for (int a = 1; a < 9; ++a) kc[w][a] = to_f32(ld_nt(k.c[a] + idx[w]));
                rh[w] = cload(S.rhat + idx[w]);
            }
#pragma unroll
            for (int w = 0; w < kSC; ++w) {
                const int L = idx[w] - lo;
                const float v[9] = {sm[L], sm[L - 1], sm[L + 1], sm[L - nx], sm[L + nx],
                                    sm[L - nx - 1], sm[L - nx + 1], sm[L + nx - 1], sm[L + nx + 1]};
                // the terms in the order of apply9_work
                float a9 = UNIT ? v[0] : kc[w][0] * v[0];
#pragma unroll
                for (int a = 1; a < 9; ++a) a9 = fma9(kc[w][a], v[a], a9);
                const T o = from_f32<T>(a9);
                if (!own[w]) continue;
                if (P2) {
                    cstore(S.y + idx[w], o);
                    acc_p2f(acc, (double)v[0], (double)to_f32(o), (double)to_f32(rh[w]));
                } else {
                    cstore(S.s + idx[w], o);
                    acc[0] = fma((double)to_f32(rh[w]), (double)to_f32(o), acc[0]);
                }
            }
        }
        unit_done<P2 ? 5 : 1, 0u>(acc, part, u0 / kUnitCells);
    }
}

template <class T>
__device__ __forceinline__ void run_chunk9(const SysView<float>& raw, const float* const (&wk)[2], int phase,
                                           int c0, int c1, float alpha, float omega, float beta,
                                           float inv_scale, float* sm, double* part) {
    const SysView<T> S = as_view<T>(raw);
    const Coef9T<T> k = work9<T>(S, wk);
    const bool staged = S.m.nx <= kStageMaxNx;
    if (phase == K_I) {
        over_units<1, 0u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kMaxDots]) {
            chunk_i_b<T>(S, u0, u1, inv_scale, acc);
        });
    } else if (phase == K_P1) {
        if (staged && S.unit) chunk_staged9<T, true, false>(S, k, c0, c1, 0.0f, sm, part);
        else if (staged) chunk_staged9<T, false, false>(S, k, c0, c1, 0.0f, sm, part);
        else
            over_units<1, 0u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kMaxDots]) {
                if (S.unit) chunk_p1_b9<T, true>(S, k, u0, u1, acc);
                else chunk_p1_b9<T, false>(S, k, u0, u1, acc);
            });
    } else if (phase == K_P2) {
        if (staged && S.unit) chunk_staged9<T, true, true>(S, k, c0, c1, alpha, sm, part);
        else if (staged) chunk_staged9<T, false, true>(S, k, c0, c1, alpha, sm, part);
        else
            over_units<5, 0u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kMaxDots]) {
                if (S.unit) chunk_p2f_b9<T, true>(S, k, u0, u1, alpha, acc);
                else chunk_p2f_b9<T, false>(S, k, u0, u1, alpha, acc);
            });
    } else {
        over_units<2, 0u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kMaxDots]) {
            chunk_p3_b<T, true>(S, u0, u1, alpha, omega, beta, acc);
        });
    }
}

// ---------------------------------------------------------------- job control
// After the inner iteration stopped (st.done): the FP32 epilogue, or the
// bookkeeping of one refinement step.  Returns the next phase.
__device__ int after_inner(State& st) {
    if (st.trial) return K_FINAL;  // a tuning trial never touches the caller's arrays
    if (!st.ir) {
        st.total = st.iter;
        st.ostatus = st.status;
        st.oreason = st.reason;
        st.inner_res = st.res_rec;
        st.scale = 1.0;
        st.xzero = st.nbzero;  // b = 0: x = 0
        return K_X;
    }
    st.total += st.iter;
    st.outer += 1;
    st.inner_res = st.res_rec;
    if (st.status == ST_BREAKDOWN && st.iter == 0) {
        st.ostatus = ST_BREAKDOWN;
        st.oreason = st.reason;
        return K_FINAL;
    }
    return K_X;
}

// After the residual pass: the final true residual (FP32 jobs), or the
// refinement decision (the same rules as the single-system solve).
__device__ int after_resid(State& st, const double (&tot)[kMaxDots]) {
    st.bb_true = tot[0];
    st.rr_true = tot[1];
    st.rmax = tot[2];
    if (!st.ir) return K_FINAL;
    if (tot[0] == 0.0) {
        st.xzero = 1;
        st.rel = 0.0;
        st.ostatus = ST_OK;
        return K_X;
    }
    const double nrel = sqrt(tot[1] / tot[0]);
    if (!isfinite(nrel)) {
        st.ostatus = ST_BREAKDOWN;
        st.oreason = RS_NONFINITE;
        st.rel = nrel;
        return K_FINAL;
    }
    st.stall = (nrel > 0.5 * st.rel) ? st.stall + 1 : 0;
    st.rel = nrel;
    if (nrel <= st.rtol_o) {
        st.ostatus = ST_OK;
        return K_FINAL;
    }
    if (st.outer >= st.outer_cap || st.total >= st.max_total || st.stall >= 3) {
        st.ostatus = ST_NOT_CONVERGED;
        return K_FINAL;
    }
    // power-of-two scale 2^ceil(log2 rmax), exactly: the inner right-hand side
    // has max |.| in (0.5, 1]
    if (st.rmax > 0.0) {
        int e;
        const double m = frexp(st.rmax, &e);  // rmax = m 2^e, m in [0.5, 1)
        st.scale = ldexp(1.0, m == 0.5 ? e - 1 : e);
    } else {
        st.scale = 1.0;
    }
    return K_I;
}

// ---------------------------------------------------------------- persistent kernel
// One launch runs systems of both operators: the system's op selects its
// phase functions.
__global__ __launch_bounds__(kThreads) void k_batched(const BSys* __restrict__ sys, const int* __restrict__ home,
                                                      BGlobal* glob, int nsys, long long spin_limit) {
    __shared__ int sh_sys, sh_chunk, sh_last, sh_stop, sh_budget, sh_direct;
    __shared__ uint32_t sh_seq, sh_nseq;
    __shared__ State sh_state;
    // the staged chunk functions' LDS
    __shared__ float sh_stage[kStageLds];
    // The search for work starts at the workgroup's home system while that
    // system is active (systems do not become active again within a launch),
    // then at the system where work was last found.
    const int h0 = home[blockIdx.x];
    bool home_live = true;
    int s = h0;
    long long idle = 0;
    if (threadIdx.x == 0) sh_direct = 0;
    // the launch's time slice, set by the arm step
    const long long slice = glob->slice, t_arm = glob->t0;
    for (;;) {
        // A one-chunk phase's completer has already taken the next phase's chunk
        // (sh_sys, sh_chunk and sh_seq are set): no search.  While it goes on
        // so, the system is resident in the workgroup: its State's current copy
        // is the LDS one (sh_state) and its budget is sh_budget; memory holds
        // them again once the system stops.
        if (threadIdx.x == 0 && !sh_direct) {
            // Each probe is a round trip to memory: the system's flag and claim
            // word are loaded together, and the launch-wide words are read only
            // when no system has work.
            sh_sys = -1;
            if (home_live) s = h0;
            for (int tries = 0; tries < nsys; ++tries, s = (s + 1 == nsys) ? 0 : s + 1) {
                const int act = cload_i(&sys[s].ctl->active);
                const unsigned long long w0 =
                    __hip_atomic_load(gbl(&sys[s].ctl->claim), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (!act && s == h0) home_live = false;
                if (!act || (int)(w0 & 0xffffffffull) >= sys[s].nchunk) continue;
                const unsigned long long w = __hip_atomic_fetch_add(
                    gbl(&sys[s].ctl->claim), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int c = (int)(w & 0xffffffffull);
                if (c < sys[s].nchunk) {
                    sh_sys = s;
                    sh_chunk = c;
                    sh_seq = (uint32_t)(w >> 32);
                    break;
                }
            }
            if (sh_sys == -1) {
                const int live = cload_i(&glob->active), err = cload_i(&glob->error);
                if (live <= 0 || err != 0) sh_sys = -2;  // nothing left in this launch
            }
        }
        __syncthreads();
        // The claim is the same for the whole workgroup: taking it as a scalar
        // lets the table entry and the system's base pointers live in scalar
        // registers, and the vector accesses take a scalar base with a 32-bit
        // lane offset.
        const int me = __builtin_amdgcn_readfirstlane(sh_sys);
        if (me == -2) return;
        if (me < 0) {
            if (++idle > spin_limit) {
                if (threadIdx.x == 0) cstore_i(&glob->error, 1);
                return;
            }
            __builtin_amdgcn_s_sleep(8);
            __syncthreads();
            continue;
        }
        idle = 0;
        const BSys& B = sys[me];
        const SysView<float> S = B.S;
        const int tag = B.tag;
        const bool op9 = __builtin_amdgcn_readfirstlane(B.op) == OP_9PT;
        const int chunk = __builtin_amdgcn_readfirstlane(sh_chunk);
        const uint32_t seq = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh_seq);
        const bool res = __builtin_amdgcn_readfirstlane(sh_direct) != 0;
        const int kind = (int)(seq & 7u);
        const int c0 = chunk * B.chunk;
        const int c1 = min(S.n, c0 + B.chunk);
        double* const part = S.red.part;
        // the State's scalars this phase reads: from the resident copy, or from memory
        if (kind == K_X) {
            const double scale = res ? sh_state.scale : cload_d(&S.st->scale);
            const bool zero = (res ? sh_state.xzero : cload_i(&S.st->xzero)) != 0;
            over_units<0, 0u>(c0, c1, part, [&](int u0, int u1, double (&)[kMaxDots]) {
                chunk_x_b(S, B.x, u0, u1, scale, zero);
            });
        } else if (kind == K_R) {
            const bool ir = (res ? sh_state.ir : cload_i(&S.st->ir)) != 0;
            over_units<3, 4u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kMaxDots]) {
                if (op9) chunk_r_b9(S, coef9_of(B.cf, B.cf9), B.b, B.x, u0, u1, ir, acc);
                else chunk_r_b(S, B.cf, B.b, B.x, u0, u1, ir, acc);
            });
        } else if (kind == K_S) {
            over_units<3, 0u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kMaxDots]) {
                if (op9) chunk_s_b9(S, coef9_of(B.cf, B.cf9), B.b, B.x, u0, u1, acc);
                else chunk_s_b(S, B.cf, B.b, B.x, u0, u1, acc);
            });
        } else {
            const float alpha = (float)(res ? sh_state.alpha : cload_d(&S.st->alpha));
            const float omega = (float)(res ? sh_state.omega : cload_d(&S.st->omega));
            const float beta = (float)(res ? sh_state.beta : cload_d(&S.st->beta));
            const float inv_scale = kind == K_I ? (float)(1.0 / (res ? sh_state.scale : cload_d(&S.st->scale))) : 1.0f;
            if (op9) {
                if (tag == 0) run_chunk9<float>(S, B.wk9, kind, c0, c1, alpha, omega, beta, inv_scale, sh_stage, part);
                else if (tag == 1)
                    run_chunk9<bf16>(S, B.wk9, kind, c0, c1, alpha, omega, beta, inv_scale, sh_stage, part);
                else run_chunk9<f16>(S, B.wk9, kind, c0, c1, alpha, omega, beta, inv_scale, sh_stage, part);
            } else {
                if (tag == 0) run_chunk<float>(S, kind, c0, c1, alpha, omega, beta, inv_scale, sh_stage, part);
                else if (tag == 1) run_chunk<bf16>(S, kind, c0, c1, alpha, omega, beta, inv_scale, sh_stage, part);
                else run_chunk<f16>(S, kind, c0, c1, alpha, omega, beta, inv_scale, sh_stage, part);
            }
        }
        // Every thread waits until its own vector stores (the units' sums
        // included) have reached memory: a workgroup barrier does not wait for
        // them, and the next phase may read them from another workgroup.  Then
        // the chunk is counted done.
        wait_stores();
        __syncthreads();
        // a phase of one chunk is complete once its chunk is: no count
        if (threadIdx.x == 0) {
            sh_direct = 0;
            if (B.nchunk == 1) {
                sh_last = 1;
            } else {
                const uint32_t t = __hip_atomic_fetch_add(gbl(&B.ctl->done_cnt), 1u, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                sh_last = (t == (uint32_t)(B.nchunk - 1));
            }
        }
        __syncthreads();
        if (!sh_last) continue;
        // this workgroup completes the phase: sum the units' sums in unit order.
        // The State's words are loaded first, so that they and the sums share
        // one memory round trip.
        // (a resident system's LDS copy is already current)
        const uint32_t stw = res ? 0u : state_fetch(S.st);
        const int nunit = (S.n + kUnitCells - 1) / kUnitCells;
        double tot[kMaxDots] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (kind == K_R) sum_range<kMaxDots, 4u, true>(part, 0, nunit, tot);
        else if (kND[kind] > 0) sum_range<kMaxDots, 0u, true>(part, 0, nunit, tot);
        // the private state copy lives in LDS: a register copy would raise the
        // register count of the whole kernel
        if (!res) state_put(stw, sh_state);
        else __syncthreads();
        if (threadIdx.x == 0) {
            State& st = sh_state;
            int next = K_FINAL;
            bool iter_done = false;
            switch (kind) {
                case K_P1: tail_p1(&st, reinterpret_cast<double(&)[1]>(tot)); next = K_P2; break;
                case K_P2: tail_p2f(&st, reinterpret_cast<double(&)[5]>(tot)); next = K_P3; break;
                case K_P3:
                    tail_p3(&st, reinterpret_cast<double(&)[2]>(tot));
                    next = K_P1;
                    iter_done = true;
                    break;
                case K_X: next = st.xzero ? K_FINAL : K_R; break;
                case K_R: next = after_resid(st, tot); break;
                case K_S:  // an FP32 job's start
                    tail_init(&st, tot[0], tot[1], st.rtol_o, st.max_total);
                    st.bb_true = tot[2];
                    st.scale = 1.0;
                    next = K_P1;
                    break;
                default: {  // K_I: the next inner solve starts
                    const int left = st.max_total - st.total;
                    tail_init(&st, tot[0], tot[0], st.inner_tol, st.inner_cap < left ? st.inner_cap : left);
                    next = K_P1;
                }
            }
            if ((kind <= K_P3 || kind == K_I || kind == K_S) && st.done) next = after_inner(st);
            int32_t budget = res ? sh_budget : cload_i(&B.ctl->budget);
            bool stop = next == K_FINAL;
            if (iter_done && next == K_P1) {
                budget -= 1;
                stop = budget <= 0;
            }
            // time slice: any phase boundary is a resumable point
            if (slice > 0 && wall_clock64() - t_arm > slice) stop = true;
            if (next == K_FINAL) st.final = 1;
            sh_stop = stop ? 1 : 0;
            sh_budget = budget;
            sh_nseq = seq_next(seq, next == K_FINAL ? K_P1 : next);
        }
        __syncthreads();
        // a system that goes on resident keeps its State in LDS only
        const bool stay = !sh_stop && B.nchunk == 1;
        if (!stay) {
            state_store(S.st, sh_state);
            __syncthreads();  // every word of the State has reached memory
        }
        if (threadIdx.x == 0) {
            const uint32_t nseq = sh_nseq;
            if (!stay) {
                __hip_atomic_store(gbl(&B.ctl->done_cnt), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                cstore_i(&B.ctl->budget, sh_budget);
            }
            if (sh_stop) {
                cstore_i(&B.ctl->active, 0);
                // Park the claim word on the phase to resume, with its chunk counter
                // already exhausted: a workgroup racing this store claims nothing.  The
                // next launch's arm step rewinds the counter.
                __hip_atomic_store(gbl(&B.ctl->claim), ((unsigned long long)nseq << 32) | (unsigned)B.nchunk,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                wait_stores();
                __hip_atomic_fetch_add(&glob->active, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else if (stay) {
                // the next phase's only chunk is taken here, and this workgroup
                // goes on with the same system.  On the way in, the claim word is
                // published with its chunk counter exhausted, so that no other
                // workgroup claims the system; it is not written again until the
                // system stops.
                if (!res)
                    __hip_atomic_store(gbl(&B.ctl->claim), ((unsigned long long)nseq << 32) | 1ull,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sh_sys = me;
                sh_chunk = 0;
                sh_seq = nseq;
                sh_direct = 1;
            } else {
                wait_stores();
                __hip_atomic_store(gbl(&B.ctl->claim), (unsigned long long)nseq << 32, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    }
}

// Arms a launch: every job that is not finished takes part with its own
// iteration budget; the global count of active jobs is set accordingly.  With
// a time slice, every job parks at its first phase boundary after `slice`
// wall-clock ticks.  A job
// whose first inner solve stopped at once (set up by the host, e.g. b = 0)
// moves on to its epilogue.
__global__ __launch_bounds__(kThreads) void k_batched_arm(const BSys* sys, BGlobal* glob, int nsys,
                                                          long long slice) {
    __shared__ int count;
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < nsys; s += kThreads) {
        State* st = sys[s].S.st;
        bool fin = st->final != 0;
        uint32_t seq = (uint32_t)(sys[s].ctl->claim >> 32);  // rewinds the chunk counter
        if (!fin && st->done && (seq & 7u) == (uint32_t)K_P1) {
            State cp = *st;
            const int next = after_inner(cp);
            if (next == K_FINAL) cp.final = 1;
            *st = cp;
            fin = cp.final != 0;
            seq = seq_next(seq, next == K_FINAL ? K_P1 : next);
        }
        sys[s].ctl->claim = (unsigned long long)seq << 32;
        sys[s].ctl->active = fin ? 0 : 1;
        sys[s].ctl->budget = sys[s].budget;
        sys[s].ctl->done_cnt = 0u;
        if (!fin) atomicAdd(&count, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        glob->active = count;
        glob->error = 0;
        glob->t0 = wall_clock64();
        glob->slice = slice;
    }
}

static_assert(sizeof(State) % 8 == 0, "State is copied in 8-byte words");

// Copies the states of nsys systems into one contiguous array, so that the
// host reads them with a single transfer.
__global__ __launch_bounds__(kThreads) void k_gather_states(State* const* src, State* dst, int nsys) {
    constexpr int W = (int)(sizeof(State) / 8);
    const int total = nsys * W;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < total; i += gridDim.x * kThreads) {
        const int s = i / W, w = i - s * W;
        reinterpret_cast<uint64_t*>(dst + s)[w] = reinterpret_cast<const uint64_t*>(src[s])[w];
    }
}

}  // namespace s7
