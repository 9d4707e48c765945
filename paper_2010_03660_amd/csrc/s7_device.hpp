// Device-side building blocks of the s7 library (gfx950, wave64).
//
// * Storage types and round-to-nearest-even conversions (FP32, BF16, FP16).
// * The cell-parallel stencil: one thread per cell, cells in their natural
//   x-fastest order, so a workgroup covers 256 consecutive cells.  All seven
//   operand values and the coefficients are loaded straight from memory.  The
//   neighbour re-reads (x+-1, y+-1, z+-1) are served by L1, L2 and the
//   Infinity Cache.  Arrays read once per pass (coefficients, r0, b) use
//   non-temporal loads, which leaves the L2 to the stencil operands.  Loads
//   are branch-free: an off-mesh neighbour reads the cell itself, and a zero
//   coefficient cancels it.
// * The BiCGStab passes: P1 (s = A p and (r0,s)), the streaming P2a
//   (q = r - alpha s and (q,q)), P2b (y = A q and four dots) and the
//   streaming P3 (x, r and p updates and two dots).
// * Deterministic hierarchical reductions: FP64 per lane, a fixed wavefront
//   DPP sequence, a fixed wave order in LDS, and per-workgroup partials,
//   summed in a fixed index order by the last workgroup to arrive (an atomic
//   ticket) or, for grids above 1024 workgroups, by a finishing kernel.
// * The scalar steps of Algorithm 1 (alpha, omega, beta, stopping and
//   breakdown tests), run by one thread of the last workgroup.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace s7 {

constexpr int kWave = 64;
constexpr int kWaves = 4;  // wavefronts per workgroup
constexpr int kThreads = kWave * kWaves;
constexpr int kMaxDots = 6;
constexpr int kGroup = 8192;  // workgroup partials summed by one workgroup of a finishing kernel

// ---------------------------------------------------------------- types
struct bf16 {
    uint16_t u;
};
using f16 = _Float16;

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(bf16 v) { return __uint_as_float(((uint32_t)v.u) << 16); }
__device__ __forceinline__ float to_f32(f16 v) { return (float)v; }

// Type tag of a storage type: part of every cache key that depends on it
// (BF16 and FP16 have the same size).
template <class T>
struct TypeTag;
template <>
struct TypeTag<float> {
    static constexpr int value = 0;
};
template <>
struct TypeTag<bf16> {
    static constexpr int value = 1;
};
template <>
struct TypeTag<f16> {
    static constexpr int value = 2;
};

template <class T>
__device__ __forceinline__ T from_f32(float f);
template <>
__device__ __forceinline__ float from_f32<float>(float f) { return f; }
template <>
__device__ __forceinline__ bf16 from_f32<bf16>(float f) {
    // round to nearest, ties to even; NaN stays a (quiet) NaN
    uint32_t u = __float_as_uint(f);
    bf16 r;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
        r.u = (uint16_t)((u >> 16) | 0x40u);
        return r;
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    r.u = (uint16_t)(u >> 16);
    return r;
}
template <>
__device__ __forceinline__ f16 from_f32<f16>(float f) { return (f16)f; }  // RNE

// ---------------------------------------------------------------- streaming access
// Every array here is device (global) memory.  A pointer the compiler cannot
// trace to a kernel argument (one read from a table in memory) is generic to
// it, and generic accesses become flat instructions with 64-bit per-lane
// addresses; seen through the global address space they become global
// instructions, which also take a scalar base with a 32-bit lane offset.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gbl(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// Non-temporal loads and stores for data touched once per pass (coefficients,
// r0, and the vectors a pass writes).  The cached path is kept for operands
// whose halo neighbours re-read them.
__device__ __forceinline__ float ld_nt(const float* p) { return __builtin_nontemporal_load(gbl(p)); }
__device__ __forceinline__ double ld_nt(const double* p) { return __builtin_nontemporal_load(gbl(p)); }
__device__ __forceinline__ f16 ld_nt(const f16* p) { return __builtin_nontemporal_load(gbl(p)); }
__device__ __forceinline__ bf16 ld_nt(const bf16* p) {
    bf16 r;
    r.u = __builtin_nontemporal_load(gbl(reinterpret_cast<const uint16_t*>(p)));
    return r;
}
// A plain (cached) load through the global address space.
__device__ __forceinline__ float ld(const float* p) { return *gbl(p); }
__device__ __forceinline__ double ld(const double* p) { return *gbl(p); }
__device__ __forceinline__ f16 ld(const f16* p) { return *gbl(p); }
__device__ __forceinline__ bf16 ld(const bf16* p) { return bf16{*gbl(reinterpret_cast<const uint16_t*>(p))}; }
__device__ __forceinline__ void st_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_nt(f16* p, f16 v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_nt(bf16* p, bf16 v) {
    __builtin_nontemporal_store(v.u, reinterpret_cast<uint16_t*>(p));
}

// Four consecutive elements (8- or 16-byte aligned) as FP32, and back.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void ld4_nt(const float* p, float (&v)[4]) {
    const f32x4 a = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
}
__device__ __forceinline__ void ld4_nt(const bf16* p, float (&v)[4]) {
    const u16x4 a = __builtin_nontemporal_load(reinterpret_cast<const u16x4*>(p));
    v[0] = __uint_as_float((uint32_t)a.x << 16);
    v[1] = __uint_as_float((uint32_t)a.y << 16);
    v[2] = __uint_as_float((uint32_t)a.z << 16);
    v[3] = __uint_as_float((uint32_t)a.w << 16);
}
__device__ __forceinline__ void ld4_nt(const f16* p, float (&v)[4]) {
    const u16x4 a = __builtin_nontemporal_load(reinterpret_cast<const u16x4*>(p));
    const uint16_t u[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = (float)__builtin_bit_cast(f16, u[i]);
}
__device__ __forceinline__ void st4_nt(float* p, const float (&v)[4]) {
    f32x4 a;
    a.x = v[0];
    a.y = v[1];
    a.z = v[2];
    a.w = v[3];
    __builtin_nontemporal_store(a, reinterpret_cast<f32x4*>(p));
}
template <class T>
__device__ __forceinline__ uint16_t bits16(T v);
template <>
__device__ __forceinline__ uint16_t bits16<bf16>(bf16 v) { return v.u; }
template <>
__device__ __forceinline__ uint16_t bits16<f16>(f16 v) { return __builtin_bit_cast(uint16_t, v); }
template <class T>
__device__ __forceinline__ void st4_nt(T* p, const T (&v)[4]) {
    u16x4 a;
    a.x = bits16(v[0]);
    a.y = bits16(v[1]);
    a.z = bits16(v[2]);
    a.w = bits16(v[3]);
    __builtin_nontemporal_store(a, reinterpret_cast<u16x4*>(p));
}

// W consecutive elements as FP32, and back: W = 4 (8- or 16-byte accesses) or
// W = 8 (16-byte accesses of 16-bit data, two 16-byte accesses of FP32).
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
template <int W, class T>
__device__ __forceinline__ void ldw_nt(const T* p, float (&v)[W]) {
    if constexpr (W == 4) {
        ld4_nt(p, v);
    } else if constexpr (sizeof(T) == 4) {
        float a[4], b[4];
        ld4_nt(p, a);
        ld4_nt(p + 4, b);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = a[j], v[4 + j] = b[j];
    } else {
        const u16x8 a = __builtin_nontemporal_load(reinterpret_cast<const u16x8*>(p));
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            T t;
            const uint16_t u = a[j];
            __builtin_memcpy(&t, &u, 2);
            v[j] = to_f32(t);
        }
    }
}
template <int W, class T>
__device__ __forceinline__ void stw_nt(T* p, const T (&v)[W]) {
    if constexpr (W == 4) {
        st4_nt(p, v);
    } else if constexpr (sizeof(T) == 4) {
        const T a[4] = {v[0], v[1], v[2], v[3]}, b[4] = {v[4], v[5], v[6], v[7]};
        st4_nt(p, a);
        st4_nt(p + 4, b);
    } else {
        u16x8 a;
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = bits16(v[j]);
        __builtin_nontemporal_store(a, reinterpret_cast<u16x8*>(p));
    }
}
// Elements per thread and step of the streaming passes: 16-byte accesses.
template <class T>
constexpr int kVec = sizeof(T) == 2 ? 8 : 4;

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The caller's seven FP32 coefficient arrays: diag, xm, xp, ym, yp, zm, zp.
struct Coef7 {
    const float* c[7];
};

// ---------------------------------------------------------------- geometry
// rnx and rplane are 1/nx and 1/(nx ny) rounded to FP64, for the index
// divisions of cell_at (make_mesh fills them).
struct Mesh {
    int nx, ny, nz;
    double rnx, rplane;
};

inline Mesh make_mesh(int nx, int ny, int nz) {
    return Mesh{nx, ny, nz, 1.0 / (double)nx, 1.0 / ((double)nx * (double)ny)};
}

// floor(a / d) for 0 <= a < 2^31 and d >= 1, with rd = fl64(1/d).  The FP64
// product is within 2^31 * 2^-52 < 1 of a/d, so the truncated estimate is off
// by at most one; the remainder test corrects it.  About a fifth of the
// instructions of a generic 32-bit division.
__device__ __forceinline__ int div_rcp(int a, int d, double rd) {
    int q = (int)((double)a * rd);
    const int r = a - q * d;
    q += r >= d ? 1 : 0;
    q -= r < 0 ? 1 : 0;
    return q;
}

// One cell of the mesh and the offsets of its six neighbours.  An off-mesh
// neighbour gets offset 0: it reads the cell itself, and its coefficient is
// zero or masked.  Threads past the end take the last cell and own nothing.
struct Cell {
    int idx;
    bool own;
    int dw, de, ds, dn, db, dt;
};

__device__ __forceinline__ Cell cell_at(int g, const Mesh& m, int n) {
    Cell c;
    c.own = g < n;
    c.idx = c.own ? g : n - 1;
    const int plane = m.nx * m.ny;
    const int k = div_rcp(c.idx, plane, m.rplane);
    const int rem = c.idx - k * plane;
    const int j = div_rcp(rem, m.nx, m.rnx);
    const int i = rem - j * m.nx;
    c.dw = i > 0 ? -1 : 0;
    c.de = i < m.nx - 1 ? 1 : 0;
    c.ds = j > 0 ? -m.nx : 0;
    c.dn = j < m.ny - 1 ? m.nx : 0;
    c.db = k > 0 ? -plane : 0;
    c.dt = k < m.nz - 1 ? plane : 0;
    return c;
}

// XCD-aware tile order of a cell-parallel stencil pass.  The chip deals the
// workgroups of a launch to its eight XCDs in turn (workgroup b to XCD b mod
// 8), and each XCD has its own L2.  In plain order the y and z neighbours of
// a workgroup's cells belong to tiles that run on other XCDs, so each XCD
// fetches them into its own L2 again.  Here workgroup b takes tile
// xcd_tile(b) instead: the tiles form rounds of 8 * run, and in each round XCD
// x sweeps the run of tiles [x run, (x + 1) run) in order.  With run about an
// eighth of a plane's tiles, every XCD works through one band of each plane
// after the other, so the rows above and below a tile and the plane below it
// were mostly fetched into the same L2 shortly before.  Tiles of an incomplete
// last round keep their own index.  run <= 1 is plain order.  The partial sums
// are stored by tile, so every sum has the same order as in plain order.
__device__ __forceinline__ int xcd_tile(int b, int nb, int run) {
    if (run <= 1) return b;
    const int span = 8 * run;
    const int w = b % span;
    const int base = b - w;
    if (base + span > nb) return b;
    return base + (w & 7) * run + (w >> 3);
}

// The seven operand values of a cell: centre, west, east, south, north,
// below, above.
template <class V>
struct Nbr {
    V c, w, e, s, n, b, t;
};

template <class T>
__device__ __forceinline__ Nbr<T> load_nbr(const T* v, const Cell& c) {
    const T* p = v + c.idx;
    return Nbr<T>{p[0], p[c.dw], p[c.de], p[c.ds], p[c.dn], p[c.db], p[c.dt]};
}

template <class T>
__device__ __forceinline__ Nbr<float> nbr_f32(const Nbr<T>& a) {
    return Nbr<float>{to_f32(a.c), to_f32(a.w), to_f32(a.e), to_f32(a.s),
                      to_f32(a.n), to_f32(a.b), to_f32(a.t)};
}

// Coefficients of a cell.  UNIT: unit diagonal (Jacobi-scaled copies, c[0]
// unused).  MASK: zero the coefficient of every off-mesh neighbour, so caller
// data on the boundary faces (even Inf/NaN) never enters.
template <class CT, bool UNIT>
struct Coefs {
    CT a[7];
};

template <class CT, bool UNIT>
__device__ __forceinline__ Coefs<CT, UNIT> load_coefs(const CT* const* c, int idx) {
    Coefs<CT, UNIT> r;
#pragma unroll
    for (int a = UNIT ? 1 : 0; a < 7; ++a) r.a[a] = ld(c[a] + idx);
    return r;
}

// The same with non-temporal loads: each coefficient is read once per pass, so
// it need not take L2 capacity from the stencil operands' neighbour reuse.
template <class CT, bool UNIT>
__device__ __forceinline__ Coefs<CT, UNIT> load_coefs_nt(const CT* const* c, int idx) {
    Coefs<CT, UNIT> r;
#pragma unroll
    for (int a = UNIT ? 1 : 0; a < 7; ++a) r.a[a] = ld_nt(c[a] + idx);
    return r;
}

// diag v + xm w + xp e + ym s + yp n + zm b + zp t, in that order, by FMA.
template <class V, class CT, bool UNIT, bool MASK>
__device__ __forceinline__ V apply7(const Coefs<CT, UNIT>& k, const Nbr<V>& v, const Cell& c) {
    V cw = (V)to_f32(k.a[1]), ce = (V)to_f32(k.a[2]), cs = (V)to_f32(k.a[3]);
    V cn = (V)to_f32(k.a[4]), cb = (V)to_f32(k.a[5]), ct = (V)to_f32(k.a[6]);
    if (MASK) {
        cw = c.dw ? cw : (V)0;
        ce = c.de ? ce : (V)0;
        cs = c.ds ? cs : (V)0;
        cn = c.dn ? cn : (V)0;
        cb = c.db ? cb : (V)0;
        ct = c.dt ? ct : (V)0;
    }
    V acc = UNIT ? v.c : (V)to_f32(k.a[0]) * v.c;
    acc = fmaT(cw, v.w, acc);
    acc = fmaT(ce, v.e, acc);
    acc = fmaT(cs, v.s, acc);
    acc = fmaT(cn, v.n, acc);
    acc = fmaT(cb, v.b, acc);
    acc = fmaT(ct, v.t, acc);
    return acc;
}

// ---------------------------------------------------------------- solver state
struct State {
    double rho, alpha, omega, beta;   // (r0, r_i), alpha_i, omega_i, beta_i
    double sigma, qy, yy, qq;         // (r0, s), (q, y), (y, y), (q, q)
    double rq, ry, rr, nb;            // (r0, q), (r0, y), (r, r), ||b|| of the iterated system
    double tol, res_rec, bb_true, rr_true;  // rtol, last ||r||/||b||, unscaled ||b||^2, ||b - A x||^2
    double rmax, scale, pad_d[2];     // max |r_s| of the last residual pass, IR scale
    int32_t iter, max_iter, done, status;
    int32_t reason, half, beta_bad, nbzero;
    // Jobs of the batch engine run their whole solve on the device: the
    // refinement loop (or the FP32 epilogue) around the inner iteration.
    double rtol_o, inner_tol, rel, inner_res;  // requested tolerance, inner tolerance,
                                               // last true relative residual, last inner residual
    int32_t total, outer, stall, inner_cap;    // iterations so far, outer steps, stalled steps
    int32_t outer_cap, max_total, final, ir;   // caps; final: the job is finished; ir: refinement
    int32_t xzero, ostatus, oreason, trial;    // x = 0 then finish; the job's status and reason;
                                               // trial: a tuning run, which ends with its iteration
};

enum : int32_t { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_BREAKDOWN = 2 };
enum : int32_t { RS_NONE = 0, RS_RHO_ZERO = 1, RS_RS_ZERO = 2, RS_YY_ZERO = 3, RS_NONFINITE = 4 };

__device__ __forceinline__ void set_breakdown(State* st, int32_t reason) {
    st->status = ST_BREAKDOWN;
    st->reason = reason;
    st->done = 1;
}

// ---------------------------------------------------------------- reductions
// Reduction scratch of one system: per-workgroup partials, second-level
// partials and one arrival counter (zero between uses).
//
// A grid-wide sum ends in a "last workgroup" step decided by an atomic ticket.
// The partials are published coherently instead of behind a release fence.
// The workgroup writes its partial with agent-scope atomic stores, which go to
// the device coherence point, not the XCD-private L2.  It waits until they
// have completed (s_waitcnt), then takes the ticket.  The last workgroup reads
// the partials with agent-scope atomic loads.  On this multi-XCD device an
// agent-scope release fence would also write back the XCD's whole L2.  At
// tens of nanoseconds per workgroup, serialized, that fence costs more than
// the pass it ends.
// Passes with at most kSingleMax workgroups finish their sums in-kernel.
// Larger passes only store their workgroup partials; a second kernel
// (k_finish) sums them in runs of kGroup and finishes with the ticket among
// its own few workgroups.  Every sum runs in a fixed index order, so the
// result never depends on arrival order.
struct Red {
    double* part;
    double* gpart;
    uint32_t* cnt;
};

constexpr int kSingleMax = 1024;

__host__ __device__ inline int red_groups(int nblocks) { return (nblocks + kGroup - 1) / kGroup; }
__host__ __device__ inline bool red_split(int nblocks) { return nblocks > kSingleMax; }

__device__ __forceinline__ void publish(double* p, double v) {
    __hip_atomic_store(gbl(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double fetch_published(const double* p) {
    return __hip_atomic_load(gbl(const_cast<double*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Waits until this thread's stores have completed; the signal fences keep the
// compiler from moving memory operations across the wait.
__device__ __forceinline__ void wait_stores() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ __forceinline__ uint32_t take_ticket(uint32_t* cnt) {
    return __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// DPP move of an FP64 value (both 32-bit halves with the same control).
// Lanes of a masked-off row get an unspecified value: no zero fill of the
// destination first, which would add two moves to every step.  The reduction
// below only reads lanes whose every input is defined.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, ROWMASK, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Wavefront reduction on the VALU (DPP), in a fixed order: pairs (quad_perm
// [1,0,3,2]), quads ([2,3,0,1]), half-rows (row_half_mirror), rows
// (row_mirror), then rows 0+1 and 2+3 (row_bcast:15 into rows 1 and 3) and
// all four (row_bcast:31 into rows 2 and 3).  The total is in lane 63, whose
// inputs are all defined; the other lanes end with unspecified values.  All
// 64 lanes must be active.  Values j with bit j of MAXMASK set reduce with
// max (of non-negative values), the others with +.
template <int ND, unsigned MAXMASK>
__device__ __forceinline__ void wave_reduce(double (&a)[ND]) {
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        const bool mx = (MAXMASK >> j) & 1u;
        double v = a[j];
        double t;
        t = dpp_f64<0xB1, 0xf>(v);
        v = mx ? fmax(v, t) : v + t;
        t = dpp_f64<0x4E, 0xf>(v);
        v = mx ? fmax(v, t) : v + t;
        t = dpp_f64<0x141, 0xf>(v);
        v = mx ? fmax(v, t) : v + t;
        t = dpp_f64<0x140, 0xf>(v);
        v = mx ? fmax(v, t) : v + t;
        t = dpp_f64<0x142, 0xa>(v);
        v = mx ? fmax(v, t) : v + t;
        t = dpp_f64<0x143, 0xc>(v);
        v = mx ? fmax(v, t) : v + t;
        a[j] = v;
    }
}

template <int ND, unsigned MAXMASK>
__device__ __forceinline__ double comb(int j, double a, double b) {
    return ((MAXMASK >> j) & 1u) ? fmax(a, b) : a + b;
}

// Workgroup sum of acc, in a fixed order: every thread stores its values in
// LDS; the first wavefront adds the four values of lane l (threads l, l+64,
// l+128, l+192, in that order) and reduces the wavefront with DPP.  Only one
// wavefront of the four runs the DPP sequence.  out is written in thread 0
// only; the other threads' out is left as it was.
// The LDS of block_reduce, one array per kernel whatever instantiations of
// block_reduce the kernel uses.
__device__ __forceinline__ double (*reduce_lds())[kThreads] {
    __shared__ double sm[kMaxDots][kThreads];
    return sm;
}

template <int ND, unsigned MAXMASK>
__device__ __forceinline__ void block_reduce(double (&acc)[ND], double (&out)[ND]) {
    double (*sm)[kThreads] = reduce_lds();
    __syncthreads();  // the previous use of sm is over
#pragma unroll
    for (int j = 0; j < ND; ++j) sm[j][threadIdx.x] = acc[j];
    __syncthreads();
    if (threadIdx.x < kWave) {
        double v[ND];
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            double t = sm[j][threadIdx.x];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) t = comb<ND, MAXMASK>(j, t, sm[j][threadIdx.x + w * kWave]);
            v[j] = t;
        }
        wave_reduce<ND, MAXMASK>(v);
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            const int lo = __builtin_amdgcn_readlane(__double2loint(v[j]), kWave - 1);
            const int hi = __builtin_amdgcn_readlane(__double2hiint(v[j]), kWave - 1);
            if (threadIdx.x == 0) out[j] = __hiloint2double(hi, lo);
        }
    }
}

// Sums src[i*ND + j] for i in [i0, i1) into out (thread 0), in a fixed order:
// thread t adds i = i0 + t, i0 + t + 256, ... in turn, then the workgroup sum.
// The loads of four such steps are issued before their values are added, so
// that a long range costs about one memory round trip per four steps.
// COHERENT: the partials were published by other workgroups of this kernel.
template <int ND, unsigned MAXMASK, bool COHERENT>
__device__ __forceinline__ void sum_range(const double* src, int i0, int i1, double (&out)[ND]) {
    constexpr int kB = 4;
    double s[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) s[j] = 0.0;
    auto ld = [&](int b, int j) {
        const double* p = &src[(size_t)b * ND + j];
        return COHERENT ? fetch_published(p) : *p;
    };
    int b = i0 + (int)threadIdx.x;
    for (; b + (kB - 1) * kThreads < i1; b += kB * kThreads) {
        double v[kB][ND];
#pragma unroll
        for (int k = 0; k < kB; ++k)
#pragma unroll
            for (int j = 0; j < ND; ++j) v[k][j] = ld(b + k * kThreads, j);
#pragma unroll
        for (int k = 0; k < kB; ++k)
#pragma unroll
            for (int j = 0; j < ND; ++j) s[j] = comb<ND, MAXMASK>(j, s[j], v[k][j]);
    }
    for (; b < i1; b += kThreads) {
#pragma unroll
        for (int j = 0; j < ND; ++j) s[j] = comb<ND, MAXMASK>(j, s[j], ld(b, j));
    }
    block_reduce<ND, MAXMASK>(s, out);
}

// In-kernel completion: the workgroup sum goes to part[bid]; the last of nblocks
// workgroups to arrive sums part[0..nblocks) into tot (thread 0) and returns
// true in all its threads.
template <int ND, unsigned MAXMASK = 0u>
__device__ bool reduce_ticket(double (&acc)[ND], double* part, uint32_t* cnt, int nblocks, int bid,
                              double (&tot)[ND]) {
    __shared__ int flag;
    double bsum[ND];
    block_reduce<ND, MAXMASK>(acc, bsum);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < ND; ++j) publish(&part[(size_t)bid * ND + j], bsum[j]);
        wait_stores();
        flag = (take_ticket(cnt) == (uint32_t)(nblocks - 1));
    }
    __syncthreads();
    if (!flag) return false;
    sum_range<ND, MAXMASK, true>(part, 0, nblocks, tot);
    if (threadIdx.x == 0) __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Split completion, first half: store the workgroup sum only.
template <int ND, unsigned MAXMASK = 0u>
__device__ __forceinline__ void reduce_store(double (&acc)[ND], double* part, int bid) {
    double bsum[ND];
    block_reduce<ND, MAXMASK>(acc, bsum);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < ND; ++j) part[(size_t)bid * ND + j] = bsum[j];
    }
}

// Grid-wide sum: in-kernel for small grids (returns true in the completing
// workgroup), or the first half of a split sum (returns false; k_finish ends it).
template <int ND, unsigned MAXMASK = 0u>
__device__ __forceinline__ bool grid_reduce(double (&acc)[ND], const Red& red, int nblocks, int bid,
                                            double (&tot)[ND]) {
    if (red_split(nblocks)) {
        reduce_store<ND, MAXMASK>(acc, red.part, bid);
        return false;
    }
    return reduce_ticket<ND, MAXMASK>(acc, red.part, red.cnt, nblocks, bid, tot);
}

// Split completion, second half, run by the finishing kernel's workgroups:
// workgroup g sums part[g*kGroup .. ) and the last one sums those sums.
template <int ND, unsigned MAXMASK = 0u>
__device__ __forceinline__ bool finish_split(const Red& red, int nblocks, double (&tot)[ND]) {
    // The group sum lands in thread 0 only; the other threads contribute zeros
    // (the identity of both + and max over non-negative values) to the ticket sum.
    double gs[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) gs[j] = 0.0;
    const int g = blockIdx.x;
    sum_range<ND, MAXMASK, false>(red.part, g * kGroup, min(nblocks, (g + 1) * kGroup), gs);
    return reduce_ticket<ND, MAXMASK>(gs, red.gpart, red.cnt, (int)gridDim.x, g, tot);
}

// ---------------------------------------------------------------- system view
// Everything one BiCGStab system needs on the device.  coef: 6 (unit
// diagonal, c[1..6]) or 7 working-precision arrays with outward links zeroed.
template <class T>
struct SysView {
    Mesh m;
    int n;
    int unit;          // 1: Jacobi-scaled (unit diagonal)
    const T* c[7];
    T *r, *rhat, *p, *s, *y, *q;
    float* d;          // FP32 correction accumulated by the iteration
    State* st;
    Red red;
    int cell_blocks;   // workgroups of the cell-parallel passes: ceil(n / 256)
    int stream_blocks; // workgroups of the streaming pass
    int pair_blocks;   // workgroups of the paired passes, ceil(n / 512); 0 if nx is odd
};

// Work split of the streaming pass: chunk b of nb covers a contiguous range
// aligned to 8 elements, so vector loads stay aligned.

// P1 at one cell: s = A p; partial (r0, s).
template <class T, bool UNIT>
__device__ __forceinline__ void cell_p1(const SysView<T>& S, int g, double (&acc)[1]) {
    const Cell c = cell_at(g, S.m, S.n);
    const Nbr<float> pv = nbr_f32(load_nbr(S.p, c));
    const Coefs<T, UNIT> k = load_coefs_nt<T, UNIT>(S.c, c.idx);
    const T rh = ld_nt(S.rhat + c.idx);
    const T sv = from_f32<T>(apply7<float, T, UNIT, false>(k, pv, c));
    if (c.own) S.s[c.idx] = sv;
    acc[0] = c.own ? (double)to_f32(rh) * (double)to_f32(sv) : 0.0;
}

// P2a, workgroup b of the streaming grid: q = r - alpha s, rounded to the
// storage type; partial (q, q) of the rounded q, for the half-step test.
template <class T>
__device__ __forceinline__ void chunk_p2a(const SysView<T>& S, int b, double (&acc)[1]) {
    const float alpha = (float)S.st->alpha;
    const T* __restrict__ r = S.r;
    const T* __restrict__ s = S.s;
    T* __restrict__ q = S.q;
    constexpr int W = kVec<T>;
    const int nv = S.n / W, step = S.stream_blocks * kThreads;
    for (int v = b * kThreads + (int)threadIdx.x; v < nv; v += step) {
        const int i = W * v;
        float rv[W], sv[W];
        ldw_nt<W>(r + i, rv);
        ldw_nt<W>(s + i, sv);
        T qv[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            qv[j] = from_f32<T>(fmaT(-alpha, sv[j], rv[j]));
            const double qd = (double)to_f32(qv[j]);
            acc[0] = fma(qd, qd, acc[0]);
        }
        stw_nt<W>(q + i, qv);
    }
    for (int i = W * nv + b * kThreads + (int)threadIdx.x; i < S.n; i += step) {
        const T qv = from_f32<T>(fmaT(-alpha, to_f32(s[i]), to_f32(r[i])));
        q[i] = qv;
        const double qd = (double)to_f32(qv);
        acc[0] = fma(qd, qd, acc[0]);
    }
}

// P2b at one cell: y = A q stored; partials (q,y), (y,y), (r0,q), (r0,y).
template <class T, bool UNIT>
__device__ __forceinline__ void cell_p2b(const SysView<T>& S, int g, double (&acc)[4]) {
    const Cell c = cell_at(g, S.m, S.n);
    const Nbr<float> qv = nbr_f32(load_nbr(S.q, c));
    const Coefs<T, UNIT> k = load_coefs_nt<T, UNIT>(S.c, c.idx);
    const double rh = (double)to_f32(ld_nt(S.rhat + c.idx));
    const T yt = from_f32<T>(apply7<float, T, UNIT, false>(k, qv, c));
    if (c.own) S.y[c.idx] = yt;
    const double yd = c.own ? (double)to_f32(yt) : 0.0;
    const double qd = c.own ? (double)qv.c : 0.0;
    acc[0] = qd * yd;
    acc[1] = yd * yd;
    acc[2] = rh * qd;
    acc[3] = rh * yd;
}

// The three-pass schedule's P2 at one cell: q = r - alpha s is formed on the
// fly at the cell and its six neighbours (FP32, not stored), y = A q stored;
// partials (q,y), (y,y), (q,q), (r0,q), (r0,y).  P3 then forms the same q
// from r and s again, with the same rounding.
template <class T, bool UNIT>
__device__ __forceinline__ void cell_p2f(const SysView<T>& S, int g, float alpha, double (&acc)[5]) {
    const Cell c = cell_at(g, S.m, S.n);
    const Nbr<float> rv = nbr_f32(load_nbr(S.r, c));
    const Nbr<float> sv = nbr_f32(load_nbr(S.s, c));
    const Coefs<T, UNIT> k = load_coefs_nt<T, UNIT>(S.c, c.idx);
    const double rh = (double)to_f32(ld_nt(S.rhat + c.idx));
    const Nbr<float> qv{fmaT(-alpha, sv.c, rv.c), fmaT(-alpha, sv.w, rv.w), fmaT(-alpha, sv.e, rv.e),
                        fmaT(-alpha, sv.s, rv.s), fmaT(-alpha, sv.n, rv.n), fmaT(-alpha, sv.b, rv.b),
                        fmaT(-alpha, sv.t, rv.t)};
    const T yt = from_f32<T>(apply7<float, T, UNIT, false>(k, qv, c));
    if (c.own) S.y[c.idx] = yt;
    const double yd = c.own ? (double)to_f32(yt) : 0.0;
    const double qd = c.own ? (double)qv.c : 0.0;
    acc[0] = qd * yd;
    acc[1] = yd * yd;
    acc[2] = qd * qd;
    acc[3] = rh * qd;
    acc[4] = rh * yd;
}

// ---------------------------------------------------------------- paired cells
// For meshes with an even nx, a stencil pass can give each thread two
// x-adjacent cells (2t, 2t+1) of the flat order.  A pair never crosses a row,
// and its own values, its y and z neighbours and its coefficients are single
// 8-byte (FP32) or 4-byte (16-bit) accesses: about half the load instructions
// of one cell per thread.  Each cell's stencil sum is formed exactly as in the
// one-cell kernels.
struct F2 {
    float a, b;
};
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ F2 ld2(const float* p) {
    const f32x2 v = *reinterpret_cast<const f32x2*>(p);
    return F2{v.x, v.y};
}
__device__ __forceinline__ F2 ld2_nt(const float* p) {
    const f32x2 v = __builtin_nontemporal_load(gbl(reinterpret_cast<const f32x2*>(p)));
    return F2{v.x, v.y};
}
__device__ __forceinline__ F2 split16(uint32_t u, const bf16*) {
    return F2{__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u)};
}
__device__ __forceinline__ F2 split16(uint32_t u, const f16*) {
    return F2{(float)__builtin_bit_cast(f16, (uint16_t)(u & 0xffffu)),
              (float)__builtin_bit_cast(f16, (uint16_t)(u >> 16))};
}
template <class T>
__device__ __forceinline__ F2 ld2(const T* p) {
    return split16(*reinterpret_cast<const uint32_t*>(p), p);
}
template <class T>
__device__ __forceinline__ F2 ld2_nt(const T* p) {
    return split16(__builtin_nontemporal_load(gbl(reinterpret_cast<const uint32_t*>(p))), p);
}
__device__ __forceinline__ void st2(float* p, float a, float b) {
    *reinterpret_cast<f32x2*>(p) = f32x2{a, b};
}
__device__ __forceinline__ void st2(bf16* p, bf16 a, bf16 b) {
    *reinterpret_cast<uint32_t*>(p) = (uint32_t)a.u | ((uint32_t)b.u << 16);
}
__device__ __forceinline__ void st2(f16* p, f16 a, f16 b) {
    *reinterpret_cast<uint32_t*>(p) =
        (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}

// Non-temporal pair stores, for stencil-pass outputs: nothing reads them back
// from the L2 within the pass, so they should not displace the neighbour planes.
__device__ __forceinline__ void st2_nt(float* p, float a, float b) {
    __builtin_nontemporal_store(f32x2{a, b}, reinterpret_cast<f32x2*>(p));
}
template <class T>
__device__ __forceinline__ void st2_nt(T* p, T a, T b) {
    using U = uint16_t;
    __builtin_nontemporal_store((uint32_t)__builtin_bit_cast(U, a) | ((uint32_t)__builtin_bit_cast(U, b) << 16),
                                reinterpret_cast<uint32_t*>(p));
}

// Pair gp of the mesh: cells 2gp and 2gp+1.  dw and de are the offsets of the
// west neighbour of the first cell and the east neighbour of the second (0
// and 1 at the mesh faces: the cell itself, whose coefficient is zero).
// Threads past the end take the last pair and own nothing.
__device__ __forceinline__ Cell cell2_at(int gp, const Mesh& m, int n) {
    Cell c;
    const int g0 = 2 * gp;
    c.own = g0 < n;
    c.idx = c.own ? g0 : n - 2;
    const int plane = m.nx * m.ny;
    const int k = div_rcp(c.idx, plane, m.rplane);
    const int rem = c.idx - k * plane;
    const int j = div_rcp(rem, m.nx, m.rnx);
    const int i = rem - j * m.nx;
    c.dw = i > 0 ? -1 : 0;
    c.de = i + 1 < m.nx - 1 ? 2 : 1;
    c.ds = j > 0 ? -m.nx : 0;
    c.dn = j < m.ny - 1 ? m.nx : 0;
    c.db = k > 0 ? -plane : 0;
    c.dt = k < m.nz - 1 ? plane : 0;
    return c;
}

template <class T>
__device__ __forceinline__ void load_nbr2(const T* v, const Cell& c, Nbr<float>& v0, Nbr<float>& v1) {
    const T* p = v + c.idx;
    const F2 ce = ld2(p), s = ld2(p + c.ds), nn = ld2(p + c.dn), b = ld2(p + c.db), t = ld2(p + c.dt);
    const float w = to_f32(p[c.dw]), e = to_f32(p[c.de]);
    v0 = Nbr<float>{ce.a, w, ce.b, s.a, nn.a, b.a, t.a};
    v1 = Nbr<float>{ce.b, ce.a, e, s.b, nn.b, b.b, t.b};
}

template <class T, bool UNIT>
__device__ __forceinline__ void load_coefs2_nt(const T* const* c, int idx, Coefs<float, UNIT>& k0,
                                               Coefs<float, UNIT>& k1) {
#pragma unroll
    for (int a = UNIT ? 1 : 0; a < 7; ++a) {
        const F2 v = ld2_nt(c[a] + idx);
        k0.a[a] = v.a;
        k1.a[a] = v.b;
    }
}

// P1 on a pair: s = A p and the pair's part of (r0, s).
template <class T, bool UNIT>
__device__ __forceinline__ void pair_p1(const SysView<T>& S, const Cell& c, double (&acc)[1]) {
    Nbr<float> p0, p1;
    load_nbr2(S.p, c, p0, p1);
    Coefs<float, UNIT> k0, k1;
    load_coefs2_nt<T, UNIT>(S.c, c.idx, k0, k1);
    const F2 rh = ld2_nt(S.rhat + c.idx);
    const T s0 = from_f32<T>(apply7<float, float, UNIT, false>(k0, p0, c));
    const T s1 = from_f32<T>(apply7<float, float, UNIT, false>(k1, p1, c));
    if (c.own) st2_nt(S.s + c.idx, s0, s1);
    acc[0] = c.own ? fma((double)rh.b, (double)to_f32(s1), (double)rh.a * (double)to_f32(s0)) : 0.0;
}

// The three-pass P2 on a pair: q = r - alpha s on the fly, y = A q stored;
// the pair's parts of (q,y), (y,y), (q,q), (r0,q), (r0,y).
template <class T, bool UNIT>
__device__ __forceinline__ void pair_p2f(const SysView<T>& S, const Cell& c, float alpha, double (&acc)[5]) {
    Nbr<float> r0, r1, s0, s1;
    load_nbr2(S.r, c, r0, r1);
    load_nbr2(S.s, c, s0, s1);
    Coefs<float, UNIT> k0, k1;
    load_coefs2_nt<T, UNIT>(S.c, c.idx, k0, k1);
    const F2 rh = ld2_nt(S.rhat + c.idx);
    auto qof = [&](const Nbr<float>& r, const Nbr<float>& s) {
        return Nbr<float>{fmaT(-alpha, s.c, r.c), fmaT(-alpha, s.w, r.w), fmaT(-alpha, s.e, r.e),
                          fmaT(-alpha, s.s, r.s), fmaT(-alpha, s.n, r.n), fmaT(-alpha, s.b, r.b),
                          fmaT(-alpha, s.t, r.t)};
    };
    const Nbr<float> q0 = qof(r0, s0), q1 = qof(r1, s1);
    const T y0 = from_f32<T>(apply7<float, float, UNIT, false>(k0, q0, c));
    const T y1 = from_f32<T>(apply7<float, float, UNIT, false>(k1, q1, c));
    if (c.own) st2_nt(S.y + c.idx, y0, y1);
    const double ya = c.own ? (double)to_f32(y0) : 0.0, yb = c.own ? (double)to_f32(y1) : 0.0;
    const double qa = c.own ? (double)q0.c : 0.0, qb = c.own ? (double)q1.c : 0.0;
    acc[0] = fma(qb, yb, qa * ya);
    acc[1] = fma(yb, yb, ya * ya);
    acc[2] = fma(qb, qb, qa * qa);
    acc[3] = fma((double)rh.b, qb, (double)rh.a * qa);
    acc[4] = fma((double)rh.b, yb, (double)rh.a * ya);
}

// ---------------------------------------------------------------- staged stencil passes
// The stencil passes in a second form (meshes with an even nx of at most
// kLdsMaxNx).  A workgroup takes a tile of kLdsTile consecutive cells of the
// flat order, [c0, c0 + kLdsTile).  It first stages the stencil operand over
// [c0 - nx, c0 + kLdsTile + nx), widened to multiples of 8 cells, into LDS as
// FP32, with zeros outside the mesh: the tile and one row on either side, so
// every x and y neighbour of a tile cell is in LDS.  P2 stages q = r - alpha s,
// formed once per cell as it is staged, instead of loading both r and s at
// every neighbour.  The staging loads are 16-byte accesses in flat order.
// Each thread then takes the pairs (2 consecutive cells) u * kThreads + tid of
// the tile: centre, west, east, south and north from LDS, below and above from
// memory.  A neighbour across a mesh face is another cell of the mesh (or a
// staged zero) whose coefficient is zero in the working copies, so the
// per-cell sum is exactly that of the flat kernels.  Measured at 600x595x1536,
// the flat P2 re-read its two operands' neighbours through the caches at about
// 1.1 ms per pass over a halo-free stream of the same arrays; staging removes
// most of that.
constexpr int kLdsTile = 4096;         // the default tile: 16 cells (8 pairs) per thread
constexpr int kLdsMaxNx = 4096;
constexpr int kLdsMaxFloats = 13056;   // staging LDS of a workgroup: 52 KiB beside the 12 KiB of the reduction

__host__ __device__ inline int lds_lo(int c0, int nx) { return (c0 - nx) >> 3 << 3; }
__host__ __device__ inline int lds_count(int nx, int tile) { return tile + 2 * nx + 16; }
inline int lds_blocks(long long n, int tile) { return (int)((n + tile - 1) / tile); }
// Whether a tile of `tile` cells and its two halo rows fit the staging LDS.
inline bool lds_fits(int nx, int tile) { return nx <= kLdsMaxNx && lds_count(nx, tile) <= kLdsMaxFloats; }

// Stages v (Q: r - alpha s with v = r, w = s) over [lo, lo + cnt) into sm.
template <class T, bool Q>
__device__ __forceinline__ void stage_rows(const T* v, const T* w, float alpha, int lo, int cnt, int n,
                                           float* sm) {
    constexpr int W = kVec<T>;
    for (int e = (int)threadIdx.x; e < cnt / W; e += kThreads) {
        const int g = lo + W * e;
        float a[W], b[W];
        if (g >= 0 && g + W <= n) {
            if constexpr (sizeof(T) == 4) {
                const f32x4 x = *reinterpret_cast<const f32x4*>(v + g);
                a[0] = x.x, a[1] = x.y, a[2] = x.z, a[3] = x.w;
                if (Q) {
                    const f32x4 y = *reinterpret_cast<const f32x4*>(w + g);
                    b[0] = y.x, b[1] = y.y, b[2] = y.z, b[3] = y.w;
                }
            } else {
                const u16x8 x = *reinterpret_cast<const u16x8*>(v + g);
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    T t;
                    const uint16_t u = x[j];
                    __builtin_memcpy(&t, &u, 2);
                    a[j] = to_f32(t);
                }
                if (Q) {
                    const u16x8 y = *reinterpret_cast<const u16x8*>(w + g);
#pragma unroll
                    for (int j = 0; j < W; ++j) {
                        T t;
                        const uint16_t u = y[j];
                        __builtin_memcpy(&t, &u, 2);
                        b[j] = to_f32(t);
                    }
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const bool in = g + j >= 0 && g + j < n;
                a[j] = in ? to_f32(v[g + j]) : 0.0f;
                b[j] = (Q && in) ? to_f32(w[g + j]) : 0.0f;
            }
        }
#pragma unroll
        for (int j = 0; j < W; ++j) sm[W * e + j] = Q ? fmaT(-alpha, b[j], a[j]) : a[j];
    }
}

// The seven operand values of the pair at LDS position L (first cell), with
// the pair's vertical neighbours vb, vt (FP32) from memory.
__device__ __forceinline__ void lds_nbr2(const float* sm, int L, int nx, F2 vb, F2 vt, Nbr<float>& v0,
                                         Nbr<float>& v1) {
    const f32x2 c = *reinterpret_cast<const f32x2*>(sm + L);
    const f32x2 s = *reinterpret_cast<const f32x2*>(sm + L - nx);
    const f32x2 nn = *reinterpret_cast<const f32x2*>(sm + L + nx);
    const float w = sm[L - 1], e = sm[L + 2];
    v0 = Nbr<float>{c.x, w, c.y, s.x, nn.x, vb.a, vt.a};
    v1 = Nbr<float>{c.y, c.x, e, s.y, nn.y, vb.b, vt.b};
}

// Offsets of the cells below and above cell idx (0 across the z faces).
__device__ __forceinline__ void z_offsets(int idx, const Mesh& m, int& db, int& dt) {
    const int plane = m.nx * m.ny;
    const int k = div_rcp(idx, plane, m.rplane);
    db = k > 0 ? -plane : 0;
    dt = k < m.nz - 1 ? plane : 0;
}

// P3, workgroup b of the streaming grid: d += alpha p + omega q;
// r = q - omega y; p = r + beta (p - omega s).  Accumulates (r0, r_{i+1}) and
// (r_{i+1}, r_{i+1}).  In place is safe: every cell reads and writes only
// itself.  Each thread takes kVec<T> consecutive cells per step (16-byte
// non-temporal accesses), and the grid strides over the arrays; the last
// n mod kVec<T> cells are scalar.
template <class T>
__device__ __forceinline__ void p3_math(float alpha, float omega, float beta, float pv, float sv,
                                        float yv, float qv, float& dv, T& rn, T& pn) {
    dv = fmaT(omega, qv, fmaT(alpha, pv, dv));
    rn = from_f32<T>(fmaT(-omega, yv, qv));
    pn = from_f32<T>(fmaT(beta, fmaT(-omega, sv, pv), to_f32(rn)));
}

// QR (three-pass schedule): q is formed from the old r and s, r - alpha s,
// instead of being read.
template <class T, bool QR>
__device__ __forceinline__ void chunk_p3(const SysView<T>& S, int b, double (&acc)[2]) {
    const float alpha = (float)S.st->alpha, omega = (float)S.st->omega, beta = (float)S.st->beta;
    T* __restrict__ p = S.p;
    const T* __restrict__ s = S.s;
    const T* __restrict__ y = S.y;
    const T* __restrict__ q = QR ? S.r : S.q;
    const T* __restrict__ rh = S.rhat;
    T* __restrict__ r = S.r;
    float* __restrict__ d = S.d;
    double a0 = 0.0, a1 = 0.0;
    constexpr int W = kVec<T>;
    const int nv = S.n / W, step = S.stream_blocks * kThreads;
    for (int v = b * kThreads + (int)threadIdx.x; v < nv; v += step) {
        const int i = W * v;
        float pv[W], sv[W], yv[W], qv[W], hv[W], dv[W];
        ldw_nt<W>(p + i, pv);
        ldw_nt<W>(s + i, sv);
        ldw_nt<W>(y + i, yv);
        ldw_nt<W>(q + i, qv);
        ldw_nt<W>(rh + i, hv);
        ldw_nt<W>(d + i, dv);
        if (QR) {
#pragma unroll
            for (int j = 0; j < W; ++j) qv[j] = fmaT(-alpha, sv[j], qv[j]);
        }
        T rn[W], pn[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            p3_math<T>(alpha, omega, beta, pv[j], sv[j], yv[j], qv[j], dv[j], rn[j], pn[j]);
            const double rd = (double)to_f32(rn[j]);
            a0 = fma((double)hv[j], rd, a0);
            a1 = fma(rd, rd, a1);
        }
        stw_nt<W>(d + i, dv);
        stw_nt<W>(r + i, rn);
        stw_nt<W>(p + i, pn);
    }
    for (int i = W * nv + b * kThreads + (int)threadIdx.x; i < S.n; i += step) {
        float dv = d[i];
        T rn, pn;
        const float sv = to_f32(s[i]);
        const float qv = QR ? fmaT(-alpha, sv, to_f32(q[i])) : to_f32(q[i]);
        p3_math<T>(alpha, omega, beta, to_f32(p[i]), sv, to_f32(y[i]), qv, dv, rn, pn);
        d[i] = dv;
        r[i] = rn;
        p[i] = pn;
        const double rd = (double)to_f32(rn);
        a0 = fma((double)to_f32(rh[i]), rd, a0);
        a1 = fma(rd, rd, a1);
    }
    acc[0] = a0;
    acc[1] = a1;
}

// ---------------------------------------------------------------- scalar steps
// After P1: alpha_i = rho_i / (r0, s_i).
__device__ __forceinline__ void tail_p1(State* st, const double (&tot)[1]) {
    const double sigma = tot[0];
    st->sigma = sigma;
    if (sigma == 0.0) {
        set_breakdown(st, RS_RS_ZERO);
        return;
    }
    const double a = st->rho / sigma;
    if (!isfinite(a)) {
        set_breakdown(st, RS_NONFINITE);
        return;
    }
    st->alpha = a;
}

// After P2a: (q, q) for the half-step test.
__device__ __forceinline__ void tail_p2a(State* st, const double (&tot)[1]) { st->qq = tot[0]; }

// After P2b: half-step test on ||q||, else omega_i = (q, y) / (y, y), and
// beta_i = (alpha_i / omega_i) rho_{i+1} / rho_i with rho_{i+1} = (r0, r_{i+1})
// expanded as (r0, q_i) - omega_i (r0, y_i), so that P3 can form p_{i+1} in the
// same pass as r_{i+1}.  P3 also computes (r0, r_{i+1}) directly.  That exact
// value becomes rho for the next iteration and drives the breakdown test.
__device__ __forceinline__ void tail_p2(State* st, const double (&tot)[4]) {
    st->qy = tot[0];
    st->yy = tot[1];
    st->rq = tot[2];
    st->ry = tot[3];
    st->beta = 0.0;
    st->beta_bad = RS_NONE;
    const double qn = sqrt(st->qq) / st->nb;
    if (qn <= st->tol) {
        st->omega = 0.0;  // P3 then adds alpha p only and sets r = q
        st->half = 1;
        return;
    }
    if (tot[1] == 0.0) {
        set_breakdown(st, RS_YY_ZERO);
        return;
    }
    const double w = tot[0] / tot[1];
    if (!isfinite(w)) {
        set_breakdown(st, RS_NONFINITE);
        return;
    }
    st->omega = w;
    const double rho_next = tot[2] - w * tot[3];
    const double beta = (st->alpha / w) * (rho_next / st->rho);
    if (rho_next == 0.0) {
        st->beta_bad = RS_RHO_ZERO;
    } else if (!isfinite(beta)) {
        st->beta_bad = RS_NONFINITE;
    } else {
        st->beta = beta;
    }
}

// Scalar step after the three-pass schedule's P2 (five sums: (q,y), (y,y),
// (q,q), (r0,q), (r0,y)).
__device__ __forceinline__ void tail_p2f(State* st, const double (&tot)[5]) {
    st->qq = tot[2];
    const double t4[4] = {tot[0], tot[1], tot[3], tot[4]};
    tail_p2(st, t4);
}

// After P3: stopping tests, then the breakdown tests on rho_{i+1}.
__device__ __forceinline__ void tail_p3(State* st, const double (&tot)[2]) {
    st->iter += 1;
    st->rr = tot[1];
    const double res = sqrt(tot[1]) / st->nb;
    st->res_rec = res;
    if (st->half) {
        st->status = ST_OK;
        st->done = 1;
        return;
    }
    if (!isfinite(res)) {
        set_breakdown(st, RS_NONFINITE);
        return;
    }
    if (res <= st->tol) {
        st->status = ST_OK;
        st->done = 1;
        return;
    }
    if (st->iter >= st->max_iter) {
        st->status = ST_NOT_CONVERGED;
        st->done = 1;
        return;
    }
    const double rho_new = tot[0];
    if (rho_new == 0.0) {
        set_breakdown(st, RS_RHO_ZERO);
        return;
    }
    if (st->beta_bad) {
        set_breakdown(st, st->beta_bad);
        return;
    }
    st->rho = rho_new;
}

// Start of a (sub)solve: r0 in place, nb^2, (r0, r0) known.
__device__ __forceinline__ void tail_init(State* st, double nb2, double rr, double tol,
                                          int max_iter) {
    st->iter = 0;
    st->max_iter = max_iter;
    st->tol = tol;
    st->done = 0;
    st->status = ST_OK;
    st->reason = RS_NONE;
    st->half = 0;
    st->beta_bad = RS_NONE;
    st->alpha = st->omega = st->beta = 0.0;
    st->nb = sqrt(nb2);
    st->rho = rr;
    st->rr = rr;
    st->nbzero = (nb2 == 0.0);
    if (nb2 == 0.0) {
        st->res_rec = 0.0;
        st->done = 1;
        return;
    }
    const double res = sqrt(rr) / st->nb;
    st->res_rec = res;
    if (!isfinite(res)) {
        set_breakdown(st, RS_NONFINITE);
    } else if (res <= tol) {
        st->done = 1;
    } else if (max_iter <= 0) {
        st->status = ST_NOT_CONVERGED;
        st->done = 1;
    }
}

// ---------------------------------------------------------------- generator
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace s7
