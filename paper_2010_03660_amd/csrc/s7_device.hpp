// Device-side building blocks of the s7 library (gfx950, wave64).
//
// * Storage types and round-to-nearest-even conversions (FP32, BF16, FP16).
// * The z-marching tile engine: one wavefront owns a 62-column x R-row tile
//   of an x-y plane and marches through a chunk of z-planes.  The planes k-1,
//   k and k+1 stay in registers.  x-neighbours come from the adjacent lane
//   (DPP wavefront shift).  y-neighbours come from the adjacent register row.
//   Lanes 0 and 63 and rows 0 and R+1 hold the tile's x/y halo.  Their values
//   are computed but never written.
// * The fused BiCGStab passes over one workgroup tile (4 wavefronts):
//   P1 (p update on the fly + s = A p + (r0,s)), P2 (q on the fly + y = A q +
//   three dots) and the streaming P3 (x, r updates + two dots).
// * Deterministic two-level reductions: FP64 per lane, a fixed wavefront
//   butterfly, a fixed wave order in LDS, per-workgroup partials, and a final
//   fixed-order sum by the last workgroup to arrive (atomic ticket).
// * The scalar steps of Algorithm 1 (alpha, omega, beta, stopping and
//   breakdown tests), run by one thread of that last workgroup.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace s7 {

constexpr int kWave = 64;
constexpr int kTileX = 62;  // output columns per wavefront: lanes 1..62
constexpr int kWaves = 4;   // wavefronts per workgroup, stacked in y
constexpr int kThreads = kWave * kWaves;
constexpr int kMaxDots = 4;

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

// ---------------------------------------------------------------- lane shifts
// DPP wavefront shifts (GFX9 wave_shr:1 / wave_shl:1).  All 64 lanes must be
// active; lanes with no source read 0.
__device__ __forceinline__ float lane_prev(float v) {  // value held by lane - 1
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_next(float v) {  // value held by lane + 1
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double lane_prev(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_next(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x130, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------- geometry
struct Mesh {
    int nx, ny, nz;
};

struct ZTiles {
    int R;         // rows per wavefront tile
    int zc;        // z-planes per tile
    int tiles_x;   // ceil(nx / 62)
    int tiles_y;   // ceil(ny / R)
    int groups_y;  // ceil(tiles_y / 4): workgroup rows
    int chunks;    // ceil(nz / zc)
    int nblocks;   // tiles_x * groups_y * chunks
};

__host__ __device__ inline ZTiles make_ztiles(Mesh m, int R, int zc) {
    ZTiles t;
    t.R = R;
    t.zc = zc;
    t.tiles_x = (m.nx + kTileX - 1) / kTileX;
    t.tiles_y = (m.ny + R - 1) / R;
    t.groups_y = (t.tiles_y + kWaves - 1) / kWaves;
    t.chunks = (m.nz + zc - 1) / zc;
    t.nblocks = t.tiles_x * t.groups_y * t.chunks;
    return t;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Renumber so that each XCD receives one contiguous run of logical tiles.  The
// tiles of a run are x-y neighbours, which share halo lines in that L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
    const int nx = 8;
    const int per = nblocks / nx, rem = nblocks % nx;
    const int xcd = bid % nx, slot = bid / nx;
    return (xcd < rem) ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

// ---------------------------------------------------------------- solver state
struct State {
    double rho, alpha, omega, beta;  // (r0, r_i), alpha_i, omega_i, beta_{i-1}
    double sigma, qy, yy, qq;        // (r0, s), (q, y), (y, y), (q, q)
    double rr, nb, tol, res_rec;     // (r, r), ||b|| of the iterated system, rtol, last ||r||/||b||
    double bb_true, rr_true, rmax, scale;  // unscaled ||b||^2, ||b - A x||^2, max |r|, IR scale
    int32_t iter, max_iter, done, status;
    int32_t reason, half, first, nbzero;
    int32_t pad[8];
    alignas(256) uint32_t ticket;  // arrival counter of the last-block reduction
};

enum : int32_t { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_BREAKDOWN = 2 };
enum : int32_t { RS_NONE = 0, RS_RHO_ZERO = 1, RS_RS_ZERO = 2, RS_YY_ZERO = 3, RS_NONFINITE = 4 };

__device__ __forceinline__ void set_breakdown(State* st, int32_t reason) {
    st->status = ST_BREAKDOWN;
    st->reason = reason;
    st->done = 1;
}

// ---------------------------------------------------------------- reductions
template <int ND>
__device__ __forceinline__ void wave_sum(double (&a)[ND]) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            double o = __shfl_xor(a[j], off, kWave);
            a[j] = a[j] + o;
        }
    }
}

// Values j with bit j of MAXMASK set reduce with max, the others with +.
template <int ND, unsigned MAXMASK>
__device__ __forceinline__ void wave_reduce(double (&a)[ND]) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            double o = __shfl_xor(a[j], off, kWave);
            a[j] = ((MAXMASK >> j) & 1u) ? fmax(a[j], o) : a[j] + o;
        }
    }
}

// Block partial of this workgroup -> partials[slot*ND + j].  Then the arrival
// ticket.  The last workgroup to arrive reduces every partial in a fixed
// order into tot[] (valid in thread 0) and resets the ticket.  Returns true in
// all threads of that workgroup.  The result does not depend on which
// workgroup arrives last.
template <int ND, unsigned MAXMASK = 0u>
__device__ bool reduce_partials(double (&acc)[ND], double* partials, uint32_t* ticket,
                                int nslots, int slot, double (&tot)[ND]) {
    __shared__ double sm[kWaves][kMaxDots];
    __shared__ int last;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    wave_reduce<ND, MAXMASK>(acc);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < ND; ++j) sm[wave][j] = acc[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            double v = sm[0][j];
#pragma unroll
            for (int w = 1; w < kWaves; ++w)
                v = ((MAXMASK >> j) & 1u) ? fmax(v, sm[w][j]) : v + sm[w][j];
            partials[(size_t)slot * ND + j] = v;
        }
        __threadfence();
        uint32_t t = atomicAdd(ticket, 1u);
        last = (t == (uint32_t)(nslots - 1));
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double s[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) s[j] = 0.0;
    for (int b = threadIdx.x; b < nslots; b += kThreads) {
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            double v = __builtin_nontemporal_load(&partials[(size_t)b * ND + j]);
            s[j] = ((MAXMASK >> j) & 1u) ? fmax(s[j], v) : s[j] + v;
        }
    }
    wave_reduce<ND, MAXMASK>(s);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < ND; ++j) sm[wave][j] = s[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            double v = sm[0][j];
#pragma unroll
            for (int w = 1; w < kWaves; ++w)
                v = ((MAXMASK >> j) & 1u) ? fmax(v, sm[w][j]) : v + sm[w][j];
            tot[j] = v;
        }
        *ticket = 0u;
    }
    return true;
}

// ---------------------------------------------------------------- stencil operator
// Coefficient access for the z-march.  CT is the stored coefficient type.  V is
// the arithmetic type.  UNIT: the diagonal is one (Jacobi-scaled system), so
// only six arrays exist: c[1..6].  MASK: force outward coefficients on the
// boundary faces to 0, so caller data there (even Inf/NaN) never enters.
// Summation order: diag v, then xm, xp, ym, yp, zm, zp, by fused multiply-add.
template <class CT, class V, bool UNIT, bool MASK>
struct StencilOp {
    const CT* c[7];
    Mesh m;
    __device__ __forceinline__ V ld(int a, int idx) const { return (V)to_f32v(c[a][idx]); }
    __device__ __forceinline__ static float to_f32v(float v) { return v; }
    __device__ __forceinline__ static float to_f32v(bf16 v) { return to_f32(v); }
    __device__ __forceinline__ static float to_f32v(f16 v) { return to_f32(v); }
    __device__ __forceinline__ V apply(int idx, int x, int y, int k, V v, V w, V e, V s, V n,
                                       V b, V t) const {
        V acc = UNIT ? v : ld(0, idx) * v;
        V cxm = ld(1, idx), cxp = ld(2, idx), cym = ld(3, idx), cyp = ld(4, idx);
        V czm = ld(5, idx), czp = ld(6, idx);
        if (MASK) {
            cxm = (x > 0) ? cxm : (V)0;
            cxp = (x < m.nx - 1) ? cxp : (V)0;
            cym = (y > 0) ? cym : (V)0;
            cyp = (y < m.ny - 1) ? cyp : (V)0;
            czm = (k > 0) ? czm : (V)0;
            czp = (k < m.nz - 1) ? czp : (V)0;
        }
        acc = fmaT(cxm, w, acc);
        acc = fmaT(cxp, e, acc);
        acc = fmaT(cym, s, acc);
        acc = fmaT(cyp, n, acc);
        acc = fmaT(czm, b, acc);
        acc = fmaT(czp, t, acc);
        return acc;
    }
};

// ---------------------------------------------------------------- z-march engine
// One wavefront: tile columns x = tx*62-1 .. tx*62+62 (lane = x - tx*62 + 1),
// rows y = ty*R-1 .. ty*R+R, planes k0-1 .. k1 (k1 exclusive end of the owned
// chunk).  src.get(idx, own) returns the operand value at a cell; own is true
// exactly once per owned cell (interior lane, interior row, owned plane).  The
// source may write its value there (P1 stores p_new).  out.emit(idx, v, Av)
// runs for every owned cell, planes in order, rows in order.
template <int R, class Src, class Op, class Out>
__device__ __forceinline__ void zmarch(const Mesh m, int tx, int ty, int k0, int k1, Src& src,
                                       const Op& op, Out& out) {
    using V = typename Src::V;
    const int lane = threadIdx.x & (kWave - 1);
    const int x = tx * kTileX - 1 + lane;
    const bool xin = (unsigned)x < (unsigned)m.nx;
    const bool xown = xin && lane >= 1 && lane <= kTileX;
    const int y0 = ty * R - 1;
    const int plane = m.nx * m.ny;
    bool yin[R + 2];
    int rowidx[R + 2];
#pragma unroll
    for (int t = 0; t < R + 2; ++t) {
        yin[t] = xin && ((unsigned)(y0 + t) < (unsigned)m.ny);
        rowidx[t] = x + m.nx * (y0 + t);
    }
    V zlo[R], cur[R + 2], nxt[R + 2];
    // plane k0 - 1 (halo plane, interior rows only)
#pragma unroll
    for (int t = 1; t <= R; ++t) {
        zlo[t - 1] = (V)0;
        if (k0 > 0 && yin[t]) zlo[t - 1] = src.get(rowidx[t] + plane * (k0 - 1), false);
    }
    // plane k0 (owned)
#pragma unroll
    for (int t = 0; t < R + 2; ++t) {
        cur[t] = (V)0;
        if (yin[t]) cur[t] = src.get(rowidx[t] + plane * k0, xown && t >= 1 && t <= R);
    }
    for (int k = k0; k < k1; ++k) {
        const int kn = k + 1;
        const bool kin = kn < m.nz;
        const bool kown = kn < k1;
#pragma unroll
        for (int t = 0; t < R + 2; ++t) {
            nxt[t] = (V)0;
            if (kin && yin[t]) nxt[t] = src.get(rowidx[t] + plane * kn, kown && xown && t >= 1 && t <= R);
        }
#pragma unroll
        for (int t = 1; t <= R; ++t) {
            const V w = lane_prev(cur[t]);
            const V e = lane_next(cur[t]);
            if (xown && yin[t]) {
                const int idx = rowidx[t] + plane * k;
                const V av = op.apply(idx, x, y0 + t, k, cur[t], w, e, cur[t - 1], cur[t + 1],
                                      zlo[t - 1], nxt[t]);
                out.emit(idx, cur[t], av);
            }
        }
#pragma unroll
        for (int t = 1; t <= R; ++t) zlo[t - 1] = cur[t];
#pragma unroll
        for (int t = 0; t < R + 2; ++t) cur[t] = nxt[t];
    }
}

// Decode a (remapped) workgroup index into this wavefront's tile.  Returns
// false if the wavefront has no rows (the last workgroup row may be short).
__device__ __forceinline__ bool wave_tile(const ZTiles& zt, const Mesh& m, int L, int& tx, int& ty,
                                          int& k0, int& k1) {
    tx = L % zt.tiles_x;
    int rest = L / zt.tiles_x;
    const int gy = rest % zt.groups_y;
    const int tz = rest / zt.groups_y;
    ty = gy * kWaves + (int)(threadIdx.x / kWave);
    k0 = tz * zt.zc;
    k1 = min(m.nz, k0 + zt.zc);
    return ty < zt.tiles_y;
}

// ---------------------------------------------------------------- sources and sinks
template <class T>
struct SrcLoad {  // plain operand v
    using V = float;
    const T* v;
    __device__ __forceinline__ float get(int idx, bool) const { return to_f32(v[idx]); }
};

struct SrcLoadF64 {
    using V = double;
    const double* v;
    __device__ __forceinline__ double get(int idx, bool) const { return v[idx]; }
};

// P1 operand: p_{i} = r_i + beta_{i-1} (p_{i-1} - omega_{i-1} s_{i-1}) (Algorithm 1,
// last update of the previous iteration); p_0 = r_0.  Rounded to the storage
// type, stored once per owned cell, and applied in its rounded form.
template <class T>
struct SrcP1 {
    using V = float;
    const T *r, *p_old, *s_old;
    T* p_new;
    float beta, omega;
    bool first;
    __device__ __forceinline__ float get(int idx, bool own) const {
        float v;
        if (first) {
            v = to_f32(r[idx]);
        } else {
            v = fmaT(beta, fmaT(-omega, to_f32(s_old[idx]), to_f32(p_old[idx])), to_f32(r[idx]));
        }
        const T vt = from_f32<T>(v);
        if (own) p_new[idx] = vt;
        return to_f32(vt);
    }
};

// P2 operand: q_i = r_i - alpha_i s_i, formed in FP32 and never stored.
template <class T>
struct SrcP2 {
    using V = float;
    const T *r, *s;
    float alpha;
    __device__ __forceinline__ float get(int idx, bool) const {
        return fmaT(-alpha, to_f32(s[idx]), to_f32(r[idx]));
    }
};

template <class T>
struct OutStore {
    T* u;
    __device__ __forceinline__ void emit(int idx, float, float av) { u[idx] = from_f32<T>(av); }
};

// P1 sink: s_i = A p_i stored; accumulates (r0, s_i).
template <class T>
struct OutP1 {
    T* s;
    const T* rhat;
    double acc[1];
    __device__ __forceinline__ void emit(int idx, float, float av) {
        const T st = from_f32<T>(av);
        s[idx] = st;
        acc[0] = fma((double)to_f32(rhat[idx]), (double)to_f32(st), acc[0]);
    }
};

// P2 sink: y_i = A q_i stored; accumulates (q, y), (y, y), (q, q).
template <class T>
struct OutP2 {
    T* y;
    double acc[3];
    __device__ __forceinline__ void emit(int idx, float q, float av) {
        const T yt = from_f32<T>(av);
        y[idx] = yt;
        const double yd = (double)to_f32(yt), qd = (double)q;
        acc[0] = fma(qd, yd, acc[0]);
        acc[1] = fma(yd, yd, acc[1]);
        acc[2] = fma(qd, qd, acc[2]);
    }
};

// ---------------------------------------------------------------- system view
// Everything one BiCGStab system needs on the device.  coef: 6 (unit
// diagonal) or 7 working-precision arrays with outward links zeroed.
template <class T>
struct SysView {
    Mesh m;
    ZTiles zt;
    int n;
    int unit;          // 1: Jacobi-scaled (unit diagonal, c[1..6] used)
    const T* c[7];
    T *r, *rhat, *y;
    T *p[2], *s[2];
    float* d;          // FP32 correction accumulated by the iteration
    State* st;
    double* partials;
    int stream_blocks; // workgroups of the streaming pass
};

// Work split of the streaming pass: chunk b of nb covers a contiguous range
// aligned to 8 elements, so vector loads stay aligned.
__host__ __device__ inline void stream_range(int n, int nb, int b, int& i0, int& i1) {
    const int n8 = (n + 7) / 8;
    const int per = (n8 + nb - 1) / nb;
    i0 = min(n, b * per * 8);
    i1 = min(n, (b + 1) * per * 8);
}

// P1 over one workgroup tile.  Returns the partial (r0, s) in acc[0].
template <class T, int R>
__device__ __forceinline__ void wg_p1(const SysView<T>& S, int L, int par, double (&acc)[1]) {
    int tx, ty, k0, k1;
    acc[0] = 0.0;
    if (!wave_tile(S.zt, S.m, L, tx, ty, k0, k1)) return;
    SrcP1<T> src{S.r, S.p[par], S.s[par], S.p[par ^ 1], (float)S.st->beta, (float)S.st->omega,
                 S.st->first != 0};
    OutP1<T> out{S.s[par ^ 1], S.rhat, {0.0}};
    if (S.unit) {
        StencilOp<T, float, true, false> op{{S.c[0], S.c[1], S.c[2], S.c[3], S.c[4], S.c[5], S.c[6]}, S.m};
        zmarch<R>(S.m, tx, ty, k0, k1, src, op, out);
    } else {
        StencilOp<T, float, false, false> op{{S.c[0], S.c[1], S.c[2], S.c[3], S.c[4], S.c[5], S.c[6]}, S.m};
        zmarch<R>(S.m, tx, ty, k0, k1, src, op, out);
    }
    acc[0] = out.acc[0];
}

// P2 over one workgroup tile (reads s of parity par^1, the one P1 wrote).
template <class T, int R>
__device__ __forceinline__ void wg_p2(const SysView<T>& S, int L, int par, double (&acc)[3]) {
    int tx, ty, k0, k1;
    acc[0] = acc[1] = acc[2] = 0.0;
    if (!wave_tile(S.zt, S.m, L, tx, ty, k0, k1)) return;
    SrcP2<T> src{S.r, S.s[par ^ 1], (float)S.st->alpha};
    OutP2<T> out{S.y, {0.0, 0.0, 0.0}};
    if (S.unit) {
        StencilOp<T, float, true, false> op{{S.c[0], S.c[1], S.c[2], S.c[3], S.c[4], S.c[5], S.c[6]}, S.m};
        zmarch<R>(S.m, tx, ty, k0, k1, src, op, out);
    } else {
        StencilOp<T, float, false, false> op{{S.c[0], S.c[1], S.c[2], S.c[3], S.c[4], S.c[5], S.c[6]}, S.m};
        zmarch<R>(S.m, tx, ty, k0, k1, src, op, out);
    }
    acc[0] = out.acc[0];
    acc[1] = out.acc[1];
    acc[2] = out.acc[2];
}

// P3 over one contiguous chunk: q = r - alpha s; d += alpha p + omega q;
// r = q - omega y.  Accumulates (r0, r_{i+1}) and (r_{i+1}, r_{i+1}).  In place is
// safe: every cell reads and writes only itself.
template <class T>
__device__ __forceinline__ void chunk_p3(const SysView<T>& S, int b, int par, double (&acc)[2]) {
    int i0, i1;
    stream_range(S.n, S.stream_blocks, b, i0, i1);
    const float alpha = (float)S.st->alpha, omega = (float)S.st->omega;
    const T* __restrict__ p = S.p[par ^ 1];
    const T* __restrict__ s = S.s[par ^ 1];
    const T* __restrict__ y = S.y;
    const T* __restrict__ rh = S.rhat;
    T* __restrict__ r = S.r;
    float* __restrict__ d = S.d;
    double a0 = 0.0, a1 = 0.0;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += kThreads) {
        const float q = fmaT(-alpha, to_f32(s[i]), to_f32(r[i]));
        d[i] = fmaT(omega, q, fmaT(alpha, to_f32(p[i]), d[i]));
        const T rn = from_f32<T>(fmaT(-omega, to_f32(y[i]), q));
        r[i] = rn;
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

// After P2: half-step test on ||q||, else omega_i = (q, y) / (y, y).
__device__ __forceinline__ void tail_p2(State* st, const double (&tot)[3]) {
    st->qy = tot[0];
    st->yy = tot[1];
    st->qq = tot[2];
    const double qn = sqrt(tot[2]) / st->nb;
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
}

// After P3: stopping tests, then beta_i = (alpha/omega) (r0, r_{i+1}) / (r0, r_i).
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
    const double beta = (st->alpha / st->omega) * (rho_new / st->rho);
    if (!isfinite(beta)) {
        set_breakdown(st, RS_NONFINITE);
        return;
    }
    st->beta = beta;
    st->rho = rho_new;
    st->first = 0;
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
    st->first = 1;
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
