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

// ---------------------------------------------------------------- streaming access
// Non-temporal loads and stores for data touched once per pass (coefficients,
// r0, and the vectors a pass writes).  The cached path is kept for operands
// whose halo neighbours re-read them.
__device__ __forceinline__ float ld_nt(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ f16 ld_nt(const f16* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ bf16 ld_nt(const bf16* p) {
    bf16 r;
    r.u = __builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p));
    return r;
}
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
// load() fetches the raw coefficients of a cell.  apply() forms
// diag v + xm w + xp e + ym s + yp n + zm b + zp t, in that order, by FMA.
template <class CT, class V, bool UNIT, bool MASK>
struct StencilOp {
    const CT* c[7];
    Mesh m;
    struct Raw {
        CT a[7];
    };
    __device__ __forceinline__ Raw load(int idx) const {
        Raw r;
#pragma unroll
        for (int a = UNIT ? 1 : 0; a < 7; ++a) r.a[a] = c[a][idx];
        return r;
    }
    __device__ __forceinline__ V apply(const Raw& r, int x, int y, int k, V v, V w, V e, V s,
                                       V n, V b, V t) const {
        V acc = UNIT ? v : (V)to_f32(r.a[0]) * v;
        V cxm = (V)to_f32(r.a[1]), cxp = (V)to_f32(r.a[2]), cym = (V)to_f32(r.a[3]);
        V cyp = (V)to_f32(r.a[4]), czm = (V)to_f32(r.a[5]), czp = (V)to_f32(r.a[6]);
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
// chunk).  Each z-step first issues every load it needs: the operand of plane
// k+1 on all R+2 rows, and the coefficients and sink inputs of plane k.  Loads
// go to clamped, in-mesh addresses and are masked afterwards with selects.  So
// no load waits behind a branch or behind a store that might alias it.  Only
// stores are predicated.
//   Src: Raw load(idx); V value(raw, idx, valid, own).  own is true exactly once
//     per owned cell (interior lane, interior row, owned plane); the source may
//     then store its value there (P1 stores p_new).
//   Op:  Raw load(idx); V apply(raw, x, y, k, v, w, e, s, n, b, t).
//   Out: Raw load(idx); void emit(raw, idx, own, v, Av); acts only where own.
// Owned cells are visited plane by plane, rows in order.
template <int R, class Src, class Op, class Out>
__device__ __forceinline__ void zmarch(const Mesh m, int tx, int ty, int k0, int k1, Src& src,
                                       const Op& op, Out& out) {
    using V = typename Src::V;
    using SR = typename Src::Raw;
    using CR = typename Op::Raw;
    using OR = typename Out::Raw;
    const int lane = threadIdx.x & (kWave - 1);
    const int x = tx * kTileX - 1 + lane;
    const bool xin = (unsigned)x < (unsigned)m.nx;
    const bool xown = xin && lane >= 1 && lane <= kTileX;
    const int xc = min(max(x, 0), m.nx - 1);
    const int y0 = ty * R - 1;
    const int plane = m.nx * m.ny;
    bool yin[R + 2];
    int rowidx[R + 2];
#pragma unroll
    for (int t = 0; t < R + 2; ++t) {
        const int y = y0 + t;
        yin[t] = xin && ((unsigned)y < (unsigned)m.ny);
        rowidx[t] = xc + m.nx * min(max(y, 0), m.ny - 1);
    }
    V zlo[R], cur[R + 2], nxt[R + 2];
    SR sr[R + 2];
    {  // planes k0 - 1 (halo plane, interior rows only) and k0 (owned)
        const int kk = max(k0 - 1, 0);
#pragma unroll
        for (int t = 1; t <= R; ++t) sr[t] = src.load(rowidx[t] + plane * kk);
#pragma unroll
        for (int t = 1; t <= R; ++t)
            zlo[t - 1] = src.value(sr[t], rowidx[t] + plane * kk, k0 > 0 && yin[t], false);
#pragma unroll
        for (int t = 0; t < R + 2; ++t) sr[t] = src.load(rowidx[t] + plane * k0);
#pragma unroll
        for (int t = 0; t < R + 2; ++t)
            cur[t] = src.value(sr[t], rowidx[t] + plane * k0, yin[t],
                               xown && yin[t] && t >= 1 && t <= R);
    }
    for (int k = k0; k < k1; ++k) {
        const int kn = k + 1;
        const bool kin = kn < m.nz;
        const bool kown = kn < k1;
        const int kc = kin ? kn : k;
        CR cr[R];
        OR orr[R];
        // ---- loads
#pragma unroll
        for (int t = 0; t < R + 2; ++t) sr[t] = src.load(rowidx[t] + plane * kc);
#pragma unroll
        for (int t = 1; t <= R; ++t) cr[t - 1] = op.load(rowidx[t] + plane * k);
#pragma unroll
        for (int t = 1; t <= R; ++t) orr[t - 1] = out.load(rowidx[t] + plane * k);
        // ---- compute and stores
#pragma unroll
        for (int t = 0; t < R + 2; ++t)
            nxt[t] = src.value(sr[t], rowidx[t] + plane * kc, kin && yin[t],
                               kown && xown && yin[t] && t >= 1 && t <= R);
#pragma unroll
        for (int t = 1; t <= R; ++t) {
            const V w = lane_prev(cur[t]);
            const V e = lane_next(cur[t]);
            const V av = op.apply(cr[t - 1], x, y0 + t, k, cur[t], w, e, cur[t - 1], cur[t + 1],
                                  zlo[t - 1], nxt[t]);
            out.emit(orr[t - 1], rowidx[t] + plane * k, xown && yin[t], cur[t], av);
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
struct NoRaw {};

template <class T>
struct SrcLoad {  // plain operand v
    using V = float;
    using Raw = T;
    const T* v;
    __device__ __forceinline__ T load(int idx) const { return v[idx]; }
    __device__ __forceinline__ float value(T a, int, bool valid, bool) const {
        return valid ? to_f32(a) : 0.0f;
    }
};

struct SrcLoadF64 {
    using V = double;
    using Raw = double;
    const double* v;
    __device__ __forceinline__ double load(int idx) const { return v[idx]; }
    __device__ __forceinline__ double value(double a, int, bool valid, bool) const {
        return valid ? a : 0.0;
    }
};

// P1 operand: p_{i} = r_i + beta_{i-1} (p_{i-1} - omega_{i-1} s_{i-1}) (Algorithm 1,
// last update of the previous iteration); p_0 = r_0.  Rounded to the storage
// type, stored once per owned cell, and applied in its rounded form.  p_old and
// s_old are read in the first iteration too (and ignored), so the loads never
// sit behind a branch.
template <class T>
struct SrcP1 {
    using V = float;
    struct Raw {
        T r, p, s;
    };
    const T *r, *p_old, *s_old;
    T* p_new;
    float beta, omega;
    bool first;
    __device__ __forceinline__ Raw load(int idx) const { return Raw{r[idx], p_old[idx], s_old[idx]}; }
    __device__ __forceinline__ float value(const Raw& a, int idx, bool valid, bool own) const {
        const float rv = to_f32(a.r);
        const float v = first ? rv : fmaT(beta, fmaT(-omega, to_f32(a.s), to_f32(a.p)), rv);
        const T vt = from_f32<T>(v);
        if (own) p_new[idx] = vt;
        return valid ? to_f32(vt) : 0.0f;
    }
};

// P2 operand: q_i = r_i - alpha_i s_i, formed in FP32 and never stored.
template <class T>
struct SrcP2 {
    using V = float;
    struct Raw {
        T r, s;
    };
    const T *r, *s;
    float alpha;
    __device__ __forceinline__ Raw load(int idx) const { return Raw{r[idx], s[idx]}; }
    __device__ __forceinline__ float value(const Raw& a, int, bool valid, bool) const {
        const float q = fmaT(-alpha, to_f32(a.s), to_f32(a.r));
        return valid ? q : 0.0f;
    }
};

template <class T>
struct OutStore {
    using Raw = NoRaw;
    T* u;
    __device__ __forceinline__ NoRaw load(int) const { return NoRaw{}; }
    __device__ __forceinline__ void emit(NoRaw, int idx, bool own, float, float av) {
        if (own) u[idx] = from_f32<T>(av);
    }
};

// P1 sink: s_i = A p_i stored; accumulates (r0, s_i).
template <class T>
struct OutP1 {
    using Raw = T;
    T* s;
    const T* rhat;
    double acc[1];
    __device__ __forceinline__ T load(int idx) const { return rhat[idx]; }
    __device__ __forceinline__ void emit(T rh, int idx, bool own, float, float av) {
        const T st = from_f32<T>(av);
        if (own) s[idx] = st;
        acc[0] = fma(own ? (double)to_f32(rh) : 0.0, (double)to_f32(st), acc[0]);
    }
};

// P2 sink: y_i = A q_i stored; accumulates (q, y), (y, y), (q, q).
template <class T>
struct OutP2 {
    using Raw = NoRaw;
    T* y;
    double acc[3];
    __device__ __forceinline__ NoRaw load(int) const { return NoRaw{}; }
    __device__ __forceinline__ void emit(NoRaw, int idx, bool own, float q, float av) {
        const T yt = from_f32<T>(av);
        if (own) y[idx] = yt;
        const double yd = own ? (double)to_f32(yt) : 0.0, qd = own ? (double)q : 0.0;
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
// safe: every cell reads and writes only itself.  Four consecutive cells per
// thread and step, with 16-byte (FP32) or 8-byte (16-bit) non-temporal accesses.
// Chunk bounds are multiples of 8 cells except at the end of the array, so the
// vector accesses stay aligned; the last chunk's tail (< 4 cells) is scalar.
template <class T>
__device__ __forceinline__ void p3_cell(const SysView<T>& S, int i, float alpha, float omega,
                                        int par, double& a0, double& a1) {
    const T* p = S.p[par ^ 1];
    const T* s = S.s[par ^ 1];
    const float q = fmaT(-alpha, to_f32(s[i]), to_f32(S.r[i]));
    S.d[i] = fmaT(omega, q, fmaT(alpha, to_f32(p[i]), S.d[i]));
    const T rn = from_f32<T>(fmaT(-omega, to_f32(S.y[i]), q));
    S.r[i] = rn;
    const double rd = (double)to_f32(rn);
    a0 = fma((double)to_f32(S.rhat[i]), rd, a0);
    a1 = fma(rd, rd, a1);
}

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
    const int nv = (i1 - i0) / 4;
    for (int v = (int)threadIdx.x; v < nv; v += kThreads) {
        const int i = i0 + 4 * v;
        float pv[4], sv[4], yv[4], rv[4], hv[4], dv[4];
        ld4_nt(p + i, pv);
        ld4_nt(s + i, sv);
        ld4_nt(y + i, yv);
        ld4_nt(r + i, rv);
        ld4_nt(rh + i, hv);
        ld4_nt(d + i, dv);
        T rn[4];
        float rnf[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float q = fmaT(-alpha, sv[j], rv[j]);
            dv[j] = fmaT(omega, q, fmaT(alpha, pv[j], dv[j]));
            rn[j] = from_f32<T>(fmaT(-omega, yv[j], q));
            rnf[j] = to_f32(rn[j]);
            const double rd = (double)rnf[j];
            a0 = fma((double)hv[j], rd, a0);
            a1 = fma(rd, rd, a1);
        }
        st4_nt(d + i, dv);
        st4_nt(r + i, rn);
    }
    for (int i = i0 + 4 * nv + (int)threadIdx.x; i < i1; i += kThreads) p3_cell(S, i, alpha, omega, par, a0, a1);
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
