// Pipelined BiCGStab (the one-reduction variant of Cools and Vanroose, 2017)
// for many systems in one persistent launch: the batched form of the solve in
// s7_pipelined.hpp, on the claim-and-complete machinery of the classical
// batched kernel (s7_batched_kernels.hpp).
//
// In the persistent kernel a phase boundary is a hand-off between workgroups:
// every chunk of the phase must be done before any chunk of the next starts.
// Of the four passes of the multi-kernel form, the two streaming ones are
// merged into the stencil pass that follows them, by forming their output at
// the stencil's neighbour cells from the vectors it is computed from:
//   A  z = t + beta (z - omega v) at the cell and its six neighbours, v = A z,
//      p, s, q, y at the cell; all ten sums of the iteration.  Its completion
//      takes every decision of the iteration (the stop test on r_i, omega,
//      beta, the next alpha).
//   B  w = y - omega (t - alpha v) at the cell and its neighbours, t = A w,
//      d += alpha p + omega q, r = q - omega y at the cell.  No sums.
// Two hand-offs per iteration, against three for the classical P1, P2, P3.
// A reads z and v at neighbour cells and writes new z and v; B does the same
// for t.  So z, v and t are kept twice and the copies alternate: a phase
// reads one copy and writes the other, and no chunk overwrites a value that
// a neighbouring chunk of the same phase still reads.  The FP32 arithmetic of
// every vector element is that of the multi-kernel form, term for term.
//
// Residual replacement every kReplace iterations, and at once after a
// candidate stop: R (r = b - A (x + d), FP64), WS (w = A r, s = A p; x += d,
// d = 0), TZ (t = A w, z = A s), V (v = A z and the sums (r0, r), (r0, w),
// (r0, s), (r0, z), (r, r), which decide a candidate stop on the true
// residual).  The start is S (r0 = b - A x0) followed by WS, TZ and V, which
// give w_0, t_0 and alpha_0.  The end is X (x += d) and the FP64 true
// residual, as for a classical FP32 job.  Sums are kept per unit of
// kUnitCells cells as in the classical kernel, so a system's iterates depend
// on nothing but the system.  FP32 storage, 7-point operator.  Included by
// the solver translation unit (s7_single.hip) after s7_pipelined.hpp.
#pragma once

namespace s7 {

// A pipelined job's control block: the State, the pipelined scalars, which
// copy of z and v (zb) and of t (tb) is current, and the iterations since the
// last replacement.  It sits where a classical job keeps its State, in the
// space before the partial sums.
struct PState {
    State st;
    PipeScalars ps;
    int32_t zb, tb, since, pad;
};
constexpr int kPStateWords = (int)(sizeof(PState) / 4);
static_assert(sizeof(PState) % 4 == 0 && kPStateWords <= kThreads, "PState is copied one word per thread");
static_assert(sizeof(PState) <= (sizeof(State) + 255) / 256 * 256, "PState fits before the partial sums");

// Phase kinds; a phase sequence number is (count << 4) | kind.  PK_S has the
// value of the classical K_S, so the shared job start kernel sets it.
enum PipeKind : int {
    PK_A = 0, PK_B = 1, PK_R = 2, PK_WS = 3, PK_TZ = 4, PK_V = 5, PK_S = 6, PK_X = 7, PK_RF = 8, PK_FINAL = 9
};
static_assert((int)PK_S == (int)K_S, "the job start kernel sets the first phase");
__host__ __device__ inline uint32_t pseq_next(uint32_t seq, int kind) {
    return (((seq >> 4) + 1u) << 4) | (uint32_t)kind;
}

// One system of a pipelined launch.
struct PSys {
    SysView<float> S;  // r, r0, p, s, y, q, d, working coefficients; S.st is the PState
    BCtl* ctl;
    float* z[2];
    float* v[2];
    float* t[2];
    float* w;
    int nchunk;
    int chunk;  // cells per work item (a multiple of kUnitCells)
    Coef7 cf;   // the caller's coefficients (residual passes)
    const double* b;
    double* x;
};

// ---------------------------------------------------------------- unit sums
// Up to kPD sums per unit of kUnitCells cells, reduced over the wavefront and
// published by lane 63 (as unit_done, with a wider stride).
constexpr int kPD = 10;
template <int ND, unsigned MAXMASK, int NA>
__device__ __forceinline__ void punit_done(const double (&acc)[NA], double* part, int unit) {
    if constexpr (ND > 0) {
        double v[ND];
#pragma unroll
        for (int j = 0; j < ND; ++j) v[j] = acc[j];
        wave_reduce<ND, MAXMASK>(v);
        if (lane_id() == kWave - 1) {
#pragma unroll
            for (int j = 0; j < ND; ++j) publish(&part[(size_t)unit * kPD + j], v[j]);
        }
    }
}

// The units of chunk [c0, c1), wavefront w taking units w, w + kWaves, ...;
// f(u0, u1, acc) sums one unit's cells into an acc of NA values.
template <int NA, int ND, unsigned MAXMASK, class F>
__device__ __forceinline__ void pover_units(int c0, int c1, double* part, F&& f) {
    for (int u0 = c0 + wave_id() * kUnitCells; u0 < c1; u0 += kUnitGroup) {
        double acc[NA];
#pragma unroll
        for (int j = 0; j < NA; ++j) acc[j] = 0.0;
        f(u0, min(c1, u0 + kUnitCells), acc);
        punit_done<ND, MAXMASK>(acc, part, u0 / kUnitCells);
    }
}

// The completer's sums over the units [0, nunit), in unit order per thread
// (thread t adds units t, t + 256, ...), then the workgroup sum of each value;
// the workgroup reduction takes at most five values at a time.  Result in
// thread 0.
template <int ND, unsigned MAXMASK>
__device__ __forceinline__ void psum_units(const double* part, int nunit, double (&out)[kPD]) {
    double s[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) s[j] = 0.0;
    for (int u = (int)threadIdx.x; u < nunit; u += kThreads) {
        double v[ND];
#pragma unroll
        for (int j = 0; j < ND; ++j) v[j] = fetch_published(&part[(size_t)u * kPD + j]);
#pragma unroll
        for (int j = 0; j < ND; ++j) s[j] = comb<ND, MAXMASK>(j, s[j], v[j]);
    }
    constexpr int L = ND < 5 ? ND : 5;
    double a[L], oa[L];
#pragma unroll
    for (int j = 0; j < L; ++j) a[j] = s[j];
    block_reduce<L, MAXMASK & 31u>(a, oa);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < L; ++j) out[j] = oa[j];
    }
    if constexpr (ND > 5) {
        constexpr int H = ND - 5;
        double b[H], ob[H];
#pragma unroll
        for (int j = 0; j < H; ++j) b[j] = s[5 + j];
        block_reduce<H, (MAXMASK >> 5)>(b, ob);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int j = 0; j < H; ++j) out[5 + j] = ob[j];
        }
    }
}

// ---------------------------------------------------------------- chunk work
// The cells of step `base` of a unit [u0, u1): lane l takes cells
// base + 64 u + l for u < kPU, so its cells come in the order l, l + 64,
// l + 128, ... whatever kPU is.  A cell at or past u1 is replaced by u0 and
// keeps nothing.  The loads of a step are issued before any of its stores.
constexpr int kPU = 2;
__device__ __forceinline__ Cell pcell(int base, int u, int u0, int u1, const Mesh& m, int n) {
    const int g = base + u * kWave + lane_id();
    Cell c = cell_at(g < u1 ? g : u0, m, n);
    c.own = g < u1;
    return c;
}

// A of one unit.  zo, vo: the current z and v; zn, vn: the other copies, which
// receive the new ones.  Sums: (r0, y), (r0, t), (r0, s), (r0, z), (r, r),
// (q, y), (y, y), (q, q), (r0, q), (r0, v).
template <bool UNIT>
__device__ void pchunk_a(const PSys& B, const float* zo, const float* vo, float* zn, float* vn, const float* t,
                         int u0, int u1, float a, float bt, float om, double (&acc)[kPD]) {
    const SysView<float>& S = B.S;
    auto zf = [&](float tt, float zz, float vx) { return fmaT(bt, fmaT(-om, vx, zz), tt); };
    for (int base = u0; base < u1; base += kPU * kWave) {
        Cell c[kPU];
        Nbr<float> z[kPU];
        Coefs<float, UNIT> k[kPU];
        float r[kPU], w[kPU], p0[kPU], s0[kPU], h[kPU], zc[kPU], tc[kPU];
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            c[u] = pcell(base, u, u0, u1, S.m, S.n);
            const int i = c[u].idx;
            const Nbr<float> tv = cload_nbr(t, c[u]), zv = cload_nbr(zo, c[u]), vv = cload_nbr(vo, c[u]);
            // z = t + beta (z - omega v) at the cell and its neighbours
            z[u] = Nbr<float>{zf(tv.c, zv.c, vv.c), zf(tv.w, zv.w, vv.w), zf(tv.e, zv.e, vv.e),
                              zf(tv.s, zv.s, vv.s), zf(tv.n, zv.n, vv.n), zf(tv.b, zv.b, vv.b),
                              zf(tv.t, zv.t, vv.t)};
            zc[u] = zv.c;
            tc[u] = tv.c;
            k[u] = load_coefs<float, UNIT>(S.c, i);
            r[u] = cload(S.r + i), w[u] = cload(B.w + i), p0[u] = cload(S.p + i), s0[u] = cload(S.s + i);
            h[u] = cload(S.rhat + i);
        }
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            if (!c[u].own) continue;
            const int i = c[u].idx;
            const float v = apply7<float, float, UNIT, false>(k[u], z[u], c[u]);
            const float p = fmaT(bt, fmaT(-om, s0[u], p0[u]), r[u]);
            const float s = fmaT(bt, fmaT(-om, zc[u], s0[u]), w[u]);
            const float q = fmaT(-a, s, r[u]);
            const float y = fmaT(-a, z[u].c, w[u]);
            cstore(S.p + i, p);
            cstore(S.s + i, s);
            cstore(zn + i, z[u].c);
            cstore(vn + i, v);
            cstore(S.q + i, q);
            cstore(S.y + i, y);
            const double hd = h[u], yd = y, qd = q, rd = r[u];
            acc[0] = fma(hd, yd, acc[0]);
            acc[1] = fma(hd, (double)tc[u], acc[1]);
            acc[2] = fma(hd, (double)s, acc[2]);
            acc[3] = fma(hd, (double)z[u].c, acc[3]);
            acc[4] = fma(rd, rd, acc[4]);
            acc[5] = fma(qd, yd, acc[5]);
            acc[6] = fma(yd, yd, acc[6]);
            acc[7] = fma(qd, qd, acc[7]);
            acc[8] = fma(hd, qd, acc[8]);
            acc[9] = fma(hd, (double)v, acc[9]);
        }
    }
}

// B of one unit, full update: to, v: the current t and v; tn receives t = A w.
template <bool UNIT>
__device__ void pchunk_b(const PSys& B, const float* to, const float* v, float* tn, int u0, int u1, float a,
                         float om) {
    const SysView<float>& S = B.S;
    auto wf = [&](float yy, float tt, float vx) { return fmaT(-om, fmaT(-a, vx, tt), yy); };
    for (int base = u0; base < u1; base += kPU * kWave) {
        Cell c[kPU];
        Nbr<float> w[kPU];
        Coefs<float, UNIT> k[kPU];
        float q[kPU], p[kPU], d[kPU], yc[kPU];
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            c[u] = pcell(base, u, u0, u1, S.m, S.n);
            const int i = c[u].idx;
            const Nbr<float> yv = cload_nbr(S.y, c[u]), tv = cload_nbr(to, c[u]), vv = cload_nbr(v, c[u]);
            // w = y - omega (t - alpha v) at the cell and its neighbours
            w[u] = Nbr<float>{wf(yv.c, tv.c, vv.c), wf(yv.w, tv.w, vv.w), wf(yv.e, tv.e, vv.e),
                              wf(yv.s, tv.s, vv.s), wf(yv.n, tv.n, vv.n), wf(yv.b, tv.b, vv.b),
                              wf(yv.t, tv.t, vv.t)};
            yc[u] = yv.c;
            k[u] = load_coefs<float, UNIT>(S.c, i);
            q[u] = cload(S.q + i), p[u] = cload(S.p + i), d[u] = cload(S.d + i);
        }
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            if (!c[u].own) continue;
            const int i = c[u].idx;
            const float tt = apply7<float, float, UNIT, false>(k[u], w[u], c[u]);
            cstore(S.d + i, fmaT(om, q[u], fmaT(a, p[u], d[u])));
            cstore(S.r + i, fmaT(-om, yc[u], q[u]));
            cstore(B.w + i, w[u].c);
            cstore(tn + i, tt);
        }
    }
}

// B of the half-step exit: d += alpha p only.
__device__ void pchunk_b_half(const PSys& B, int u0, int u1, float a) {
    const SysView<float>& S = B.S;
    for (int i = u0 + lane_id(); i < u1; i += kWave) cstore(S.d + i, fmaT(a, cload(S.p + i), cload(S.d + i)));
}

// R: r = fl32((b - A (x + d)) / diag) in FP64 with the caller's coefficients;
// x + d is the value the next phase stores into x.
__device__ void pchunk_r(const PSys& B, int u0, int u1) {
    const SysView<float>& S = B.S;
    for (int base = u0; base < u1; base += kPU * kWave) {
        Cell c[kPU];
        Nbr<double> xv[kPU];
        Coefs<float, false> k[kPU];
        double bi[kPU];
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            c[u] = pcell(base, u, u0, u1, S.m, S.n);
            const double* px = B.x + c[u].idx;
            const float* pd = S.d + c[u].idx;
            auto xd = [&](int o) { return cload(px + o) + (double)cload(pd + o); };
            xv[u] = Nbr<double>{xd(0), xd(c[u].dw), xd(c[u].de), xd(c[u].ds), xd(c[u].dn), xd(c[u].db), xd(c[u].dt)};
            k[u] = load_coefs<float, false>(B.cf.c, c[u].idx);
            bi[u] = *gbl(B.b + c[u].idx);
        }
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            if (!c[u].own) continue;
            const double r0 = bi[u] - apply7<double, float, false, true>(k[u], xv[u], c[u]);
            cstore(S.r + c[u].idx, (float)(S.unit ? r0 / (double)k[u].a[0] : r0));
        }
    }
}

// WS: w = A r, s = A p; x += d, d = 0.
template <bool UNIT>
__device__ void pchunk_ws(const PSys& B, int u0, int u1) {
    const SysView<float>& S = B.S;
    for (int base = u0; base < u1; base += kPU * kWave) {
        Cell c[kPU];
        Nbr<float> rv[kPU], pv[kPU];
        Coefs<float, UNIT> k[kPU];
        float dv[kPU];
        double xv[kPU];
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            c[u] = pcell(base, u, u0, u1, S.m, S.n);
            const int i = c[u].idx;
            rv[u] = cload_nbr(S.r, c[u]), pv[u] = cload_nbr(S.p, c[u]);
            k[u] = load_coefs<float, UNIT>(S.c, i);
            dv[u] = cload(S.d + i);
            xv[u] = cload(B.x + i);
        }
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            if (!c[u].own) continue;
            const int i = c[u].idx;
            cstore(B.w + i, apply7<float, float, UNIT, false>(k[u], rv[u], c[u]));
            cstore(S.s + i, apply7<float, float, UNIT, false>(k[u], pv[u], c[u]));
            cstore(B.x + i, xv[u] + (double)dv[u]);
            cstore(S.d + i, 0.0f);
        }
    }
}

// TZ: t = A w, z = A s (into the current copies).
template <bool UNIT>
__device__ void pchunk_tz(const PSys& B, float* t, float* z, int u0, int u1) {
    const SysView<float>& S = B.S;
    for (int base = u0; base < u1; base += kPU * kWave) {
        Cell c[kPU];
        Nbr<float> wv[kPU], sv[kPU];
        Coefs<float, UNIT> k[kPU];
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            c[u] = pcell(base, u, u0, u1, S.m, S.n);
            wv[u] = cload_nbr(B.w, c[u]), sv[u] = cload_nbr(S.s, c[u]);
            k[u] = load_coefs<float, UNIT>(S.c, c[u].idx);
        }
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            if (!c[u].own) continue;
            cstore(t + c[u].idx, apply7<float, float, UNIT, false>(k[u], wv[u], c[u]));
            cstore(z + c[u].idx, apply7<float, float, UNIT, false>(k[u], sv[u], c[u]));
        }
    }
}

// V: v = A z; sums (r0, r), (r0, w), (r0, s), (r0, z), (r, r).
template <bool UNIT>
__device__ void pchunk_v(const PSys& B, const float* z, float* v, int u0, int u1, double (&acc)[kPD]) {
    const SysView<float>& S = B.S;
    for (int base = u0; base < u1; base += kPU * kWave) {
        Cell c[kPU];
        Nbr<float> zv[kPU];
        Coefs<float, UNIT> k[kPU];
        float h[kPU], r[kPU], w[kPU], s[kPU];
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            c[u] = pcell(base, u, u0, u1, S.m, S.n);
            const int i = c[u].idx;
            zv[u] = cload_nbr(z, c[u]);
            k[u] = load_coefs<float, UNIT>(S.c, i);
            h[u] = cload(S.rhat + i), r[u] = cload(S.r + i), w[u] = cload(B.w + i), s[u] = cload(S.s + i);
        }
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            if (!c[u].own) continue;
            cstore(v + c[u].idx, apply7<float, float, UNIT, false>(k[u], zv[u], c[u]));
            const double hd = h[u], rd = r[u];
            acc[0] = fma(hd, rd, acc[0]);
            acc[1] = fma(hd, (double)w[u], acc[1]);
            acc[2] = fma(hd, (double)s[u], acc[2]);
            acc[3] = fma(hd, (double)zv[u].c, acc[3]);
            acc[4] = fma(rd, rd, acc[4]);
        }
    }
}

// ---------------------------------------------------------------- staged A and B
// For systems with an even nx of at most kStageMaxNx, A and B take the chunk
// one unit group (kStageTile cells) at a time, as the classical staged passes
// do: the group's stencil operand (z for A, w for B) is formed once per cell,
// with one row either side, from its three vectors into LDS; then wavefront w
// takes unit w of the group on x-adjacent cell pairs, reading the centre and
// the x and y neighbours from LDS and forming the z neighbours from coherent
// loads.  Lane l visits the unit's pairs l, l + 64, ... in that order.
//
// sm[g - lo] = f1 (f2 x2[g] + x1[g]) + x0[g] for g in [lo, lo + cnt), 0
// outside the system (A: x0, x1, x2 = t, z, v and f1, f2 = beta, -omega; B:
// y, t, v and -omega, -alpha).  The values were written by other workgroups
// of the launch, so the 16-byte loads bypass the XCD's L2 (volatile, system
// scope); two steps' loads are issued before their LDS stores.
__device__ __forceinline__ f32x4 vload4(const float* p) {
    return *(volatile __attribute__((address_space(1))) f32x4*)gbl(reinterpret_cast<f32x4*>(const_cast<float*>(p)));
}
__device__ void stage3(const float* x0, const float* x1, const float* x2, float f1, float f2, int lo, int cnt, int n,
                       float* sm) {
    auto comb3 = [&](float a0, float a1, float a2) { return fmaT(f1, fmaT(f2, a2, a1), a0); };
    const int nv = cnt / 4;
    for (int e0 = (int)threadIdx.x; e0 < nv; e0 += 2 * kThreads) {
        float a[2][3][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = e0 + h * kThreads;
            const int g = lo + 4 * e;
            if (e < nv && g >= 0 && g + 4 <= n) {
                const f32x4 u = vload4(x0 + g), v = vload4(x1 + g), w = vload4(x2 + g);
                a[h][0][0] = u.x, a[h][0][1] = u.y, a[h][0][2] = u.z, a[h][0][3] = u.w;
                a[h][1][0] = v.x, a[h][1][1] = v.y, a[h][1][2] = v.z, a[h][1][3] = v.w;
                a[h][2][0] = w.x, a[h][2][1] = w.y, a[h][2][2] = w.z, a[h][2][3] = w.w;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const bool in = e < nv && g + j >= 0 && g + j < n;
                    a[h][0][j] = in ? cload(x0 + g + j) : 0.0f;
                    a[h][1][j] = in ? cload(x1 + g + j) : 0.0f;
                    a[h][2][j] = in ? cload(x2 + g + j) : 0.0f;
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = e0 + h * kThreads;
            if (e >= nv) break;
#pragma unroll
            for (int j = 0; j < 4; ++j) sm[4 * e + j] = comb3(a[h][0][j], a[h][1][j], a[h][2][j]);
        }
    }
}

// The combined operand of the pair at idx + off (the cells below or above).
__device__ __forceinline__ F2 comb3_2(const float* x0, const float* x1, const float* x2, float f1, float f2, int i) {
    const F2 a = cload2(x0 + i), b = cload2(x1 + i), c = cload2(x2 + i);
    return F2{fmaT(f1, fmaT(f2, c.a, b.a), a.a), fmaT(f1, fmaT(f2, c.b, b.b), a.b)};
}

// A of the chunk [c0, c1), staged (sums as pchunk_a, per unit).
template <bool UNIT>
__device__ void pstaged_a(const PSys& B, const float* zo, const float* vo, float* zn, float* vn, const float* t,
                          int c0, int c1, float a, float bt, float om, float* sm, double* part) {
    const SysView<float>& S = B.S;
    const int nx = S.m.nx;
    for (int t0 = c0; t0 < c1; t0 += kStageTile) {
        const int t1 = min(c1, t0 + kStageTile);
        const int lo = (t0 - nx) >> 3 << 3, hi = (t1 + nx + 7) >> 3 << 3;
        __syncthreads();  // the previous group's reads of sm are over
        stage3(t, zo, vo, bt, -om, lo, hi - lo, S.n, sm);
        __syncthreads();
        const int u0 = t0 + wave_id() * kUnitCells;
        if (u0 >= t1) continue;  // the same for the whole wavefront
        const int u1 = min(t1, u0 + kUnitCells);
        double acc[kPD] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        constexpr int kSP = 2;  // pairs per lane and step
        for (int u = 0; u < kUnitCells / (2 * kWave); u += kSP) {
            int idx[kSP];
            bool own[kSP];
            Coefs<float, UNIT> k0[kSP], k1[kSP];
            F2 zb[kSP], zt[kSP], r[kSP], w[kSP], p[kSP], s[kSP], h[kSP], zc[kSP], tc[kSP];
#pragma unroll
            for (int q = 0; q < kSP; ++q) {
                const int i = u0 + 2 * ((u + q) * kWave + lane_id());
                own[q] = i < u1;
                idx[q] = own[q] ? i : u0;
                int db, dt;
                z_offsets(idx[q], S.m, db, dt);
                zb[q] = comb3_2(t, zo, vo, bt, -om, idx[q] + db);
                zt[q] = comb3_2(t, zo, vo, bt, -om, idx[q] + dt);
                load_coefs2_nt<float, UNIT>(S.c, idx[q], k0[q], k1[q]);
                r[q] = cload2(S.r + idx[q]), w[q] = cload2(B.w + idx[q]), p[q] = cload2(S.p + idx[q]);
                s[q] = cload2(S.s + idx[q]), h[q] = cload2(S.rhat + idx[q]);
                zc[q] = cload2(zo + idx[q]), tc[q] = cload2(t + idx[q]);
            }
#pragma unroll
            for (int q = 0; q < kSP; ++q) {
                if (!own[q]) continue;
                const int i = idx[q];
                Nbr<float> z0, z1;
                lds_nbr2(sm, i - lo, nx, zb[q], zt[q], z0, z1);
                const Cell none{};
                const float v0 = apply7<float, float, UNIT, false>(k0[q], z0, none);
                const float v1 = apply7<float, float, UNIT, false>(k1[q], z1, none);
                const float pa = fmaT(bt, fmaT(-om, s[q].a, p[q].a), r[q].a);
                const float pb = fmaT(bt, fmaT(-om, s[q].b, p[q].b), r[q].b);
                const float sa = fmaT(bt, fmaT(-om, zc[q].a, s[q].a), w[q].a);
                const float sb = fmaT(bt, fmaT(-om, zc[q].b, s[q].b), w[q].b);
                const float qa = fmaT(-a, sa, r[q].a), qb = fmaT(-a, sb, r[q].b);
                const float ya = fmaT(-a, z0.c, w[q].a), yb = fmaT(-a, z1.c, w[q].b);
                cstore2(S.p + i, pa, pb);
                cstore2(S.s + i, sa, sb);
                cstore2(zn + i, z0.c, z1.c);
                cstore2(vn + i, v0, v1);
                cstore2(S.q + i, qa, qb);
                cstore2(S.y + i, ya, yb);
                const float hs[2] = {h[q].a, h[q].b}, ys[2] = {ya, yb}, ts[2] = {tc[q].a, tc[q].b};
                const float ss[2] = {sa, sb}, zs[2] = {z0.c, z1.c}, rs[2] = {r[q].a, r[q].b};
                const float qs[2] = {qa, qb}, vs[2] = {v0, v1};
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const double hd = hs[e], yd = ys[e], qd = qs[e], rd = rs[e];
                    acc[0] = fma(hd, yd, acc[0]);
                    acc[1] = fma(hd, (double)ts[e], acc[1]);
                    acc[2] = fma(hd, (double)ss[e], acc[2]);
                    acc[3] = fma(hd, (double)zs[e], acc[3]);
                    acc[4] = fma(rd, rd, acc[4]);
                    acc[5] = fma(qd, yd, acc[5]);
                    acc[6] = fma(yd, yd, acc[6]);
                    acc[7] = fma(qd, qd, acc[7]);
                    acc[8] = fma(hd, qd, acc[8]);
                    acc[9] = fma(hd, (double)vs[e], acc[9]);
                }
            }
        }
        punit_done<kPD, 0u>(acc, part, u0 / kUnitCells);
    }
}

// B of the chunk [c0, c1), full update, staged.
template <bool UNIT>
__device__ void pstaged_b(const PSys& B, const float* to, const float* v, float* tn, int c0, int c1, float a,
                          float om, float* sm) {
    const SysView<float>& S = B.S;
    const int nx = S.m.nx;
    for (int t0 = c0; t0 < c1; t0 += kStageTile) {
        const int t1 = min(c1, t0 + kStageTile);
        const int lo = (t0 - nx) >> 3 << 3, hi = (t1 + nx + 7) >> 3 << 3;
        __syncthreads();
        stage3(S.y, to, v, -om, -a, lo, hi - lo, S.n, sm);
        __syncthreads();
        const int u0 = t0 + wave_id() * kUnitCells;
        if (u0 >= t1) continue;
        const int u1 = min(t1, u0 + kUnitCells);
        constexpr int kSP = 2;
        for (int u = 0; u < kUnitCells / (2 * kWave); u += kSP) {
            int idx[kSP];
            bool own[kSP];
            Coefs<float, UNIT> k0[kSP], k1[kSP];
            F2 wb[kSP], wt[kSP], q2[kSP], p2[kSP], d2[kSP], y2[kSP];
#pragma unroll
            for (int q = 0; q < kSP; ++q) {
                const int i = u0 + 2 * ((u + q) * kWave + lane_id());
                own[q] = i < u1;
                idx[q] = own[q] ? i : u0;
                int db, dt;
                z_offsets(idx[q], S.m, db, dt);
                wb[q] = comb3_2(S.y, to, v, -om, -a, idx[q] + db);
                wt[q] = comb3_2(S.y, to, v, -om, -a, idx[q] + dt);
                load_coefs2_nt<float, UNIT>(S.c, idx[q], k0[q], k1[q]);
                q2[q] = cload2(S.q + idx[q]), p2[q] = cload2(S.p + idx[q]), d2[q] = cload2(S.d + idx[q]);
                y2[q] = cload2(S.y + idx[q]);
            }
#pragma unroll
            for (int q = 0; q < kSP; ++q) {
                if (!own[q]) continue;
                const int i = idx[q];
                Nbr<float> w0, w1;
                lds_nbr2(sm, i - lo, nx, wb[q], wt[q], w0, w1);
                const Cell none{};
                const float ta = apply7<float, float, UNIT, false>(k0[q], w0, none);
                const float tb = apply7<float, float, UNIT, false>(k1[q], w1, none);
                cstore2(S.d + i, fmaT(om, q2[q].a, fmaT(a, p2[q].a, d2[q].a)),
                        fmaT(om, q2[q].b, fmaT(a, p2[q].b, d2[q].b)));
                cstore2(S.r + i, fmaT(-om, y2[q].a, q2[q].a), fmaT(-om, y2[q].b, q2[q].b));
                cstore2(B.w + i, w0.c, w1.c);
                cstore2(tn + i, ta, tb);
            }
        }
    }
}

// The phases of chunk [c0, c1) that apply the working operator.
template <bool UNIT>
__device__ __forceinline__ void prun_chunk(const PSys& B, int kind, int c0, int c1, int zb, int tb, float alpha,
                                           float beta, float omega, int flag, float* sm) {
    double* const part = B.S.red.part;
    const bool staged = B.S.pair_blocks > 0 && B.S.m.nx <= kStageMaxNx;
    if (kind == PK_A && staged) {
        pstaged_a<UNIT>(B, B.z[zb], B.v[zb], B.z[zb ^ 1], B.v[zb ^ 1], B.t[tb], c0, c1, alpha, beta, omega, sm, part);
    } else if (kind == PK_B && staged && flag == 2) {
        pstaged_b<UNIT>(B, B.t[tb], B.v[zb], B.t[tb ^ 1], c0, c1, alpha, omega, sm);
    } else if (kind == PK_A) {
        pover_units<kPD, 10, 0u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kPD]) {
            pchunk_a<UNIT>(B, B.z[zb], B.v[zb], B.z[zb ^ 1], B.v[zb ^ 1], B.t[tb], u0, u1, alpha, beta, omega, acc);
        });
    } else if (kind == PK_B) {
        pover_units<1, 0, 0u>(c0, c1, part, [&](int u0, int u1, double (&)[1]) {
            if (flag == 2) pchunk_b<UNIT>(B, B.t[tb], B.v[zb], B.t[tb ^ 1], u0, u1, alpha, omega);
            else pchunk_b_half(B, u0, u1, alpha);
        });
    } else if (kind == PK_WS) {
        pover_units<1, 0, 0u>(c0, c1, part, [&](int u0, int u1, double (&)[1]) { pchunk_ws<UNIT>(B, u0, u1); });
    } else if (kind == PK_TZ) {
        pover_units<1, 0, 0u>(c0, c1, part,
                              [&](int u0, int u1, double (&)[1]) { pchunk_tz<UNIT>(B, B.t[tb], B.z[zb], u0, u1); });
    } else {  // PK_V
        pover_units<kPD, 5, 0u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kPD]) {
            pchunk_v<UNIT>(B, B.z[zb], B.v[zb], u0, u1, acc);
        });
    }
}

// ---------------------------------------------------------------- control block copies
__device__ __forceinline__ uint32_t pstate_fetch(const PState* src) {
    const int w = (int)threadIdx.x;
    return w < kPStateWords
               ? __hip_atomic_load(gbl(const_cast<uint32_t*>(reinterpret_cast<const uint32_t*>(src) + w)),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
               : 0u;
}
__device__ __forceinline__ void pstate_put(uint32_t word, PState& dst) {
    const int w = (int)threadIdx.x;
    if (w < kPStateWords) reinterpret_cast<uint32_t*>(&dst)[w] = word;
    __syncthreads();
}
__device__ __forceinline__ void pstate_store(PState* dst, const PState& src) {
    const int w = (int)threadIdx.x;
    if (w < kPStateWords) {
        __hip_atomic_store(gbl(reinterpret_cast<uint32_t*>(dst) + w), reinterpret_cast<const uint32_t*>(&src)[w],
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_stores();
    }
}

// The decisions at the end of a phase (thread 0, on the workgroup's copy of
// the control block).  Returns the next phase.
__device__ int pipe_complete(PState& P, int kind, const double (&tot)[kPD]) {
    State& st = P.st;
    PipeScalars& ps = P.ps;
    int next = PK_FINAL;
    bool inner_end = false;  // the iteration has stopped: the epilogue follows
    switch (kind) {
        case PK_S:
            tail_init(&st, tot[0], tot[1], st.rtol_o, st.max_total);
            st.bb_true = tot[2];
            st.scale = 1.0;
            ps = PipeScalars{};
            P.zb = P.tb = P.since = 0;
            if (st.done) inner_end = true;
            else next = PK_WS;
            break;
        case PK_R: next = PK_WS; break;
        case PK_WS: next = PK_TZ; break;
        case PK_TZ: next = PK_V; break;
        case PK_V:
            P.since = 0;
            tail_rr(&st, &ps, reinterpret_cast<const double(&)[5]>(tot));
            if (st.done) inner_end = true;
            else next = PK_A;
            break;
        case PK_A:
            tail_k1(&ps, reinterpret_cast<const double(&)[4]>(tot));
            tail_k2(&st, &ps, reinterpret_cast<const double(&)[6]>(tot[4]));
            P.zb ^= 1;
            if (ps.flag != 0) next = PK_B;  // the update is applied, stop or not
            else if (st.done) inner_end = true;
            else next = PK_R;  // a candidate stop: the true residual decides
            break;
        case PK_B:
            if (ps.flag == 2) P.tb ^= 1;
            P.since += 1;
            st.alpha = ps.alpha_next;
            ps.flag = 0;
            if (st.done) inner_end = true;
            else next = (ps.verify || P.since >= kReplace) ? PK_R : PK_A;
            break;
        case PK_X: next = st.xzero ? PK_FINAL : PK_RF; break;
        default:  // PK_RF
            (void)after_resid(st, reinterpret_cast<const double(&)[kMaxDots]>(tot));
            next = PK_FINAL;
    }
    if (inner_end) next = after_inner(st) == K_FINAL ? PK_FINAL : PK_X;
    if (next == PK_FINAL) st.final = 1;
    return next;
}

// ---------------------------------------------------------------- persistent kernel
// Workgroups claim (system, chunk) work items as in k_batched; the last chunk
// of a phase completes it.  A launch runs every system to its end.
__global__ __launch_bounds__(kThreads) void k_batched_pipe(const PSys* __restrict__ sys, const int* __restrict__ home,
                                                           BGlobal* glob, int nsys, long long spin_limit) {
    __shared__ int sh_sys, sh_chunk, sh_last, sh_stop, sh_direct;
    __shared__ uint32_t sh_seq, sh_nseq;
    __shared__ PState sh_p;
    // the staged phases' LDS
    __shared__ float sh_stage[kStageLds];
    // the search for work starts at the home system while it is active (as in k_batched)
    const int h0 = home[blockIdx.x];
    bool home_live = true;
    int s = h0;
    long long idle = 0;
    if (threadIdx.x == 0) sh_direct = 0;
    for (;;) {
        // a one-chunk phase's completer has already taken the next phase's chunk
        if (threadIdx.x == 0 && !sh_direct) {
            sh_sys = -1;
            if (home_live) s = h0;
            for (int tries = 0; tries < nsys; ++tries, s = (s + 1 == nsys) ? 0 : s + 1) {
                const int act = cload_i(&sys[s].ctl->active);
                const unsigned long long w0 =
                    __hip_atomic_load(gbl(&sys[s].ctl->claim), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (!act && s == h0) home_live = false;
                if (!act || (int)(w0 & 0xffffffffull) >= sys[s].nchunk) continue;
                const unsigned long long w = __hip_atomic_fetch_add(gbl(&sys[s].ctl->claim), 1ull, __ATOMIC_RELAXED,
                                                                    __HIP_MEMORY_SCOPE_AGENT);
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
                if (live <= 0 || err != 0) sh_sys = -2;
            }
        }
        __syncthreads();
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
        const PSys& B = sys[me];
        const SysView<float> S = B.S;
        PState* const pst = reinterpret_cast<PState*>(S.st);
        const int chunk = __builtin_amdgcn_readfirstlane(sh_chunk);
        const uint32_t seq = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh_seq);
        // resident (as in k_batched): the control block's current copy is sh_p
        const bool res = __builtin_amdgcn_readfirstlane(sh_direct) != 0;
        const int kind = (int)(seq & 15u);
        const int c0 = chunk * B.chunk;
        const int c1 = min(S.n, c0 + B.chunk);
        double* const part = S.red.part;
        if (kind == PK_S) {
            pover_units<kMaxDots, 3, 0u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kMaxDots]) {
                chunk_s_b(S, B.cf, B.b, B.x, u0, u1, acc);
            });
        } else if (kind == PK_R) {
            pover_units<1, 0, 0u>(c0, c1, part, [&](int u0, int u1, double (&)[1]) { pchunk_r(B, u0, u1); });
        } else if (kind == PK_X) {
            const double scale = res ? sh_p.st.scale : cload_d(&S.st->scale);
            const bool zero = (res ? sh_p.st.xzero : cload_i(&S.st->xzero)) != 0;
            pover_units<1, 0, 0u>(c0, c1, part, [&](int u0, int u1, double (&)[1]) {
                chunk_x_b(S, B.x, u0, u1, scale, zero);
            });
        } else if (kind == PK_RF) {
            pover_units<kMaxDots, 3, 4u>(c0, c1, part, [&](int u0, int u1, double (&acc)[kMaxDots]) {
                chunk_r_b(S, B.cf, B.b, B.x, u0, u1, false, acc);
            });
        } else {
            // the scalars and copy indices this phase reads, set by the last completion
            const int zb = __builtin_amdgcn_readfirstlane(res ? sh_p.zb : cload_i(&pst->zb));
            const int tb = __builtin_amdgcn_readfirstlane(res ? sh_p.tb : cload_i(&pst->tb));
            const int flag = __builtin_amdgcn_readfirstlane(res ? sh_p.ps.flag : cload_i(&pst->ps.flag));
            const float alpha = (float)(res ? sh_p.st.alpha : cload_d(&S.st->alpha));
            const float beta = (float)(res ? sh_p.st.beta : cload_d(&S.st->beta));
            const float omega = (float)(res ? sh_p.st.omega : cload_d(&S.st->omega));
            if (S.unit) prun_chunk<true>(B, kind, c0, c1, zb, tb, alpha, beta, omega, flag, sh_stage);
            else prun_chunk<false>(B, kind, c0, c1, zb, tb, alpha, beta, omega, flag, sh_stage);
        }
        // every thread's stores (the unit sums included) reach memory before the
        // chunk is counted done
        wait_stores();
        __syncthreads();
        if (threadIdx.x == 0) {
            sh_direct = 0;
            if (B.nchunk == 1) {
                sh_last = 1;  // a phase of one chunk: no count
            } else {
                const uint32_t t =
                    __hip_atomic_fetch_add(gbl(&B.ctl->done_cnt), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sh_last = (t == (uint32_t)(B.nchunk - 1));
            }
        }
        __syncthreads();
        if (!sh_last) continue;
        // this workgroup completes the phase (a resident system's LDS copy is current)
        const uint32_t pw = res ? 0u : pstate_fetch(pst);
        const int nunit = (S.n + kUnitCells - 1) / kUnitCells;
        double tot[kPD] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (kind == PK_A) psum_units<10, 0u>(part, nunit, tot);
        else if (kind == PK_V) psum_units<5, 0u>(part, nunit, tot);
        else if (kind == PK_S) psum_units<3, 0u>(part, nunit, tot);
        else if (kind == PK_RF) psum_units<3, 4u>(part, nunit, tot);
        if (!res) pstate_put(pw, sh_p);
        else __syncthreads();
        if (threadIdx.x == 0) {
            const int next = pipe_complete(sh_p, kind, tot);
            sh_stop = next == PK_FINAL ? 1 : 0;
            sh_nseq = pseq_next(seq, next == PK_FINAL ? PK_A : next);
        }
        __syncthreads();
        // a system that goes on resident keeps its control block in LDS only
        const bool stay = !sh_stop && B.nchunk == 1;
        if (!stay) {
            pstate_store(pst, sh_p);
            __syncthreads();  // every word of the control block has reached memory
        }
        if (threadIdx.x == 0) {
            if (!stay) __hip_atomic_store(gbl(&B.ctl->done_cnt), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t nseq = sh_nseq;
            if (sh_stop) {
                cstore_i(&B.ctl->active, 0);
                __hip_atomic_store(gbl(&B.ctl->claim), ((unsigned long long)nseq << 32) | (unsigned)B.nchunk,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                wait_stores();
                __hip_atomic_fetch_add(&glob->active, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else if (stay) {
                // the next phase's only chunk is taken here (as in k_batched); the
                // claim word, published on the way in with its counter exhausted,
                // is not written again until the system stops
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

// Arms a pipelined launch: every unfinished system takes part.
__global__ __launch_bounds__(kThreads) void k_batched_pipe_arm(const PSys* sys, BGlobal* glob, int nsys) {
    __shared__ int count;
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < nsys; s += kThreads) {
        const bool fin = sys[s].S.st->final != 0;
        const uint32_t seq = (uint32_t)(sys[s].ctl->claim >> 32);  // rewinds the chunk counter
        sys[s].ctl->claim = (unsigned long long)seq << 32;
        sys[s].ctl->active = fin ? 0 : 1;
        sys[s].ctl->budget = 0;
        sys[s].ctl->done_cnt = 0u;
        if (!fin) atomicAdd(&count, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        glob->active = count;
        glob->error = 0;
        glob->t0 = wall_clock64();
        glob->slice = 0;
    }
}

// ---------------------------------------------------------------- host
// A system's slice: the classical FP32 layout (its State space holds the
// PState), then z, v and t twice each and w.
static size_t pipe_batch_bytes(const Layout& Lo) {
    return align256(Lo.bytes) + 7 * align256(Lo.n * sizeof(float));
}

// Tables: [BGlobal][PSys x cap][State* x cap][State x cap][JobStart x cap][home x kMaxPersistentGrid].
static size_t pt_sys() { return align256(sizeof(BGlobal)); }
static size_t pt_sptr(int cap) { return pt_sys() + align256((size_t)cap * sizeof(PSys)); }
static size_t pt_gather(int cap) { return pt_sptr(cap) + align256((size_t)cap * sizeof(State*)); }
static size_t pt_jobs(int cap) { return pt_gather(cap) + align256((size_t)cap * sizeof(State)); }
static size_t pt_home(int cap) { return pt_jobs(cap) + align256((size_t)cap * sizeof(JobStart)); }
static size_t pipe_table_bytes(int cap) { return pt_home(cap) + align256((size_t)kMaxPersistentGrid * sizeof(int)); }

static PSys psys_entry(const EngineJob& j, const s7_options& o, int chunk) {
    PSys P;
    std::memset(&P, 0, sizeof(P));
    P.S = make_view<float>(j.d, j.lo, o.jacobi, j.ws);
    P.ctl = reinterpret_cast<BCtl*>(j.ws + j.lo.off_ctl);
    const size_t base = align256(j.lo.bytes), span = align256(j.lo.n * sizeof(float));
    auto vec = [&](int k) { return reinterpret_cast<float*>(j.ws + base + (size_t)k * span); };
    P.z[0] = vec(0), P.z[1] = vec(1), P.v[0] = vec(2), P.v[1] = vec(3), P.t[0] = vec(4), P.t[1] = vec(5);
    P.w = vec(6);
    P.nchunk = (int)((j.lo.n + chunk - 1) / chunk);
    P.chunk = chunk;
    for (int a = 0; a < 7; ++a) P.cf.c[a] = j.coef[a];
    P.b = j.b;
    P.x = j.x;
    return P;
}

// Runs the jobs (workspace slices filled in) in one pipelined launch.
static int run_pipe_batch(std::vector<EngineJob*>& jobs, char* tables, int cap, const s7_options& o,
                          hipStream_t s) {
    const int nsys = (int)jobs.size();
    if (nsys == 0) return S7_OK;
    for (EngineJob* j : jobs) {
        // the unit sums use kPD values per unit of the classical partial space
        const size_t nunit = (j->lo.n + kUnitCells - 1) / kUnitCells;
        if (nunit * kPD * sizeof(double) > j->lo.off_gpart - j->lo.off_part) {
            set_error("pipelined batch: partial space too small");
            return S7_EHIP;
        }
    }
    // 1) job starts: working coefficient copies, State, first phase S
    std::vector<JobStart> starts;
    std::vector<State*> sptr;
    size_t max_n = 1;
    for (EngineJob* j : jobs) {
        JobStart J = job_entry(*j, o);
        J.first = PK_S;
        starts.push_back(J);
        sptr.push_back(reinterpret_cast<State*>(j->ws + j->lo.off_state));
        max_n = std::max(max_n, j->lo.n);
    }
    JobStart* dj = reinterpret_cast<JobStart*>(tables + pt_jobs(cap));
    S7_HIP(hipMemcpyAsync(dj, starts.data(), starts.size() * sizeof(JobStart), hipMemcpyHostToDevice, s));
    S7_HIP(hipMemcpyAsync(tables + pt_sptr(cap), sptr.data(), sptr.size() * sizeof(State*), hipMemcpyHostToDevice,
                          s));
    const int gx = (int)std::min<size_t>(128, (max_n + kThreads - 1) / kThreads);
    for (int k = 0; k < nsys; k += 65535) {
        const unsigned ny = (unsigned)std::min(65535, nsys - k);
        hipLaunchKernelGGL(k_jobs_start, dim3(gx, ny), dim3(kThreads), 0, s, (const JobStart*)(dj + k));
    }
    S7_CHECK_LAUNCH();
    // 2) one persistent launch runs every job to its end; the kernel keeps three
    // workgroups resident per CU (its register count allows three wavefronts per SIMD)
    const int grid_cap = 768;
    const std::vector<int> chunks = launch_chunks(jobs, chunk_cells_of(o), grid_cap, o.chunk_cells == 0);
    std::vector<PSys> table;
    long long total_chunks = 0;
    for (int i = 0; i < nsys; ++i) {
        table.push_back(psys_entry(*jobs[i], o, chunks[i]));
        total_chunks += table.back().nchunk;
    }
    BGlobal* glob = reinterpret_cast<BGlobal*>(tables);
    PSys* dsys = reinterpret_cast<PSys*>(tables + pt_sys());
    S7_HIP(hipMemcpyAsync(dsys, table.data(), table.size() * sizeof(PSys), hipMemcpyHostToDevice, s));
    const int grid = (int)std::max(1LL, std::min<long long>(total_chunks, grid_cap));
    // home systems in proportion to cell count, as for the classical kernel
    std::vector<double> cells;
    for (const PSys& b : table) cells.push_back((double)b.S.n);
    const std::vector<int> home = weighted_homes(cells, grid);
    int* dhome = reinterpret_cast<int*>(tables + pt_home(cap));
    S7_HIP(hipMemcpyAsync(dhome, home.data(), home.size() * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_batched_pipe_arm, dim3(1), dim3(kThreads), 0, s, (const PSys*)dsys, glob, nsys);
    hipLaunchKernelGGL(k_batched_pipe, dim3(grid), dim3(kThreads), 0, s, (const PSys*)dsys, (const int*)dhome, glob,
                       nsys, (long long)5000000);
    S7_CHECK_LAUNCH();
    BGlobal hg;
    S7_HIP(hipMemcpyAsync(&hg, glob, sizeof(hg), hipMemcpyDeviceToHost, s));
    S7_HIP(hipStreamSynchronize(s));
    if (hg.error) {
        set_error("pipelined batched launch: a workgroup exceeded its wait bound");
        return S7_EHIP;
    }
    // 3) every job's State, in one transfer
    State* gather = reinterpret_cast<State*>(tables + pt_gather(cap));
    hipLaunchKernelGGL(k_gather_states, dim3((nsys * (int)(sizeof(State) / 8) + kThreads - 1) / kThreads),
                       dim3(kThreads), 0, s, (State* const*)(tables + pt_sptr(cap)), gather, nsys);
    S7_CHECK_LAUNCH();
    std::vector<State> h((size_t)nsys);
    S7_HIP(hipMemcpyAsync(h.data(), gather, (size_t)nsys * sizeof(State), hipMemcpyDeviceToHost, s));
    S7_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nsys; ++i) {
        if (!h[i].final) {
            set_error("pipelined batched launch: system %d did not finish", i);
            return S7_EHIP;
        }
        finish_job(*jobs[i], h[i]);
        jobs[i]->info.schedule = 4;
    }
    return S7_OK;
}

}  // namespace s7

extern "C" {

size_t s7_batched_workspace_bytes_pipelined(int32_t nsys, const s7_dims* d, const s7_options* opt) {
    if (nsys < 1 || !d) return 0;
    s7_options o;
    options_or_default(opt, o);
    size_t total = align256(pipe_table_bytes(nsys));
    for (int i = 0; i < nsys; ++i) {
        if (!dims_ok(d[i])) return 0;
        total += align256(pipe_batch_bytes(make_layout(d[i], S7_FP32, o)));
    }
    return total;
}

int s7_bicgstab_solve_batched_pipelined(int32_t nsys, const s7_dims* d, const float* const* coef,
                                        const double* const* b, double* const* x, const double* rtol,
                                        const int32_t* max_iter, void* ws, size_t ws_bytes, const s7_options* opt,
                                        s7_info* info, void* stream) {
    clear_error();
    s7_options o;
    options_or_default(opt, o);
    if (nsys < 1 || !d || !coef || !b || !x || !rtol || !max_iter || !ws || ((uintptr_t)ws & 255u) != 0) {
        set_error("s7_bicgstab_solve_batched_pipelined: invalid argument");
        return S7_EINVAL;
    }
    for (int i = 0; i < nsys; ++i) {
        bool ok = dims_ok(d[i]) && b[i] && x[i] && rtol[i] > 0.0 && max_iter[i] >= 0;
        for (int a = 0; a < 7 && ok; ++a) ok = coef[7 * i + a] != nullptr;
        if (!ok) {
            set_error("s7_bicgstab_solve_batched_pipelined: invalid argument for system %d", i);
            return S7_EINVAL;
        }
    }
    const size_t need = s7_batched_workspace_bytes_pipelined(nsys, d, &o);
    if (ws_bytes < need) {
        set_error("s7_bicgstab_solve_batched_pipelined: workspace too small (%zu < %zu)", ws_bytes, need);
        return S7_EINVAL;
    }
    char* w = (char*)ws;
    const hipStream_t s = (hipStream_t)stream;
    const long long split = split_cells_of(o);
    std::vector<EngineJob> jobs((size_t)nsys);
    std::vector<EngineJob*> shared;
    size_t off = align256(pipe_table_bytes(nsys));
    const double t0 = now_ms();
    for (int i = 0; i < nsys; ++i) {
        EngineJob& j = jobs[i];
        std::memset(&j, 0, sizeof(j));
        j.d = d[i];
        for (int a = 0; a < 7; ++a) j.coef[a] = coef[7 * i + a];
        j.b = b[i];
        j.x = x[i];
        j.rtol = rtol[i];
        j.max_iter = max_iter[i];
        j.prec = S7_FP32;
        j.ws = w + off;
        j.lo = make_layout(d[i], S7_FP32, o);
        j.ws_bytes = pipe_batch_bytes(j.lo);
        j.t_start_ms = t0;
        j.op = OP_7PT;
        off += align256(j.ws_bytes);
        if ((long long)d[i].nx * d[i].ny * d[i].nz < split) shared.push_back(&j);
    }
    int rc = run_pipe_batch(shared, w, nsys, o, s);
    if (rc) return rc;
    int worst = S7_OK;
    for (int i = 0; i < nsys; ++i) {
        EngineJob& j = jobs[i];
        if ((long long)d[i].nx * d[i].ny * d[i].nz >= split) {
            // a large system alone, on the multi-kernel pipelined path in its slice
            rc = s7_bicgstab_solve_pipelined(j.d, j.coef, j.b, j.x, j.rtol, j.max_iter, j.ws, j.ws_bytes, &o,
                                             &j.info, stream);
            if (rc < 0) return rc;
        }
        if (info) info[i] = j.info;
        if (j.info.status > worst) worst = j.info.status;
    }
    return worst;
}

}  // extern "C"
