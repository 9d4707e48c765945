// Design probe (diagnostic): the P2 pass of the three-pass iteration,
// q = r - alpha s formed on the fly and y = A q with its five sums (Algorithm 1,
// the stencil of section IV "SpMV (3D)"), in the alternative kernel designs
// that were measured against the one the solver uses.  Each design computes the
// same y, term for term in the order of apply7 (unit diagonal, then w, e, s,
// n, b, t by FMA), so their outputs agree bit for bit; only the order of the
// FP64 sums differs.  The designs:
//   0  flat cell pairs: every neighbour of r and s loaded from memory;
//   1  one-plane tiles: a workgroup stages q over 2048 consecutive cells and one
//      row either side in LDS, the z neighbours from memory (the solver's
//      staged form), in plain or band-per-XCD tile order;
//   2  two-plane tiles: the same xy range of planes 2k and 2k+1 staged
//      together, so the z neighbour between them comes from LDS;
//   3  z-march: a workgroup walks H planes of one 2048-cell in-plane tile, q of
//      the planes below and above in registers, the current plane (tile and one
//      row either side) in a double-buffered LDS ring, the next plane prefetched.
// Coefficients are unit-diagonal working copies with the outward links zeroed
// on the faces (as the solver's Jacobi-scaled copies).  Limits: nx a multiple
// of 8 and at most 1024.
#include <algorithm>

#include "s7_host.hpp"

namespace s7 {
namespace {

typedef float q4 __attribute__((ext_vector_type(4)));
typedef float q2 __attribute__((ext_vector_type(2)));

constexpr int kT = 2048;      // in-plane cells per tile
constexpr int kNxMax = 1024;  // widest row the LDS layouts hold

struct PArr {
    const float *r, *s, *rh;
    float* y;
    const float* c[7];  // c[1..6]: w, e, s, n, b, t
    double* part;       // five sums per workgroup
};

__device__ __forceinline__ void sums_pair(double (&acc)[5], bool own, float qa, float qb, float ya, float yb, F2 rh) {
    const double y0 = own ? (double)ya : 0.0, y1 = own ? (double)yb : 0.0;
    const double q0 = own ? (double)qa : 0.0, q1 = own ? (double)qb : 0.0;
    acc[0] += fma(q1, y1, q0 * y0);
    acc[1] += fma(y1, y1, y0 * y0);
    acc[2] += fma(q1, q1, q0 * q0);
    acc[3] += fma((double)rh.b, q1, (double)rh.a * q0);
    acc[4] += fma((double)rh.b, y1, (double)rh.a * y0);
}

// Design 0.
__global__ __launch_bounds__(kThreads) void kd_pairs(PArr A, Mesh m, int n, float alpha) {
    const Cell c = cell2_at(blockIdx.x * kThreads + threadIdx.x, m, n);
    Nbr<float> r0, r1, s0, s1;
    load_nbr2(A.r, c, r0, r1);
    load_nbr2(A.s, c, s0, s1);
    Coefs<float, true> k0, k1;
    load_coefs2_nt<float, true>(A.c, c.idx, k0, k1);
    const F2 rh = ld2_nt(A.rh + c.idx);
    auto qof = [&](const Nbr<float>& r, const Nbr<float>& s) {
        return Nbr<float>{fmaT(-alpha, s.c, r.c), fmaT(-alpha, s.w, r.w), fmaT(-alpha, s.e, r.e),
                          fmaT(-alpha, s.s, r.s), fmaT(-alpha, s.n, r.n), fmaT(-alpha, s.b, r.b),
                          fmaT(-alpha, s.t, r.t)};
    };
    const Nbr<float> q0 = qof(r0, s0), q1 = qof(r1, s1);
    const float y0 = apply7<float, float, true, false>(k0, q0, c);
    const float y1 = apply7<float, float, true, false>(k1, q1, c);
    if (c.own) st2_nt(A.y + c.idx, y0, y1);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    sums_pair(acc, c.own, q0.c, q1.c, y0, y1, rh);
    reduce_store<5>(acc, A.part, blockIdx.x);
}

// q over [lo, lo + 4 cnt4) into qs, zero outside [0, n); lo is a multiple of 4.
__device__ __forceinline__ void stage_q4(const PArr& A, float alpha, int lo, int cnt4, int n, float* qs) {
    for (int v = (int)threadIdx.x; v < cnt4; v += kThreads) {
        const int g = lo + 4 * v;
        q4 q = q4{0.f, 0.f, 0.f, 0.f};
        if (g >= 0 && g + 3 < n) {
            const q4 rv = *reinterpret_cast<const q4*>(A.r + g);
            const q4 sv = *reinterpret_cast<const q4*>(A.s + g);
            q = q4{fmaT(-alpha, sv.x, rv.x), fmaT(-alpha, sv.y, rv.y), fmaT(-alpha, sv.z, rv.z),
                   fmaT(-alpha, sv.w, rv.w)};
        }
        *reinterpret_cast<q4*>(&qs[4 * v]) = q;
    }
}

__device__ __forceinline__ F2 q_mem(const PArr& A, int i, float alpha) {
    const F2 r = ld2(A.r + i), s = ld2(A.s + i);
    return F2{fmaT(-alpha, s.a, r.a), fmaT(-alpha, s.b, r.b)};
}

// y and the sums of the pair at idx: centre, x and y neighbours from the staged
// plane qs (L = the pair's index in it), z neighbours qb and qt.
__device__ __forceinline__ void pair_from_lds(const PArr& A, const float* qs, int L, int nx, int idx, bool own,
                                              F2 qb, F2 qt, double (&acc)[5]) {
    const q2 qc = *reinterpret_cast<const q2*>(&qs[L]);
    const q2 qsn = *reinterpret_cast<const q2*>(&qs[L - nx]);
    const q2 qno = *reinterpret_cast<const q2*>(&qs[L + nx]);
    const float qw = qs[L - 1], qe = qs[L + 2];
    Coefs<float, true> k0, k1;
    load_coefs2_nt<float, true>(A.c, idx, k0, k1);
    const F2 rh = ld2_nt(A.rh + idx);
    float y0 = qc.x, y1 = qc.y;
    y0 = fmaT(k0.a[1], qw, y0);
    y0 = fmaT(k0.a[2], qc.y, y0);
    y0 = fmaT(k0.a[3], qsn.x, y0);
    y0 = fmaT(k0.a[4], qno.x, y0);
    y0 = fmaT(k0.a[5], qb.a, y0);
    y0 = fmaT(k0.a[6], qt.a, y0);
    y1 = fmaT(k1.a[1], qc.x, y1);
    y1 = fmaT(k1.a[2], qe, y1);
    y1 = fmaT(k1.a[3], qsn.y, y1);
    y1 = fmaT(k1.a[4], qno.y, y1);
    y1 = fmaT(k1.a[5], qb.b, y1);
    y1 = fmaT(k1.a[6], qt.b, y1);
    if (own) st2_nt(A.y + idx, y0, y1);
    sums_pair(acc, own, qc.x, qc.y, y0, y1, rh);
}

// Design 1: tile t covers cells [t kT, (t + 1) kT).
__global__ __launch_bounds__(kThreads) void kd_tile1(PArr A, Mesh m, int n, float alpha, int nb, int run) {
    __shared__ float qs[kT + 2 * kNxMax + 8];
    const int nx = m.nx, plane = nx * m.ny;
    const int t = xcd_tile(blockIdx.x, nb, run);
    const int c0 = t * kT, lo = c0 - nx;
    stage_q4(A, alpha, lo, (kT + 2 * nx) / 4, n, qs);
    __syncthreads();
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int u = 0; u < kT / (2 * kThreads); ++u) {
        const int cell = c0 + 2 * (u * kThreads + (int)threadIdx.x);
        const bool own = cell < n;
        const int idx = own ? cell : n - 2;
        const int k = div_rcp(idx, plane, m.rplane);
        const int db = k > 0 ? -plane : 0, dt = k < m.nz - 1 ? plane : 0;
        pair_from_lds(A, qs, idx - lo, nx, idx, own, q_mem(A, idx + db, alpha), q_mem(A, idx + dt, alpha), acc);
    }
    reduce_store<5>(acc, A.part, t);
}

// Design 2: tile t = (pair of planes kk, xy tile j) covers the in-plane cells
// [j kT, min((j + 1) kT, P)) of planes 2 kk and 2 kk + 1.
__global__ __launch_bounds__(kThreads) void kd_tile2(PArr A, Mesh m, int n, float alpha, int nb, int run,
                                                     int tpp) {
    constexpr int LB = kT + 2 * kNxMax + 8;
    __shared__ float qs[2][LB];
    const int nx = m.nx, P = nx * m.ny, nz = m.nz;
    const int t = xcd_tile(blockIdx.x, nb, run);
    const int kk = t / tpp, j = t - kk * tpp;
    const int k0 = 2 * kk;
    const bool two = k0 + 1 < nz;
    const int x0 = j * kT, x1 = min(P, x0 + kT);
    const int cnt4 = (x1 - x0 + 2 * nx + 3) / 4;
    stage_q4(A, alpha, k0 * P + x0 - nx, cnt4, n, qs[0]);
    if (two) stage_q4(A, alpha, (k0 + 1) * P + x0 - nx, cnt4, n, qs[1]);
    __syncthreads();
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int a = 0; a < 2; ++a) {
        if (a == 1 && !two) break;
        const int k = k0 + a;
        const int base = k * P;
        for (int u = 0; u < kT / (2 * kThreads); ++u) {
            const int xy = x0 + 2 * (u * kThreads + (int)threadIdx.x);
            const bool own = xy < x1;
            const int xyc = own ? xy : x0;
            const int idx = base + xyc;
            const int L = xyc - x0 + nx;
            F2 qb, qt;
            if (a == 0) {
                qb = q_mem(A, k > 0 ? idx - P : idx, alpha);
                if (two) {
                    const q2 v = *reinterpret_cast<const q2*>(&qs[1][L]);
                    qt = F2{v.x, v.y};
                } else {
                    qt = q_mem(A, idx, alpha);
                }
            } else {
                const q2 v = *reinterpret_cast<const q2*>(&qs[0][L]);
                qb = F2{v.x, v.y};
                qt = q_mem(A, k < nz - 1 ? idx + P : idx, alpha);
            }
            pair_from_lds(A, qs[a], L, nx, idx, own, qb, qt, acc);
        }
    }
    reduce_store<5>(acc, A.part, t);
}

__device__ __forceinline__ q4 q_of4(float alpha, q4 r, q4 s) {
    return q4{fmaT(-alpha, s.x, r.x), fmaT(-alpha, s.y, r.y), fmaT(-alpha, s.z, r.z), fmaT(-alpha, s.w, r.w)};
}
__device__ __forceinline__ q4 ld4(const float* p) { return *reinterpret_cast<const q4*>(p); }
__device__ __forceinline__ q4 ld4nt(const float* p) { return __builtin_nontemporal_load(reinterpret_cast<const q4*>(p)); }

// Design 3: workgroup b takes in-plane tile b mod tpp of planes [k0, k0 + H)
// with k0 = (b / tpp) H; each thread owns two quads of the tile.  The ring
// holds [one row before | tile | one row after] of the current plane.
__global__ __launch_bounds__(kThreads) void kd_zmarch(PArr A, Mesh m, float alpha, int tpp, int H) {
    constexpr int LB = kT + 2 * kNxMax;
    __shared__ float ring[2][LB];
    const int nx = m.nx, P = nx * m.ny, nz = m.nz;
    const int tile = (int)blockIdx.x % tpp, zb = (int)blockIdx.x / tpp;
    const int c0 = tile * kT;
    const int k0 = zb * H, k1 = min(k0 + H, nz);
    const int tid = (int)threadIdx.x;
    const int hq = nx / 2;  // halo quads of a plane: one row either side
    int oo[2], ho[2], hp[2];
    bool ov[2], hv[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        oo[u] = c0 + 4 * (tid + kThreads * u);
        ov[u] = oo[u] < P;
        const int h = tid + kThreads * u;
        const bool has = h < hq;
        const int off = h < hq / 2 ? c0 - nx + 4 * h : c0 + kT + 4 * (h - hq / 2);
        hv[u] = has && off >= 0 && off < P;
        ho[u] = hv[u] ? off : 0;
        hp[u] = !has ? -1 : (h < hq / 2 ? 4 * h : nx + kT + 4 * (h - hq / 2));
    }
    auto own_q = [&](int k, q4 (&q)[2]) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            q[u] = q4{0.f, 0.f, 0.f, 0.f};
            if (k >= 0 && k < nz && ov[u]) {
                const size_t g = (size_t)k * P + oo[u];
                q[u] = q_of4(alpha, ld4(A.r + g), ld4(A.s + g));
            }
        }
    };
    auto halo_q = [&](int k, q4 (&q)[2]) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            q[u] = q4{0.f, 0.f, 0.f, 0.f};
            if (k >= 0 && k < nz && hv[u]) {
                const size_t g = (size_t)k * P + ho[u];
                q[u] = q_of4(alpha, ld4(A.r + g), ld4(A.s + g));
            }
        }
    };
    auto put = [&](int b, const q4 (&own)[2], const q4 (&hal)[2]) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            *reinterpret_cast<q4*>(&ring[b][nx + 4 * (tid + kThreads * u)]) = own[u];
            if (hp[u] >= 0) *reinterpret_cast<q4*>(&ring[b][hp[u]]) = hal[u];
        }
    };
    q4 qm[2], qc[2], qp[2], hn[2];
    own_q(k0 - 1, qm);
    own_q(k0, qc);
    {
        q4 h0[2];
        halo_q(k0, h0);
        put(0, qc, h0);
    }
    own_q(k0 + 1, qp);
    halo_q(k0 + 1, hn);
    __syncthreads();
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = k0; k < k1; ++k) {
        const int b = (k - k0) & 1;
        // plane k + 1 into the other ring half, plane k + 2 prefetched, while plane k is computed
        q4 qn[2], hnn[2];
        const bool more = k + 1 < k1;
        if (more) {
            own_q(k + 2, qn);
            halo_q(k + 2, hnn);
            put(b ^ 1, qp, hn);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (!ov[u]) continue;
            const int L = nx + 4 * (tid + kThreads * u);
            const size_t g = (size_t)k * P + oo[u];
            const q4 sn = *reinterpret_cast<const q4*>(&ring[b][L - nx]);
            const q4 nn = *reinterpret_cast<const q4*>(&ring[b][L + nx]);
            const float w = ring[b][L - 1], e = ring[b][L + 4];
            q4 cf[7];
#pragma unroll
            for (int a = 1; a < 7; ++a) cf[a] = ld4nt(A.c[a] + g);
            const q4 rh = ld4nt(A.rh + g);
            const float qcv[4] = {qc[u].x, qc[u].y, qc[u].z, qc[u].w};
            const float wv[4] = {w, qc[u].x, qc[u].y, qc[u].z};
            const float ev[4] = {qc[u].y, qc[u].z, qc[u].w, e};
            const float sv[4] = {sn.x, sn.y, sn.z, sn.w};
            const float nv[4] = {nn.x, nn.y, nn.z, nn.w};
            const float bv[4] = {qm[u].x, qm[u].y, qm[u].z, qm[u].w};
            const float tv[4] = {qp[u].x, qp[u].y, qp[u].z, qp[u].w};
            const float rhv[4] = {rh.x, rh.y, rh.z, rh.w};
            float y[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float a = qcv[j];
                a = fmaT(cf[1][j], wv[j], a);
                a = fmaT(cf[2][j], ev[j], a);
                a = fmaT(cf[3][j], sv[j], a);
                a = fmaT(cf[4][j], nv[j], a);
                a = fmaT(cf[5][j], bv[j], a);
                a = fmaT(cf[6][j], tv[j], a);
                y[j] = a;
                const double yd = a, qd = qcv[j];
                acc[0] = fma(qd, yd, acc[0]);
                acc[1] = fma(yd, yd, acc[1]);
                acc[2] = fma(qd, qd, acc[2]);
                acc[3] = fma((double)rhv[j], qd, acc[3]);
                acc[4] = fma((double)rhv[j], yd, acc[4]);
            }
            __builtin_nontemporal_store(q4{y[0], y[1], y[2], y[3]}, reinterpret_cast<q4*>(A.y + g));
        }
        if (more) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                qm[u] = qc[u];
                qc[u] = qp[u];
                qp[u] = qn[u];
                hn[u] = hnn[u];
            }
        }
        __syncthreads();
    }
    reduce_store<5>(acc, A.part, blockIdx.x);
}

// Workgroups of a design's launch (0 for an unknown design).
long long design_grid(int kind, int param, const Mesh& m, int n) {
    const int P = m.nx * m.ny;
    const int tpp = (P + kT - 1) / kT;
    switch (kind) {
        case 0: return ((long long)n / 2 + kThreads - 1) / kThreads;
        case 1: return ((long long)n + kT - 1) / kT;
        case 2: return (long long)tpp * ((m.nz + 1) / 2);
        case 3: return param >= 1 ? (long long)tpp * ((m.nz + param - 1) / param) : 0;
        default: return 0;
    }
}

void design_launch(int kind, int param, const PArr& A, const Mesh& m, int n, float alpha, hipStream_t s) {
    const int P = m.nx * m.ny;
    const int tpp = (P + kT - 1) / kT;
    const int grid = (int)design_grid(kind, param, m, n);
    // band-per-XCD tile order: runs of an eighth of a plane's tiles
    const int run = param == 0 ? std::max(1, tpp / 8) : 1;
    if (kind == 0) hipLaunchKernelGGL(kd_pairs, dim3(grid), dim3(kThreads), 0, s, A, m, n, alpha);
    else if (kind == 1) hipLaunchKernelGGL(kd_tile1, dim3(grid), dim3(kThreads), 0, s, A, m, n, alpha, grid, run);
    else if (kind == 2)
        hipLaunchKernelGGL(kd_tile2, dim3(grid), dim3(kThreads), 0, s, A, m, n, alpha, grid, run, tpp);
    else hipLaunchKernelGGL(kd_zmarch, dim3(grid), dim3(kThreads), 0, s, A, m, alpha, tpp, param);
}

}  // namespace
}  // namespace s7

using namespace s7;

extern "C" {

size_t s7_p2_design_part_bytes(int32_t kind, int32_t param, s7_dims d) {
    if (!dims_ok(d)) return 0;
    const Mesh m = make_mesh(d.nx, d.ny, d.nz);
    return (size_t)design_grid(kind, param, m, d.nx * d.ny * d.nz) * 5 * sizeof(double);
}

int s7_p2_design_probe(int32_t kind, int32_t param, s7_dims d, const float* const coef[6], const float* r,
                       const float* s, const float* rhat, float alpha, float* y, double* part, size_t part_bytes,
                       int32_t reps, float* ms, void* stream) {
    clear_error();
    if (!dims_ok(d) || d.nx % 8 != 0 || d.nx > kNxMax || kind < 0 || kind > 3 || (kind == 3 && param < 1) ||
        ((kind == 1 || kind == 2) && param != 0 && param != 1) || !coef || !r || !s || !rhat || !y || !part ||
        reps < 1 || !ms) {
        set_error("s7_p2_design_probe: invalid argument");
        return S7_EINVAL;
    }
    for (int a = 0; a < 6; ++a) {
        if (!coef[a] || ((uintptr_t)coef[a] & 15u) != 0) {
            set_error("s7_p2_design_probe: coefficient %d missing or not 16-byte aligned", a);
            return S7_EINVAL;
        }
    }
    if (((uintptr_t)r | (uintptr_t)s | (uintptr_t)rhat | (uintptr_t)y) & 15u) {
        set_error("s7_p2_design_probe: arrays must be 16-byte aligned");
        return S7_EINVAL;
    }
    const size_t need = s7_p2_design_part_bytes(kind, param, d);
    if (part_bytes < need) {
        set_error("s7_p2_design_probe: partial buffer too small (%zu < %zu)", part_bytes, need);
        return S7_EINVAL;
    }
    const Mesh m = make_mesh(d.nx, d.ny, d.nz);
    const int n = d.nx * d.ny * d.nz;
    PArr A;
    A.r = r;
    A.s = s;
    A.rh = rhat;
    A.y = y;
    A.c[0] = nullptr;
    for (int a = 0; a < 6; ++a) A.c[a + 1] = coef[a];
    A.part = part;
    const hipStream_t st = (hipStream_t)stream;
    design_launch(kind, param, A, m, n, alpha, st);  // warm-up
    S7_CHECK_LAUNCH();
    hipEvent_t e0, e1;
    S7_HIP(hipEventCreate(&e0));
    S7_HIP(hipEventCreate(&e1));
    int rc = S7_OK;
    if (hipEventRecord(e0, st) != hipSuccess) rc = S7_EHIP;
    for (int k = 0; k < reps && rc == S7_OK; ++k) design_launch(kind, param, A, m, n, alpha, st);
    if (rc == S7_OK && (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
                        hipEventSynchronize(e1) != hipSuccess))
        rc = S7_EHIP;
    float t = 0.f;
    if (rc == S7_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = S7_EHIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        set_error("s7_p2_design_probe: launch or timing failed");
        return rc;
    }
    *ms = t / (float)reps;
    return S7_OK;
}

}  // extern "C"
