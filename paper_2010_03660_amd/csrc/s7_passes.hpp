// The kernels of the single-system iteration's passes: P1 (s = A p), P2 (the
// four-pass P2a and P2b, and the three-pass P2 that forms q on the fly), P3 (the
// x, r and p updates), each in its flat, cell-pair and LDS-staged forms, and the
// finishing kernel of a split grid sum.  Every pass ends in the device-side
// scalar step of Algorithm 1 that its sums feed (s7_device.hpp).  Included by
// the solver translation unit (s7_single.hip) only.
#pragma once

#include "s7_device.hpp"

namespace s7 {

// Second half of a split grid sum (see Red), followed by the scalar step of the
// pass whose partials it sums.
enum FinishKind { FIN_P1 = 1, FIN_P2 = 2, FIN_INIT = 3, FIN_RESID = 4, FIN_P2F = 5 };

template <int ND, unsigned MAXMASK, int KIND>
__global__ __launch_bounds__(kThreads) void k_finish(Red red, int nblocks, State* st, double tol,
                                                     int max_iter) {
    if ((KIND == FIN_P1 || KIND == FIN_P2 || KIND == FIN_P2F) && st->done) return;
    double tot[ND];
    if (!finish_split<ND, MAXMASK>(red, nblocks, tot) || threadIdx.x != 0) return;
    if constexpr (KIND == FIN_P1) {
        tail_p1(st, reinterpret_cast<double(&)[1]>(tot));
    } else if constexpr (KIND == FIN_P2) {
        tail_p2(st, reinterpret_cast<double(&)[4]>(tot));
    } else if constexpr (KIND == FIN_P2F) {
        tail_p2f(st, reinterpret_cast<double(&)[5]>(tot));
    } else if constexpr (KIND == FIN_INIT) {
        tail_init(st, tot[0], tot[1], tol, max_iter);
        st->bb_true = tot[2];
        st->scale = 1.0;
    } else {
        st->bb_true = tot[0];
        st->rr_true = tot[1];
        st->rmax = tot[2];
    }
}

template <class T, bool UNIT>
__global__ __launch_bounds__(kThreads) void k_p1(SysView<T> S, int run) {
    if (S.st->done) return;
    const int t = xcd_tile(blockIdx.x, S.cell_blocks, run);
    double acc[1];
    cell_p1<T, UNIT>(S, t * kThreads + threadIdx.x, acc);
    double tot[1];
    if (grid_reduce<1>(acc, S.red, S.cell_blocks, t, tot) && threadIdx.x == 0)
        tail_p1(S.st, tot);
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_p2a(SysView<T> S) {
    if (S.st->done) return;
    double acc[1] = {0.0};
    chunk_p2a<T>(S, blockIdx.x, acc);
    double tot[1];
    if (grid_reduce<1>(acc, S.red, S.stream_blocks, blockIdx.x, tot) && threadIdx.x == 0)
        tail_p2a(S.st, tot);
}

template <class T, bool UNIT>
__global__ __launch_bounds__(kThreads) void k_p2(SysView<T> S, int run) {
    if (S.st->done) return;
    const int t = xcd_tile(blockIdx.x, S.cell_blocks, run);
    double acc[4];
    cell_p2b<T, UNIT>(S, t * kThreads + threadIdx.x, acc);
    double tot[4];
    if (grid_reduce<4>(acc, S.red, S.cell_blocks, t, tot) && threadIdx.x == 0)
        tail_p2(S.st, tot);
}

template <class T, bool UNIT>
__global__ __launch_bounds__(kThreads) void k_p1_pair(SysView<T> S, int run) {
    if (S.st->done) return;
    const int t = xcd_tile(blockIdx.x, S.pair_blocks, run);
    double acc[1];
    pair_p1<T, UNIT>(S, cell2_at(t * kThreads + threadIdx.x, S.m, S.n), acc);
    double tot[1];
    if (grid_reduce<1>(acc, S.red, S.pair_blocks, t, tot) && threadIdx.x == 0)
        tail_p1(S.st, tot);
}

template <class T, bool UNIT>
__global__ __launch_bounds__(kThreads) void k_p2f_pair(SysView<T> S, int run) {
    if (S.st->done) return;
    const int t = xcd_tile(blockIdx.x, S.pair_blocks, run);
    double acc[5];
    pair_p2f<T, UNIT>(S, cell2_at(t * kThreads + threadIdx.x, S.m, S.n), (float)S.st->alpha, acc);
    double tot[5];
    if (grid_reduce<5>(acc, S.red, S.pair_blocks, t, tot) && threadIdx.x == 0)
        tail_p2f(S.st, tot);
}

template <class T, bool UNIT>
__global__ __launch_bounds__(kThreads) void k_p2f(SysView<T> S, int run) {
    if (S.st->done) return;
    const int t = xcd_tile(blockIdx.x, S.cell_blocks, run);
    double acc[5];
    cell_p2f<T, UNIT>(S, t * kThreads + threadIdx.x, (float)S.st->alpha, acc);
    double tot[5];
    if (grid_reduce<5>(acc, S.red, S.cell_blocks, t, tot) && threadIdx.x == 0)
        tail_p2f(S.st, tot);
}

// The staged stencil passes (TILE cells per workgroup: 2048, 4096 or 8192; the
// dynamic LDS holds lds_count(nx, TILE) floats).  Each thread sums its pairs' products first, in pair
// order, then the workgroup and the grid sums follow as in the flat passes.
template <class T, bool UNIT, int TILE>
__global__ __launch_bounds__(kThreads) void k_p1_lds(SysView<T> S, int nblocks, int run) {
    extern __shared__ float stage[];
    if (S.st->done) return;
    const int tile = xcd_tile(blockIdx.x, nblocks, run);
    const int nx = S.m.nx, c0 = tile * TILE, lo = lds_lo(c0, nx);
    const int hi = (c0 + TILE + nx + 7) >> 3 << 3;
    stage_rows<T, false>(S.p, nullptr, 0.0f, lo, hi - lo, S.n, stage);
    __syncthreads();
    double acc[1] = {0.0};
    const Cell none{};
#pragma unroll 2
    for (int u = 0; u < TILE / (2 * kThreads); ++u) {
        const int idx = c0 + 2 * (u * kThreads + (int)threadIdx.x);
        if (idx >= S.n) break;
        int db, dt;
        z_offsets(idx, S.m, db, dt);
        const F2 pb = ld2(S.p + idx + db), pt = ld2(S.p + idx + dt);
        Nbr<float> p0, p1;
        lds_nbr2(stage, idx - lo, nx, pb, pt, p0, p1);
        Coefs<float, UNIT> k0, k1;
        load_coefs2_nt<T, UNIT>(S.c, idx, k0, k1);
        const F2 rh = ld2_nt(S.rhat + idx);
        const T s0 = from_f32<T>(apply7<float, float, UNIT, false>(k0, p0, none));
        const T s1 = from_f32<T>(apply7<float, float, UNIT, false>(k1, p1, none));
        st2_nt(S.s + idx, s0, s1);
        acc[0] += fma((double)rh.b, (double)to_f32(s1), (double)rh.a * (double)to_f32(s0));
    }
    double tot[1];
    if (grid_reduce<1>(acc, S.red, nblocks, tile, tot) && threadIdx.x == 0) tail_p1(S.st, tot);
}

template <class T, bool UNIT, int TILE>
__global__ __launch_bounds__(kThreads) void k_p2f_lds(SysView<T> S, int nblocks, int run) {
    extern __shared__ float stage[];
    if (S.st->done) return;
    const float alpha = (float)S.st->alpha;
    const int tile = xcd_tile(blockIdx.x, nblocks, run);
    const int nx = S.m.nx, c0 = tile * TILE, lo = lds_lo(c0, nx);
    const int hi = (c0 + TILE + nx + 7) >> 3 << 3;
    stage_rows<T, true>(S.r, S.s, alpha, lo, hi - lo, S.n, stage);
    __syncthreads();
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const Cell none{};
#pragma unroll 2
    for (int u = 0; u < TILE / (2 * kThreads); ++u) {
        const int idx = c0 + 2 * (u * kThreads + (int)threadIdx.x);
        if (idx >= S.n) break;
        int db, dt;
        z_offsets(idx, S.m, db, dt);
        const F2 rb = ld2(S.r + idx + db), sb = ld2(S.s + idx + db);
        const F2 rt = ld2(S.r + idx + dt), st = ld2(S.s + idx + dt);
        const F2 qb{fmaT(-alpha, sb.a, rb.a), fmaT(-alpha, sb.b, rb.b)};
        const F2 qt{fmaT(-alpha, st.a, rt.a), fmaT(-alpha, st.b, rt.b)};
        Nbr<float> q0, q1;
        lds_nbr2(stage, idx - lo, nx, qb, qt, q0, q1);
        Coefs<float, UNIT> k0, k1;
        load_coefs2_nt<T, UNIT>(S.c, idx, k0, k1);
        const F2 rh = ld2_nt(S.rhat + idx);
        const T y0 = from_f32<T>(apply7<float, float, UNIT, false>(k0, q0, none));
        const T y1 = from_f32<T>(apply7<float, float, UNIT, false>(k1, q1, none));
        st2_nt(S.y + idx, y0, y1);
        const double ya = (double)to_f32(y0), yb = (double)to_f32(y1);
        const double qa = (double)q0.c, qb2 = (double)q1.c;
        acc[0] += fma(qb2, yb, qa * ya);
        acc[1] += fma(yb, yb, ya * ya);
        acc[2] += fma(qb2, qb2, qa * qa);
        acc[3] += fma((double)rh.b, qb2, (double)rh.a * qa);
        acc[4] += fma((double)rh.b, yb, (double)rh.a * ya);
    }
    double tot[5];
    if (grid_reduce<5>(acc, S.red, nblocks, tile, tot) && threadIdx.x == 0) tail_p2f(S.st, tot);
}

template <class T, bool QR>
__global__ __launch_bounds__(kThreads) void k_p3(SysView<T> S) {
    if (S.st->done) return;
    double acc[2];
    chunk_p3<T, QR>(S, blockIdx.x, acc);
    double tot[2];
    if (grid_reduce<2>(acc, S.red, S.stream_blocks, blockIdx.x, tot) && threadIdx.x == 0)
        tail_p3(S.st, tot);
}

}  // namespace s7
