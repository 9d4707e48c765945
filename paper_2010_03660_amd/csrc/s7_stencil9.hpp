// The 2D 9-point operator of section IV ("SpMV (2D)"): BiCGStab (Algorithm 1)
// on an nx x ny mesh whose rows hold the main diagonal, the four axis
// neighbours (w, e, s, n) and the four corners (sw, se, nw, ne).  The paper
// sketches this second mapping and sizes it at 4800^2 and 22800^2 meshes.
//
// FP32 storage, or BF16/FP16 storage inside FP64 iterative refinement (the
// outer loop shared with the 3D solver).  The iteration is the three-pass
// schedule of the 3D solver, one cell per thread in the two stencil passes:
// P1 s = A p with (r0, s); P2 forms q = r - alpha s at the cell and its eight
// neighbours, y = A q, and the five sums; P3 is the 3D streaming pass
// unchanged (it touches no coefficient).  Working coefficient copies are
// Jacobi-scaled with every outward link (axis or corner) zeroed, so all nine
// loads of a cell stay in the mesh and need no test: an off-mesh neighbour
// reads the cell itself, times zero.  Included by the solver translation
// unit (s7_single.hip) only, after the pieces it shares with the 3D path
// (State, reductions, P3, refinement loop, x update, graph cache).
#pragma once

#include "s7_stencil9_device.hpp"

namespace s7 {

// ---------------------------------------------------------------- kernels
__global__ __launch_bounds__(kThreads) void k9_apply_f32(Coef9 cf, const float* v, float* u, Mesh m, int n) {
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, m, n);
    float x[9];
    load9(v, c, x);
    const float av = apply9_masked<float>(cf, c, x);
    if (c.own) u[c.idx] = av;
}

__global__ __launch_bounds__(kThreads) void k9_apply_f64(Coef9 cf, const double* v, double* u, Mesh m, int n) {
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, m, n);
    double x[9];
    load9(v, c, x);
    const double av = apply9_masked<double>(cf, c, x);
    if (c.own) u[c.idx] = av;
}

// Working copies in storage type T: c[a] / diag for a = 1..8 with Jacobi
// scaling, else all nine; outward links zeroed; rounded once to T.
template <class T>
__global__ __launch_bounds__(kThreads) void k9_prep(Coef9 src, T* dst0, size_t span, Mesh m, int n,
                                                    int jacobi) {
    const int first = jacobi ? 1 : 0;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        const Cell c = cell_at(i, m, n);
        bool in[9];
        inside9(c, in);
        const float dg = src.c[0][i];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            if (a < first) continue;
            float v = in[a] ? src.c[a][i] : 0.0f;
            if (jacobi) v = v / dg;
            dst0[(size_t)(a - first) * span + i] = from_f32<T>(v);
        }
    }
}

// r0 = b - A x0 in FP64 with the caller's coefficients, Jacobi-scaled, rounded
// to FP32 into r, r0 and p; d = 0.  Sums ||b_s||^2, (r,r) of the rounded r,
// ||b||^2 unscaled.
__global__ __launch_bounds__(kThreads) void k9_init(Coef9 cf, const double* b, const double* x0,
                                                    SysView<float> S, int jacobi, double tol, int max_iter) {
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, S.m, S.n);
    double xv[9];
    load9(x0, c, xv);
    const double bi = b[c.idx];
    double r0 = bi - apply9_masked<double>(cf, c, xv), bs = bi;
    if (jacobi) {
        const double dg = (double)cf.c[0][c.idx];
        r0 = r0 / dg;
        bs = bs / dg;
    }
    const float rf = (float)r0;
    if (c.own) {
        S.r[c.idx] = rf;
        S.rhat[c.idx] = rf;
        S.p[c.idx] = rf;
        S.d[c.idx] = 0.0f;
    }
    double acc[3] = {c.own ? bs * bs : 0.0, c.own ? (double)rf * (double)rf : 0.0, c.own ? bi * bi : 0.0};
    double tot[3];
    if (grid_reduce<3>(acc, S.red, S.cell_blocks, blockIdx.x, tot) && threadIdx.x == 0) {
        tail_init(S.st, tot[0], tot[1], tol, max_iter);
        S.st->bb_true = tot[2];
        S.st->scale = 1.0;
    }
}

// P1: s = A p, rounded to T; (r0, s) of the rounded s.
template <class T, bool UNIT>
__global__ __launch_bounds__(kThreads) void k9_p1(SysView<T> S, Coef9T<T> k) {
    if (S.st->done) return;
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, S.m, S.n);
    float pv[9];
    load9f(S.p, c, pv);
    const T sv = from_f32<T>(apply9_work<T, UNIT>(k, c.idx, pv));
    const float rh = to_f32(ld_nt(S.rhat + c.idx));
    if (c.own) S.s[c.idx] = sv;
    double acc[1] = {c.own ? (double)rh * (double)to_f32(sv) : 0.0};
    double tot[1];
    if (grid_reduce<1>(acc, S.red, S.cell_blocks, blockIdx.x, tot) && threadIdx.x == 0) tail_p1(S.st, tot);
}

// P2: q = r - alpha s at the nine points (FP32), y = A q rounded to T;
// (q,y), (y,y), (q,q), (r0,q), (r0,y).
template <class T, bool UNIT>
__global__ __launch_bounds__(kThreads) void k9_p2f(SysView<T> S, Coef9T<T> k) {
    if (S.st->done) return;
    const float alpha = (float)S.st->alpha;
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, S.m, S.n);
    float rv[9], sv[9], q[9];
    load9f(S.r, c, rv);
    load9f(S.s, c, sv);
#pragma unroll
    for (int a = 0; a < 9; ++a) q[a] = fma9(-alpha, sv[a], rv[a]);
    const T yv = from_f32<T>(apply9_work<T, UNIT>(k, c.idx, q));
    const double rh = (double)to_f32(ld_nt(S.rhat + c.idx));
    if (c.own) S.y[c.idx] = yv;
    const double qd = c.own ? (double)q[0] : 0.0, yd = c.own ? (double)to_f32(yv) : 0.0;
    double acc[5] = {qd * yd, yd * yd, qd * qd, rh * qd, rh * yd};
    double tot[5];
    if (grid_reduce<5>(acc, S.red, S.cell_blocks, blockIdx.x, tot) && threadIdx.x == 0) tail_p2f(S.st, tot);
}

// True residual r = b - A x in FP64 with the caller's coefficients.  Sums
// ||b||^2, ||r||^2, max |fl32(r_s)|.  If dst is not null, r_s = r / diag (Jacobi)
// goes there as FP32: the right-hand side of the next refinement step.
__global__ __launch_bounds__(kThreads) void k9_resid(Coef9 cf, const double* b, const double* x, float* dst,
                                                     Mesh m, int n, int nblocks, State* st, Red red, int jacobi) {
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, m, n);
    double xv[9];
    load9(x, c, xv);
    const double bi = b[c.idx];
    const double r0 = bi - apply9_masked<double>(cf, c, xv);
    const double rs = jacobi ? r0 / (double)cf.c[0][c.idx] : r0;
    const float rf = (float)rs;
    if (dst && c.own) dst[c.idx] = rf;
    double acc[3] = {c.own ? bi * bi : 0.0, c.own ? r0 * r0 : 0.0, c.own ? (double)fabsf(rf) : 0.0};
    double tot[3];
    if (grid_reduce<3, 4u>(acc, red, nblocks, blockIdx.x, tot) && threadIdx.x == 0) {
        st->bb_true = tot[0];
        st->rr_true = tot[1];
        st->rmax = tot[2];
    }
}

// The seeded recipe of the 2D 9-point inputs: off-diagonal a (aid 19 + a) is
// -(0.5 + m 2^-24) with m the top 23 bits of the cell hash; the diagonal is
// fl32(sum |off| + 0.1), the eight magnitudes summed in FP64 in order; x* as in
// 3D (aid 7).
__global__ __launch_bounds__(kThreads) void k9_gen(Coef9 out, double* xstar, int n, uint64_t seed) {
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        double sum = 0.0;
        float off[8];
#pragma unroll
        for (int a = 1; a <= 8; ++a) {
            const uint64_t h = gen_hash(seed, 19 + a, (uint64_t)i);
            const float v = (float)(-(__dadd_rn(0.5, __dmul_rn((double)(h >> 41), 0x1p-24))));
            off[a - 1] = v;
            sum = __dadd_rn(sum, fabs((double)v));
        }
        if (out.c[0]) const_cast<float*>(out.c[0])[i] = (float)__dadd_rn(sum, 0.1);
#pragma unroll
        for (int a = 1; a <= 8; ++a)
            if (out.c[a]) const_cast<float*>(out.c[a])[i] = off[a - 1];
        if (xstar) {
            const uint64_t h = gen_hash(seed, 7, (uint64_t)i);
            xstar[i] = __dadd_rn(-1.0, __dmul_rn((double)(h >> 40), 0x1p-23));
        }
    }
}

// ---------------------------------------------------------------- driver
static bool dims2_ok(int32_t nx, int32_t ny) {
    return nx >= 1 && ny >= 1 && (long long)nx * ny <= kMaxCells;
}

static Layout make_layout9(int32_t nx, int32_t ny, int prec, const s7_options& o) {
    return make_layout(s7_dims{nx, ny, 1}, prec, o, o.jacobi ? 8 : 9);
}

// The working copies inside the workspace, in storage type T.
template <class T>
static Coef9T<T> work_coefs9(const Layout& L, int jacobi, char* ws) {
    Coef9T<T> k{};
    const size_t span = align256(L.n * L.elt);
    const int first = jacobi ? 1 : 0;
    for (int a = first; a < 9; ++a)
        k.c[a] = reinterpret_cast<const T*>(ws + L.off_coef + (size_t)(a - first) * span);
    return k;
}

template <class T>
static void launch_iter9(const SysView<T>& S, const Coef9T<T>& k, int pass, hipStream_t s) {
    const int nb = S.cell_blocks;
    if (pass == 0) {
        if (S.unit) hipLaunchKernelGGL((k9_p1<T, true>), dim3(nb), dim3(kThreads), 0, s, S, k);
        else hipLaunchKernelGGL((k9_p1<T, false>), dim3(nb), dim3(kThreads), 0, s, S, k);
        launch_finish<1, 0u, FIN_P1>(S.red, nb, S.st, s);
    } else if (pass == 1) {
        if (S.unit) hipLaunchKernelGGL((k9_p2f<T, true>), dim3(nb), dim3(kThreads), 0, s, S, k);
        else hipLaunchKernelGGL((k9_p2f<T, false>), dim3(nb), dim3(kThreads), 0, s, S, k);
        launch_finish<5, 0u, FIN_P2F>(S.red, nb, S.st, s);
    } else {
        hipLaunchKernelGGL((k_p3<T, true>), dim3(S.stream_blocks), dim3(kThreads), 0, s, S);
    }
}

// Inner iterations from the State set by the start (FP32) or by k_ir_init
// (refinement), K per host check: graph replays, or with profile direct
// launches timed per pass into the slots of the 3D three-pass schedule.
template <class T>
static int iterate9(const SysView<T>& S, const Coef9T<T>& k, const s7_options& o, hipStream_t s, State* h,
                    s7_info* info) {
    int rc = read_state(S.st, h, s);
    if (rc || h->done) return rc;
    const int K = o.graph_iters > 0 ? o.graph_iters : auto_graph_iters((size_t)S.n, (int)sizeof(T));
    const long long max_launches = (long long)h->max_iter / K + 3;
    if (o.profile) {
        const int slot[3] = {0, 2, 3};
        std::vector<hipEvent_t> ev((size_t)4 * K);
        for (auto& e : ev) S7_HIP(hipEventCreate(&e));
        for (long long l = 0; l < max_launches && !h->done; ++l) {
            const int it0 = h->iter;
            for (int j = 0; j < K; ++j) {
                for (int p = 0; p < 3; ++p) {
                    S7_HIP(hipEventRecord(ev[4 * j + p], s));
                    launch_iter9<T>(S, k, p, s);
                }
                S7_HIP(hipEventRecord(ev[4 * j + 3], s));
            }
            S7_CHECK_LAUNCH();
            if ((rc = read_state(S.st, h, s))) return rc;
            for (int j = 0; info && j < K && j < h->iter - it0; ++j)
                for (int p = 0; p < 3; ++p) {
                    float ms = 0.f;
                    S7_HIP(hipEventElapsedTime(&ms, ev[4 * j + p], ev[4 * j + p + 1]));
                    info->pass_ms[slot[p]] += ms;
                    info->pass_count[slot[p]] += 1;
                }
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
    } else {
        std::vector<uintptr_t> key = {0x92u, (uintptr_t)TypeTag<T>::value, (uintptr_t)K, (uintptr_t)S.m.nx,
                                      (uintptr_t)S.m.ny, (uintptr_t)S.unit, (uintptr_t)S.st, (uintptr_t)S.red.part,
                                      (uintptr_t)S.r, (uintptr_t)k.c[1], (uintptr_t)S.d,
                                      (uintptr_t)S.stream_blocks};
        GraphRef g;
        rc = cached_graph(key, [&](hipStream_t cs) {
            for (int j = 0; j < K; ++j)
                for (int p = 0; p < 3; ++p) launch_iter9<T>(S, k, p, cs);
        }, &g);
        if (rc) return rc;
        for (long long l = 0; l < max_launches && !h->done; ++l) {
            S7_HIP(hipGraphLaunch(g->exec, s));
            if ((rc = read_state(S.st, h, s))) return rc;
        }
    }
    if (!h->done) {
        set_error("iteration driver did not reach a final state");
        return S7_EHIP;
    }
    return S7_OK;
}

static void resid9_launch(const Coef9& cf, const double* b, const double* x, float* dst, const Mesh& m, int n,
                          int cell_blocks, State* st, const Red& red, int jacobi, hipStream_t s) {
    hipLaunchKernelGGL(k9_resid, dim3(cell_blocks), dim3(kThreads), 0, s, cf, b, x, dst, m, n, cell_blocks, st, red,
                       jacobi);
    launch_finish<3, 4u, FIN_RESID>(red, cell_blocks, st, s);
}

// Clears the State and writes the working coefficient copies.
template <class T>
static void start9(const Coef9& cf, const SysView<T>& S, const Coef9T<T>& k, const Layout& Lo, int jacobi,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_zero_state, dim3(1), dim3(kThreads), 0, s, S.st, S.red.cnt, 1);
    hipLaunchKernelGGL((k9_prep<T>), dim3(grid_for(S.n)), dim3(kThreads), 0, s, cf,
                       const_cast<T*>(k.c[jacobi ? 1 : 0]), align256(Lo.n * Lo.elt) / Lo.elt, S.m, S.n, jacobi);
}

static int solve9(int32_t nx, int32_t ny, const Coef9& cf, const double* b, double* x, double rtol,
                  int max_iter, char* ws, const Layout& Lo, const s7_options& o, s7_info* info,
                  hipStream_t s) {
    const s7_dims d{nx, ny, 1};
    SysView<float> S = make_view<float>(d, Lo, o.jacobi, ws);
    const Coef9 k = work_coefs9<float>(Lo, o.jacobi, ws);
    auto t0 = std::chrono::steady_clock::now();
    start9<float>(cf, S, k, Lo, o.jacobi, s);
    hipLaunchKernelGGL(k9_init, dim3(S.cell_blocks), dim3(kThreads), 0, s, cf, b, x, S, o.jacobi, rtol, max_iter);
    launch_finish<3, 0u, FIN_INIT>(S.red, S.cell_blocks, S.st, s, rtol, max_iter);
    S7_CHECK_LAUNCH();
    State h;
    int rc = iterate9<float>(S, k, o, s, &h, info);
    if (rc) return rc;
    hipLaunchKernelGGL(k_update_x, dim3(S.stream_blocks), dim3(kThreads), 0, s, x, S.d, S.n, 1.0, S.st);
    resid9_launch(cf, b, x, nullptr, S.m, S.n, S.cell_blocks, S.st, S.red, o.jacobi, s);
    S7_CHECK_LAUNCH();
    if ((rc = read_state(S.st, &h, s))) return rc;
    auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->status = h.status;
        info->reason = h.reason;
        info->rel_res_rec = h.res_rec;
        info->iters = h.iter;
        info->outer_iters = 1;
        info->schedule = SCHED_THREE;
        info->rel_res_true = h.bb_true > 0 ? sqrt(h.rr_true / h.bb_true) : 0.0;
        info->t_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    return h.status;
}

// 16-bit storage inside FP64 iterative refinement (reading 13), the outer loop
// shared with the 3D solver.
template <class T>
static int solve9_ir(int32_t nx, int32_t ny, const Coef9& cf, const double* b, double* x, double rtol,
                     int max_iter, char* ws, const Layout& Lo, const s7_options& o, s7_info* info,
                     hipStream_t s, int prec) {
    const s7_dims d{nx, ny, 1};
    SysView<T> S = make_view<T>(d, Lo, o.jacobi, ws);
    const Coef9T<T> k = work_coefs9<T>(Lo, o.jacobi, ws);
    start9<T>(cf, S, k, Lo, o.jacobi, s);
    S7_CHECK_LAUNCH();
    return refine<T>(S, x, rtol, max_iter, o, prec, SCHED_THREE, info, s,
                     [&]() -> int {
                         resid9_launch(cf, b, x, S.d, S.m, S.n, S.cell_blocks, S.st, S.red, o.jacobi, s);
                         S7_CHECK_LAUNCH();
                         return S7_OK;
                     },
                     [&](State* h) { return iterate9<T>(S, k, o, s, h, info); });
}

static bool coef9_ok(const float* const coef[9]) {
    if (!coef) return false;
    for (int a = 0; a < 9; ++a)
        if (!coef[a]) return false;
    return true;
}

}  // namespace s7

extern "C" {

int s7_stencil9_apply(int32_t nx, int32_t ny, const float* const coef[9], const float* v, float* u,
                      void* stream) {
    clear_error();
    if (!dims2_ok(nx, ny) || !coef9_ok(coef) || !v || !u || v == u) {
        set_error("s7_stencil9_apply: invalid argument");
        return S7_EINVAL;
    }
    Coef9 cf;
    for (int a = 0; a < 9; ++a) cf.c[a] = coef[a];
    const int n = nx * ny;
    hipLaunchKernelGGL(k9_apply_f32, dim3(cell_blocks_for(n)), dim3(kThreads), 0, (hipStream_t)stream, cf, v, u,
                       make_mesh(nx, ny, 1), n);
    S7_CHECK_LAUNCH();
    return S7_OK;
}

size_t s7_workspace_bytes_2d9(int32_t nx, int32_t ny, int32_t prec, const s7_options* opt) {
    if (!dims2_ok(nx, ny) || prec < S7_FP32 || prec > S7_FP16_IR) return 0;
    s7_options o;
    options_or_default(opt, o);
    return make_layout9(nx, ny, prec, o).bytes;
}

int s7_bicgstab_solve_2d9(int32_t nx, int32_t ny, const float* const coef[9], const double* b, double* x,
                          double rtol, int32_t max_iter, int32_t prec, void* ws, size_t ws_bytes,
                          const s7_options* opt, s7_info* info, void* stream) {
    clear_error();
    if (info) std::memset(info, 0, sizeof(*info));
    s7_options o;
    options_or_default(opt, o);
    if (!dims2_ok(nx, ny) || !coef9_ok(coef) || !b || !x || !ws || !(rtol > 0.0) || max_iter < 0 ||
        prec < S7_FP32 || prec > S7_FP16_IR || ((uintptr_t)ws & 255u) != 0) {
        set_error("s7_bicgstab_solve_2d9: invalid argument");
        return S7_EINVAL;
    }
    const Layout Lo = make_layout9(nx, ny, prec, o);
    if (ws_bytes < Lo.bytes) {
        set_error("s7_bicgstab_solve_2d9: workspace too small (%zu < %zu)", ws_bytes, Lo.bytes);
        return S7_EINVAL;
    }
    Coef9 cf;
    for (int a = 0; a < 9; ++a) cf.c[a] = coef[a];
    hipStream_t st = (hipStream_t)stream;
    if (prec == S7_FP32) return solve9(nx, ny, cf, b, x, rtol, max_iter, (char*)ws, Lo, o, info, st);
    if (prec == S7_BF16_IR) return solve9_ir<bf16>(nx, ny, cf, b, x, rtol, max_iter, (char*)ws, Lo, o, info, st, prec);
    return solve9_ir<f16>(nx, ny, cf, b, x, rtol, max_iter, (char*)ws, Lo, o, info, st, prec);
}

size_t s7_batched_workspace_bytes_2d9(int32_t nsys, const int32_t* nx, const int32_t* ny, int32_t prec,
                                      const s7_options* opt) {
    if (nsys < 1 || !nx || !ny || prec < S7_FP32 || prec > S7_FP16_IR) return 0;
    s7_options o;
    options_or_default(opt, o);
    size_t total = align256(engine_table_bytes(nsys));
    for (int i = 0; i < nsys; ++i) {
        if (!dims2_ok(nx[i], ny[i])) return 0;
        total += align256(make_layout9(nx[i], ny[i], prec, o).bytes);
    }
    return total;
}

int s7_bicgstab_solve_batched_2d9(int32_t nsys, const int32_t* nx, const int32_t* ny, const float* const* coef,
                                  const double* const* b, double* const* x, const double* rtol,
                                  const int32_t* max_iter, int32_t prec, void* ws, size_t ws_bytes,
                                  const s7_options* opt, s7_info* info, void* stream) {
    clear_error();
    s7_options o;
    options_or_default(opt, o);
    if (nsys < 1 || !nx || !ny || !coef || !b || !x || !rtol || !max_iter || !ws ||
        ((uintptr_t)ws & 255u) != 0 || prec < S7_FP32 || prec > S7_FP16_IR) {
        set_error("s7_bicgstab_solve_batched_2d9: invalid argument");
        return S7_EINVAL;
    }
    for (int i = 0; i < nsys; ++i) {
        if (!dims2_ok(nx[i], ny[i]) || !coef9_ok(coef + 9 * (size_t)i) || !b[i] || !x[i] || !(rtol[i] > 0.0) ||
            max_iter[i] < 0) {
            set_error("s7_bicgstab_solve_batched_2d9: invalid argument for system %d", i);
            return S7_EINVAL;
        }
    }
    const size_t need = s7_batched_workspace_bytes_2d9(nsys, nx, ny, prec, &o);
    if (ws_bytes < need) {
        set_error("s7_bicgstab_solve_batched_2d9: workspace too small (%zu < %zu)", ws_bytes, need);
        return S7_EINVAL;
    }
    char* w = (char*)ws;
    const long long split = split_cells_of(o);
    std::vector<EngineJob> jobs((size_t)nsys);
    std::vector<char> big((size_t)nsys, 0);
    size_t off = align256(engine_table_bytes(nsys));
    const double t0 = now_ms();
    for (int i = 0; i < nsys; ++i) {
        EngineJob& j = jobs[i];
        std::memset(&j, 0, sizeof(j));
        j.d = s7_dims{nx[i], ny[i], 1};
        for (int a = 0; a < 7; ++a) j.coef[a] = coef[9 * (size_t)i + a];
        j.coef9[0] = coef[9 * (size_t)i + 7];
        j.coef9[1] = coef[9 * (size_t)i + 8];
        j.b = b[i];
        j.x = x[i];
        j.rtol = rtol[i];
        j.max_iter = max_iter[i];
        j.prec = prec;
        j.ws = w + off;
        j.ws_bytes = make_layout9(nx[i], ny[i], prec, o).bytes;
        j.t_start_ms = t0;
        big[i] = (long long)nx[i] * ny[i] >= split;
        off += align256(j.ws_bytes);
    }
    return run_batch(jobs, big, OP_9PT, w, o, (hipStream_t)stream, info, "s7_bicgstab_solve_batched_2d9",
                     [&](EngineJob& j) {
                         const float* c9[9];
                         for (int a = 0; a < 7; ++a) c9[a] = j.coef[a];
                         c9[7] = j.coef9[0];
                         c9[8] = j.coef9[1];
                         return s7_bicgstab_solve_2d9(j.d.nx, j.d.ny, c9, j.b, j.x, j.rtol, j.max_iter, prec, j.ws,
                                                      j.ws_bytes, &o, &j.info, stream);
                     });
}

int s7_generate_problem_2d9(int32_t nx, int32_t ny, uint64_t seed, float* const coef[9], double* xstar,
                            double* b, void* stream) {
    clear_error();
    if (!dims2_ok(nx, ny) || (b && (!coef || !xstar))) {
        set_error("s7_generate_problem_2d9: invalid argument");
        return S7_EINVAL;
    }
    Coef9 cf{};
    bool all = coef != nullptr;
    for (int a = 0; a < 9; ++a) {
        cf.c[a] = coef ? coef[a] : nullptr;
        all = all && cf.c[a];
    }
    if (b && !all) {
        set_error("s7_generate_problem_2d9: b needs all coefficient arrays and xstar");
        return S7_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int n = nx * ny;
    hipLaunchKernelGGL(k9_gen, dim3(grid_for(n)), dim3(kThreads), 0, s, cf, xstar, n, seed);
    S7_CHECK_LAUNCH();
    if (b) {
        hipLaunchKernelGGL(k9_apply_f64, dim3(cell_blocks_for(n)), dim3(kThreads), 0, s, cf, (const double*)xstar,
                           b, make_mesh(nx, ny, 1), n);
        S7_CHECK_LAUNCH();
    }
    return S7_OK;
}

}  // extern "C"
