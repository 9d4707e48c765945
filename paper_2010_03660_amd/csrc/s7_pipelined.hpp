// Pipelined BiCGStab (Cools and Vanroose, "The communication-hiding pipelined
// BiCGStab method for the parallel solution of large unsymmetric linear
// systems", Parallel Computing 65, 2017) on the 7-point operator, in the form
// with a single reduction per iteration.  In exact arithmetic its iterates are
// those of Algorithm 1; the matrix products are carried forward by
// recurrences: s = A p, z = A s, w = A r, t = A w, v = A z, y = A q.
//
// FP32 storage and arithmetic, FP64 inner products, Jacobi scaling as in the
// classical solver.  Four passes per iteration:
//   K1 (streaming)  p = r + beta (p - omega s), s = w + beta (s - omega z),
//                   z = t + beta (z - omega v), q = r - alpha s, y = w - alpha z;
//                   sums (r0,y), (r0,t), (r0,s), (r0,z)
//   K2 (stencil)    v = A z; sums (r,r), (q,y), (y,y), (q,q), (r0,q), (r0,v).
//                   Its completion takes every decision of the iteration: the
//                   stopping test on r_i, the half-step test, omega, and from
//                   the ten sums rho_{i+1}, beta_i, (r0, A p_{i+1}), alpha_{i+1}
//   K3 (streaming)  d += alpha p + omega q, r = q - omega y,
//                   w = y - omega (t - alpha v)
//   K4 (stencil)    t = A w
// The ten sums belong to one reduction point of the method; they are taken in
// two kernels because K1 forms y, s and z, and K2 forms v.  The stopping test
// on r_i is decided in iteration i's K2 (after half an iteration's work, which
// is then not applied), as in the oracle's variant.
//
// Residual replacement (Cools, Yetkin, Agullo, Giraud and Vanroose, "Analyzing
// the effect of local rounding error propagation on the maximal attainable
// accuracy of the pipelined Conjugate Gradient method", SIAM J. Matrix Anal.
// Appl. 39, 2018, applied here to BiCGStab): in FP32 storage the recurrences
// for the matrix products drift from A, and the true residual stalls orders of
// magnitude above the recurrence residual.  Every kReplace iterations the
// iteration folds d into x and recomputes r = b - A x (FP64), w = A r,
// t = A w, s = A p, z = A s, v = A z from their definitions, then rho and
// (r0, A p) from the new vectors.
//
// Verified stops.  A stop that the recurrences decide (||r_i|| or ||q_i|| at
// most the tolerance, or rho_{i+1} = 0 with a small residual) is only a
// candidate unless r_i was replaced since the last update: the iteration then
// idles until the next replacement, whose true residual decides.  At most the
// tolerance, the solve ends with S7_OK; otherwise it goes on from the replaced
// vectors with the search direction restarted (beta = 0: p = r, s = w, z = t)
// until the true residual meets the tolerance or the iteration cap ends it.
// With x kept in FP64 and r recomputed from it, the true residual keeps
// falling below the FP32 storage floor, as in iterative refinement.  Included
// by the solver translation unit (s7_single.hip) only.
#pragma once

namespace s7 {

// Scalars of the pipelined iteration beyond the State: the sums K1 takes, the
// next alpha, and which update K3 applies (0 none, 1 half step, 2 full).
struct PipeScalars {
    double ry, rt, rs, rz;
    double alpha_next;
    int32_t flag;
    int32_t verify;  // 1: a candidate stop waits for the next replacement
    int32_t fresh;   // 1: r was replaced and no update has been applied since
    int32_t pad;
};

struct PipeView {
    float *z, *w, *t, *v;
    PipeScalars* ps;
};

enum PipeFinish : int { PF_W0 = 1, PF_K1 = 2, PF_K2 = 3, PF_RR = 4 };

constexpr int kReplace = 10;  // iterations between residual replacements

// After w_0 = A r_0: sigma_0 = (r0, w_0), alpha_0 = rho_0 / sigma_0.
__device__ __forceinline__ void tail_w0(State* st, PipeScalars* ps, const double (&tot)[1]) {
    st->sigma = tot[0];
    st->beta = 0.0;
    st->omega = 0.0;
    ps->flag = 0;
    if (tot[0] == 0.0) {
        set_breakdown(st, RS_RS_ZERO);
        return;
    }
    const double a = st->rho / tot[0];
    if (!isfinite(a)) {
        set_breakdown(st, RS_NONFINITE);
        return;
    }
    st->alpha = a;
    ps->alpha_next = a;
}

// After a replacement: rho = (r0, r), (r0, A p_{i+1}) = (r0, w) + beta ((r0, s) - omega (r0, z)).
// tot[4] = (r, r) of the replaced r decides a candidate stop.
__device__ __forceinline__ void tail_rr(State* st, PipeScalars* ps, const double (&tot)[5]) {
    ps->fresh = 1;
    if (ps->verify) {
        ps->verify = 0;
        const double res = sqrt(tot[4]) / st->nb;
        if (!isfinite(res)) {
            set_breakdown(st, RS_NONFINITE);
            return;
        }
        if (res <= st->tol) {
            st->res_rec = res;
            st->status = ST_OK;
            st->done = 1;
            return;
        }
        if (st->iter >= st->max_iter) {
            st->res_rec = res;
            st->status = ST_NOT_CONVERGED;
            st->done = 1;
            return;
        }
        st->half = 0;
        st->beta = 0.0;  // restart the direction from the true residual
        st->omega = 0.0;
    }
    const double rho = tot[0];
    const double sig = tot[1] + st->beta * (tot[2] - st->omega * tot[3]);
    double a;
    if (sig != 0.0) {
        a = rho / sig;
    } else if (rho == 0.0) {
        a = 0.0;  // r = 0: the next reduction stops on ||r||
    } else {
        set_breakdown(st, RS_RS_ZERO);
        return;
    }
    if (!isfinite(a)) {
        set_breakdown(st, RS_NONFINITE);
        return;
    }
    st->rho = rho;
    st->sigma = sig;
    st->alpha = a;
    ps->alpha_next = a;
}

__device__ __forceinline__ void tail_k1(PipeScalars* ps, const double (&tot)[4]) {
    ps->ry = tot[0];
    ps->rt = tot[1];
    ps->rs = tot[2];
    ps->rz = tot[3];
}

// The decisions of iteration i, in the oracle variant's order.
__device__ __forceinline__ void tail_k2(State* st, PipeScalars* ps, const double (&tot)[6]) {
    const double rr = tot[0], qy = tot[1], yy = tot[2], qq = tot[3], rq = tot[4], rv = tot[5];
    const double res = sqrt(rr) / st->nb;
    st->rr = rr;
    st->res_rec = res;
    ps->flag = 0;
    if (!isfinite(res)) {
        set_breakdown(st, RS_NONFINITE);
        return;
    }
    if (res <= st->tol) {
        if (ps->fresh) {  // r_i is the replaced true residual
            st->status = ST_OK;
            st->done = 1;
        } else {
            ps->verify = 1;
        }
        return;
    }
    if (st->iter >= st->max_iter) {
        st->status = ST_NOT_CONVERGED;
        st->done = 1;
        return;
    }
    const double qn = sqrt(qq) / st->nb;
    if (qn <= st->tol) {  // half-step exit: x += alpha p, then the true residual decides
        st->iter += 1;
        st->res_rec = qn;
        st->half = 1;
        st->omega = 0.0;
        ps->flag = 1;
        ps->fresh = 0;
        ps->verify = 1;
        return;
    }
    if (yy == 0.0) {
        set_breakdown(st, RS_YY_ZERO);
        return;
    }
    const double om = qy / yy;
    if (!isfinite(om)) {
        set_breakdown(st, RS_NONFINITE);
        return;
    }
    st->omega = om;
    st->qy = qy;
    st->yy = yy;
    st->qq = qq;
    st->iter += 1;
    ps->flag = 2;  // the full update of this iteration is applied whatever follows
    ps->fresh = 0;
    const double a = st->alpha;
    const double rho_new = rq - om * ps->ry;
    if (rho_new == 0.0) {
        const double est = qq - 2.0 * om * qy + om * om * yy;
        const double rn = sqrt(est > 0.0 ? est : 0.0) / st->nb;
        if (rn <= st->tol) {
            st->res_rec = rn;
            ps->verify = 1;
        } else {
            set_breakdown(st, RS_RHO_ZERO);
        }
        return;
    }
    const double bt = (a / om) * (rho_new / st->rho);
    const double sig = ps->ry - om * (ps->rt - a * rv) + bt * (ps->rs - om * ps->rz);
    if (!isfinite(bt) || !isfinite(sig)) {
        set_breakdown(st, RS_NONFINITE);
        return;
    }
    if (sig == 0.0) {
        set_breakdown(st, RS_RS_ZERO);
        return;
    }
    const double an = rho_new / sig;
    if (!isfinite(an)) {
        set_breakdown(st, RS_NONFINITE);
        return;
    }
    st->beta = bt;
    st->sigma = sig;
    st->rho = rho_new;
    ps->alpha_next = an;
}

// The iteration's kernels idle once the solve has stopped, and while a
// candidate stop waits for the next replacement; the replacement's only once
// it has stopped.
__device__ __forceinline__ bool pipe_idle(const State* st, const PipeScalars* ps) { return st->done || ps->verify; }

template <int ND, int KIND>
__global__ __launch_bounds__(kThreads) void kp_finish(Red red, int nblocks, State* st, PipeScalars* ps) {
    if ((KIND == PF_K1 || KIND == PF_K2) ? pipe_idle(st, ps) : st->done != 0) return;
    double tot[ND];
    if (finish_split<ND>(red, nblocks, tot) && threadIdx.x == 0) {
        if constexpr (KIND == PF_W0) tail_w0(st, ps, reinterpret_cast<double(&)[1]>(tot));
        else if constexpr (KIND == PF_K1) tail_k1(ps, reinterpret_cast<double(&)[4]>(tot));
        else if constexpr (KIND == PF_RR) tail_rr(st, ps, reinterpret_cast<double(&)[5]>(tot));
        else tail_k2(st, ps, reinterpret_cast<double(&)[6]>(tot));
    }
}

template <int ND, int KIND>
static void pipe_finish(const SysView<float>& S, const PipeView& P, hipStream_t s) {
    if (red_split(S.cell_blocks))
        hipLaunchKernelGGL((kp_finish<ND, KIND>), dim3(red_groups(S.cell_blocks)), dim3(kThreads), 0, s, S.red,
                           S.cell_blocks, S.st, P.ps);
}

// s, z, v and the pipelined scalars start at zero (with beta = 0 the first
// iteration then reads only r, w and t).
__global__ __launch_bounds__(kThreads) void kp_zero(float* s, float* z, float* v, PipeScalars* ps, int n) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *ps = PipeScalars{};
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        s[i] = 0.0f;
        z[i] = 0.0f;
        v[i] = 0.0f;
    }
}

// u = A in at one cell with the working copies (unit diagonal if UNIT).
template <bool UNIT>
__device__ __forceinline__ float pipe_apply(const SysView<float>& S, const float* in, const Cell& c) {
    const Nbr<float> v = load_nbr(in, c);
    const Coefs<float, UNIT> k = load_coefs_nt<float, UNIT>(S.c, c.idx);
    return apply7<float, float, UNIT, false>(k, v, c);
}

// w_0 = A r_0 and (r0, w_0).
template <bool UNIT>
__global__ __launch_bounds__(kThreads) void kp_w0(SysView<float> S, PipeView P) {
    if (S.st->done) return;
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, S.m, S.n);
    const float w = pipe_apply<UNIT>(S, S.r, c);
    if (c.own) P.w[c.idx] = w;
    double acc[1] = {c.own ? (double)S.rhat[c.idx] * (double)w : 0.0};
    double tot[1];
    if (grid_reduce<1>(acc, S.red, S.cell_blocks, blockIdx.x, tot) && threadIdx.x == 0) tail_w0(S.st, P.ps, tot);
}

__global__ __launch_bounds__(kThreads) void kp_k1(SysView<float> S, PipeView P) {
    if (pipe_idle(S.st, P.ps)) return;
    const float a = (float)S.st->alpha, bt = (float)S.st->beta, om = (float)S.st->omega;
    const int i = blockIdx.x * kThreads + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < S.n) {
        const float r = S.r[i], w = P.w[i], t = P.t[i];
        const float p = __builtin_fmaf(bt, __builtin_fmaf(-om, S.s[i], S.p[i]), r);
        const float s = __builtin_fmaf(bt, __builtin_fmaf(-om, P.z[i], S.s[i]), w);
        const float z = __builtin_fmaf(bt, __builtin_fmaf(-om, P.v[i], P.z[i]), t);
        const float q = __builtin_fmaf(-a, s, r);
        const float y = __builtin_fmaf(-a, z, w);
        S.p[i] = p;
        S.s[i] = s;
        P.z[i] = z;
        S.q[i] = q;
        S.y[i] = y;
        const double h = (double)S.rhat[i];
        acc[0] = h * (double)y;
        acc[1] = h * (double)t;
        acc[2] = h * (double)s;
        acc[3] = h * (double)z;
    }
    double tot[4];
    if (grid_reduce<4>(acc, S.red, S.cell_blocks, blockIdx.x, tot) && threadIdx.x == 0) tail_k1(P.ps, tot);
}

template <bool UNIT>
__global__ __launch_bounds__(kThreads) void kp_k2(SysView<float> S, PipeView P) {
    if (pipe_idle(S.st, P.ps)) return;
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, S.m, S.n);
    const float v = pipe_apply<UNIT>(S, P.z, c);
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (c.own) {
        P.v[c.idx] = v;
        const double r = S.r[c.idx], q = S.q[c.idx], y = S.y[c.idx], h = S.rhat[c.idx];
        acc[0] = r * r;
        acc[1] = q * y;
        acc[2] = y * y;
        acc[3] = q * q;
        acc[4] = h * q;
        acc[5] = h * (double)v;
    }
    double tot[6];
    if (grid_reduce<6>(acc, S.red, S.cell_blocks, blockIdx.x, tot) && threadIdx.x == 0) tail_k2(S.st, P.ps, tot);
}

__global__ __launch_bounds__(kThreads) void kp_k3(SysView<float> S, PipeView P) {
    const int flag = P.ps->flag;
    if (flag == 0) return;
    const float a = (float)S.st->alpha, om = (float)S.st->omega;
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= S.n) return;
    if (flag == 1) {
        S.d[i] = __builtin_fmaf(a, S.p[i], S.d[i]);
        return;
    }
    const float q = S.q[i], y = S.y[i];
    S.d[i] = __builtin_fmaf(om, q, __builtin_fmaf(a, S.p[i], S.d[i]));
    S.r[i] = __builtin_fmaf(-om, y, q);
    P.w[i] = __builtin_fmaf(-om, __builtin_fmaf(-a, P.v[i], P.t[i]), y);
}

// t = A w.  One thread first moves the next alpha into place and clears the
// update flag (K3 has read both).
template <bool UNIT>
__global__ __launch_bounds__(kThreads) void kp_k4(SysView<float> S, PipeView P) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        S.st->alpha = P.ps->alpha_next;
        P.ps->flag = 0;
    }
    if (pipe_idle(S.st, P.ps)) return;
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, S.m, S.n);
    const float t = pipe_apply<UNIT>(S, P.w, c);
    if (c.own) P.t[c.idx] = t;
}

// ---------------------------------------------------------------- replacement
// x += d in FP64, d = 0.
__global__ __launch_bounds__(kThreads) void kp_fold(double* x, float* d, int n, const State* st) {
    if (st->done) return;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        x[i] = x[i] + (double)d[i];
        d[i] = 0.0f;
    }
}

// out = A in.
template <bool UNIT>
__global__ __launch_bounds__(kThreads) void kp_apply(SysView<float> S, const float* in, float* out) {
    if (S.st->done) return;
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, S.m, S.n);
    const float u = pipe_apply<UNIT>(S, in, c);
    if (c.own) out[c.idx] = u;
}

// r = fl32((b - A x) / diag) in FP64 with the caller's coefficients: the
// replaced residual of the iterated system.
__global__ __launch_bounds__(kThreads) void kp_resid(Coef7 cf, const double* b, const double* x, float* r,
                                                     Mesh m, int n, const State* st, int jacobi) {
    if (st->done) return;
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, m, n);
    const Nbr<double> xv = load_nbr(x, c);
    const Coefs<float, false> k = load_coefs_nt<float, false>(cf.c, c.idx);
    const double r0 = ld_nt(b + c.idx) - apply7<double, float, false, true>(k, xv, c);
    if (c.own) r[c.idx] = (float)(jacobi ? r0 / (double)k.a[0] : r0);
}

// (r0, r), (r0, w), (r0, s), (r0, z) and (r, r) of the replaced vectors.
__global__ __launch_bounds__(kThreads) void kp_rr(SysView<float> S, PipeView P) {
    if (S.st->done) return;
    const int i = blockIdx.x * kThreads + threadIdx.x;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < S.n) {
        const double h = (double)S.rhat[i], r = (double)S.r[i];
        acc[0] = h * r;
        acc[1] = h * (double)P.w[i];
        acc[2] = h * (double)S.s[i];
        acc[3] = h * (double)P.z[i];
        acc[4] = r * r;
    }
    double tot[5];
    if (grid_reduce<5>(acc, S.red, S.cell_blocks, blockIdx.x, tot) && threadIdx.x == 0) tail_rr(S.st, P.ps, tot);
}

// ---------------------------------------------------------------- driver
static size_t pipe_bytes(const Layout& Lo) {
    return align256(Lo.bytes) + 4 * align256(Lo.n * sizeof(float)) + align256(sizeof(PipeScalars));
}

static PipeView make_pipe_view(const Layout& Lo, char* ws) {
    const size_t base = align256(Lo.bytes), span = align256(Lo.n * sizeof(float));
    PipeView P;
    P.z = reinterpret_cast<float*>(ws + base);
    P.w = reinterpret_cast<float*>(ws + base + span);
    P.t = reinterpret_cast<float*>(ws + base + 2 * span);
    P.v = reinterpret_cast<float*>(ws + base + 3 * span);
    P.ps = reinterpret_cast<PipeScalars*>(ws + base + 4 * span);
    return P;
}

static void pipe_iteration(const SysView<float>& S, const PipeView& P, hipStream_t s) {
    const int nb = S.cell_blocks;
    hipLaunchKernelGGL(kp_k1, dim3(nb), dim3(kThreads), 0, s, S, P);
    pipe_finish<4, PF_K1>(S, P, s);
    if (S.unit) hipLaunchKernelGGL(kp_k2<true>, dim3(nb), dim3(kThreads), 0, s, S, P);
    else hipLaunchKernelGGL(kp_k2<false>, dim3(nb), dim3(kThreads), 0, s, S, P);
    pipe_finish<6, PF_K2>(S, P, s);
    hipLaunchKernelGGL(kp_k3, dim3(nb), dim3(kThreads), 0, s, S, P);
    if (S.unit) hipLaunchKernelGGL(kp_k4<true>, dim3(nb), dim3(kThreads), 0, s, S, P);
    else hipLaunchKernelGGL(kp_k4<false>, dim3(nb), dim3(kThreads), 0, s, S, P);
}

template <bool UNIT>
static void pipe_apply_launch(const SysView<float>& S, const float* in, float* out, hipStream_t s) {
    hipLaunchKernelGGL(kp_apply<UNIT>, dim3(S.cell_blocks), dim3(kThreads), 0, s, S, in, out);
}

// The replacement step (its kernels do nothing once the solve has stopped).
static void pipe_replace(const SysView<float>& S, const PipeView& P, const Coef7& cf, const double* b, double* x,
                         int jacobi, hipStream_t s) {
    hipLaunchKernelGGL(kp_fold, dim3(S.stream_blocks), dim3(kThreads), 0, s, x, S.d, S.n, S.st);
    hipLaunchKernelGGL(kp_resid, dim3(S.cell_blocks), dim3(kThreads), 0, s, cf, b, (const double*)x, S.r, S.m, S.n,
                       (const State*)S.st, jacobi);
    auto ap = S.unit ? pipe_apply_launch<true> : pipe_apply_launch<false>;
    ap(S, S.r, P.w, s);
    ap(S, P.w, P.t, s);
    ap(S, S.p, S.s, s);
    ap(S, S.s, P.z, s);
    ap(S, P.z, P.v, s);
    hipLaunchKernelGGL(kp_rr, dim3(S.cell_blocks), dim3(kThreads), 0, s, S, P);
    pipe_finish<5, PF_RR>(S, P, s);
}

static int solve_pipelined(s7_dims d, const Coef7& cf, const double* b, double* x, double rtol, int max_iter,
                           char* ws, const Layout& Lo, const s7_options& o, s7_info* info, hipStream_t s) {
    SysView<float> S = make_view<float>(d, Lo, o.jacobi, ws);
    const PipeView P = make_pipe_view(Lo, ws);
    int rc = start_solve<float>(cf, S, Lo, o.jacobi, s);
    if (rc) return rc;
    auto t0 = std::chrono::steady_clock::now();
    hipLaunchKernelGGL(kp_zero, dim3(grid_for(S.n)), dim3(kThreads), 0, s, S.s, P.z, P.v, P.ps, S.n);
    hipLaunchKernelGGL(k_init_f32, dim3(S.cell_blocks), dim3(kThreads), 0, s, cf, b, x, S, o.jacobi, rtol,
                       max_iter);
    launch_finish<3, 0u, FIN_INIT>(S.red, S.cell_blocks, S.st, s, rtol, max_iter);
    if (S.unit) hipLaunchKernelGGL(kp_w0<true>, dim3(S.cell_blocks), dim3(kThreads), 0, s, S, P);
    else hipLaunchKernelGGL(kp_w0<false>, dim3(S.cell_blocks), dim3(kThreads), 0, s, S, P);
    pipe_finish<1, PF_W0>(S, P, s);
    if (S.unit) hipLaunchKernelGGL(kp_k4<true>, dim3(S.cell_blocks), dim3(kThreads), 0, s, S, P);
    else hipLaunchKernelGGL(kp_k4<false>, dim3(S.cell_blocks), dim3(kThreads), 0, s, S, P);
    S7_CHECK_LAUNCH();
    State h;
    if ((rc = read_state(S.st, &h, s))) return rc;
    if (!h.done) {
        // a graph replays G groups of kReplace iterations and one replacement
        const int G = std::max(1, (o.graph_iters > 0 ? o.graph_iters : auto_graph_iters((size_t)S.n, 4)) / kReplace);
        const int K = G * kReplace;
        const long long max_launches = (long long)h.max_iter / K + 3;
        std::vector<uintptr_t> key = {0x71u, (uintptr_t)K, (uintptr_t)S.m.nx, (uintptr_t)S.m.ny, (uintptr_t)S.m.nz,
                                      (uintptr_t)S.unit, (uintptr_t)S.st, (uintptr_t)S.red.part, (uintptr_t)S.r,
                                      (uintptr_t)S.c[1], (uintptr_t)P.z, (uintptr_t)x, (uintptr_t)b};
        for (int a = 0; a < 7; ++a) key.push_back((uintptr_t)cf.c[a]);
        GraphRef g;
        rc = cached_graph(key, [&](hipStream_t cs) {
            for (int k = 0; k < G; ++k) {
                for (int j = 0; j < kReplace; ++j) pipe_iteration(S, P, cs);
                pipe_replace(S, P, cf, b, x, o.jacobi, cs);
            }
        }, &g);
        if (rc) return rc;
        for (long long l = 0; l < max_launches && !h.done; ++l) {
            S7_HIP(hipGraphLaunch(g->exec, s));
            if ((rc = read_state(S.st, &h, s))) return rc;
        }
        if (!h.done) {
            set_error("iteration driver did not reach a final state");
            return S7_EHIP;
        }
    }
    hipLaunchKernelGGL(k_update_x, dim3(S.stream_blocks), dim3(kThreads), 0, s, x, S.d, S.n, 1.0, S.st);
    S7_CHECK_LAUNCH();
    rc = resid_launch<float>(cf, b, x, nullptr, S, o.jacobi, s);
    if (rc) return rc;
    if ((rc = read_state(S.st, &h, s))) return rc;
    auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->status = h.status;
        info->reason = h.reason;
        info->rel_res_rec = h.res_rec;
        info->iters = h.iter;
        info->outer_iters = 1;
        info->schedule = 4;
        info->rel_res_true = h.bb_true > 0 ? sqrt(h.rr_true / h.bb_true) : 0.0;
        info->t_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    return h.status;
}

}  // namespace s7

extern "C" {

size_t s7_workspace_bytes_pipelined(s7_dims d, const s7_options* opt) {
    if (!dims_ok(d)) return 0;
    s7_options o;
    options_or_default(opt, o);
    return pipe_bytes(make_layout(d, S7_FP32, o));
}

int s7_bicgstab_solve_pipelined(s7_dims d, const float* const coef[7], const double* b, double* x, double rtol,
                                int32_t max_iter, void* ws, size_t ws_bytes, const s7_options* opt, s7_info* info,
                                void* stream) {
    clear_error();
    if (info) std::memset(info, 0, sizeof(*info));
    s7_options o;
    options_or_default(opt, o);
    if (!dims_ok(d) || !coef_ok(coef) || !b || !x || !ws || !(rtol > 0.0) || max_iter < 0 ||
        ((uintptr_t)ws & 255u) != 0) {
        set_error("s7_bicgstab_solve_pipelined: invalid argument");
        return S7_EINVAL;
    }
    const Layout Lo = make_layout(d, S7_FP32, o);
    const size_t need = pipe_bytes(Lo);
    if (ws_bytes < need) {
        set_error("s7_bicgstab_solve_pipelined: workspace too small (%zu < %zu)", ws_bytes, need);
        return S7_EINVAL;
    }
    Coef7 cf;
    for (int a = 0; a < 7; ++a) cf.c[a] = coef[a];
    return solve_pipelined(d, cf, b, x, rtol, max_iter, (char*)ws, Lo, o, info, (hipStream_t)stream);
}

}  // extern "C"
