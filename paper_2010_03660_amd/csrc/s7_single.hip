// Single-system path of the s7 library: stencil apply, the generator, and the
// BiCGStab solve (FP32, and BF16/FP16 inside FP64 iterative refinement).
//
// Per iteration, Algorithm 1 runs as three passes.  Each ends in a device-side
// scalar step:
//   P1  s_i = A p_i; partial (r0, s_i)                               -> alpha_i
//   P2a q_i = r_i - alpha s_i (streaming)
//   P2b y_i = A q_i; partials (q,y), (y,y), (q,q), (r0,q), (r0,y) -> omega_i, beta_i, half-step test
//   P3  x += alpha p + omega q; r_{i+1} = q - omega y;
//       p_{i+1} = r_{i+1} + beta (p_i - omega s_i); partials (r0,r), (r,r) -> stopping tests
// P1 and P2b are cell-parallel stencils; P2a and P3 stream.  The scalars stay on the
// device.  The host reads only the `done` word, once per captured graph of K
// iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "s7_host.hpp"
#include "s7_batched_kernels.hpp"
#include "s7_passes.hpp"

namespace s7 {

// ============================================================== error state
static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}
void clear_error() { g_err.clear(); }

void options_or_default(const s7_options* in, s7_options& out) {
    if (in) {
        out = *in;
    } else {
        s7_default_options(&out);
    }
}

Layout make_layout(s7_dims d, int prec, const s7_options& o, int ncoef) {
    Layout L;
    L.n = (size_t)d.nx * d.ny * d.nz;
    L.elt = elt_size(prec);
    L.ncoef = ncoef > 0 ? ncoef : (o.jacobi ? 6 : 7);
    L.cell_blocks = cell_blocks_for((long long)L.n);
    L.stream_blocks = stream_blocks_for((long long)L.n, o.stream_blocks);
    // partials for any streaming split up to kSingleMax, so the workspace size
    // does not depend on the (tunable) split
    const int nb = L.cell_blocks > kSingleMax ? L.cell_blocks : kSingleMax;
    L.groups = red_groups(nb);  // workgroups of the finishing kernel of a split sum
    size_t off = 0;
    L.off_state = off;
    off = align256(off + sizeof(State));
    L.off_part = off;
    off = align256(off + (size_t)nb * kMaxDots * sizeof(double));
    L.off_gpart = off;
    off = align256(off + (size_t)L.groups * kMaxDots * sizeof(double));
    L.off_cnt = off;
    off = align256(off + sizeof(uint32_t));
    L.off_ctl = off;
    off = align256(off + sizeof(BCtl));
    L.off_coef = off;
    off = align256(off + (size_t)L.ncoef * align256(L.n * L.elt));
    L.off_vec = off;
    off = align256(off + (size_t)6 * align256(L.n * L.elt));
    L.off_d = off;
    off = align256(off + L.n * sizeof(float));
    L.bytes = off;
    return L;
}

template <class T>
static SysView<T> make_view(s7_dims d, const Layout& L, int jacobi, char* ws) {
    SysView<T> S;
    S.m = make_mesh(d.nx, d.ny, d.nz);
    S.n = (int)L.n;
    S.unit = jacobi ? 1 : 0;
    const size_t span = align256(L.n * L.elt);
    const int first = jacobi ? 1 : 0;
    for (int a = 0; a < 7; ++a)
        S.c[a] = a < first ? nullptr : reinterpret_cast<const T*>(ws + L.off_coef + (a - first) * span);
    auto vec = [&](int i) { return reinterpret_cast<T*>(ws + L.off_vec + i * span); };
    S.r = vec(0);
    S.rhat = vec(1);
    S.p = vec(2);
    S.s = vec(3);
    S.y = vec(4);
    S.q = vec(5);
    S.d = reinterpret_cast<float*>(ws + L.off_d);
    S.st = reinterpret_cast<State*>(ws + L.off_state);
    S.red = Red{reinterpret_cast<double*>(ws + L.off_part), reinterpret_cast<double*>(ws + L.off_gpart),
                reinterpret_cast<uint32_t*>(ws + L.off_cnt)};
    S.cell_blocks = L.cell_blocks;
    S.stream_blocks = L.stream_blocks;
    S.pair_blocks = d.nx % 2 == 0 ? (int)((L.n + 2 * kThreads - 1) / (2 * kThreads)) : 0;
    return S;
}

// ============================================================== kernels

// Clears the solver state and the reduction counters (a kernel rather than a
// memset, so that the same clear is valid inside captured graphs).
__global__ __launch_bounds__(kThreads) void k_zero_state(State* st, uint32_t* cnt, int ncnt) {
    uint32_t* w = reinterpret_cast<uint32_t*>(st);
    for (int i = threadIdx.x; i < (int)(sizeof(State) / 4); i += kThreads) w[i] = 0u;
    for (int i = threadIdx.x; i < ncnt; i += kThreads) cnt[i] = 0u;
}

// Working-precision coefficient copies.  jacobi: c[a] / diag for a = 1..6 (unit
// diagonal).  Otherwise all seven.  Outward links on the boundary faces are
// zeroed, so the iteration never needs face tests.
template <class T>
__global__ __launch_bounds__(kThreads) void k_prep_coef(Coef7 src, T* dst0, size_t span_elems,
                                                        Mesh m, int jacobi) {
    const int first = jacobi ? 1 : 0;
    const int n = m.nx * m.ny * m.nz;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        const Cell c = cell_at(i, m, n);
        const bool in[7] = {true, c.dw != 0, c.de != 0, c.ds != 0, c.dn != 0, c.db != 0, c.dt != 0};
        const float dg = src.c[0][i];
#pragma unroll
        for (int a = 0; a < 7; ++a) {
            if (a < first) continue;
            float v = in[a] ? src.c[a][i] : 0.0f;
            if (jacobi) v = v / dg;
            dst0[(size_t)(a - first) * span_elems + i] = from_f32<T>(v);
        }
    }
}

// r0 = b - A x0 in FP64 with the caller's FP32 coefficients.  Optionally
// Jacobi-scaled.  Rounded to FP32 into r, r_hat and p, and d = 0.  Partials:
// ||b_s||^2, (r,r) of the rounded r, ||b||^2 unscaled.
__global__ __launch_bounds__(kThreads) void k_init_f32(Coef7 cf, const double* b, const double* x0,
                                                       SysView<float> S, int jacobi, double tol,
                                                       int max_iter) {
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, S.m, S.n);
    const Nbr<double> xv = load_nbr(x0, c);
    const Coefs<float, false> k = load_coefs_nt<float, false>(cf.c, c.idx);
    const double bi = ld_nt(b + c.idx);
    const double ax = apply7<double, float, false, true>(k, xv, c);
    double r0 = bi - ax, bs = bi;
    if (jacobi) {
        const double dg = (double)k.a[0];
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
    double acc[3] = {c.own ? bs * bs : 0.0, c.own ? (double)rf * (double)rf : 0.0,
                     c.own ? bi * bi : 0.0};
    double tot[3];
    if (grid_reduce<3>(acc, S.red, S.cell_blocks, blockIdx.x, tot) && threadIdx.x == 0) {
        tail_init(S.st, tot[0], tot[1], tol, max_iter);
        S.st->bb_true = tot[2];
        S.st->scale = 1.0;
    }
}

// True residual r = b - A x in FP64 (caller's coefficients, unscaled).
// Partials: ||b||^2, ||r||^2, max |r_s| (r_s = r / diag with Jacobi).  If dst is
// not null, r_s goes there as FP32: the right-hand side of the next refinement
// step.
__global__ __launch_bounds__(kThreads) void k_resid(Coef7 cf, const double* b, const double* x,
                                                    float* dst, Mesh m, int n, int nblocks,
                                                    State* st, Red red, int jacobi) {
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, m, n);
    const Nbr<double> xv = load_nbr(x, c);
    const Coefs<float, false> k = load_coefs_nt<float, false>(cf.c, c.idx);
    const double bi = ld_nt(b + c.idx);
    const double r0 = bi - apply7<double, float, false, true>(k, xv, c);
    const double rs = jacobi ? r0 / (double)k.a[0] : r0;
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

// Start of an inner solve of the refinement: r = r_hat = p = fl_T(rs / scale)
// from the FP32 residual in d, then d = 0.
template <class T>
__global__ __launch_bounds__(kThreads) void k_ir_init(SysView<T> S, float inv_scale, double tol,
                                                      int max_iter) {
    double acc[1] = {0.0};
    const int step = S.stream_blocks * kThreads;
    // kVec<T> cells per thread and step with 16-byte accesses, then the tail
    constexpr int W = kVec<T>;
    const int nv = S.n / W;
    const float zero[W] = {};
    for (int v = (int)(blockIdx.x * kThreads + threadIdx.x); v < nv; v += step) {
        const int i = W * v;
        float dv[W];
        ldw_nt<W>(S.d + i, dv);
        T rt[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            rt[j] = from_f32<T>(dv[j] * inv_scale);
            const double x = (double)to_f32(rt[j]);
            acc[0] = fma(x, x, acc[0]);
        }
        stw_nt<W>(S.r + i, rt);
        stw_nt<W>(S.rhat + i, rt);
        stw_nt<W>(S.p + i, rt);
        stw_nt<W>(S.d + i, zero);
    }
    for (int i = W * nv + (int)(blockIdx.x * kThreads + threadIdx.x); i < S.n; i += step) {
        const T rt = from_f32<T>(S.d[i] * inv_scale);
        S.r[i] = rt;
        S.rhat[i] = rt;
        S.p[i] = rt;
        S.d[i] = 0.0f;
        const double v = (double)to_f32(rt);
        acc[0] = fma(v, v, acc[0]);
    }
    double tot[1];
    if (grid_reduce<1>(acc, S.red, S.stream_blocks, blockIdx.x, tot) && threadIdx.x == 0)
        tail_init(S.st, tot[0], tot[0], tol, max_iter);
}

// x += scale * d (FP64), or x = 0 when b = 0.
// x += scale d in FP64 (x = 0 when b was zero).  Four cells per thread and
// step with 16-byte accesses when x is 16-byte aligned (d, in the workspace,
// always is); the caller's x may be only 8-byte aligned, which takes the
// scalar loop.
typedef double f64x2 __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(kThreads) void k_update_x(double* x, const float* d, int n,
                                                       double scale, const State* st) {
    const bool zero = st->nbzero != 0;
    const int step = (int)gridDim.x * kThreads;
    int head = 0;
    if ((reinterpret_cast<uintptr_t>(x) & 15u) == 0) {
        const int nv = n / 4;
        for (int v = (int)(blockIdx.x * kThreads + threadIdx.x); v < nv; v += step) {
            const int i = 4 * v;
            float dv[4];
            ld4_nt(d + i, dv);
            f64x2* px = reinterpret_cast<f64x2*>(x + i);
            f64x2 a = __builtin_nontemporal_load(px), b = __builtin_nontemporal_load(px + 1);
            a.x = zero ? 0.0 : fma(scale, (double)dv[0], a.x);
            a.y = zero ? 0.0 : fma(scale, (double)dv[1], a.y);
            b.x = zero ? 0.0 : fma(scale, (double)dv[2], b.x);
            b.y = zero ? 0.0 : fma(scale, (double)dv[3], b.y);
            __builtin_nontemporal_store(a, px);
            __builtin_nontemporal_store(b, px + 1);
        }
        head = 4 * nv;
    }
    for (int i = head + (int)(blockIdx.x * kThreads + threadIdx.x); i < n; i += step)
        x[i] = zero ? 0.0 : fma(scale, (double)d[i], x[i]);
}

__global__ __launch_bounds__(kThreads) void k_fill0(double* x, int n) {
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) x[i] = 0.0;
}

__global__ __launch_bounds__(kThreads) void k_stencil_apply(Coef7 cf, const float* v, float* u,
                                                            Mesh m, int n) {
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, m, n);
    const Nbr<float> vv = load_nbr(v, c);
    const Coefs<float, false> k = load_coefs<float, false>(cf.c, c.idx);
    const float av = apply7<float, float, false, true>(k, vv, c);
    if (c.own) u[c.idx] = av;
}

// u = A v on x-adjacent cell pairs, v staged in LDS: a tile of TILE cells and
// one row either side, as in the solver's staged passes; below and above come
// from memory.  The caller's coefficients are used as given, so a neighbour
// across a mesh face has both its coefficient and its value set to zero (the
// staged neighbour there is another cell of the mesh): every cell's sum is the
// flat kernel's, term by term, for finite v.
template <int TILE>
__global__ __launch_bounds__(kThreads) void k_apply_lds(Coef7 cf, const float* v, float* u, Mesh m, int n,
                                                        int nblocks, int run) {
    extern __shared__ float stage[];
    const int tile = xcd_tile(blockIdx.x, nblocks, run);
    const int nx = m.nx, c0 = tile * TILE, lo = lds_lo(c0, nx);
    const int hi = (c0 + TILE + nx + 7) >> 3 << 3;
    stage_rows<float, false>(v, nullptr, 0.0f, lo, hi - lo, n, stage);
    __syncthreads();
    const int plane = nx * m.ny;
#pragma unroll 2
    for (int q = 0; q < TILE / (2 * kThreads); ++q) {
        const int idx = c0 + 2 * (q * kThreads + (int)threadIdx.x);
        if (idx >= n) break;
        const int k = div_rcp(idx, plane, m.rplane);
        const int rem = idx - k * plane;
        const int j = div_rcp(rem, nx, m.rnx);
        const int i = rem - j * nx;
        Cell f0{}, f1{};  // the faces each cell of the pair touches (nonzero: inside)
        f0.dw = i > 0 ? -1 : 0;
        f0.de = 1;
        f1.dw = -1;
        f1.de = i + 1 < nx - 1 ? 1 : 0;
        f0.ds = f1.ds = j > 0 ? -nx : 0;
        f0.dn = f1.dn = j < m.ny - 1 ? nx : 0;
        f0.db = f1.db = k > 0 ? -plane : 0;
        f0.dt = f1.dt = k < m.nz - 1 ? plane : 0;
        const F2 vb = ld2(v + idx + f0.db), vt = ld2(v + idx + f0.dt);
        Nbr<float> v0, v1;
        lds_nbr2(stage, idx - lo, nx, vb, vt, v0, v1);
        v0.w = f0.dw ? v0.w : 0.0f;
        v1.e = f1.de ? v1.e : 0.0f;
        v0.s = f0.ds ? v0.s : 0.0f;
        v1.s = f0.ds ? v1.s : 0.0f;
        v0.n = f0.dn ? v0.n : 0.0f;
        v1.n = f0.dn ? v1.n : 0.0f;
        v0.b = f0.db ? v0.b : 0.0f;
        v1.b = f0.db ? v1.b : 0.0f;
        v0.t = f0.dt ? v0.t : 0.0f;
        v1.t = f0.dt ? v1.t : 0.0f;
        Coefs<float, false> k0, k1;
        load_coefs2_nt<float, false>(cf.c, idx, k0, k1);
        const float a0 = apply7<float, float, false, true>(k0, v0, f0);
        const float a1 = apply7<float, float, false, true>(k1, v1, f1);
        st2_nt(u + idx, a0, a1);
    }
}

__global__ __launch_bounds__(kThreads) void k_apply_f64(Coef7 cf, const double* v, double* u,
                                                        Mesh m, int n) {
    const Cell c = cell_at(blockIdx.x * kThreads + threadIdx.x, m, n);
    const Nbr<double> vv = load_nbr(v, c);
    const Coefs<float, false> k = load_coefs<float, false>(cf.c, c.idx);
    const double av = apply7<double, float, false, true>(k, vv, c);
    if (c.own) u[c.idx] = av;
}

// ---- generator (recipe of the synthetic inputs; see s7.h)
__device__ __forceinline__ uint64_t gen_hash(uint64_t seed, int aid, uint64_t cell) {
    const uint64_t key = splitmix64(seed ^ ((uint64_t)aid << 56));
    return splitmix64(key ^ cell);
}

__device__ __forceinline__ double smooth01(double t) {
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    return __dmul_rn(__dmul_rn(t, t), __dsub_rn(3.0, __dmul_rn(2.0, t)));
}

__global__ __launch_bounds__(kThreads) void k_gen_coef(Coef7 out, double* xstar, Mesh m,
                                                       uint64_t seed, int recipe) {
    const int n = m.nx * m.ny * m.nz;
    float* c[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) c[a] = const_cast<float*>(out.c[a]);
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        const int k = i / (m.nx * m.ny);
        double f = 1.0;
        if (recipe == 1) {
            const double lo = (double)(m.nz / 4), hi = (double)((3 * m.nz) / 4), w = 4.0;
            const double kd = (double)k;
            const double s = __dmul_rn(smooth01(__ddiv_rn(__dsub_rn(kd, __dsub_rn(lo, w)), w)),
                                       smooth01(__ddiv_rn(__dsub_rn(__dadd_rn(__dsub_rn(hi, 1.0), w), kd), w)));
            f = __dadd_rn(1.0, __dmul_rn(9.0, s));
        }
        double sum = 0.0;
        float off[6];
#pragma unroll
        for (int a = 1; a <= 6; ++a) {
            const uint64_t h = gen_hash(seed, a, (uint64_t)i);
            const double mm = (double)(h >> 41);
            float v = (float)(-(__dadd_rn(0.5, __dmul_rn(mm, 0x1p-24))));
            if (recipe == 1 && a >= 5) v = (float)__dmul_rn((double)v, f);
            off[a - 1] = v;
            sum = __dadd_rn(sum, fabs((double)v));
        }
        const float dg = (float)__dadd_rn(sum, 0.1);
        if (c[0]) c[0][i] = dg;
#pragma unroll
        for (int a = 1; a <= 6; ++a)
            if (c[a]) c[a][i] = off[a - 1];
        if (xstar) {
            const uint64_t h = gen_hash(seed, 7, (uint64_t)i);
            xstar[i] = __dadd_rn(-1.0, __dmul_rn((double)(h >> 40), 0x1p-23));
        }
    }
}

// ============================================================== graph cache
namespace {

// An instantiated graph.  Holders keep it alive: a graph evicted from the
// cache while another thread still launches it is destroyed with its last user.
struct GraphExec {
    hipGraphExec_t exec = nullptr;
    ~GraphExec() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};
using GraphRef = std::shared_ptr<GraphExec>;

struct GraphEntry {
    std::vector<uintptr_t> key;
    GraphRef g;
};

std::mutex g_graph_mu;
std::list<GraphEntry> g_graphs;
constexpr size_t kMaxGraphs = 32;
hipStream_t g_capture_stream[16] = {};

int capture_stream(hipStream_t* out) {
    int dev = 0;
    S7_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 16) {
        set_error("device index %d out of range", dev);
        return S7_EINVAL;
    }
    if (!g_capture_stream[dev]) S7_HIP(hipStreamCreateWithFlags(&g_capture_stream[dev], hipStreamNonBlocking));
    *out = g_capture_stream[dev];
    return S7_OK;
}

}  // namespace

// Returns a cached executable graph for `key` on the current device,
// capturing `body` on first use.  The caller keeps *out until its launches
// have completed.
template <class F>
int cached_graph(std::vector<uintptr_t> key, F body, GraphRef* out) {
    int dev = 0;
    S7_HIP(hipGetDevice(&dev));
    key.push_back((uintptr_t)dev);
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it) {
        if (it->key == key) {
            g_graphs.splice(g_graphs.begin(), g_graphs, it);
            *out = g_graphs.front().g;
            return S7_OK;
        }
    }
    hipStream_t cs;
    int rc = capture_stream(&cs);
    if (rc) return rc;
    hipGraph_t graph;
    S7_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    body(cs);
    hipError_t le = hipGetLastError();
    hipError_t ce = hipStreamEndCapture(cs, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
        set_error("graph capture failed: %s / %s", hipGetErrorString(le), hipGetErrorString(ce));
        return S7_EHIP;
    }
    hipGraphExec_t exec;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
        set_error("hipGraphInstantiate failed: %s", hipGetErrorString(ie));
        return S7_EHIP;
    }
    GraphRef ref = std::make_shared<GraphExec>();
    ref->exec = exec;
    if (g_graphs.size() >= kMaxGraphs) g_graphs.pop_back();
    g_graphs.push_front(GraphEntry{key, ref});
    *out = ref;
    return S7_OK;
}

// ============================================================== drivers
static int auto_graph_iters(size_t n, int elt) {
    const double us = (double)n * (elt == 4 ? 112.0 : 60.0) / 5.0e6 + 15.0;
    int k = (int)(2000.0 / us);
    if (k < 2) k = 2;
    if (k > 64) k = 64;
    return k;
}

template <int ND, unsigned MAXMASK, int KIND>
static void launch_finish(const Red& red, int nblocks, State* st, hipStream_t s, double tol = 0.0,
                          int max_iter = 0) {
    if (red_split(nblocks))
        hipLaunchKernelGGL((k_finish<ND, MAXMASK, KIND>), dim3(red_groups(nblocks)), dim3(kThreads),
                           0, s, red, nblocks, st, tol, max_iter);
}

// The launches of one iteration: 0 P1, 1 P2a, 2 P2b, 3 P3 (each with the
// finishing kernel of a split sum where one is needed).  The three-pass
// schedule has no P2a: its pass 2 forms q on the fly, and its P3 forms q again.
constexpr int kPasses = 4;
enum Schedule { SCHED_AUTO = 0, SCHED_THREE = 1, SCHED_FOUR = 2, SCHED_PAIRS = 3, SCHED_LDS = 5 };

// Tiles per XCD run of a stencil pass (xcd_tile): the option if above 1, an
// eighth of a plane's tiles for -1, else plain order.  Measured at
// 600x595x1536 and 256^3, runs of 44, 87 (an eighth of a plane) and 174 tiles
// left the paired passes' times within 2 % of plain order, so plain order is
// the default.
static int tile_run(int xcd_run, const Mesh& m, int tile_cells) {
    if (xcd_run > 1) return xcd_run;
    if (xcd_run != -1) return 1;
    const long long r = (long long)m.nx * m.ny / (8LL * tile_cells);
    return r < 1 ? 1 : (r > (1 << 20) ? (1 << 20) : (int)r);
}

// The staged passes' tile for this mesh: the requested one (2048, 4096 or 8192
// cells) if its LDS fits, else the largest of 4096 and 2048 that fits; 0 when
// the staged passes do not apply (odd nx, or rows too long for the LDS).
static int lds_tile_for(int requested, int nx, bool even) {
    if (!even) return 0;
    if ((requested == 2048 || requested == 4096 || requested == 8192) && lds_fits(nx, requested))
        return requested;
    for (int t : {kLdsTile, 2048})
        if (lds_fits(nx, t)) return t;
    return 0;
}

// The schedule of an iteration: the option if set (one that does not apply to
// the mesh falls back to cell pairs, and cell pairs to single cells when nx is
// odd); by default the staged passes on meshes of at least kLdsMinCells cells
// where they apply, else cell pairs.  Below that size the staged passes'
// workgroups are too few to fill the chip.
constexpr long long kLdsMinCells = 4LL << 20;

template <class T>
static int effective_schedule(const s7_options& o, const SysView<T>& S) {
    if (o.schedule == SCHED_THREE || o.schedule == SCHED_FOUR) return o.schedule;
    const bool staged = lds_tile_for(o.lds_tile, S.m.nx, S.pair_blocks > 0) > 0;
    if (o.schedule == SCHED_LDS && staged) return SCHED_LDS;
    if (o.schedule == SCHED_AUTO && staged && (long long)S.n >= kLdsMinCells) return SCHED_LDS;
    return S.pair_blocks > 0 ? SCHED_PAIRS : SCHED_THREE;
}

// Launch parameters of an iteration's passes: the schedule, the XCD tile order
// and the staged passes' tile.
struct PassLaunch {
    int sched, xr, tile;
};

template <class T>
static PassLaunch pass_launch(const s7_options& o, const SysView<T>& S) {
    const int sched = effective_schedule(o, S);
    return PassLaunch{sched, o.xcd_run, sched == SCHED_LDS ? lds_tile_for(o.lds_tile, S.m.nx, true) : 0};
}

template <class T, int TILE>
static void launch_staged(const SysView<T>& S, int pass, int xr, hipStream_t s) {
    const int nb = lds_blocks(S.n, TILE);
    const size_t lds = (size_t)lds_count(S.m.nx, TILE) * sizeof(float);
    const int run = tile_run(xr, S.m, TILE);
    if (pass == 0) {
        if (S.unit) hipLaunchKernelGGL((k_p1_lds<T, true, TILE>), dim3(nb), dim3(kThreads), lds, s, S, nb, run);
        else hipLaunchKernelGGL((k_p1_lds<T, false, TILE>), dim3(nb), dim3(kThreads), lds, s, S, nb, run);
        launch_finish<1, 0u, FIN_P1>(S.red, nb, S.st, s);
    } else {
        if (S.unit) hipLaunchKernelGGL((k_p2f_lds<T, true, TILE>), dim3(nb), dim3(kThreads), lds, s, S, nb, run);
        else hipLaunchKernelGGL((k_p2f_lds<T, false, TILE>), dim3(nb), dim3(kThreads), lds, s, S, nb, run);
        launch_finish<5, 0u, FIN_P2F>(S.red, nb, S.st, s);
    }
}

template <class T>
static void launch_pass(const SysView<T>& S, int pass, const PassLaunch& L, hipStream_t s) {
    const int sched = L.sched, xr = L.xr;
    // With 16-bit storage the staged P1 measured slower than the paired one (its
    // single operand is read in 4-byte pairs either way), so it keeps the pairs.
    if (sched == SCHED_LDS && L.tile > 0 && (pass == 2 || (pass == 0 && sizeof(T) == 4))) {
        if (L.tile == 2048) launch_staged<T, 2048>(S, pass, xr, s);
        else if (L.tile == 8192) launch_staged<T, 8192>(S, pass, xr, s);
        else launch_staged<T, kLdsTile>(S, pass, xr, s);
        return;
    }
    if ((sched == SCHED_PAIRS || sched == SCHED_LDS) && S.pair_blocks > 0 && pass != 3) {
        if (pass == 1) return;
        const int nb = S.pair_blocks;
        const int run = tile_run(xr, S.m, 2 * kThreads);
        if (pass == 0) {
            if (S.unit) hipLaunchKernelGGL((k_p1_pair<T, true>), dim3(nb), dim3(kThreads), 0, s, S, run);
            else hipLaunchKernelGGL((k_p1_pair<T, false>), dim3(nb), dim3(kThreads), 0, s, S, run);
            launch_finish<1, 0u, FIN_P1>(S.red, nb, S.st, s);
        } else {
            if (S.unit) hipLaunchKernelGGL((k_p2f_pair<T, true>), dim3(nb), dim3(kThreads), 0, s, S, run);
            else hipLaunchKernelGGL((k_p2f_pair<T, false>), dim3(nb), dim3(kThreads), 0, s, S, run);
            launch_finish<5, 0u, FIN_P2F>(S.red, nb, S.st, s);
        }
        return;
    }
    const int run = tile_run(xr, S.m, kThreads);
    if (sched == SCHED_THREE || sched == SCHED_PAIRS || sched == SCHED_LDS) {
        if (pass == 1) return;
        if (pass == 2) {
            if (S.unit)
                hipLaunchKernelGGL((k_p2f<T, true>), dim3(S.cell_blocks), dim3(kThreads), 0, s, S, run);
            else
                hipLaunchKernelGGL((k_p2f<T, false>), dim3(S.cell_blocks), dim3(kThreads), 0, s, S, run);
            launch_finish<5, 0u, FIN_P2F>(S.red, S.cell_blocks, S.st, s);
            return;
        }
        if (pass == 3) {
            hipLaunchKernelGGL((k_p3<T, true>), dim3(S.stream_blocks), dim3(kThreads), 0, s, S);
            return;
        }
    }
    if (pass == 0) {
        if (S.unit)
            hipLaunchKernelGGL((k_p1<T, true>), dim3(S.cell_blocks), dim3(kThreads), 0, s, S, run);
        else
            hipLaunchKernelGGL((k_p1<T, false>), dim3(S.cell_blocks), dim3(kThreads), 0, s, S, run);
        launch_finish<1, 0u, FIN_P1>(S.red, S.cell_blocks, S.st, s);
    } else if (pass == 1) {
        hipLaunchKernelGGL((k_p2a<T>), dim3(S.stream_blocks), dim3(kThreads), 0, s, S);
    } else if (pass == 2) {
        if (S.unit)
            hipLaunchKernelGGL((k_p2<T, true>), dim3(S.cell_blocks), dim3(kThreads), 0, s, S, run);
        else
            hipLaunchKernelGGL((k_p2<T, false>), dim3(S.cell_blocks), dim3(kThreads), 0, s, S, run);
        launch_finish<4, 0u, FIN_P2>(S.red, S.cell_blocks, S.st, s);
    } else {
        hipLaunchKernelGGL((k_p3<T, false>), dim3(S.stream_blocks), dim3(kThreads), 0, s, S);
    }
}

static int read_state(const State* dst, State* host, hipStream_t s) {
    S7_HIP(hipMemcpyAsync(host, dst, sizeof(State), hipMemcpyDeviceToHost, s));
    S7_HIP(hipStreamSynchronize(s));
    return S7_OK;
}

// Runs BiCGStab iterations from an initialised state until the device says done.
template <class T>
static int run_iterations(const SysView<T>& S, const s7_options& o, hipStream_t stream,
                          State* host, s7_info* info, bool direct = false) {
    int rc = read_state(S.st, host, stream);
    if (rc) return rc;
    if (host->done) return S7_OK;
    const int K = o.graph_iters > 0 ? o.graph_iters : auto_graph_iters((size_t)S.n, (int)sizeof(T));
    const long long max_launches = (long long)host->max_iter / K + 3;
    const PassLaunch PL = pass_launch(o, S);
    const int sched = PL.sched;
    if (direct) {
        // plain launches: no graph (its instantiation allocates) and no events
        for (long long l = 0; l < max_launches; ++l) {
            for (int j = 0; j < K; ++j)
                for (int p = 0; p < kPasses; ++p) launch_pass<T>(S, p, PL, stream);
            S7_CHECK_LAUNCH();
            rc = read_state(S.st, host, stream);
            if (rc) return rc;
            if (host->done) break;
        }
    } else if (o.profile) {
        constexpr int NP = kPasses;
        std::vector<hipEvent_t> ev((size_t)(NP + 1) * K);
        for (auto& e : ev) S7_HIP(hipEventCreate(&e));
        for (long long l = 0; l < max_launches; ++l) {
            const int it0 = host->iter;
            for (int j = 0; j < K; ++j) {
                for (int p = 0; p < NP; ++p) {
                    S7_HIP(hipEventRecord(ev[(NP + 1) * j + p], stream));
                    launch_pass<T>(S, p, PL, stream);
                }
                S7_HIP(hipEventRecord(ev[(NP + 1) * j + NP], stream));
            }
            S7_CHECK_LAUNCH();
            rc = read_state(S.st, host, stream);
            if (rc) return rc;
            const int ran = host->iter - it0;
            if (info) {
                for (int j = 0; j < K && j < ran; ++j) {
                    for (int p = 0; p < NP; ++p) {
                        if (sched != SCHED_FOUR && p == 1) continue;  // no P2a in this schedule
                        float ms = 0.f;
                        S7_HIP(hipEventElapsedTime(&ms, ev[(NP + 1) * j + p], ev[(NP + 1) * j + p + 1]));
                        info->pass_ms[p] += ms;
                        info->pass_count[p] += 1;
                    }
                }
            }
            if (host->done) break;
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
    } else {
        std::vector<uintptr_t> key = {0x52u, (uintptr_t)TypeTag<T>::value, (uintptr_t)K,
                                      (uintptr_t)S.m.nx, (uintptr_t)S.m.ny, (uintptr_t)S.m.nz,
                                      (uintptr_t)S.unit, (uintptr_t)S.st, (uintptr_t)S.red.part,
                                      (uintptr_t)S.r, (uintptr_t)S.c[1], (uintptr_t)S.d,
                                      (uintptr_t)S.stream_blocks, (uintptr_t)sched,
                                      (uintptr_t)(intptr_t)PL.xr, (uintptr_t)PL.tile};
        GraphRef g;
        rc = cached_graph(key, [&](hipStream_t cs) {
            for (int j = 0; j < K; ++j)
                for (int p = 0; p < kPasses; ++p) launch_pass<T>(S, p, PL, cs);
        }, &g);
        if (rc) return rc;
        for (long long l = 0; l < max_launches; ++l) {
            S7_HIP(hipGraphLaunch(g->exec, stream));
            rc = read_state(S.st, host, stream);
            if (rc) return rc;
            if (host->done) break;
        }
    }
    if (!host->done) {
        set_error("iteration driver did not reach a final state");
        return S7_EHIP;
    }
    return S7_OK;
}

static int grid_for(size_t n) {
    size_t g = (n + kThreads - 1) / kThreads;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

template <class T>
static int resid_launch(const Coef7& cf, const double* b, const double* x, float* dst,
                        const SysView<T>& S, int jacobi, hipStream_t s) {
    hipLaunchKernelGGL(k_resid, dim3(S.cell_blocks), dim3(kThreads), 0, s, cf, b, x, dst, S.m, S.n,
                       S.cell_blocks, S.st, S.red, jacobi);
    launch_finish<3, 4u, FIN_RESID>(S.red, S.cell_blocks, S.st, s);
    S7_CHECK_LAUNCH();
    return S7_OK;
}

template <class T>
static int start_solve(const Coef7& cf, const SysView<T>& S, const Layout& Lo, int jacobi,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_zero_state, dim3(1), dim3(kThreads), 0, s, S.st, S.red.cnt, 1);
    const size_t span_elems = align256(Lo.n * Lo.elt) / Lo.elt;
    hipLaunchKernelGGL((k_prep_coef<T>), dim3(grid_for(S.n)), dim3(kThreads), 0, s, cf,
                       const_cast<T*>(S.c[jacobi ? 1 : 0]), span_elems, S.m, jacobi);
    S7_CHECK_LAUNCH();
    return S7_OK;
}

// ============================================================== autotuning trials
// A trial runs iterations on synthetic contents written into the workspace:
// unit diagonal, off-diagonals -0.15 with the outward links of boundary cells
// zeroed (as for real coefficients; row sums 0.1 inside the mesh, so the
// system is well conditioned), r = r0 = p = 1.  Its State marks it as a trial
// with tolerance -1: it never converges, and if it stopped anyway (a breakdown)
// it would end there.  So the caller's arrays are never read or written.
template <class T>
__global__ __launch_bounds__(kThreads) void k_tune_fill(SysView<T> S) {
    const T one = from_f32<T>(1.0f), zero = from_f32<T>(0.0f), off = from_f32<T>(-0.15f);
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < S.n; i += gridDim.x * kThreads) {
        const Cell c = cell_at(i, S.m, S.n);
        const bool in[7] = {true, c.dw != 0, c.de != 0, c.ds != 0, c.dn != 0, c.db != 0, c.dt != 0};
        for (int a = S.unit ? 1 : 0; a < 7; ++a)
            const_cast<T*>(S.c[a])[i] = a == 0 ? one : (in[a] ? off : zero);
        S.r[i] = one;
        S.rhat[i] = one;
        S.p[i] = one;
        S.s[i] = zero;
        S.y[i] = zero;
        S.q[i] = zero;
        S.d[i] = 0.0f;
    }
}

__global__ void k_tune_state(State* st, uint32_t* cnt, int n) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    *st = State{};
    st->rho = (double)n;
    st->nb = sqrt((double)n);
    st->tol = -1.0;
    st->max_iter = 1 << 30;
    st->trial = 1;
    *cnt = 0u;
}

// Fills the workspace with a trial system and arms its State.
template <class T>
static int tune_prepare(const SysView<T>& S, hipStream_t s) {
    hipLaunchKernelGGL((k_tune_fill<T>), dim3(grid_for(S.n)), dim3(kThreads), 0, s, S);
    hipLaunchKernelGGL(k_tune_state, dim3(1), dim3(64), 0, s, S.st, S.red.cnt, S.n);
    S7_CHECK_LAUNCH();
    return S7_OK;
}

// Picks the launch parameters of the single-system solve for the size class of
// d: first the pass form (the staged passes with tiles of 2048, 4096 and 8192
// cells, i.e. 8, 16 or 32 cells per thread, each in plain and band-per-XCD tile
// order; cell pairs; single cells in three and in four passes) at the default
// streaming split, then the streaming split (256, 512 or 1024 workgroups) for
// the best form.  Each candidate runs one warm-up and K timed iterations on
// the trial system.  best = {schedule, stream_blocks, lds_tile, xcd_run}.
template <class T>
static int tune_single(s7_dims d, const Layout& Lo, int jacobi, int xr, char* ws, hipStream_t s,
                       int (&best)[4]) {
    const TuneKey key{TUNE_SINGLE, TypeTag<T>::value, jacobi, size_bucket((double)Lo.n), 0};
    if (tune_lookup(key, best)) return S7_OK;
    SysView<T> S = make_view<T>(d, Lo, jacobi, ws);
    const int K = std::max(2, std::min(12, auto_graph_iters(Lo.n, (int)sizeof(T)) / 2));
    hipEvent_t e0, e1;
    S7_HIP(hipEventCreate(&e0));
    S7_HIP(hipEventCreate(&e1));
    const bool even = S.pair_blocks > 0;
    std::vector<PassLaunch> forms;
    for (int tile : {2048, 4096, 8192}) {
        if (!even || lds_tile_for(tile, S.m.nx, true) != tile) continue;
        for (int x : {1, -1}) forms.push_back(PassLaunch{SCHED_LDS, x, tile});
    }
    if (even) forms.push_back(PassLaunch{SCHED_PAIRS, xr, 0});
    forms.push_back(PassLaunch{SCHED_THREE, xr, 0});
    forms.push_back(PassLaunch{SCHED_FOUR, xr, 0});
    int rc = S7_OK;
    // one timed trial: iterations per millisecond, or a negative value if the
    // trial system stopped (then the time says nothing)
    auto trial = [&](const PassLaunch& L, int sb, float* out_ms) -> int {
        S.stream_blocks = sb;
        int r = tune_prepare<T>(S, s);
        if (r) return r;
        for (int p = 0; p < kPasses; ++p) launch_pass<T>(S, p, L, s);
        if (hipEventRecord(e0, s) != hipSuccess) return S7_EHIP;
        for (int j = 0; j < K; ++j)
            for (int p = 0; p < kPasses; ++p) launch_pass<T>(S, p, L, s);
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return S7_EHIP;
        State h;
        if ((r = read_state(S.st, &h, s))) return r;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        *out_ms = (h.done || h.iter != K + 1) ? -1.0f : ms / (float)K;
        char line[200];
        std::snprintf(line, sizeof line, "single tag=%d unit=%d dims=%dx%dx%d schedule=%d lds_tile=%d xcd_run=%d "
                      "stream_blocks=%d ms_per_iteration=%.4f", TypeTag<T>::value, jacobi, d.nx, d.ny, d.nz,
                      L.sched, L.tile, L.xr, sb, *out_ms);
        tune_log(line);
        return S7_OK;
    };
    const int sb0 = stream_blocks_for((long long)Lo.n, 0);
    PassLaunch bestL = forms.front();
    float best_ms = INFINITY;
    for (const PassLaunch& L : forms) {
        float ms;
        if ((rc = trial(L, sb0, &ms))) break;
        if (ms >= 0.0f && ms < best_ms) {
            best_ms = ms;
            bestL = L;
        }
    }
    int best_sb = sb0;
    if (!rc && best_ms < INFINITY) {
        for (int cap : {512, 1024}) {
            const int sb = stream_blocks_for((long long)Lo.n, cap);
            if (sb == sb0) continue;
            float ms;
            if ((rc = trial(bestL, sb, &ms))) break;
            if (ms >= 0.0f && ms < best_ms) {
                best_ms = ms;
                best_sb = sb;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        set_error("autotuning trial failed");
        return rc;
    }
    if (best_ms == INFINITY) {  // no timing: the defaults
        s7_options def;
        s7_default_options(&def);
        const PassLaunch L = pass_launch(def, S);
        bestL = PassLaunch{L.sched, xr, L.tile};
    }
    best[0] = bestL.sched;
    best[1] = best_sb;
    best[2] = bestL.tile;
    best[3] = bestL.xr;
    tune_store(key, best);
    return S7_OK;
}

static int solve_fp32(s7_dims d, const Coef7& cf, const double* b, double* x, double rtol,
                      int max_iter, char* ws, const Layout& Lo, const s7_options& o,
                      s7_info* info, hipStream_t s, bool direct = false) {
    SysView<float> S = make_view<float>(d, Lo, o.jacobi, ws);
    int rc = start_solve<float>(cf, S, Lo, o.jacobi, s);
    if (rc) return rc;
    auto t0 = std::chrono::steady_clock::now();
    hipLaunchKernelGGL(k_init_f32, dim3(S.cell_blocks), dim3(kThreads), 0, s, cf, b, x, S, o.jacobi,
                       rtol, max_iter);
    launch_finish<3, 0u, FIN_INIT>(S.red, S.cell_blocks, S.st, s, rtol, max_iter);
    S7_CHECK_LAUNCH();
    State h;
    rc = run_iterations<float>(S, o, s, &h, info, direct);
    if (rc) return rc;
    hipLaunchKernelGGL(k_update_x, dim3(S.stream_blocks), dim3(kThreads), 0, s, x, S.d, S.n, 1.0, S.st);
    S7_CHECK_LAUNCH();
    rc = resid_launch<float>(cf, b, x, nullptr, S, o.jacobi, s);
    if (rc) return rc;
    rc = read_state(S.st, &h, s);
    if (rc) return rc;
    auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->status = h.status;
        info->reason = h.reason;
        info->rel_res_rec = h.res_rec;
        info->iters = h.iter;
        info->outer_iters = 1;
        info->schedule = effective_schedule(o, S);
        info->lds_tile = pass_launch(o, S).tile;
        info->xcd_run = o.xcd_run;
        info->rel_res_true = h.bb_true > 0 ? sqrt(h.rr_true / h.bb_true) : 0.0;
        info->t_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    return h.status;
}

// The outer loop of iterative refinement (reading 13), for any operator:
// resid() forms the FP64 residual b - A x into State (||b||^2, ||r||^2,
// max |r_s|) and r_s into d as FP32; iterate(h) runs an inner solve from the
// State that k_ir_init set, leaving it in *h.
template <class T, class Resid, class Iterate>
static int refine(const SysView<T>& S, double* x, double rtol, int max_iter, const s7_options& o, int prec,
                  int schedule, s7_info* info, hipStream_t s, Resid resid, Iterate iterate) {
    auto t0 = std::chrono::steady_clock::now();
    const double inner_tol = o.inner_rtol > 0 ? o.inner_rtol : (prec == S7_FP16_IR ? 5e-3 : 1e-2);
    const int inner_cap = o.inner_max_iter > 0 ? o.inner_max_iter : 100;
    const int outer_cap = o.outer_max_iter > 0 ? o.outer_max_iter : 30;
    int total = 0, outer = 0, status = S7_NOT_CONVERGED, reason = 0;
    double rel = INFINITY, inner_res = 0.0;
    int stall = 0;
    State h;
    int rc;
    for (;;) {
        if ((rc = resid())) return rc;
        if ((rc = read_state(S.st, &h, s))) return rc;
        if (h.bb_true == 0.0) {
            hipLaunchKernelGGL(k_fill0, dim3(grid_for(S.n)), dim3(kThreads), 0, s, x, S.n);
            S7_CHECK_LAUNCH();
            rel = 0.0;
            status = S7_OK;
            break;
        }
        const double nrel = sqrt(h.rr_true / h.bb_true);
        if (!std::isfinite(nrel)) {
            status = S7_BREAKDOWN;
            reason = S7_REASON_NONFINITE;
            rel = nrel;
            break;
        }
        stall = (nrel > 0.5 * rel) ? stall + 1 : 0;
        rel = nrel;
        if (rel <= rtol) {
            status = S7_OK;
            break;
        }
        if (outer >= outer_cap || total >= max_iter || stall >= 3) {
            status = S7_NOT_CONVERGED;
            break;
        }
        // power-of-two scale 2^ceil(log2 rmax), exactly: the inner right-hand side
        // has max |.| in (0.5, 1]
        double scale = 1.0;
        if (h.rmax > 0) {
            int e;
            const double m = std::frexp(h.rmax, &e);  // rmax = m 2^e, m in [0.5, 1)
            scale = std::ldexp(1.0, m == 0.5 ? e - 1 : e);
        }
        hipLaunchKernelGGL((k_ir_init<T>), dim3(S.stream_blocks), dim3(kThreads), 0, s, S,
                           (float)(1.0 / scale), inner_tol,
                           inner_cap < max_iter - total ? inner_cap : max_iter - total);
        S7_CHECK_LAUNCH();
        if ((rc = iterate(&h))) return rc;
        total += h.iter;
        outer += 1;
        inner_res = h.res_rec;
        if (h.status == S7_BREAKDOWN && h.iter == 0) {
            status = S7_BREAKDOWN;
            reason = h.reason;
            break;
        }
        hipLaunchKernelGGL(k_update_x, dim3(S.stream_blocks), dim3(kThreads), 0, s, x, S.d, S.n,
                           scale, S.st);
        S7_CHECK_LAUNCH();
    }
    S7_HIP(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->status = status;
        info->reason = reason;
        info->iters = total;
        info->outer_iters = outer;
        info->schedule = schedule;
        info->rel_res_true = rel;
        info->rel_res_rec = inner_res;
        info->t_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    return status;
}

template <class T>
static int solve_ir(s7_dims d, const Coef7& cf, const double* b, double* x, double rtol,
                    int max_iter, char* ws, const Layout& Lo, const s7_options& o,
                    s7_info* info, hipStream_t s, int prec) {
    SysView<T> S = make_view<T>(d, Lo, o.jacobi, ws);
    int rc = start_solve<T>(cf, S, Lo, o.jacobi, s);
    if (rc) return rc;
    const int rc2 = refine<T>(S, x, rtol, max_iter, o, prec, effective_schedule(o, S), info, s,
                              [&]() { return resid_launch<T>(cf, b, x, S.d, S, o.jacobi, s); },
                              [&](State* h) { return run_iterations<T>(S, o, s, h, info); });
    if (info) {
        info->lds_tile = pass_launch(o, S).tile;
        info->xcd_run = o.xcd_run;
    }
    return rc2;
}

// ============================================================== batch engine
// A job is J_NEW until it is in a start launch, then J_RUN: the device
// runs the rest of its solve (iterations, refinement steps, epilogue).
enum JobStage { J_NEW = 0, J_RUN = 1 };

// Engine tables: [BGlobal][BSys x cap][State* x cap][State x cap][JobStart x cap][home x kMaxPersistentGrid].
static size_t off_sys() { return align256(sizeof(BGlobal)); }
static size_t off_sptr(int cap) { return off_sys() + align256((size_t)cap * sizeof(BSys)); }
static size_t off_sgather(int cap) { return off_sptr(cap) + align256((size_t)cap * sizeof(State*)); }

static size_t off_jobs(int cap) { return off_sgather(cap) + align256((size_t)cap * sizeof(State)); }

static size_t off_home(int cap) { return off_jobs(cap) + align256((size_t)cap * sizeof(JobStart)); }

// The most workgroups of a persistent launch (the home table's length).
constexpr int kMaxPersistentGrid = 1024;

size_t engine_table_bytes(int capacity) {
    return off_home(capacity) + align256((size_t)kMaxPersistentGrid * sizeof(int));
}

static int chunk_cells_of(const s7_options& o);

// Pinned host buffers for the engines' state reads, kept for the life of the
// process: every batched call builds an engine, and pinning fresh host memory
// for each call cost more than the call's other host work.
static std::mutex g_pinned_mu;
static std::vector<std::pair<size_t, void*>> g_pinned_free;

static void* pinned_take(size_t bytes) {
    {
        std::lock_guard<std::mutex> lk(g_pinned_mu);
        for (size_t i = 0; i < g_pinned_free.size(); ++i) {
            if (g_pinned_free[i].first >= bytes) {
                void* p = g_pinned_free[i].second;
                g_pinned_free.erase(g_pinned_free.begin() + (long)i);
                return p;
            }
        }
    }
    void* p = nullptr;
    return hipHostMalloc(&p, bytes, hipHostMallocDefault) == hipSuccess ? p : nullptr;
}

static void pinned_give(void* p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    g_pinned_free.emplace_back(bytes, p);
}

BatchEngine::BatchEngine(char* tables, int capacity, const s7_options& o, hipStream_t stream,
                         bool use_graph)
    : tables_(tables), cap_(capacity), o_(o), st_(stream), graph_(use_graph),
      chunk_(chunk_cells_of(o)), grid_cap_(1024) {
    host_states_ = static_cast<State*>(pinned_take((size_t)capacity * sizeof(State)));  // null: read_states reports it
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
        ticks_per_ms_ = (double)khz;
}

BatchEngine::~BatchEngine() {
    pinned_give(host_states_, (size_t)cap_ * sizeof(State));
}

static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int BatchEngine::add(EngineJob* j) {
    if ((int)jobs_.size() >= cap_) {
        set_error("batch engine: more than %d resident systems", cap_);
        return S7_EAGAIN;
    }
    j->lo = make_layout(j->d, j->prec, o_, j->op == OP_9PT ? (o_.jacobi ? 8 : 9) : 0);
    j->stage = J_NEW;
    j->tag = j->prec == S7_FP32 ? 0 : (j->prec == S7_BF16_IR ? 1 : 2);
    j->finished = 0;
    std::memset(&j->info, 0, sizeof(j->info));
    if (j->t_start_ms <= 0.0) j->t_start_ms = now_ms();
    jobs_.push_back(j);
    return S7_OK;
}

// Cells per work item.  Every chunk costs a claim and a completion, each a
// round trip to memory on the system's own control words, so chunks are
// large by default: a small system is one or two chunks, done by one
// workgroup with no hand-off, and the batch itself supplies the parallelism.
// A chunk is a whole number of the units whose sums the phases keep.
static int chunk_cells_of(const s7_options& o) {
    int c = o.chunk_cells > 0 ? o.chunk_cells : 16384;
    if (c > (1 << 24)) c = 1 << 24;  // chunk start + chunk_cells stays within 32 bits
    c = (c + kUnitCells - 1) / kUnitCells * kUnitCells;
    return c;
}

// The chunk of each system in a launch.  While the resident set has fewer
// work items than the persistent grid has workgroups (light load), a system
// of few chunks has its chunks halved, down to one unit group and up to
// kShrinkChunks chunks, so that a lone system is spread over more workgroups.
// Larger systems keep their chunks: the claims and completions of one
// system's chunks are atomics on the same control words, which serialize.
// The sums are kept per unit, so this changes no result.  An explicit
// options.chunk_cells is kept as given.
constexpr long long kShrinkChunks = 32;
static std::vector<int> launch_chunks(const std::vector<EngineJob*>& jobs, int chunk, int grid_cap, bool adapt) {
    std::vector<int> c(jobs.size(), chunk);
    if (!adapt) return c;
    long long items = 0;
    for (const EngineJob* j : jobs) items += (long long)((j->lo.n + chunk - 1) / chunk);
    if (items >= grid_cap) return c;
    for (size_t i = 0; i < jobs.size(); ++i) {
        const long long n = (long long)jobs[i]->lo.n;
        while (c[i] >= 2 * kUnitGroup && c[i] % (2 * kUnitCells) == 0 && (n + c[i] / 2 - 1) / (c[i] / 2) <= kShrinkChunks)
            c[i] /= 2;
    }
    return c;
}

// The start-table entry of a new job: coefficient copies, State and control
// words, and the first phase (the FP32 start S, or the FP64 residual R that
// begins refinement).
static JobStart job_entry(const EngineJob& j, const s7_options& o) {
    const int op = j.op;
    JobStart J{};
    SysView<float> S = make_view<float>(j.d, j.lo, o.jacobi, j.ws);  // pointer members only
    for (int a = 0; a < 7; ++a) J.cf.c[a] = j.coef[a];
    J.cf9[0] = j.coef9[0];
    J.cf9[1] = j.coef9[1];
    J.op = op;
    J.coef_dst = const_cast<float*>(S.c[o.jacobi ? 1 : 0]);
    J.span = align256(j.lo.n * j.lo.elt) / j.lo.elt;
    J.m = S.m;
    J.n = S.n;
    J.jacobi = o.jacobi ? 1 : 0;
    J.tag = j.tag;
    J.ir = j.prec == S7_FP32 ? 0 : 1;
    J.first = J.ir ? (int)K_R : (int)K_S;
    J.st = S.st;
    J.cnt = S.red.cnt;
    J.ctl = reinterpret_cast<BCtl*>(j.ws + j.lo.off_ctl);
    J.rtol = j.rtol;
    J.inner_tol = o.inner_rtol > 0 ? o.inner_rtol : (j.prec == S7_FP16_IR ? 5e-3 : 1e-2);
    J.inner_cap = o.inner_max_iter > 0 ? o.inner_max_iter : 100;
    J.outer_cap = o.outer_max_iter > 0 ? o.outer_max_iter : 30;
    J.max_total = j.max_iter;
    return J;
}

#define S7_BY_PREC(j, call)                                           \
    ((j).prec == S7_FP32 ? call<float> : ((j).prec == S7_BF16_IR ? call<bf16> : call<f16>))

// The table entry of a resident job in a persistent launch.
static BSys sys_entry(const EngineJob& j, const s7_options& o, int chunk, int budget) {
    const int op = j.op;
    BSys b;
    std::memset(&b, 0, sizeof(b));
    b.op = op;
    b.S = make_view<float>(j.d, j.lo, o.jacobi, j.ws);
    b.ctl = reinterpret_cast<BCtl*>(j.ws + j.lo.off_ctl);
    b.nchunk = (int)((j.lo.n + chunk - 1) / chunk);
    b.chunk = chunk;
    b.tag = j.tag;
    b.budget = budget;
    for (int a = 0; a < 7; ++a) b.cf.c[a] = j.coef[a];
    b.b = j.b;
    b.x = j.x;
    if (op == OP_9PT) {
        // the working copies of coefficients 7 and 8 follow the first seven
        const size_t span = align256(j.lo.n * j.lo.elt);
        const int first = o.jacobi ? 1 : 0;
        for (int i = 0; i < 2; ++i) {
            b.cf9[i] = j.coef9[i];
            b.wk9[i] = reinterpret_cast<const float*>(j.ws + j.lo.off_coef + (size_t)(7 + i - first) * span);
        }
    }
    return b;
}

static void finish_job(EngineJob& j, const State& h) {
    const int op = j.op;
    s7_info& inf = j.info;
    std::memset(&inf, 0, sizeof(inf));
    inf.iters = h.total;
    inf.outer_iters = h.ir ? h.outer : 1;
    // the persistent kernel's phases: cell pairs for the 7-point operator with an even nx
    inf.schedule = op == OP_7PT && j.d.nx % 2 == 0 ? SCHED_PAIRS : SCHED_THREE;
    inf.status = h.ostatus;
    inf.reason = h.oreason;
    inf.rel_res_rec = h.inner_res;
    if (h.ir) inf.rel_res_true = h.rel;
    else inf.rel_res_true = h.bb_true > 0 ? sqrt(h.rr_true / h.bb_true) : 0.0;
    inf.t_ms = now_ms() - j.t_start_ms;
    j.finished = 1;
}

// Every resident job's State, in job order: one gather kernel and one transfer.
int BatchEngine::read_states(std::vector<State>& h) {
    const int n = (int)jobs_.size();
    h.resize((size_t)n);
    if (n == 0) return S7_OK;
    if (!host_states_) {
        set_error("batch engine: pinned host buffer unavailable");
        return S7_EHIP;
    }
    State** dptr = reinterpret_cast<State**>(tables_ + off_sptr(cap_));
    State* dst = reinterpret_cast<State*>(tables_ + off_sgather(cap_));
    hipLaunchKernelGGL(k_gather_states, dim3((n * (int)(sizeof(State) / 8) + kThreads - 1) / kThreads),
                       dim3(kThreads), 0, st_, (State* const*)dptr, dst, n);
    S7_CHECK_LAUNCH();
    S7_HIP(hipMemcpyAsync(host_states_, dst, (size_t)n * sizeof(State), hipMemcpyDeviceToHost, st_));
    S7_HIP(hipStreamSynchronize(st_));
    std::memcpy(h.data(), host_states_, (size_t)n * sizeof(State));
    return S7_OK;
}

// Each workgroup's home system, where its search for work starts while that
// system is active: the systems in table order, each taking a share of the
// grid's workgroups in proportion to its cell count.  A large system thus has
// many workgroups returning to it from the start, instead of the uniform share
// that leaves it running alone at the end of the launch.
static std::vector<int> weighted_homes(const std::vector<double>& cells, int grid) {
    const int nsys = (int)cells.size();
    std::vector<double> cum((size_t)nsys + 1, 0.0);
    for (int i = 0; i < nsys; ++i) cum[(size_t)i + 1] = cum[(size_t)i] + cells[(size_t)i];
    std::vector<int> home((size_t)grid);
    for (int b = 0; b < grid; ++b) {
        const double at = (b + 0.5) / grid * cum[(size_t)nsys];
        const int h = (int)(std::upper_bound(cum.begin() + 1, cum.end(), at) - (cum.begin() + 1));
        home[(size_t)b] = h < nsys ? h : nsys - 1;
    }
    return home;
}

int BatchEngine::launch(const std::vector<BSys>& table, int epoch_key, int chunk, int grid_cap,
                        long long slice) {
    BGlobal* glob = reinterpret_cast<BGlobal*>(tables_);
    BSys* dsys = reinterpret_cast<BSys*>(tables_ + off_sys());
    S7_HIP(hipMemcpyAsync(dsys, table.data(), table.size() * sizeof(BSys), hipMemcpyHostToDevice, st_));
    const int nsys = (int)table.size();
    long long total_chunks = 0;
    for (const BSys& b : table) total_chunks += b.nchunk;
    int grid = (int)(total_chunks < grid_cap ? total_chunks : grid_cap);
    if (grid < 1) grid = 1;
    if (grid > kMaxPersistentGrid) grid = kMaxPersistentGrid;
    std::vector<double> cells;
    for (const BSys& b : table) cells.push_back((double)b.S.n);
    const std::vector<int> home = weighted_homes(cells, grid);
    int* dhome = reinterpret_cast<int*>(tables_ + off_home(cap_));
    S7_HIP(hipMemcpyAsync(dhome, home.data(), home.size() * sizeof(int), hipMemcpyHostToDevice, st_));
    const long long spin_limit = 5000000;
    auto body = [&](hipStream_t cs) {
        hipLaunchKernelGGL(k_batched_arm, dim3(1), dim3(kThreads), 0, cs, (const BSys*)dsys, glob, nsys,
                           slice);
        hipLaunchKernelGGL(k_batched, dim3(grid), dim3(kThreads), 0, cs, (const BSys*)dsys, (const int*)dhome,
                           glob, nsys, spin_limit);
    };
    GraphRef g;  // held until the launch has completed
    if (graph_) {
        // the table is re-uploaded before every replay, so the key needs only its shape
        std::vector<uintptr_t> key = {0x53u, (uintptr_t)tables_, (uintptr_t)nsys, (uintptr_t)epoch_key,
                                      (uintptr_t)grid, (uintptr_t)chunk, (uintptr_t)slice};
        int rc = cached_graph(key, body, &g);
        if (rc) return rc;
        S7_HIP(hipGraphLaunch(g->exec, st_));
    } else {
        // the serving loop: the resident set changes from step to step
        body(st_);
        S7_CHECK_LAUNCH();
    }
    BGlobal hg;
    S7_HIP(hipMemcpyAsync(&hg, glob, sizeof(hg), hipMemcpyDeviceToHost, st_));
    S7_HIP(hipStreamSynchronize(st_));
    if (hg.error) {
        set_error("batched launch: a workgroup exceeded its wait bound");
        return S7_EHIP;
    }
    return S7_OK;
}

// A trial system in the job's workspace; the 9-point operator's two extra
// working copies are zero (the trial is the 5-point part).
template <class T>
static int tune_prepare_job(const EngineJob& j, const s7_options& o, hipStream_t s) {
    const int rc = tune_prepare<T>(make_view<T>(j.d, j.lo, o.jacobi, j.ws), s);
    if (rc || j.op != OP_9PT) return rc;
    const size_t span = align256(j.lo.n * j.lo.elt);
    const int first = o.jacobi ? 1 : 0;
    S7_HIP(hipMemsetAsync(j.ws + j.lo.off_coef + (size_t)(7 - first) * span, 0, 2 * span, s));
    return S7_OK;
}

int BatchEngine::tune() {
    if (jobs_.empty()) return S7_OK;
    double total = 0.0;
    for (const EngineJob* j : jobs_) {
        if (j->stage != J_NEW) {
            set_error("batch engine: tune() after the first step");
            return S7_EINVAL;
        }
        total += (double)j->lo.n;
    }
    const TuneKey key{jobs_[0]->op == OP_9PT ? TUNE_BATCH9 : TUNE_BATCH, jobs_[0]->tag, o_.jacobi, size_bucket(total),
                      size_bucket((double)jobs_.size())};
    int best[4] = {0, 0, 0, 0};
    if (tune_lookup(key, best)) {
        chunk_ = best[0];
        grid_cap_ = best[1];
        return S7_OK;
    }
    const bool graph = graph_;
    graph_ = false;  // trials launch directly
    hipEvent_t e0, e1;
    S7_HIP(hipEventCreate(&e0));
    S7_HIP(hipEventCreate(&e1));
    const int K = 4;
    float best_ms = INFINITY;
    best[0] = chunk_;
    best[1] = grid_cap_;
    int rc = S7_OK;
    for (int chunk : {1024, 2048, 4096, 8192, 16384, 32768, 65536}) {
        for (int gcap : {256, 512, 768, 1024}) {
            std::vector<BSys> table;
            long long chunks = 0;
            for (EngineJob* j : jobs_) {
                if ((rc = S7_BY_PREC(*j, tune_prepare_job)(*j, o_, st_))) break;
                hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, st_,
                                   reinterpret_cast<BCtl*>(j->ws + j->lo.off_ctl), (int)K_P1);
                const BSys b = sys_entry(*j, o_, chunk, K);
                chunks += b.nchunk;
                table.push_back(b);
            }
            if (rc) break;
            if (gcap > 256 && chunks <= gcap / 2) continue;  // about the same grid as a smaller cap
            if (hipEventRecord(e0, st_) != hipSuccess) { rc = S7_EHIP; break; }
            if ((rc = launch(table, K, chunk, gcap))) break;
            if (hipEventRecord(e1, st_) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                rc = S7_EHIP;
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            char line[160];
            std::snprintf(line, sizeof line, "batch op=%d tag=%d systems=%d chunk_cells=%d grid_cap=%d ms=%.4f",
                          jobs_[0]->op, jobs_[0]->tag, (int)jobs_.size(), chunk, gcap, ms);
            tune_log(line);
            if (ms < best_ms) {
                best_ms = ms;
                best[0] = chunk;
                best[1] = gcap;
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    graph_ = graph;
    if (rc) return rc;
    tune_store(key, best);
    chunk_ = best[0];
    grid_cap_ = best[1];
    return S7_OK;
}

int BatchEngine::step(int epoch_iters, double slice_ms) {
    if (jobs_.empty()) return S7_OK;
    int rc;
    // 1) start new jobs, all in one launch; the state pointer table follows the
    // resident set
    std::vector<State*> sptr;
    std::vector<JobStart> starts;
    size_t max_n = 1;
    for (EngineJob* j : jobs_) {
        sptr.push_back(reinterpret_cast<State*>(j->ws + j->lo.off_state));
        if (j->stage != J_NEW) continue;
        starts.push_back(job_entry(*j, o_));
        max_n = std::max(max_n, j->lo.n);
        j->stage = J_RUN;
    }
    S7_HIP(hipMemcpyAsync(tables_ + off_sptr(cap_), sptr.data(), sptr.size() * sizeof(State*),
                          hipMemcpyHostToDevice, st_));
    if (!starts.empty()) {
        JobStart* dj = reinterpret_cast<JobStart*>(tables_ + off_jobs(cap_));
        S7_HIP(hipMemcpyAsync(dj, starts.data(), starts.size() * sizeof(JobStart), hipMemcpyHostToDevice, st_));
        const int gx = (int)std::min<size_t>(128, (max_n + kThreads - 1) / kThreads);
        for (size_t k = 0; k < starts.size(); k += 65535) {  // the grid's y extent is at most 65535
            const unsigned ny = (unsigned)std::min<size_t>(65535, starts.size() - k);
            hipLaunchKernelGGL(k_jobs_start, dim3(gx, ny), dim3(kThreads), 0, st_, (const JobStart*)(dj + k));
        }
        S7_CHECK_LAUNCH();
    }
    // 2) one persistent launch over every resident job
    std::vector<BSys> table;
    const std::vector<int> chunks = launch_chunks(jobs_, chunk_, grid_cap_, o_.chunk_cells == 0);
    for (size_t i = 0; i < jobs_.size(); ++i)
        table.push_back(sys_entry(*jobs_[i], o_, chunks[i], epoch_iters > 0 ? epoch_iters : (1 << 30)));
    const int chunk = chunk_;
    const long long slice = epoch_iters > 0 ? 0 : (long long)(slice_ms * ticks_per_ms_);
    rc = launch(table, epoch_iters, chunk, grid_cap_, slice);
    if (rc) return rc;
    // 3) finished jobs leave
    std::vector<State> h;
    rc = read_states(h);
    if (rc) return rc;
    std::vector<EngineJob*> keep;
    for (size_t i = 0; i < jobs_.size(); ++i) {
        if (h[i].final) finish_job(*jobs_[i], h[i]);
        else keep.push_back(jobs_[i]);
    }
    jobs_.swap(keep);
    return S7_OK;
}

// A system of split_cells cells or more gains nothing from the shared launch:
// its phases already fill the chip, and at thousands of chunks per phase the
// claim and completion atomics on its control words, which serialize, cost
// more than the pass itself.  It runs alone on the multi-kernel path, in its
// own slice of the workspace, after the shared launch.  The choice depends
// only on the system's own size, so a system's result still does not depend
// on the rest of the batch.
static long long split_cells_of(const s7_options& o) {
    return o.split_cells < 0 ? (1ll << 62) : (o.split_cells > 0 ? o.split_cells : 1ll << 21);
}

// Runs a batch whose jobs are filled in (workspace slices included): the jobs
// marked in `big` run one by one through `alone`, after the others have run
// together on one engine.  Fills info[i] and returns the worst status.
template <class Alone>
static int run_batch(std::vector<EngineJob>& jobs, const std::vector<char>& big, int op, char* w,
                     const s7_options& o, hipStream_t s, s7_info* info, const char* who, Alone alone) {
    const int nsys = (int)jobs.size();
    BatchEngine eng(w, nsys, o, s, /*use_graph=*/true);
    for (int i = 0; i < nsys; ++i) {
        if (big[i]) continue;
        EngineJob& j = jobs[i];
        j.op = op;
        const int rc = eng.add(&j);
        if (rc) return rc;
    }
    if (o.tune && o.chunk_cells == 0 && eng.resident() > 0) {
        const int rc = eng.tune();
        if (rc) return rc;
    }
    int guard = 0;
    while (eng.resident() > 0) {
        const int rc = eng.step(1 << 30);
        if (rc) return rc;
        if (++guard > 100000) {
            set_error("%s: no progress", who);
            return S7_EHIP;
        }
    }
    for (int i = 0; i < nsys; ++i) {
        if (!big[i]) continue;
        const int rc = alone(jobs[i]);
        if (rc < 0) return rc;
    }
    int worst = S7_OK;
    for (int i = 0; i < nsys; ++i) {
        if (info) info[i] = jobs[i].info;
        if (jobs[i].info.status > worst) worst = jobs[i].info.status;
    }
    return worst;
}

}  // namespace s7

// ============================================================== C ABI
using namespace s7;

extern "C" {

void s7_default_options(s7_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->jacobi = 1;
}

const char* s7_last_error(void) { return g_err.c_str(); }

int32_t s7_version(void) { return 0x010000; }

static bool coef_ok(const float* const coef[7]) {
    if (!coef) return false;
    for (int a = 0; a < 7; ++a)
        if (!coef[a]) return false;
    return true;
}

constexpr int kApplyMinCells = 1 << 18;

int s7_stencil_apply(s7_dims d, const float* const coef[7], const float* v, float* u, void* stream) {
    clear_error();
    if (!dims_ok(d) || !coef_ok(coef) || !v || !u || v == u) {
        set_error("s7_stencil_apply: invalid argument");
        return S7_EINVAL;
    }
    const Mesh m = make_mesh(d.nx, d.ny, d.nz);
    const int n = d.nx * d.ny * d.nz;
    Coef7 cf;
    bool aligned = ((uintptr_t)v & 15u) == 0 && ((uintptr_t)u & 7u) == 0;
    for (int a = 0; a < 7; ++a) {
        cf.c[a] = coef[a];
        aligned = aligned && ((uintptr_t)coef[a] & 7u) == 0;
    }
    // The staged pairs for an even nx whose rows fit the LDS, on meshes large
    // enough to fill the chip with 2048-cell tiles, when v allows 16-byte and
    // the rest 8-byte accesses; single cells otherwise.
    constexpr int kApplyTile = 2048;
    if (d.nx % 2 == 0 && lds_fits(d.nx, kApplyTile) && n >= kApplyMinCells && aligned) {
        const int nb = lds_blocks(n, kApplyTile);
        const size_t lds = (size_t)lds_count(d.nx, kApplyTile) * sizeof(float);
        hipLaunchKernelGGL((k_apply_lds<kApplyTile>), dim3(nb), dim3(kThreads), lds, (hipStream_t)stream, cf, v, u,
                           m, n, nb, tile_run(-1, m, kApplyTile));
    } else {
        hipLaunchKernelGGL(k_stencil_apply, dim3(cell_blocks_for(n)), dim3(kThreads), 0,
                           (hipStream_t)stream, cf, v, u, m, n);
    }
    S7_CHECK_LAUNCH();
    return S7_OK;
}

size_t s7_workspace_bytes(s7_dims d, int32_t prec, const s7_options* opt) {
    if (!dims_ok(d) || prec < S7_FP32 || prec > S7_FP16_IR) return 0;
    s7_options o;
    options_or_default(opt, o);
    return make_layout(d, prec, o).bytes;
}

int s7_bicgstab_solve(s7_dims d, const float* const coef[7], const double* b, double* x,
                      double rtol, int32_t max_iter, int32_t prec, void* ws, size_t ws_bytes,
                      const s7_options* opt, s7_info* info, void* stream) {
    clear_error();
    if (info) std::memset(info, 0, sizeof(*info));
    s7_options o;
    options_or_default(opt, o);
    if (!dims_ok(d) || !coef_ok(coef) || !b || !x || !ws || !(rtol > 0.0) || max_iter < 0 ||
        prec < S7_FP32 || prec > S7_FP16_IR || ((uintptr_t)ws & 255u) != 0) {
        set_error("s7_bicgstab_solve: invalid argument");
        return S7_EINVAL;
    }
    Layout Lo = make_layout(d, prec, o);
    if (ws_bytes < Lo.bytes) {
        set_error("s7_bicgstab_solve: workspace too small (%zu < %zu)", ws_bytes, Lo.bytes);
        return S7_EINVAL;
    }
    Coef7 cf;
    for (int a = 0; a < 7; ++a) cf.c[a] = coef[a];
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)ws;
    if (o.tune && (o.schedule == 0 || o.stream_blocks == 0)) {
        int best[4];
        const int rc = prec == S7_FP32      ? tune_single<float>(d, Lo, o.jacobi, o.xcd_run, w, s, best)
                       : prec == S7_BF16_IR ? tune_single<bf16>(d, Lo, o.jacobi, o.xcd_run, w, s, best)
                                            : tune_single<f16>(d, Lo, o.jacobi, o.xcd_run, w, s, best);
        if (rc) return rc;
        if (o.schedule == 0) {
            o.schedule = best[0];
            if (o.lds_tile == 0) o.lds_tile = best[2];
            if (o.xcd_run == 0) o.xcd_run = best[3];
        }
        if (o.stream_blocks == 0) o.stream_blocks = best[1];
        Lo = make_layout(d, prec, o);
    }
    if (prec == S7_FP32) return solve_fp32(d, cf, b, x, rtol, max_iter, w, Lo, o, info, s);
    if (prec == S7_BF16_IR) return solve_ir<bf16>(d, cf, b, x, rtol, max_iter, w, Lo, o, info, s, prec);
    return solve_ir<f16>(d, cf, b, x, rtol, max_iter, w, Lo, o, info, s, prec);
}

// ============================================================== solve without allocation
// The workspace of s7_bicgstab_solve_noalloc: a fixed array in device memory,
// one copy per GPU, held until the process ends.  Its name stands for the array
// in device code only; host code reaches it through the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[S7_NOALLOC_WS_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];

static int scratch_for_current_device(void** out) {
    int dev = 0;
    S7_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("s7_bicgstab_solve_noalloc: device index %d out of range", dev);
        return S7_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return S7_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return S7_OK;
}

int s7_bicgstab_solve_noalloc(s7_dims d, const float* const coef[7], const double* b, double* x,
                              double rtol, int32_t max_iter, const s7_options* opt, s7_info* info,
                              void* stream) {
    clear_error();
    if (info) std::memset(info, 0, sizeof(*info));
    s7_options o;
    options_or_default(opt, o);
    o.tune = 0;     // tuning trials time with events
    o.profile = 0;  // per-pass timing creates events
    if (!dims_ok(d) || !coef_ok(coef) || !b || !x || !(rtol > 0.0) || max_iter < 0) {
        set_error("s7_bicgstab_solve_noalloc: invalid argument");
        return S7_EINVAL;
    }
    const Layout Lo = make_layout(d, S7_FP32, o);
    if (Lo.bytes > (size_t)S7_NOALLOC_WS_BYTES) {
        set_error("s7_bicgstab_solve_noalloc: the system needs %zu workspace bytes, more than the "
                  "%zu of the fixed workspace", Lo.bytes, (size_t)S7_NOALLOC_WS_BYTES);
        return S7_EINVAL;
    }
    void* ws = nullptr;
    const int rc = scratch_for_current_device(&ws);
    if (rc) return rc;
    Coef7 cf;
    for (int a = 0; a < 7; ++a) cf.c[a] = coef[a];
    return solve_fp32(d, cf, b, x, rtol, max_iter, (char*)ws, Lo, o, info, (hipStream_t)stream, true);
}

int s7_generate_problem(s7_dims d, uint64_t seed, int32_t recipe, float* const coef[7],
                        double* xstar, double* b, void* stream) {
    clear_error();
    if (!dims_ok(d) || (recipe != 0 && recipe != 1)) {
        set_error("s7_generate_problem: invalid argument");
        return S7_EINVAL;
    }
    const Mesh m = make_mesh(d.nx, d.ny, d.nz);
    Coef7 cf;
    bool all = coef != nullptr;
    for (int a = 0; a < 7; ++a) {
        cf.c[a] = coef ? coef[a] : nullptr;
        all = all && cf.c[a];
    }
    if (b && (!all || !xstar)) {
        set_error("s7_generate_problem: b needs all coefficient arrays and xstar");
        return S7_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int n = d.nx * d.ny * d.nz;
    hipLaunchKernelGGL(k_gen_coef, dim3(grid_for(n)), dim3(kThreads), 0, s, cf, xstar, m, seed, recipe);
    S7_CHECK_LAUNCH();
    if (b) {
        hipLaunchKernelGGL(k_apply_f64, dim3(cell_blocks_for(n)), dim3(kThreads), 0, s, cf,
                           (const double*)xstar, b, m, n);
        S7_CHECK_LAUNCH();
    }
    return S7_OK;
}

size_t s7_batched_workspace_bytes(int32_t nsys, const s7_dims* d, int32_t prec, const s7_options* opt) {
    if (nsys < 1 || !d || prec < S7_FP32 || prec > S7_FP16_IR) return 0;
    s7_options o;
    options_or_default(opt, o);
    size_t total = align256(engine_table_bytes(nsys));
    for (int i = 0; i < nsys; ++i) {
        if (!dims_ok(d[i])) return 0;
        total += align256(make_layout(d[i], prec, o).bytes);
    }
    return total;
}

int s7_bicgstab_solve_batched(int32_t nsys, const s7_dims* d, const float* const* coef,
                              const double* const* b, double* const* x, const double* rtol,
                              const int32_t* max_iter, int32_t prec, void* ws, size_t ws_bytes,
                              const s7_options* opt, s7_info* info, void* stream) {
    clear_error();
    s7_options o;
    options_or_default(opt, o);
    if (nsys < 1 || !d || !coef || !b || !x || !rtol || !max_iter || !ws ||
        ((uintptr_t)ws & 255u) != 0 || prec < S7_FP32 || prec > S7_FP16_IR) {
        set_error("s7_bicgstab_solve_batched: invalid argument");
        return S7_EINVAL;
    }
    for (int i = 0; i < nsys; ++i) {
        bool ok = dims_ok(d[i]) && b[i] && x[i] && rtol[i] > 0.0 && max_iter[i] >= 0;
        for (int a = 0; a < 7 && ok; ++a) ok = coef[7 * i + a] != nullptr;
        if (!ok) {
            set_error("s7_bicgstab_solve_batched: invalid argument for system %d", i);
            return S7_EINVAL;
        }
    }
    const size_t need = s7_batched_workspace_bytes(nsys, d, prec, &o);
    if (ws_bytes < need) {
        set_error("s7_bicgstab_solve_batched: workspace too small (%zu < %zu)", ws_bytes, need);
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
        j.d = d[i];
        for (int a = 0; a < 7; ++a) j.coef[a] = coef[7 * i + a];
        j.b = b[i];
        j.x = x[i];
        j.rtol = rtol[i];
        j.max_iter = max_iter[i];
        j.prec = prec;
        j.ws = w + off;
        j.ws_bytes = make_layout(d[i], prec, o).bytes;
        j.t_start_ms = t0;
        big[i] = (long long)d[i].nx * d[i].ny * d[i].nz >= split;
        off += align256(j.ws_bytes);
    }
    return run_batch(jobs, big, OP_7PT, w, o, (hipStream_t)stream, info, "s7_bicgstab_solve_batched",
                     [&](EngineJob& j) {
                         return s7_bicgstab_solve(j.d, j.coef, j.b, j.x, j.rtol, j.max_iter, prec, j.ws,
                                                  j.ws_bytes, &o, &j.info, stream);
                     });
}

}  // extern "C"

// The 2D 9-point operator (section IV, "SpMV (2D)"), on the same machinery.
#include "s7_stencil9.hpp"
// Pipelined BiCGStab (one reduction per iteration), on the 7-point operator.
#include "s7_pipelined.hpp"
// Pipelined BiCGStab for many systems in one persistent launch.
#include "s7_batched_pipe.hpp"
