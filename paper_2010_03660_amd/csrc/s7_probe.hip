// STREAM-style bandwidth probes (McCalpin's STREAM kernels: copy, triad, plus a
// read-only sum and an 6-read/2-write pattern shaped like the P3 update).  They
// measure the HBM rate that plain streaming code reaches on this device, the
// practical ceiling that the roofline fractions of the solver kernels are read
// against.
#include "s7_host.hpp"

namespace s7 {

typedef float pf2 __attribute__((ext_vector_type(2)));
typedef float pf4 __attribute__((ext_vector_type(4)));

template <int W>
struct VecF;
template <>
struct VecF<1> {
    using T = float;
};
template <>
struct VecF<2> {
    using T = pf2;
};
template <>
struct VecF<4> {
    using T = pf4;
};

__device__ __forceinline__ float vsum(float a) { return a; }
__device__ __forceinline__ float vsum(pf2 a) { return a.x + a.y; }
__device__ __forceinline__ float vsum(pf4 a) { return (a.x + a.y) + (a.z + a.w); }

__device__ __forceinline__ float vfma(float s, float a, float b) { return __builtin_fmaf(s, a, b); }
__device__ __forceinline__ pf2 vfma(float s, pf2 a, pf2 b) {
    pf2 r;
    r.x = __builtin_fmaf(s, a.x, b.x);
    r.y = __builtin_fmaf(s, a.y, b.y);
    return r;
}
__device__ __forceinline__ pf4 vfma(float s, pf4 a, pf4 b) {
    pf4 r;
    r.x = __builtin_fmaf(s, a.x, b.x);
    r.y = __builtin_fmaf(s, a.y, b.y);
    r.z = __builtin_fmaf(s, a.z, b.z);
    r.w = __builtin_fmaf(s, a.w, b.w);
    return r;
}

// kind & 3: 0 sum(a), 1 c = a, 2 c = a + s b, 3 six reads and two writes
// kind & 4: non-temporal stores; kind & 8: non-temporal loads
// (a..f read, a and b written back: the access pattern of the BiCGStab x/r update)
template <class T, bool NT>
__device__ __forceinline__ T ldv(const T* p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}
template <class T, bool NT>
__device__ __forceinline__ void stv(T* p, T v) {
    if (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <int W, bool NTL, bool NTS>
__global__ __launch_bounds__(256) void k_probe(int kind, float* a, float* b, float* c,
                                               size_t nvec, float* sink) {
    using T = typename VecF<W>::T;
    T* A = reinterpret_cast<T*>(a);
    T* B = reinterpret_cast<T*>(b);
    T* Cw = reinterpret_cast<T*>(c);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    float acc = 0.f;
    if (kind == 0) {
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride)
            acc += vsum(ldv<T, NTL>(A + i));
    } else if (kind == 1) {
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride)
            stv<T, NTS>(Cw + i, ldv<T, NTL>(A + i));
    } else if (kind == 2) {
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride)
            stv<T, NTS>(Cw + i, vfma(0.5f, ldv<T, NTL>(B + i), ldv<T, NTL>(A + i)));
    } else {
        // six streams carved from the three buffers: a = [a0 | a1], b = [b0 | b1], c = [c0 | c1]
        const size_t h = nvec / 2;
        T* A0 = A;
        T* B0 = B;
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < h; i += stride) {
            T x0 = ldv<T, NTL>(A0 + i), x1 = ldv<T, NTL>(A0 + i + h);
            T y0 = ldv<T, NTL>(B0 + i), y1 = ldv<T, NTL>(B0 + i + h);
            T z0 = ldv<T, NTL>(Cw + i), z1 = ldv<T, NTL>(Cw + i + h);
            T q = vfma(-0.5f, y0, x0);
            stv<T, NTS>(A0 + i, vfma(0.25f, z0, vfma(0.5f, y1, x1)));
            stv<T, NTS>(B0 + i, vfma(-0.5f, z1, q));
        }
    }
    if (acc == 12345.678f) sink[0] = acc;  // keeps the read-only loop alive
}

}  // namespace s7

using namespace s7;

extern "C" int s7_bandwidth_probe(int32_t kind, int32_t width, float* a, float* b, float* c,
                                  size_t n, int32_t blocks, void* stream) {
    clear_error();
    const int base = kind & 3;
    const bool ntl = (kind & 8) != 0, nts = (kind & 4) != 0;
    if (kind < 0 || kind > 15 || !(width == 1 || width == 2 || width == 4) || !a || blocks < 1 ||
        (base >= 1 && !c) || (base >= 2 && !b) || n % 8 != 0) {
        set_error("s7_bandwidth_probe: invalid argument");
        return S7_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t nvec = n / width;
    float* sink = c ? c : a;
#define S7_PROBE_LAUNCH(W, L, S) \
    hipLaunchKernelGGL((k_probe<W, L, S>), dim3(blocks), dim3(256), 0, s, base, a, b, c, nvec, sink)
#define S7_PROBE_W(W)                            \
    do {                                         \
        if (ntl && nts) S7_PROBE_LAUNCH(W, true, true);   \
        else if (ntl) S7_PROBE_LAUNCH(W, true, false);    \
        else if (nts) S7_PROBE_LAUNCH(W, false, true);    \
        else S7_PROBE_LAUNCH(W, false, false);            \
    } while (0)
    if (width == 1)
        S7_PROBE_W(1);
    else if (width == 2)
        S7_PROBE_W(2);
    else
        S7_PROBE_W(4);
#undef S7_PROBE_W
#undef S7_PROBE_LAUNCH
    S7_CHECK_LAUNCH();
    return S7_OK;
}
