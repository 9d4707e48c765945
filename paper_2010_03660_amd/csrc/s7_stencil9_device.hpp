// Device building blocks of the 2D 9-point operator (section IV, "SpMV
// (2D)"): on an nx x ny mesh, row (i,j) holds the main diagonal and eight
// off-diagonals in the order {diag, w, e, s, n, sw, se, nw, ne}.  Shared by
// the single-system solver and the persistent kernel.
#pragma once

#include "s7_device.hpp"

namespace s7 {

// Nine coefficient arrays in the order {diag, w, e, s, n, sw, se, nw, ne}:
// the caller's (FP32), or the working copies in the storage type T.
template <class T>
struct Coef9T {
    const T* c[9];
};
using Coef9 = Coef9T<float>;

// Offsets of the nine points from the cell; an off-mesh neighbour maps to the
// cell itself (its coefficient is zero or masked).
__device__ __forceinline__ void offsets9(const Cell& c, int (&o)[9]) {
    o[0] = 0;
    o[1] = c.dw;
    o[2] = c.de;
    o[3] = c.ds;
    o[4] = c.dn;
    o[5] = (c.dw && c.ds) ? c.dw + c.ds : 0;
    o[6] = (c.de && c.ds) ? c.de + c.ds : 0;
    o[7] = (c.dw && c.dn) ? c.dw + c.dn : 0;
    o[8] = (c.de && c.dn) ? c.de + c.dn : 0;
}

// Whether each of the nine links stays in the mesh.
__device__ __forceinline__ void inside9(const Cell& c, bool (&in)[9]) {
    in[0] = true;
    in[1] = c.dw != 0;
    in[2] = c.de != 0;
    in[3] = c.ds != 0;
    in[4] = c.dn != 0;
    in[5] = in[1] && in[3];
    in[6] = in[2] && in[3];
    in[7] = in[1] && in[4];
    in[8] = in[2] && in[4];
}

template <class V>
__device__ __forceinline__ void load9(const V* v, const Cell& c, V (&x)[9]) {
    int o[9];
    offsets9(c, o);
    const V* p = v + c.idx;
#pragma unroll
    for (int a = 0; a < 9; ++a) x[a] = p[o[a]];
}

// The nine values of a working vector in storage type T, widened to FP32.
template <class T>
__device__ __forceinline__ void load9f(const T* v, const Cell& c, float (&x)[9]) {
    int o[9];
    offsets9(c, o);
    const T* p = v + c.idx;
#pragma unroll
    for (int a = 0; a < 9; ++a) x[a] = to_f32(p[o[a]]);
}

__device__ __forceinline__ float fma9(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma9(double a, double b, double c) { return fma(a, b, c); }

// (A v) at one cell with the caller's coefficients; outward links masked.
// Terms in the order diag, w, e, s, n, sw, se, nw, ne.
template <class V>
__device__ __forceinline__ V apply9_masked(const Coef9& cf, const Cell& c, const V (&x)[9]) {
    bool in[9];
    inside9(c, in);
    V acc = (V)*gbl(cf.c[0] + c.idx) * x[0];
#pragma unroll
    for (int a = 1; a < 9; ++a) acc = fma9(in[a] ? (V)*gbl(cf.c[a] + c.idx) : (V)0, x[a], acc);
    return acc;
}

// (A v) at one cell with the working copies (outward links already zero).
// UNIT: Jacobi-scaled, the diagonal is one and c[0] is not stored.
template <class T, bool UNIT>
__device__ __forceinline__ float apply9_work(const Coef9T<T>& k, int idx, const float (&x)[9]) {
    float acc = UNIT ? x[0] : to_f32(ld_nt(k.c[0] + idx)) * x[0];
#pragma unroll
    for (int a = 1; a < 9; ++a) acc = fma9(to_f32(ld_nt(k.c[a] + idx)), x[a], acc);
    return acc;
}

// The caller's nine coefficient arrays of a 2D system: the first seven travel
// in a Coef7, the last two beside it.
__host__ __device__ inline Coef9 coef9_of(const Coef7& c7, const float* const (&extra)[2]) {
    Coef9 k;
    for (int a = 0; a < 7; ++a) k.c[a] = c7.c[a];
    k.c[7] = extra[0];
    k.c[8] = extra[1];
    return k;
}

}  // namespace s7
