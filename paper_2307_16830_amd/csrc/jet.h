// Second-order forward-mode automatic differentiation for the model templates (Section III-B: derivatives of
// the repeated templates are generated from their value expressions, not derived by hand).
//
// Jet<K> carries a value, its gradient and the lower triangle of its Hessian with respect to K local inputs of
// one template instance.  Arithmetic and the elementary functions the ACOPF templates use propagate all three
// by the chain and product rules, so a template written once as a function of a generic number type yields
// its value (instantiated with double), its Jacobian entries (the gradient) and its Hessian entries (the
// lower triangle, index (i, j), i >= j, at i (i + 1) / 2 + j) in one evaluation.
#pragma once

#include <hip/hip_runtime.h>

namespace opf {

template <int K>
struct Jet {
    static constexpr int NH = K * (K + 1) / 2;
    double v;
    double g[K];
    double h[NH];
    __device__ __forceinline__ static constexpr int hi(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }
    __device__ __forceinline__ Jet() : v(0.0) {
#pragma unroll
        for (int i = 0; i < K; i++) g[i] = 0.0;
#pragma unroll
        for (int q = 0; q < NH; q++) h[q] = 0.0;
    }
    __device__ __forceinline__ Jet(double c) : Jet() { v = c; }
    // the k-th independent input with value x
    __device__ __forceinline__ static Jet input(double x, int k) {
        Jet r(x);
        r.g[k] = 1.0;
        return r;
    }
};

template <int K>
__device__ __forceinline__ Jet<K> operator+(const Jet<K>& a, const Jet<K>& b) {
    Jet<K> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < K; i++) r.g[i] = a.g[i] + b.g[i];
#pragma unroll
    for (int q = 0; q < Jet<K>::NH; q++) r.h[q] = a.h[q] + b.h[q];
    return r;
}

template <int K>
__device__ __forceinline__ Jet<K> operator-(const Jet<K>& a, const Jet<K>& b) {
    Jet<K> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < K; i++) r.g[i] = a.g[i] - b.g[i];
#pragma unroll
    for (int q = 0; q < Jet<K>::NH; q++) r.h[q] = a.h[q] - b.h[q];
    return r;
}

template <int K>
__device__ __forceinline__ Jet<K> operator-(const Jet<K>& a) {
    Jet<K> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < K; i++) r.g[i] = -a.g[i];
#pragma unroll
    for (int q = 0; q < Jet<K>::NH; q++) r.h[q] = -a.h[q];
    return r;
}

template <int K>
__device__ __forceinline__ Jet<K> operator*(double c, const Jet<K>& a) {
    Jet<K> r;
    r.v = c * a.v;
#pragma unroll
    for (int i = 0; i < K; i++) r.g[i] = c * a.g[i];
#pragma unroll
    for (int q = 0; q < Jet<K>::NH; q++) r.h[q] = c * a.h[q];
    return r;
}

template <int K>
__device__ __forceinline__ Jet<K> operator*(const Jet<K>& a, double c) { return c * a; }

template <int K>
__device__ __forceinline__ Jet<K> operator+(const Jet<K>& a, double c) {
    Jet<K> r = a;
    r.v += c;
    return r;
}

template <int K>
__device__ __forceinline__ Jet<K> operator+(double c, const Jet<K>& a) { return a + c; }

// product rule: (ab)' = a'b + ab',  (ab)'' = a''b + a'b'^T + b'a'^T + ab''
template <int K>
__device__ __forceinline__ Jet<K> operator*(const Jet<K>& a, const Jet<K>& b) {
    Jet<K> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < K; i++) r.g[i] = a.g[i] * b.v + a.v * b.g[i];
#pragma unroll
    for (int i = 0; i < K; i++)
#pragma unroll
        for (int j = 0; j <= i; j++) {
            const int q = Jet<K>::hi(i, j);
            r.h[q] = a.h[q] * b.v + a.v * b.h[q] + a.g[i] * b.g[j] + a.g[j] * b.g[i];
        }
    return r;
}

// f(a) for a scalar function with f(a.v), f'(a.v), f''(a.v) given: chain rule
template <int K>
__device__ __forceinline__ Jet<K> chain(const Jet<K>& a, double f0, double f1, double f2) {
    Jet<K> r;
    r.v = f0;
#pragma unroll
    for (int i = 0; i < K; i++) r.g[i] = f1 * a.g[i];
#pragma unroll
    for (int i = 0; i < K; i++)
#pragma unroll
        for (int j = 0; j <= i; j++) {
            const int q = Jet<K>::hi(i, j);
            r.h[q] = f1 * a.h[q] + f2 * a.g[i] * a.g[j];
        }
    return r;
}

// sine and cosine of one argument together (one sincos of the value)
template <int K>
__device__ __forceinline__ void sincos(const Jet<K>& a, Jet<K>* s, Jet<K>* c) {
    double sv, cv;
    ::sincos(a.v, &sv, &cv);
    *s = chain(a, sv, cv, -sv);
    *c = chain(a, cv, -sv, -cv);
}

__device__ __forceinline__ void sincos(double a, double* s, double* c) { ::sincos(a, s, c); }

}  // namespace opf
