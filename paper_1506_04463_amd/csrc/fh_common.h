// Shared device/host helpers of the feasthip library: complex arithmetic,
// error handling, device buffers.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

namespace fh {

// ---------------------------------------------------------------------------
// complex numbers: interleaved (re, im), 2*sizeof(T) aligned so that a pair
// moves in one vector load
// ---------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) Cx {
    T re, im;
};
using zd = Cx<double>;
using cf = Cx<float>;

template <typename T> __host__ __device__ __forceinline__ Cx<T> cx(T r, T i) { return Cx<T>{r, i}; }
template <typename T> __host__ __device__ __forceinline__ Cx<T> czero() { return Cx<T>{T(0), T(0)}; }
template <typename T> __host__ __device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ __forceinline__ Cx<T> operator-(Cx<T> a) { return {-a.re, -a.im}; }
template <typename T> __host__ __device__ __forceinline__ Cx<T> operator*(Cx<T> a, Cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ __forceinline__ Cx<T> operator*(T s, Cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ __forceinline__ Cx<T> conj(Cx<T> a) { return {a.re, -a.im}; }
template <typename T> __host__ __device__ __forceinline__ T abs2(Cx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T> __host__ __device__ __forceinline__ T cabs(Cx<T> a) { return hypot(a.re, a.im); }
// |re| + |im|  (LAPACK's cabs1, used for pivoting and deflation tests)
template <typename T> __host__ __device__ __forceinline__ T cabs1(Cx<T> a) { return fabs(a.re) + fabs(a.im); }
// a / b, scaled to avoid overflow (Smith's method)
template <typename T> __host__ __device__ __forceinline__ Cx<T> cdiv(Cx<T> a, Cx<T> b) {
    if (fabs(b.re) >= fabs(b.im)) {
        T r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    } else {
        T r = b.re / b.im, d = b.im + b.re * r;
        return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
    }
}
// principal square root
template <typename T> __host__ __device__ __forceinline__ Cx<T> csqrt(Cx<T> a) {
    T m = hypot(a.re, a.im);
    if (m == T(0)) return {T(0), T(0)};
    T r = sqrt(T(0.5) * (m + fabs(a.re)));
    if (a.re >= T(0)) return {r, a.im / (T(2) * r)};
    return {fabs(a.im) / (T(2) * r), a.im >= T(0) ? r : -r};
}
// acc += a * b  /  acc -= a * b  /  acc += conj(a) * b
template <typename T> __host__ __device__ __forceinline__ void cfma(Cx<T>& acc, Cx<T> a, Cx<T> b) {
    acc.re = fma(a.re, b.re, acc.re); acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im); acc.im = fma(a.im, b.re, acc.im);
}
template <typename T> __host__ __device__ __forceinline__ void cfms(Cx<T>& acc, Cx<T> a, Cx<T> b) {
    acc.re = fma(-a.re, b.re, acc.re); acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(-a.re, b.im, acc.im); acc.im = fma(-a.im, b.re, acc.im);
}
template <typename T> __host__ __device__ __forceinline__ void cfma_conj(Cx<T>& acc, Cx<T> a, Cx<T> b) {
    acc.re = fma(a.re, b.re, acc.re); acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im); acc.im = fma(-a.im, b.re, acc.im);
}
template <typename T, typename S> __host__ __device__ __forceinline__ Cx<T> ccast(Cx<S> a) { return {T(a.re), T(a.im)}; }

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define FH_HIP(call)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            throw ::fh::Error(100, std::string(#call) + ": " + hipGetErrorString(e_) + " at " + \
                                       __FILE__ + ":" + std::to_string(__LINE__));              \
    } while (0)

#define FH_LAUNCH_CHECK() FH_HIP(hipGetLastError())

#define FH_REQUIRE(cond, code, msg)                  \
    do {                                             \
        if (!(cond)) throw ::fh::Error((code), (msg)); \
    } while (0)

// ---------------------------------------------------------------------------
// device buffer (grow-only)
// ---------------------------------------------------------------------------
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void* ensure(size_t b) {
        if (b <= bytes && p) return p;
        release();
        if (b == 0) b = 256;
        FH_HIP(hipMalloc(&p, b));
        bytes = b;
        return p;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

inline unsigned ceil_div(size_t a, size_t b) { return unsigned((a + b - 1) / b); }

}  // namespace fh
