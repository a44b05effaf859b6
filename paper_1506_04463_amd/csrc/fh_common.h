// Shared device/host helpers of the feasthip library: complex arithmetic,
// error handling, device buffers.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <memory>
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
// device-memory source of a handle: the caller's allocator callbacks (e.g.
// torch's caching allocator) or, without them, hipMalloc / hipFree.  Every
// entry point makes its handle's source current on the calling thread
// (MemScope); a DBuf allocates from the current source and keeps a reference
// to it for the free, so a buffer may outlive the call (and the handle) that
// allocated it.
// ---------------------------------------------------------------------------
struct MemSource {
    void* (*alloc)(size_t bytes, void* stream, void* user) = nullptr;
    void (*free)(void* ptr, size_t bytes, void* stream, void* user) = nullptr;
    void* user = nullptr;
    void* stream = nullptr;   // the handle's stream (updated at every call)
};
using MemSourceP = std::shared_ptr<MemSource>;
inline MemSourceP& tl_mem() {
    static thread_local MemSourceP m;
    return m;
}
struct MemScope {
    MemSourceP prev;
    MemScope(const MemSourceP& m, void* stream) : prev(tl_mem()) {
        if (m) m->stream = stream;
        tl_mem() = m;
    }
    ~MemScope() { tl_mem() = prev; }
};

// ---------------------------------------------------------------------------
// device buffer (grow-only)
// ---------------------------------------------------------------------------
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    MemSourceP src;           // the source p came from (null: hipMalloc)
    void* st = nullptr;       // stream passed to the source's alloc
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) {
            if (src && src->free) {
                // hipFree waits for the device; a caller's allocator may hand the
                // block out again at once, so wait for work still using it
                (void)hipDeviceSynchronize();
                src->free(p, bytes, st, src->user);
            } else {
                (void)hipFree(p);
            }
        }
        p = nullptr;
        bytes = 0;
        src.reset();
        st = nullptr;
    }
    void* ensure(size_t b) {
        if (b <= bytes && p) return p;
        release();
        if (b == 0) b = 256;
        const MemSourceP& m = tl_mem();
        if (m && m->alloc) {
            p = m->alloc(b, m->stream, m->user);
            if (!p) throw Error(100, "device allocator returned no memory for " + std::to_string(b) + " bytes");
            src = m;
            st = m->stream;
        } else {
            FH_HIP(hipMalloc(&p, b));
        }
        bytes = b;
        return p;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

inline unsigned ceil_div(size_t a, size_t b) { return unsigned((a + b - 1) / b); }

}  // namespace fh
