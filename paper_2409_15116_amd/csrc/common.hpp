// Shared definitions of the HIP library: complex helpers, error plumbing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/bse.h"

namespace bse {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
const char *last_error();

struct Err {
    bse_status st;
};

#define BSE_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::bse::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                  \
            throw ::bse::Err{BSE_ERR_HIP};                                         \
        }                                                                          \
    } while (0)

#define BSE_LAUNCH_CHECK()                                                         \
    do {                                                                           \
        hipError_t e_ = hipGetLastError();                                         \
        if (e_ != hipSuccess) {                                                    \
            ::bse::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                  \
            throw ::bse::Err{BSE_ERR_HIP};                                         \
        }                                                                          \
    } while (0)

#define BSE_REQUIRE(cond, code, ...)                                               \
    do {                                                                           \
        if (!(cond)) {                                                             \
            ::bse::set_error(__VA_ARGS__);                                         \
            throw ::bse::Err{code};                                                \
        }                                                                          \
    } while (0)

// ---------------------------------------------------------------- complex
template <typename T> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename T> using cplx = typename cplx_t<T>::type;

template <typename C> __host__ __device__ inline C cmake(decltype(C::x) a, decltype(C::x) b) {
    C r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename C> __device__ inline C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ inline C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ inline C cmul(C a, C b) {
    return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ inline C cconj(C a) { return cmake<C>(a.x, -a.y); }
// multiply by s*i (s = +1 or -1)
template <typename C> __device__ inline C cmul_si(C a, decltype(C::x) s) {
    return cmake<C>(-s * a.y, s * a.x);
}
template <typename C> __device__ inline C cscale(C a, decltype(C::x) s) {
    return cmake<C>(a.x * s, a.y * s);
}

inline unsigned div_up(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace bse
