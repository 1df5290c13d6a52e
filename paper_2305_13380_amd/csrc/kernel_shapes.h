// Smoothing kernels of the neighbour loops. Section 3.1 lists the Wendland
// C2, C4 and C6 functions and the cubic, quartic and quintic B-splines, with
// one smoothing length h for all of them and a kernel-dependent cut-off
// H = gamma_k h (h twice the kernel's standard deviation). In u = r/H on the
// support [0, 1]:
//
//     W(r, h)     =  kW H^-3 w(u)
//     dW/dr       = -kD H^-4 mdw(u)
//     (dW/dr) / r = -kD H^-5 phi(u),      phi(u) = mdw(u) / u
//
// kW makes W integrate to one over space; kD / kW is the factor taken out of
// -w'. The density loop needs w and phi (its gradient sums carry x_ij, and
// its h-derivative sums u^2 phi); the force loop needs mdw. Arguments are in
// [0, 1] (callers clamp u at 1, where every function vanishes). The spline
// pieces are the splines' truncated-power sums multiplied out on each
// interval between knots: no cancellation near u = 0 and no division there;
// phi divides by u only on intervals that stay away from 0. Both pieces are
// evaluated and one is picked by a bit mask: with a plain conditional the
// compiler forms predicated blocks in the unrolled pair loops, and the
// spline loops then need about 180 instead of about 128 registers.
#pragma once

#include <hip/hip_runtime.h>

namespace sphx {

enum KernelKind : int {
    kWendlandC2 = 0,
    kWendlandC4 = 1,
    kWendlandC6 = 2,
    kCubicSpline = 3,
    kQuarticSpline = 4,
    kQuinticSpline = 5,
    kKernelKinds = 6
};

// a where pick, else b, by bit masks: both operands are computed first, and
// no branch or predicated block is left for the compiler to form
__device__ __forceinline__ float pick(bool pick_a, float a, float b)
{
    const int m = -int(pick_a);
    return __int_as_float((__float_as_int(a) & m) | (__float_as_int(b) & ~m));
}

template <int K>
struct Kern;

// Wendland C2: w = (1-u)^4 (1 + 4u), -w' = 20 u (1-u)^3.
template <>
struct Kern<kWendlandC2> {
    static constexpr float kW = 3.3422538049298023f;   // 21 / (2 pi)
    static constexpr float kD = 66.845076098596050f;   // 20 kW
    __device__ static __forceinline__ float w(float u)
    {
        const float t = 1.0f - u, t2 = t * t;
        return t2 * t2 * (1.0f + 4.0f * u);
    }
    __device__ static __forceinline__ float phi(float u)
    {
        const float t = 1.0f - u;
        return t * t * t;
    }
    __device__ static __forceinline__ float mdw(float u) { return u * phi(u); }
};

// Wendland C4: w = (1-u)^6 (1 + 6u + 35/3 u^2), -w' = 56/3 u (1-u)^5 (1 + 5u).
template <>
struct Kern<kWendlandC4> {
    static constexpr float kW = 4.9238560519055130f;   // 495 / (32 pi)
    static constexpr float kD = 91.911979635569580f;   // 56/3 kW
    __device__ static __forceinline__ float w(float u)
    {
        const float t = 1.0f - u, t2 = t * t;
        return (t2 * t2) * t2 * (1.0f + u * (6.0f + (35.0f / 3.0f) * u));
    }
    __device__ static __forceinline__ float phi(float u)
    {
        const float t = 1.0f - u, t2 = t * t;
        return (t2 * t2) * t * (1.0f + 5.0f * u);
    }
    __device__ static __forceinline__ float mdw(float u) { return u * phi(u); }
};

// Wendland C6: w = (1-u)^8 (1 + 8u + 25u^2 + 32u^3),
// -w' = 22 u (1-u)^7 (1 + 7u + 16u^2).
template <>
struct Kern<kWendlandC6> {
    static constexpr float kW = 6.7889530412636600f;   // 1365 / (64 pi)
    static constexpr float kD = 149.35696690780054f;   // 22 kW
    __device__ static __forceinline__ float w(float u)
    {
        const float t = 1.0f - u, t2 = t * t, t4 = t2 * t2;
        return (t4 * t4) * (1.0f + u * (8.0f + u * (25.0f + 32.0f * u)));
    }
    __device__ static __forceinline__ float phi(float u)
    {
        const float t = 1.0f - u, t2 = t * t;
        return (t2 * t2) * (t2 * t) * (1.0f + u * (7.0f + 16.0f * u));
    }
    __device__ static __forceinline__ float mdw(float u) { return u * phi(u); }
};

// Cubic B-spline: w = (1-u)^3 - 4 (1/2-u)_+^3;
// -w' = 6u - 9u^2 below the knot, 3 (1-u)^2 above.
template <>
struct Kern<kCubicSpline> {
    static constexpr float kW = 5.0929581789406510f;   // 16 / pi
    static constexpr float kD = kW;
    __device__ static __forceinline__ float w(float u)
    {
        const float t = 1.0f - u, a = fmaxf(0.5f - u, 0.0f);
        return t * t * t - 4.0f * (a * a * a);
    }
    __device__ static __forceinline__ float phi(float u)
    {
        const float t = 1.0f - u;
        const float in = 6.0f - 9.0f * u;
        const float out = 3.0f * (t * t) * __builtin_amdgcn_rcpf(fmaxf(u, 0.5f));
        return pick(u < 0.5f, in, out);
    }
    __device__ static __forceinline__ float mdw(float u)
    {
        const float t = 1.0f - u;
        return pick(u < 0.5f, u * (6.0f - 9.0f * u), 3.0f * (t * t));
    }
};

// Quartic B-spline: w = (1-u)^4 - 5 (3/5-u)_+^4 + 10 (1/5-u)_+^4;
// -w' = 24/5 u - 24 u^3 below 1/5, 4 (1-u)^3 - 20 (3/5-u)_+^3 above.
template <>
struct Kern<kQuarticSpline> {
    static constexpr float kW = 9.7140468195736900f;   // 15625 / (512 pi)
    static constexpr float kD = kW;
    __device__ static __forceinline__ float w(float u)
    {
        const float t = 1.0f - u, a = fmaxf(0.6f - u, 0.0f), b = fmaxf(0.2f - u, 0.0f);
        const float t2 = t * t, a2 = a * a, b2 = b * b;
        return t2 * t2 - 5.0f * (a2 * a2) + 10.0f * (b2 * b2);
    }
    __device__ static __forceinline__ float outer(float u)
    {
        const float t = 1.0f - u, a = fmaxf(0.6f - u, 0.0f);
        return 4.0f * (t * t * t) - 20.0f * (a * a * a);
    }
    __device__ static __forceinline__ float phi(float u)
    {
        const float in = 4.8f - 24.0f * (u * u);
        const float out = outer(u) * __builtin_amdgcn_rcpf(fmaxf(u, 0.2f));
        return pick(u < 0.2f, in, out);
    }
    __device__ static __forceinline__ float mdw(float u)
    {
        return pick(u < 0.2f, u * (4.8f - 24.0f * (u * u)), outer(u));
    }
};

// Quintic B-spline: w = (1-u)^5 - 6 (2/3-u)_+^5 + 15 (1/3-u)_+^5;
// -w' = 40/9 u - 40 u^3 + 50 u^4 below 1/3, 5 (1-u)^4 - 30 (2/3-u)_+^4 above.
template <>
struct Kern<kQuinticSpline> {
    static constexpr float kW = 17.403593027098754f;   // 2187 / (40 pi)
    static constexpr float kD = kW;
    __device__ static __forceinline__ float w(float u)
    {
        const float t = 1.0f - u, a = fmaxf((2.0f / 3.0f) - u, 0.0f),
                    b = fmaxf((1.0f / 3.0f) - u, 0.0f);
        const float t2 = t * t, a2 = a * a, b2 = b * b;
        return (t2 * t2) * t - 6.0f * ((a2 * a2) * a) + 15.0f * ((b2 * b2) * b);
    }
    __device__ static __forceinline__ float outer(float u)
    {
        const float t = 1.0f - u, a = fmaxf((2.0f / 3.0f) - u, 0.0f);
        const float t2 = t * t, a2 = a * a;
        return 5.0f * (t2 * t2) - 30.0f * (a2 * a2);
    }
    __device__ static __forceinline__ float inner(float u)
    {
        return (40.0f / 9.0f) + (u * u) * (50.0f * u - 40.0f);
    }
    __device__ static __forceinline__ float phi(float u)
    {
        const float in = inner(u);
        const float out = outer(u) * __builtin_amdgcn_rcpf(fmaxf(u, 1.0f / 3.0f));
        return pick(u < (1.0f / 3.0f), in, out);
    }
    __device__ static __forceinline__ float mdw(float u)
    {
        return pick(u < (1.0f / 3.0f), u * inner(u), outer(u));
    }
};

}  // namespace sphx

// Runs CALL with the constant KK set to the kernel kind k (host code; the
// context has checked that k is one of the kinds).
#define SPHX_WITH_KERNEL(k, CALL)                                                        \
    switch (k) {                                                                         \
    case ::sphx::kWendlandC2: { constexpr int KK = ::sphx::kWendlandC2; CALL; } break;     \
    case ::sphx::kWendlandC4: { constexpr int KK = ::sphx::kWendlandC4; CALL; } break;     \
    case ::sphx::kWendlandC6: { constexpr int KK = ::sphx::kWendlandC6; CALL; } break;     \
    case ::sphx::kCubicSpline: { constexpr int KK = ::sphx::kCubicSpline; CALL; } break;   \
    case ::sphx::kQuarticSpline: { constexpr int KK = ::sphx::kQuarticSpline; CALL; } break; \
    default: { constexpr int KK = ::sphx::kQuinticSpline; CALL; } break;                  \
    }
