// Shared device and host helpers of libttsvd (gfx950 / CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cfloat>

#include "ttsvd.h"

namespace ttsvd {

constexpr int kWave = 64;

// ------------------------------------------------------------ element types

// Storage type tag for bfloat16 (raw bits; round-to-nearest-even on store).
struct bf16 {
    uint16_t bits;
};

template <typename T> struct Elem;
template <> struct Elem<double> {
    using acc = double;
    __device__ static inline double load(const double *p) { return *p; }
    __device__ static inline void store(double *p, double v) { *p = v; }
};
template <> struct Elem<float> {
    using acc = float;
    __device__ static inline float load(const float *p) { return *p; }
    __device__ static inline void store(float *p, float v) { *p = v; }
};
template <> struct Elem<bf16> {
    using acc = float;
    __device__ static inline float load(const bf16 *p) {
        return __uint_as_float(static_cast<uint32_t>(p->bits) << 16);
    }
    __device__ static inline void store(bf16 *p, float v) {
        uint32_t u = __float_as_uint(v);
        // round to nearest, ties to even; NaN stays NaN (quiet bit kept)
        uint32_t r = ((u >> 16) & 1u) + 0x7fffu;
        uint32_t o = ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu))
                         ? ((u >> 16) | 0x40u)
                         : ((u + r) >> 16);
        p->bits = static_cast<uint16_t>(o);
    }
};

// Smallest positive normalized number of the accumulation type: the eps_FP
// safeguard of the Householder reflector (Algorithm 6).
template <typename T> struct EpsFP;
template <> struct EpsFP<double> {
    __device__ static constexpr double value() { return DBL_MIN; }
};
template <> struct EpsFP<float> {
    __device__ static constexpr float value() { return FLT_MIN; }
};

__device__ inline double dev_sqrt(double x) { return __builtin_sqrt(x); }
__device__ inline float dev_sqrt(float x) { return __builtin_sqrtf(x); }

// ------------------------------------------------------- wave reductions

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

constexpr int cpow2(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}
constexpr int clog2(int n) {
    int q = 0;
    while ((1 << q) < n) ++q;
    return q;
}

// All-reduce of N values per lane over the 64 lanes of a wave.  On return
// every lane holds the N sums in p[].  Reduce-scatter by recursive halving
// (lane bit 5 keeps the upper half of the list at the first stage, bit 4 at
// the second, ...), a butterfly over the remaining lane bits, then an
// all-gather through lds (>= cpow2(N) values of per-wave scratch).
template <int N, typename T>
__device__ inline void wave_allreduce_vec(T (&p)[N], T *lds) {
    constexpr int NP = cpow2(N);
    constexpr int Q = clog2(NP);
    static_assert(NP <= kWave, "at most 64 values");
    const int lane = lane_id();
    T b[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) b[i] = (i < N) ? p[i] : T(0);
#pragma unroll
    for (int t = 0; t < Q; ++t) {
        const int d = 32 >> t;
        const int half = NP >> (t + 1);
        const bool hi = (lane & d) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            T send = hi ? b[i] : b[half + i];
            T keep = hi ? b[half + i] : b[i];
            b[i] = keep + __shfl_xor(send, d, kWave);
        }
    }
#pragma unroll
    for (int d = (32 >> Q); d >= 1; d >>= 1) b[0] += __shfl_xor(b[0], d, kWave);
    const int key = lane >> (6 - Q);
    if ((lane & ((64 >> Q) - 1)) == 0) lds[key] = b[0];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int i = 0; i < N; ++i) p[i] = lds[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace ttsvd

// ----------------------------------------------------------- host helpers

namespace ttsvd {

// Records msg as the calling thread's last error and returns code.
int set_error(int code, const char *fmt, ...);
void clear_error();

#define TTSVD_HIP_TRY(expr)                                                    \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess)                                                  \
            return ::ttsvd::set_error(TTSVD_EHIP, "%s failed: %s (%s:%d)",     \
                                      #expr, hipGetErrorString(e_), __FILE__,  \
                                      __LINE__);                               \
    } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline size_t dtype_size(int dt) {
    return dt == TTSVD_F64 ? 8 : dt == TTSVD_F32 ? 4 : dt == TTSVD_BF16 ? 2 : 0;
}

}  // namespace ttsvd
