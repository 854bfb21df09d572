// Shared device and host helpers of libttsvd (gfx950 / CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cfloat>
#include <type_traits>

#include "ttsvd.h"

namespace ttsvd {

constexpr int kWave = 64;

// ------------------------------------------------------------ element types

// Storage type tag for bfloat16 (raw bits; round-to-nearest-even on store).
struct bf16 {
    uint16_t bits;
};

template <typename T> struct Elem;
// load / store widen and narrow between the storage and accumulation types;
// round(v) is the value that store(p, v) leaves for a later load(p).
template <> struct Elem<double> {
    using acc = double;
    __device__ static inline double load(const double *p) { return *p; }
    __device__ static inline void store(double *p, double v) { *p = v; }
    __device__ static inline double round(double v) { return v; }
};
template <> struct Elem<float> {
    using acc = float;
    __device__ static inline float load(const float *p) { return *p; }
    __device__ static inline void store(float *p, float v) { *p = v; }
    __device__ static inline float round(float v) { return v; }
};
template <> struct Elem<bf16> {
    using acc = float;
    __device__ static inline float load(const bf16 *p) {
        return __uint_as_float(static_cast<uint32_t>(p->bits) << 16);
    }
    // bf16 bits of v: round to nearest, ties to even; NaN stays NaN (quiet bit kept)
    __device__ static inline uint32_t bits(float v) {
        uint32_t u = __float_as_uint(v);
        uint32_t r = ((u >> 16) & 1u) + 0x7fffu;
        return ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) ? ((u >> 16) | 0x40u)
                                                                      : ((u + r) >> 16);
    }
    __device__ static inline void store(bf16 *p, float v) {
        p->bits = static_cast<uint16_t>(bits(v));
    }
    __device__ static inline float round(float v) { return __uint_as_float(bits(v) << 16); }
};

// *p widened to the accumulation type if ok, else zero.  p must be a valid
// address whatever ok is (callers clamp the index): the load is then issued
// unconditionally and the zero is a select, so the independent loads of a
// tile stay in flight together.  (A load guarded by ok becomes a branch per
// load, and for bf16 the widening shift inside that branch waits for the
// load before the next one can issue.)
template <typename Tin>
__device__ __forceinline__ typename Elem<Tin>::acc load_or_zero(const Tin *p, bool ok) {
    using A = typename Elem<Tin>::acc;
    const A v = Elem<Tin>::load(p);
    return ok ? v : A(0);
}

// Smallest positive normalized number of the accumulation type: the eps_FP
// safeguard of the Householder reflector (Algorithm 6).
template <typename T> struct EpsFP;
template <> struct EpsFP<double> {
    __device__ static constexpr double value() { return DBL_MIN; }
};
template <> struct EpsFP<float> {
    __device__ static constexpr float value() { return FLT_MIN; }
};

// 1/sqrt(x) and 1/x from the hardware estimates refined by Newton steps
// (x normal and positive; each step squares the relative error): two steps
// in FP64, one in FP32.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}
__device__ __forceinline__ float rsqrt_nr(float x) {
    float y = __builtin_amdgcn_rsqf(x);
    const float e = fmaf(-x * y, y, 1.0f);
    return fmaf(0.5f * y, e, y);
}
// One Newton step only (relative error ~2^-48 from the ~2^-24 estimates):
// enough where the value steers an iteration rather than entering a result.
__device__ __forceinline__ double rsqrt_nr1(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}
__device__ __forceinline__ double rcp_nr1(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
__device__ __forceinline__ float rcp_nr(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

__device__ inline double dev_sqrt(double x) { return __builtin_sqrt(x); }
__device__ inline float dev_sqrt(float x) { return __builtin_sqrtf(x); }

// ------------------------------------------------------- wave reductions

// threadIdx.x.  A translation unit that defines TTSVD_PERSISTENT_KERNEL (the
// batched persistent kernel, compiled into its own code object) puts it behind
// an empty asm statement: values derived from it are then computed where a
// body uses them instead of being hoisted to the start of the kernel, where
// those of every inlined body would be live at once.  The statement emits no
// instruction.
__device__ __forceinline__ int thread_id() {
    int t = (int)threadIdx.x;
#ifdef TTSVD_PERSISTENT_KERNEL
    __asm__ volatile("" : "+v"(t));
#endif
    return t;
}

__device__ inline int lane_id() { return thread_id() & (kWave - 1); }


__host__ __device__ __forceinline__ constexpr int cpow2(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}
__host__ __device__ __forceinline__ constexpr int clog2(int n) {
    int q = 0;
    while ((1 << q) < n) ++q;
    return q;
}

// Compile-time loop: calls f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Halving exchange across lane halves (distance 32) or across 16-lane rows
// within each half (distance 16) with the gfx950 permlane swaps: lanes whose
// distance bit is 0 return lo(l) + lo(partner), the others hi(partner) + hi(l).
template <int D>
__device__ __forceinline__ uint32_t swap_u32_lo(uint32_t lo, uint32_t hi, uint32_t &hi_out) {
    if constexpr (D == 32) {
        auto r = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
        hi_out = r[1];
        return r[0];
    } else {
        auto r = __builtin_amdgcn_permlane16_swap(lo, hi, false, false);
        hi_out = r[1];
        return r[0];
    }
}
template <int D>
__device__ __forceinline__ double swap_add(double lo, double hi) {
    uint32_t h0, h1;
    const uint32_t l0 = swap_u32_lo<D>(__double2loint(lo), __double2loint(hi), h0);
    const uint32_t l1 = swap_u32_lo<D>(__double2hiint(lo), __double2hiint(hi), h1);
    return __hiloint2double(l1, l0) + __hiloint2double(h1, h0);
}
template <int D>
__device__ __forceinline__ float swap_add(float lo, float hi) {
    uint32_t h0;
    const uint32_t l0 = swap_u32_lo<D>(__float_as_uint(lo), __float_as_uint(hi), h0);
    return __uint_as_float(l0) + __uint_as_float(h0);
}

// DPP lane exchange inside 16-lane rows (VALU latency, no LDS traffic).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, true));
}

// Value of the partner lane at "distance" D < 16.  Each control is a perfect
// matching that pairs the lanes with bit D clear with those with bit D set:
// D = 1, 2: quad_perm xor; D = 4: row_half_mirror (i <-> 7 - i in each 8
// lanes); D = 8: row_ror:8 (i <-> i ^ 8 in each 16 lanes).
template <int D, typename T>
__device__ __forceinline__ T partner(T x) {
    static_assert(D == 1 || D == 2 || D == 4 || D == 8, "distance");
    if constexpr (D == 1) return dpp_mov<0xB1>(x);
    else if constexpr (D == 2) return dpp_mov<0x4E>(x);
    else if constexpr (D == 4) return dpp_mov<0x141>(x);
    else return dpp_mov<0x128>(x);
}

// x + (value of the partner lane at distance D), D in {1, 2, 4, 8, 16, 32}.
template <int D, typename T>
__device__ __forceinline__ T butterfly_add(T x) {
    if constexpr (D >= 16) return swap_add<D>(x, x);
    else return x + partner<D>(x);
}

// Value of lane `src` (wave-uniform) in every lane, via v_readlane.
__device__ __forceinline__ double read_lane(double x, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), src);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float read_lane(float x, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}

// Sum over the 64 lanes of a wave, returned in every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    v = butterfly_add<1>(v);
    v = butterfly_add<2>(v);
    v = butterfly_add<4>(v);
    v = butterfly_add<8>(v);
    v = butterfly_add<16>(v);
    v = butterfly_add<32>(v);
    return v;
}

// Sum over aligned groups of G lanes (G in {1, 2, 4, 8, 16, 32, 64}).
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
    if constexpr (G >= 2) v = butterfly_add<1>(v);
    if constexpr (G >= 4) v = butterfly_add<2>(v);
    if constexpr (G >= 8) v = butterfly_add<4>(v);
    if constexpr (G >= 16) v = butterfly_add<8>(v);
    if constexpr (G >= 32) v = butterfly_add<16>(v);
    if constexpr (G >= 64) v = butterfly_add<32>(v);
    return v;
}

// Reduce-scatter of N values per lane over the 64 lanes of a wave (the first
// half of wave_allreduce_vec below, kept separate so that the cooperative
// TSQR bodies compile exactly as before), by recursive halving (lane bit 5 keeps the upper half of the list at the first
// stage, bit 4 at the second, ...) and a butterfly over the remaining lane
// bits.  Returns, in every lane, the full sum of value number
// lane >> (6 - log2(cpow2(N))) (zero for numbers >= N).
template <int N, typename T>
__device__ __forceinline__ T wave_reduce_keys(const T (&p)[N]) {
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
            if (t == 0) {
                b[i] = swap_add<32>(b[i], b[half + i]);
            } else if (t == 1) {
                b[i] = swap_add<16>(b[i], b[half + i]);
            } else {
                T send = hi ? b[i] : b[half + i];
                T keep = hi ? b[half + i] : b[i];
                if (t == 2) send = partner<8>(send);
                else if (t == 3) send = partner<4>(send);
                else if (t == 4) send = partner<2>(send);
                else send = partner<1>(send);
                b[i] = keep + send;
            }
        }
    }
    if (Q <= 0) b[0] = butterfly_add<32>(b[0]);
    if (Q <= 1) b[0] = butterfly_add<16>(b[0]);
    if (Q <= 2) b[0] = butterfly_add<8>(b[0]);
    if (Q <= 3) b[0] = butterfly_add<4>(b[0]);
    if (Q <= 4) b[0] = butterfly_add<2>(b[0]);
    if (Q <= 5) b[0] = butterfly_add<1>(b[0]);
    return b[0];
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
            if (t == 0) {
                b[i] = swap_add<32>(b[i], b[half + i]);
            } else if (t == 1) {
                b[i] = swap_add<16>(b[i], b[half + i]);
            } else {
                T send = hi ? b[i] : b[half + i];
                T keep = hi ? b[half + i] : b[i];
                if (t == 2) send = partner<8>(send);
                else if (t == 3) send = partner<4>(send);
                else if (t == 4) send = partner<2>(send);
                else send = partner<1>(send);
                b[i] = keep + send;
            }
        }
    }
    // butterfly over the lane bits not used by the halving stages
    if (Q <= 0) b[0] = butterfly_add<32>(b[0]);
    if (Q <= 1) b[0] = butterfly_add<16>(b[0]);
    if (Q <= 2) b[0] = butterfly_add<8>(b[0]);
    if (Q <= 3) b[0] = butterfly_add<4>(b[0]);
    if (Q <= 4) b[0] = butterfly_add<2>(b[0]);
    if (Q <= 5) b[0] = butterfly_add<1>(b[0]);
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
