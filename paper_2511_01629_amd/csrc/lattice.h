// lattice.h -- compile-time velocity sets and population storage types for
// the gfx950 kernels.
//
// D2Q9 is numbered as in the velocity-set figure of sec. 2.2 (0 rest, 1..4
// the axes counter-clockwise from +x, 5..8 the diagonals); D3Q19 is rest, the
// six faces, then the twelve edges with opposite directions adjacent.  The
// weights go by speed: 4/9, 1/9, 1/36 (D2Q9) and 1/3, 1/18, 1/36 (D3Q19).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

struct D2Q9 {
    static constexpr int Q = 9, D = 2;
    static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

struct D3Q19 {
    static constexpr int Q = 19, D = 3;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

// ---------------------------------------------------------------- storage
// Storage tags: the raw element type in HBM and its conversion to/from the
// arithmetic type.  FP16 uses the IEEE binary16 conversion of the compiler
// (round to nearest even); BF16 rounds to nearest even by integer arithmetic.
struct StF64 { using raw = double; };
struct StF32 { using raw = float; };
struct StF16 { using raw = _Float16; };
struct StBF16 { using raw = uint16_t; };

template <class S, class T> __device__ __forceinline__ T ld(const typename S::raw *p);
template <class S, class T> __device__ __forceinline__ void st(typename S::raw *p, T v);

template <> __device__ __forceinline__ double ld<StF64, double>(const double *p) { return __builtin_nontemporal_load(p); }
template <> __device__ __forceinline__ float ld<StF32, float>(const float *p) { return __builtin_nontemporal_load(p); }
template <> __device__ __forceinline__ float ld<StF16, float>(const _Float16 *p)
{
    return (float)__builtin_nontemporal_load(p);
}
template <> __device__ __forceinline__ float ld<StBF16, float>(const uint16_t *p)
{
    uint32_t b = (uint32_t)__builtin_nontemporal_load(p) << 16;
    return __uint_as_float(b);
}

template <> __device__ __forceinline__ void st<StF64, double>(double *p, double v) { __builtin_nontemporal_store(v, p); }
template <> __device__ __forceinline__ void st<StF32, float>(float *p, float v) { __builtin_nontemporal_store(v, p); }
template <> __device__ __forceinline__ void st<StF16, float>(_Float16 *p, float v)
{
    __builtin_nontemporal_store((_Float16)v, p);
}
// FP32 -> BF16, round to nearest even, NaN kept quiet (the top 16 bits with
// the quiet bit set): gfx950 converts in one instruction (v_cvt_pk_bf16_f32),
// which gives the same bits as the integer form (add 0x7FFF plus the kept
// lowest bit, keep the top half) on every input, NaNs and denormals included
// (checked over 2^24 bit patterns and every rounding edge on MI355X).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float v)
{
    const __bf16 b = (__bf16)v;
    return __builtin_bit_cast(uint16_t, b);
}
template <> __device__ __forceinline__ void st<StBF16, float>(uint16_t *p, float v)
{
    __builtin_nontemporal_store(f32_to_bf16_rne(v), p);
}

// Plain (cached) variants for the small side kernels.
template <class S, class T> __device__ __forceinline__ T ldc(const typename S::raw *p);
template <> __device__ __forceinline__ double ldc<StF64, double>(const double *p) { return *p; }
template <> __device__ __forceinline__ float ldc<StF32, float>(const float *p) { return *p; }
template <> __device__ __forceinline__ float ldc<StF16, float>(const _Float16 *p) { return (float)*p; }
template <> __device__ __forceinline__ float ldc<StBF16, float>(const uint16_t *p)
{
    return __uint_as_float((uint32_t)*p << 16);
}

// Raw element <-> arithmetic type without a memory access (LDS staging);
// the same conversions as ld / st.
template <class S, class T> __device__ __forceinline__ T from_raw(typename S::raw r);
template <class S, class T> __device__ __forceinline__ typename S::raw to_raw(T v);
template <> __device__ __forceinline__ double from_raw<StF64, double>(double r) { return r; }
template <> __device__ __forceinline__ float from_raw<StF32, float>(float r) { return r; }
template <> __device__ __forceinline__ float from_raw<StF16, float>(_Float16 r) { return (float)r; }
template <> __device__ __forceinline__ float from_raw<StBF16, float>(uint16_t r) { return __uint_as_float((uint32_t)r << 16); }
template <> __device__ __forceinline__ double to_raw<StF64, double>(double v) { return v; }
template <> __device__ __forceinline__ float to_raw<StF32, float>(float v) { return v; }
template <> __device__ __forceinline__ _Float16 to_raw<StF16, float>(float v) { return (_Float16)v; }
template <> __device__ __forceinline__ uint16_t to_raw<StBF16, float>(float v) { return f32_to_bf16_rne(v); }

constexpr uint16_t FLUID = 0xFFFFu; // owner-map value of a fluid node

} // namespace lbm
