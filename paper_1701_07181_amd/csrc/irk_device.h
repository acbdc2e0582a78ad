// irk_device.h -- device helpers shared by the gfx950 kernels.
#pragma once
#include "irk_internal.h"

namespace irk {

// Global address space.  Pointers taken from the device-side descriptor are
// generic; casting them lets the compiler emit global_* (not flat_*) memory
// instructions, which do not share the LDS wait counter.
#define GAS __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ GAS T *gp(T *p) { return (GAS T *)(p); }

// Native vector types (plain clang vectors load from any address space).
typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Storage tags for the 16-bit factor formats.
struct bf16s { uint16_t u; };
struct f16s { uint16_t u; };

// ---------------------------------------------------------------------------
// 16-byte loads of V consecutive elements converted to the compute type.
// Blocks are stored column-major with a leading dimension that is a multiple
// of V, so every load is one aligned dwordx4.
// ---------------------------------------------------------------------------
// 16-byte loads of one column piece of a matrix block, converted to the
// compute type.  Every caller streams blocks that are read once per pass
// (Jacobian, mass, pivot and cross blocks), so the loads are nontemporal:
// the blocks do not displace the stage vectors, which neighbouring elements
// re-read, from the caches.
template <typename TS> struct Vec16;

template <> struct Vec16<double> {
    static constexpr int V = 2;
    using st = double;
    template <typename TC>
    __device__ __forceinline__ static void load(const GAS double *p, TC *o) {
        const dbl2 v = __builtin_nontemporal_load(reinterpret_cast<const GAS dbl2 *>(p));
        o[0] = (TC)v.x; o[1] = (TC)v.y;
    }
};

template <> struct Vec16<float> {
    static constexpr int V = 4;
    using st = float;
    template <typename TC>
    __device__ __forceinline__ static void load(const GAS float *p, TC *o) {
        const flt4 v = __builtin_nontemporal_load(reinterpret_cast<const GAS flt4 *>(p));
        o[0] = (TC)v.x; o[1] = (TC)v.y; o[2] = (TC)v.z; o[3] = (TC)v.w;
    }
};

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ float f16_to_f32(uint32_t h) {
    _Float16 x;
    uint16_t hh = (uint16_t)h;
    __builtin_memcpy(&x, &hh, 2);
    return (float)x;
}

template <> struct Vec16<bf16s> {
    static constexpr int V = 8;
    using st = uint16_t;
    template <typename TC>
    __device__ __forceinline__ static void load(const GAS uint16_t *p, TC *o) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const GAS u32x4 *>(p));
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            o[2 * q] = (TC)bf16_to_f32(w[q] & 0xffffu);
            o[2 * q + 1] = (TC)bf16_to_f32(w[q] >> 16);
        }
    }
};

template <> struct Vec16<f16s> {
    static constexpr int V = 8;
    using st = uint16_t;
    template <typename TC>
    __device__ __forceinline__ static void load(const GAS uint16_t *p, TC *o) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const GAS u32x4 *>(p));
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            o[2 * q] = (TC)f16_to_f32(w[q] & 0xffffu);
            o[2 * q + 1] = (TC)f16_to_f32(w[q] >> 16);
        }
    }
};

// FP32 -> BF16, round to nearest even, NaN kept quiet.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// FP32 -> FP16 bits, IEEE round to nearest even with subnormals, overflow to
// infinity.  Computed exactly in FP64: the FP32 magnitude d is scaled so
// that its half-precision significand becomes an integer, rounded with rint
// (round half to even), and re-encoded.
__device__ __forceinline__ uint16_t f32_to_f16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    const uint16_t sign = (uint16_t)((u >> 16) & 0x8000u);
    const double d = fabs((double)f);
    if (d != d) return (uint16_t)(sign | 0x7e00u);                 // NaN
    if (d >= 65520.0) return (uint16_t)(sign | 0x7c00u);           // rounds to infinity
    if (d < 0x1p-14) {                                             // half subnormal (or zero)
        const double q = rint(d * 0x1p24);                         // units of 2^-24, q <= 1024
        return (uint16_t)(sign | (uint16_t)q);                     // q = 1024 is the smallest normal
    }
    int ex = ilogb(d);                                             // -14 .. 15
    double r = rint(ldexp(d, 10 - ex));                            // [1024, 2048]
    if (r == 2048.0) { r = 1024.0; ++ex; }
    if (ex > 15) return (uint16_t)(sign | 0x7c00u);
    return (uint16_t)(sign | (uint16_t)((ex + 15) << 10) | (uint16_t)(r - 1024.0));
}

// leading dimension and base pointers by storage type
template <typename TS> __device__ __forceinline__ int ld_of(const SysDesc &d);
template <> __device__ __forceinline__ int ld_of<double>(const SysDesc &d) { return d.ld; }
template <> __device__ __forceinline__ int ld_of<float>(const SysDesc &d) { return d.ld32; }
template <> __device__ __forceinline__ int ld_of<bf16s>(const SysDesc &d) { return d.ld16; }
template <> __device__ __forceinline__ int ld_of<f16s>(const SysDesc &d) { return d.ld16; }

template <typename TS> __device__ __forceinline__ const GAS typename Vec16<TS>::st *jac_of(const SysDesc &d);
template <> __device__ __forceinline__ const GAS double *jac_of<double>(const SysDesc &d) { return gp((const double *)d.Jc); }
template <> __device__ __forceinline__ const GAS float *jac_of<float>(const SysDesc &d) { return gp((const float *)d.Jc32); }
template <typename TS> __device__ __forceinline__ const GAS typename Vec16<TS>::st *mass_of(const SysDesc &d);
template <> __device__ __forceinline__ const GAS double *mass_of<double>(const SysDesc &d) { return gp((const double *)d.Mc); }
template <> __device__ __forceinline__ const GAS float *mass_of<float>(const SysDesc &d) { return gp((const float *)d.Mc32); }

template <typename TS> __device__ __forceinline__ const GAS typename Vec16<TS>::st *piv_of(const SysDesc &d);
template <> __device__ __forceinline__ const GAS double *piv_of<double>(const SysDesc &d) { return gp((const double *)d.P64); }
template <> __device__ __forceinline__ const GAS float *piv_of<float>(const SysDesc &d) { return gp((const float *)d.P32); }
template <> __device__ __forceinline__ const GAS uint16_t *piv_of<bf16s>(const SysDesc &d) { return gp((const uint16_t *)d.P16); }
template <> __device__ __forceinline__ const GAS uint16_t *piv_of<f16s>(const SysDesc &d) { return gp((const uint16_t *)d.P16); }
template <typename TS> __device__ __forceinline__ const GAS typename Vec16<TS>::st *cross_of(const SysDesc &d);
template <> __device__ __forceinline__ const GAS double *cross_of<double>(const SysDesc &d) { return gp((const double *)d.C64); }
template <> __device__ __forceinline__ const GAS float *cross_of<float>(const SysDesc &d) { return gp((const float *)d.C32); }
template <> __device__ __forceinline__ const GAS uint16_t *cross_of<bf16s>(const SysDesc &d) { return gp((const uint16_t *)d.C16); }
template <> __device__ __forceinline__ const GAS uint16_t *cross_of<f16s>(const SysDesc &d) { return gp((const uint16_t *)d.C16); }

// per-block scale of the FP16S format (1 for every other format)
template <typename TS, typename TC>
__device__ __forceinline__ TC block_scale(const int *e, long long blk) { return (TC)1; }
template <>
__device__ __forceinline__ float block_scale<f16s, float>(const int *e, long long blk) {
    return ldexpf(1.0f, -gp(e)[blk]);
}

// ---------------------------------------------------------------------------
// wave / workgroup reductions (fixed order, so results are deterministic)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace irk
