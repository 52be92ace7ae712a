// Plane stores: non-temporal (the plane is written once and read later by a
// different pass), bfloat16 rounded to nearest even from FP32.
#pragma once

#include <hip/hip_runtime.h>

namespace fdas {

template <class P>
struct plane_store;
template <>
struct plane_store<float> {
    static __device__ __forceinline__ void put(float *p, float v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct plane_store<double> {
    static __device__ __forceinline__ void put(double *p, double v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct plane_store<__bf16> {
    static __device__ __forceinline__ void put(__bf16 *p, float v) {
        const __bf16 b = (__bf16)v;
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, b), (unsigned short *)p);
    }
};

}  // namespace fdas
