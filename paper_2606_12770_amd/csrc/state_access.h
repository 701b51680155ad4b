// State-vector loads and stores with an optional nontemporal hint, for the
// tile passes and the plain gate kernels, which read and write each amplitude
// they touch once.  (The dense block pass keeps plain accesses: with the hint
// its complex128 form was 17% slower and its complex64 form unchanged.)
// The hint is a template parameter: two branches over the same addresses would
// be merged by the compiler into one access without the hint.
#pragma once
#include <hip/hip_runtime.h>

namespace svi {

template <bool NT>
__device__ __forceinline__ float2 load_state(const float2 *p)
{
    if constexpr (NT) {
        typedef float v2 __attribute__((ext_vector_type(2)));
        const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
        return make_float2(v.x, v.y);
    } else {
        return *p;
    }
}

template <bool NT>
__device__ __forceinline__ double2 load_state(const double2 *p)
{
    if constexpr (NT) {
        typedef double v2 __attribute__((ext_vector_type(2)));
        const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
        return make_double2(v.x, v.y);
    } else {
        return *p;
    }
}

template <bool NT>
__device__ __forceinline__ void store_state(float2 *p, float2 x)
{
    if constexpr (NT) {
        typedef float v2 __attribute__((ext_vector_type(2)));
        v2 v;
        v.x = x.x;
        v.y = x.y;
        __builtin_nontemporal_store(v, reinterpret_cast<v2 *>(p));
    } else {
        *p = x;
    }
}

template <bool NT>
__device__ __forceinline__ void store_state(double2 *p, double2 x)
{
    if constexpr (NT) {
        typedef double v2 __attribute__((ext_vector_type(2)));
        v2 v;
        v.x = x.x;
        v.y = x.y;
        __builtin_nontemporal_store(v, reinterpret_cast<v2 *>(p));
    } else {
        *p = x;
    }
}

}  // namespace svi
