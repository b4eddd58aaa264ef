// Device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mf {

// Pointers read out of a FrontNum are generic to the compiler, so their accesses
// become flat instructions, which count on the same wait counter as LDS: every
// LDS access would then wait for all front loads in flight, and the loads would
// wait for one another.  Front storage is device global memory; casting to the
// global address space gives global loads and stores with their own in-order
// counter.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
    return (gptr<T>)p;
}

// Position of parent (pre-pivot) row i inside child c's contribution block, or -1.
// dseg: start of c's segment inside the parent's delayed-in block; dout: c's
// delayed-out count; im: c's inverse nominal map (indexed by parent nominal row).
__device__ __forceinline__ int child_pos(int i, int npiv_p, int din_p, int dseg, int dout, const int32_t* im) {
    if (i < npiv_p) {
        int t = im[i];
        return t >= 0 ? dout + t : -1;
    }
    int d = i - npiv_p;
    if (d < din_p) {
        d -= dseg;
        return (d >= 0 && d < dout) ? d : -1;
    }
    int t = im[i - din_p];
    return t >= 0 ? dout + t : -1;
}

// Uniform broadcast of lane l's double (two 32-bit readlanes).
__device__ __forceinline__ double readlane_d(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

}  // namespace mf
