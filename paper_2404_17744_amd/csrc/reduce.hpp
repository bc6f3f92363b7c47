// Workgroup-wide maximum of non-negative doubles, published with one atomic per
// workgroup.  Many atomics on one address serialise in the L2, so the waves of a
// workgroup combine through LDS first.
#pragma once
#include <hip/hip_runtime.h>

namespace thcsox {

// Every thread of the workgroup must call this (it contains a barrier).
// NWAVES = workgroup size / 64.  *addr holds the bits of a non-negative double,
// so the unsigned integer maximum is the floating-point maximum.
template <int NWAVES>
__device__ __forceinline__ void block_atomic_max(double v, unsigned long long* addr) {
  __shared__ double wmax[NWAVES];
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wmax[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = wmax[0];
    for (int w = 1; w < NWAVES; ++w) m = fmax(m, wmax[w]);
    atomicMax(addr, (unsigned long long)__double_as_longlong(m));
  }
}

}  // namespace thcsox
