// Register-staged operand panels for the matrix-core kernels: a ROWS x BK
// slice of a K-major array (rows of k-contiguous elements) is fetched with raw
// buffer loads into registers and later written to LDS rows of stride
// lds_ld<T>() for fragment reads.  Rows outside the valid range read as zero
// (their offsets point past the buffer), so no load needs a branch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mfma.hpp"

namespace thcsox {
namespace {

constexpr int NT = 256;   // threads per workgroup (4 wavefronts)
constexpr int BK = 32;    // k extent of one staged panel

// LDS row stride (elements).  16-bit operands use unpadded 64-byte rows whose
// four 16-byte chunks are XOR-swizzled per row (see lds_chunk); 32/64-bit
// operands use padded rows.
template <typename T> constexpr int lds_ld() {
  return BK + (sizeof(T) == 8 ? 2 : sizeof(T) == 4 ? 4 : 0);
}

__device__ __forceinline__ double pow2_scale_f(const unsigned long long* amax) {
  if (amax == nullptr) return 1.0;
  const unsigned long long b = *amax;
  if (b == 0ull) return 1.0;
  const double x = __longlong_as_double((long long)b);
  if (!(x < 1e300)) return 1.0;
  return ldexp(1.0, -ilogb(x));
}

typedef unsigned int u4 __attribute__((ext_vector_type(4)));
constexpr uint32_t OOB = 0x80000000u;   // buffer offset that reads as zero

// Raw buffer resource over [base, base + bytes): loads beyond it return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  const int n = bytes > 0x7fffffff ? 0x7fffffff : (int)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n, 0x00020000);
}

typedef int i4 __attribute__((ext_vector_type(4)));
// raw buffer resource words over [base, base + bytes) (reads past it return zero)
__device__ __forceinline__ i4 raw_rsrc(const void* base, int bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  return i4{(int)(uint32_t)a, (int)((a >> 32) & 0xffff), bytes, 0x00020000};
}
// LDS byte address of a __shared__ location (the low half of its flat address)
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)reinterpret_cast<uint64_t>(p);
}
// Memory-to-LDS load of 16 bytes per lane (lane l lands at LDS lds + 16 l), issued
// in inline assembly: the compiler does not track it, so it inserts no waits for
// it before other LDS accesses (it cannot tell other LDS data apart from the
// buffer being loaded).  The kernel waits for these loads itself (s_waitcnt
// vmcnt(0) before each barrier) and touches the loaded buffer only after that
// barrier.  Nothing else in the kernel uses m0.
__device__ __forceinline__ void dma16_untracked(const i4& rsrc, uint32_t lds, uint32_t voff,
                                                uint32_t soff) {
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
  __asm__ volatile("s_mov_b32 m0, %0\n\tbuffer_load_dwordx4 %1, %2, %3 offen lds"
                   :: "s"(lds), "v"(voff), "s"(rsrc), "s"(soff) : "memory", "m0");
#pragma clang diagnostic pop
}

// A ROWS x BK panel of a K-major array, staged through registers in 16-byte
// units.  Each thread's byte offsets inside the panel are fixed for the whole
// kernel (rows past the valid range point out of the buffer and load zero).
template <typename T, int ROWS>
struct Panel {
  static constexpr int EPU = 16 / (int)sizeof(T), UPR = BK / EPU, NU = ROWS * UPR;
  static constexpr int PER = (NU + NT - 1) / NT;
  uint32_t off[PER];
  u4 r[PER];
  __device__ __forceinline__ void init(int64_t row_stride, int valid_rows, int tid) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int u = tid + i * NT;
      const int row = u / UPR, c = (u % UPR) * EPU;
      off[i] = (u < NU && row < valid_rows)
                   ? (uint32_t)(((int64_t)row * row_stride + c) * (int64_t)sizeof(T))
                   : OOB;
    }
  }
  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, int k0) {
#pragma unroll
    for (int i = 0; i < PER; ++i)
      r[i] = __builtin_amdgcn_raw_buffer_load_b128(rs, off[i], k0 * (int)sizeof(T), 0);
  }
  __device__ __forceinline__ void store(T* s, int tid) const {
    constexpr int LD = lds_ld<T>();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int u = tid + i * NT;
      const int row = u / UPR;
      const int c = (sizeof(T) == 2 ? lds_chunk(row, u % UPR) : u % UPR) * EPU;
      if (NU % NT == 0 || u < NU) *reinterpret_cast<u4*>(s + row * LD + c) = r[i];
    }
  }
};

}  // namespace
}  // namespace thcsox
