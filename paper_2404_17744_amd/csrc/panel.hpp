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

// Exact split of an FP32 value into 16-bit planes (x - hi is exact in FP32).
template <int M> __device__ __forceinline__ void split_f(float x, typename ModeT<M>::T* o);
template <> __device__ __forceinline__ void split_f<MODE_F16X2>(float x, _Float16* o) {
  const _Float16 h = (_Float16)x;
  o[0] = h;
  o[1] = (_Float16)(x - (float)h);
}
template <> __device__ __forceinline__ void split_f<MODE_BF16X3>(float x, __bf16* o) {
  const __bf16 h = (__bf16)x;
  const float r1 = x - (float)h;
  const __bf16 m = (__bf16)r1;
  o[0] = h;
  o[1] = m;
  o[2] = (__bf16)(r1 - (float)m);
}

// A ROWS x BK panel of an FP32 array, split into the planes of mode M (after
// scaling by a power of two) when written to LDS.
template <int M, int ROWS>
struct PanelF32 {
  using T = typename ModeT<M>::T;
  static constexpr int NP = ModeT<M>::NP;
  static constexpr int UPR = BK / 4, NU = ROWS * UPR, PER = (NU + NT - 1) / NT;
  uint32_t off[PER];
  f4 r[PER];
  __device__ __forceinline__ void init(int64_t row_stride, int valid_rows, int tid) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int u = tid + i * NT;
      const int row = u / UPR, c = (u % UPR) * 4;
      off[i] = (u < NU && row < valid_rows) ? (uint32_t)(((int64_t)row * row_stride + c) * 4)
                                            : OOB;
    }
  }
  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, int k0) {
#pragma unroll
    for (int i = 0; i < PER; ++i)
      r[i] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, off[i], k0 * 4, 0));
  }
  __device__ __forceinline__ void store(T* const* s, float scale, int tid) const {
    constexpr int LD = lds_ld<T>();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int u = tid + i * NT;
      const int row = u / UPR, c4 = u % UPR;   // 4-element piece: chunk c4 / 2, half c4 % 2
      const int c = lds_chunk(row, c4 >> 1) * 8 + (c4 & 1) * 4;
      if (NU % NT == 0 || u < NU) {
        T o[4][NP];
#pragma unroll
        for (int e = 0; e < 4; ++e) split_f<M>(r[i][e] * scale, o[e]);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          typedef T T4 __attribute__((ext_vector_type(4)));
          T4 w = {o[0][p], o[1][p], o[2][p], o[3][p]};
          *reinterpret_cast<T4*>(s[p] + row * LD + c) = w;
        }
      }
    }
  }
};

}  // namespace
}  // namespace thcsox
