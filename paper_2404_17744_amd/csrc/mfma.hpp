// Matrix-core building blocks for gfx950 (CDNA4): operand formats, MFMA calls
// and the 16x16 output layout of each instruction.
//
// Every contraction in this library is written as C[i][j] = sum_k A[i][k] B[j][k]
// on 16x16 output tiles held by one 64-lane wavefront.  Operand element types:
//
//   mode        element   planes  k per MFMA   instruction
//   MODE_F64    double    1       4            v_mfma_f64_16x16x4_f64
//   MODE_F32    float     1       4            v_mfma_f32_16x16x4_f32
//   MODE_BF16X3 __bf16    3       32           v_mfma_f32_16x16x32_bf16 (6 products)
//   MODE_F16X2  _Float16  2       32           v_mfma_f32_16x16x32_f16  (3 products)
//
// A split operand x is stored as planes x0 + x1 (+ x2), each plane an array of
// the same shape; the product a*b is formed from the plane products whose order
// of magnitude is at least the last plane's (all except those below it).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace thcsox {

enum Mode { MODE_F64 = 0, MODE_F32 = 1, MODE_BF16X3 = 2, MODE_F16X2 = 3 };

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <int M> struct ModeT;
template <> struct ModeT<MODE_F64> {
  using T = double; using Frag = double; using Acc = d4;
  static constexpr int NP = 1, KS = 4;
};
template <> struct ModeT<MODE_F32> {
  using T = float; using Frag = float; using Acc = f4;
  static constexpr int NP = 1, KS = 4;
};
template <> struct ModeT<MODE_BF16X3> {
  using T = __bf16; using Frag = bf16x8; using Acc = f4;
  static constexpr int NP = 3, KS = 32;
};
template <> struct ModeT<MODE_F16X2> {
  using T = _Float16; using Frag = f16x8; using Acc = f4;
  static constexpr int NP = 2, KS = 32;
};

__device__ __forceinline__ d4 mfma1(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma1(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma1(bf16x8 a, bf16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma1(f16x8 a, f16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Number of plane products per operand product and the plane pair of product p.
// The order runs from the smallest terms to the leading one.
template <int NP> struct Products;
template <> struct Products<1> {
  static constexpr int N = 1;
  __device__ static constexpr int a(int) { return 0; }
  __device__ static constexpr int b(int) { return 0; }
};
template <> struct Products<2> {
  static constexpr int N = 3;   // x1*y0, x0*y1, x0*y0
  __device__ static constexpr int a(int p) { return p == 0 ? 1 : 0; }
  __device__ static constexpr int b(int p) { return p == 1 ? 1 : 0; }
};
template <> struct Products<3> {
  static constexpr int N = 6;   // x0*y2, x1*y1, x2*y0, x0*y1, x1*y0, x0*y0
  __device__ static constexpr int a(int p) {
    return p == 0 ? 0 : p == 1 ? 1 : p == 2 ? 2 : p == 3 ? 0 : p == 4 ? 1 : 0;
  }
  __device__ static constexpr int b(int p) {
    return p == 0 ? 2 : p == 1 ? 1 : p == 2 ? 0 : p == 3 ? 1 : p == 4 ? 0 : 0;
  }
};

// Row of element r (0..3) held by lane l in a 16x16 output tile; column is l & 15.
template <int M> __device__ __forceinline__ int out_row(int lane, int r) {
  if constexpr (M == MODE_F64) return (lane >> 4) + 4 * r;
  else return 4 * (lane >> 4) + r;
}

// Physical 16-byte chunk of logical chunk c (0..3) in row r of a 16-bit LDS
// tile with 64-byte rows.  Fragment reads touch 16 consecutive rows at one
// logical chunk; with this map any 8 (or 16) consecutive rows land on distinct
// bank groups for 128-byte (or 256-byte) wide LDS banking, and the four chunks
// of one row stay distinct (so whole-row writes are conflict-free too).
__device__ __forceinline__ int lds_chunk(int r, int c) { return c ^ (((r >> 1) ^ (r >> 3)) & 3); }

// Load one operand fragment from an LDS tile stored row-major as
// s[row][ldk_s] (k contiguous): rows i0..i0+15, k range starting at kk.
// 16-bit tiles hold one 32-wide k range per row (kk = 0) as four 16-byte
// chunks placed by lds_chunk.
template <int M>
__device__ __forceinline__ typename ModeT<M>::Frag
lds_frag(const typename ModeT<M>::T* s, int ldk_s, int i0, int kk, int lane) {
  using MT = ModeT<M>;
  if constexpr (MT::KS == 4) {
    return s[(i0 + (lane & 15)) * ldk_s + kk + (lane >> 4)];
  } else {
    const int r = i0 + (lane & 15);
    const int c = lds_chunk(r, lane >> 4);
    const typename MT::Frag* p =
        reinterpret_cast<const typename MT::Frag*>(s + r * ldk_s + kk + 8 * c);
    return *p;
  }
}

// Split of an FP64 value into the planes of a mode (value already scaled).
template <int M> struct Split;
template <> struct Split<MODE_F64> {
  __device__ static void run(double x, double* o) { o[0] = x; }
};
template <> struct Split<MODE_F32> {
  __device__ static void run(double x, float* o) { o[0] = (float)x; }
};
template <> struct Split<MODE_BF16X3> {
  __device__ static void run(double x, __bf16* o) {
    __bf16 h = (__bf16)(float)x;
    double r1 = x - (double)(float)h;
    __bf16 m = (__bf16)(float)r1;
    double r2 = r1 - (double)(float)m;
    o[0] = h; o[1] = m; o[2] = (__bf16)(float)r2;
  }
};
template <> struct Split<MODE_F16X2> {
  __device__ static void run(double x, _Float16* o) {
    _Float16 h = (_Float16)(float)x;
    double r = x - (double)(float)h;
    o[0] = h; o[1] = (_Float16)(float)r;
  }
};

}  // namespace thcsox
