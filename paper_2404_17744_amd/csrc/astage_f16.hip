// The A stage in the fp16x2 mode:
//
//   A_Pqv = sum_s U_Pqs G_sv(beta - tau)
//
// as C(i, j) = alpha * sum_k Aop[i][k] Bop[j][k] with Aop the rows (P, q) of U
// and Bop the rows v of G(beta - tau)^T, both K-major fp16 planes (x = x0 + x1,
// products x1 y0 + x0 y1 + x0 y0 on the f16 matrix cores, FP32 accumulation).
// The result is written in FP32, and max |C| is max-reduced for the scaling
// that the fused stage applies when it splits A.
//
// A workgroup of eight waves (two per SIMD) owns 128 rows of U and TN = 64 WBN
// columns (v), WBN <= 5; wave (wm, wn) holds 64 x 16 WBN of it.  Each 32-wide
// k stage of both operands (U: 16 KiB, G: TN x 128 B) is loaded from memory
// straight into one of two LDS buffers, one stage ahead of the matrix cores;
// the fragments of the next stage are read while the second half of the
// current stage's MFMAs run.  The MFMA takes the G fragment as its row operand, so a lane's output
// elements run along i = (P, q): stores of 16 lanes cover 64 contiguous bytes.
#include "kernels.hpp"
#include "mfma.hpp"
#include "panel.hpp"

namespace thcsox {
namespace {

constexpr int AM = 128;             // rows of U per workgroup
constexpr int AKC = 32;             // k per stage
constexpr int ANW = 8, ANT = 64 * ANW;

constexpr int AMAXN = 320;          // columns per workgroup at most (WBN <= 5)
struct ABuf {
  _Float16 u[2][AM * AKC];              // [plane][row * 32 + physical chunk * 8 + e]
  _Float16 g[2][AMAXN * AKC];
};

template <int WBN> struct AFrags {
  f16x8 u[2][4], g[2][WBN];   // [plane][tile]
};

__device__ __forceinline__ void a_vm_lds_barrier() {
  __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ double a_wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <int WBN>
__device__ __forceinline__ void astage_body(const GemmKArgs& g, ABuf& b0, ABuf& b1) {
  constexpr int TN = 64 * WBN;
  static_assert(TN <= AMAXN, "at most 320 columns per workgroup");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int nib = (g.M + AM - 1) / AM;
  const int i0 = (blockIdx.x % nib) * AM, j0 = (blockIdx.x / nib) * TN;
  const int rows_i = min(AM, g.M - i0), rows_j = min(TN, g.N - j0);
  const int kst = g.kpad / AKC;

  const _Float16* A = static_cast<const _Float16*>(g.A) + (int64_t)i0 * g.lda;
  const _Float16* B = static_cast<const _Float16*>(g.B) + (int64_t)j0 * g.ldb;
  __amdgpu_buffer_rsrc_t rA[2], rB[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    rA[p] = make_rsrc(A + p * g.a_plane, (int64_t)AM * g.lda * 2);
    rB[p] = make_rsrc(B + p * g.b_plane, (int64_t)TN * g.ldb * 2);
  }
  // memory-to-LDS slabs of 16 rows: U has 8 per plane (wave w moves slab w of
  // both planes), G has TN / 16 per plane, 8 WBN in all (wave w moves the
  // slabs w + 8 j, j < WBN, counted across the two planes)
  constexpr int GSP = TN / 16;               // G slabs per plane
  uint32_t du, dg[WBN];
  {
    const int row = wave * 16 + (lane >> 2);
    const int c = lds_chunk(row, lane & 3);
    du = row < rows_i ? (uint32_t)((row * g.lda + 8 * c) * 2) : OOB;
  }
#pragma unroll
  for (int j = 0; j < WBN; ++j) {
    const int slab = (wave + ANW * j) % GSP;
    const int row = slab * 16 + (lane >> 2);
    const int c = lds_chunk(row, lane & 3);
    dg[j] = row < rows_j ? (uint32_t)((row * g.ldb + 8 * c) * 2) : OOB;
  }
  auto dma = [&](ABuf& bf, int k0) {
#pragma unroll
    for (int p = 0; p < 2; ++p)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rA[p], &bf.u[p][wave * 16 * AKC], 16, du, k0 * 2, 0, 0);
#pragma unroll
    for (int j = 0; j < WBN; ++j) {
      const int s = wave + ANW * j, p = s / GSP, slab = s % GSP;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(p ? rB[1] : rB[0], &bf.g[p][slab * 16 * AKC], 16,
                                               dg[j], k0 * 2, 0, 0);
    }
  };

  int ui[4], gj[WBN];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = wm * 64 + 16 * t + (lane & 15);
    ui[t] = r * AKC + lds_chunk(r, lane >> 4) * 8;
  }
#pragma unroll
  for (int t = 0; t < WBN; ++t) {
    const int r = wn * 16 * WBN + 16 * t + (lane & 15);
    gj[t] = r * AKC + lds_chunk(r, lane >> 4) * 8;
  }
  using Frags = AFrags<WBN>;
  auto read_frags = [&](Frags& fr, const ABuf& bf) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
#pragma unroll
      for (int t = 0; t < 4; ++t) fr.u[p][t] = *reinterpret_cast<const f16x8*>(&bf.u[p][ui[t]]);
#pragma unroll
      for (int t = 0; t < WBN; ++t) fr.g[p][t] = *reinterpret_cast<const f16x8*>(&bf.g[p][gj[t]]);
    }
  };
  // acc[tj][ti]: rows v (tile tj), columns i (tile ti)
  f4 acc[WBN][4];
#pragma unroll
  for (int a = 0; a < WBN; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = f4{0.f, 0.f, 0.f, 0.f};
  constexpr int NQ = 4 * WBN * 3;
  auto mfma_range = [&](const Frags& fr, int q0, int q1) {
#pragma unroll
    for (int q = q0; q < q1; ++q) {
      const int tile = q / 3, pp = q % 3;
      const int tj = tile / 4, ti = tile % 4;
      const int pg = pp == 0 ? 1 : 0, pu = pp == 1 ? 1 : 0;
      acc[tj][ti] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.g[pg][tj], fr.u[pu][ti],
                                                           acc[tj][ti], 0, 0, 0);
    }
  };

  Frags f0, f1;
  // stage s lives in buffer s mod 2; kst is even
  int lk = 0;
  auto next_k = [&]() {
    const int k = lk;
    lk = min(lk + 1, kst - 1);
    return k * AKC;
  };
  dma(b0, next_k());
  dma(b1, next_k());
  a_vm_lds_barrier();
  read_frags(f0, b0);
  auto stage = [&](ABuf& cur, ABuf& nxt, Frags& fc, Frags& fn) {
    mfma_range(fc, 0, NQ / 2);
    // the next stage has landed in nxt; every wave is done reading cur
    a_vm_lds_barrier();
    dma(cur, next_k());
    read_frags(fn, nxt);
    mfma_range(fc, NQ / 2, NQ);
  };
  for (int ks = 0; ks < kst; ks += 2) {
    stage(b0, b1, f0, f1);
    stage(b1, b0, f1, f0);
  }
  // the last (repeated) memory-to-LDS loads land before the workgroup may end
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");

  double lmax = 0.0;
  float* C = static_cast<float*>(g.C);
  const int ib = i0 + wm * 64 + (lane & 15);
  const int jb = j0 + wn * 16 * WBN + 4 * (lane >> 4);
#pragma unroll
  for (int ti = 0; ti < 4; ++ti) {
    const int i = ib + 16 * ti;
    if (i >= g.M) continue;
    const int64_t ibase = ((int64_t)i / g.ci_in) * g.ci_out + ((int64_t)i % g.ci_in);
#pragma unroll
    for (int tj = 0; tj < WBN; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jb + 16 * tj + r;
        if (j < g.N) {
          const float v = (float)(g.alpha * (double)acc[tj][ti][r]);
          C[ibase + (int64_t)j * g.c_j] = v;
          lmax = fmax(lmax, fabs((double)v));
        }
      }
  }
  if (g.amax != nullptr) {
    lmax = a_wave_max(lmax);
    if (lane == 0) atomicMax(g.amax, (unsigned long long)__double_as_longlong(lmax));
  }
}

// one kernel per column count (the body is a device template)
#define THCSOX_ASTAGE_KERNEL(W)                                                         \
  __global__ __launch_bounds__(ANT) __attribute__((amdgpu_waves_per_eu(2, 2)))          \
  void astage_f16_kernel_##W(GemmKArgs g) {                                            \
    __shared__ __attribute__((aligned(16))) ABuf b0;                                    \
    __shared__ __attribute__((aligned(16))) ABuf b1;                                    \
    astage_body<W>(g, b0, b1);                                                          \
  }
THCSOX_ASTAGE_KERNEL(2)
THCSOX_ASTAGE_KERNEL(3)
THCSOX_ASTAGE_KERNEL(4)
THCSOX_ASTAGE_KERNEL(5)
#undef THCSOX_ASTAGE_KERNEL

inline unsigned a_cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <int WBN>
hipError_t a_launch(void (*kernel)(GemmKArgs), const GemmKArgs& g, hipStream_t s) {
  const unsigned grid = a_cdiv(g.M, AM) * a_cdiv(g.N, 64 * WBN);
  kernel<<<grid, ANT, 0, s>>>(g);
  return hipGetLastError();
}

}  // namespace

hipError_t astage_f16(const GemmKArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.kpad % (2 * AKC) != 0) return hipErrorInvalidValue;
  // 32-bit buffer offsets inside one workgroup's rows
  if ((int64_t)AM * g.lda * 2 > 0x7fffffffLL || (int64_t)320 * g.ldb * 2 > 0x7fffffffLL)
    return hipErrorInvalidValue;
  if (g.N <= 128) return a_launch<2>(astage_f16_kernel_2, g, s);
  if (g.N <= 192) return a_launch<3>(astage_f16_kernel_3, g, s);
  if (g.N <= 256) return a_launch<4>(astage_f16_kernel_4, g, s);
  return a_launch<5>(astage_f16_kernel_5, g, s);   // 320 columns per workgroup, more beyond
}

}  // namespace thcsox
