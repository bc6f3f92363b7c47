// GEMM over K-major operand planes on matrix cores, used for the A stage
//     A_Pqv = sum_s U_Pqs G_sv(-tau)
// as C(i, j) = alpha * sum_k Aop[i][k] Bop[j][k] with the rows of U as Aop
// (i = (P, q), naux * n rows, streamed once) and the rows of G(-tau)^T as Bop
// (j = v, n rows, re-read from L2 by every workgroup).  A workgroup owns a
// (32 WTI) x (32 WTJ) tile; the next 32-wide k panel is prefetched into
// registers while the current one runs on the matrix cores.
#include "kernels.hpp"
#include "mfma.hpp"
#include "panel.hpp"
#include "reduce.hpp"

namespace thcsox {
namespace {

template <int M, int WTI, int WTJ, typename OutT>
__global__ __launch_bounds__(NT) void gemmk_kernel(GemmKArgs g) {
  using MT = ModeT<M>;
  using T = typename MT::T;
  constexpr int NP = MT::NP, KS = MT::KS, LD = lds_ld<T>(), ES = (int)sizeof(T);
  constexpr int TM = 32 * WTI, TN = 32 * WTJ;
  using PR = Products<NP>;
  __shared__ __attribute__((aligned(16))) T sA[NP][TM * LD];
  __shared__ __attribute__((aligned(16))) T sB[NP][TN * LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int nib = (g.M + TM - 1) / TM;
  const int i0 = (blockIdx.x % nib) * TM, j0 = (blockIdx.x / nib) * TN;

  const T* A = static_cast<const T*>(g.A) + (int64_t)i0 * g.lda;
  const T* B = static_cast<const T*>(g.B) + (int64_t)j0 * g.ldb;
  __amdgpu_buffer_rsrc_t rA[NP], rB[NP];
  Panel<T, TM> pA[NP];
  Panel<T, TN> pB[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    rA[p] = make_rsrc(A + p * g.a_plane, (int64_t)TM * g.lda * ES);
    rB[p] = make_rsrc(B + p * g.b_plane, (int64_t)TN * g.ldb * ES);
    pA[p].init(g.lda, min(TM, g.M - i0), tid);
    pB[p].init(g.ldb, min(TN, g.N - j0), tid);
  }
  typename MT::Acc acc[WTI][WTJ];
#pragma unroll
  for (int ti = 0; ti < WTI; ++ti)
#pragma unroll
    for (int tj = 0; tj < WTJ; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[ti][tj][r] = 0;

  const int nst = g.kpad / BK;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    pA[p].load(rA[p], 0);
    pB[p].load(rB[p], 0);
  }
  for (int ks = 0; ks < nst; ++ks) {
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      pA[p].store(sA[p], tid);
      pB[p].store(sB[p], tid);
    }
    __syncthreads();
    if (ks + 1 < nst) {
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        pA[p].load(rA[p], (ks + 1) * BK);
        pB[p].load(rB[p], (ks + 1) * BK);
      }
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += KS) {
      typename MT::Frag fa[WTI][NP], fb[WTJ][NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
#pragma unroll
        for (int ti = 0; ti < WTI; ++ti)
          fa[ti][p] = lds_frag<M>(sA[p], LD, wr * 16 * WTI + 16 * ti, kk, lane);
#pragma unroll
        for (int tj = 0; tj < WTJ; ++tj)
          fb[tj][p] = lds_frag<M>(sB[p], LD, wc * 16 * WTJ + 16 * tj, kk, lane);
      }
#pragma unroll
      for (int q = 0; q < PR::N; ++q)
#pragma unroll
        for (int ti = 0; ti < WTI; ++ti)
#pragma unroll
          for (int tj = 0; tj < WTJ; ++tj)
            acc[ti][tj] = mfma1(fa[ti][PR::a(q)], fb[tj][PR::b(q)], acc[ti][tj]);
    }
  }

  double lmax = 0.0;
  OutT* C = static_cast<OutT*>(g.C);
  if constexpr (__is_same(OutT, __bf16)) {
    // three bf16 planes; a lane's four outputs are four consecutive rows i of one
    // column j: one 8-byte store per plane when they lie in one block of ci_in
    // rows and the address is 8-byte aligned, else one store per element
    typedef __bf16 b4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int ti = 0; ti < WTI; ++ti)
#pragma unroll
      for (int tj = 0; tj < WTJ; ++tj) {
        const int ib = i0 + wr * 16 * WTI + 16 * ti + out_row<M>(lane, 0);
        const int j = j0 + wc * 16 * WTJ + 16 * tj + (lane & 15);
        if (j >= g.N) continue;
        b4 pl[3];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          __bf16 x[3];
          Split<MODE_BF16X3>::run(g.alpha * (double)acc[ti][tj][r], x);
#pragma unroll
          for (int p = 0; p < 3; ++p) pl[p][r] = x[p];
        }
        const int64_t o = ((int64_t)ib / g.ci_in) * g.ci_out + ((int64_t)ib % g.ci_in) + (int64_t)j * g.c_j;
        if (ib + 3 < g.M && ib % g.ci_in + 3 < g.ci_in && (o & 3) == 0 && (g.c_plane & 3) == 0) {
#pragma unroll
          for (int p = 0; p < 3; ++p) *reinterpret_cast<b4*>(C + o + p * g.c_plane) = pl[p];
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = ib + r;
            if (i >= g.M) break;
            const int64_t oi = ((int64_t)i / g.ci_in) * g.ci_out + ((int64_t)i % g.ci_in) + (int64_t)j * g.c_j;
#pragma unroll
            for (int p = 0; p < 3; ++p) C[oi + p * g.c_plane] = pl[p][r];
          }
        }
      }
    return;
  }
#pragma unroll
  for (int ti = 0; ti < WTI; ++ti)
#pragma unroll
    for (int tj = 0; tj < WTJ; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr * 16 * WTI + 16 * ti + out_row<M>(lane, r);
        const int j = j0 + wc * 16 * WTJ + 16 * tj + (lane & 15);
        if (i < g.M && j < g.N) {
          const int64_t o = ((int64_t)i / g.ci_in) * g.ci_out + ((int64_t)i % g.ci_in) + (int64_t)j * g.c_j;
          const OutT v = (OutT)(g.alpha * (double)acc[ti][tj][r]);
          C[o] = v;
          lmax = fmax(lmax, fabs((double)v));
        }
      }
  if (g.amax != nullptr) block_atomic_max<NT / 64>(lmax, g.amax);
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <int M, int WTI, int WTJ>
hipError_t launch(bool out_f64, const GemmKArgs& g, hipStream_t s) {
  const unsigned grid = cdiv(g.M, 32 * WTI) * cdiv(g.N, 32 * WTJ);
  if (out_f64) gemmk_kernel<M, WTI, WTJ, double><<<grid, NT, 0, s>>>(g);
  else gemmk_kernel<M, WTI, WTJ, float><<<grid, NT, 0, s>>>(g);
  return hipGetLastError();
}

template <int M>
hipError_t launch_mode(bool out_f64, const GemmKArgs& g, hipStream_t s) {
  // all of the B rows in one workgroup when they fit 320, else 160 per workgroup
  if (g.N <= 320) return launch<M, 2, 10>(out_f64, g, s);
  return launch<M, 2, 5>(out_f64, g, s);
}

}  // namespace

hipError_t gemm_kmajor_bf3(const GemmKArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int wtj = g.N <= 320 ? 10 : 5;
  const unsigned grid = cdiv(g.M, 128) * cdiv(g.N, 32 * wtj);
  if (wtj == 10) gemmk_kernel<MODE_BF16X3, 4, 10, __bf16><<<grid, NT, 0, s>>>(g);
  else gemmk_kernel<MODE_BF16X3, 4, 5, __bf16><<<grid, NT, 0, s>>>(g);
  return hipGetLastError();
}

hipError_t gemm_kmajor(int mode, bool out_f64, const GemmKArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  switch (mode) {
    case MODE_F64: return launch<MODE_F64, 2, 5>(out_f64, g, s);
    case MODE_F32: return launch_mode<MODE_F32>(out_f64, g, s);
    case MODE_BF16X3: return launch_mode<MODE_BF16X3>(out_f64, g, s);
    case MODE_F16X2: return launch_mode<MODE_F16X2>(out_f64, g, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace thcsox
