// The fused B/C/D stage of the THC-SOX sequence (one tau point), FP64 mode, and
// the dispatch of the other modes' kernels:
//
//   D_PR = sum_v C_RvP B_PRv,   B_PRv = sum_q G_Rq A_Pqv,   C_RvP = sum_w U_Rvw G_wP
//
// A workgroup owns a TR (R) x TP (P) tile of D and a range of v.  For every v
// it forms both length-n contractions on matrix cores,
//   accB[R][P] = sum_q Gt[R][q] A[v][P][q]      accC[R][P] = sum_w U[R][v][w] GXt[P][w]
// which land in the same MFMA output layout, so B o C is a register-to-register
// product.  In FP64 mode it is accumulated in FP64 registers; the template also
// holds a reduced-precision form (FP32 registers for at most FLUSH_V consecutive
// v, then added into the workgroup's FP64 tile of D) that is not launched: only
// the FP64 mode runs this kernel.  Neither B (naux^2 n) nor
// C ever reaches memory.  Operands are staged through LDS one (v, 32-wide k chunk) stage at a
// time; the next stage's global loads are issued before the current stage's
// MFMAs (register prefetch), so loads overlap the matrix work.
#include <algorithm>
#include <type_traits>

#include "kernels.hpp"
#include "mfma.hpp"
#include "panel.hpp"

namespace thcsox {
namespace {

constexpr int FLUSH_V = 8;   // v per FP32 partial sum of D before it is added in FP64
constexpr int NXCD = 8;      // accelerator complex dies of an MI355X

// MFMA tiles per wave (rows x cols); the workgroup is 2 x 2 waves.  Sized so
// that two stages of operand panels fit the 160 KiB of LDS.  BAND: R blocks per
// band of the tile walk (measured at n = 300: 1 is 5 % faster than 4 for FP64).
template <int M> struct FusedCfg;
template <> struct FusedCfg<MODE_F64> { static constexpr int WTI = 2, WTJ = 2, BAND = 1; };
// (the FP32 and fp16x2 modes run the two-v kernel of fused_f16.hip, bf16x3 that of
// fused_bf3.hip)

template <int M>
__global__ __launch_bounds__(NT) void fused_kernel(FusedArgs f) {
  using MT = ModeT<M>;
  using T = typename MT::T;
  constexpr int NP = MT::NP, KS = MT::KS, LD = lds_ld<T>();
  constexpr int WTI = FusedCfg<M>::WTI, WTJ = FusedCfg<M>::WTJ;
  constexpr int TR = 32 * WTI, TP = 32 * WTJ;
  constexpr int ES = (int)sizeof(T);
  using PR = Products<NP>;
  // two stages of panels: one is read by the matrix cores while the next is written
  __shared__ __attribute__((aligned(16))) T sG[2][NP][TR * LD];
  __shared__ __attribute__((aligned(16))) T sU[2][NP][TR * LD];
  __shared__ __attribute__((aligned(16))) T sA[2][NP][TP * LD];
  __shared__ __attribute__((aligned(16))) T sX[2][NP][TP * LD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  // XCD-aware placement.  Workgroups are dealt round-robin to the XCDs, so
  // workgroup b runs on XCD b % NXCD.  Each XCD takes vsplit / NXCD partial
  // slots z = xcd, xcd + NXCD, ... (a block of consecutive v ranges, below)
  // for every tile, and walks the tiles in bands of BAND R
  // blocks, P block by P block: the workgroups resident on one XCD at a time
  // form a compact BAND x (CUs per XCD / BAND) block of tiles at the same v,
  // which share the U_v and A_v panels through that XCD's L2.
  const int nrb = (f.naux + TR - 1) / TR, npb = (f.naux + TP - 1) / TP;
  const int tiles = nrb * npb;
  const int b = blockIdx.x;
  const int xcd = b % NXCD, local = b / NXCD;
  const int z = xcd + NXCD * (local / tiles);
  const int to = local % tiles;
  constexpr int BAND = FusedCfg<M>::BAND;
  const int band = to / (BAND * npb);
  const int rb0 = band * BAND, bh = min(BAND, nrb - rb0);
  const int within = to - rb0 * npb;
  const int P0 = (within / bh) * TP, R0 = (rb0 + within % bh) * TR;
  // symmetric D: a tile wholly below the diagonal is the mirror of one above it
  if (f.sym != nullptr && *f.sym != 0 && R0 >= P0 + TP) return;
  // v range: XCD x owns the consecutive ranges x q .. x q + q - 1 (q = vsplit / NXCD),
  // and the ranges split n as evenly as floor division allows, so every XCD gets
  // the same number of v to within one; range r is [r n / vsplit, (r + 1) n / vsplit)
  const int vr = (z % NXCD) * (f.vsplit / NXCD) + z / NXCD;
  const int v_lo = (int)((int64_t)vr * f.n / f.vsplit);
  const int v_hi = (int)((int64_t)(vr + 1) * f.n / f.vsplit);
  const int kst = f.ldk / BK;
  const int nstage = (v_hi > v_lo) ? (v_hi - v_lo) * kst : 0;
  const int64_t ldk = f.ldk;
  const int64_t u_row = (int64_t)f.n * ldk;        // elements between R rows of U
  const int64_t a_v = (int64_t)f.naux * ldk;       // elements between v slabs of A
  const int rows_r = min(TR, f.naux - R0), rows_p = min(TP, f.naux - P0);

  const T* Gt = static_cast<const T*>(f.Gt) + R0 * ldk;
  const T* GX = static_cast<const T*>(f.GXt) + P0 * ldk;
  const T* U = static_cast<const T*>(f.U) + R0 * u_row;
  __amdgpu_buffer_rsrc_t rG[NP], rX[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    rG[p] = make_rsrc(Gt + p * f.g_plane, TR * ldk * ES);
    rX[p] = make_rsrc(GX + p * f.g_plane, TP * ldk * ES);
  }

  Panel<T, TR> pG[NP], pU[NP];
  Panel<T, TP> pX[NP];
  Panel<T, TP> pA[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    pG[p].init(ldk, rows_r, tid);
    pU[p].init(u_row, rows_r, tid);
    pX[p].init(ldk, rows_p, tid);
    pA[p].init(ldk, rows_p, tid);
  }

  auto load_stage = [&](int v, int k0) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      pG[p].load(rG[p], k0);
      pX[p].load(rX[p], k0);
      pU[p].load(make_rsrc(U + p * f.u_plane + v * ldk, TR * u_row * ES), k0);
    }
#pragma unroll
    for (int p = 0; p < NP; ++p)
      pA[p].load(make_rsrc(static_cast<const T*>(f.A) + p * f.a_plane + v * a_v + P0 * ldk,
                           TP * ldk * ES),
                 k0);
  };

  using DAcc = typename std::conditional<M == MODE_F64, double, float>::type;
  typename MT::Acc accB[WTI][WTJ], accC[WTI][WTJ];
  DAcc accD[WTI][WTJ][4];
#pragma unroll
  for (int ti = 0; ti < WTI; ++ti)
#pragma unroll
    for (int tj = 0; tj < WTJ; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        accB[ti][tj][r] = 0;
        accC[ti][tj][r] = 0;
        accD[ti][tj][r] = 0;
      }
  double* D = f.Dpart + (int64_t)z * f.naux * f.naux;
  float* D32 = reinterpret_cast<float*>(f.Dpart) + (int64_t)z * f.naux * f.naux;
  // add (or, the first time, store) the register partial sums into the FP64 tile
  auto flush = [&](bool first) {
#pragma unroll
    for (int ti = 0; ti < WTI; ++ti)
#pragma unroll
      for (int tj = 0; tj < WTJ; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int R = R0 + wr * 16 * WTI + 16 * ti + out_row<M>(lane, r);
          const int P = P0 + wc * 16 * WTJ + 16 * tj + (lane & 15);
          if (R < f.naux && P < f.naux) {
            if (f.dpart_f32) {   // one range = one FP32 partial sum (first is true)
              D32[(int64_t)R * f.naux + P] = (float)accD[ti][tj][r];
            } else {
              double* d = D + (int64_t)R * f.naux + P;
              *d = (first ? 0.0 : *d) + (double)accD[ti][tj][r];
            }
          }
          accD[ti][tj][r] = 0;
        }
  };
  int nv = 0;

  // stage sequence: (v, ks) for v in [v_lo, v_hi), ks in [0, kst); (lv, lk) is the
  // next stage to fetch from global memory
  int lv = v_lo, lk = 0;
  auto fetch_next = [&]() {
    load_stage(lv, lk * BK);
    if (++lk == kst) { lk = 0; ++lv; }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      pG[p].store(sG[buf][p], tid);
      pU[p].store(sU[buf][p], tid);
      pX[p].store(sX[buf][p], tid);
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) pA[p].store(sA[buf][p], tid);
  };
  // acc[ti][tj] += sum_k rows(sr) x rows(sc) over this stage's 32-wide k range
  auto gemm = [&](typename MT::Acc (&acc)[WTI][WTJ], T (*sr)[TR * LD], T (*sc)[TP * LD]) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += KS) {
      typename MT::Frag fr[WTI][NP], fc[WTJ][NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
#pragma unroll
        for (int ti = 0; ti < WTI; ++ti)
          fr[ti][p] = lds_frag<M>(sr[p], LD, wr * 16 * WTI + 16 * ti, kk, lane);
#pragma unroll
        for (int tj = 0; tj < WTJ; ++tj)
          fc[tj][p] = lds_frag<M>(sc[p], LD, wc * 16 * WTJ + 16 * tj, kk, lane);
      }
#pragma unroll
      for (int q = 0; q < PR::N; ++q)
#pragma unroll
        for (int ti = 0; ti < WTI; ++ti)
#pragma unroll
          for (int tj = 0; tj < WTJ; ++tj)
            acc[ti][tj] = mfma1(fr[ti][PR::a(q)], fc[tj][PR::b(q)], acc[ti][tj]);
    }
  };

  if (nstage > 0) {
    fetch_next();
    put(0);
  }
  if (nstage > 1) fetch_next();
  __syncthreads();
  int t = 0;
  for (int v = v_lo; v < v_hi; ++v) {
#pragma unroll
    for (int ti = 0; ti < WTI; ++ti)
#pragma unroll
      for (int tj = 0; tj < WTJ; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          accB[ti][tj][r] = 0;
          accC[ti][tj][r] = 0;
        }
    for (int ks = 0; ks < kst; ++ks, ++t) {
      const int cur = t & 1;
      gemm(accB, sG[cur], sA[cur]);
      // while those run: stage t+1 (already in registers) into the other buffer,
      // and start fetching stage t+2
      if (t + 1 < nstage) put(cur ^ 1);
      if (t + 2 < nstage) fetch_next();
      gemm(accC, sU[cur], sX[cur]);
      __syncthreads();
    }
    // all k of this v done: D += B o C
#pragma unroll
    for (int ti = 0; ti < WTI; ++ti)
#pragma unroll
      for (int tj = 0; tj < WTJ; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          accD[ti][tj][r] = fma((DAcc)accB[ti][tj][r], (DAcc)accC[ti][tj][r], accD[ti][tj][r]);
    ++nv;
    if (M != MODE_F64 && (nv % FLUSH_V == 0) && v + 1 < v_hi) flush(nv == FLUSH_V);
  }
  // final flush (also writes zeros for an empty v range)
  flush(M == MODE_F64 || nv <= FLUSH_V);
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

template <int M> void tile_of(int* rows, int* cols) {
  *rows = 32 * FusedCfg<M>::WTI;
  *cols = 32 * FusedCfg<M>::WTJ;
}

void fused_tile(int mode, int* rows, int* cols) {
  switch (mode) {
    case MODE_F64: tile_of<MODE_F64>(rows, cols); break;
    default: fused_f16_tile(rows, cols); break;   // FP32, fp16x2 and bf16x3: 128 x 128
  }
}

int fused_xcds() { return NXCD; }

hipError_t sox_fused(int mode, const FusedArgs& f, hipStream_t s) {
  if (mode == MODE_F16X2 || mode == MODE_F32) return sox_fused_pairs(mode, f, s);   // own checks
  if (mode == MODE_BF16X3) return sox_fused_bf3(f, s);
  int TR, TP;
  fused_tile(mode, &TR, &TP);
  if (f.vsplit % NXCD != 0 || (int64_t)f.vsplit * f.vchunk < f.n) return hipErrorInvalidValue;
  // FP32 partial tiles only where each range is one FP32 partial sum
  if (f.dpart_f32 && (mode == MODE_F64 || f.vchunk > FLUSH_V)) return hipErrorInvalidValue;
  // buffer offsets inside one tile's rows of U are 32-bit
  if ((int64_t)std::max(TR, TP) * f.n * f.ldk * 8 > 0x7fffffffLL) return hipErrorInvalidValue;
  dim3 grid(cdiv(f.naux, TP) * cdiv(f.naux, TR) * f.vsplit);
  switch (mode) {
    case MODE_F64: fused_kernel<MODE_F64><<<grid, NT, 0, s>>>(f); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace thcsox
