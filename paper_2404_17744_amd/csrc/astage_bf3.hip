// The A stage in the bf16x3 mode:
//
//   A_Pqv = sum_s U_Pqs G_sv(beta - tau)
//
// as C(i, j) = sum_k Uop[i][k] Gop[j][k] with Uop the rows i = (P, q) of U and
// Gop the rows v of G(beta - tau)^T, each three K-major bf16 planes x = x0 + x1
// + x2 (rows of ldk elements, planes u_plane and gb_plane elements apart).  The
// six plane products x_a y_b with a + b <= 2 run on the bf16 matrix cores
// (16x16x32, FP32 accumulation), and every FP32 result is split again into the
// three bf16 planes of A: rows (v, P) with k = q, planes a_plane elements apart,
// which is what the fused stage loads.
//
// G lives in registers.  Wave w of a workgroup keeps the fragments of NCT
// 16-column tiles (columns v) for every k chunk and plane, 12 NCT KST registers
// (360 at NCT = 3 and ldk = 320), so a workgroup covers 64 NCT columns.  Past 12
// tiles (n > 192) the columns form two blocks, the first 12 tiles (NCT = 3) and
// the rest (NCT1 <= 2), each served by its own workgroups; a wave whose tiles lie
// past n computes zeros that are never stored.  Only U streams through LDS: a
// step is 32 rows of the padded row space i = P ldk + q (one 32-wide q chunk of
// one P, all KST k chunks, three planes: 6 KST KiB), loaded from memory straight
// into one of two LDS buffers one step ahead.  Rows q >= n read U as zero and
// give the zero rows of A that pad the fused stage's k range.
//
// Workers are persistent, one per compute unit.  The steps form eight
// contiguous ranges, one per XCD; on an XCD the workers of the two column blocks
// walk its range at the same pace (their numbers in the ratio of the blocks'
// tiles per wave), so a step of U is fetched from HBM about once and served to
// the other block from that XCD's L2.
//
// Epilogue: the MFMA takes the U fragment as its row operand, so a lane's four
// outputs are four consecutive q of one v: one 8-byte store per plane.  The
// first half of a step is stored as soon as it is split, the second half is held
// in registers and stored at the top of the next step, so that both complete
// under matrix work.
#include <algorithm>

#include "kernels.hpp"
#include "mfma.hpp"
#include "panel.hpp"

namespace thcsox {
namespace {

constexpr int BRM = 32;              // rows i per step
constexpr int BNW = 4, BNT = 64 * BNW;
constexpr int BMAXT = 20;            // column tiles of both blocks at most (ldk <= 320)

// One step of U: [plane][k chunk][row][32], 64-byte rows whose four 16-byte
// pieces are placed by lds_chunk (16 rows read at one logical piece hit distinct
// banks).
template <int KST> struct B3Buf {
  __bf16 u[3][KST][BRM * 32];
};

__device__ __forceinline__ void b3_barrier() {
  __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

// One worker: the steps first, first + stride, ... below last, columns from
// 16 tile0 on (wave w: tiles tile0 + NCT w .. + NCT - 1).
template <int KST, int NCT>
__device__ __forceinline__ void astage_b3_body(const AStageB3Args& g, B3Buf<KST>& b0,
                                               B3Buf<KST>& b1, int tile0, int first, int last,
                                               int stride) {
  constexpr int LDK = 32 * KST;
  using PR = Products<3>;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nst = __builtin_amdgcn_readfirstlane(first < last ? (last - 1 - first) / stride + 1 : 0);
  if (nst == 0) return;
  const int lr = lane & 15, kc = lane >> 4;
  const int vb = 16 * (tile0 + NCT * wave);   // first column of this wave

  // this wave's G fragments: column v = vb + 16 t + lane % 16, k = 32 c + 8 (lane
  // / 16) .. + 7 of plane p; rows v >= n lie past the end of the resource and
  // read as zero
  __amdgpu_buffer_rsrc_t rG[3];
#pragma unroll
  for (int p = 0; p < 3; ++p)
    rG[p] = make_rsrc(static_cast<const __bf16*>(g.Gb) + p * g.gb_plane, (int64_t)g.n * LDK * 2);
  bf16x8 gr[NCT][KST][3];
  // the first fragments live in AGPRs (the matrix cores read them there), as many
  // as fit beside the accumulators; the rest in VGPRs
  constexpr int NF = 3 * NCT * KST;
  constexpr int NG_A = (256 - 4 * NCT) / 4 < NF ? (256 - 4 * NCT) / 4 : NF;
  auto in_agpr = [](int t, int c, int p) { return (t * KST + c) * 3 + p < NG_A; };
  // (loaded in batches of 16, the AGPR moves of a batch after the next batch is
  // issued, so that each waits for about one batch's latency)
  constexpr int GB = 16;
  auto gload = [&](int f) {
    const int t = f / (3 * KST), c = (f / 3) % KST, p = f % 3;
    const uint32_t gv = (uint32_t)(((vb + 16 * t + lr) * LDK + 8 * kc) * 2);
    gr[t][c][p] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rG[p], gv, c * 64, 0));
  };
#pragma unroll
  for (int f = 0; f < GB && f < NF; ++f) gload(f);
#pragma unroll
  for (int f0 = 0; f0 < NF; f0 += GB) {
#pragma unroll
    for (int f = f0 + GB; f < f0 + 2 * GB && f < NF; ++f) gload(f);
#pragma unroll
    for (int f = f0; f < f0 + GB && f < NF; ++f) {
      const int t = f / (3 * KST), c = (f / 3) % KST, p = f % 3;
      if (in_agpr(t, c, p)) __asm__ volatile("" : "+a"(gr[t][c][p]));
    }
  }

  // memory to LDS: one instruction moves 16 rows of one k chunk of one plane (16
  // rows x 64 bytes); per plane the 2 KST instructions m = 2 c + h (rows 16 h ..
  // 16 h + 15 of chunk c) go to the waves in turn.  Lane l lands at row 16 h + l /
  // 4, physical piece l % 4, and loads the logical piece lds_chunk maps there.
  const __bf16* const Ub = static_cast<const __bf16*>(g.U);
  uint32_t dvoff[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int row = 16 * h + (lane >> 2);
    dvoff[h] = (uint32_t)((row * LDK + 8 * lds_chunk(row, lane & 3)) * 2);
  }
  auto dma = [&](B3Buf<KST>& bf, int s) {
    const int st = first + s * stride, P = st / KST, q0 = 32 * (st - P * KST);
    const int nv = min(BRM, g.n - q0);   // rows q < n of this step (none past n)
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const i4 r = raw_rsrc(Ub + p * g.u_plane + ((int64_t)P * g.n + q0) * LDK, nv > 0 ? nv * LDK * 2 : 0);
#pragma unroll
      for (int i = 0; i < (2 * KST + BNW - 1) / BNW; ++i) {
        const int m = wave + BNW * i;
        if (m < 2 * KST) {
          const int c = m >> 1, h = m & 1;
          dma16_untracked(r, lds_addr(&bf.u[p][c][16 * h * 32]), dvoff[h], c * 64);
        }
      }
    }
  };

  // fragment (row 16 a + lane % 16, k piece lane / 16) of a chunk
  int uoff[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) uoff[a] = (16 * a + lr) * 32 + 8 * lds_chunk(16 * a + lr, kc);
  // the two 16-row halves of a step run one after the other on the same
  // accumulators (16 x 16 NCT of A per wave)
  f4 acc[NCT];
  auto compute = [&](const B3Buf<KST>& bf, int a) {
    // the fragments of chunk c + 1 are read while chunk c's MFMAs run
    bf16x8 u[3], un[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) un[p] = *reinterpret_cast<const bf16x8*>(&bf.u[p][0][uoff[a]]);
#pragma unroll
    for (int c = 0; c < KST; ++c) {
#pragma unroll
      for (int p = 0; p < 3; ++p) u[p] = un[p];
      if (c + 1 < KST) {
#pragma unroll
        for (int p = 0; p < 3; ++p) un[p] = *reinterpret_cast<const bf16x8*>(&bf.u[p][c + 1][uoff[a]]);
      }
#pragma unroll
      for (int q = 0; q < PR::N; ++q) {
        const int pu = PR::a(q), pg = PR::b(q);
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
          if (in_agpr(t, c, pg)) __asm__ volatile("" : "+a"(gr[t][c][pg]));
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              u[pu], gr[t][c][pg], (c == 0 && q == 0) ? f4{0.f, 0.f, 0.f, 0.f} : acc[t], 0, 0, 0);
        }
      }
    }
  };

  // stores: the lane's four q of column v at (v c_j + 16 a + 4 (lane / 16)) elements
  // from the step's piece of row (0, P) of a plane (offsets below 2^31: checked on
  // the host); columns v >= n lie past the end of the resource and are dropped
  __bf16* const A = static_cast<__bf16*>(g.A);
  const int64_t c_j = (int64_t)g.naux * LDK;
  uint32_t cvoff[NCT];
#pragma unroll
  for (int t = 0; t < NCT; ++t) cvoff[t] = (uint32_t)(((vb + 16 * t + lr) * c_j + 4 * kc) * 2);
  auto store_half = [&](int s, int a, const bf16x4 (&x)[NCT][3]) {
    const int st = first + s * stride, P = st / KST, q0 = 32 * (st - P * KST);
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const __amdgpu_buffer_rsrc_t rC =
          make_rsrc(A + p * g.a_plane + (int64_t)P * LDK + q0, (int64_t)(g.n - 1) * c_j * 2 + 64);
#pragma unroll
      for (int t = 0; t < NCT; ++t)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x[t][p]), rC, cvoff[t] + 32 * a, 0, 0);
    }
  };
  // the three planes of the accumulators (x = x0 + x1 + x2; the first
  // difference is exact in FP32)
  auto split = [&](bf16x4 (&x)[NCT][3]) {
#pragma unroll
    for (int t = 0; t < NCT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float v = acc[t][r];
        const __bf16 h = (__bf16)v;
        const float r1 = v - (float)h;
        const __bf16 m = (__bf16)r1;
        x[t][0][r] = h;
        x[t][1][r] = m;
        x[t][2][r] = (__bf16)(r1 - (float)m);
      }
  };
  // half 0 of a step is stored at once (it completes under half 1's matrix work),
  // half 1 is held and stored at the top of the next step
  bf16x4 hold[NCT][3];
  // a half whose rows are all past n (pad rows of A) is zero without its MFMAs
  auto run_step = [&](B3Buf<KST>& bf, int s) {
    const int st = first + s * stride, q0 = 32 * (st - (st / KST) * KST);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      if (q0 + 16 * a < g.n) {
        compute(bf, a);
      } else {
#pragma unroll
        for (int t = 0; t < NCT; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
      }
      if (a == 0) {
        bf16x4 x[NCT][3];
        split(x);
        store_half(s, 0, x);
      } else {
        split(hold);
      }
    }
  };

  // one step ahead: at the top of step s its loads have landed (every wave's) and
  // every wave is done with the other buffer, which then takes the loads of step
  // s + 1; the held half of step s - 1 is stored first
  dma(b0, 0);
  for (int s = 0; s < nst; s += 2) {
    b3_barrier();
    if (s > 0) store_half(s - 1, 1, hold);
    if (s + 1 < nst) dma(b1, s + 1);
    run_step(b0, s);
    if (s + 1 >= nst) { store_half(s, 1, hold); break; }
    b3_barrier();
    store_half(s, 1, hold);
    if (s + 2 < nst) dma(b0, s + 2);
    run_step(b1, s + 1);
    if (s + 2 >= nst) store_half(s + 1, 1, hold);
  }
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// KST k chunks; NCT0 tiles per wave in the first column block, NCT1 in the second
// (0: one block).  Workgroup b runs on XCD b mod 8; slots b / 8 below wx0 serve
// the first block, the next wx1 the second.
template <int KST, int NCT0, int NCT1>
__global__ __launch_bounds__(BNT) __attribute__((amdgpu_waves_per_eu(1, 1)))
void astage_bf3r_kernel(AStageB3Args g) {
  __shared__ __attribute__((aligned(16))) B3Buf<KST> b0;
  __shared__ __attribute__((aligned(16))) B3Buf<KST> b1;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int nstep = g.naux * KST;
  const int lo = (int)((int64_t)nstep * xcd / 8), hi = (int)((int64_t)nstep * (xcd + 1) / 8);
  if (NCT1 == 0 || slot < g.wx0) {
    astage_b3_body<KST, NCT0>(g, b0, b1, 0, lo + slot, hi, g.wx0);
  } else if constexpr (NCT1 > 0) {
    astage_b3_body<KST, NCT1>(g, b0, b1, 4 * NCT0, lo + slot - g.wx0, hi, g.wx1);
  }
}

inline int tiles_per_wave(int tiles) { return (tiles + BNW - 1) / BNW; }

template <int KST, int NCT0, int NCT1>
hipError_t b3_launch(AStageB3Args g, hipStream_t s) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int wx = std::max(1, cus / 8);   // workers per XCD
  if (NCT1 == 0) {
    g.wx0 = wx; g.wx1 = 0;
  } else {
    g.wx0 = std::min(wx - 1, std::max(1, (wx * NCT0 + (NCT0 + NCT1) / 2) / (NCT0 + NCT1)));
    g.wx1 = std::max(1, wx - g.wx0);
  }
  astage_bf3r_kernel<KST, NCT0, NCT1><<<8 * (g.wx0 + g.wx1), BNT, 0, s>>>(g);
  return hipGetLastError();
}

}  // namespace

bool astage_bf3_fits(int n, int naux, int ldk) {
  if (n <= 0 || naux <= 0 || ldk % 32 != 0 || ldk < n || ldk > 32 * 10 || ldk >= n + 32) return false;
  // byte offsets of the stores (columns up to 16 BMAXT) and of U's rows in 32 bits
  return (int64_t)16 * BMAXT * naux * ldk * 2 < 0x7fffffffLL;
}

hipError_t astage_bf3(const AStageB3Args& g, hipStream_t s) {
  if (g.naux <= 0 || g.n <= 0) return hipSuccess;
  if (!astage_bf3_fits(g.n, g.naux, g.ldk)) return hipErrorInvalidValue;
  // ldk = 32 ceil(n / 32): the tile counts follow from the chunk count
  const int tiles = (g.n + 15) / 16;
  const int nct0 = tiles > 12 ? 3 : tiles_per_wave(tiles);
  const int nct1 = tiles > 12 ? tiles_per_wave(tiles - 12) : 0;
  auto pick = [&](int k, int a, int b) { return g.ldk == 32 * k && nct0 == a && nct1 == b; };
  if (pick(1, 1, 0)) return b3_launch<1, 1, 0>(g, s);
  if (pick(2, 1, 0)) return b3_launch<2, 1, 0>(g, s);
  if (pick(3, 2, 0)) return b3_launch<3, 2, 0>(g, s);
  if (pick(4, 2, 0)) return b3_launch<4, 2, 0>(g, s);
  if (pick(5, 3, 0)) return b3_launch<5, 3, 0>(g, s);
  if (pick(6, 3, 0)) return b3_launch<6, 3, 0>(g, s);
  if (pick(7, 3, 1)) return b3_launch<7, 3, 1>(g, s);
  if (pick(8, 3, 1)) return b3_launch<8, 3, 1>(g, s);
  if (pick(9, 3, 2)) return b3_launch<9, 3, 2>(g, s);
  if (pick(10, 3, 2)) return b3_launch<10, 3, 2>(g, s);
  return hipErrorInvalidValue;
}

}  // namespace thcsox
