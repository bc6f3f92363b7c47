// The fused B/C/D stage in the fp16x2 mode, 128 x 128 tiles of D per workgroup:
//
//   D_PR = sum_v C_RvP B_PRv,   B_PRv = sum_q G_Rq A_Pqv,   C_RvP = sum_w U_Rvw G_wP
//
// Every operand is a power-of-two scaled value split into two fp16 planes
// x = x0 + x1; a product is formed from the plane products x1 y0 + x0 y1 + x0 y0
// on the f16 matrix cores (16x16x32, FP32 accumulation).
//
// Eight waves (two per SIMD) in a 2 x 4 arrangement each own a 64 x 32 sub-tile
// (4 x 2 MFMA tiles) of accB, accC and the FP32 partial sum of D; everything a
// wave holds fits its 256 registers, so the two waves of a SIMD hide each
// other's LDS and memory latency.  A stage is one v and one
// 32-wide k chunk: four panels (G rows R, U_v rows R, A_v rows P, GX rows P) of
// 128 rows x 32 k in two fp16 planes, 64 KiB, double buffered in LDS (128 KiB).
// The fp16 panels are loaded from memory directly into LDS; the A panel arrives
// as FP32 in registers and is split while it is written to LDS.
//
// The loop is software pipelined so that the matrix cores, the LDS and the
// memory system work at the same time.  With cur = t mod 2, stage t runs as
//   phase 1: fragments of the C product (stage t)   <- LDS buffer cur,
//            matrix cores: B product, first 32 of 48 MFMAs;
//   phase 2: A of stage t+1 (registers) -> LDS buffer cur^1,
//            matrix cores: last 16 MFMAs of B, first 16 of C;
//   wait for this wave's loads, barrier;
//   phase 3: fragments of the B product (stage t+1) <- LDS buffer cur^1,
//            loads of stage t+2 -> LDS buffer cur and registers,
//            matrix cores: last 32 MFMAs of C.
// The loop body has no branches: past the last stage the loads repeat the last
// stage and the extra panels written to LDS are never used.  The operand row
// length (ldk) is a multiple of 64, so each v takes an even number of stages
// and the loop runs two stages per trip with the buffers fixed at compile time.
#include "kernels.hpp"
#include "mfma.hpp"
#include "panel.hpp"

namespace thcsox {
namespace {

constexpr int TT = 128;        // tile edge of D (R and P)
constexpr int WR_ = 2, WP_ = 4;                 // waves along R and along P
constexpr int NW = WR_ * WP_, NTH = 64 * NW;
constexpr int WBR = TT / 16 / WR_, WBP = TT / 16 / WP_;   // MFMA tiles per wave
constexpr int KC = 32;         // k per stage (one f16 MFMA)
constexpr int PANEL = TT * KC; // halves per panel plane
constexpr int FLUSH16 = 8;     // v per FP32 partial sum of D
constexpr int NXCD16 = 8;
constexpr int BAND16 = 2;   // R blocks per band (measured: 2 beats 1, 3, 4, 5, 6, 8, 15)

typedef _Float16 h4 __attribute__((ext_vector_type(4)));

// One LDS stage buffer: [panel G, U, A, X][plane][row * 32 + physical chunk * 8 + e].
// The two buffers are separate objects and every access names one of them at
// compile time, so the compiler can tell that reads of one buffer do not wait
// for memory-to-LDS loads still landing in the other.
struct Buf {
  _Float16 s[4][2][PANEL];
};

__device__ __forceinline__ void vm_lds_barrier() {
  // This wave's memory loads (including those that write LDS) and LDS accesses
  // complete, then the workgroup barrier.
  __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(NW / 4, NW / 4)))
void fused_f16_kernel(FusedArgs f) {
  __shared__ __attribute__((aligned(16))) Buf sb0;
  __shared__ __attribute__((aligned(16))) Buf sb1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WP_, wc = wave % WP_;

  // tile and v range: XCD-aware order (workgroup b runs on XCD b mod 8; each XCD
  // owns the partial slots z = xcd, xcd + 8, ..., a block of consecutive v ranges
  // (below), and walks the tiles in bands of BAND16
  // R blocks so its resident workgroups share U_v and A_v panels in its L2)
  const int nb = (f.naux + TT - 1) / TT;
  const int tiles = nb * nb;
  const int b = blockIdx.x;
  const int xcd = b % NXCD16, local = b / NXCD16;
  const int z = xcd + NXCD16 * (local / tiles);
  const int to = local % tiles;
  const int band = to / (BAND16 * nb);
  const int rb0 = band * BAND16, bh = min(BAND16, nb - rb0);
  const int within = to - rb0 * nb;
  const int P0 = (within / bh) * TT, R0 = (rb0 + within % bh) * TT;
  if (f.sym != nullptr && *f.sym != 0 && R0 >= P0 + TT) return;

  // v range: XCD x owns the consecutive ranges x q .. x q + q - 1 (q = vsplit / NXCD16),
  // and the ranges split n as evenly as floor division allows, so every XCD gets
  // the same number of v to within one; range r is [r n / vsplit, (r + 1) n / vsplit)
  const int vr = (z % NXCD16) * (f.vsplit / NXCD16) + z / NXCD16;
  const int v_lo = (int)((int64_t)vr * f.n / f.vsplit);
  const int v_hi = (int)((int64_t)(vr + 1) * f.n / f.vsplit);
  const int kst = f.ldk / KC;
  const int nstage = (v_hi > v_lo) ? (v_hi - v_lo) * kst : 0;
  const int64_t ldk = f.ldk;
  const int64_t u_row = (int64_t)f.n * ldk;     // elements between R rows of U
  const int64_t a_v = (int64_t)f.naux * ldk;    // elements between v slabs of A
  const float a_scale = (float)pow2_scale_f(f.amax_a);
  const int rows_r = min(TT, f.naux - R0), rows_p = min(TT, f.naux - P0);

  const _Float16* Gt = static_cast<const _Float16*>(f.Gt) + R0 * ldk;
  const _Float16* GX = static_cast<const _Float16*>(f.GXt) + P0 * ldk;
  const _Float16* U = static_cast<const _Float16*>(f.U) + R0 * u_row;
  const float* A = static_cast<const float*>(f.A) + P0 * ldk;
  __amdgpu_buffer_rsrc_t rG[2], rX[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    rG[p] = make_rsrc(Gt + p * f.g_plane, TT * ldk * 2);
    rX[p] = make_rsrc(GX + p * f.g_plane, TT * ldk * 2);
  }

  // The fp16 panels (G, U_v, GX) go from memory straight into LDS (buffer loads
  // with the LDS destination): wave w moves the 16-row slabs w, w + NW, ... of
  // each panel plane (one slab with eight waves); lane l lands at slab row l / 4, physical chunk l % 4, so it
  // loads the logical chunk that the swizzle maps there.  Rows past the end of
  // naux read as zero (their offsets point out of the buffer).
  constexpr int SL = 8 / NW;   // 16-row slabs per wave and panel plane
  uint32_t dg[SL], du[SL], dx[SL];
#pragma unroll
  for (int j = 0; j < SL; ++j) {
    const int row = (wave + NW * j) * 16 + (lane >> 2);
    const int c = lds_chunk(row, lane & 3);   // the map is its own inverse
    dg[j] = row < rows_r ? (uint32_t)((row * ldk + 8 * c) * 2) : OOB;
    du[j] = row < rows_r ? (uint32_t)((row * u_row + 8 * c) * 2) : OOB;
    dx[j] = row < rows_p ? (uint32_t)((row * ldk + 8 * c) * 2) : OOB;
  }
  auto dma = [&](Buf& b, int v, int k0) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const __amdgpu_buffer_rsrc_t rU =
          make_rsrc(U + p * f.u_plane + (int64_t)v * ldk, (int64_t)TT * u_row * 2);
#pragma unroll
      for (int j = 0; j < SL; ++j) {
        const int slab = (wave + NW * j) * 16 * KC;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rG[p], &b.s[0][p][slab], 16, dg[j], k0 * 2, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rU, &b.s[1][p][slab], 16, du[j], k0 * 2, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rX[p], &b.s[3][p][slab], 16, dx[j], k0 * 2, 0, 0);
      }
    }
  };
  // the FP32 A panel is staged through registers (1024 / NTH units of 4 floats
  // per thread: row u/8, piece u%8, u = tid + NTH i) and split when written to LDS
  constexpr int AU = 1024 / NTH;
  uint32_t offa[AU];
  int lda_[AU];
#pragma unroll
  for (int i = 0; i < AU; ++i) {
    const int u = tid + i * NTH, row = u >> 3, c4 = u & 7;
    offa[i] = row < rows_p ? (uint32_t)((row * ldk + 4 * c4) * 4) : OOB;
    lda_[i] = row * KC + lds_chunk(row, c4 >> 1) * 8 + (c4 & 1) * 4;
  }
  f4 ra[AU];
  auto fetch_a = [&](int v, int k0) {
    const __amdgpu_buffer_rsrc_t rA = make_rsrc(A + (int64_t)v * a_v, (int64_t)TT * ldk * 4);
#pragma unroll
    for (int i = 0; i < AU; ++i)
      ra[i] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rA, offa[i], k0 * 4, 0));
  };
  auto put_a = [&](Buf& b) {
#pragma unroll
    for (int i = 0; i < AU; ++i) {
      h4 hi, lo;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float x = ra[i][e] * a_scale;
        const _Float16 h = (_Float16)x;
        hi[e] = h;
        lo[e] = (_Float16)(x - (float)h);
      }
      *reinterpret_cast<h4*>(&b.s[2][0][lda_[i]]) = hi;
      *reinterpret_cast<h4*>(&b.s[2][1][lda_[i]]) = lo;
    }
  };

  // fragment reads: R side rows wr*64 + 16 ti, P side rows wc*64 + 16 tj
  int fr_off[WBR], fc_off[WBP];
#pragma unroll
  for (int t = 0; t < WBR; ++t) {
    const int r = wr * 16 * WBR + 16 * t + (lane & 15);
    fr_off[t] = r * KC + lds_chunk(r, lane >> 4) * 8;
  }
#pragma unroll
  for (int t = 0; t < WBP; ++t) {
    const int c = wc * 16 * WBP + 16 * t + (lane & 15);
    fc_off[t] = c * KC + lds_chunk(c, lane >> 4) * 8;
  }
  struct Frags { f16x8 r[2][WBR], c[2][WBP]; };   // [plane][tile]
  Frags fB, fC;
  auto read_frags = [&](Frags& fr, const Buf& b, int pr, int pc) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
#pragma unroll
      for (int t = 0; t < WBR; ++t)
        fr.r[p][t] = *reinterpret_cast<const f16x8*>(&b.s[pr][p][fr_off[t]]);
#pragma unroll
      for (int t = 0; t < WBP; ++t)
        fr.c[p][t] = *reinterpret_cast<const f16x8*>(&b.s[pc][p][fc_off[t]]);
    }
  };

  f4 accB[WBR][WBP], accC[WBR][WBP];
  float accD[WBR][WBP][4];
#pragma unroll
  for (int i = 0; i < WBR; ++i)
#pragma unroll
    for (int j = 0; j < WBP; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) accD[i][j][r] = 0.f;

  // MFMA number q (0..47) of one product: tile (q / 3) of the 4 x 4, plane pair q % 3
  constexpr int NQ = WBR * WBP * 3;   // MFMAs per product and stage
  auto mfma_range = [&](f4 (&acc)[WBR][WBP], const Frags& fr, int q0, int q1) {
#pragma unroll
    for (int q = q0; q < q1; ++q) {
      const int tile = q / 3, pp = q % 3;
      const int ti = tile / WBP, tj = tile % WBP;
      const int pa = pp == 0 ? 1 : 0, pb = pp == 1 ? 1 : 0;
      acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.r[pa][ti], fr.c[pb][tj],
                                                           acc[ti][tj], 0, 0, 0);
    }
  };

  // this lane's first element of D: row R0 + wr*64 + 4*(lane/16), column P0 + wc*64 + lane%16
  const int Rl = R0 + wr * 16 * WBR + 4 * (lane >> 4), Pl = P0 + wc * 16 * WBP + (lane & 15);
  const int64_t dl_off = (int64_t)z * f.naux * f.naux + (int64_t)Rl * f.naux + Pl;
  double* const Dl = f.Dpart + dl_off;
  float* const Dl32 = reinterpret_cast<float*>(f.Dpart) + dl_off;
  auto flush = [&](bool first) {
#pragma unroll
    for (int ti = 0; ti < WBR; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool row_ok = Rl + 16 * ti + r < f.naux;
#pragma unroll
        for (int tj = 0; tj < WBP; ++tj) {
          if (row_ok && Pl + 16 * tj < f.naux) {
            if (f.dpart_f32) {   // one range = one FP32 partial sum (first is true)
              Dl32[(16 * ti + r) * f.naux + 16 * tj] = accD[ti][tj][r];
            } else {
              double* d = Dl + (16 * ti + r) * f.naux + 16 * tj;
              *d = (first ? 0.0 : *d) + (double)accD[ti][tj][r];
            }
          }
          accD[ti][tj][r] = 0.f;
        }
      }
  };

  // next stage to fetch, clamped to the last one
  int lv = v_lo, lk = 0;
  auto advance = [&]() {
    const bool last = (lv == v_hi - 1) && (lk == kst - 1);
    const bool wrap = (lk == kst - 1);
    lk = last ? lk : (wrap ? 0 : lk + 1);
    lv = last ? lv : (wrap ? lv + 1 : lv);
  };

  if (nstage > 0) {
    dma(sb0, lv, lk * KC);
    fetch_a(lv, lk * KC);
    advance();
    put_a(sb0);
    dma(sb1, lv, lk * KC);
    fetch_a(lv, lk * KC);
    advance();
    vm_lds_barrier();
    read_frags(fB, sb0, 0, 2);
  }
  // one stage; `cur` holds stage t, `nxt` receives stage t+1 (already loading)
  auto stage = [&](Buf& cur, Buf& nxt) {
    // phase 1: C fragments of stage t; B product
    read_frags(fC, cur, 1, 3);
    mfma_range(accB, fB, 0, 2 * NQ / 3);
    // phase 2: A of stage t+1 into the other buffer; C product starts
    mfma_range(accB, fB, 2 * NQ / 3, NQ);
    put_a(nxt);
    mfma_range(accC, fC, 0, NQ / 3);
    // stage t+1 complete in LDS (its memory-to-LDS loads were issued one phase 3 ago)
    vm_lds_barrier();
    // phase 3: B fragments of stage t+1; stage t+2 loads into this buffer
    read_frags(fB, nxt, 0, 2);
    dma(cur, lv, lk * KC);
    fetch_a(lv, lk * KC);
    advance();
    mfma_range(accC, fC, NQ / 3, NQ);
  };
  int nv = 0;
  for (int v = v_lo; v < v_hi; ++v) {
#pragma unroll
    for (int i = 0; i < WBR; ++i)
#pragma unroll
      for (int j = 0; j < WBP; ++j) {
        accB[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        accC[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
    // kst is even, so every v starts on buffer 0
    for (int ks = 0; ks < kst; ks += 2) {
      stage(sb0, sb1);
      stage(sb1, sb0);
    }
#pragma unroll
    for (int i = 0; i < WBR; ++i)
#pragma unroll
      for (int j = 0; j < WBP; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) accD[i][j][r] = fmaf(accB[i][j][r], accC[i][j][r], accD[i][j][r]);
    ++nv;
    if ((nv % FLUSH16 == 0) && v + 1 < v_hi) flush(nv == FLUSH16);
  }
  // the last (repeated) memory-to-LDS loads land before the workgroup may end
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
  flush(nv <= FLUSH16);   // also writes zeros for an empty v range
}

inline unsigned cdiv16(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

void fused_f16_tile(int* rows, int* cols) {
  *rows = TT;
  *cols = TT;
}

hipError_t sox_fused_f16(const FusedArgs& f, hipStream_t s) {
  if (!f.a_f32 || f.vsplit % NXCD16 != 0 || (int64_t)f.vsplit * f.vchunk < f.n ||
      (f.dpart_f32 && f.vchunk > FLUSH16) ||
      f.ldk % (2 * KC) != 0)
    return hipErrorInvalidValue;
  // buffer offsets inside one tile's rows of U (fp16) and A (FP32) are 32-bit
  if ((int64_t)TT * f.n * f.ldk * 2 > 0x7fffffffLL || (int64_t)TT * f.ldk * 4 > 0x7fffffffLL)
    return hipErrorInvalidValue;
  const unsigned nb = cdiv16(f.naux, TT);
  fused_f16_kernel<<<dim3(nb * nb * f.vsplit), NTH, 0, s>>>(f);
  return hipGetLastError();
}

}  // namespace thcsox
