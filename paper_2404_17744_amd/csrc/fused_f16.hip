// The fused B/C/D stage in the fp16x2 and FP32 modes, 128 x 128 tiles of D per
// workgroup:
//
//   D_PR = sum_v C_RvP B_PRv,   B_PRv = sum_q G_Rq A_Pqv,   C_RvP = sum_w U_Rvw G_wP
//
// fp16x2: every operand is a power-of-two scaled value split into two fp16
// planes x = x0 + x1; a product is formed from the plane products x1 y0 + x0 y1
// + x0 y0 on the f16 matrix cores (16x16x32, FP32 accumulation).  The operands
// are K-major rows with the two planes interleaved per 32-wide k chunk (layout
// c32: row r, plane p, k at r * 2 ldk + (k / 32) * 64 + 32 p + k % 32), so one
// 128-byte request fetches both planes of a row's chunk.  FP32: plain K-major
// FP32 rows, whose 32-wide k chunks are 128 bytes too, so both modes share the
// loads, the LDS layout and the schedule below; a chunk is eight 16x16x4 FP32
// MFMAs per tile instead of three 16x16x32 f16 ones.
//
// Work split.  A workgroup owns a 128 x 128 tile of D and a range of v, taken
// two v at a time: the k loop of a pair forms B and C for both v at once, so
// the v-independent panels (G rows R, GX rows P) are loaded once per pair and
// feed four products.  Four waves (one per SIMD) in a 2 x 2 arrangement each
// own 64 x 64 of the tile: the four accumulator sets B1, B2, C1, C2 (256
// registers) live in the matrix-core registers (AGPRs), fragments in the
// ordinary ones.  The partial sum of D (FP32, at most 8 v) lives in LDS, one
// private 16-byte slot per lane and MFMA tile, and is updated once per pair:
// D += B1 o C1 + B2 o C2.
//
// Pipeline.  A k chunk is two half stages, each three panels of 128 rows x 32 k
// x 2 planes (FP32: one plane of 4-byte elements; 48 KiB either way): the B half (G, A_v1, A_v2) in LDS buffer sB and the C
// half (GX, U_v1, U_v2) in sC.  With 64 KiB for D the workgroup uses the full
// 160 KiB of LDS.  Chunk t runs as
//   phase B(t): barrier (C(t) is in sC, every wave has read B(t) from sB);
//               loads of B(t+1) -> sB; fragments of C(t) <- sC;
//               matrix cores: B1, B2 += products of B(t) (fragments read before)
//   phase C(t): barrier (B(t+1) is in sB, every wave has read C(t) from sC);
//               loads of C(t+1) -> sC; fragments of B(t+1) <- sB;
//               matrix cores: C1, C2 += products of C(t)
// so each half stage is loaded one phase ahead of its fragment reads, and each
// fragment is read one phase ahead of its products.  The first chunk of a pair
// starts the accumulators from zero inside the MFMA (no register clearing).
// Past the last chunk the loads repeat it (never used).
#include "kernels.hpp"
#include "mfma.hpp"
#include "panel.hpp"

namespace thcsox {
namespace {

constexpr int TT = 128;          // tile edge of D (R and P)
constexpr int NW = 4, NTH = 64 * NW;
constexpr int KC = 32;           // k per chunk (one f16 MFMA)
constexpr int PANEL = TT * KC * 2;   // halves per panel (both planes)
constexpr int FLUSH_PAIRS = 4;   // pairs per FP32 partial sum of D (8 v)
constexpr int NXCD16 = 8;

// One half stage: three panels, each [row][plane][32] (128-byte rows) with the
// eight 16-byte chunks of a row permuted by sw8.
struct Half {
  _Float16 s[3][PANEL];
};

// Physical 16-byte chunk of logical chunk c (= 4 plane + k / 8) in LDS row r.
// Fragment reads take 16 consecutive rows at one logical chunk; XOR-ing the
// chunk with (r / 2) mod 8 places the 16 rows' chunks at all eight positions of
// two consecutive 128-byte rows (rocprofv3 counts no LDS bank conflicts).
__device__ __forceinline__ int sw8(int r, int c) { return c ^ ((r >> 1) & 7); }

__device__ __forceinline__ void vm_lds_barrier() {
  // this wave's memory loads (including those that write LDS) and LDS accesses
  // complete, then the workgroup barrier
  __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// M = MODE_F16X2 or MODE_F32.  sB: G, A_v1, A_v2; sC: GX, U_v1, U_v2; sD: the
// partial sum of D.
template <int M>
__device__ __forceinline__ void fused_pair_body(const FusedArgs& f, Half& sB, Half& sC, f4* sD) {
  constexpr bool F32 = M == MODE_F32;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int naux = f.naux, n = f.n, ldk = f.ldk;

  // tile and pair range: XCD-aware order (workgroup b runs on XCD b mod 8; each
  // XCD owns the partial slots z = xcd, xcd + 8, ..., a block of consecutive
  // pair ranges, and walks the tiles of one slot in bands of two R blocks, P by
  // P with R fastest, so its resident workgroups share panels in its L2).  With
  // symmetric D only the tiles on or above the diagonal are walked (nb (nb + 1)
  // / 2 of them; the grid has nb^2 per slot, the rest exit at once).  The
  // integer divisions run on the vector unit; readfirstlane marks their results
  // uniform so that buffer resources and offsets stay scalar.
  const int nb = (naux + TT - 1) / TT;
  const bool symm = f.sym != nullptr && *f.sym != 0;
  const int ntl = symm ? nb * (nb + 1) / 2 : nb * nb;
  const int b = blockIdx.x;
  const int xcd = b % NXCD16, local = b / NXCD16;
  if (local >= ntl * (f.vsplit / NXCD16)) return;
  const int z = __builtin_amdgcn_readfirstlane(xcd + NXCD16 * (local / ntl));
  int t = local % ntl, r0 = 0;
  for (;;) {   // the band of rows r0, r0 + 1 (one row at the end when nb is odd)
    const int rows = min(2, nb - r0);
    const int cnt = symm ? (rows == 2 ? 2 * (nb - r0) - 1 : nb - r0) : rows * nb;
    if (t < cnt) break;
    t -= cnt;
    r0 += 2;
  }
  int rb, pb;
  if (symm) {   // (r0, r0), then (r0, p), (r0 + 1, p) for p > r0
    rb = t == 0 ? r0 : r0 + (t - 1) % 2;
    pb = t == 0 ? r0 : r0 + 1 + (t - 1) / 2;
  } else {
    const int rows = min(2, nb - r0);
    rb = r0 + t % rows;
    pb = t / rows;
  }
  const int P0 = __builtin_amdgcn_readfirstlane(pb * TT);
  const int R0 = __builtin_amdgcn_readfirstlane(rb * TT);

  // pair range: XCD x owns the consecutive ranges x q .. x q + q - 1
  // (q = vsplit / 8); range r is pairs [r np / vsplit, (r + 1) np / vsplit)
  const int npair = (n + 1) / 2;
  const int vr = (z % NXCD16) * (f.vsplit / NXCD16) + z / NXCD16;
  const int p_lo = __builtin_amdgcn_readfirstlane((int)((int64_t)vr * npair / f.vsplit));
  const int p_hi = __builtin_amdgcn_readfirstlane((int)((int64_t)(vr + 1) * npair / f.vsplit));
  const int npr = p_hi - p_lo;
  const int kst = ldk / KC;
  const int ld2 = 2 * ldk;   // halves per c32 row
  const int rows_r = min(TT, naux - R0), rows_p = min(TT, naux - P0);

  const _Float16* Gt = static_cast<const _Float16*>(f.Gt);
  const _Float16* GX = static_cast<const _Float16*>(f.GXt);
  const __amdgpu_buffer_rsrc_t rG = make_rsrc(Gt + (int64_t)R0 * ld2, (int64_t)rows_r * ld2 * 2);
  const __amdgpu_buffer_rsrc_t rX = make_rsrc(GX + (int64_t)P0 * ld2, (int64_t)rows_p * ld2 * 2);
  const _Float16* Ubase = static_cast<const _Float16*>(f.U) + (int64_t)R0 * n * ld2;
  const _Float16* Abase = static_cast<const _Float16*>(f.A) + (int64_t)P0 * ld2;
  const int64_t a_v = (int64_t)naux * ld2;   // halves between v slabs of A

  // memory -> LDS: one instruction moves 8 rows x 128 bytes; wave w moves the
  // 8-row slabs w, w + 4, w + 8, w + 12 of each panel.  Lane l lands at slab row
  // l / 8, physical chunk l % 8, and loads the logical chunk sw8 maps there.
  // Rows past the valid range lie beyond the buffer resource and read as zero.
  uint32_t dR[4], dU[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = (wave + NW * j) * 8 + (lane >> 3);
    const int c = sw8(row, lane & 7);
    dR[j] = (uint32_t)((row * ld2 + 8 * c) * 2);
    dU[j] = (uint32_t)((row * (n * ld2) + 8 * c) * 2);
  }
  // per pair: A slabs v1, v2 (rows P) and U rows (R, v1), (R, v2); a missing
  // second v (odd n) gets empty resources, so its panels read as zero and B2 = 0
  __amdgpu_buffer_rsrc_t rA1, rA2, rU1, rU2;
  const int64_t a_bytes = (int64_t)rows_p * ld2 * 2;
  const int64_t u_bytes = ((int64_t)(rows_r - 1) * n * ld2 + ld2) * 2;
  auto set_pair = [&](int pr) {
    const int v1 = 2 * (p_lo + pr);
    const bool two = v1 + 1 < n;
    rA1 = make_rsrc(Abase + (int64_t)v1 * a_v, a_bytes);
    rA2 = make_rsrc(Abase + (int64_t)(v1 + 1) * a_v, two ? a_bytes : 0);
    rU1 = make_rsrc(Ubase + (int64_t)v1 * ld2, u_bytes);
    rU2 = make_rsrc(Ubase + (int64_t)(v1 + 1) * ld2, two ? u_bytes : 0);
  };
  auto dmaB = [&](int k0) {
    const int so = k0 * 4;   // bytes to the k chunk (both planes)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int slab = (wave + NW * j) * 8 * 64;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rG, &sB.s[0][slab], 16, dR[j], so, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rA1, &sB.s[1][slab], 16, dR[j], so, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rA2, &sB.s[2][slab], 16, dR[j], so, 0, 0);
    }
  };
  auto dmaC = [&](int k0) {
    const int so = k0 * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int slab = (wave + NW * j) * 8 * 64;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rX, &sC.s[0][slab], 16, dR[j], so, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rU1, &sC.s[1][slab], 16, dU[j], so, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rU2, &sC.s[2][slab], 16, dU[j], so, 0, 0);
    }
  };

  // fp16x2: fragment (row r, plane p, k chunk lane / 16) at halves r * 64 + sw8(r, 4 p +
  // lane / 16) * 8.  FP32: the 16x16x4 MFMA takes one k per lane group, and any
  // assignment of the chunk's 32 k to its eight MFMAs j and four lane groups serves
  // when both operands use it: lane group g takes k = 8 g + j, two 16-byte reads
  // at logical chunks 2 g and 2 g + 1 (in "planes" 0 and 1 below).  sw8 depends on
  // r mod 16 only, so the rows of tile t are 16 t * 64 halves further.
  const int lr = lane & 15, kc = lane >> 4;
  const int rr = wr * 64 + lr, rc = wc * 64 + lr;
  const int c0 = F32 ? 2 * kc : kc, c1 = F32 ? 2 * kc + 1 : 4 + kc;
  const int fr0 = rr * 64 + sw8(rr, c0) * 8, fr1 = rr * 64 + sw8(rr, c1) * 8;
  const int fc0 = rc * 64 + sw8(rc, c0) * 8, fc1 = rc * 64 + sw8(rc, c1) * 8;
  // fragments of one half stage: the shared operand s (G or GX) and the per-v
  // operands m1, m2 (A_v or U_v), [plane][tile]
  struct Frags { f16x8 s[2][4], m1[2][4], m2[2][4]; };
  Frags fb, fc;
  auto rd = [&](const _Float16* base, int off, int t) {
    return *reinterpret_cast<const f16x8*>(base + off + t * 16 * 64);
  };
  auto readB = [&](Frags& fr) {   // G (R side), A_v1, A_v2 (P side)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      fr.s[0][t] = rd(sB.s[0], fr0, t);  fr.s[1][t] = rd(sB.s[0], fr1, t);
      fr.m1[0][t] = rd(sB.s[1], fc0, t); fr.m1[1][t] = rd(sB.s[1], fc1, t);
      fr.m2[0][t] = rd(sB.s[2], fc0, t); fr.m2[1][t] = rd(sB.s[2], fc1, t);
    }
  };
  auto readC = [&](Frags& fr) {   // GX (P side), U_v1, U_v2 (R side)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      fr.s[0][t] = rd(sC.s[0], fc0, t);  fr.s[1][t] = rd(sC.s[0], fc1, t);
      fr.m1[0][t] = rd(sC.s[1], fr0, t); fr.m1[1][t] = rd(sC.s[1], fr1, t);
      fr.m2[0][t] = rd(sC.s[2], fr0, t); fr.m2[1][t] = rd(sC.s[2], fr1, t);
    }
  };

  // accumulators [ti][tj]: rows R of tile ti, columns P of tile tj (cleared once
  // here; each pair then starts them from zero inside its first MFMAs)
  f4 B1[4][4], B2[4][4], C1[4][4], C2[4][4];
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) B1[ti][tj] = B2[ti][tj] = C1[ti][tj] = C2[ti][tj] = zero;
  // FP32: operand j (k = 8 g + j) of a fragment pair
  auto el = [](const f16x8& lo, const f16x8& hi, int j) {
    return j < 4 ? __builtin_bit_cast(f4, lo)[j] : __builtin_bit_cast(f4, hi)[j - 4];
  };
  // B products: acc[ti][tj] += G[ti] . A_m[tj] (fp16x2: planes x1 y0 + x0 y1 + x0 y0;
  // FP32: eight 16x16x4 products, the two v interleaved)
  auto mfmaB = [&](const Frags& fr, bool first) {
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
        if constexpr (F32) {
          f4 a1 = first ? zero : B1[ti][tj];
          f4 a2 = first ? zero : B2[ti][tj];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const float g = el(fr.s[0][ti], fr.s[1][ti], j);
            a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(g, el(fr.m1[0][tj], fr.m1[1][tj], j), a1, 0, 0, 0);
            a2 = __builtin_amdgcn_mfma_f32_16x16x4f32(g, el(fr.m2[0][tj], fr.m2[1][tj], j), a2, 0, 0, 0);
          }
          B1[ti][tj] = a1;
          B2[ti][tj] = a2;
        } else {
          f4 a1 = first ? zero : B1[ti][tj];
          a1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.s[1][ti], fr.m1[0][tj], a1, 0, 0, 0);
          a1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.s[0][ti], fr.m1[1][tj], a1, 0, 0, 0);
          B1[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.s[0][ti], fr.m1[0][tj], a1, 0, 0, 0);
          f4 a2 = first ? zero : B2[ti][tj];
          a2 = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.s[1][ti], fr.m2[0][tj], a2, 0, 0, 0);
          a2 = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.s[0][ti], fr.m2[1][tj], a2, 0, 0, 0);
          B2[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.s[0][ti], fr.m2[0][tj], a2, 0, 0, 0);
        }
      }
  };
  // C products: acc[ti][tj] += U_m[ti] . GX[tj]
  auto mfmaC = [&](const Frags& fr, bool first) {
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
        if constexpr (F32) {
          f4 a1 = first ? zero : C1[ti][tj];
          f4 a2 = first ? zero : C2[ti][tj];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const float x = el(fr.s[0][tj], fr.s[1][tj], j);
            a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(el(fr.m1[0][ti], fr.m1[1][ti], j), x, a1, 0, 0, 0);
            a2 = __builtin_amdgcn_mfma_f32_16x16x4f32(el(fr.m2[0][ti], fr.m2[1][ti], j), x, a2, 0, 0, 0);
          }
          C1[ti][tj] = a1;
          C2[ti][tj] = a2;
        } else {
          f4 a1 = first ? zero : C1[ti][tj];
          a1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.m1[1][ti], fr.s[0][tj], a1, 0, 0, 0);
          a1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.m1[0][ti], fr.s[1][tj], a1, 0, 0, 0);
          C1[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.m1[0][ti], fr.s[0][tj], a1, 0, 0, 0);
          f4 a2 = first ? zero : C2[ti][tj];
          a2 = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.m2[1][ti], fr.s[0][tj], a2, 0, 0, 0);
          a2 = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.m2[0][ti], fr.s[1][tj], a2, 0, 0, 0);
          C2[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.m2[0][ti], fr.s[0][tj], a2, 0, 0, 0);
        }
      }
  };

  // the partial sum of D: slot (wave, tile) of each lane, 64 lanes x 16 bytes
  f4* const Dw = sD + wave * 16 * 64 + lane;
  auto dzero = [&]() {
#pragma unroll
    for (int t = 0; t < 16; ++t) Dw[t * 64] = zero;
  };
  auto dupdate = [&]() {
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
        f4 d = Dw[(ti * 4 + tj) * 64];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          d[r] = fmaf(B1[ti][tj][r], C1[ti][tj][r], d[r]);
          d[r] = fmaf(B2[ti][tj][r], C2[ti][tj][r], d[r]);
        }
        Dw[(ti * 4 + tj) * 64] = d;
      }
  };
  // D tile -> partial tile z (FP32 store, or FP64 add unless first): thread t
  // takes column P0 + t % 128 and rows R0 + t / 128 + 2 i, reading each element
  // from the LDS slot of the lane that formed it (lane 16 (R % 16 / 4) + P % 16
  // of wave 2 (R / 64) + P / 64, tile (R % 64 / 16, P % 64 / 16), element R % 4),
  // so the global writes are coalesced rows.  Barriers before (other waves'
  // slots) and after (the slots may be cleared next).
  auto flush = [&](bool first) {
    __syncthreads();
    const float* sDf = reinterpret_cast<const float*>(sD);
    const int Pt = tid & (TT - 1), P = P0 + Pt;
    const int pslot = (Pt >> 6) * 16 * 64 + ((Pt >> 4) & 3) * 64 + (Pt & 15);
    const int64_t zo = (int64_t)z * naux * naux + P;
    for (int Rt = tid >> 7; Rt < TT; Rt += NTH / TT) {
      const int R = R0 + Rt;
      if (R < naux && P < naux) {
        const int slot = pslot + (Rt >> 6) * 2 * 16 * 64 + ((Rt >> 4) & 3) * 4 * 64 + ((Rt >> 2) & 3) * 16;
        const float v = sDf[slot * 4 + (Rt & 3)];
        const int64_t o = zo + (int64_t)R * naux;
        if (f.dpart_f32) {   // one range = one FP32 partial sum (first is true)
          reinterpret_cast<float*>(f.Dpart)[o] = v;
        } else {
          f.Dpart[o] = (first ? 0.0 : f.Dpart[o]) + (double)v;
        }
      }
    }
    __syncthreads();
  };

  dzero();
  // fetch cursor over (pair, chunk), clamped to the last chunk
  int cp = 0, ck = 0;
  auto advance = [&]() {
    const bool last = (cp == npr - 1) && (ck == kst - 1);
    const bool wrap = (ck == kst - 1);
    ck = last ? ck : (wrap ? 0 : ck + 1);
    if (wrap && !last) set_pair(++cp);
  };
  if (npr > 0) {
    set_pair(0);
    dmaB(0);
    dmaC(0);
    advance();
    vm_lds_barrier();
    readB(fb);
  }
  // interleave a phase's 12 memory-to-LDS loads with its first MFMAs, one load
  // per MPL of them: a load the texture unit cannot take yet stalls its wave,
  // and with one wave per SIMD nothing else would keep the matrix core busy
  // meanwhile, while loads issued late have less time to land (measured at n =
  // 300: fp16x2, 96 MFMAs per phase, fastest at 3 of 1, 2, 3, 4, 8; FP32, 256
  // MFMAs per phase, at 16 of 10, 12, 16, 21)
  constexpr int MPL = F32 ? 16 : 3;
  auto spread = [&]() {
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);     // one memory instruction
      __builtin_amdgcn_sched_group_barrier(0x008, MPL, 0);   // MPL MFMAs
    }
  };
  auto chunk = [&](bool first) {
    vm_lds_barrier();
    dmaB(ck * KC);
    readC(fc);
    mfmaB(fb, first);
    spread();
    vm_lds_barrier();
    dmaC(ck * KC);
    advance();
    readB(fb);
    mfmaC(fc, first);
    spread();
  };
  int done = 0;
  for (int pr = 0; pr < npr; ++pr) {
    chunk(true);
    for (int k = 1; k < kst; ++k) chunk(false);
    dupdate();
    ++done;
    if (done % FLUSH_PAIRS == 0 && pr + 1 < npr) {
      flush(done == FLUSH_PAIRS);
      dzero();
    }
  }
  // the last (repeated) memory-to-LDS loads land before the workgroup may end
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
  flush(done <= FLUSH_PAIRS);   // also writes zeros for an empty range
}

__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(1, 1)))
void fused_f16_kernel(FusedArgs f) {
  __shared__ __attribute__((aligned(16))) Half sB;
  __shared__ __attribute__((aligned(16))) Half sC;
  __shared__ __attribute__((aligned(16))) f4 sD[NW * 16 * 64];
  fused_pair_body<MODE_F16X2>(f, sB, sC, sD);
}

__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(1, 1)))
void fused_f32_kernel(FusedArgs f) {
  __shared__ __attribute__((aligned(16))) Half sB;
  __shared__ __attribute__((aligned(16))) Half sC;
  __shared__ __attribute__((aligned(16))) f4 sD[NW * 16 * 64];
  fused_pair_body<MODE_F32>(f, sB, sC, sD);
}

inline unsigned cdiv16(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

void fused_f16_tile(int* rows, int* cols) {
  *rows = TT;
  *cols = TT;
}

hipError_t sox_fused_pairs(int mode, const FusedArgs& f, hipStream_t s) {
  if (mode != MODE_F16X2 && mode != MODE_F32) return hipErrorInvalidValue;
  const int npair = (f.n + 1) / 2;
  const int pairs_max = (npair + f.vsplit - 1) / f.vsplit;   // longest pair range
  if (f.vsplit % NXCD16 != 0 || f.ldk % KC != 0 || f.ldk < f.n ||
      (f.dpart_f32 && pairs_max > FLUSH_PAIRS))
    return hipErrorInvalidValue;
  // buffer offsets inside one tile's rows of U (rows of 4 ldk bytes) are 32-bit
  if ((int64_t)TT * f.n * f.ldk * 4 > 0x7fffffffLL) return hipErrorInvalidValue;
  const unsigned nb = cdiv16(f.naux, TT);
  if (mode == MODE_F16X2) fused_f16_kernel<<<dim3(nb * nb * f.vsplit), NTH, 0, s>>>(f);
  else fused_f32_kernel<<<dim3(nb * nb * f.vsplit), NTH, 0, s>>>(f);
  return hipGetLastError();
}

}  // namespace thcsox
