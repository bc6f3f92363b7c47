// The fused B/C/D stage in the bf16x3 mode, 128 x 128 tiles of D per workgroup:
//
//   D_PR = sum_v C_RvP B_PRv,   B_PRv = sum_q G_Rq A_Pqv,   C_RvP = sum_w U_Rvw G_wP
//
// Every operand is split into three bf16 planes x = x0 + x1 + x2 (about the 24
// bits of an FP32 significand; bf16 keeps FP32's exponent range, so A needs no
// scale); a product is formed from the six plane products x0 y2 + x1 y1 + x2 y0
// + x0 y1 + x1 y0 + x0 y0 on the bf16 matrix cores (16x16x32, FP32
// accumulation).  The operands are K-major rows, one array per plane.
//
// Work split.  A workgroup owns a 128 x 128 tile of D and a range of v, one v at
// a time.  Four waves (one per SIMD) in a 2 x 2 arrangement each own 64 x 64 of
// the tile: the accumulators of B and C (128 registers) live in the matrix-core
// registers (AGPRs), the fragments of the three planes in the ordinary ones.  The
// partial sum of D (FP32, at most 8 v) lives in LDS, one private 16-byte slot per
// lane and MFMA tile, updated once per v: D += B o C.  (The fp16x2 kernel takes
// two v per pass in the same registers and LDS: two planes of two v there, three
// planes of one v here.)
//
// Pipeline.  A k chunk is two half stages, each two panels of 128 rows x 32 k x
// 3 planes (48 KiB): the B half (G, A_v) in LDS buffer sB and the C half (GX,
// U_v) in sC; with 64 KiB for D the workgroup uses the full 160 KiB of LDS.  A
// plane of a panel is 128 rows of 64 bytes, each row's four 16-byte chunks
// placed by lds_chunk.  Chunk t runs as
//   phase B(t): barrier (C(t) is in sC, every wave has read B(t) from sB);
//               loads of B(t+1) -> sB; fragments of C(t) <- sC;
//               matrix cores: B += products of B(t) (fragments read before)
//   phase C(t): barrier (B(t+1) is in sB, every wave has read C(t) from sC);
//               loads of C(t+1) -> sC; fragments of B(t+1) <- sB;
//               matrix cores: C += products of C(t)
// so each half stage is loaded one phase ahead of its fragment reads, and each
// fragment is read one phase ahead of its products.  The first chunk of a v
// starts the accumulators from zero inside the MFMA.  Past the last chunk the
// loads repeat it (never used).
#include "kernels.hpp"
#include "mfma.hpp"
#include "panel.hpp"

namespace thcsox {
namespace {

constexpr int TT = 128;          // tile edge of D (R and P)
constexpr int NW = 4, NTH = 64 * NW;
constexpr int KC = 32;           // k per chunk (one bf16 MFMA)
constexpr int NPL = 3;           // bf16 planes
constexpr int PP = TT * KC;      // elements of one plane of a panel
constexpr int FLUSH_V = 8;       // v per FP32 partial sum of D
constexpr int NXCD = 8;

// One half stage: panel 0 is the v-independent operand (G or GX), panel 1 the
// per-v one (A_v or U_v); [panel][plane][row * 32 + k].
struct Half3 {
  __bf16 s[2][NPL][PP];
};

__device__ __forceinline__ void bf3_vm_lds_barrier() {
  // this wave's memory loads (including those that write LDS) and LDS accesses
  // complete, then the workgroup barrier
  __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(1, 1)))
void fused_bf3_kernel(FusedArgs f) {
  __shared__ __attribute__((aligned(16))) Half3 sB;   // G, A_v
  __shared__ __attribute__((aligned(16))) Half3 sC;   // GX, U_v
  __shared__ __attribute__((aligned(16))) f4 sD[NW * 16 * 64];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int naux = f.naux, n = f.n, ldk = f.ldk;

  // tile and v range: XCD-aware order (workgroup b runs on XCD b mod 8; each XCD
  // owns the partial slots z = xcd, xcd + 8, ..., a block of consecutive v
  // ranges, and walks the tiles of one slot in bands of two R blocks, P by P
  // with R fastest, so its resident workgroups share panels in its L2).  With
  // symmetric D only the tiles on or above the diagonal are walked.  The integer
  // divisions run on the vector unit; readfirstlane marks their results uniform.
  const int nb = (naux + TT - 1) / TT;
  const bool symm = f.sym != nullptr && *f.sym != 0;
  const int ntl = symm ? nb * (nb + 1) / 2 : nb * nb;
  const int b = blockIdx.x;
  const int xcd = b % NXCD, local = b / NXCD;
  if (local >= ntl * (f.vsplit / NXCD)) return;
  const int z = __builtin_amdgcn_readfirstlane(xcd + NXCD * (local / ntl));
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

  // v range: XCD x owns the consecutive ranges x q .. x q + q - 1 (q = vsplit /
  // 8); range r is v in [r n / vsplit, (r + 1) n / vsplit)
  const int vr = (z % NXCD) * (f.vsplit / NXCD) + z / NXCD;
  const int v_lo = __builtin_amdgcn_readfirstlane((int)((int64_t)vr * n / f.vsplit));
  const int v_hi = __builtin_amdgcn_readfirstlane((int)((int64_t)(vr + 1) * n / f.vsplit));
  const int nv = v_hi - v_lo;
  const int kst = ldk / KC;
  const int rows_r = min(TT, naux - R0), rows_p = min(TT, naux - P0);

  // operand planes (rows past the valid range lie beyond the buffer resources
  // and read as zero)
  const __bf16* Gt = static_cast<const __bf16*>(f.Gt);
  const __bf16* GX = static_cast<const __bf16*>(f.GXt);
  const __bf16* Ub = static_cast<const __bf16*>(f.U);
  const __bf16* Ab = static_cast<const __bf16*>(f.A);
  __amdgpu_buffer_rsrc_t rG[NPL], rX[NPL];
#pragma unroll
  for (int p = 0; p < NPL; ++p) {
    rG[p] = make_rsrc(Gt + p * f.g_plane + (int64_t)R0 * ldk, (int64_t)rows_r * ldk * 2);
    rX[p] = make_rsrc(GX + p * f.g_plane + (int64_t)P0 * ldk, (int64_t)rows_p * ldk * 2);
  }
  const int64_t a_bytes = (int64_t)rows_p * ldk * 2;
  const int64_t u_bytes = ((int64_t)(rows_r - 1) * n * ldk + ldk) * 2;
  // per v: A rows (v, P) and U rows (R, v)
  __amdgpu_buffer_rsrc_t rA[NPL], rU[NPL];
  auto set_v = [&](int iv) {
    const int v = v_lo + iv;
#pragma unroll
    for (int p = 0; p < NPL; ++p) {
      rA[p] = make_rsrc(Ab + p * f.a_plane + ((int64_t)v * naux + P0) * ldk, a_bytes);
      rU[p] = make_rsrc(Ub + p * f.u_plane + ((int64_t)R0 * n + v) * ldk, u_bytes);
    }
  };

  // memory -> LDS: one instruction moves 16 rows x 64 bytes of one plane; wave w
  // moves the 16-row slabs w and w + 4 of each plane of each panel.  Lane l
  // lands at slab row l / 4, physical chunk l % 4, and loads the logical chunk
  // lds_chunk maps there (the map is its own inverse for a given row).
  uint32_t dR[2], dU[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int row = (wave + NW * j) * 16 + (lane >> 2);
    const int c = lds_chunk(row, lane & 3);
    dR[j] = (uint32_t)((row * ldk + 8 * c) * 2);
    dU[j] = (uint32_t)((row * (n * ldk) + 8 * c) * 2);
  }
  auto dmaB = [&](int k0) {
    const int so = k0 * 2;   // bytes to the k chunk
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int slab = (wave + NW * j) * 16 * 32;
#pragma unroll
      for (int p = 0; p < NPL; ++p) {
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rG[p], &sB.s[0][p][slab], 16, dR[j], so, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rA[p], &sB.s[1][p][slab], 16, dR[j], so, 0, 0);
      }
    }
  };
  auto dmaC = [&](int k0) {
    const int so = k0 * 2;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int slab = (wave + NW * j) * 16 * 32;
#pragma unroll
      for (int p = 0; p < NPL; ++p) {
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rX[p], &sC.s[0][p][slab], 16, dR[j], so, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rU[p], &sC.s[1][p][slab], 16, dU[j], so, 0, 0);
      }
    }
  };

  // fragment (row r, k chunk lane / 16) of a plane at r * 32 + lds_chunk(r, lane / 16) * 8.
  // For r = 64 h + 16 t + lane % 16 the map depends on t only through t mod 2
  // (it flips bit 1 of the chunk), so even and odd tiles take two offsets.
  const int lr = lane & 15, kc = lane >> 4;
  auto frag_off = [&](int base, int tpar) {
    const int r = base + 16 * tpar + lr;
    return (r - 16 * tpar) * 32 + lds_chunk(r, kc) * 8;
  };
  const int fR[2] = {frag_off(wr * 64, 0), frag_off(wr * 64, 1)};   // R side rows
  const int fP[2] = {frag_off(wc * 64, 0), frag_off(wc * 64, 1)};   // P side rows
  // fragments of one half stage: the shared operand s (G or GX) and the per-v
  // operand m (A_v or U_v), [plane][tile]
  struct Frags { bf16x8 s[NPL][4], m[NPL][4]; };
  Frags fb, fc;
  auto rd = [&](const __bf16* base, const int* off, int t) {
    return *reinterpret_cast<const bf16x8*>(base + off[t & 1] + t * 16 * 32);
  };
  auto readB = [&](Frags& fr) {   // G (R side), A_v (P side)
#pragma unroll
    for (int p = 0; p < NPL; ++p)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        fr.s[p][t] = rd(sB.s[0][p], fR, t);
        fr.m[p][t] = rd(sB.s[1][p], fP, t);
      }
  };
  auto readC = [&](Frags& fr) {   // GX (P side), U_v (R side)
#pragma unroll
    for (int p = 0; p < NPL; ++p)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        fr.s[p][t] = rd(sC.s[0][p], fP, t);
        fr.m[p][t] = rd(sC.s[1][p], fR, t);
      }
  };

  // accumulators [ti][tj]: rows R of tile ti, columns P of tile tj (cleared once
  // here; each v then starts them from zero inside its first MFMAs)
  f4 B[4][4], C[4][4];
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) B[ti][tj] = C[ti][tj] = zero;
  using PR = Products<NPL>;   // plane pairs, smallest terms first
  // B products: B[ti][tj] += G[ti] . A_v[tj]
  auto mfmaB = [&](const Frags& fr, bool first) {
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
        f4 a = first ? zero : B[ti][tj];
#pragma unroll
        for (int q = 0; q < PR::N; ++q)
          a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.s[PR::a(q)][ti], fr.m[PR::b(q)][tj], a,
                                                      0, 0, 0);
        B[ti][tj] = a;
      }
  };
  // C products: C[ti][tj] += U_v[ti] . GX[tj]
  auto mfmaC = [&](const Frags& fr, bool first) {
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
        f4 a = first ? zero : C[ti][tj];
#pragma unroll
        for (int q = 0; q < PR::N; ++q)
          a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.m[PR::a(q)][ti], fr.s[PR::b(q)][tj], a,
                                                      0, 0, 0);
        C[ti][tj] = a;
      }
  };

  // the partial sum of D: slot (wave, tile) of each lane, 64 lanes x 16 bytes
  f4* const Dw = sD + wave * 16 * 64 + lane;
  auto dzero = [&]() {
#pragma unroll
    for (int tt = 0; tt < 16; ++tt) Dw[tt * 64] = zero;
  };
  auto dupdate = [&]() {
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
        f4 d = Dw[(ti * 4 + tj) * 64];
#pragma unroll
        for (int r = 0; r < 4; ++r) d[r] = fmaf(B[ti][tj][r], C[ti][tj][r], d[r]);
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
  // fetch cursor over (v, chunk), clamped to the last chunk
  int cv = 0, ck = 0;
  auto advance = [&]() {
    const bool last = (cv == nv - 1) && (ck == kst - 1);
    const bool wrap = (ck == kst - 1);
    ck = last ? ck : (wrap ? 0 : ck + 1);
    if (wrap && !last) set_v(++cv);
  };
  if (nv > 0) {
    set_v(0);
    dmaB(0);
    dmaC(0);
    advance();
    bf3_vm_lds_barrier();
    readB(fb);
  }
  // spread a phase's 12 memory-to-LDS loads over its 96 MFMAs (one per 8)
  auto spread = [&]() {
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);   // one memory instruction
      __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);   // eight MFMAs
    }
  };
  auto chunk = [&](bool first) {
    bf3_vm_lds_barrier();
    dmaB(ck * KC);
    readC(fc);
    mfmaB(fb, first);
    spread();
    bf3_vm_lds_barrier();
    dmaC(ck * KC);
    advance();
    readB(fb);
    mfmaC(fc, first);
    spread();
  };
  int done = 0;
  for (int iv = 0; iv < nv; ++iv) {
    chunk(true);
    for (int k = 1; k < kst; ++k) chunk(false);
    dupdate();
    ++done;
    if (done % FLUSH_V == 0 && iv + 1 < nv) {
      flush(done == FLUSH_V);
      dzero();
    }
  }
  // the last (repeated) memory-to-LDS loads land before the workgroup may end
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
  flush(done <= FLUSH_V);   // also writes zeros for an empty range
}

inline unsigned cdiv_bf3(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

hipError_t sox_fused_bf3(const FusedArgs& f, hipStream_t s) {
  const int vmax = (f.n + f.vsplit - 1) / f.vsplit;   // longest v range
  if (f.vsplit % NXCD != 0 || f.ldk % KC != 0 || f.ldk < f.n ||
      (f.dpart_f32 && vmax > FLUSH_V))
    return hipErrorInvalidValue;
  // buffer offsets inside one tile's rows of U (rows of 2 ldk bytes) are 32-bit
  if ((int64_t)TT * f.n * f.ldk * 2 > 0x7fffffffLL) return hipErrorInvalidValue;
  const unsigned nb = cdiv_bf3(f.naux, TT);
  fused_bf3_kernel<<<dim3(nb * nb * f.vsplit), NTH, 0, s>>>(f);
  return hipGetLastError();
}

}  // namespace thcsox
