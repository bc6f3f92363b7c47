// The A stage in the fp16x2 mode:
//
//   A_Pqv = sum_s U_Pqs G_sv(beta - tau)
//
// for one or more tau points ("sets") per launch, as C(i, j) = sum_k Uop[i][k]
// Gop[j][k] with Uop the rows (P, q) of U and Gop the rows v of G(beta - tau)^T,
// both K-major fp16 operands in the c32 layout (the two planes x = x0 + x1
// interleaved per 32-wide k chunk: row r, plane p, k at r * 2 ldk + (k / 32) *
// 64 + 32 p + k % 32); products x1 y0 + x0 y1 + x0 y0 on the f16 matrix cores,
// FP32 accumulation.  The result is scaled by the power of two taken from
// amax[set] (a bound on |A| placed near 2^14, computed before the launch) and
// written as fp16 planes in the same c32 layout, rows (v, P) with k = q, which
// is what the fused stage loads.
//
// Rows are walked in the padded row space of A, i = P ldk + q: a 128-row tile is
// four whole 32-wide chunks of one v row set, so no output line is shared by two
// workgroups (rows n <= q < ldk read U as zero and write zeros).
// A workgroup of eight waves (two per SIMD) works on 128 rows at a time and TN =
// 64 WBN columns (v), WBN <= 5; wave (wm, wn) holds 64 x 16 WBN of it.  The grid
// is persistent (about one workgroup per compute unit): a workgroup walks its
// row tiles with one continuous stream of stages, so the loads of the next tile
// overlap the last stages and the stores of the current one.  The workgroups
// that walk the same row tiles for different sets (or column blocks) are placed
// on one XCD, so U is fetched from HBM about once per launch and served from
// that XCD's L2 to the others.  Each 32-wide k stage of both operands (U: 16 KiB,
// G: TN x 128 B) is loaded from memory straight into one of two LDS buffers, one
// stage ahead of the matrix cores; the fragments of the next stage are read while
// the second half of the current stage's MFMAs run.  The MFMA takes the U
// fragment as its row operand, so a lane's four outputs are four consecutive
// rows i of one v: one 8-byte store per plane.
#include <algorithm>

#include "kernels.hpp"
#include "mfma.hpp"
#include "panel.hpp"

namespace thcsox {
namespace {

constexpr int AM = 128;             // rows of U per workgroup
constexpr int AKC = 32;             // k per stage
constexpr int ANW = 8, ANT = 64 * ANW;

constexpr int AMAXN = 320;          // columns per workgroup at most (WBN <= 5)
// staging row of one v in the epilogue: 64 rows i x 2 planes (c32 order) plus
// 8 halves of padding (rows 272 bytes apart: 16 rows start on distinct banks)
constexpr int STG_LD = 136;
// One stage: U rows and G rows, each [row][plane][32] (128 bytes: both planes of
// the row's k chunk) with the eight 16-byte chunks of a row permuted by sw8a.
struct ABuf {
  _Float16 u[AM * 2 * AKC];
  _Float16 g[AMAXN * 2 * AKC];
};
// Physical 16-byte chunk of logical chunk c (= 4 plane + k / 8) in LDS row r;
// 16 consecutive rows read at one logical chunk land on all eight positions of
// two rows (depends on r mod 16 only).
__device__ __forceinline__ int sw8a(int r, int c) { return c ^ ((r >> 1) & 7); }

template <int WBN> struct AFrags {
  f16x8 u[2][4], g[2][WBN];   // [plane][tile]
};

__device__ __forceinline__ void a_vm_lds_barrier() {
  __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int WBN>
__device__ __forceinline__ void astage_body(const AStageArgs& g, ABuf& b0, ABuf& b1,
                                            _Float16* sstage) {
  constexpr int TN = 64 * WBN;
  static_assert(TN <= AMAXN, "at most 320 columns per workgroup");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform in the wave
  const int wm = wave >> 2, wn = wave & 3;
  const int M = g.naux * g.ldk;                 // padded rows (checked < 2^31 on the host)
  const int nib = (M + AM - 1) / AM;
  // block -> (part x, row worker y), parts = (set, column block): the X parts of
  // worker y are the blocks 8 (X (y / 8) + x) + y % 8, which share an XCD (blocks
  // are dealt to the eight XCDs round-robin)
  // (the integer divisions run on the vector unit: readfirstlane tells the
  // compiler that the results are uniform, so the buffer resources stay scalar)
  const int ncol = (g.n + TN - 1) / TN, X = g.nsets * ncol;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int x = __builtin_amdgcn_readfirstlane(slot % X);
  const int first = __builtin_amdgcn_readfirstlane((slot / X) * 8 + xcd);
  const int stride = __builtin_amdgcn_readfirstlane(gridDim.x / X);
  const int set = __builtin_amdgcn_readfirstlane(x / ncol);
  const int j0 = __builtin_amdgcn_readfirstlane((x % ncol) * TN);
  const int ntile = __builtin_amdgcn_readfirstlane(first < nib ? (nib - 1 - first) / stride + 1 : 0);
  if (ntile == 0) return;
  const int rows_j = min(TN, g.n - j0);
  const int kst = g.ldk / AKC;
  const int64_t ldk = g.ldk;

  const int64_t ld2 = 2 * ldk;   // halves per c32 row
  const _Float16* B = static_cast<const _Float16*>(g.Gb) + set * g.gb_set + j0 * ld2;
  const __amdgpu_buffer_rsrc_t rB = make_rsrc(B, rows_j * ld2 * 2);
  // memory to LDS: one instruction moves 8 rows x 128 bytes (both planes of a k
  // chunk); lane l lands at row l / 8 of the slab, physical chunk l % 8, and
  // loads the logical chunk sw8a maps there.  U: 16 slabs, wave w moves slabs
  // 2 w and 2 w + 1; G: TN / 8 slabs, wave w moves slabs w + 8 j, j < WBN.
  const int lrow = lane >> 3;
  uint32_t dg[WBN];
#pragma unroll
  for (int j = 0; j < WBN; ++j) {
    const int row = (wave + ANW * j) * 8 + lrow;
    dg[j] = row < rows_j ? (uint32_t)((row * ld2 + 8 * sw8a(row, lane & 7)) * 2) : OOB;
  }
  // the U rows of the tile being fetched: this lane's rows i = i0 + urow[h] are U
  // rows P n + q (none for q >= n), addressed from the tile's first P
  const _Float16* Ub = static_cast<const _Float16*>(g.U);
  const int64_t urows = (int64_t)g.naux * g.n;
  __amdgpu_buffer_rsrc_t rU;
  uint32_t du[2] = {OOB, OOB};
  auto set_tile = [&](int t) {
    const int i0 = (first + t * stride) * AM;
    const int P0 = __builtin_amdgcn_readfirstlane(i0 / g.ldk);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int urow = (2 * wave + h) * 8 + lrow;
      const int i = i0 + urow, P = i / g.ldk, q = i - P * g.ldk;
      du[h] = (P < g.naux && q < g.n)
                  ? (uint32_t)((((P - P0) * g.n + q) * ld2 + 8 * sw8a(urow, lane & 7)) * 2)
                  : OOB;
    }
    const int64_t r0 = (int64_t)P0 * g.n;
    rU = make_rsrc(Ub + r0 * ld2, (urows - r0) * ld2 * 2);
  };
  // stage k of the current fetch tile -> LDS buffer (chunk k is 64 k halves into a c32 row)
  auto dma = [&](ABuf& bf, int k) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rU, &bf.u[(2 * wave + h) * 8 * 64], 16, du[h],
                                               k * 64 * 2, 0, 0);
#pragma unroll
    for (int j = 0; j < WBN; ++j)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rB, &bf.g[(wave + ANW * j) * 8 * 64], 16, dg[j],
                                               k * 64 * 2, 0, 0);
  };

  // fragment (row r, plane p, k chunk lane / 16) at halves r * 64 + sw8a(r, 4 p + lane / 16) * 8;
  // the rows of tile t are 16 t * 64 halves further
  const int lr = lane & 15, kc = lane >> 4;
  const int ru = wm * 64 + lr, rg = wn * 16 * WBN + lr;
  const int ui0 = ru * 64 + sw8a(ru, kc) * 8, ui1 = ru * 64 + sw8a(ru, 4 + kc) * 8;
  const int gj0 = rg * 64 + sw8a(rg, kc) * 8, gj1 = rg * 64 + sw8a(rg, 4 + kc) * 8;
  using Frags = AFrags<WBN>;
  auto read_frags = [&](Frags& fr, const ABuf& bf) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      fr.u[0][t] = *reinterpret_cast<const f16x8*>(&bf.u[ui0 + t * 16 * 64]);
      fr.u[1][t] = *reinterpret_cast<const f16x8*>(&bf.u[ui1 + t * 16 * 64]);
    }
#pragma unroll
    for (int t = 0; t < WBN; ++t) {
      fr.g[0][t] = *reinterpret_cast<const f16x8*>(&bf.g[gj0 + t * 16 * 64]);
      fr.g[1][t] = *reinterpret_cast<const f16x8*>(&bf.g[gj1 + t * 16 * 64]);
    }
  };
  // acc[tj][ti]: rows i (tile ti), columns v (tile tj)
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
      acc[tj][ti] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr.u[pu][ti], fr.g[pg][tj],
                                                           acc[tj][ti], 0, 0, 0);
    }
  };

  // the scale of A: 2^-ilogb(amax[set]); amax is a bound on |A| times 2^-14, so
  // every scaled value stays below 2^15 and fp16 keeps 11 + 11 bits of it
  const float a_scale = (float)pow2_scale_f(g.amax + set);
  _Float16* C = g.A + set * g.a_set;
  const int64_t c_j = (int64_t)g.naux * ld2;   // halves between v rows of A
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  // write the finished tile t.  A wave's 64 rows i (a multiple of 64, so two
  // whole 32-wide chunks) of one v row are 256 contiguous bytes of A.  Per 16
  // columns: each lane puts its four consecutive rows of both planes into the
  // wave's staging rows (v, c32 order), then reads back 16-byte pieces so that
  // 16 lanes store one v row's 256 bytes.
  _Float16* const stg = sstage + wave * 16 * STG_LD;
  const int kq = lane >> 4, vl = lane & 15;
  auto store_tile = [&](int t) {
    const int ib = (first + t * stride) * AM + wm * 64;   // this wave's first row i
    const bool ok = ib < M;   // M is a multiple of 64: all 64 rows or none
    _Float16* const Crow = C + 64 * (int64_t)(ib >> 5);
#pragma unroll
    for (int tj = 0; tj < WBN; ++tj) {
#pragma unroll
      for (int ti = 0; ti < 4; ++ti) {
        const int il = 16 * ti + 4 * kq;   // local row of element r = 0
        h4 hi, lo;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float x = acc[tj][ti][r] * a_scale;
          const _Float16 h = (_Float16)x;
          hi[r] = h;
          lo[r] = (_Float16)(x - (float)h);
        }
        _Float16* o = stg + vl * STG_LD + (il >> 5) * 64 + (il & 31);
        *reinterpret_cast<h4*>(o) = hi;
        *reinterpret_cast<h4*>(o + 32) = lo;
        acc[tj][ti] = f4{0.f, 0.f, 0.f, 0.f};
      }
      // this wave's staging writes complete before its lanes read other lanes' rows
      __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int v = 4 * q + kq;
        const u4 d = *reinterpret_cast<const u4*>(stg + v * STG_LD + vl * 8);
        const int j = j0 + wn * 16 * WBN + 16 * tj + v;
        if (ok && j < g.n) *reinterpret_cast<u4*>(Crow + (int64_t)j * c_j + vl * 8) = d;
      }
      __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
  };

  Frags f0, f1;
  // one stream of stages over (tile, k), the stage in buffer (stage index) mod 2;
  // kst is even, so every tile starts on buffer 0.  Past the end the loads repeat
  // the last stage (never used).
  int ft = 0, fk = 0;
  set_tile(0);
  auto fetch_next = [&](ABuf& bf) {
    dma(bf, fk);
    const bool last = (ft == ntile - 1) && (fk == kst - 1);
    const bool wrap = (fk == kst - 1);
    if (wrap && !last) set_tile(++ft);
    fk = last ? fk : (wrap ? 0 : fk + 1);
  };
  fetch_next(b0);
  fetch_next(b1);
  a_vm_lds_barrier();
  read_frags(f0, b0);
  auto stage = [&](ABuf& cur, ABuf& nxt, Frags& fc, Frags& fn) {
    mfma_range(fc, 0, NQ / 2);
    // the next stage has landed in nxt; every wave is done reading cur
    a_vm_lds_barrier();
    fetch_next(cur);
    read_frags(fn, nxt);
    mfma_range(fc, NQ / 2, NQ);
  };
  for (int t = 0; t < ntile; ++t) {
    for (int ks = 0; ks < kst; ks += 2) {
      stage(b0, b1, f0, f1);
      stage(b1, b0, f1, f0);
    }
    store_tile(t);
  }
  // the last (repeated) memory-to-LDS loads land before the workgroup may end
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// one kernel per column count (the body is a device template)
#define THCSOX_ASTAGE_KERNEL(W)                                                         \
  __global__ __launch_bounds__(ANT) __attribute__((amdgpu_waves_per_eu(2, 2)))          \
  void astage_f16_kernel_##W(AStageArgs g) {                                            \
    __shared__ __attribute__((aligned(16))) ABuf b0;                                    \
    __shared__ __attribute__((aligned(16))) ABuf b1;                                    \
    __shared__ __attribute__((aligned(16))) _Float16 sstage[ANW * 16 * STG_LD];         \
    astage_body<W>(g, b0, b1, sstage);                                                  \
  }
THCSOX_ASTAGE_KERNEL(2)
THCSOX_ASTAGE_KERNEL(3)
THCSOX_ASTAGE_KERNEL(4)
THCSOX_ASTAGE_KERNEL(5)
#undef THCSOX_ASTAGE_KERNEL

inline unsigned a_cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <int WBN>
hipError_t a_launch(void (*kernel)(AStageArgs), const AStageArgs& g, hipStream_t s) {
  // persistent row workers, a multiple of eight (one per XCD in each group of
  // eight), with all parts of a worker on one XCD: about one workgroup per
  // compute unit (the LDS holds one)
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const unsigned X = a_cdiv(g.n, 64 * WBN) * (unsigned)g.nsets;
  const unsigned nib = a_cdiv((int64_t)g.naux * g.ldk, AM);
  unsigned workers = std::min(nib, (unsigned)std::max(1, cus) / X);
  workers = std::max(8u, workers / 8 * 8);
  kernel<<<X * workers, ANT, 0, s>>>(g);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Register-resident variant for ldk <= 320 (n <= 320).  G(beta - tau)^T of one
// set is at most 320 x 320 x 2 planes of fp16 (400 KiB), which fits in the
// register file of one compute unit (4 waves x 512 registers x 64 lanes x 4 B =
// 512 KiB): wave w keeps the MFMA fragments of columns v in [16 NCT w, 16 NCT (w
// + 1)) for every k chunk and plane (4 KST^2 registers, the compiler places them
// in both register files; the matrix cores read AGPR operands directly).  Only
// U then streams through LDS: a step is 32 rows i = P ldk + q of the padded row
// space (one 32-wide q chunk of one P, all KST k chunks: 40 KiB at ldk = 320),
// double-buffered one step ahead.  Per step a wave issues 2 x NCT x KST x 3
// MFMAs against 2 x KST x 2 fragment reads, and the workgroup moves 4 KST KiB
// from L2 to LDS; the streaming variant above re-reads its G panels from L2 for
// every 128-row tile (2.5 times the U bytes at ldk = 320).
//
// Epilogue: the step's 32 rows of one v are one 128-byte line of A (both planes
// of chunk q / 32 of row (v, P)); each wave stages its 16 NCT lines in LDS and
// stores them as 16-byte pieces, eight lanes per line.  The stores of a step are
// issued at the start of the next one (after its loads), so their completion
// overlaps that step's matrix work.
constexpr int RM = 32;          // rows i per step
constexpr int RNW = 4, RNT = 64 * RNW;

template <int KST> struct RBuf {
  _Float16 u[KST][RM * 64];     // [chunk][row][plane][32], 16-byte chunks permuted by sw8a
  // the lines of A computed from u: [wave][line v][plane][32 rows], the eight
  // 16-byte pieces of line v permuted by XOR with v % 8
  _Float16 stg[RNW][16 * (KST / 2)][64];
};

// M = MODE_F16X2, or MODE_F32: FP32 K-major rows, whose 32-wide k chunks are
// 128 bytes as in c32, so the loads, the LDS layout and the stores are the same;
// a chunk is eight 16x16x4 FP32 MFMAs per tile (lane group g takes k = 8 g + j,
// 32 contiguous bytes, in both operands), and A is written unscaled as FP32.
template <int M, int KST>
__device__ __forceinline__ void astage_r_body(const AStageArgs& g, RBuf<KST>& b0, RBuf<KST>& b1) {
  constexpr bool F32 = M == MODE_F32;
  constexpr int NCT = KST / 2;              // 16-column tiles per wave: 4 waves cover ldk columns
  constexpr int LDK = 32 * KST;
  constexpr int LD2 = 2 * LDK;              // halves per c32 row
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nstep = g.naux * KST;
  // block -> (set x, worker y); the sets of worker y are the blocks 8 (X (y / 8) +
  // x) + y % 8, on one XCD, so U is fetched from HBM once for all of them
  const int X = g.nsets;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int set = __builtin_amdgcn_readfirstlane(slot % X);
  const int first = __builtin_amdgcn_readfirstlane((slot / X) * 8 + xcd);
  const int stride = __builtin_amdgcn_readfirstlane(gridDim.x / X);
  const int nst = __builtin_amdgcn_readfirstlane(first < nstep ? (nstep - 1 - first) / stride + 1 : 0);
  if (nst == 0) return;

  // this wave's G fragments: column v = 16 (NCT wave + t) + lane % 16, k = 32 c +
  // 8 (lane / 16) .. + 7 of plane p (zero for v >= n)
  // (rows v >= n lie past the end of the buffer resource and read as zero)
  const __amdgpu_buffer_rsrc_t rG = make_rsrc(static_cast<const _Float16*>(g.Gb) + set * g.gb_set,
                                              (int64_t)g.n * LD2 * 2);
  f16x8 gr[NCT][KST][2];
  // the first fragments live in AGPRs (the matrix cores read them there), as many
  // as fit beside the accumulators; the rest and all other values in VGPRs
  constexpr int NG_A = (256 - 4 * NCT) / 4 < 2 * NCT * KST ? (256 - 4 * NCT) / 4 : 2 * NCT * KST;
  auto in_agpr = [](int t, int c, int p) { return (t * KST + c) * 2 + p < NG_A; };
  // (loaded in batches of 16, the AGPR moves of a batch after the next batch is
  // issued, so that they wait for about one batch's latency each)
  constexpr int NF = 2 * NCT * KST, GB = 16;
  // (FP32: the two 16-byte pieces 2 (lane / 16) and 2 (lane / 16) + 1 of the chunk)
  auto gload = [&](int f) {
    const int t = f / (2 * KST), c = (f / 2) % KST, p = f % 2;
    const int v = 16 * (NCT * wave + t) + (lane & 15);
    const uint32_t gv = (uint32_t)((v * LD2 + (F32 ? 16 : 8) * (lane >> 4)) * 2);
    gr[t][c][p] = __builtin_bit_cast(
        f16x8, __builtin_amdgcn_raw_buffer_load_b128(rG, gv, (c * 64 + (F32 ? 8 : 32) * p) * 2, 0));
  };
#pragma unroll
  for (int f = 0; f < GB && f < NF; ++f) gload(f);
#pragma unroll
  for (int f0 = 0; f0 < NF; f0 += GB) {
#pragma unroll
    for (int f = f0 + GB; f < f0 + 2 * GB && f < NF; ++f) gload(f);
#pragma unroll
    for (int f = f0; f < f0 + GB && f < NF; ++f) {
      const int t = f / (2 * KST), c = (f / 2) % KST, p = f % 2;
      if (in_agpr(t, c, p)) __asm__ volatile("" : "+a"(gr[t][c][p]));
    }
  }

  // memory to LDS: wave w moves rows 8 w .. 8 w + 7 of every chunk (one
  // instruction per chunk: 8 rows x 128 bytes); lane l lands at row 8 w + l / 8,
  // physical 16-byte chunk l % 8, and loads the logical chunk sw8a maps there
  const _Float16* Ub = static_cast<const _Float16*>(g.U);
  const int drow = 8 * wave + (lane >> 3);
  const uint32_t dvoff = (uint32_t)((drow * LD2 + 8 * sw8a(drow, lane & 7)) * 2);
  auto dma = [&](RBuf<KST>& bf, int s) {
    const int st = first + s * stride, P = st / KST, q0 = 32 * (st - P * KST);
    const int nv = min(RM, g.n - q0);   // rows q < n of this step (none past n)
    const i4 r = raw_rsrc(Ub + ((int64_t)P * g.n + q0) * LD2, nv > 0 ? nv * LD2 * 2 : 0);
#pragma unroll
    for (int c = 0; c < KST; ++c) dma16_untracked(r, lds_addr(&bf.u[c][8 * wave * 64]), dvoff, c * 128);
  };

  // fragment (row 16 a + lane % 16, plane p, k chunk lane / 16) of chunk c
  const int lr = lane & 15, kc = lane >> 4;
  // (the permutation depends on the row mod 16, so half a is 16 rows further)
  int uoff[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) uoff[p] = lr * 64 + sw8a(lr, F32 ? 2 * kc + p : 4 * p + kc) * 8;
  // the two 16-row halves of a step run one after the other on the same
  // accumulators (16 x 16 NCT of A per wave)
  f4 acc[NCT];
  auto compute = [&](const RBuf<KST>& bf, int a) {
    // the fragments of chunk c + 1 are read while chunk c's MFMAs run
    f16x8 u[2], un[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) un[p] = *reinterpret_cast<const f16x8*>(&bf.u[0][uoff[p] + a * 16 * 64]);
#pragma unroll
    for (int c = 0; c < KST; ++c) {
#pragma unroll
      for (int p = 0; p < 2; ++p) u[p] = un[p];
      if (c + 1 < KST) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
          un[p] = *reinterpret_cast<const f16x8*>(&bf.u[c + 1][uoff[p] + a * 16 * 64]);
      }
      if constexpr (F32) {
        auto el = [](const f16x8& lo, const f16x8& hi, int e) {
          return e < 4 ? __builtin_bit_cast(f4, lo)[e] : __builtin_bit_cast(f4, hi)[e - 4];
        };
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
          for (int t = 0; t < NCT; ++t) {
            if (in_agpr(t, c, e / 4)) __asm__ volatile("" : "+a"(gr[t][c][e / 4]));
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                el(u[0], u[1], e), el(gr[t][c][0], gr[t][c][1], e),
                (c == 0 && e == 0) ? f4{0.f, 0.f, 0.f, 0.f} : acc[t], 0, 0, 0);
          }
      } else {
#pragma unroll
        for (int pp = 0; pp < 3; ++pp) {
          const int pg = pp == 0 ? 1 : 0, pu = pp == 1 ? 1 : 0;
#pragma unroll
          for (int t = 0; t < NCT; ++t) {
            if (in_agpr(t, c, pg)) __asm__ volatile("" : "+a"(gr[t][c][pg]));
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                u[pu], gr[t][c][pg], (c == 0 && pp == 0) ? f4{0.f, 0.f, 0.f, 0.f} : acc[t], 0, 0, 0);
          }
        }
      }
    }
  };

  // the scale of A (fp16x2): 2^-ilogb(amax[set]), amax a bound on |A| times 2^-14
  const float a_scale = F32 ? 1.f : (float)pow2_scale_f(g.amax + set);
  _Float16* const C = g.A + set * g.a_set;
  const int64_t c_j = (int64_t)g.naux * LD2;   // halves between v rows of A
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  // store offsets (bytes): lane part (line 16 NCT wave + lane / 8, piece lane % 8)
  // and eight lines further per store (offsets below 2^31: checked on the host)
  const uint32_t cvoff = (uint32_t)(((16 * NCT * wave + (lane >> 3)) * c_j + 8 * (lane & 7)) * 2);
  const int cjstep = (int)(8 * c_j * 2);
  // half a of the step: each lane's four consecutive rows of both planes into the
  // wave's staging lines (v, c32 order)
  auto stage_half = [&](RBuf<KST>& bf, int a) {
    _Float16* const stg = &bf.stg[wave][0][0];
    if constexpr (F32) {
      // rows 16 a + 4 kc .. + 3: logical piece 4 a + kc of the line
#pragma unroll
      for (int t = 0; t < NCT; ++t)
        *reinterpret_cast<f4*>(stg + (16 * t + lr) * 64 + 8 * ((4 * a + kc) ^ (lr & 7))) = acc[t];
      return;
    }
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
      h4 hi, lo;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float x = acc[t][r] * a_scale;
        const _Float16 h = (_Float16)x;
        hi[r] = h;
        lo[r] = (_Float16)(x - (float)h);
      }
      // rows 16 a + 4 kc .. + 3: logical piece 2 a + kc / 2 (plane 0), 4 more (plane 1)
      _Float16* o = stg + (16 * t + lr) * 64 + 4 * (kc & 1);
      *reinterpret_cast<h4*>(o + 8 * ((2 * a + (kc >> 1)) ^ (lr & 7))) = hi;
      *reinterpret_cast<h4*>(o + 8 * ((4 + 2 * a + (kc >> 1)) ^ (lr & 7))) = lo;
    }
  };
  // the staged lines of step s: 16-byte pieces, eight lanes per line
  auto store_step = [&](const RBuf<KST>& bf, int s) {
    const int st = first + s * stride, P = st / KST, c0 = st - P * KST;
    const _Float16* const stg = &bf.stg[wave][0][0];
    // this wave's staging writes complete before its lanes read other lanes' lines
    __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    // line of v at v c_j halves from the step's piece of row (0, P); rows v >= n
    // lie past the end of the resource and are not written
    const __amdgpu_buffer_rsrc_t rC =
        make_rsrc(C + (int64_t)P * LD2 + c0 * 64, (int64_t)(g.n - 1) * c_j * 2 + 128);
#pragma unroll
    for (int j = 0; j < 2 * NCT; ++j) {
      // line 8 j + lane / 8 (line % 8 = lane / 8), logical piece lane % 8
      const u4 d = *reinterpret_cast<const u4*>(stg + (8 * j + (lane >> 3)) * 64 +
                                                8 * ((lane & 7) ^ (lane >> 3)));
      __builtin_amdgcn_raw_buffer_store_b128(d, rC, cvoff, j * cjstep, 0);
    }
    // the reads are done before the next step's staging writes
    __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  };
  // a half whose rows are all past n (pad rows of A) is zero without its MFMAs
  auto run_step = [&](RBuf<KST>& bf, int s) {
    const int st = first + s * stride, q0 = 32 * (st - (st / KST) * KST);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      if (q0 + 16 * a < g.n) {
        compute(bf, a);
      } else {
#pragma unroll
        for (int t = 0; t < NCT; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
      }
      stage_half(bf, a);
    }
  };

  // one step ahead: at the top of step s its loads have landed (every wave's) and
  // every wave is done with the other buffer, whose staged lines (step s - 1) are
  // then stored before it takes the loads of step s + 1.  (The staging lines sit
  // in the buffer they are computed from: LDS accesses that alias no pending
  // memory-to-LDS load would otherwise wait for all of them.)
  dma(b0, 0);
  for (int s = 0; s < nst; s += 2) {
    a_vm_lds_barrier();
    if (s > 0) store_step(b1, s - 1);
    if (s + 1 < nst) dma(b1, s + 1);
    run_step(b0, s);
    if (s + 1 >= nst) { store_step(b0, s); break; }
    a_vm_lds_barrier();
    store_step(b0, s);
    if (s + 2 < nst) dma(b0, s + 2);
    run_step(b1, s + 1);
    if (s + 2 >= nst) store_step(b1, s + 1);
  }
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

#define THCSOX_ASTAGE_R_KERNEL(NAME, M, K)                                              \
  __global__ __launch_bounds__(RNT) __attribute__((amdgpu_waves_per_eu(1, 1)))          \
  void NAME(AStageArgs g) {                                                             \
    __shared__ __attribute__((aligned(16))) RBuf<K> b0;                                 \
    __shared__ __attribute__((aligned(16))) RBuf<K> b1;                                 \
    astage_r_body<M, K>(g, b0, b1);                                                     \
  }
THCSOX_ASTAGE_R_KERNEL(astage_f16r_kernel_2, MODE_F16X2, 2)
THCSOX_ASTAGE_R_KERNEL(astage_f16r_kernel_4, MODE_F16X2, 4)
THCSOX_ASTAGE_R_KERNEL(astage_f16r_kernel_6, MODE_F16X2, 6)
THCSOX_ASTAGE_R_KERNEL(astage_f16r_kernel_8, MODE_F16X2, 8)
THCSOX_ASTAGE_R_KERNEL(astage_f16r_kernel_10, MODE_F16X2, 10)
THCSOX_ASTAGE_R_KERNEL(astage_f32r_kernel_2, MODE_F32, 2)
THCSOX_ASTAGE_R_KERNEL(astage_f32r_kernel_4, MODE_F32, 4)
THCSOX_ASTAGE_R_KERNEL(astage_f32r_kernel_6, MODE_F32, 6)
THCSOX_ASTAGE_R_KERNEL(astage_f32r_kernel_8, MODE_F32, 8)
THCSOX_ASTAGE_R_KERNEL(astage_f32r_kernel_10, MODE_F32, 10)
#undef THCSOX_ASTAGE_R_KERNEL

hipError_t r_launch(void (*kernel)(AStageArgs), const AStageArgs& g, hipStream_t s) {
  // persistent step workers, a multiple of eight, the sets of a worker on one XCD
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const unsigned X = (unsigned)g.nsets;
  const unsigned nstep = (unsigned)g.naux * (unsigned)(g.ldk / RM);
  unsigned workers = std::min(nstep, (unsigned)std::max(1, cus) / X);
  workers = std::max(8u, workers / 8 * 8);
  kernel<<<X * workers, RNT, 0, s>>>(g);
  return hipGetLastError();
}

}  // namespace

hipError_t astage_f16(const AStageArgs& g, hipStream_t s) {
  if (g.naux <= 0 || g.n <= 0 || g.nsets <= 0) return hipSuccess;
  if (g.ldk % (2 * AKC) != 0 || g.ldk < g.n) return hipErrorInvalidValue;
  // 32-bit row indices and buffer offsets inside one tile (c32 rows of 4 ldk bytes)
  if ((int64_t)g.naux * g.ldk + AM > 0x7fffffffLL ||
      (int64_t)(AM + 2 * g.n) * g.ldk * 4 > 0x7fffffffLL || (int64_t)320 * g.ldk * 4 > 0x7fffffffLL)
    return hipErrorInvalidValue;
  // G in registers while ldk <= 320 and the byte offsets of A's rows (v, P) fit in
  // 31 bits (the stores address a set from the step's row piece)
  if ((int64_t)g.n * g.naux * g.ldk * 4 < 0x7fffffffLL) switch (g.ldk) {
    case 64: return r_launch(astage_f16r_kernel_2, g, s);
    case 128: return r_launch(astage_f16r_kernel_4, g, s);
    case 192: return r_launch(astage_f16r_kernel_6, g, s);
    case 256: return r_launch(astage_f16r_kernel_8, g, s);
    case 320: return r_launch(astage_f16r_kernel_10, g, s);
    default: break;
  }
  if (g.n <= 128) return a_launch<2>(astage_f16_kernel_2, g, s);
  if (g.n <= 192) return a_launch<3>(astage_f16_kernel_3, g, s);
  if (g.n <= 256) return a_launch<4>(astage_f16_kernel_4, g, s);
  return a_launch<5>(astage_f16_kernel_5, g, s);   // 320 columns per workgroup, more beyond
}

bool astage_f32_fits(int n, int naux, int ldk) {
  return n > 0 && naux > 0 && ldk >= n && ldk % 64 == 0 && ldk <= 320 &&
         (int64_t)n * naux * ldk * 4 < 0x7fffffffLL;
}

hipError_t astage_f32(const AStageArgs& g, hipStream_t s) {
  if (g.naux <= 0 || g.n <= 0) return hipSuccess;
  if (g.nsets != 1 || !astage_f32_fits(g.n, g.naux, g.ldk)) return hipErrorInvalidValue;
  switch (g.ldk) {
    case 64: return r_launch(astage_f32r_kernel_2, g, s);
    case 128: return r_launch(astage_f32r_kernel_4, g, s);
    case 192: return r_launch(astage_f32r_kernel_6, g, s);
    case 256: return r_launch(astage_f32r_kernel_8, g, s);
    default: return r_launch(astage_f32r_kernel_10, g, s);
  }
}

}  // namespace thcsox
