// Kernel launchers of libthcsox (host-side declarations).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace thcsox {

// Strided FP64 GEMM on matrix cores, batched over grid.z:
//   C(i,j) = alpha * sum_k A(i,k) B(k,j) + beta * C(i,j)
//   A(i,k) = A[b*a_b + i*a_i + k*a_k],  B(k,j) = B[b*b_b + k*b_k + j*b_j],
//   C(i,j) = C[b*c_b + i*c_i + (j / cj_in) * cj_out + (j % cj_in) * c_j].
// beta == 0 never reads C.
struct Gemm64Args {
  int M, N, K, batch;
  double alpha, beta;
  const double* A; int64_t a_i, a_k, a_b;
  const double* B; int64_t b_k, b_j, b_b;
  double* C; int64_t c_i, c_j, c_b; int64_t cj_in, cj_out;
};
hipError_t gemm64(const Gemm64Args& g, hipStream_t s);

// GEMM over K-major operand planes in one of the four modes:
//   C(i,j) = alpha * sum_{k < kpad} A[i][k] B[j][k]   (operand pad must be zero)
//   A rows:  A + p*a_plane + i*lda          (i < M)
//   B rows:  B + p*b_plane + j*ldb          (j < N)
//   C(i,j) = C[(i / ci_in) * ci_out + (i % ci_in) + j * c_j]  (OutT = double or float)
// If amax != nullptr, the largest |C(i,j)| is max-reduced into *amax (as the
// bits of a non-negative double).
struct GemmKArgs {
  int M, N, kpad;
  double alpha;
  const void* A; int64_t lda, a_plane;
  const void* B; int64_t ldb, b_plane;
  void* C; int64_t ci_in, ci_out, c_j;
  unsigned long long* amax;
  int64_t c_plane;   // gemm_kmajor_bf3: elements between the output planes
};
hipError_t gemm_kmajor(int mode, bool out_f64, const GemmKArgs& g, hipStream_t s);
// The same product in the bf16x3 mode with the output split into three bf16
// planes (C + p * c_plane, p < 3) instead of FP32 (no scale: bf16 keeps FP32's
// exponent range); amax is not used.
hipError_t gemm_kmajor_bf3(const GemmKArgs& g, hipStream_t s);
// The A stage of the fp16x2 mode for nsets tau points at once:
//   A[set][v][P][q] = scale[set] * sum_s U[P][q][s] Gb[set][v][s]   (q < n; rows n <= q < ldk get 0)
// All operands are fp16 planes in the c32 layout (row r, plane p, k at
// r * 2 ldk + (k / 32) * 64 + 32 p + k % 32): U rows (P, q), Gb rows (set, v)
// (G(beta - tau)^T, gb_set = n * 2 ldk halves apart), A rows (set, v, P) with
// k = q (a_set halves apart).  scale[set] = 2^-ilogb(amax[set]); amax[set] must
// bound max |A| / 2^14 (see ascale_bound).  ldk must be a multiple of 64.
struct AStageArgs {
  int naux, n, ldk, nsets;
  const void* U;
  const void* Gb; int64_t gb_set;
  _Float16* A; int64_t a_set;
  const unsigned long long* amax;
};
hipError_t astage_f16(const AStageArgs& a, hipStream_t s);
// The same stage in the FP32 mode for one tau point (nsets = 1; amax, a_set
// unused): U, Gb and A are FP32 K-major rows of ldk elements (A passed as the
// address of its FP32 array), A written unscaled.  Only for ldk a multiple of 64
// up to 320 with A's byte offsets in 31 bits (astage_f32_fits); otherwise
// hipErrorInvalidValue (use gemm_kmajor).
bool astage_f32_fits(int n, int naux, int ldk);
hipError_t astage_f32(const AStageArgs& a, hipStream_t s);
// The A stage of the bf16x3 mode for one tau point:
//   A[p][v][P][q] = plane p of the bf16x3 split of sum_s U[P][q][s] Gb[v][s]
//   (q < n; rows n <= q < ldk get 0)
// U rows (P, q) and Gb rows v (G(beta - tau)^T) are three bf16 planes of ldk
// elements per row (u_plane, gb_plane elements apart), A rows (v, P) with k = q
// (a_plane apart).  Only for ldk = 32 ceil(n / 32) <= 320 with byte offsets in
// 31 bits (astage_bf3_fits); otherwise hipErrorInvalidValue (use gemm_kmajor_bf3).
struct AStageB3Args {
  int naux, n, ldk;
  const void* U; int64_t u_plane;
  const void* Gb; int64_t gb_plane;
  void* A; int64_t a_plane;
  int wx0, wx1;   // set by the launcher
};
bool astage_bf3_fits(int n, int naux, int ldk);
hipError_t astage_bf3(const AStageB3Args& a, hipStream_t s);

// The fused B/C/D stage for one tau point (v split over grid.z):
//   Dpart[z][R][P] = sum_{v in split z} (sum_q Gt[R][q] A[v][P][q]) (sum_w U[R][v][w] GXt[P][w])
// A holds the mode's planes (fp16x2: scaled by the power of two taken from
// *amax_a, which the reduction divides out; otherwise unscaled).  In the fp16x2
// mode every operand is in the c32 layout and the plane strides are unused; in
// the fp16x2 and FP32 modes the v split counts pairs of v: split z covers the
// pairs [z' np / vsplit, (z' + 1) np / vsplit) (np = ceil(n / 2)).
struct FusedArgs {
  int n, naux, ldk, vsplit, vchunk;
  const void* Gt; const void* GXt; int64_t g_plane;   // [naux][ldk] planes
  const void* U; int64_t u_plane;                      // [naux][n][ldk] planes
  const void* A; int64_t a_plane;                      // [n][naux][ldk] planes
  const unsigned long long* amax_a;
  double* Dpart;                                       // [vsplit][naux][naux]
  // Dpart holds FP32 partial tiles (reinterpreted as float*).  Only with v ranges
  // of at most 8 in the reduced-precision modes: each range is then one FP32
  // partial sum, so storing it as FP32 is exact.
  bool dpart_f32;
  // If sym != nullptr and *sym != 0, D is symmetric (G(tau) and G(beta - tau)
  // symmetric): tiles lying wholly below the diagonal (every R > every P) are
  // skipped and their Dpart entries are left untouched.
  const int* sym;
};
hipError_t sox_fused(int mode, const FusedArgs& f, hipStream_t s);
void fused_tile(int mode, int* rows, int* cols);   // D tile one workgroup owns (R x P)
// the two-v kernel of the fp16x2 and FP32 modes, used by sox_fused for them
hipError_t sox_fused_pairs(int mode, const FusedArgs& f, hipStream_t s);
// the bf16x3 kernel (three bf16 planes, one v per pass), used by sox_fused for
// that mode
hipError_t sox_fused_bf3(const FusedArgs& f, hipStream_t s);
void fused_f16_tile(int* rows, int* cols);
int fused_xcds();   // vsplit must be a multiple of this (one v range per XCD in turn)

// Split rows of an FP64 source into the planes of a mode, scaled by the power of
// two 2^-floor(log2(amax[r2 * amax_s2])) (scale 1 if amax is null or zero):
//   src(r1,r2,c) = src[r1*s1 + r2*s2 + c*sc],  dst plane p:
//   dst[p*d_plane + r1*d1 + r2*d2 + c] for c < cols, zero for cols <= c < ldk.
// With c32 (fp16x2 only) the planes are interleaved per 32-wide chunk instead:
//   element c of plane p at dst[r1*d1 + r2*d2 + (c / 32) * 64 + 32 p + c % 32].
struct SplitArgs {
  int rows1, rows2, cols, ldk;
  const void* src; bool src_f32; int64_t s1, s2, sc;
  void* dst; int64_t d1, d2, d_plane;
  const unsigned long long* amax; int64_t amax_s2;
  bool c32;
};
hipError_t split_planes(int mode, const SplitArgs& a, hipStream_t s);

// amax[b] = max |x[b*stride + i]| for i < len, for b < batch (max-reduced).
hipError_t absmax64(const double* x, int64_t len, int64_t stride, int batch,
                    unsigned long long* amax, hipStream_t s);
hipError_t fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
// *out = max over rows r < rows of sum_{c < len} x[r ld + c]^2 (max-reduced, bits;
// *out must hold 0 or an earlier maximum).
hipError_t rownorm2_max(const double* x, int64_t rows, int len, int64_t ld,
                        unsigned long long* out, hipStream_t s);
// out[b] = max over columns v of sum_s G_b[s][v]^2 for the n x n matrices
// G_b = G + b stride, b < nb (stride may be negative; out zeroed by the caller).
hipError_t colnorm2_max(const double* G, int n, int64_t stride, int nb, unsigned long long* out,
                        hipStream_t s);
// The A-stage scale of the fp16x2 mode, before A exists: for b < nb,
//   amax_a[b] = 2^-14 (1 + 2^-10) sqrt(*unorm2) su sqrt(gnorm2[b]) sg_b
// with su = 2^-ilogb(*amax_u), sg_b = 2^-ilogb(amax_gb[b gb_stride]): unorm2 and
// gnorm2 are the largest squared row norms of U and of G(beta - tau)^T, so by
// Cauchy-Schwarz the scale 2^-ilogb(amax_a[b]) keeps every |A| below 2^15.
hipError_t ascale_bound(const unsigned long long* unorm2, const unsigned long long* amax_u,
                        const unsigned long long* gnorm2, const unsigned long long* amax_gb,
                        int64_t gb_stride, int nb, unsigned long long* amax_a, hipStream_t s);

// Sthc[R][P] = -factor * sum_z Dpart[z][R][P], factor = product of the inverse
// operand scales (see scale_factor in the kernel source).
// With sym != nullptr and *sym != 0 (symmetric D, lower tiles skipped by the
// fused stage), entries with R > P are taken from the mirrored position P, R.
struct DReduceArgs {
  int naux, vsplit;
  const double* Dpart;   // FP64 partial tiles, or FP32 ones if dpart_f32
  bool dpart_f32;
  double* Sthc; int64_t s_ld;
  const unsigned long long* amax_gt; const unsigned long long* amax_gx;
  const unsigned long long* amax_gb; const unsigned long long* amax_a;
  const unsigned long long* amax_u;
  // the U of the C product when it differs from the A product's (two cores); null: amax_u
  const unsigned long long* amax_u2;
  const int* sym;
};
hipError_t dreduce(const DReduceArgs& a, hipStream_t s);

// asym[k] = max |G[k] - G[k]^T| (as the bits of a non-negative double), k < m.
hipError_t asym64(const double* G, int n, int m, unsigned long long* asym, hipStream_t s);
// flag[k] = 1 if both G[k] and G[m-1-k] are symmetric to within rtol of the
// largest element of G on the whole grid (asym[k] <= rtol * max_j amax[j]), else 0.
hipError_t sym_flags(const unsigned long long* asym, const unsigned long long* amax, int m,
                     double rtol, int* flag, hipStream_t s);

// KR[(q - q0)*n + s][Q] = X[q][Q] * X[s][Q] for q in [q0, q1).
hipError_t khatri_rao(const double* X, int n, int naux, int q0, int q1, double* KR,
                      hipStream_t s);

// Inverse of one real n x n matrix (row-major, n <= 9216) by the Dyson step's
// blocked Gauss-Jordan elimination with partial pivoting on a complex copy.
// Work: Am [n n] double2, piv and perm [n] ints, flag [1] int, set to 1 for a
// zero or non-finite pivot (read it after synchronising).
hipError_t gj_inverse_real(const double* M, int n, double* Minv, double2* Am, int* piv, int* perm,
                           int* flag, hipStream_t s);

// Pi0[e] (+)= sum_b w[b] Pi[b][e] over nb blocks of len elements, b in order
// (accumulate = 0: Pi0 is overwritten).
hipError_t weighted_block_sum(const double* Pi, const double* w, int nb, int64_t len,
                              double* Pi0, int accumulate, hipStream_t s);
// A[i][i] += 1 for i < n (row-major n x n).
hipError_t add_identity(double* A, int n, hipStream_t s);

// tr[k] = sum_pq G[m-1-k][q][p] Sigma[k][p][q]; then E = -1/2 sum_k w[k] tr[k].
hipError_t energy_partials(const double* G, const double* S, int n, int m, double* tr,
                           hipStream_t s);
hipError_t energy_final(const double* tr, const double* w, int m, double* E, hipStream_t s);

}  // namespace thcsox
