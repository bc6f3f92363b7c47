// C interface of libthcsox: plan construction (the U precontraction), the
// per-tau SOX pipeline and the Galitskii-Migdal energy.  See include/thcsox.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/thcsox.h"
#include "error.hpp"
#include "direct.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace thcsox {
namespace {
thread_local std::string g_last_error;
}
int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
void clear_error() { g_last_error.clear(); }
}  // namespace thcsox

using namespace thcsox;

namespace {

int fail(int code, const std::string& msg) { return set_error(code, msg); }

// G(tau) counts as symmetric when max |G(tau) - G(tau)^T| <= rtol max |G| (the
// largest element on the whole grid); the symmetric-D path then changes Sigma
// by at most about that amount relative to its largest element:
// 1e-12 for FP64 plans, 1e-10 for the reduced-precision ones (whose own
// rounding error is about 1e-8).  A Green's function from a Dyson step carries
// an asymmetry of that order from the rounding of the inversion.
constexpr double SYM_RTOL_F64 = 1e-12;
constexpr double SYM_RTOL_MIXED = 1e-10;

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(THCSOX_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

int check_dev(const void* p, const char* name) {
  if (p == nullptr) return fail(THCSOX_EINVAL, std::string(name) + " is NULL");
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(THCSOX_ENOTDEV, std::string(name) + " is not device memory");
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
    return fail(THCSOX_ENOTDEV, std::string(name) + " is not device memory");
  return 0;
}

size_t elem_size(int mode) {
  switch (mode) {
    case MODE_F64: return 8;
    case MODE_F32: return 4;
    default: return 2;
  }
}
int n_planes(int mode) { return mode == MODE_BF16X3 ? 3 : mode == MODE_F16X2 ? 2 : 1; }

// Device scratch of the allocation-free energy entry point: the per-tau traces
// Tr[G(beta - tau_k) Sigma(tau_k)].  Each GPU holds its own copy for the life of
// the process.  In host code the name stands for the host-side shadow only; the
// device address comes from hipGetSymbolAddress (scratch_on_current_device).
constexpr int NOALLOC_MAX_NTAU = 4096;
static __device__ __align__(256) double scratch[NOALLOC_MAX_NTAU];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int scratch_on_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return fail(THCSOX_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(THCSOX_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return fail(THCSOX_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

}  // namespace

struct thcsox_plan_s {
  int n = 0, naux = 0, m = 0, mode = 0, ldk = 0, np = 1;
  double beta = 0;
  size_t esize = 8;
  hipStream_t stream = nullptr;
  std::vector<void*> allocs;
  size_t bytes = 0, limit = 0;

  double* X = nullptr;      // [n][naux]
  double* V = nullptr;      // [naux][naux] (the direct term)
  double* dbuf = nullptr;   // direct term: 3 x [tbd][naux][naux], allocated on first use
  double* ebuf = nullptr;   // basis energy: 2 x [ntau][n][n] coefficients, on first use
  double* ecoef = nullptr;  // basis energy: [2][ntau][ntau] (rows reversed, then as given)
  double* esign = nullptr;  // basis energy: [ntau]
  int tbd = 0;              // tau points per direct-term batch
  // screened exchange (allocated on first use): the second U (from the screened
  // core W, same layout and precision as U) and its max |.|, the static
  // polarization Pi0, 1 + V Pi0 and its inverse, and the Gauss-Jordan work
  void* Uw = nullptr;
  unsigned long long* amax_w = nullptr;
  double* Pi0 = nullptr;
  double* Mscr = nullptr;
  double* Minv = nullptr;
  double2* Am = nullptr;
  int* gj = nullptr;        // [2 naux + 1]: pivots, permutation, flag
  double* w = nullptr;      // [m]
  void* U = nullptr;        // planes of [naux][n][ldk] (fp16x2: c32 rows [naux][n])
  int64_t u_plane = 0;
  void* A = nullptr;        // planes of [n][naux][ldk] (fp16x2: [a_sets] c32 rows [n][naux])
  int64_t a_plane = 0;
  int a_sets = 1;           // tau points per A-stage launch (fp16x2: 2 while A is small)
  // fp16x2: the largest squared row norms of U ([0]) and of the screened core's
  // U ([1]), and of G(beta - tau)^T for each tau of a batch ([2 ..]): the A
  // stage's scale is taken from their product before A is formed
  unsigned long long* norm2 = nullptr;
  int tb = 1;               // tau points per projection / back-projection batch
  void* Gt = nullptr;       // planes of [tb][naux][ldk] (fp16x2: c32 rows [tb][naux])
  void* GX = nullptr;
  int64_t g_plane = 0;
  void* Gb = nullptr;       // planes of [tb][n][ldk]: G(beta - tau)^T (fp16x2: c32 rows)
  int64_t gb_plane = 0;
  double* Gt64 = nullptr;   // [tb][naux][n]
  double* GX64 = nullptr;   // [tb][naux][n]
  double* Dpart = nullptr;  // [vsplit][naux][naux], FP64 or (dpart_f32) FP32
  bool dpart_f32 = false;
  int vsplit = 1, vchunk = 1;
  double* Sthc = nullptr;   // [tb][naux][naux]
  double* T1 = nullptr;     // [tb][n][naux]
  // max-abs values as the bits of non-negative doubles: [0] U, then five arrays
  // of m per-tau entries: Gt, GX, A, G[k], asymmetry of G[k]
  unsigned long long* amax = nullptr;
  int* symflag = nullptr;   // [m]: 1 where the symmetric-D path applies
  int sym_mode = THCSOX_SYM_AUTO;
  unsigned long long* am_gt() { return amax + 1; }
  unsigned long long* am_gx() { return amax + 1 + m; }
  unsigned long long* am_a() { return amax + 1 + 2 * (int64_t)m; }
  unsigned long long* am_g() { return amax + 1 + 3 * (int64_t)m; }
  unsigned long long* am_asym() { return amax + 1 + 4 * (int64_t)m; }
  // optional per-stage timing with events on the plan's stream
  bool profiling = false;
  struct Timer {
    std::vector<hipEvent_t> start, stop;
    size_t used = 0;
  } timers[THCSOX_NSTAGES];
  double* tr = nullptr;     // [m]
  double* E = nullptr;      // [1]

  template <typename T>
  int alloc(T** p, size_t count) {
    size_t b = count * sizeof(T);
    if (b == 0) b = 16;
    b = (b + 255) & ~size_t(255);
    if (limit && bytes + b > limit)
      return fail(THCSOX_ENOMEM, "workspace_limit of " + std::to_string(limit) +
                                     " bytes is too small (need more than " +
                                     std::to_string(bytes + b) + ")");
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, b);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(THCSOX_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed: " +
                                     hipGetErrorString(e));
    }
    allocs.push_back(q);
    bytes += b;
    *p = static_cast<T*>(q);
    return 0;
  }
  ~thcsox_plan_s() {
    for (auto& t : timers) {
      for (hipEvent_t e : t.start) (void)hipEventDestroy(e);
      for (hipEvent_t e : t.stop) (void)hipEventDestroy(e);
    }
    for (void* q : allocs) (void)hipFree(q);
  }
  hipError_t mark(int stage, bool begin) {
    if (!profiling) return hipSuccess;
    Timer& t = timers[stage];
    if (begin && t.used == t.start.size()) {
      hipEvent_t a, b;
      hipError_t e = hipEventCreate(&a);
      if (e != hipSuccess) return e;
      if ((e = hipEventCreate(&b)) != hipSuccess) return e;
      t.start.push_back(a);
      t.stop.push_back(b);
    }
    if (begin) return hipEventRecord(t.start[t.used], stream);
    return hipEventRecord(t.stop[t.used++], stream);
  }
};

namespace {

#define TRY(expr)            \
  do {                       \
    int rc_ = (expr);        \
    if (rc_ != 0) return rc_; \
  } while (0)

// U_Pqs = sum_Q V_PQ X_qQ X_sQ in FP64, chunked over q, stored in the operand
// planes Uout (the plan's U, or the second U of a screened core).  Split modes
// first take max|U| into *amax_slot (pass 0; fp16x2 also the largest squared row
// norm into *norm_slot), then store (pass 1).
int build_u(thcsox_plan_s* p, const double* V, void* Uout, unsigned long long* amax_slot,
            unsigned long long* norm_slot) {
  const int n = p->n, naux = p->naux, ldk = p->ldk;
  const hipStream_t s = p->stream;
  size_t per_q = (size_t)n * naux * sizeof(double);
  int qb = (int)std::max<size_t>(1, std::min<size_t>((size_t)n, (size_t(256) << 20) / per_q));
  double* KR = nullptr;
  TRY(p->alloc(&KR, (size_t)qb * n * naux));
  double* Uc = nullptr;
  if (p->mode != MODE_F64) TRY(p->alloc(&Uc, (size_t)qb * n * naux));
  HIP_TRY(fill_u64(amax_slot, 1, 0ull, s));
  const bool c32 = p->mode == MODE_F16X2;
  if (c32) HIP_TRY(fill_u64(norm_slot, 1, 0ull, s));
  const int64_t lrow = c32 ? 2 * (int64_t)ldk : ldk;   // elements per operand row
  const int passes = p->mode == MODE_F64 ? 1 : 2;
  for (int pass = 0; pass < passes; ++pass) {
    for (int q0 = 0; q0 < n; q0 += qb) {
      const int q1 = std::min(n, q0 + qb), qc = q1 - q0;
      HIP_TRY(khatri_rao(p->X, n, naux, q0, q1, KR, s));
      Gemm64Args g{};
      g.M = naux; g.N = qc * n; g.K = naux; g.batch = 1; g.alpha = 1.0; g.beta = 0.0;
      g.A = V; g.a_i = naux; g.a_k = 1;
      g.B = KR; g.b_k = 1; g.b_j = naux;
      if (p->mode == MODE_F64) {
        g.C = static_cast<double*>(Uout) + (int64_t)q0 * ldk;
        g.c_i = (int64_t)n * ldk; g.c_j = 1; g.cj_in = n; g.cj_out = ldk;
      } else {
        g.C = Uc; g.c_i = (int64_t)qc * n; g.c_j = 1; g.cj_in = (int64_t)qc * n; g.cj_out = 0;
      }
      HIP_TRY(gemm64(g, s));
      if (p->mode == MODE_F64) continue;
      if (pass == 0) {
        HIP_TRY(absmax64(Uc, (int64_t)naux * qc * n, 0, 1, amax_slot, s));
        // rows (P, q) of the chunk are the consecutive n-element rows of Uc
        if (c32) HIP_TRY(rownorm2_max(Uc, (int64_t)naux * qc, n, n, norm_slot, s));
      } else {
        SplitArgs a{};
        a.rows1 = naux; a.rows2 = qc; a.cols = n; a.ldk = ldk;
        a.src = Uc; a.src_f32 = false; a.s1 = (int64_t)qc * n; a.s2 = n; a.sc = 1;
        a.dst = static_cast<char*>(Uout) + (size_t)q0 * lrow * p->esize;
        a.d1 = (int64_t)n * lrow; a.d2 = lrow; a.d_plane = p->u_plane;
        a.amax = amax_slot; a.c32 = c32;
        HIP_TRY(split_planes(p->mode, a, s));
      }
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  // the temporaries are the last two allocations: release them
  for (int t = 0; t < (p->mode == MODE_F64 ? 1 : 2); ++t) {
    void* q = p->allocs.back();
    p->allocs.pop_back();
    (void)hipFree(q);
  }
  p->bytes -= ((size_t)qb * n * naux * sizeof(double) + 255) / 256 * 256 *
              (p->mode == MODE_F64 ? 1 : 2);
  return 0;
}

// Sigma[b] = X Sig_thc[b] X^T for nb tau points at once (FP64 matrix cores);
// Sig_thc[b] = St + b * st_stride, Sigma[b] = Sig + b * n * n (beta_out = 1: Sigma[b] +=).
int backproject_batch(thcsox_plan_s* p, const double* St, int64_t st_stride, double* Sig,
                      int nb, double beta_out = 0.0, double alpha_out = 1.0) {
  const int n = p->n, naux = p->naux;
  const hipStream_t s = p->stream;
  Gemm64Args b{};
  b.M = n; b.N = naux; b.K = naux; b.batch = nb; b.alpha = 1.0; b.beta = 0.0;
  b.A = p->X; b.a_i = naux; b.a_k = 1; b.a_b = 0;
  b.B = St; b.b_k = naux; b.b_j = 1; b.b_b = st_stride;
  b.C = p->T1; b.c_i = naux; b.c_j = 1; b.cj_in = naux; b.cj_out = 0; b.c_b = (int64_t)n * naux;
  HIP_TRY(gemm64(b, s));
  b.N = n;
  b.A = p->T1; b.a_i = naux; b.a_k = 1; b.a_b = (int64_t)n * naux;
  b.B = p->X; b.b_k = 1; b.b_j = naux; b.b_b = 0;
  b.C = Sig; b.c_i = n; b.c_j = 1; b.cj_in = n; b.cj_out = 0; b.c_b = (int64_t)n * n;
  b.alpha = alpha_out;
  b.beta = beta_out;   // 1: add to what Sig holds
  HIP_TRY(gemm64(b, s));
  return 0;
}

// The core matrices of the two interaction lines of the exchange diagram, as
// their U planes: UA on the line (pr|qs) (enters A), UC on (tu|vw) (enters C).
// SOX has the plan's U on both; the symmetric-D path needs UA == UC.
struct Cores {
  const void* UA; const unsigned long long* amaxA;
  const void* UC; const unsigned long long* amaxC;
  const unsigned long long* normA;   // fp16x2: largest squared row norm of UA
};

// Tau points k0 <= k < k1 (k1 - k0 <= tb): Sigma[k] (and Sig_thc[k]) from G,
// Sigma[k] = alpha_out X Sig_thc X^T + beta_out Sigma[k].
// Needs the per-tau max |G[k]| and the symmetry flags of every k (set by the caller).
int sigma_batch(thcsox_plan_s* p, const double* G, double* Sigma, double* Sthc_out, int k0,
                int k1, const Cores& cores, double alpha_out = 1.0, double beta_out = 0.0) {
  const bool same_core = cores.UA == cores.UC;
  const int n = p->n, naux = p->naux, ldk = p->ldk, m = p->m, mode = p->mode;
  const int nb = k1 - k0;
  const hipStream_t s = p->stream;
  const int64_t nn = (int64_t)n * n, an = (int64_t)naux * n, aa = (int64_t)naux * naux;
  const size_t es = p->esize;
  HIP_TRY(p->mark(THCSOX_STAGE_PROJECT, true));
  HIP_TRY(fill_u64(p->am_gt() + k0, nb, 0ull, s));
  HIP_TRY(fill_u64(p->am_gx() + k0, nb, 0ull, s));
  HIP_TRY(fill_u64(p->am_a() + k0, nb, 0ull, s));

  // projections of the batch: Gt[b][R][q] = sum_u X[u][R] G[k0+b][u][q],
  // GX[b][P][w] = sum_p G[k0+b][w][p] X[p][P]
  Gemm64Args g{};
  g.M = naux; g.N = n; g.K = n; g.batch = nb; g.alpha = 1.0; g.beta = 0.0;
  g.A = p->X; g.a_i = 1; g.a_k = naux; g.a_b = 0;
  g.B = G + (int64_t)k0 * nn; g.b_k = n; g.b_j = 1; g.b_b = nn;
  g.C = p->Gt64; g.c_i = n; g.c_j = 1; g.cj_in = n; g.cj_out = 0; g.c_b = an;
  HIP_TRY(gemm64(g, s));
  g.b_k = 1; g.b_j = n;
  g.C = p->GX64;
  HIP_TRY(gemm64(g, s));
  HIP_TRY(absmax64(p->Gt64, an, an, nb, p->am_gt() + k0, s));
  HIP_TRY(absmax64(p->GX64, an, an, nb, p->am_gx() + k0, s));

  // fp16x2 keeps the two planes of each 32-wide chunk together (c32 rows of 2 ldk)
  const bool c32 = mode == MODE_F16X2;
  const int64_t lrow = c32 ? 2 * (int64_t)ldk : ldk;
  SplitArgs sa{};
  sa.rows1 = naux; sa.rows2 = nb; sa.cols = n; sa.ldk = ldk;
  sa.src_f32 = false; sa.s1 = n; sa.s2 = an; sa.sc = 1;
  sa.d1 = lrow; sa.d2 = (int64_t)naux * lrow; sa.d_plane = p->g_plane; sa.c32 = c32;
  sa.src = p->Gt64; sa.dst = p->Gt; sa.amax = p->am_gt() + k0; sa.amax_s2 = 1;
  HIP_TRY(split_planes(mode, sa, s));
  sa.src = p->GX64; sa.dst = p->GX; sa.amax = p->am_gx() + k0;
  HIP_TRY(split_planes(mode, sa, s));
  // G(beta - tau)^T of each tau of the batch: row v holds G[m-1-k][s][v] over s
  sa.rows1 = n; sa.src = G + (int64_t)(m - 1 - k0) * nn; sa.s1 = 1; sa.s2 = -nn; sa.sc = n;
  sa.d2 = (int64_t)n * lrow; sa.dst = p->Gb; sa.d_plane = p->gb_plane;
  sa.amax = p->am_g() + (m - 1 - k0); sa.amax_s2 = -1;
  HIP_TRY(split_planes(mode, sa, s));
  if (c32) {
    // the A stage's scale for each tau of the batch, from the row norms of U and
    // of G(beta - tau)^T (the columns of G(beta - tau))
    unsigned long long* gn = p->norm2 + 2;
    HIP_TRY(fill_u64(gn, nb, 0ull, s));
    HIP_TRY(colnorm2_max(G + (int64_t)(m - 1 - k0) * nn, n, -nn, nb, gn, s));
    HIP_TRY(ascale_bound(cores.normA, cores.amaxA, gn, p->am_g() + (m - 1 - k0), -1, nb,
                         p->am_a() + k0, s));
  }
  HIP_TRY(p->mark(THCSOX_STAGE_PROJECT, false));

  // fp16x2 scales A by a power of two (bound taken before the A stage); the
  // bf16x3 A stage writes three unscaled bf16 planes (FP32's exponent range)
  const bool scaled_a = mode == MODE_F16X2;
  for (int b = 0; b < nb; ++b) {
    const int k = k0 + b, kb = m - 1 - k;
    const int* sym = same_core && p->sym_mode == THCSOX_SYM_AUTO ? p->symflag + k : nullptr;
    // A[v][P][q] = sum_s U[P][q][s] G(beta - tau)[s][v]: rows (P,q) of U against rows v of Gb
    // (fp16x2: for up to a_sets tau points at once, into set b % a_sets of A)
    const int aset = mode == MODE_F16X2 ? b % p->a_sets : 0;
    const int64_t a_set = (int64_t)n * naux * lrow;   // fp16x2: halves per set of A
    if (aset == 0) {
      HIP_TRY(p->mark(THCSOX_STAGE_A, true));
      if (mode == MODE_F16X2) {
        AStageArgs ast{};
        ast.naux = naux; ast.n = n; ast.ldk = ldk; ast.nsets = std::min(p->a_sets, nb - b);
        ast.U = cores.UA;
        ast.Gb = static_cast<const char*>(p->Gb) + (size_t)b * n * lrow * es;
        ast.gb_set = (int64_t)n * lrow;
        ast.A = static_cast<_Float16*>(p->A); ast.a_set = a_set;
        ast.amax = p->am_a() + k;
        HIP_TRY(astage_f16(ast, s));
      } else if (mode == MODE_F32 && astage_f32_fits(n, naux, ldk)) {
        AStageArgs ast{};
        ast.naux = naux; ast.n = n; ast.ldk = ldk; ast.nsets = 1;
        ast.U = cores.UA;
        ast.Gb = static_cast<const char*>(p->Gb) + (size_t)b * n * ldk * es;
        ast.A = static_cast<_Float16*>(p->A);
        HIP_TRY(astage_f32(ast, s));
      } else if (mode == MODE_BF16X3 && astage_bf3_fits(n, naux, ldk)) {
        AStageB3Args ab{};
        ab.naux = naux; ab.n = n; ab.ldk = ldk;
        ab.U = cores.UA; ab.u_plane = p->u_plane;
        ab.Gb = static_cast<const char*>(p->Gb) + (size_t)b * n * ldk * es;
        ab.gb_plane = p->gb_plane;
        ab.A = p->A; ab.a_plane = p->a_plane;
        HIP_TRY(astage_bf3(ab, s));
      } else {
        GemmKArgs ga{};
        ga.M = naux * n; ga.N = n; ga.kpad = ldk; ga.alpha = 1.0;
        ga.A = cores.UA; ga.lda = ldk; ga.a_plane = p->u_plane;
        ga.B = static_cast<const char*>(p->Gb) + (size_t)b * n * ldk * es;
        ga.ldb = ldk; ga.b_plane = p->gb_plane;
        ga.ci_in = n; ga.ci_out = ldk; ga.c_j = (int64_t)naux * ldk;
        ga.C = p->A;
        ga.amax = nullptr;
        if (mode == MODE_BF16X3) {
          ga.c_plane = p->a_plane;
          HIP_TRY(gemm_kmajor_bf3(ga, s));
        } else {
          HIP_TRY(gemm_kmajor(mode, mode == MODE_F64, ga, s));
        }
      }
      HIP_TRY(p->mark(THCSOX_STAGE_A, false));
    }

    FusedArgs f{};
    f.n = n; f.naux = naux; f.ldk = ldk; f.vsplit = p->vsplit; f.vchunk = p->vchunk;
    f.Gt = static_cast<const char*>(p->Gt) + (size_t)b * naux * lrow * es;
    f.GXt = static_cast<const char*>(p->GX) + (size_t)b * naux * lrow * es;
    f.g_plane = p->g_plane;
    f.U = cores.UC; f.u_plane = p->u_plane;
    // A already in the mode's planes (fp16x2: split and scaled by the A stage)
    f.A = c32 ? static_cast<const void*>(static_cast<const _Float16*>(p->A) + aset * a_set) : p->A;
    f.a_plane = p->a_plane;
    f.amax_a = scaled_a ? p->am_a() + k : nullptr;
    f.Dpart = p->Dpart; f.dpart_f32 = p->dpart_f32;
    f.sym = sym;
    HIP_TRY(p->mark(THCSOX_STAGE_FUSED, true));
    HIP_TRY(sox_fused(mode, f, s));
    HIP_TRY(p->mark(THCSOX_STAGE_FUSED, false));

    HIP_TRY(p->mark(THCSOX_STAGE_BACK, true));
    DReduceArgs d{};
    d.naux = naux; d.vsplit = p->vsplit; d.Dpart = p->Dpart; d.dpart_f32 = p->dpart_f32;
    d.Sthc = Sthc_out ? Sthc_out + (int64_t)k * aa : p->Sthc + (int64_t)b * aa;
    d.s_ld = naux;
    d.amax_gt = p->am_gt() + k; d.amax_gx = p->am_gx() + k; d.amax_gb = p->am_g() + kb;
    d.amax_a = scaled_a ? p->am_a() + k : nullptr;
    d.amax_u = (mode == MODE_F64) ? nullptr : cores.amaxA;
    d.amax_u2 = (mode == MODE_F64) ? nullptr : cores.amaxC;
    d.sym = sym;
    HIP_TRY(dreduce(d, s));
    HIP_TRY(p->mark(THCSOX_STAGE_BACK, false));
  }

  HIP_TRY(p->mark(THCSOX_STAGE_BACK, true));
  const double* St = Sthc_out ? Sthc_out + (int64_t)k0 * aa : p->Sthc;
  TRY(backproject_batch(p, St, aa, Sigma + (int64_t)k0 * nn, nb, beta_out, alpha_out));
  HIP_TRY(p->mark(THCSOX_STAGE_BACK, false));
  return 0;
}

// Gt = X^T G[k] X into the direct-term buffer A and Gbt = X^T G[m-1-k] X into
// buffer B for k0 <= k < k1 (k1 - k0 <= tbd), then Pi = Gt o Gbt^T into buffer C.
int bubble_batch(thcsox_plan_s* p, const double* G, int k0, int k1) {
  const int n = p->n, naux = p->naux, m = p->m, nb = k1 - k0;
  const hipStream_t s = p->stream;
  const int64_t nn = (int64_t)n * n, aa = (int64_t)naux * naux;
  double* bufA = p->dbuf;
  double* bufB = p->dbuf + (int64_t)p->tbd * aa;
  double* bufC = bufB + (int64_t)p->tbd * aa;
  // T = X^T G for the batch (into Gt64, [nb][naux][n]) and Gt = T X; the same
  // for the mirrored points, walking G backwards
  for (int mirror = 0; mirror < 2; ++mirror) {
    Gemm64Args g{};
    g.M = naux; g.N = n; g.K = n; g.batch = nb; g.alpha = 1.0; g.beta = 0.0;
    g.A = p->X; g.a_i = 1; g.a_k = naux; g.a_b = 0;
    g.B = mirror ? G + (int64_t)(m - 1 - k0) * nn : G + (int64_t)k0 * nn;
    g.b_k = n; g.b_j = 1; g.b_b = mirror ? -nn : nn;
    g.C = p->Gt64; g.c_i = n; g.c_j = 1; g.cj_in = n; g.cj_out = 0; g.c_b = (int64_t)naux * n;
    HIP_TRY(gemm64(g, s));
    g.M = naux; g.N = naux; g.K = n;
    g.A = p->Gt64; g.a_i = n; g.a_k = 1; g.a_b = (int64_t)naux * n;
    g.B = p->X; g.b_k = naux; g.b_j = 1; g.b_b = 0;
    g.C = mirror ? bufB : bufA; g.c_i = naux; g.c_j = 1; g.cj_in = naux; g.cj_out = 0; g.c_b = aa;
    HIP_TRY(gemm64(g, s));
  }
  HIP_TRY(bubble_pi(bufA, bufB, bufC, naux, nb, s));
  return 0;
}

// GF2 direct (bubble) term for tau points k0 <= k < k1 (k1 - k0 <= tbd), FP64:
//   Gt = X^T G[k] X, Gbt = X^T G[m-1-k] X, Pi = Gt o Gbt^T, W = V Pi V,
//   Sigma[k] = X (W o Gt) X^T.
int direct_batch(thcsox_plan_s* p, const double* G, double* Sigma, int k0, int k1,
                 bool accumulate) {
  const int n = p->n, naux = p->naux, nb = k1 - k0;
  const hipStream_t s = p->stream;
  const int64_t nn = (int64_t)n * n, aa = (int64_t)naux * naux;
  double* bufA = p->dbuf;                          // Gt
  double* bufB = p->dbuf + (int64_t)p->tbd * aa;   // Gbt, then V Pi
  double* bufC = bufB + (int64_t)p->tbd * aa;      // Pi, then W, then W o Gt
  TRY(bubble_batch(p, G, k0, k1));
  // W = (V Pi) V
  Gemm64Args g{};
  g.M = naux; g.N = naux; g.K = naux; g.batch = nb; g.alpha = 1.0; g.beta = 0.0;
  g.A = p->V; g.a_i = naux; g.a_k = 1; g.a_b = 0;
  g.B = bufC; g.b_k = naux; g.b_j = 1; g.b_b = aa;
  g.C = bufB; g.c_i = naux; g.c_j = 1; g.cj_in = naux; g.cj_out = 0; g.c_b = aa;
  HIP_TRY(gemm64(g, s));
  g.A = bufB; g.a_i = naux; g.a_k = 1; g.a_b = aa;
  g.B = p->V; g.b_k = naux; g.b_j = 1; g.b_b = 0;
  g.C = bufC;
  HIP_TRY(gemm64(g, s));
  HIP_TRY(hadamard64(bufC, bufA, bufC, (int64_t)nb * aa, s));
  return backproject_batch(p, bufC, aa, Sigma + (int64_t)k0 * nn, nb, accumulate ? 1.0 : 0.0);
}

// The direct term's three batch buffers of naux^2 per tau point (also the
// screened exchange's polarization batches), allocated on first use: about
// 1 GB per batch at most, and no more than what the workspace limit leaves
// (alloc refuses one point that does not fit with THCSOX_ENOMEM).
int ensure_direct_buffers(thcsox_plan_s* p) {
  if (p->dbuf != nullptr) return 0;
  const double per_tau = 3.0 * 8.0 * (double)p->naux * p->naux;
  double cap = 1.0e9;
  if (p->limit) cap = std::min(cap, (double)p->limit - (double)p->bytes - 256.0);
  p->tbd = (int)std::max(1.0, std::min((double)p->tb, std::floor(cap / per_tau)));
  return p->alloc(&p->dbuf, (size_t)3 * p->tbd * p->naux * p->naux);
}

// Per-call preparation of G for the exchange contractions: max |G[k]| of every
// tau point (the power-of-two scales) and, under THCSOX_SYM_AUTO, the flags of
// the symmetric-D path.
int prepare_g(thcsox_plan_s* p, const double* G_dev) {
  const hipStream_t s = p->stream;
  const int64_t nn = (int64_t)p->n * p->n;
  HIP_TRY(fill_u64(p->am_g(), p->m, 0ull, s));
  HIP_TRY(absmax64(G_dev, nn, nn, p->m, p->am_g(), s));
  if (p->sym_mode == THCSOX_SYM_AUTO) {
    HIP_TRY(asym64(G_dev, p->n, p->m, p->am_asym(), s));
    HIP_TRY(sym_flags(p->am_asym(), p->am_g(), p->m,
                      p->mode == MODE_F64 ? SYM_RTOL_F64 : SYM_RTOL_MIXED, p->symflag, s));
  }
  return 0;
}

}  // namespace

extern "C" {

const char* thcsox_last_error(void) { return g_last_error.c_str(); }

int thcsox_plan(thcsox_plan_t* out, int n, int naux, int ntau, double beta,
                const double* tau_host, const double* wq_host, const double* X_dev,
                const double* V_dev, int precision, size_t workspace_limit, void* hip_stream) {
  clear_error();
  if (out == nullptr) return fail(THCSOX_EINVAL, "out is NULL");
  *out = nullptr;
  if (n <= 0 || naux <= 0 || ntau <= 0)
    return fail(THCSOX_EINVAL, "n, naux and ntau must be positive");
  if (!(beta > 0.0) || !std::isfinite(beta)) return fail(THCSOX_EINVAL, "beta must be > 0");
  if (precision < THCSOX_FP64 || precision > THCSOX_FP16X2)
    return fail(THCSOX_EINVAL, "unknown precision " + std::to_string(precision));
  {
    // The fused kernels address one tile's rows of U with 32-bit buffer offsets
    // (tile rows x n x ldk elements; their launchers check the same bound).
    // Refuse larger n here, before anything is allocated.
    int TR = 0, TP = 0;
    fused_tile(precision, &TR, &TP);
    auto fits = [&](int64_t nn) {
      const int64_t l = precision == THCSOX_FP16X2 ? (nn + 63) / 64 * 64 : (nn + 31) / 32 * 32;
      // bytes per k of an operand row addressed by one resource: FP64 8; FP32 4;
      // fp16x2 4 (both planes in one c32 row); bf16x3 2 (one resource per plane)
      const int64_t es = precision == THCSOX_FP64 ? 8 : precision == THCSOX_BF16X3 ? 2 : 4;
      // in double: exact near the bound, and no wrap-around for huge n
      return (double)std::max(TR, TP) * (double)nn * (double)l * (double)es <= 2147483647.0;
    };
    if (!fits(n)) {
      int64_t lo = 1, hi = n;   // fits(lo), !fits(hi)
      while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        (fits(mid) ? lo : hi) = mid;
      }
      return fail(THCSOX_EINVAL, "n = " + std::to_string(n) +
                                     " is beyond the 32-bit buffer offsets of the fused "
                                     "kernels in this precision (n <= " + std::to_string(lo) + ")");
    }
  }
  if (tau_host == nullptr || wq_host == nullptr)
    return fail(THCSOX_EINVAL, "tau_host and wq_host are required");
  {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, tau_host) == hipSuccess && a.type == hipMemoryTypeDevice)
      return fail(THCSOX_ENOTDEV, "tau_host must be host memory");
    (void)hipGetLastError();
    if (hipPointerGetAttributes(&a, wq_host) == hipSuccess && a.type == hipMemoryTypeDevice)
      return fail(THCSOX_ENOTDEV, "wq_host must be host memory");
    (void)hipGetLastError();
  }
  for (int k = 0; k < ntau; ++k) {
    if (!(tau_host[k] > 0.0 && tau_host[k] < beta))
      return fail(THCSOX_EINVAL, "tau[" + std::to_string(k) + "] is outside (0, beta)");
    if (k > 0 && !(tau_host[k] > tau_host[k - 1]))
      return fail(THCSOX_EINVAL, "tau grid is not ascending");
    if (std::fabs(tau_host[k] + tau_host[ntau - 1 - k] - beta) > 1e-12 * beta)
      return fail(THCSOX_EINVAL, "tau grid is not mirror symmetric");
    if (!std::isfinite(wq_host[k])) return fail(THCSOX_EINVAL, "non-finite weight");
  }
  TRY(check_dev(X_dev, "X_dev"));
  TRY(check_dev(V_dev, "V_dev"));

  thcsox_plan_s* p = new (std::nothrow) thcsox_plan_s();
  if (!p) return fail(THCSOX_ENOMEM, "host allocation failed");
  auto bail = [&](int rc) { delete p; return rc; };
  p->n = n; p->naux = naux; p->m = ntau; p->beta = beta; p->mode = precision;
  // operand row length: n rounded up to the k step of the matrix-core stages
  // (64 for fp16x2, whose fused kernel takes two 32-wide stages per trip)
  p->ldk = precision == THCSOX_FP16X2 ? (n + 63) / 64 * 64 : (n + 31) / 32 * 32;
  p->np = n_planes(precision);
  p->esize = elem_size(precision);
  p->stream = static_cast<hipStream_t>(hip_stream);
  p->limit = workspace_limit;
  const int64_t ldk = p->ldk;

  {
    // v split: a multiple of the XCD count (each XCD owns whole v ranges),
    // chosen so the last round of workgroups on each XCD is nearly full.
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int nx = fused_xcds();
    const int per_xcd = std::max(1, cus / nx);
    int TR = 64, TP = 64;
    fused_tile(precision, &TR, &TP);
    const long tiles = (long)((naux + TR - 1) / TR) * ((naux + TP - 1) / TP);
    int best = nx;
    double best_eff = -1.0;
    // the fp16x2 and FP32 kernel takes v in pairs and splits the pairs
    const bool pairs = precision == THCSOX_FP16X2 || precision == THCSOX_FP32;
    const int nv = pairs ? (n + 1) / 2 : n;
    for (int vs = nx; vs <= std::max(nx, std::min(8 * nx, nv)); vs += nx) {
      const long wg = tiles * (vs / nx);                 // workgroups per XCD
      const long rounds = (wg + per_xcd - 1) / per_xcd;
      double eff = (double)wg / (double)(rounds * per_xcd);
      eff *= 1.0 - 0.002 * vs;                           // mild preference for long v ranges
      if (eff > best_eff) { best_eff = eff; best = vs; }
    }
    // The reduced-precision kernels keep an FP32 partial sum of D for 8 v and
    // then add it into the partial tile; with v ranges of at most 8 each
    // workgroup writes its tile once, never reads it back, and the tile can be
    // FP32.  Use that split when the partial-D buffer stays small (measured at
    // n = 300, naux = 1800: 2-4 % faster than the balance choice above, full
    // and symmetric paths).
    if (precision != THCSOX_FP64) {
      const int per = pairs ? 4 : 8;   // pairs or v per range
      const int vs8 = ((nv + per - 1) / per + nx - 1) / nx * nx;
      const double dbytes = 4.0 * vs8 * (double)naux * naux;   // FP32 partial tiles
      const bool fits = dbytes <= 2.0e9 &&
                        (workspace_limit == 0 || dbytes <= 0.25 * (double)workspace_limit);
      if (fits && vs8 > best) best = vs8;
    }
    p->vsplit = best;
    // longest v range (ranges are balanced over the XCDs)
    p->vchunk = pairs ? 2 * ((nv + best - 1) / best) : (n + best - 1) / best;
    // ranges of at most 8 v are one FP32 partial sum each: store them as FP32
    p->dpart_f32 = precision != THCSOX_FP64 && p->vchunk <= 8;
  }

  int rc = 0;
  const size_t es = p->esize, np = p->np;
  p->u_plane = (int64_t)naux * n * ldk;
  p->a_plane = (int64_t)n * naux * ldk;
  // the fp16x2 A stage forms two tau points per launch (U read once for both)
  // while their FP32 A arrays take at most 2 GB together
  if (precision == THCSOX_FP16X2 && ntau > 1 && 8.0 * p->a_plane <= 2.0e9) p->a_sets = 2;
  {
    // tau batch of the projections and back-projection: up to 16 points within ~2 GB
    const double per_tau = 8.0 * (2.0 * naux * n + (double)naux * naux + (double)n * naux) +
                           (double)p->np * p->esize * ((2.0 * naux + n) * ldk);
    double cap = 2.0e9;
    if (workspace_limit > 0) {
      // what the plan keeps besides the batch buffers, plus 1 MiB of slack
      // the U build's temporaries (Khatri-Rao chunk, and its FP64 result in the split
      // modes) are allocated last and freed after the build, so they count too
      const double per_q = 8.0 * n * naux;
      const double qb = std::max(1.0, std::min((double)n, std::floor((double)(size_t(256) << 20) / per_q)));
      const double temps = qb * per_q * (precision == THCSOX_FP64 ? 1.0 : 2.0);
      // (X, V and the per-tau scalars in FP64, U, A, the partial tiles)
      const double fixed = 8.0 * ((double)n * naux + (double)naux * naux + 7.0 * ntau + 2.0) +
                           (double)p->np * p->esize * naux * n * ldk +
                           (double)p->np * p->esize * p->a_sets * n * naux * ldk +
                           (p->dpart_f32 ? 4.0 : 8.0) * p->vsplit * (double)naux * naux +
                           temps + (1 << 20);
      cap = std::min(cap, (double)workspace_limit - fixed);
    }
    p->tb = (int)std::max(1.0, std::min({16.0, (double)ntau, std::floor(cap / per_tau)}));
  }
  p->g_plane = (int64_t)p->tb * naux * ldk;
  p->gb_plane = (int64_t)p->tb * n * ldk;
  char* tmp = nullptr;
  if ((rc = p->alloc(&p->X, (size_t)n * naux))) return bail(rc);
  if ((rc = p->alloc(&p->w, (size_t)ntau))) return bail(rc);
  if ((rc = p->alloc(&p->amax, (size_t)1 + 5 * (size_t)ntau))) return bail(rc);
  if ((rc = p->alloc(&p->symflag, (size_t)ntau))) return bail(rc);
  if ((rc = p->alloc(&p->tr, (size_t)ntau))) return bail(rc);
  if ((rc = p->alloc(&p->E, 1))) return bail(rc);
  if ((rc = p->alloc(&tmp, np * es * (size_t)p->u_plane))) return bail(rc);
  p->U = tmp;
  if ((rc = p->alloc(&tmp, np * es * (size_t)p->a_sets * p->a_plane))) return bail(rc);
  p->A = tmp;
  if (precision == THCSOX_FP16X2 && (rc = p->alloc(&p->norm2, (size_t)2 + p->tb)))
    return bail(rc);
  if ((rc = p->alloc(&tmp, np * es * (size_t)p->g_plane))) return bail(rc);
  p->Gt = tmp;
  if ((rc = p->alloc(&tmp, np * es * (size_t)p->g_plane))) return bail(rc);
  p->GX = tmp;
  if ((rc = p->alloc(&tmp, np * es * (size_t)p->gb_plane))) return bail(rc);
  p->Gb = tmp;
  if ((rc = p->alloc(&p->Gt64, (size_t)p->tb * naux * n))) return bail(rc);
  if ((rc = p->alloc(&p->GX64, (size_t)p->tb * naux * n))) return bail(rc);
  {
    const size_t dn = (size_t)p->vsplit * naux * naux;
    if ((rc = p->alloc(&p->Dpart, p->dpart_f32 ? (dn + 1) / 2 : dn))) return bail(rc);
  }
  if ((rc = p->alloc(&p->Sthc, (size_t)p->tb * naux * naux))) return bail(rc);
  if ((rc = p->alloc(&p->T1, (size_t)p->tb * n * naux))) return bail(rc);

  const hipStream_t s = p->stream;
  auto hip_bail = [&](hipError_t e, const char* what) {
    delete p;
    return fail(THCSOX_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipMemcpyAsync(p->X, X_dev, sizeof(double) * n * naux, hipMemcpyDeviceToDevice, s)))
    return hip_bail(e, "copy X");
  if ((e = hipMemcpyAsync(p->w, wq_host, sizeof(double) * ntau, hipMemcpyHostToDevice, s)))
    return hip_bail(e, "copy weights");
  // zero the operand pads once (stages only ever write the first n of ldk columns)
  if ((e = hipMemsetAsync(p->U, 0, np * es * (size_t)p->u_plane, s))) return hip_bail(e, "zero U");
  if (p->A && (e = hipMemsetAsync(p->A, 0, np * es * (size_t)p->a_sets * p->a_plane, s)))
    return hip_bail(e, "zero A");
  if ((e = hipMemsetAsync(p->symflag, 0, sizeof(int) * (size_t)ntau, s)))
    return hip_bail(e, "zero flags");
  if ((rc = p->alloc(&p->V, (size_t)naux * naux))) return bail(rc);
  if ((e = hipMemcpyAsync(p->V, V_dev, sizeof(double) * (size_t)naux * naux,
                          hipMemcpyDeviceToDevice, s)))
    return hip_bail(e, "copy V");
  if ((rc = build_u(p, V_dev, p->U, p->amax, p->norm2))) return bail(rc);
  if ((e = hipStreamSynchronize(s))) return hip_bail(e, "plan synchronise");
  *out = p;
  return 0;
}

int thcsox_sigma_sox(thcsox_plan_t p, const double* G_dev, double* Sigma_dev,
                     double* Sigma_thc_dev, int k_begin, int k_end) {
  clear_error();
  if (p == nullptr) return fail(THCSOX_EINVAL, "plan is NULL");
  if (k_begin < 0 || k_end > p->m || k_begin >= k_end)
    return fail(THCSOX_EINVAL, "need 0 <= k_begin < k_end <= ntau");
  TRY(check_dev(G_dev, "G_dev"));
  TRY(check_dev(Sigma_dev, "Sigma_dev"));
  if (Sigma_thc_dev) TRY(check_dev(Sigma_thc_dev, "Sigma_thc_dev"));
  const size_t gbytes = sizeof(double) * (size_t)p->m * p->n * p->n;
  const char* g0 = reinterpret_cast<const char*>(G_dev);
  const char* s0 = reinterpret_cast<const char*>(Sigma_dev);
  if (s0 < g0 + gbytes && g0 < s0 + gbytes) return fail(THCSOX_EINVAL, "Sigma aliases G");
  TRY(prepare_g(p, G_dev));
  for (int k = k_begin; k < k_end; k += p->tb)
    TRY(sigma_batch(p, G_dev, Sigma_dev, Sigma_thc_dev, k, std::min(k_end, k + p->tb),
                    Cores{p->U, p->amax, p->U, p->amax, p->norm2}));
  return 0;
}

int thcsox_backproject(thcsox_plan_t p, const double* Sigma_thc_dev, double* Sigma_dev,
                       int k_begin, int k_end) {
  clear_error();
  if (p == nullptr) return fail(THCSOX_EINVAL, "plan is NULL");
  if (k_begin < 0 || k_end > p->m || k_begin >= k_end)
    return fail(THCSOX_EINVAL, "need 0 <= k_begin < k_end <= ntau");
  TRY(check_dev(Sigma_thc_dev, "Sigma_thc_dev"));
  TRY(check_dev(Sigma_dev, "Sigma_dev"));
  const int64_t nn = (int64_t)p->n * p->n, aa = (int64_t)p->naux * p->naux;
  for (int k = k_begin; k < k_end; k += p->tb)
    TRY(backproject_batch(p, Sigma_thc_dev + k * aa, aa, Sigma_dev + k * nn,
                          std::min(k_end, k + p->tb) - k));
  return 0;
}

int thcsox_sigma_direct(thcsox_plan_t p, const double* G_dev, double* Sigma_dev, int k_begin,
                        int k_end, int accumulate) {
  clear_error();
  if (p == nullptr) return fail(THCSOX_EINVAL, "plan is NULL");
  if (k_begin < 0 || k_end > p->m || k_begin >= k_end)
    return fail(THCSOX_EINVAL, "need 0 <= k_begin < k_end <= ntau");
  TRY(check_dev(G_dev, "G_dev"));
  TRY(check_dev(Sigma_dev, "Sigma_dev"));
  const size_t gbytes = sizeof(double) * (size_t)p->m * p->n * p->n;
  const char* g0 = reinterpret_cast<const char*>(G_dev);
  const char* s0 = reinterpret_cast<const char*>(Sigma_dev);
  if (s0 < g0 + gbytes && g0 < s0 + gbytes) return fail(THCSOX_EINVAL, "Sigma aliases G");
  TRY(ensure_direct_buffers(p));
  for (int k = k_begin; k < k_end; k += p->tbd)
    TRY(direct_batch(p, G_dev, Sigma_dev, k, std::min(k_end, k + p->tbd), accumulate != 0));
  return 0;
}

int thcsox_static_screening(thcsox_plan_t p, const double* G_dev, double* W_dev) {
  clear_error();
  if (p == nullptr) return fail(THCSOX_EINVAL, "plan is NULL");
  TRY(check_dev(G_dev, "G_dev"));
  TRY(check_dev(W_dev, "W_dev"));
  const int naux = p->naux, m = p->m;
  if (naux > 9216) return fail(THCSOX_EINVAL, "naux > 9216 is beyond the screening solve");
  const int64_t aa = (int64_t)naux * naux;
  const hipStream_t s = p->stream;
  TRY(ensure_direct_buffers(p));
  if (p->Pi0 == nullptr) {
    TRY(p->alloc(&p->Pi0, (size_t)aa));
    TRY(p->alloc(&p->Mscr, (size_t)aa));
    TRY(p->alloc(&p->Minv, (size_t)aa));
    TRY(p->alloc(&p->Am, (size_t)aa));
    TRY(p->alloc(&p->gj, (size_t)2 * naux + 1));
  }
  // Pi0 = sum_k w_k Pi(tau_k), batch by batch, in the order of k
  const double* bufC = p->dbuf + 2 * (int64_t)p->tbd * aa;
  for (int k0 = 0; k0 < m; k0 += p->tbd) {
    const int k1 = std::min(m, k0 + p->tbd);
    TRY(bubble_batch(p, G_dev, k0, k1));
    HIP_TRY(weighted_block_sum(bufC, p->w + k0, k1 - k0, aa, p->Pi0, k0 > 0 ? 1 : 0, s));
  }
  // W = (1 + V Pi0)^-1 V
  Gemm64Args g{};
  g.M = naux; g.N = naux; g.K = naux; g.batch = 1; g.alpha = 1.0; g.beta = 0.0;
  g.A = p->V; g.a_i = naux; g.a_k = 1;
  g.B = p->Pi0; g.b_k = naux; g.b_j = 1;
  g.C = p->Mscr; g.c_i = naux; g.c_j = 1; g.cj_in = naux; g.cj_out = 0;
  HIP_TRY(gemm64(g, s));
  HIP_TRY(add_identity(p->Mscr, naux, s));
  int* piv = p->gj;
  int* perm = p->gj + naux;
  int* flag = p->gj + 2 * naux;
  HIP_TRY(gj_inverse_real(p->Mscr, naux, p->Minv, p->Am, piv, perm, flag, s));
  g.A = p->Minv; g.B = p->V; g.C = W_dev;
  HIP_TRY(gemm64(g, s));
  int hflag = 0;
  HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hflag) return fail(THCSOX_ENONFINITE, "1 + V Pi0 is singular");
  return 0;
}

int thcsox_sigma_screened(thcsox_plan_t p, const double* G_dev, const double* W_dev, int kind,
                          double* Sigma_dev, int k_begin, int k_end) {
  clear_error();
  if (p == nullptr) return fail(THCSOX_EINVAL, "plan is NULL");
  if (kind != THCSOX_SOSEX && kind != THCSOX_G3W2)
    return fail(THCSOX_EINVAL, "unknown screened-exchange kind " + std::to_string(kind));
  if (k_begin < 0 || k_end > p->m || k_begin >= k_end)
    return fail(THCSOX_EINVAL, "need 0 <= k_begin < k_end <= ntau");
  TRY(check_dev(G_dev, "G_dev"));
  TRY(check_dev(W_dev, "W_dev"));
  TRY(check_dev(Sigma_dev, "Sigma_dev"));
  const size_t gbytes = sizeof(double) * (size_t)p->m * p->n * p->n;
  const char* g0 = reinterpret_cast<const char*>(G_dev);
  const char* s0 = reinterpret_cast<const char*>(Sigma_dev);
  if (s0 < g0 + gbytes && g0 < s0 + gbytes) return fail(THCSOX_EINVAL, "Sigma aliases G");
  const hipStream_t s = p->stream;
  if (p->Uw == nullptr) {
    char* tmp = nullptr;
    TRY(p->alloc(&tmp, (size_t)p->np * p->esize * (size_t)p->u_plane));
    p->Uw = tmp;
    TRY(p->alloc(&p->amax_w, 1));
    // the operand pads stay zero (every build writes only the first n of ldk columns)
    HIP_TRY(hipMemsetAsync(p->Uw, 0, (size_t)p->np * p->esize * (size_t)p->u_plane, s));
  }
  TRY(build_u(p, W_dev, p->Uw, p->amax_w, p->norm2 ? p->norm2 + 1 : nullptr));
  TRY(prepare_g(p, G_dev));
  const Cores vw{p->U, p->amax, p->Uw, p->amax_w, p->norm2};
  const Cores wv{p->Uw, p->amax_w, p->U, p->amax, p->norm2 ? p->norm2 + 1 : nullptr};
  const Cores ww{p->Uw, p->amax_w, p->Uw, p->amax_w, p->norm2 ? p->norm2 + 1 : nullptr};
  for (int k = k_begin; k < k_end; k += p->tb) {
    const int k1 = std::min(k_end, k + p->tb);
    if (kind == THCSOX_SOSEX) {
      TRY(sigma_batch(p, G_dev, Sigma_dev, nullptr, k, k1, vw, 0.5, 0.0));
      TRY(sigma_batch(p, G_dev, Sigma_dev, nullptr, k, k1, wv, 0.5, 1.0));
    } else {
      TRY(sigma_batch(p, G_dev, Sigma_dev, nullptr, k, k1, ww));
    }
  }
  return 0;
}

int thcsox_energy(thcsox_plan_t p, const double* G_dev, const double* Sigma_dev,
                  double* E_host) {
  clear_error();
  if (p == nullptr) return fail(THCSOX_EINVAL, "plan is NULL");
  if (E_host == nullptr) return fail(THCSOX_EINVAL, "E_host is NULL");
  TRY(check_dev(G_dev, "G_dev"));
  TRY(check_dev(Sigma_dev, "Sigma_dev"));
  const hipStream_t s = p->stream;
  HIP_TRY(energy_partials(G_dev, Sigma_dev, p->n, p->m, p->tr, s));
  HIP_TRY(energy_final(p->tr, p->w, p->m, p->E, s));
  HIP_TRY(hipMemcpyAsync(E_host, p->E, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

int thcsox_energy_noalloc(const double* G_dev, const double* Sigma_dev, const double* w_dev,
                          int n, int ntau, double* E_dev, void* hip_stream) {
  clear_error();
  if (n <= 0 || ntau <= 0) return fail(THCSOX_EINVAL, "n and ntau must be positive");
  if (ntau > NOALLOC_MAX_NTAU)
    return fail(THCSOX_EINVAL, "ntau = " + std::to_string(ntau) +
                                   " exceeds the allocation-free scratch (at most " +
                                   std::to_string(NOALLOC_MAX_NTAU) + " tau points)");
  TRY(check_dev(G_dev, "G_dev"));
  TRY(check_dev(Sigma_dev, "Sigma_dev"));
  TRY(check_dev(w_dev, "w_dev"));
  TRY(check_dev(E_dev, "E_dev"));
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (s != nullptr) {
    // the scratch address belongs to the current device; so must the stream
    int cur = -1;
    hipDevice_t sd = -1;
    HIP_TRY(hipGetDevice(&cur));
    HIP_TRY(hipStreamGetDevice(s, &sd));
    if (sd != cur) return fail(THCSOX_EINVAL, "hip_stream belongs to another device");
  }
  double* tr = nullptr;
  TRY(scratch_on_current_device(&tr));
  // every tr[k], k < ntau, is written before it is read: nothing to clear
  HIP_TRY(energy_partials(G_dev, Sigma_dev, n, ntau, tr, s));
  HIP_TRY(energy_final(tr, w_dev, ntau, E_dev, s));
  return 0;
}

int thcsox_energy_basis(thcsox_plan_t p, const double* G_dev, const double* Sigma_dev,
                        const double* coef_host, const double* sign_host, double* E_host) {
  clear_error();
  if (p == nullptr) return fail(THCSOX_EINVAL, "plan is NULL");
  if (E_host == nullptr || coef_host == nullptr || sign_host == nullptr)
    return fail(THCSOX_EINVAL, "NULL argument");
  TRY(check_dev(G_dev, "G_dev"));
  TRY(check_dev(Sigma_dev, "Sigma_dev"));
  const int m = p->m, n = p->n;
  const int64_t nn = (int64_t)n * n, mm = (int64_t)m * m;
  for (int l = 0; l < m; ++l)
    if (sign_host[l] != 1.0 && sign_host[l] != -1.0) return fail(THCSOX_EINVAL, "sign must be +-1");
  for (int64_t i = 0; i < mm; ++i)
    if (!std::isfinite(coef_host[i])) return fail(THCSOX_EINVAL, "coef has a non-finite entry");
  // allocated on first use; a failed allocation leaves the others for the next call
  if (p->ebuf == nullptr) TRY(p->alloc(&p->ebuf, (size_t)(2 * m * nn)));
  if (p->ecoef == nullptr) TRY(p->alloc(&p->ecoef, (size_t)(2 * mm)));
  if (p->esign == nullptr) TRY(p->alloc(&p->esign, (size_t)m));
  // g = C G with the rows of C reversed, sigma = C Sigma: the trace kernel pairs
  // index k of its first operand with index m-1-k of the second, so it meets
  // g_l with sigma_l
  std::vector<double> c2;
  try {   // no exception may cross the C interface
    c2.resize((size_t)(2 * mm));
  } catch (const std::bad_alloc&) {
    return fail(THCSOX_ENOMEM, "host allocation failed");
  }
  for (int l = 0; l < m; ++l)
    for (int k = 0; k < m; ++k) {
      c2[(size_t)(m - 1 - l) * m + k] = coef_host[(size_t)l * m + k];
      c2[(size_t)mm + (size_t)l * m + k] = coef_host[(size_t)l * m + k];
    }
  const hipStream_t s = p->stream;
  HIP_TRY(hipMemcpyAsync(p->ecoef, c2.data(), sizeof(double) * c2.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(p->esign, sign_host, sizeof(double) * m, hipMemcpyHostToDevice, s));
  for (int t = 0; t < 2; ++t) {
    Gemm64Args g{};
    g.M = m; g.N = (int)nn; g.K = m; g.batch = 1; g.alpha = 1.0; g.beta = 0.0;
    g.A = p->ecoef + t * mm; g.a_i = m; g.a_k = 1;
    g.B = t == 0 ? G_dev : Sigma_dev; g.b_k = nn; g.b_j = 1;
    g.C = p->ebuf + t * m * nn; g.c_i = nn; g.c_j = 1; g.cj_in = nn; g.cj_out = 0;
    HIP_TRY(gemm64(g, s));
  }
  HIP_TRY(energy_partials(p->ebuf, p->ebuf + m * nn, n, m, p->tr, s));
  HIP_TRY(energy_final(p->tr, p->esign, m, p->E, s));
  HIP_TRY(hipMemcpyAsync(E_host, p->E, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return 0;
}

int thcsox_destroy(thcsox_plan_t p) {
  if (p == nullptr) return 0;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  delete p;
  return 0;
}

int thcsox_plan_info(thcsox_plan_t p, thcsox_plan_info_t* info) {
  clear_error();
  if (p == nullptr || info == nullptr) return fail(THCSOX_EINVAL, "NULL argument");
  const double n = p->n, na = p->naux;
  info->n = p->n; info->naux = p->naux; info->ntau = p->m; info->precision = p->mode;
  info->tau_batch = p->tb;
  info->bytes = p->bytes;
  info->mac_per_tau = 2 * na * na * n * n + na * n * n * n + 2 * na * na * n + 3 * na * n * n;
  info->fused_mac_per_tau = 2 * na * na * n * n;
  info->fused_bytes_per_tau =
      (double)p->np * p->esize * (2 * na * n * n + 2 * na * n);
  info->vsplit = p->vsplit;
  info->vrange = p->vchunk;
  info->partial_f32 = p->dpart_f32 ? 1 : 0;
  return 0;
}

int thcsox_set_symmetry(thcsox_plan_t p, int mode) {
  clear_error();
  if (p == nullptr) return fail(THCSOX_EINVAL, "plan is NULL");
  if (mode != THCSOX_SYM_AUTO && mode != THCSOX_SYM_OFF)
    return fail(THCSOX_EINVAL, "unknown symmetry mode " + std::to_string(mode));
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->sym_mode = mode;
  return 0;
}

int thcsox_symmetric_flags(thcsox_plan_t p, int* flags_host) {
  clear_error();
  if (p == nullptr || flags_host == nullptr) return fail(THCSOX_EINVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (p->sym_mode != THCSOX_SYM_AUTO) {
    for (int k = 0; k < p->m; ++k) flags_host[k] = 0;
    return 0;
  }
  HIP_TRY(hipMemcpy(flags_host, p->symflag, sizeof(int) * p->m, hipMemcpyDeviceToHost));
  return 0;
}

int thcsox_profile(thcsox_plan_t p, int enable) {
  clear_error();
  if (p == nullptr) return fail(THCSOX_EINVAL, "plan is NULL");
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->profiling = enable != 0;
  for (auto& t : p->timers) t.used = 0;
  return 0;
}

int thcsox_stage_times(thcsox_plan_t p, double* ms, int* launches) {
  clear_error();
  if (p == nullptr || ms == nullptr || launches == nullptr)
    return fail(THCSOX_EINVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(p->stream));
  for (int st = 0; st < THCSOX_NSTAGES; ++st) {
    auto& t = p->timers[st];
    double tot = 0.0;
    for (size_t i = 0; i < t.used; ++i) {
      float e = 0.f;
      HIP_TRY(hipEventElapsedTime(&e, t.start[i], t.stop[i]));
      tot += e;
    }
    ms[st] = tot;
    launches[st] = (int)t.used;
    t.used = 0;
  }
  return 0;
}

}  // extern "C"
