// Device kernels of libthcsox for gfx950.  Host launchers are declared in
// kernels.hpp; the C interface that sequences them is in thcsox.hip.
#include "kernels.hpp"
#include "mfma.hpp"
#include "reduce.hpp"

namespace thcsox {

namespace {

constexpr int NT = 256;   // threads per workgroup (4 wavefronts of 64)

__device__ __forceinline__ double pow2_scale(const unsigned long long* amax) {
  if (amax == nullptr) return 1.0;
  unsigned long long b = *amax;
  if (b == 0ull) return 1.0;
  double x = __longlong_as_double((long long)b);
  if (!(x < 1e300)) return 1.0;   // inf / nan: leave unscaled, the result shows it
  return ldexp(1.0, -ilogb(x));
}

// ---------------------------------------------------------------------------
// Strided FP64 GEMM (projections, back-projection, U precontraction, Dyson
// transforms): 64 x 64 tiles of C, k steps of 32, four waves of 32 x 32 on the
// f64 matrix cores.  The next k step is loaded into registers while the current
// one is multiplied out of LDS.  Operands are read in pairs of doubles (16-byte
// loads) along their contiguous dimension: AM = 0 when A is contiguous in k
// (a_k == 1), 1 when contiguous in i (a_i == 1); BM = 0 when B is contiguous in j
// (b_j == 1), 1 when contiguous in k (b_k == 1).  VEC is false when a stride or
// base is odd (then the pairs are two 8-byte loads).
// ---------------------------------------------------------------------------
constexpr int G64_BK = 32, G64_LD = G64_BK + 1;
typedef double d2 __attribute__((ext_vector_type(2)));

template <bool VEC>
__device__ __forceinline__ d2 g64_pair(const double* p, int x, int lim) {
  // elements x, x + 1 along the contiguous dimension (zero past lim)
  if (VEC && x + 1 < lim) {
    const double2 v = *reinterpret_cast<const double2*>(p + x);
    return d2{v.x, v.y};
  }
  return d2{x < lim ? p[x] : 0.0, x + 1 < lim ? p[x + 1] : 0.0};
}

template <int AM, int BM, bool VEC>
__global__ __launch_bounds__(NT) void gemm64_kernel(Gemm64Args g) {
  __shared__ double sA[64 * G64_LD];   // [i][k]
  __shared__ double sB[64 * G64_LD];   // [j][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int64_t b = blockIdx.z;
  const double* A = g.A + b * g.a_b;
  const double* B = g.B + b * g.b_b;
  d4 acc[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = d4{0.0, 0.0, 0.0, 0.0};

  // 1024 pairs per operand and k step, four per thread
  d2 ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + NT * t;
      if (AM == 0) {   // row i, k pair
        const int i = e >> 4, k = 2 * (e & 15), gi = i0 + i;
        ra[t] = gi < g.M ? g64_pair<VEC>(A + (int64_t)gi * g.a_i, k0 + k, g.K) : d2{0.0, 0.0};
      } else {         // column k, i pair
        const int k = e >> 5, i = 2 * (e & 31), gk = k0 + k;
        ra[t] = gk < g.K ? g64_pair<VEC>(A + (int64_t)gk * g.a_k, i0 + i, g.M) : d2{0.0, 0.0};
      }
      if (BM == 0) {   // row k, j pair
        const int k = e >> 5, j = 2 * (e & 31), gk = k0 + k;
        rb[t] = gk < g.K ? g64_pair<VEC>(B + (int64_t)gk * g.b_k, j0 + j, g.N) : d2{0.0, 0.0};
      } else {         // column j, k pair
        const int j = e >> 4, k = 2 * (e & 15), gj = j0 + j;
        rb[t] = gj < g.N ? g64_pair<VEC>(B + (int64_t)gj * g.b_j, k0 + k, g.K) : d2{0.0, 0.0};
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + NT * t;
      if (AM == 0) {
        const int i = e >> 4, k = 2 * (e & 15);
        sA[i * G64_LD + k] = ra[t][0];
        sA[i * G64_LD + k + 1] = ra[t][1];
      } else {
        const int k = e >> 5, i = 2 * (e & 31);
        sA[i * G64_LD + k] = ra[t][0];
        sA[(i + 1) * G64_LD + k] = ra[t][1];
      }
      if (BM == 0) {
        const int k = e >> 5, j = 2 * (e & 31);
        sB[j * G64_LD + k] = rb[t][0];
        sB[(j + 1) * G64_LD + k] = rb[t][1];
      } else {
        const int j = e >> 4, k = 2 * (e & 15);
        sB[j * G64_LD + k] = rb[t][0];
        sB[j * G64_LD + k + 1] = rb[t][1];
      }
    }
  };

  load(0);
  for (int k0 = 0; k0 < g.K; k0 += G64_BK) {
    store();
    __syncthreads();
    if (k0 + G64_BK < g.K) load(k0 + G64_BK);   // in flight while this step is multiplied
#pragma unroll
    for (int kk = 0; kk < G64_BK; kk += 4) {
      double a[2], bb[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = sA[(32 * wr + 16 * t + (lane & 15)) * G64_LD + kk + (lane >> 4)];
        bb[t] = sB[(32 * wc + 16 * t + (lane & 15)) * G64_LD + kk + (lane >> 4)];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = mfma1(a[ti], bb[tj], acc[ti][tj]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 32 * wr + 16 * ti + out_row<MODE_F64>(lane, r);
        const int j = j0 + 32 * wc + 16 * tj + (lane & 15);
        if (i < g.M && j < g.N) {
          const int64_t idx = b * g.c_b + (int64_t)i * g.c_i + ((int64_t)j / g.cj_in) * g.cj_out +
                              ((int64_t)j % g.cj_in) * g.c_j;
          double v = g.alpha * acc[ti][tj][r];
          if (g.beta != 0.0) v += g.beta * g.C[idx];
          g.C[idx] = v;
        }
      }
}

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(NT) void split_kernel(SplitArgs a) {
  using T = typename ModeT<M>::T;
  constexpr int NP = ModeT<M>::NP;
  const int64_t row = blockIdx.x;
  const int64_t r1 = row / a.rows2, r2 = row % a.rows2;
  const double sc = pow2_scale(a.amax ? a.amax + r2 * a.amax_s2 : nullptr);
  T* dst = static_cast<T*>(a.dst);
  const int64_t so = r1 * a.s1 + r2 * a.s2;
  const int64_t dof = r1 * a.d1 + r2 * a.d2;
  for (int c = threadIdx.x; c < a.ldk; c += NT) {
    double x = 0.0;
    if (c < a.cols) {
      x = a.src_f32 ? (double)static_cast<const float*>(a.src)[so + (int64_t)c * a.sc]
                    : static_cast<const double*>(a.src)[so + (int64_t)c * a.sc];
      x *= sc;
    }
    T o[NP];
    Split<M>::run(x, o);
    if (a.c32) {   // planes interleaved per 32-wide chunk
#pragma unroll
      for (int p = 0; p < NP; ++p) dst[dof + (c >> 5) * 64 + 32 * p + (c & 31)] = o[p];
    } else {
#pragma unroll
      for (int p = 0; p < NP; ++p) dst[p * a.d_plane + dof + c] = o[p];
    }
  }
}

// out = max over rows r < rows of sum_{c < len} x[r ld + c]^2 (max-reduced, bits)
__global__ __launch_bounds__(NT) void rownorm2_kernel(const double* x, int64_t rows, int len,
                                                      int64_t ld, unsigned long long* out) {
  double m = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x; r < rows; r += (int64_t)gridDim.x * NT) {
    const double* xr = x + r * ld;
    double s = 0.0;
    for (int c = 0; c < len; ++c) s = fma(xr[c], xr[c], s);
    m = fmax(m, s);
  }
  block_atomic_max<NT / 64>(m, out);
}

// out[b] = max over columns v < n of sum_{s < n} G_b[s n + v]^2, G_b = G + b stride
__global__ __launch_bounds__(NT) void colnorm2_kernel(const double* G, int n, int64_t stride,
                                                      unsigned long long* out) {
  const double* g = G + (int64_t)blockIdx.x * stride;
  double m = 0.0;
  for (int v = threadIdx.x; v < n; v += NT) {
    double s = 0.0;
    for (int r = 0; r < n; ++r) s = fma(g[(int64_t)r * n + v], g[(int64_t)r * n + v], s);
    m = fmax(m, s);
  }
  block_atomic_max<NT / 64>(m, out + blockIdx.x);
}

// amax_a[b] = bound_b * 2^-14, bound_b = (1 + 2^-10) |U row|max su |Gb row|max(b) sg(b):
// by Cauchy-Schwarz |A| <= bound_b for A formed from the scaled planes.
__global__ void ascale_kernel(const unsigned long long* unorm2, const unsigned long long* amax_u,
                              const unsigned long long* gnorm2, const unsigned long long* amax_gb,
                              int64_t gb_stride, int nb, unsigned long long* amax_a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double un = sqrt(__longlong_as_double((long long)*unorm2));
  const double gn = sqrt(__longlong_as_double((long long)gnorm2[b]));
  const double bound = (1.0 + 0x1p-10) * un * pow2_scale(amax_u) * gn *
                       pow2_scale(amax_gb + (int64_t)b * gb_stride);
  amax_a[b] = (unsigned long long)__double_as_longlong(bound * 0x1p-14);
}

__global__ __launch_bounds__(NT) void absmax_kernel(const double* x, int64_t len, int64_t stride,
                                                    unsigned long long* amax) {
  const int64_t b = blockIdx.y;
  const double* xb = x + b * stride;
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < len; i += (int64_t)gridDim.x * NT)
    m = fmax(m, fabs(xb[i]));
  block_atomic_max<NT / 64>(m, amax + b);
}

__global__ void fill_u64_kernel(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// One workgroup per 32 x 32 tile of Sthc: sum the partial D tiles over z and
// scale.  With the symmetric path only the tiles on and above the diagonal are
// read: each writes itself and (through LDS) its transpose below the diagonal,
// and inside a diagonal tile the entries with R > P come from the mirrored
// position.
constexpr int DT = 32;          // reduction tile edge
constexpr int DRP = NT / DT;    // rows per pass
constexpr int DEL = DT / DRP;   // elements per thread
__device__ __forceinline__ void add4(const float* p, double* acc) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  acc[0] += v.x; acc[1] += v.y; acc[2] += v.z; acc[3] += v.w;
}
__device__ __forceinline__ void add4(const double* p, double* acc) {
  const double2 v0 = *reinterpret_cast<const double2*>(p);
  const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
  acc[0] += v0.x; acc[1] += v0.y; acc[2] += v1.x; acc[3] += v1.y;
}

template <typename T>
__global__ __launch_bounds__(NT) void dreduce_kernel(DReduceArgs a) {
  __shared__ double t[DT][DT + 1];
  const double f = pow2_scale(a.amax_gt) * pow2_scale(a.amax_gx) * pow2_scale(a.amax_gb) *
                   pow2_scale(a.amax_a) * pow2_scale(a.amax_u) *
                   pow2_scale(a.amax_u2 != nullptr ? a.amax_u2 : a.amax_u);
  const double inv = 1.0 / f;   // exact: a power of two
  const int64_t nn = (int64_t)a.naux * a.naux;
  const bool sym = a.sym != nullptr && *a.sym != 0;
  const int nt = (a.naux + DT - 1) / DT;
  const int rb = blockIdx.x / nt, pb = blockIdx.x % nt;
  // symmetric D: the tiles below the diagonal are written by their transposes
  if (sym && rb > pb) return;
  // sum over z: thread = (row ar, four consecutive columns ac..ac+3), 16-byte
  // loads when the row length allows
  const int ar = threadIdx.x / (DT / 4), ac = 4 * (threadIdx.x % (DT / 4));
  const int gr = rb * DT + ar, gc = pb * DT + ac;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (gr < a.naux) {
    const T* D0 = reinterpret_cast<const T*>(a.Dpart) + (int64_t)gr * a.naux + gc;
    if (a.naux % 4 == 0 && gc + 3 < a.naux) {
#pragma unroll 4
      for (int z = 0; z < a.vsplit; ++z) add4(D0 + z * nn, acc);
    } else {
      for (int z = 0; z < a.vsplit; ++z)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (gc + e < a.naux) acc[e] += (double)D0[z * nn + e];
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) t[ar][ac + e] = acc[e];
  __syncthreads();
  const int col = threadIdx.x % DT, row0 = threadIdx.x / DT;
#pragma unroll
  for (int i = 0; i < DEL; ++i) {
    const int lr = row0 + DRP * i, lc = col;
    // element (R, P) of tile (rb, pb); on a symmetric diagonal tile the lower
    // half comes from the upper
    const int R = rb * DT + lr, P = pb * DT + lc;
    if (R < a.naux && P < a.naux) {
      const double v = (sym && rb == pb && R > P) ? t[lc][lr] : t[lr][lc];
      a.Sthc[(int64_t)R * a.s_ld + P] = -inv * v;
    }
    // symmetric, off the diagonal: element (R2, P2) of the transposed tile (pb, rb)
    if (sym && rb < pb) {
      const int R2 = pb * DT + lr, P2 = rb * DT + lc;
      if (R2 < a.naux && P2 < a.naux) a.Sthc[(int64_t)R2 * a.s_ld + P2] = -inv * t[lc][lr];
    }
  }
}

// max |G[k][i][j] - G[k][j][i]| over j > i; a row of workgroups per k strides over G[k].
__global__ __launch_bounds__(NT) void asym_kernel(const double* G, int n,
                                                  unsigned long long* asym) {
  const int k = blockIdx.y;
  const double* g = G + (int64_t)k * n * n;
  double m = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.x * NT) {
    const int i = (int)(e / n), j = (int)(e % n);
    if (j > i) m = fmax(m, fabs(g[(int64_t)i * n + j] - g[(int64_t)j * n + i]));
  }
  block_atomic_max<NT / 64>(m, asym + k);
}

__global__ void sym_flags_kernel(const unsigned long long* asym, const unsigned long long* amax,
                                 int m, double rtol, int* flag) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  // the reference magnitude is the largest |G| on the whole grid: Sigma's error
  // is measured against its largest element, which comes from the largest G
  double gmax = 0.0;
  for (int j = 0; j < m; ++j) gmax = fmax(gmax, __longlong_as_double((long long)amax[j]));
  auto ok = [&](int j) { return __longlong_as_double((long long)asym[j]) <= rtol * gmax; };
  flag[k] = (ok(k) && ok(m - 1 - k)) ? 1 : 0;
}

__global__ __launch_bounds__(NT) void khatri_rao_kernel(const double* X, int n, int naux, int q0,
                                                        double* KR) {
  const int64_t row = blockIdx.x;          // (q - q0) * n + s
  const int q = q0 + (int)(row / n), s = (int)(row % n);
  for (int Q = threadIdx.x; Q < naux; Q += NT)
    KR[row * naux + Q] = X[(int64_t)q * naux + Q] * X[(int64_t)s * naux + Q];
}

__global__ __launch_bounds__(NT) void energy_partials_kernel(const double* G, const double* S,
                                                             int n, int m, double* tr) {
  __shared__ double red[NT];
  const int k = blockIdx.x;
  const double* Gb = G + (int64_t)(m - 1 - k) * n * n;
  const double* Sk = S + (int64_t)k * n * n;
  double acc = 0.0;
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = threadIdx.x; e < nn; e += NT) {
    const int64_t p = e / n, q = e % n;
    acc = fma(Gb[q * n + p], Sk[e], acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) tr[k] = red[0];
}

__global__ void energy_final_kernel(const double* tr, const double* w, int m, double* E) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < m; ++k) s = fma(w[k], tr[k], s);
    *E = -0.5 * s;
  }
}

__global__ __launch_bounds__(NT) void weighted_block_sum_kernel(const double* __restrict__ Pi,
                                                                const double* __restrict__ w,
                                                                int nb, int64_t len,
                                                                double* __restrict__ Pi0,
                                                                int accumulate) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < len; e += (int64_t)gridDim.x * NT) {
    double acc = accumulate ? Pi0[e] : 0.0;
    for (int b = 0; b < nb; ++b) acc = fma(w[b], Pi[(int64_t)b * len + e], acc);
    Pi0[e] = acc;
  }
}

__global__ __launch_bounds__(NT) void add_identity_kernel(double* A, int n) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < n) A[(int64_t)i * n + i] += 1.0;
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

hipError_t weighted_block_sum(const double* Pi, const double* w, int nb, int64_t len,
                              double* Pi0, int accumulate, hipStream_t s) {
  if (len <= 0) return hipSuccess;
  const int64_t b = (len + NT - 1) / NT;
  weighted_block_sum_kernel<<<(unsigned)(b > 4096 ? 4096 : b), NT, 0, s>>>(Pi, w, nb, len, Pi0,
                                                                          accumulate);
  return hipGetLastError();
}

hipError_t add_identity(double* A, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  add_identity_kernel<<<cdiv(n, NT), NT, 0, s>>>(A, n);
  return hipGetLastError();
}

hipError_t gemm64(const Gemm64Args& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (g.K <= 0) return hipErrorInvalidValue;
  // the contiguous dimension of each operand
  int am, bm;
  if (g.a_k == 1) am = 0;
  else if (g.a_i == 1) am = 1;
  else return hipErrorInvalidValue;
  if (g.b_j == 1) bm = 0;
  else if (g.b_k == 1) bm = 1;
  else return hipErrorInvalidValue;
  // 16-byte loads need even strides and 16-byte aligned bases (tile starts are even)
  auto even = [](int64_t x) { return (x & 1) == 0; };
  const int64_t a_other = am == 0 ? g.a_i : g.a_k, b_other = bm == 0 ? g.b_k : g.b_j;
  const bool vec = even(a_other) && even(g.a_b) && even(b_other) && even(g.b_b) &&
                   (reinterpret_cast<uintptr_t>(g.A) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(g.B) & 15) == 0;
  dim3 grid(cdiv(g.N, 64), cdiv(g.M, 64), g.batch);
  const int sel = am * 4 + bm * 2 + (vec ? 1 : 0);
  switch (sel) {
    case 0: gemm64_kernel<0, 0, false><<<grid, NT, 0, s>>>(g); break;
    case 1: gemm64_kernel<0, 0, true><<<grid, NT, 0, s>>>(g); break;
    case 2: gemm64_kernel<0, 1, false><<<grid, NT, 0, s>>>(g); break;
    case 3: gemm64_kernel<0, 1, true><<<grid, NT, 0, s>>>(g); break;
    case 4: gemm64_kernel<1, 0, false><<<grid, NT, 0, s>>>(g); break;
    case 5: gemm64_kernel<1, 0, true><<<grid, NT, 0, s>>>(g); break;
    case 6: gemm64_kernel<1, 1, false><<<grid, NT, 0, s>>>(g); break;
    default: gemm64_kernel<1, 1, true><<<grid, NT, 0, s>>>(g); break;
  }
  return hipGetLastError();
}

hipError_t split_planes(int mode, const SplitArgs& a, hipStream_t s) {
  const int64_t rows = (int64_t)a.rows1 * a.rows2;
  if (rows <= 0) return hipSuccess;
  dim3 grid((unsigned)rows);
  switch (mode) {
    case MODE_F64: split_kernel<MODE_F64><<<grid, NT, 0, s>>>(a); break;
    case MODE_F32: split_kernel<MODE_F32><<<grid, NT, 0, s>>>(a); break;
    case MODE_BF16X3: split_kernel<MODE_BF16X3><<<grid, NT, 0, s>>>(a); break;
    case MODE_F16X2: split_kernel<MODE_F16X2><<<grid, NT, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t absmax64(const double* x, int64_t len, int64_t stride, int batch,
                    unsigned long long* amax, hipStream_t s) {
  if (len <= 0 || batch <= 0) return hipSuccess;
  // a few workgroups per row: one atomic each
  unsigned bx = cdiv(len, NT);
  if (bx > 64) bx = 64;
  absmax_kernel<<<dim3(bx, batch), NT, 0, s>>>(x, len, stride, amax);
  return hipGetLastError();
}

hipError_t rownorm2_max(const double* x, int64_t rows, int len, int64_t ld,
                        unsigned long long* out, hipStream_t s) {
  if (rows <= 0 || len <= 0) return hipSuccess;
  unsigned b = cdiv(rows, NT);
  if (b > 1024) b = 1024;
  rownorm2_kernel<<<b, NT, 0, s>>>(x, rows, len, ld, out);
  return hipGetLastError();
}

hipError_t colnorm2_max(const double* G, int n, int64_t stride, int nb, unsigned long long* out,
                        hipStream_t s) {
  if (nb <= 0 || n <= 0) return hipSuccess;
  colnorm2_kernel<<<nb, NT, 0, s>>>(G, n, stride, out);
  return hipGetLastError();
}

hipError_t ascale_bound(const unsigned long long* unorm2, const unsigned long long* amax_u,
                        const unsigned long long* gnorm2, const unsigned long long* amax_gb,
                        int64_t gb_stride, int nb, unsigned long long* amax_a, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  ascale_kernel<<<cdiv(nb, 64), 64, 0, s>>>(unorm2, amax_u, gnorm2, amax_gb, gb_stride, nb, amax_a);
  return hipGetLastError();
}

hipError_t fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  unsigned b = cdiv(n, NT);
  if (b > 4096) b = 4096;
  fill_u64_kernel<<<b, NT, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t dreduce(const DReduceArgs& a, hipStream_t s) {
  if (a.naux <= 0) return hipSuccess;
  const unsigned nt = cdiv(a.naux, DT);
  if (a.dpart_f32) dreduce_kernel<float><<<nt * nt, NT, 0, s>>>(a);
  else dreduce_kernel<double><<<nt * nt, NT, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t asym64(const double* G, int n, int m, unsigned long long* asym, hipStream_t s) {
  if (n <= 0 || m <= 0) return hipSuccess;
  unsigned bx = cdiv((int64_t)n * n, NT);
  if (bx > 256) bx = 256;
  fill_u64_kernel<<<cdiv(m, NT), NT, 0, s>>>(asym, m, 0ull);
  asym_kernel<<<dim3(bx, m), NT, 0, s>>>(G, n, asym);
  return hipGetLastError();
}

hipError_t sym_flags(const unsigned long long* asym, const unsigned long long* amax, int m,
                     double rtol, int* flag, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  sym_flags_kernel<<<cdiv(m, 64), 64, 0, s>>>(asym, amax, m, rtol, flag);
  return hipGetLastError();
}

hipError_t khatri_rao(const double* X, int n, int naux, int q0, int q1, double* KR,
                      hipStream_t s) {
  const int64_t rows = (int64_t)(q1 - q0) * n;
  if (rows <= 0) return hipSuccess;
  khatri_rao_kernel<<<(unsigned)rows, NT, 0, s>>>(X, n, naux, q0, KR);
  return hipGetLastError();
}

hipError_t energy_partials(const double* G, const double* S, int n, int m, double* tr,
                           hipStream_t s) {
  energy_partials_kernel<<<m, NT, 0, s>>>(G, S, n, m, tr);
  return hipGetLastError();
}

hipError_t energy_final(const double* tr, const double* w, int m, double* E, hipStream_t s) {
  energy_final_kernel<<<1, 64, 0, s>>>(tr, w, m, E);
  return hipGetLastError();
}

}  // namespace thcsox
