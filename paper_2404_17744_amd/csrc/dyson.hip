// One self-consistency step in FP64 on the GPU: Sigma(tau) -> Sigma(i w_n) ->
// Dyson equation (Sec. "Definitions", Eq. Dyson, orthonormal basis) ->
// G(i w_n) -> G(tau) and the density matrix.
//
// tau grid: the m roots of the Chebyshev polynomial T_m mapped to [0, beta].
//   forward : Sigma(i w_n) = sum_l T_nl c_l, c = Chebyshev interpolation
//             coefficients of Sigma(tau) through the roots, and
//             T_nl = int_0^beta exp(i w_n tau) T_l(2 tau / beta - 1) dtau,
//             w_n = (2n+1) pi / beta, n = 0 .. nw-1.
//   Dyson   : G(i w_n) = [(i w_n + mu) 1 - F - Sigma(i w_n)]^-1
//   backward: real coefficients minimising sum_n |sum_l T_nl c_l - G(i w_n)|^2,
//             G(tau_k) = sum_l c_l T_l(x_k),  gamma = -G(beta^-) = -sum_l c_l.
// The three linear maps are folded into two real matrices built on the host
// at plan time (Wf: [2 nw][m], Wb: [m + 1][2 nw]); each step is then two FP64
// matrix-core GEMMs around a batched complex Gauss-Jordan inversion.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/thcsox.h"
#include "error.hpp"
#include "kernels.hpp"

using namespace thcsox;

namespace {

constexpr int NT = 256;

// ----------------------------------------------------------------------------
// Host tables (FP64)
// ----------------------------------------------------------------------------

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_q).
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  x.resize(q);
  w.resize(q);
  for (int i = 0; i < q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = q * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= q; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    const double dp = q * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

struct Tables {
  std::vector<double> Wf;   // [2 nw][m]: rows 0..nw-1 real part, nw..2nw-1 imaginary part
  std::vector<double> Wb;   // [m + 1][2 nw]: G(tau_k) rows, then the gamma row
};

// T[n][l] = int_0^beta exp(i w_n tau) T_l(2 tau/beta - 1) dtau by composite
// Gauss-Legendre over equal panels in x = 2 tau / beta - 1.
std::vector<std::complex<double>> cheb_matsubara(int m, int nw, double beta) {
  const int q = 16;
  const double amax = (2.0 * nw - 1.0) * M_PI / 2.0;          // largest w_n beta / 2
  const int panels = std::max(64, (int)std::ceil(amax / M_PI * 4.0) + 2 * m);
  std::vector<double> gx, gw;
  gauss_legendre(q, gx, gw);
  const int npt = panels * q;
  std::vector<double> xs(npt), ws(npt);
  for (int p = 0; p < panels; ++p) {
    const double a = -1.0 + 2.0 * p / panels, h = 1.0 / panels;   // half width
    for (int i = 0; i < q; ++i) {
      xs[p * q + i] = a + h + h * gx[i];
      ws[p * q + i] = h * gw[i];
    }
  }
  std::vector<double> Tl((size_t)npt * m);   // T_l(x) by recurrence
  for (int i = 0; i < npt; ++i) {
    double t0 = 1.0, t1 = xs[i];
    Tl[(size_t)i * m] = 1.0;
    if (m > 1) Tl[(size_t)i * m + 1] = t1;
    for (int l = 2; l < m; ++l) {
      const double t2 = 2.0 * xs[i] * t1 - t0;
      Tl[(size_t)i * m + l] = t2;
      t0 = t1;
      t1 = t2;
    }
  }
  std::vector<std::complex<double>> T((size_t)nw * m);
  std::vector<std::complex<double>> acc(m);
  for (int n = 0; n < nw; ++n) {
    const double wn = (2.0 * n + 1.0) * M_PI / beta;
    std::fill(acc.begin(), acc.end(), std::complex<double>(0.0, 0.0));
    for (int i = 0; i < npt; ++i) {
      const double tau = 0.5 * beta * (1.0 + xs[i]);
      const std::complex<double> e = std::polar(ws[i] * 0.5 * beta, wn * tau);
      const double* t = &Tl[(size_t)i * m];
      for (int l = 0; l < m; ++l) acc[l] += e * t[l];
    }
    for (int l = 0; l < m; ++l) T[(size_t)n * m + l] = acc[l];
  }
  return T;
}

// Least-squares pseudo-inverse P = (A^T A)^-1 A^T of a tall A [r][c] by
// Householder QR: A = Q R, P = R^-1 Q^T.
std::vector<double> pinv_qr(std::vector<double> A, int r, int c) {
  std::vector<double> Qt((size_t)r * r, 0.0);   // accumulate Q^T applied to identity rows
  for (int i = 0; i < r; ++i) Qt[(size_t)i * r + i] = 1.0;
  std::vector<double> v(r);
  for (int k = 0; k < c; ++k) {
    double norm = 0.0;
    for (int i = k; i < r; ++i) norm += A[(size_t)i * c + k] * A[(size_t)i * c + k];
    norm = std::sqrt(norm);
    const double akk = A[(size_t)k * c + k];
    const double alpha = akk > 0 ? -norm : norm;
    for (int i = 0; i < r; ++i) v[i] = 0.0;
    v[k] = akk - alpha;
    for (int i = k + 1; i < r; ++i) v[i] = A[(size_t)i * c + k];
    double vn = 0.0;
    for (int i = k; i < r; ++i) vn += v[i] * v[i];
    if (vn == 0.0) continue;
    // H = I - 2 v v^T / (v^T v) applied to A (columns k..c-1) and to Qt
    for (int j = k; j < c; ++j) {
      double s = 0.0;
      for (int i = k; i < r; ++i) s += v[i] * A[(size_t)i * c + j];
      s = 2.0 * s / vn;
      for (int i = k; i < r; ++i) A[(size_t)i * c + j] -= s * v[i];
    }
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int i = k; i < r; ++i) s += v[i] * Qt[(size_t)i * r + j];
      s = 2.0 * s / vn;
      for (int i = k; i < r; ++i) Qt[(size_t)i * r + j] -= s * v[i];
    }
  }
  // P = R^-1 (first c rows of Qt), R upper triangular in A[0..c-1][0..c-1]
  std::vector<double> P((size_t)c * r);
  for (int j = 0; j < r; ++j) {
    for (int i = c - 1; i >= 0; --i) {
      double s = Qt[(size_t)i * r + j];
      for (int k2 = i + 1; k2 < c; ++k2) s -= A[(size_t)i * c + k2] * P[(size_t)k2 * r + j];
      P[(size_t)i * r + j] = s / A[(size_t)i * c + i];
    }
  }
  return P;
}

Tables build_tables(int m, int nw, double beta) {
  std::vector<double> x(m);
  for (int k = 0; k < m; ++k) x[k] = -std::cos((2.0 * k + 1.0) * M_PI / (2.0 * m));
  std::vector<double> Tev((size_t)m * m);   // Tev[k][l] = T_l(x_k)
  for (int k = 0; k < m; ++k) {
    double t0 = 1.0, t1 = x[k];
    Tev[(size_t)k * m] = 1.0;
    if (m > 1) Tev[(size_t)k * m + 1] = t1;
    for (int l = 2; l < m; ++l) {
      const double t2 = 2.0 * x[k] * t1 - t0;
      Tev[(size_t)k * m + l] = t2;
      t0 = t1;
      t1 = t2;
    }
  }
  const auto T = cheb_matsubara(m, nw, beta);
  Tables tb;
  // forward: c_l = (2 - delta_l0)/m sum_k T_l(x_k) F_k ; F(i w_n) = sum_l T_nl c_l
  tb.Wf.assign((size_t)2 * nw * m, 0.0);
  for (int n = 0; n < nw; ++n)
    for (int k = 0; k < m; ++k) {
      std::complex<double> s(0.0, 0.0);
      for (int l = 0; l < m; ++l)
        s += T[(size_t)n * m + l] * ((l == 0 ? 1.0 : 2.0) / m) * Tev[(size_t)k * m + l];
      tb.Wf[(size_t)n * m + k] = s.real();
      tb.Wf[(size_t)(nw + n) * m + k] = s.imag();
    }
  // backward: c = pinv([Re T; Im T]) [Re G; Im G]
  std::vector<double> A((size_t)2 * nw * m);
  for (int n = 0; n < nw; ++n)
    for (int l = 0; l < m; ++l) {
      A[(size_t)n * m + l] = T[(size_t)n * m + l].real();
      A[(size_t)(nw + n) * m + l] = T[(size_t)n * m + l].imag();
    }
  const auto P = pinv_qr(A, 2 * nw, m);   // [m][2nw]
  tb.Wb.assign((size_t)(m + 1) * 2 * nw, 0.0);
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < 2 * nw; ++j) {
      double s = 0.0;
      for (int l = 0; l < m; ++l) s += Tev[(size_t)k * m + l] * P[(size_t)l * 2 * nw + j];
      tb.Wb[(size_t)k * 2 * nw + j] = s;
    }
  for (int j = 0; j < 2 * nw; ++j) {
    double s = 0.0;
    for (int l = 0; l < m; ++l) s += P[(size_t)l * 2 * nw + j];
    tb.Wb[(size_t)m * 2 * nw + j] = -s;   // gamma = -sum_l c_l
  }
  return tb;
}

// tables depend only on (m, nw, beta): cache them for repeated plans
const Tables& tables_for(int m, int nw, double beta) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, double>, Tables> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple(m, nw, beta);
  auto it = cache.find(key);
  if (it == cache.end()) it = cache.emplace(key, build_tables(m, nw, beta)).first;
  return it->second;
}

// ----------------------------------------------------------------------------
// Kernels
// ----------------------------------------------------------------------------

// Am[w] = (i w_w + mu) 1 - F - Sigma(i w_w) as complex [n][n]; wfreq[w] = w_w.
__global__ __launch_bounds__(NT) void build_a(const double* __restrict__ S, const double* __restrict__ F,
                                              double mu, const double* __restrict__ wfreq, int n,
                                              int nw, double2* __restrict__ Am) {
  const int w = blockIdx.y;
  const double wn = wfreq[w];
  const int64_t nn = (int64_t)n * n;
  const double* Sre = S + (int64_t)w * nn;
  const double* Sim = S + (int64_t)(nw + w) * nn;
  double2* A = Am + (int64_t)w * nn;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < nn; e += (int64_t)gridDim.x * NT) {
    const int64_t i = e / n, j = e % n;
    double re = -F[e] - Sre[e], im = -Sim[e];
    if (i == j) {
      re += mu;
      im += wn;
    }
    A[e] = make_double2(re, im);
  }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place Gauss-Jordan inversion with partial pivoting, blocked by panels of
// GJ_B columns.  For the panel [k, k + bw):
//   gje_panel: the n x bw panel sits in LDS; for each of its columns c the pivot
//     is the largest |a_ic| over the rows i >= c not yet used as pivot rows, rows c
//     and piv[c] are swapped in full (the panel in LDS, the other columns in
//     memory), and the column is eliminated from the panel columns only: the
//     pivot row is scaled by 1/p, every other row loses a_ic/p times it, and
//     column c becomes the matching column of the inverse (1/p at the pivot,
//     -a_ic/p elsewhere).  The panel ends as W, the panel's columns of the
//     product of the panel's elimination matrices.
//   gje_trail: every other column j gets the same eliminations at once,
//     A[:, j] += (W - E) A[panel rows, j] with E the panel rows' unit columns.
// After the last panel the matrix holds the inverse with its columns permuted by
// the row interchanges; gje_perm and extract_inv undo them (last first).
// One workgroup per frequency in gje_panel; flag[0] is set to 1 for a zero or
// non-finite pivot.
constexpr int GJ_B = 8;          // panel width
constexpr int GJ_LDS = 9216;     // double2 panel elements in LDS (144 KiB): bw * n <= GJ_LDS
constexpr int GJ_TCB = 64;       // columns per gje_trail workgroup
constexpr int GJ_TRC = 32;       // rows per staged chunk of W

__global__ __launch_bounds__(NT) void gje_panel(double2* __restrict__ Am, int n, int k, int bw,
                                                int* __restrict__ piv, int* __restrict__ flag) {
  __shared__ double2 P[GJ_LDS];  // column-major: P[t * n + i] = A[i][k + t]
  __shared__ double bval[NT];
  __shared__ int bidx[NT];
  __shared__ double2 prow[GJ_B];
  const int tid = threadIdx.x, w = blockIdx.x;
  double2* A = Am + (int64_t)w * n * n;
  for (int e = tid; e < n * bw; e += NT) {
    const int i = e / bw, t = e % bw;
    P[t * n + i] = A[(int64_t)i * n + k + t];
  }
  __syncthreads();
  for (int t = 0; t < bw; ++t) {
    const int c = k + t;
    double best = -1.0;
    int bi = c;
    for (int i = c + tid; i < n; i += NT) {
      const double2 a = P[t * n + i];
      const double v = a.x * a.x + a.y * a.y;
      if (v > best) { best = v; bi = i; }
    }
    bval[tid] = best;
    bidx[tid] = bi;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
      if (tid < o) {
        const double v2 = bval[tid + o];
        const int i2 = bidx[tid + o];
        if (v2 > bval[tid] || (v2 == bval[tid] && i2 < bidx[tid])) {
          bval[tid] = v2;
          bidx[tid] = i2;
        }
      }
      __syncthreads();
    }
    const int r = bidx[0];
    if (tid == 0) {
      piv[(int64_t)w * n + c] = r;
      if (!(bval[0] > 0.0) || !isfinite(bval[0])) atomicExch(flag, 1);
    }
    if (r != c) {
      for (int tt = tid; tt < bw; tt += NT) {
        const double2 x = P[tt * n + c];
        P[tt * n + c] = P[tt * n + r];
        P[tt * n + r] = x;
      }
      for (int j = tid; j < n; j += NT) {
        if (j >= k && j < k + bw) continue;
        const double2 x = A[(int64_t)c * n + j];
        A[(int64_t)c * n + j] = A[(int64_t)r * n + j];
        A[(int64_t)r * n + j] = x;
      }
    }
    __syncthreads();
    if (tid < bw) {
      const double2 p = P[t * n + c];
      const double d = p.x * p.x + p.y * p.y;
      const double2 pinv = d > 0.0 ? make_double2(p.x / d, -p.y / d) : make_double2(0.0, 0.0);
      prow[tid] = tid == t ? pinv : cmul(P[tid * n + c], pinv);
    }
    __syncthreads();
    const double2 pinv = prow[t];
    for (int i = tid; i < n; i += NT) {
      if (i == c) {
        for (int tt = 0; tt < bw; ++tt) P[tt * n + c] = prow[tt];
      } else {
        const double2 f = P[t * n + i];
        for (int tt = 0; tt < bw; ++tt) {
          if (tt == t) continue;
          const double2 q = cmul(f, prow[tt]);
          P[tt * n + i].x -= q.x;
          P[tt * n + i].y -= q.y;
        }
        const double2 q = cmul(f, pinv);
        P[t * n + i] = make_double2(-q.x, -q.y);
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < n * bw; e += NT) {
    const int i = e / bw, t = e % bw;
    A[(int64_t)i * n + k + t] = P[t * n + i];
  }
}

// A[:, j] += (W - E) A[k .. k+bw-1, j] for the columns j outside the panel; the
// workgroup owns GJ_TCB columns (all rows) of one frequency, so the panel rows it
// reads first are not yet overwritten.
__global__ __launch_bounds__(NT) void gje_trail(double2* __restrict__ Am, int n, int k, int bw) {
  __shared__ double2 X[GJ_B][GJ_TCB];
  __shared__ double2 Wl[GJ_TRC][GJ_B];
  const int tid = threadIdx.x, w = blockIdx.y;
  double2* A = Am + (int64_t)w * n * n;
  const int jj = tid % GJ_TCB, q = tid / GJ_TCB;
  const int j0 = blockIdx.x * GJ_TCB, j = j0 + jj;
  const bool active = j < n && (j < k || j >= k + bw);
  for (int e = tid; e < bw * GJ_TCB; e += NT) {
    const int t = e / GJ_TCB, c2 = e % GJ_TCB;
    X[t][c2] = j0 + c2 < n ? A[(int64_t)(k + t) * n + j0 + c2] : make_double2(0.0, 0.0);
  }
  for (int i0 = 0; i0 < n; i0 += GJ_TRC) {
    __syncthreads();
    for (int e = tid; e < GJ_TRC * bw; e += NT) {
      const int ii = e / bw, t = e % bw, i = i0 + ii;
      double2 v = i < n ? A[(int64_t)i * n + k + t] : make_double2(0.0, 0.0);
      if (i == k + t) v.x -= 1.0;
      Wl[ii][t] = v;
    }
    __syncthreads();
    if (active) {
      for (int ii = q; ii < GJ_TRC && i0 + ii < n; ii += NT / GJ_TCB) {
        double2 a = A[(int64_t)(i0 + ii) * n + j];
        for (int t = 0; t < bw; ++t) {
          const double2 wv = Wl[ii][t], x = X[t][jj];
          a.x = fma(wv.x, x.x, fma(-wv.y, x.y, a.x));
          a.y = fma(wv.x, x.y, fma(wv.y, x.x, a.y));
        }
        A[(int64_t)(i0 + ii) * n + j] = a;
      }
    }
  }
}

// perm[w][j]: the column of the eliminated matrix that is column j of the
// inverse (the row interchanges applied as column interchanges, last first).
__global__ __launch_bounds__(NT) void gje_perm(const int* __restrict__ piv, int n, int nw,
                                               int* __restrict__ perm) {
  const int w = blockIdx.x * NT + threadIdx.x;
  if (w >= nw) return;
  int* pm = perm + (int64_t)w * n;
  const int* pv = piv + (int64_t)w * n;
  for (int j = 0; j < n; ++j) pm[j] = j;
  for (int c = n - 1; c >= 0; --c) {
    const int r = pv[c];
    if (r != c) {
      const int x = pm[c];
      pm[c] = pm[r];
      pm[r] = x;
    }
  }
}

// Gstack[w][ij] = Re G(i w)_ij, Gstack[nw + w][ij] = Im G(i w)_ij.
__global__ __launch_bounds__(NT) void extract_inv(const double2* __restrict__ Am,
                                                  const int* __restrict__ perm, int n, int nw,
                                                  double* __restrict__ Gs) {
  const int w = blockIdx.y;
  const int64_t nn = (int64_t)n * n;
  const double2* A = Am + (int64_t)w * nn;
  const int* pm = perm + (int64_t)w * n;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < nn; e += (int64_t)gridDim.x * NT) {
    const int64_t i = e / n, j = e % n;
    const double2 v = A[i * n + pm[j]];
    Gs[(int64_t)w * nn + e] = v.x;
    Gs[(int64_t)(nw + w) * nn + e] = v.y;
  }
}

// tr[w] = Re Tr G(i w_w), tr[nw + w] = Im Tr G(i w_w): the diagonal of each
// inverse, read through the column permutation (one workgroup per frequency).
__global__ __launch_bounds__(NT) void inv_traces(const double2* __restrict__ Am,
                                                 const int* __restrict__ perm, int n, int nw,
                                                 double* __restrict__ tr) {
  __shared__ double r_re[NT], r_im[NT];
  const int w = blockIdx.x;
  const double2* A = Am + (int64_t)w * n * n;
  const int* pm = perm + (int64_t)w * n;
  double re = 0.0, im = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) {
    const double2 v = A[(int64_t)i * n + pm[i]];
    re += v.x;
    im += v.y;
  }
  r_re[threadIdx.x] = re;
  r_im[threadIdx.x] = im;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      r_re[threadIdx.x] += r_re[threadIdx.x + o];
      r_im[threadIdx.x] += r_im[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tr[w] = r_re[0];
    tr[nw + w] = r_im[0];
  }
}

// out = sum_pq A[p][q] B[q][p] (one workgroup, fixed order).
__global__ __launch_bounds__(NT) void trace_ab(const double* A, const double* B, int n, double* out) {
  __shared__ double red[NT];
  double s = 0.0;
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = threadIdx.x; e < nn; e += NT) {
    const int64_t p = e / n, q = e % n;
    s = fma(A[e], B[q * n + p], s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

int dfail(int code, const std::string& m) { return set_error(code, m); }

__global__ __launch_bounds__(NT) void real_to_complex(const double* __restrict__ M, int64_t nn,
                                                      double2* __restrict__ Am) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < nn; e += (int64_t)gridDim.x * NT)
    Am[e] = make_double2(M[e], 0.0);
}

// Minv[i][j] = Re of the eliminated matrix at column perm[j] (one matrix)
__global__ __launch_bounds__(NT) void extract_real_inv(const double2* __restrict__ Am,
                                                       const int* __restrict__ perm, int n,
                                                       double* __restrict__ Minv) {
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < nn; e += (int64_t)gridDim.x * NT) {
    const int64_t i = e / n, j = e % n;
    Minv[e] = Am[i * n + perm[j]].x;
  }
}

}  // namespace

namespace thcsox {
hipError_t gj_inverse_real(const double* M, int n, double* Minv, double2* Am, int* piv, int* perm,
                           int* flag, hipStream_t s) {
  if (n <= 0 || n > GJ_LDS) return hipErrorInvalidValue;
  const int64_t nn = (int64_t)n * n;
  const unsigned bx = (unsigned)std::min<int64_t>(1024, (nn + NT - 1) / NT);
  real_to_complex<<<bx, NT, 0, s>>>(M, nn, Am);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = hipMemsetAsync(flag, 0, sizeof(int), s)) != hipSuccess) return e;
  int bw = GJ_B;
  while (bw > 1 && (int64_t)bw * n > GJ_LDS) bw /= 2;
  for (int k = 0; k < n; k += bw) {
    const int w = std::min(bw, n - k);
    gje_panel<<<1, NT, 0, s>>>(Am, n, k, w, piv, flag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    gje_trail<<<dim3((unsigned)((n + GJ_TCB - 1) / GJ_TCB), 1), NT, 0, s>>>(Am, n, k, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  gje_perm<<<1, NT, 0, s>>>(piv, n, 1, perm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  extract_real_inv<<<bx, NT, 0, s>>>(Am, perm, n, Minv);
  return hipGetLastError();
}
}  // namespace thcsox

struct thcsox_dyson_s {
  int n = 0, m = 0, nw = 0, panel = GJ_B;
  double beta = 0, mu = 0;
  hipStream_t stream = nullptr;
  double* F = nullptr;     // [n][n]
  double* Wf = nullptr;    // [2nw][m]
  double* Wb = nullptr;    // [m+1][2nw]
  double* wfreq = nullptr; // [nw] the frequencies w_j
  double* Siw = nullptr;   // [2nw][n n]
  double2* Am = nullptr;   // [nw][n][n]
  int* piv = nullptr;      // [nw][n]
  int* perm = nullptr;     // [nw][n]
  double* Gs = nullptr;    // [2nw][n n]
  double* Gout = nullptr;  // [m+1][n n]
  int* flag = nullptr;
  double* scal = nullptr;
  double* traces = nullptr;   // [2 nw]
  double* Dw = nullptr;       // [2nw][n n], commutator DIIS: Sigma_out - Sigma_in in frequency
  bool have_g = false;        // Gs holds the G(i w) of a completed step
  std::vector<double> gamma_row;   // the gamma row of Wb (host)
  std::vector<void*> allocs;
  ~thcsox_dyson_s() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {
template <typename T>
int dalloc(thcsox_dyson_s* d, T** p, size_t count) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(16, count * sizeof(T)));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return dfail(THCSOX_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  d->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return 0;
}

#define DTRY(expr)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return dfail(THCSOX_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)
}  // namespace

namespace {

// Sigma(i w) (real and imaginary rows) = Wf . Sigma(tau)
int dy_forward(thcsox_dyson_s* d, const double* Sigma_dev) {
  const int64_t nn = (int64_t)d->n * d->n;
  Gemm64Args g{};
  g.M = 2 * d->nw; g.N = (int)nn; g.K = d->m; g.batch = 1; g.alpha = 1.0; g.beta = 0.0;
  g.A = d->Wf; g.a_i = d->m; g.a_k = 1;
  g.B = Sigma_dev; g.b_k = nn; g.b_j = 1;
  g.C = d->Siw; g.c_i = nn; g.c_j = 1; g.cj_in = nn; g.cj_out = 0;
  DTRY(gemm64(g, d->stream));
  return 0;
}

// G(i w) = [(i w + mu) 1 - F - Sigma(i w)]^-1 for every frequency, left in Am
// (columns permuted by perm); flag set for a singular matrix.
int dy_invert(thcsox_dyson_s* d, double mu) {
  const int n = d->n, nw = d->nw;
  const int64_t nn = (int64_t)n * n;
  const hipStream_t s = d->stream;
  const unsigned bx = (unsigned)std::min<int64_t>(64, (nn + NT - 1) / NT);
  build_a<<<dim3(bx, nw), NT, 0, s>>>(d->Siw, d->F, mu, d->wfreq, n, nw, d->Am);
  DTRY(hipGetLastError());
  DTRY(hipMemsetAsync(d->flag, 0, sizeof(int), s));
  const int bw = d->panel;
  for (int k = 0; k < n; k += bw) {
    const int w = std::min(bw, n - k);
    gje_panel<<<nw, NT, 0, s>>>(d->Am, n, k, w, d->piv, d->flag);
    DTRY(hipGetLastError());
    gje_trail<<<dim3((unsigned)((n + GJ_TCB - 1) / GJ_TCB), nw), NT, 0, s>>>(d->Am, n, k, w);
    DTRY(hipGetLastError());
  }
  gje_perm<<<(unsigned)((nw + NT - 1) / NT), NT, 0, s>>>(d->piv, n, nw, d->perm);
  DTRY(hipGetLastError());
  return 0;
}

// Tr gamma of the inverses in Am: gamma = sum_j Wb[m][j] [Re G; Im G]_j, so only
// the traces of the G(i w) are needed.  Synchronises the stream.
int dy_electrons(thcsox_dyson_s* d, double* N) {
  inv_traces<<<d->nw, NT, 0, d->stream>>>(d->Am, d->perm, d->n, d->nw, d->traces);
  DTRY(hipGetLastError());
  std::vector<double> tr((size_t)2 * d->nw);
  int flag = 0;
  DTRY(hipMemcpyAsync(tr.data(), d->traces, sizeof(double) * tr.size(), hipMemcpyDeviceToHost,
                      d->stream));
  DTRY(hipMemcpyAsync(&flag, d->flag, sizeof(int), hipMemcpyDeviceToHost, d->stream));
  DTRY(hipStreamSynchronize(d->stream));
  if (flag) return dfail(THCSOX_ENONFINITE, "singular matrix in the Dyson solve");
  double acc = 0.0;
  for (size_t j = 0; j < tr.size(); ++j) acc += d->gamma_row[j] * tr[j];
  *N = acc;
  return 0;
}

// unpack the inverses, fit back to tau: G_dev[m][n][n] and gamma_dev[n][n]
int dy_backward(thcsox_dyson_s* d, double* G_dev, double* gamma_dev) {
  const int n = d->n, m = d->m, nw = d->nw;
  const int64_t nn = (int64_t)n * n;
  const hipStream_t s = d->stream;
  const unsigned bx = (unsigned)std::min<int64_t>(64, (nn + NT - 1) / NT);
  extract_inv<<<dim3(bx, nw), NT, 0, s>>>(d->Am, d->perm, n, nw, d->Gs);
  DTRY(hipGetLastError());
  d->have_g = true;
  // [G(tau_0) .. G(tau_{m-1}); gamma] = Wb . [Re G(i w); Im G(i w)]
  Gemm64Args g{};
  g.M = m + 1; g.N = (int)nn; g.K = 2 * nw; g.batch = 1; g.alpha = 1.0; g.beta = 0.0;
  g.A = d->Wb; g.a_i = 2 * nw; g.a_k = 1;
  g.B = d->Gs; g.b_k = nn; g.b_j = 1;
  g.C = d->Gout; g.c_i = nn; g.c_j = 1; g.cj_in = nn; g.cj_out = 0;
  DTRY(gemm64(g, s));
  DTRY(hipMemcpyAsync(G_dev, d->Gout, sizeof(double) * m * nn, hipMemcpyDeviceToDevice, s));
  if (gamma_dev)
    DTRY(hipMemcpyAsync(gamma_dev, d->Gout + (int64_t)m * nn, sizeof(double) * nn,
                        hipMemcpyDeviceToDevice, s));
  int flag = 0;
  DTRY(hipMemcpyAsync(&flag, d->flag, sizeof(int), hipMemcpyDeviceToHost, s));
  DTRY(hipStreamSynchronize(s));
  if (flag) return dfail(THCSOX_ENONFINITE, "singular matrix in the Dyson solve");
  return 0;
}

}  // namespace

namespace {
// The plan on given transform tables (Wf [2 nw][m], Wb [m + 1][2 nw]) and
// frequencies wf[nw]; F_dev is checked to be device memory.
int dyson_create(thcsox_dyson_t* out, int n, int m, int nw, double beta, double mu,
                 const std::vector<double>& wf, const std::vector<double>& Wf,
                 const std::vector<double>& Wb, const double* F_dev, void* hip_stream) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, F_dev) != hipSuccess ||
      (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)) {
    (void)hipGetLastError();
    return dfail(THCSOX_ENOTDEV, "F_dev is not device memory");
  }
  auto* d = new (std::nothrow) thcsox_dyson_s();
  if (d == nullptr) return dfail(THCSOX_ENOMEM, "host allocation failed");
  d->n = n; d->m = m; d->nw = nw; d->beta = beta; d->mu = mu;
  while (d->panel > 1 && (int64_t)d->panel * n > GJ_LDS) d->panel /= 2;
  d->stream = static_cast<hipStream_t>(hip_stream);
  const int64_t nn = (int64_t)n * n;
  int rc;
  if ((rc = dalloc(d, &d->F, nn)) || (rc = dalloc(d, &d->Wf, (size_t)2 * d->nw * d->m)) ||
      (rc = dalloc(d, &d->Wb, (size_t)(d->m + 1) * 2 * d->nw)) ||
      (rc = dalloc(d, &d->wfreq, (size_t)d->nw)) ||
      (rc = dalloc(d, &d->Siw, (size_t)2 * d->nw * nn)) ||
      (rc = dalloc(d, &d->Am, (size_t)d->nw * nn)) ||
      (rc = dalloc(d, &d->piv, (size_t)d->nw * n)) ||
      (rc = dalloc(d, &d->perm, (size_t)d->nw * n)) ||
      (rc = dalloc(d, &d->Gs, (size_t)2 * d->nw * nn)) ||
      (rc = dalloc(d, &d->Gout, (size_t)(d->m + 1) * nn)) || (rc = dalloc(d, &d->flag, 1)) ||
      (rc = dalloc(d, &d->scal, 1)) || (rc = dalloc(d, &d->traces, (size_t)2 * d->nw))) {
    delete d;
    return rc;
  }
  d->gamma_row.assign(Wb.begin() + (size_t)d->m * 2 * d->nw, Wb.begin() + (size_t)(d->m + 1) * 2 * d->nw);
  hipError_t e;
  if ((e = hipMemcpyAsync(d->F, F_dev, sizeof(double) * nn, hipMemcpyDeviceToDevice, d->stream)) ||
      (e = hipMemcpyAsync(d->Wf, Wf.data(), sizeof(double) * Wf.size(),
                          hipMemcpyHostToDevice, d->stream)) ||
      (e = hipMemcpyAsync(d->Wb, Wb.data(), sizeof(double) * Wb.size(),
                          hipMemcpyHostToDevice, d->stream)) ||
      (e = hipMemcpyAsync(d->wfreq, wf.data(), sizeof(double) * wf.size(),
                          hipMemcpyHostToDevice, d->stream)) ||
      (e = hipStreamSynchronize(d->stream))) {
    delete d;
    return dfail(THCSOX_EDEVICE, std::string("dyson plan: ") + hipGetErrorString(e));
  }
  *out = d;
  return 0;
}
}  // namespace

extern "C" {

int thcsox_dyson_plan(thcsox_dyson_t* out, int n, int ntau, int n_matsubara, double beta,
                      double mu, const double* tau_host, const double* F_dev, void* hip_stream) {
  clear_error();
  if (out == nullptr) return dfail(THCSOX_EINVAL, "out is NULL");
  *out = nullptr;
  if (n <= 0 || ntau <= 1 || n_matsubara <= 0 || !(beta > 0.0))
    return dfail(THCSOX_EINVAL, "need n > 0, ntau > 1, n_matsubara > 0, beta > 0");
  if ((int64_t)n > GJ_LDS)
    return dfail(THCSOX_EINVAL, "n too large for the in-LDS panel of the Dyson inversion (n <= 9216)");
  if (2 * n_matsubara < ntau)
    return dfail(THCSOX_EINVAL, "need 2 n_matsubara >= ntau for the least-squares fit");
  if (tau_host == nullptr || F_dev == nullptr) return dfail(THCSOX_EINVAL, "NULL argument");
  for (int k = 0; k < ntau; ++k) {
    const double x = -std::cos((2.0 * k + 1.0) * M_PI / (2.0 * ntau));
    if (std::fabs(tau_host[k] - 0.5 * beta * (1.0 + x)) > 1e-12 * beta)
      return dfail(THCSOX_EINVAL, "tau grid is not the Chebyshev-root grid");
  }
  try {   // host tables: no exception may cross the C interface
    const Tables& tb = tables_for(ntau, n_matsubara, beta);
    std::vector<double> wf(n_matsubara);
    for (int j = 0; j < n_matsubara; ++j) wf[j] = (2.0 * j + 1.0) * M_PI / beta;
    return dyson_create(out, n, ntau, n_matsubara, beta, mu, wf, tb.Wf, tb.Wb, F_dev, hip_stream);
  } catch (const std::bad_alloc&) {
    return dfail(THCSOX_ENOMEM, "host allocation failed");
  }
}

int thcsox_dyson_plan_sampled(thcsox_dyson_t* out, int n, int ntau, int nfreq, double beta,
                              double mu, const int* freq_n_host, const double* Wf_host,
                              const double* Wb_host, const double* F_dev, void* hip_stream) {
  clear_error();
  if (out == nullptr) return dfail(THCSOX_EINVAL, "out is NULL");
  *out = nullptr;
  if (n <= 0 || ntau <= 1 || nfreq <= 0 || !(beta > 0.0))
    return dfail(THCSOX_EINVAL, "need n > 0, ntau > 1, nfreq > 0, beta > 0");
  if ((int64_t)n > GJ_LDS)
    return dfail(THCSOX_EINVAL, "n too large for the in-LDS panel of the Dyson inversion (n <= 9216)");
  if (2 * nfreq < ntau) return dfail(THCSOX_EINVAL, "need 2 nfreq >= ntau for the fit");
  if (freq_n_host == nullptr || Wf_host == nullptr || Wb_host == nullptr || F_dev == nullptr)
    return dfail(THCSOX_EINVAL, "NULL argument");
  for (int j = 0; j < nfreq; ++j)
    if (freq_n_host[j] < 0 || (j > 0 && freq_n_host[j] <= freq_n_host[j - 1]))
      return dfail(THCSOX_EINVAL, "freq_n must be ascending and >= 0");
  try {   // host copies of the tables: no exception may cross the C interface
    std::vector<double> Wf(Wf_host, Wf_host + (size_t)2 * nfreq * ntau);
    std::vector<double> Wb(Wb_host, Wb_host + (size_t)(ntau + 1) * 2 * nfreq);
    for (double v : Wf)
      if (!std::isfinite(v)) return dfail(THCSOX_EINVAL, "Wf has a non-finite entry");
    for (double v : Wb)
      if (!std::isfinite(v)) return dfail(THCSOX_EINVAL, "Wb has a non-finite entry");
    // the plan's last table row gives gamma = -G(beta^-) directly
    for (size_t j = (size_t)ntau * 2 * nfreq; j < Wb.size(); ++j) Wb[j] = -Wb[j];
    std::vector<double> wf(nfreq);
    for (int j = 0; j < nfreq; ++j) wf[j] = (2.0 * freq_n_host[j] + 1.0) * M_PI / beta;
    return dyson_create(out, n, ntau, nfreq, beta, mu, wf, Wf, Wb, F_dev, hip_stream);
  } catch (const std::bad_alloc&) {
    return dfail(THCSOX_ENOMEM, "host allocation failed");
  }
}

int thcsox_dyson_step(thcsox_dyson_t d, const double* Sigma_dev, double* G_dev, double* gamma_dev) {
  clear_error();
  if (d == nullptr || Sigma_dev == nullptr || G_dev == nullptr)
    return dfail(THCSOX_EINVAL, "NULL argument");
  int rc;
  if ((rc = dy_forward(d, Sigma_dev)) || (rc = dy_invert(d, d->mu))) return rc;
  return dy_backward(d, G_dev, gamma_dev);
}

int thcsox_dyson_step_mu(thcsox_dyson_t d, const double* Sigma_dev, double nelec, double tol,
                         double* mu_io, double* G_dev, double* gamma_dev, int* evals_out) {
  clear_error();
  if (d == nullptr || Sigma_dev == nullptr || G_dev == nullptr || mu_io == nullptr)
    return dfail(THCSOX_EINVAL, "NULL argument");
  if (!(nelec >= 0.0) || !(nelec <= d->n) || !(tol > 0.0) || !std::isfinite(*mu_io))
    return dfail(THCSOX_EINVAL, "need 0 <= nelec <= n, tol > 0 and a finite starting mu");
  int rc;
  if ((rc = dy_forward(d, Sigma_dev))) return rc;
  // f(mu) = Tr gamma(mu) - nelec, one Dyson solve per evaluation; the last
  // evaluated mu is the answer, so its inverses are the ones left in Am
  int evals = 0;
  auto f = [&](double mu, double* val) -> int {
    int r;
    if ((r = dy_invert(d, mu)) || (r = dy_electrons(d, val))) return r;
    *val -= nelec;
    ++evals;
    return 0;
  };
  constexpr int MAX_EVAL = 80;
  constexpr double STEP = 0.1;   // first bracketing step (Ha), doubled while the sign holds
  double a = *mu_io, fa, b, fb, mu = a;
  bool done = false;
  if ((rc = f(a, &fa))) return rc;
  if (std::fabs(fa) <= tol) done = true;
  if (!done) {
    double step = fa > 0 ? -STEP : STEP;
    b = a + step;
    if ((rc = f(b, &fb))) return rc;
    while (fa * fb > 0 && evals < MAX_EVAL) {
      a = b;
      fa = fb;
      step *= 2.0;
      b = a + step;
      if ((rc = f(b, &fb))) return rc;
    }
    mu = b;
    if (std::fabs(fb) <= tol) done = true;
    else if (fa * fb > 0) return dfail(THCSOX_ENONFINITE, "no bracket for the chemical potential");
  }
  // Illinois variant of regula falsi on the bracket (a, b)
  while (!done) {
    if (evals >= MAX_EVAL) return dfail(THCSOX_ENONFINITE, "chemical potential search did not converge");
    const double c = (a * fb - b * fa) / (fb - fa);
    double fc;
    if ((rc = f(c, &fc))) return rc;
    mu = c;
    if (std::fabs(fc) <= tol || std::fabs(b - a) <= 1e-14 * (1.0 + std::fabs(c))) break;
    if (fc * fb < 0) {
      a = b;
      fa = fb;
    } else {
      fa *= 0.5;
    }
    b = c;
    fb = fc;
  }
  d->mu = mu;
  *mu_io = mu;
  if (evals_out) *evals_out = evals;
  return dy_backward(d, G_dev, gamma_dev);
}

int thcsox_dyson_commutator(thcsox_dyson_t d, const double* Sigma_in_dev,
                            const double* Sigma_out_dev, double* e_dev) {
  clear_error();
  if (d == nullptr || Sigma_in_dev == nullptr || Sigma_out_dev == nullptr || e_dev == nullptr)
    return dfail(THCSOX_EINVAL, "NULL argument");
  for (const void* q : {(const void*)Sigma_in_dev, (const void*)Sigma_out_dev, (const void*)e_dev}) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, q) != hipSuccess ||
        (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)) {
      (void)hipGetLastError();
      return dfail(THCSOX_ENOTDEV, "arrays must be device memory");
    }
  }
  if (!d->have_g) return dfail(THCSOX_EINVAL, "no Dyson step has been taken on this plan");
  const int n = d->n, nw = d->nw, m = d->m;
  const int64_t nn = (int64_t)n * n;
  const hipStream_t s = d->stream;
  if (d->Dw == nullptr) {
    int rc = dalloc(d, &d->Dw, (size_t)2 * nw * nn);
    if (rc) return rc;
  }
  // D(i w) = Wf (Sigma_out - Sigma_in), as [Re; Im] rows
  Gemm64Args g{};
  g.M = 2 * nw; g.N = (int)nn; g.K = m; g.batch = 1; g.alpha = 1.0; g.beta = 0.0;
  g.A = d->Wf; g.a_i = m; g.a_k = 1;
  g.B = Sigma_out_dev; g.b_k = nn; g.b_j = 1;
  g.C = d->Dw; g.c_i = nn; g.c_j = 1; g.cj_in = nn; g.cj_out = 0;
  DTRY(gemm64(g, s));
  g.B = Sigma_in_dev; g.alpha = -1.0; g.beta = 1.0;
  DTRY(gemm64(g, s));
  // e = G D - D G per frequency, G = Gr + i Gi from the last step (d->Gs), D = Dr + i Di:
  //   Re e = Gr Dr - Gi Di - Dr Gr + Di Gi,  Im e = Gr Di + Gi Dr - Dr Gi - Di Gr
  const double* Gr = d->Gs;
  const double* Gi = d->Gs + (int64_t)nw * nn;
  const double* Dr = d->Dw;
  const double* Di = d->Dw + (int64_t)nw * nn;
  double* er = e_dev;
  double* ei = e_dev + (int64_t)nw * nn;
  struct Term { const double* A; const double* B; double alpha; double* C; };
  const Term terms[8] = {{Gr, Dr, 1.0, er}, {Gi, Di, -1.0, er}, {Dr, Gr, -1.0, er}, {Di, Gi, 1.0, er},
                         {Gr, Di, 1.0, ei}, {Gi, Dr, 1.0, ei}, {Dr, Gi, -1.0, ei}, {Di, Gr, -1.0, ei}};
  for (int t = 0; t < 8; ++t) {
    Gemm64Args b{};
    b.M = n; b.N = n; b.K = n; b.batch = nw; b.alpha = terms[t].alpha;
    b.beta = (t == 0 || t == 4) ? 0.0 : 1.0;
    b.A = terms[t].A; b.a_i = n; b.a_k = 1; b.a_b = nn;
    b.B = terms[t].B; b.b_k = n; b.b_j = 1; b.b_b = nn;
    b.C = terms[t].C; b.c_i = n; b.c_j = 1; b.cj_in = n; b.cj_out = 0; b.c_b = nn;
    DTRY(gemm64(b, s));
  }
  return 0;
}

int thcsox_dyson_onebody(thcsox_dyson_t d, const double* gamma_dev, double* E1_host) {
  clear_error();
  if (d == nullptr || gamma_dev == nullptr || E1_host == nullptr)
    return dfail(THCSOX_EINVAL, "NULL argument");
  trace_ab<<<1, NT, 0, d->stream>>>(d->F, gamma_dev, d->n, d->scal);
  DTRY(hipGetLastError());
  DTRY(hipMemcpyAsync(E1_host, d->scal, sizeof(double), hipMemcpyDeviceToHost, d->stream));
  DTRY(hipStreamSynchronize(d->stream));
  return 0;
}

int thcsox_dyson_destroy(thcsox_dyson_t d) {
  if (d == nullptr) return 0;
  (void)hipStreamSynchronize(d->stream);
  delete d;
  return 0;
}

}  // extern "C"
