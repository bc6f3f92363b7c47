// The IR (intermediate representation) basis of the fermionic logistic kernel
// and its sparse-sampling grids, built on the host (the grids the paper's loop
// runs on; computational-details section and the references it cites).
//
//   K(x, y) = exp(-Lambda y (x + 1) / 2) / (1 + exp(-Lambda y)),   x, y in [-1, 1],
//   x = 2 tau / beta - 1, omega = wmax y, Lambda = beta wmax.
//
// K(-x, -y) = K(x, y), so its singular functions are even or odd and the
// expansion splits into two half-domain problems on [0, 1]^2 with the kernels
// K(x, y) + K(x, -y) (even) and K(x, y) - K(x, -y) (odd).  Each is discretised
// by Gauss-Legendre rules on segments that halve towards x = 1 and towards
// y = 0 (K varies on the scale 1 / Lambda there), weighted by the square roots
// of the quadrature weights, and decomposed by a one-sided Jacobi SVD, which
// rotates column pairs until they are orthogonal.  The functions are then
// evaluated anywhere by the Nystrom form u_l(x) = (1 / s_l) int K(x, y) v_l(y) dy,
// and their Matsubara transforms come from the closed form of each term:
// int_0^beta exp(i w_n tau) K(tau, omega) dtau = 1 / (omega - i w_n).
//
// Sampling: the tau points are the roots of u_L (the first function past the
// cut s_l / s_0 >= eps), the Matsubara points the n >= 0 where the transform of
// one of u_{L-3} .. u_L changes sign, and n = 0.  (At low n the highest
// functions' transforms are at their FP64 noise level; the sign changes of the
// top two alone leave some fits badly conditioned, the top four do not.)
#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/thcsox.h"
#include "error.hpp"

struct thcsox_ir_s {
  int L = 0, nf = 0;
  std::vector<double> tau, Wf, Wb, coef, sign, sv;
  std::vector<int> freq;
};

namespace thcsox {
namespace {

constexpr int IRQ = 16;   // Gauss-Legendre nodes per segment

void gauss_rule(std::vector<double>& t, std::vector<double>& w) {
  const int q = IRQ;
  t.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    t[q - 1 - i] = z;
    w[q - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// nodes and weights of the composite rule over the given breakpoints
void composite(const std::vector<double>& br, std::vector<double>& x, std::vector<double>& w) {
  std::vector<double> t, wt;
  gauss_rule(t, wt);
  x.clear();
  w.clear();
  for (size_t s = 0; s + 1 < br.size(); ++s) {
    const double h = 0.5 * (br[s + 1] - br[s]), c = 0.5 * (br[s + 1] + br[s]);
    for (int i = 0; i < IRQ; ++i) {
      x.push_back(c + h * t[i]);
      w.push_back(h * wt[i]);
    }
  }
}

double kern(double x, double y, double lam) {
  if (y >= 0) return std::exp(-lam * y * (x + 1.0) / 2.0) / (1.0 + std::exp(-lam * y));
  return std::exp(lam * y * (1.0 - x) / 2.0) / (1.0 + std::exp(lam * y));
}

// One-sided Jacobi SVD of the M x N matrix A (column-major, column j at
// A + j M): column pairs are rotated until orthogonal, so that A V = U diag(s).
// Returns s and V (N x N, column-major); A is overwritten by U diag(s).
// False if a sweep still rotated after the sweep limit (not converged).
bool jacobi_svd(int M, int N, std::vector<double>& A, std::vector<double>& V,
                std::vector<double>& s) {
  V.assign((size_t)N * N, 0.0);
  for (int j = 0; j < N; ++j) V[(size_t)j * N + j] = 1.0;
  std::vector<double> nrm(N);
  bool converged = false;
  for (int sweep = 0; sweep < 80 && !converged; ++sweep) {
    for (int j = 0; j < N; ++j) {
      double a = 0.0;
      const double* c = &A[(size_t)j * M];
      for (int r = 0; r < M; ++r) a += c[r] * c[r];
      nrm[j] = a;
    }
    bool rotated = false;
    for (int i = 0; i < N - 1; ++i)
      for (int j = i + 1; j < N; ++j) {
        double* ci = &A[(size_t)i * M];
        double* cj = &A[(size_t)j * M];
        double g = 0.0;
        for (int r = 0; r < M; ++r) g += ci[r] * cj[r];
        const double a = nrm[i], b = nrm[j];
        if (g == 0.0 || std::fabs(g) <= 4e-16 * std::sqrt(a * b)) continue;
        rotated = true;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int r = 0; r < M; ++r) {
          const double x = ci[r], y = cj[r];
          ci[r] = c * x - sn * y;
          cj[r] = sn * x + c * y;
        }
        double* vi = &V[(size_t)i * N];
        double* vj = &V[(size_t)j * N];
        for (int r = 0; r < N; ++r) {
          const double x = vi[r], y = vj[r];
          vi[r] = c * x - sn * y;
          vj[r] = sn * x + c * y;
        }
        nrm[i] = a - t * g;
        nrm[j] = b + t * g;
      }
    converged = !rotated;
  }
  s.assign(N, 0.0);
  for (int j = 0; j < N; ++j) {
    double a = 0.0;
    const double* c = &A[(size_t)j * M];
    for (int r = 0; r < M; ++r) a += c[r] * c[r];
    s[j] = std::sqrt(a);
  }
  return converged;
}

// Pseudo-inverse of the M x N row-major matrix B (M >= N, full column rank) by
// the Jacobi SVD: pinv = V diag(1/s) U^T, returned N x M row-major (empty if
// the SVD did not converge).  *cond (if given) receives s_max / s_min.
std::vector<double> pinv_svd(const std::vector<double>& B, int M, int N, double* cond = nullptr) {
  std::vector<double> A((size_t)M * N), V, s;
  for (int r = 0; r < M; ++r)
    for (int c = 0; c < N; ++c) A[(size_t)c * M + r] = B[(size_t)r * N + c];
  if (!jacobi_svd(M, N, A, V, s)) return {};
  if (cond) {
    const double smax = *std::max_element(s.begin(), s.end());
    const double smin = *std::min_element(s.begin(), s.end());
    *cond = smin > 0 ? smax / smin : INFINITY;
  }
  std::vector<double> P((size_t)N * M, 0.0);
  for (int k = 0; k < N; ++k) {
    if (s[k] == 0.0) continue;
    const double inv2 = 1.0 / (s[k] * s[k]);   // column k of A is u_k s_k
    for (int i = 0; i < N; ++i) {
      const double vik = V[(size_t)k * N + i] * inv2;
      for (int r = 0; r < M; ++r) P[(size_t)i * M + r] += vik * A[(size_t)k * M + r];
    }
  }
  return P;
}

// One singular function: parity (0 even, 1 odd), singular value, and the
// Nystrom weights c_j = sqrt(w_j) V_jl / (s_l sqrt 2) on the half grid y_j.
struct Fn {
  int parity;
  double s;
  std::vector<double> c;
};

struct Basis {
  double beta, wmax, lam;
  std::vector<double> y;   // half grid in y
  std::vector<double> xh;  // half grid in x (root brackets)
  std::vector<Fn> fn;      // sorted by s, descending
  // u_l(x), x in [-1, 1]
  double u(int l, double x) const {
    const Fn& f = fn[l];
    double acc = 0.0;
    const double sg = f.parity ? -1.0 : 1.0;
    for (size_t j = 0; j < y.size(); ++j)
      acc += f.c[j] * (kern(x, y[j], lam) + sg * kern(x, -y[j], lam));
    return acc;
  }
  double u_tau(int l, double tau) const {
    return std::sqrt(2.0 / beta) * u(l, 2.0 * tau / beta - 1.0);
  }
  // the transform at i nu: purely imaginary (even) or purely real (odd)
  void uhat(int l, long n, double* re, double* im) const {
    const Fn& f = fn[l];
    const double nu = (2.0 * n + 1.0) * M_PI / beta;
    double acc = 0.0;
    for (size_t j = 0; j < y.size(); ++j) {
      const double om = wmax * y[j], den = om * om + nu * nu;
      acc += f.c[j] * (f.parity ? 2.0 * om / den : 2.0 * nu / den);
    }
    acc *= std::sqrt(2.0 / beta);
    *re = f.parity ? acc : 0.0;
    *im = f.parity ? 0.0 : acc;
  }
  double uhat_part(int l, long n) const {
    double re, im;
    uhat(l, n, &re, &im);
    return fn[l].parity ? re : im;
  }
};

int build_basis(double beta, double wmax, double eps, Basis& B, int& L) {
  B.beta = beta;
  B.wmax = wmax;
  B.lam = beta * wmax;
  const double hmin = 0.25 / B.lam;
  std::vector<double> bx{0.0}, by{0.0};
  // x: 0, 1/2, 3/4, ..., 1 - 2^-k, 1 (halving towards the edge)
  for (double h = 0.5; ; h *= 0.5) {
    bx.push_back(1.0 - h);
    if (h <= hmin) break;
  }
  bx.push_back(1.0);
  // y: 0, 2^-k, ..., 1/4, 1/2, 1 (halving towards the centre)
  std::vector<double> d;
  for (double h = 1.0; ; h *= 0.5) {
    d.push_back(h);
    if (h <= hmin) break;
  }
  for (auto it = d.rbegin(); it != d.rend(); ++it) by.push_back(*it);
  std::vector<double> wx, wy;
  composite(bx, B.xh, wx);
  composite(by, B.y, wy);
  const int M = (int)B.xh.size(), N = (int)B.y.size();
  std::vector<Fn> all;
  for (int par = 0; par < 2; ++par) {
    std::vector<double> A((size_t)M * N), V, s;
    const double sg = par ? -1.0 : 1.0;
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < M; ++i)
        A[(size_t)j * M + i] = std::sqrt(wx[i] * wy[j]) *
                               (kern(B.xh[i], B.y[j], B.lam) + sg * kern(B.xh[i], -B.y[j], B.lam));
    if (!jacobi_svd(M, N, A, V, s))
      return set_error(THCSOX_EINVAL, "IR basis: the Jacobi SVD did not converge");
    for (int k = 0; k < N; ++k) {
      Fn f;
      f.parity = par;
      f.s = s[k];
      f.c.resize(N);
      for (int j = 0; j < N; ++j)
        f.c[j] = s[k] > 0 ? std::sqrt(wy[j]) * V[(size_t)k * N + j] / (s[k] * std::sqrt(2.0)) : 0.0;
      all.push_back(std::move(f));
    }
  }
  std::sort(all.begin(), all.end(), [](const Fn& a, const Fn& b) { return a.s > b.s; });
  L = 0;
  while (L < (int)all.size() && all[L].s >= eps * all[0].s) ++L;
  if (L + 1 > (int)all.size() || L < 4)
    return set_error(THCSOX_EINVAL, "IR basis: eps outside the range the discretisation resolves");
  all.resize(L + 1);
  B.fn = std::move(all);
  // sign convention: u_l(x = 1) > 0
  for (int l = 0; l <= L; ++l)
    if (B.u(l, 1.0) < 0)
      for (double& c : B.fn[l].c) c = -c;
  return 0;
}

// the roots of u_L on (-1, 1), ascending (mirror-symmetric by parity)
int tau_roots(const Basis& B, int L, std::vector<double>& xr) {
  // brackets: the half-grid nodes and the midpoints between them
  std::vector<double> xs{0.0};
  for (size_t i = 0; i < B.xh.size(); ++i) {
    const double prev = xs.back();
    xs.push_back(0.5 * (prev + B.xh[i]));
    xs.push_back(B.xh[i]);
  }
  xs.push_back(1.0);
  std::vector<double> pos;
  double fa = B.u(L, xs[0]);
  for (size_t i = 0; i + 1 < xs.size(); ++i) {
    const double fb = B.u(L, xs[i + 1]);
    {
      // a sign change strictly inside (a zero at x = 0 is the odd-parity root added below)
      if ((fa < 0) != (fb < 0) && fa != 0.0 && fb != 0.0) {
        double a = xs[i], b = xs[i + 1], ga = fa;
        for (int it = 0; it < 200; ++it) {
          const double mid = 0.5 * (a + b);
          if (mid <= a || mid >= b) break;
          const double gm = B.u(L, mid);
          if ((gm < 0) == (ga < 0)) {
            a = mid;
            ga = gm;
          } else {
            b = mid;
          }
        }
        pos.push_back(0.5 * (a + b));
      }
    }
    fa = fb;
  }
  // u_L has parity (-1)^L: an odd L adds the root at x = 0
  xr.clear();
  for (auto it = pos.rbegin(); it != pos.rend(); ++it) xr.push_back(-*it);
  if (B.fn[L].parity == 1) xr.push_back(0.0);
  for (double p : pos) xr.push_back(p);
  if ((int)xr.size() != L)
    return set_error(THCSOX_EINVAL, "IR basis: u_L has " + std::to_string(xr.size()) +
                                        " roots, expected " + std::to_string(L));
  return 0;
}

std::vector<int> matsubara_points(const Basis& B, int L) {
  const long nmax = (long)(10.0 * B.lam / (2.0 * M_PI)) + 10;
  std::vector<int> pts{0};
  for (int l = L - 3; l <= L; ++l) {
    double prev = B.uhat_part(l, 0);
    for (long n = 1; n <= nmax; ++n) {
      const double cur = B.uhat_part(l, n);
      if ((prev < 0 && cur > 0) || (prev > 0 && cur < 0)) pts.push_back((int)n);
      prev = cur;
    }
  }
  std::sort(pts.begin(), pts.end());
  pts.erase(std::unique(pts.begin(), pts.end()), pts.end());
  return pts;
}

}  // namespace
}  // namespace thcsox

using namespace thcsox;

namespace {
int ir_create(thcsox_ir_t* out, double beta, double wmax, double eps) {
  if (!(beta > 0.0) || !(wmax > 0.0) || !(eps >= 1e-13 && eps < 1.0) || !(beta * wmax <= 1e7))
    return set_error(THCSOX_EINVAL, "need beta > 0, wmax > 0, beta wmax <= 1e7, 1e-13 <= eps < 1");
  Basis B;
  int L = 0, rc;
  if ((rc = build_basis(beta, wmax, eps, B, L))) return rc;
  std::vector<double> xr;
  if ((rc = tau_roots(B, L, xr))) return rc;
  auto* g = new (std::nothrow) thcsox_ir_s();
  if (g == nullptr) return set_error(THCSOX_ENOMEM, "host allocation failed");
  g->L = L;
  g->tau.resize(L);
  for (int k = 0; k < L; ++k) g->tau[k] = 0.5 * beta * (xr[k] + 1.0);
  g->freq = matsubara_points(B, L);
  const int nf = (int)g->freq.size();
  g->nf = nf;
  if (2 * nf < L) {
    delete g;
    return set_error(THCSOX_EINVAL, "IR basis: too few Matsubara sampling points");
  }
  // Ut[k][l] = u_l(tau_k); the coefficients from tau values: C = Ut^-1
  std::vector<double> Ut((size_t)L * L);
  for (int k = 0; k < L; ++k)
    for (int l = 0; l < L; ++l) Ut[(size_t)k * L + l] = B.u_tau(l, g->tau[k]);
  double cond_t = 0.0, cond_w = 0.0;
  g->coef = pinv_svd(Ut, L, L, &cond_t);   // [L][L]
  if (g->coef.empty()) {
    delete g;
    return set_error(THCSOX_EINVAL, "IR basis: the Jacobi SVD of the tau sampling matrix did not converge");
  }
  // [Re; Im] transform rows: H[j][l] = Re uhat_l(n_j), H[nf + j][l] = Im uhat_l(n_j)
  std::vector<double> H((size_t)2 * nf * L);
  for (int j = 0; j < nf; ++j)
    for (int l = 0; l < L; ++l) {
      double re, im;
      B.uhat(l, g->freq[j], &re, &im);
      H[(size_t)j * L + l] = re;
      H[(size_t)(nf + j) * L + l] = im;
    }
  // forward: F(i w) = H C F(tau)
  g->Wf.assign((size_t)2 * nf * L, 0.0);
  for (int r = 0; r < 2 * nf; ++r)
    for (int l = 0; l < L; ++l) {
      const double h = H[(size_t)r * L + l];
      if (h == 0.0) continue;
      for (int k = 0; k < L; ++k) g->Wf[(size_t)r * L + k] += h * g->coef[(size_t)l * L + k];
    }
  // backward: coefficients = pinv(H) [Re; Im] F, then F(tau_k) and F(beta^-)
  const std::vector<double> P = pinv_svd(H, 2 * nf, L, &cond_w);   // [L][2 nf]
  if (P.empty()) {
    delete g;
    return set_error(THCSOX_EINVAL, "IR basis: the Jacobi SVD of the frequency sampling matrix did not converge");
  }
  // the sampling rule can fail where the highest functions' transforms are at
  // their noise level (too small an eps for FP64 at this Lambda): refuse a grid
  // whose fits would amplify errors by more than 1e4
  if (!(cond_t <= 1e4) || !(cond_w <= 1e4)) {
    delete g;
    return set_error(THCSOX_EINVAL, "IR basis: ill-conditioned sampling (condition numbers " +
                                        std::to_string(cond_t) + " in tau, " + std::to_string(cond_w) +
                                        " in frequency); choose a larger eps");
  }
  g->Wb.assign((size_t)(L + 1) * 2 * nf, 0.0);
  for (int k = 0; k <= L; ++k) {
    for (int l = 0; l < L; ++l) {
      const double ul = k < L ? Ut[(size_t)k * L + l] : B.u_tau(l, beta);
      for (int r = 0; r < 2 * nf; ++r) g->Wb[(size_t)k * 2 * nf + r] += ul * P[(size_t)l * 2 * nf + r];
    }
  }
  g->sign.resize(L);
  g->sv.resize(L);
  for (int l = 0; l < L; ++l) {
    g->sign[l] = B.fn[l].parity ? -1.0 : 1.0;
    g->sv[l] = B.fn[l].s * std::sqrt(0.5 * beta * wmax);   // in tau and omega units
  }
  *out = g;
  return 0;
}
}  // namespace

extern "C" {

int thcsox_ir_create(thcsox_ir_t* out, double beta, double wmax, double eps) {
  clear_error();
  if (out == nullptr) return set_error(THCSOX_EINVAL, "out is NULL");
  *out = nullptr;
  // host vectors throughout: no exception may cross the C interface
  try {
    return ir_create(out, beta, wmax, eps);
  } catch (const std::bad_alloc&) {
    return set_error(THCSOX_ENOMEM, "host allocation failed");
  }
}

int thcsox_ir_sizes(thcsox_ir_t g, int* ntau, int* nfreq) {
  clear_error();
  if (g == nullptr || ntau == nullptr || nfreq == nullptr)
    return set_error(THCSOX_EINVAL, "NULL argument");
  *ntau = g->L;
  *nfreq = g->nf;
  return 0;
}

int thcsox_ir_get(thcsox_ir_t g, double* tau, int* freq_n, double* Wf, double* Wb, double* coef,
                  double* sign, double* sv) {
  clear_error();
  if (g == nullptr) return set_error(THCSOX_EINVAL, "NULL grid");
  auto put = [](const std::vector<double>& v, double* d) {
    if (d) std::copy(v.begin(), v.end(), d);
  };
  put(g->tau, tau);
  if (freq_n) std::copy(g->freq.begin(), g->freq.end(), freq_n);
  put(g->Wf, Wf);
  put(g->Wb, Wb);
  put(g->coef, coef);
  put(g->sign, sign);
  put(g->sv, sv);
  return 0;
}

int thcsox_ir_destroy(thcsox_ir_t g) {
  delete g;
  return 0;
}

}  // extern "C"
