// Convergence aids of the self-consistency loop (the paper's loop combines
// self-energies linearly: damping and DIIS): damping, and Pulay DIIS on the
// self-energy residual r = Sigma_out - Sigma_in.  Device arrays of doubles; the
// (depth + 1)^2 DIIS system is solved on the host.
#include <hip/hip_runtime.h>
#include <new>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/thcsox.h"
#include "error.hpp"

using namespace thcsox;

namespace {

constexpr int NT = 256;
constexpr int DOT_BLOCKS = 1024;   // fixed, so the summation order is fixed

// y = a x + b y
__global__ __launch_bounds__(NT) void axpby_kernel(int64_t n, double a, const double* __restrict__ x,
                                                   double b, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    y[i] = fma(a, x[i], b * y[i]);
}

// y = a x (y is not read)
__global__ __launch_bounds__(NT) void scale_kernel(int64_t n, double a, const double* __restrict__ x,
                                                   double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    y[i] = a * x[i];
}

// z = x - y
__global__ __launch_bounds__(NT) void sub_kernel(int64_t n, const double* __restrict__ x,
                                                 const double* __restrict__ y, double* __restrict__ z) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    z[i] = x[i] - y[i];
}

// part[b] = sum over the grid-stride elements of workgroup b of x y (fixed order)
__global__ __launch_bounds__(NT) void dot_partials(int64_t n, const double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   double* __restrict__ part) {
  __shared__ double red[NT];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    acc = fma(x[i], y[i], acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NT) void sum_partials(const double* __restrict__ part, int np,
                                                   double* __restrict__ out) {
  __shared__ double red[NT];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += NT) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (n + NT - 1) / NT));
}

int lfail(int code, const std::string& m) { return set_error(code, m); }

#define LTRY(expr)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return lfail(THCSOX_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

bool is_device(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Solve the bordered system [B 1; 1^T 0] [c; l] = [0; 1] (k x k block B) by
// Gaussian elimination with partial pivoting; false if it is singular.
bool solve_bordered(const std::vector<double>& B, int k, std::vector<double>& c) {
  const int m = k + 1;
  std::vector<double> M((size_t)m * (m + 1), 0.0);
  double scale = 0.0;
  for (int i = 0; i < k; ++i) scale = std::max(scale, std::fabs(B[(size_t)i * k + i]));
  if (!(scale > 0.0)) scale = 1.0;
  for (int i = 0; i < k; ++i) {
    for (int j = 0; j < k; ++j) M[(size_t)i * (m + 1) + j] = B[(size_t)i * k + j] / scale;
    M[(size_t)i * (m + 1) + k] = 1.0;
    M[(size_t)k * (m + 1) + i] = 1.0;
  }
  M[(size_t)k * (m + 1) + m] = 1.0;   // right-hand side [0 ... 0 1]
  for (int col = 0; col < m; ++col) {
    int p = col;
    for (int r = col + 1; r < m; ++r)
      if (std::fabs(M[(size_t)r * (m + 1) + col]) > std::fabs(M[(size_t)p * (m + 1) + col])) p = r;
    if (!(std::fabs(M[(size_t)p * (m + 1) + col]) > 1e-14)) return false;
    if (p != col)
      for (int j = 0; j <= m; ++j) std::swap(M[(size_t)p * (m + 1) + j], M[(size_t)col * (m + 1) + j]);
    for (int r = 0; r < m; ++r) {
      if (r == col) continue;
      const double f = M[(size_t)r * (m + 1) + col] / M[(size_t)col * (m + 1) + col];
      for (int j = col; j <= m; ++j) M[(size_t)r * (m + 1) + j] -= f * M[(size_t)col * (m + 1) + j];
    }
  }
  c.assign(k, 0.0);
  for (int i = 0; i < k; ++i) c[i] = M[(size_t)i * (m + 1) + m] / M[(size_t)i * (m + 1) + i];
  return true;
}

}  // namespace

struct thcsox_diis_s {
  int64_t len = 0;     // doubles per extrapolated vector
  int64_t len_e = 0;   // doubles per residual (len for the Pulay residual)
  bool explicit_residual = false;   // residuals given by the caller (thcsox_diis_step_res)
  int depth = 0;
  hipStream_t stream = nullptr;
  std::vector<double*> in, res;   // ring of device arrays
  std::vector<int> order;         // ring slots, oldest first
  std::vector<double> dots;       // [depth][depth] <res_slot_i, res_slot_j>
  double* part = nullptr;         // [DOT_BLOCKS]
  double* scalar = nullptr;
  ~thcsox_diis_s() {
    for (double* p : in) (void)hipFree(p);
    for (double* p : res) (void)hipFree(p);
    (void)hipFree(part);
    (void)hipFree(scalar);
  }
};

namespace {
int dot_dev(thcsox_diis_s* d, const double* x, const double* y, double* out) {
  dot_partials<<<DOT_BLOCKS, NT, 0, d->stream>>>(d->len_e, x, y, d->part);
  LTRY(hipGetLastError());
  sum_partials<<<1, NT, 0, d->stream>>>(d->part, DOT_BLOCKS, d->scalar);
  LTRY(hipGetLastError());
  LTRY(hipMemcpyAsync(out, d->scalar, sizeof(double), hipMemcpyDeviceToHost, d->stream));
  LTRY(hipStreamSynchronize(d->stream));
  return 0;
}
}  // namespace

extern "C" {

int thcsox_mix(int64_t len, double alpha, const double* sigma_out, double* sigma_io,
               void* hip_stream) {
  clear_error();
  if (len < 0 || sigma_out == nullptr || sigma_io == nullptr)
    return lfail(THCSOX_EINVAL, "need len >= 0 and non-NULL arrays");
  if (len == 0) return 0;
  if (!is_device(sigma_out) || !is_device(sigma_io))
    return lfail(THCSOX_ENOTDEV, "arrays must be device memory");
  axpby_kernel<<<grid_for(len), NT, 0, static_cast<hipStream_t>(hip_stream)>>>(
      len, 1.0 - alpha, sigma_out, alpha, sigma_io);
  LTRY(hipGetLastError());
  return 0;
}

static int thcsox_diis_create_impl(thcsox_diis_t* out, int64_t len, int64_t len_e,
                                   bool explicit_residual, int depth, void* hip_stream) {
  clear_error();
  if (out == nullptr) return lfail(THCSOX_EINVAL, "out is NULL");
  *out = nullptr;
  if (len <= 0 || len_e <= 0 || depth < 1)
    return lfail(THCSOX_EINVAL, "need len > 0, len_e > 0 and depth >= 1");
  auto* d = new thcsox_diis_s();
  d->len = len;
  d->len_e = len_e;
  d->explicit_residual = explicit_residual;
  d->depth = depth;
  d->stream = static_cast<hipStream_t>(hip_stream);
  d->dots.assign((size_t)depth * depth, 0.0);
  auto alloc = [&](double** p, size_t n) -> bool {
    if (hipMalloc(p, n * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return false;
    }
    return true;
  };
  bool ok = alloc(&d->part, DOT_BLOCKS) && alloc(&d->scalar, 1);
  for (int i = 0; ok && i < depth; ++i) {
    double *a = nullptr, *b = nullptr;
    ok = alloc(&a, (size_t)len) && alloc(&b, (size_t)len_e);
    if (a) d->in.push_back(a);
    if (b) d->res.push_back(b);
  }
  if (!ok) {
    delete d;
    return lfail(THCSOX_ENOMEM, "hipMalloc failed for the DIIS history");
  }
  *out = d;
  return 0;
}

int thcsox_diis_create(thcsox_diis_t* out, int64_t len, int depth, void* hip_stream) {
  try {   // host containers: no exception may cross the C interface
    return thcsox_diis_create_impl(out, len, len, false, depth, hip_stream);
  } catch (const std::bad_alloc&) {
    return lfail(THCSOX_ENOMEM, "host allocation failed");
  }
}

int thcsox_diis_create_res(thcsox_diis_t* out, int64_t len, int64_t len_res, int depth,
                           void* hip_stream) {
  try {
    return thcsox_diis_create_impl(out, len, len_res, true, depth, hip_stream);
  } catch (const std::bad_alloc&) {
    return lfail(THCSOX_ENOMEM, "host allocation failed");
  }
}

// the slot for a new history entry: a free one, else the oldest
static int take_slot(thcsox_diis_s* d) {
  int slot;
  if ((int)d->order.size() < d->depth) {
    slot = (int)d->order.size();
  } else {
    slot = d->order.front();
    d->order.erase(d->order.begin());
  }
  return slot;
}

static int diis_extrapolate(thcsox_diis_s* d, int slot, double* sigma_next, int* n_used_out);

static int thcsox_diis_step_impl(thcsox_diis_t d, const double* sigma_in, const double* sigma_out,
                     double* sigma_next, int* n_used_out) {
  clear_error();
  if (d == nullptr || sigma_in == nullptr || sigma_out == nullptr || sigma_next == nullptr)
    return lfail(THCSOX_EINVAL, "NULL argument");
  if (d->explicit_residual)
    return lfail(THCSOX_EINVAL, "this history takes explicit residuals (thcsox_diis_step_res)");
  if (sigma_next == sigma_out) return lfail(THCSOX_EINVAL, "sigma_next may not alias sigma_out");
  if (!is_device(sigma_in) || !is_device(sigma_out) || !is_device(sigma_next))
    return lfail(THCSOX_ENOTDEV, "arrays must be device memory");
  const hipStream_t s = d->stream;
  const unsigned gb = grid_for(d->len);
  const int slot = take_slot(d);
  LTRY(hipMemcpyAsync(d->in[slot], sigma_in, sizeof(double) * d->len, hipMemcpyDeviceToDevice, s));
  sub_kernel<<<gb, NT, 0, s>>>(d->len, sigma_out, sigma_in, d->res[slot]);
  LTRY(hipGetLastError());
  d->order.push_back(slot);
  return diis_extrapolate(d, slot, sigma_next, n_used_out);
}

static int thcsox_diis_step_res_impl(thcsox_diis_t d, const double* residual,
                                     const double* sigma_out, double* sigma_next,
                                     int* n_used_out) {
  clear_error();
  if (d == nullptr || residual == nullptr || sigma_out == nullptr || sigma_next == nullptr)
    return lfail(THCSOX_EINVAL, "NULL argument");
  if (!d->explicit_residual)
    return lfail(THCSOX_EINVAL, "this history forms its own residuals (thcsox_diis_step)");
  if (!is_device(residual) || !is_device(sigma_out) || !is_device(sigma_next))
    return lfail(THCSOX_ENOTDEV, "arrays must be device memory");
  const hipStream_t s = d->stream;
  const int slot = take_slot(d);
  // the history keeps Sigma_out itself (the ring named `in`) and the residual
  LTRY(hipMemcpyAsync(d->in[slot], sigma_out, sizeof(double) * d->len, hipMemcpyDeviceToDevice, s));
  LTRY(hipMemcpyAsync(d->res[slot], residual, sizeof(double) * d->len_e, hipMemcpyDeviceToDevice, s));
  d->order.push_back(slot);
  return diis_extrapolate(d, slot, sigma_next, n_used_out);
}

// New row of residual dot products for `slot`, coefficients over the newest
// entries (the oldest dropped while the bordered system is singular), and
// sigma_next = sum_i c_i Sigma_out_i.  Synchronises the stream.
static int diis_extrapolate(thcsox_diis_s* d, int slot, double* sigma_next, int* n_used_out) {
  const hipStream_t s = d->stream;
  const unsigned gb = grid_for(d->len);
  // new row of residual dot products
  for (int o : d->order) {
    double v;
    int rc = dot_dev(d, d->res[slot], d->res[o], &v);
    if (rc) return rc;
    d->dots[(size_t)slot * d->depth + o] = v;
    d->dots[(size_t)o * d->depth + slot] = v;
  }
  // coefficients over the newest entries; drop the oldest while singular
  std::vector<double> c;
  int first = 0;
  const int total = (int)d->order.size();
  for (; first < total; ++first) {
    const int k = total - first;
    std::vector<double> B((size_t)k * k);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j)
        B[(size_t)i * k + j] = d->dots[(size_t)d->order[first + i] * d->depth + d->order[first + j]];
    if (solve_bordered(B, k, c)) break;
  }
  if (first == total) return lfail(THCSOX_ENONFINITE, "DIIS system is singular");
  // sigma_next = sum_i c_i Sigma_out_i: (in_i + res_i) for the Pulay residual,
  // the stored Sigma_out_i for explicit residuals; sigma_next may alias the
  // caller's inputs, whose copies are already in the history
  const int k = total - first;
  for (int i = 0; i < k; ++i) {
    const int o = d->order[first + i];
    if (i == 0) scale_kernel<<<gb, NT, 0, s>>>(d->len, c[i], d->in[o], sigma_next);
    else axpby_kernel<<<gb, NT, 0, s>>>(d->len, c[i], d->in[o], 1.0, sigma_next);
    LTRY(hipGetLastError());
    if (!d->explicit_residual) {
      axpby_kernel<<<gb, NT, 0, s>>>(d->len, c[i], d->res[o], 1.0, sigma_next);
      LTRY(hipGetLastError());
    }
  }
  LTRY(hipStreamSynchronize(s));
  if (n_used_out) *n_used_out = k;
  return 0;
}

int thcsox_diis_step(thcsox_diis_t d, const double* sigma_in, const double* sigma_out,
                     double* sigma_next, int* n_used_out) {
  try {   // host containers: no exception may cross the C interface
    return thcsox_diis_step_impl(d, sigma_in, sigma_out, sigma_next, n_used_out);
  } catch (const std::bad_alloc&) {
    return lfail(THCSOX_ENOMEM, "host allocation failed");
  }
}

int thcsox_diis_step_res(thcsox_diis_t d, const double* residual, const double* sigma_out,
                         double* sigma_next, int* n_used_out) {
  try {
    return thcsox_diis_step_res_impl(d, residual, sigma_out, sigma_next, n_used_out);
  } catch (const std::bad_alloc&) {
    return lfail(THCSOX_ENOMEM, "host allocation failed");
  }
}

int thcsox_diis_destroy(thcsox_diis_t d) {
  if (d == nullptr) return 0;
  (void)hipStreamSynchronize(d->stream);
  delete d;
  return 0;
}

}  // extern "C"
