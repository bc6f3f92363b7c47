// Residual MLP of the learned warm start: training and inference on the GPU.
//
// The network maps the tau-profile of one THC pair's first-iteration
// self-energy (m values, divided by the pair's largest magnitude over tau) to
// the profile of the converged one (divided by the same number):
//     z1 = x W1^T + b1,  h1 = silu(z1)          W1: [H][m]
//     z2 = h1 W2^T + b2, h2 = silu(z2)          W2: [H][H]
//     y  = x + h2 W3^T + b3                     W3: [m][H]
// loss = mean over the batch and m of (y - target)^2, silu(z) = z / (1 + e^-z).
// Weights, activations and accumulation are FP32; the GEMMs run on FP32 matrix
// cores.  Parameters are one packed array: W1, b1, W2, b2, W3, b3.
#include <hip/hip_runtime.h>
#include <new>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/thcsox.h"
#include "error.hpp"
#include "mfma.hpp"

using namespace thcsox;

namespace {

constexpr int NT = 256;

// C(i,j) = alpha * sum_k A(i,k) B(k,j) + beta * C(i,j), FP32 matrix cores.
// A(i,k) = A[i*a_i + k*a_k], B(k,j) = B[k*b_k + j*b_j], C(i,j) = C[i*ldc + j].
struct G32 {
  int M, N, K;
  float alpha, beta;
  const float* A; int64_t a_i, a_k;
  const float* B; int64_t b_k, b_j;
  float* C; int64_t ldc;
};

__global__ __launch_bounds__(NT) void gemm32_kernel(G32 g) {
  constexpr int BK = 16, LD = 17;
  __shared__ float sA[64 * LD];
  __shared__ float sB[64 * LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  f4 acc[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
    for (int e = tid; e < 64 * BK; e += NT) {
      int i, k;
      if (g.a_k == 1) { i = e >> 4; k = e & 15; } else { i = e & 63; k = e >> 6; }
      const int gi = i0 + i, gk = k0 + k;
      sA[i * LD + k] = (gi < g.M && gk < g.K) ? g.A[(int64_t)gi * g.a_i + (int64_t)gk * g.a_k] : 0.f;
    }
#pragma unroll
    for (int e = tid; e < 64 * BK; e += NT) {
      int j, k;
      if (g.b_j == 1) { j = e & 63; k = e >> 6; } else { j = e >> 4; k = e & 15; }
      const int gj = j0 + j, gk = k0 + k;
      sB[j * LD + k] = (gj < g.N && gk < g.K) ? g.B[(int64_t)gk * g.b_k + (int64_t)gj * g.b_j] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      float a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = sA[(32 * wr + 16 * t + (lane & 15)) * LD + kk + (lane >> 4)];
        b[t] = sB[(32 * wc + 16 * t + (lane & 15)) * LD + kk + (lane >> 4)];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = mfma1(a[ti], b[tj], acc[ti][tj]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 32 * wr + 16 * ti + out_row<MODE_F32>(lane, r);
        const int j = j0 + 32 * wc + 16 * tj + (lane & 15);
        if (i < g.M && j < g.N) {
          float* c = g.C + (int64_t)i * g.ldc + j;
          *c = g.alpha * acc[ti][tj][r] + (g.beta != 0.f ? g.beta * *c : 0.f);
        }
      }
}

hipError_t gemm32(const G32& g, hipStream_t s) {
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
  gemm32_kernel<<<grid, NT, 0, s>>>(g);
  return hipGetLastError();
}

__device__ __forceinline__ float silu(float z) { return z / (1.f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.f / (1.f + __expf(-z));
  return s * (1.f + z * (1.f - s));
}

// z[b][j] += bias[j]; h = silu(z)
__global__ void bias_silu(float* z, float* h, const float* bias, int64_t rows, int cols) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < rows * cols; e += (int64_t)gridDim.x * NT) {
    const float v = z[e] + bias[e % cols];
    z[e] = v;
    h[e] = silu(v);
  }
}

// y[b][c] += x[b][c] + bias[c]
__global__ void residual_out(float* y, const float* x, const float* bias, int64_t rows, int cols) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < rows * cols; e += (int64_t)gridDim.x * NT)
    y[e] += x[e] + bias[e % cols];
}

// d = 2 (y - t) / N and per-block sums of (y - t)^2
__global__ void mse_grad(const float* y, const float* t, float* d, int64_t count, float inv_n,
                         double* partial) {
  __shared__ double red[NT];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < count; e += (int64_t)gridDim.x * NT) {
    const float r = y[e] - t[e];
    d[e] = 2.f * r * inv_n;
    s += (double)r * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sum_partials(const double* partial, int nb, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += partial[i];
    *out = s;
  }
}

// dz = dh * silu'(z)
__global__ void silu_back(const float* dh, const float* z, float* dz, int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < count; e += (int64_t)gridDim.x * NT)
    dz[e] = dh[e] * dsilu(z[e]);
}

// g[c] = sum_b d[b][c] (one thread per column, fixed order)
__global__ void colsum(const float* d, int64_t rows, int cols, float* g) {
  const int c = blockIdx.x * NT + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int64_t b = 0; b < rows; ++b) s += d[b * cols + c];
  g[c] = s;
}

__global__ void adam(float* p, const float* g, float* m1, float* m2, int64_t count, float lr,
                     float b1, float b2, float eps, float c1, float c2) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < count; e += (int64_t)gridDim.x * NT) {
    const float gi = g[e];
    const float a = b1 * m1[e] + (1.f - b1) * gi;
    const float v = b2 * m2[e] + (1.f - b2) * gi * gi;
    m1[e] = a;
    m2[e] = v;
    p[e] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
  }
}

// scale[e] = max_k |S[k][e]| over the m tau points of pair e (1 if all zero);
// consecutive threads take consecutive pairs, so every read of a tau slice is coalesced
__global__ void pair_scale_kernel(const double* S, int m, int64_t aa, double* scale) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < aa; e += (int64_t)gridDim.x * NT) {
    double mx = 0.0;
    for (int k = 0; k < m; ++k) mx = fmax(mx, fabs(S[(int64_t)k * aa + e]));
    scale[e] = mx > 0.0 ? mx : 1.0;
  }
}

// x[b][k] = S[k][pair_b] / scale[pair_b]; pair_b = pairs[b] (or b if pairs is null)
__global__ void pair_gather_kernel(const double* S, int m, int64_t aa, const double* scale,
                                   const int64_t* pairs, int64_t npairs, float* x) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < npairs * m;
       e += (int64_t)gridDim.x * NT) {
    const int64_t b = e / m;
    const int k = (int)(e % m);
    const int64_t pr = pairs ? pairs[b] : b;
    x[e] = (pr >= 0 && pr < aa) ? (float)(S[(int64_t)k * aa + pr] / scale[pr]) : 0.f;
  }
}

// S[k][pair] = y[pair][k] * scale[pair] for every pair
__global__ void pair_scatter_kernel(const float* y, int m, int64_t aa, const double* scale,
                                    double* S) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < aa * m; e += (int64_t)gridDim.x * NT) {
    const int k = (int)(e / aa);
    const int64_t pr = e % aa;
    S[e] = (double)y[pr * m + k] * scale[pr];
  }
}

unsigned blocks_for(int64_t n) {
  int64_t b = (n + NT - 1) / NT;
  return (unsigned)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

}  // namespace

struct thcsox_mlp_s {
  int m = 0, H = 0, maxb = 0;
  int64_t np = 0;
  int64_t oW1, ob1, oW2, ob2, oW3, ob3;
  hipStream_t stream = nullptr;
  float *P = nullptr, *Gr = nullptr, *M1 = nullptr, *M2 = nullptr;
  float *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *Y = nullptr, *D = nullptr;
  float *DH = nullptr, *DZ = nullptr;
  double *part = nullptr, *loss = nullptr;
  int step = 0;
  std::vector<void*> allocs;
  ~thcsox_mlp_s() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {

template <typename T>
int malloc_into(thcsox_mlp_s* q, T** p, size_t count) {
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, std::max<size_t>(16, count * sizeof(T)));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(THCSOX_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  q->allocs.push_back(v);
  *p = static_cast<T*>(v);
  return 0;
}

#define MTRY(expr)                                                                        \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return set_error(THCSOX_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// forward for rows [0, B) of x; activations kept for the backward pass
int forward(thcsox_mlp_s* q, const float* x, float* y, int B) {
  const hipStream_t s = q->stream;
  const int m = q->m, H = q->H;
  G32 g{};
  g.alpha = 1.f; g.beta = 0.f;
  g.M = B; g.N = H; g.K = m; g.A = x; g.a_i = m; g.a_k = 1;
  g.B = q->P + q->oW1; g.b_k = 1; g.b_j = m; g.C = q->Z1; g.ldc = H;
  MTRY(gemm32(g, s));
  bias_silu<<<blocks_for((int64_t)B * H), NT, 0, s>>>(q->Z1, q->H1, q->P + q->ob1, B, H);
  g.M = B; g.N = H; g.K = H; g.A = q->H1; g.a_i = H; g.a_k = 1;
  g.B = q->P + q->oW2; g.b_k = 1; g.b_j = H; g.C = q->Z2; g.ldc = H;
  MTRY(gemm32(g, s));
  bias_silu<<<blocks_for((int64_t)B * H), NT, 0, s>>>(q->Z2, q->H2, q->P + q->ob2, B, H);
  g.M = B; g.N = m; g.K = H; g.A = q->H2; g.a_i = H; g.a_k = 1;
  g.B = q->P + q->oW3; g.b_k = 1; g.b_j = H; g.C = y; g.ldc = m;
  MTRY(gemm32(g, s));
  residual_out<<<blocks_for((int64_t)B * m), NT, 0, s>>>(y, x, q->P + q->ob3, B, m);
  MTRY(hipGetLastError());
  return 0;
}

// gradients of the mean-squared loss into q->Gr, loss into q->loss
int backward(thcsox_mlp_s* q, const float* x, const float* t, int B) {
  const hipStream_t s = q->stream;
  const int m = q->m, H = q->H;
  const int64_t cnt = (int64_t)B * m;
  const unsigned nb = blocks_for(cnt);
  mse_grad<<<nb, NT, 0, s>>>(q->Y, t, q->D, cnt, 1.f / (float)cnt, q->part);
  sum_partials<<<1, 64, 0, s>>>(q->part, (int)nb, q->loss);
  G32 g{};
  g.alpha = 1.f; g.beta = 0.f;
  // gW3[c][j] = sum_b D[b][c] H2[b][j]
  g.M = m; g.N = H; g.K = B; g.A = q->D; g.a_i = 1; g.a_k = m;
  g.B = q->H2; g.b_k = H; g.b_j = 1; g.C = q->Gr + q->oW3; g.ldc = H;
  MTRY(gemm32(g, s));
  colsum<<<(m + NT - 1) / NT, NT, 0, s>>>(q->D, B, m, q->Gr + q->ob3);
  // dH2 = D W3
  g.M = B; g.N = H; g.K = m; g.A = q->D; g.a_i = m; g.a_k = 1;
  g.B = q->P + q->oW3; g.b_k = H; g.b_j = 1; g.C = q->DH; g.ldc = H;
  MTRY(gemm32(g, s));
  silu_back<<<blocks_for((int64_t)B * H), NT, 0, s>>>(q->DH, q->Z2, q->DZ, (int64_t)B * H);
  // gW2 = DZ2^T H1
  g.M = H; g.N = H; g.K = B; g.A = q->DZ; g.a_i = 1; g.a_k = H;
  g.B = q->H1; g.b_k = H; g.b_j = 1; g.C = q->Gr + q->oW2; g.ldc = H;
  MTRY(gemm32(g, s));
  colsum<<<(H + NT - 1) / NT, NT, 0, s>>>(q->DZ, B, H, q->Gr + q->ob2);
  // dH1 = DZ2 W2
  g.M = B; g.N = H; g.K = H; g.A = q->DZ; g.a_i = H; g.a_k = 1;
  g.B = q->P + q->oW2; g.b_k = H; g.b_j = 1; g.C = q->DH; g.ldc = H;
  MTRY(gemm32(g, s));
  silu_back<<<blocks_for((int64_t)B * H), NT, 0, s>>>(q->DH, q->Z1, q->DZ, (int64_t)B * H);
  // gW1 = DZ1^T X
  g.M = H; g.N = m; g.K = B; g.A = q->DZ; g.a_i = 1; g.a_k = H;
  g.B = x; g.b_k = m; g.b_j = 1; g.C = q->Gr + q->oW1; g.ldc = m;
  MTRY(gemm32(g, s));
  colsum<<<(H + NT - 1) / NT, NT, 0, s>>>(q->DZ, B, H, q->Gr + q->ob1);
  MTRY(hipGetLastError());
  return 0;
}

}  // namespace

extern "C" {

static int thcsox_mlp_create_impl(thcsox_mlp_t* out, int m, int hidden, int max_batch,
                      const float* params_host, void* hip_stream) {
  clear_error();
  if (out == nullptr || params_host == nullptr) return set_error(THCSOX_EINVAL, "NULL argument");
  *out = nullptr;
  if (m <= 0 || hidden <= 0 || max_batch <= 0) return set_error(THCSOX_EINVAL, "bad sizes");
  auto* q = new thcsox_mlp_s();
  q->m = m; q->H = hidden; q->maxb = max_batch;
  q->stream = static_cast<hipStream_t>(hip_stream);
  const int64_t H = hidden;
  q->oW1 = 0; q->ob1 = q->oW1 + H * m; q->oW2 = q->ob1 + H; q->ob2 = q->oW2 + H * H;
  q->oW3 = q->ob2 + H; q->ob3 = q->oW3 + (int64_t)m * H; q->np = q->ob3 + m;
  const int64_t B = max_batch;
  int rc;
  if ((rc = malloc_into(q, &q->P, q->np)) || (rc = malloc_into(q, &q->Gr, q->np)) ||
      (rc = malloc_into(q, &q->M1, q->np)) || (rc = malloc_into(q, &q->M2, q->np)) ||
      (rc = malloc_into(q, &q->Z1, B * H)) || (rc = malloc_into(q, &q->H1, B * H)) ||
      (rc = malloc_into(q, &q->Z2, B * H)) || (rc = malloc_into(q, &q->H2, B * H)) ||
      (rc = malloc_into(q, &q->Y, B * m)) || (rc = malloc_into(q, &q->D, B * m)) ||
      (rc = malloc_into(q, &q->DH, B * H)) || (rc = malloc_into(q, &q->DZ, B * H)) ||
      (rc = malloc_into(q, &q->part, 4096)) || (rc = malloc_into(q, &q->loss, 1))) {
    delete q;
    return rc;
  }
  hipError_t e;
  if ((e = hipMemcpyAsync(q->P, params_host, sizeof(float) * q->np, hipMemcpyHostToDevice,
                          q->stream)) ||
      (e = hipMemsetAsync(q->M1, 0, sizeof(float) * q->np, q->stream)) ||
      (e = hipMemsetAsync(q->M2, 0, sizeof(float) * q->np, q->stream)) ||
      (e = hipStreamSynchronize(q->stream))) {
    delete q;
    return set_error(THCSOX_EDEVICE, std::string("mlp create: ") + hipGetErrorString(e));
  }
  *out = q;
  return 0;
}

int thcsox_mlp_create(thcsox_mlp_t* out, int m, int hidden, int max_batch,
                      const float* params_host, void* hip_stream) {
  try {   // host containers: no exception may cross the C interface
    return thcsox_mlp_create_impl(out, m, hidden, max_batch, params_host, hip_stream);
  } catch (const std::bad_alloc&) {
    return set_error(THCSOX_ENOMEM, "host allocation failed");
  }
}

int thcsox_mlp_forward(thcsox_mlp_t q, const float* x_dev, float* y_dev, int batch) {
  clear_error();
  if (q == nullptr || x_dev == nullptr || y_dev == nullptr || batch < 0)
    return set_error(THCSOX_EINVAL, "bad argument");
  for (int b0 = 0; b0 < batch; b0 += q->maxb) {
    const int B = std::min(q->maxb, batch - b0);
    const int rc = forward(q, x_dev + (int64_t)b0 * q->m, y_dev + (int64_t)b0 * q->m, B);
    if (rc) return rc;
  }
  return 0;
}

int thcsox_mlp_gradients(thcsox_mlp_t q, const float* x_dev, const float* target_dev, int batch,
                         float* grads_host, double* loss_host) {
  clear_error();
  if (q == nullptr || x_dev == nullptr || target_dev == nullptr || batch <= 0 ||
      batch > q->maxb)
    return set_error(THCSOX_EINVAL, "bad argument (batch must be in 1..max_batch)");
  int rc = forward(q, x_dev, q->Y, batch);
  if (rc) return rc;
  if ((rc = backward(q, x_dev, target_dev, batch))) return rc;
  double sse = 0.0;
  MTRY(hipMemcpyAsync(&sse, q->loss, sizeof(double), hipMemcpyDeviceToHost, q->stream));
  if (grads_host)
    MTRY(hipMemcpyAsync(grads_host, q->Gr, sizeof(float) * q->np, hipMemcpyDeviceToHost,
                        q->stream));
  MTRY(hipStreamSynchronize(q->stream));
  if (loss_host) *loss_host = sse / ((double)batch * q->m);
  return 0;
}

int thcsox_mlp_train_step(thcsox_mlp_t q, const float* x_dev, const float* target_dev, int batch,
                          float lr, double* loss_host) {
  clear_error();
  if (q == nullptr || x_dev == nullptr || target_dev == nullptr || batch <= 0 ||
      batch > q->maxb)
    return set_error(THCSOX_EINVAL, "bad argument (batch must be in 1..max_batch)");
  int rc = forward(q, x_dev, q->Y, batch);
  if (rc) return rc;
  if ((rc = backward(q, x_dev, target_dev, batch))) return rc;
  q->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)q->step), c2 = 1.f - std::pow(b2, (float)q->step);
  adam<<<blocks_for(q->np), NT, 0, q->stream>>>(q->P, q->Gr, q->M1, q->M2, q->np, lr, b1, b2,
                                                1e-8f, c1, c2);
  MTRY(hipGetLastError());
  if (loss_host) {
    double sse = 0.0;
    MTRY(hipMemcpyAsync(&sse, q->loss, sizeof(double), hipMemcpyDeviceToHost, q->stream));
    MTRY(hipStreamSynchronize(q->stream));
    *loss_host = sse / ((double)batch * q->m);
  }
  return 0;
}

int thcsox_mlp_params(thcsox_mlp_t q, float* params_host) {
  clear_error();
  if (q == nullptr || params_host == nullptr) return set_error(THCSOX_EINVAL, "NULL argument");
  MTRY(hipMemcpyAsync(params_host, q->P, sizeof(float) * q->np, hipMemcpyDeviceToHost, q->stream));
  MTRY(hipStreamSynchronize(q->stream));
  return 0;
}

int thcsox_pair_scale(int m, int naux, const double* S_dev, double* scale_dev, void* hip_stream) {
  clear_error();
  if (m <= 0 || naux <= 0 || S_dev == nullptr || scale_dev == nullptr)
    return set_error(THCSOX_EINVAL, "bad argument");
  const int64_t aa = (int64_t)naux * naux;
  pair_scale_kernel<<<blocks_for(aa), NT, 0, static_cast<hipStream_t>(hip_stream)>>>(
      S_dev, m, aa, scale_dev);
  MTRY(hipGetLastError());
  return 0;
}

int thcsox_pair_gather(int m, int naux, const double* S_dev, const double* scale_dev,
                       const long long* pairs_dev, long long npairs, float* x_dev, void* hip_stream) {
  clear_error();
  const int64_t aa = (int64_t)naux * naux;
  if (m <= 0 || naux <= 0 || S_dev == nullptr || scale_dev == nullptr || x_dev == nullptr ||
      npairs < 0 || (pairs_dev == nullptr && npairs > aa))
    return set_error(THCSOX_EINVAL, "bad argument");
  pair_gather_kernel<<<blocks_for(npairs * m), NT, 0, static_cast<hipStream_t>(hip_stream)>>>(
      S_dev, m, aa, scale_dev, reinterpret_cast<const int64_t*>(pairs_dev), npairs, x_dev);
  MTRY(hipGetLastError());
  return 0;
}

int thcsox_pair_scatter(int m, int naux, const float* y_dev, const double* scale_dev,
                        double* S_dev, void* hip_stream) {
  clear_error();
  if (m <= 0 || naux <= 0 || S_dev == nullptr || scale_dev == nullptr || y_dev == nullptr)
    return set_error(THCSOX_EINVAL, "bad argument");
  const int64_t aa = (int64_t)naux * naux;
  pair_scatter_kernel<<<blocks_for(aa * m), NT, 0, static_cast<hipStream_t>(hip_stream)>>>(
      y_dev, m, aa, scale_dev, S_dev);
  MTRY(hipGetLastError());
  return 0;
}

int thcsox_mlp_destroy(thcsox_mlp_t q) {
  if (q == nullptr) return 0;
  (void)hipStreamSynchronize(q->stream);
  delete q;
  return 0;
}

}  // extern "C"
