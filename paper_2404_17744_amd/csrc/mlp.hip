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

// ---------------------------------------------------------------------------
// Inference with bf16 weights: one fused kernel per 64 rows on the bf16 matrix
// cores (16x16x32, FP32 accumulation); the hidden activations never leave LDS.
// Each layer's input (x, h1, h2) is rounded to bf16 (nearest, ties to even);
// bias, silu and the residual add on the exact FP32 x stay in FP32.
//
// Eight waves: in layers 1 and 2 wave w owns the hidden units [16 HT w,
// 16 HT (w + 1)) of all 64 rows, taking the weight rows as the MFMA's first
// operand and the activation rows (from LDS) as its second, so a lane's four
// results are four consecutive hidden units of one row: one 8-byte LDS write of
// the next layer's bf16 input.  Layer 3's m x 64 output tiles are dealt to the
// waves in turn; a lane's results are four consecutive outputs of one row, one
// 16-byte store.
constexpr int IRB = 64;               // rows per workgroup
constexpr int INW = 8, INTH = 64 * INW;
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x4 to_bf16x4(float a, float b, float c, float d) {
  return bf16x4{(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d};
}

template <int HT, int MT>   // hidden width H = 128 HT, m = 16 MT
__global__ __launch_bounds__(INTH) void mlp_infer_bf16_kernel(
    const float* __restrict__ x, float* __restrict__ y, int64_t batch,
    const __bf16* __restrict__ W1, const float* __restrict__ b1,
    const __bf16* __restrict__ W2, const float* __restrict__ b2,
    const __bf16* __restrict__ W3, const float* __restrict__ b3) {
  constexpr int H = 128 * HT, m = 16 * MT;
  constexpr int XLD = m + 8, HLD = H + 8;   // padded rows (in bf16): 16-lane reads hit distinct banks
  __shared__ __attribute__((aligned(16))) __bf16 xs[IRB * XLD];
  __shared__ __attribute__((aligned(16))) __bf16 hs[IRB * HLD];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t r0 = (int64_t)blockIdx.x * IRB;
  const int rows = (int)(batch - r0 < IRB ? batch - r0 : IRB);
  for (int e = tid; e < IRB * m / 4; e += INTH) {
    const int r = e / (m / 4), c = 4 * (e % (m / 4));
    const f4 v = r < rows ? *reinterpret_cast<const f4*>(x + (r0 + r) * m + c) : f4{0.f, 0.f, 0.f, 0.f};
    *reinterpret_cast<bf16x4*>(&xs[r * XLD + c]) = to_bf16x4(v[0], v[1], v[2], v[3]);
  }
  __syncthreads();
  const int fr = lane & 15, fk = 8 * (lane >> 4);   // fragment row, k offset
  const int hid0 = 16 * HT * wave;
  f4 acc[HT][4];
  // one hidden layer: acc = W rows [hid0, hid0 + 16 HT) . act^T over K, act in LDS
  auto layer = [&](const __bf16* __restrict__ W, const __bf16* act, int ld, int K) {
#pragma unroll
    for (int t = 0; t < HT; ++t)
#pragma unroll
      for (int p = 0; p < 4; ++p) acc[t][p] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
      bf16x8 a[HT], b[4];
#pragma unroll
      for (int t = 0; t < HT; ++t)
        a[t] = *reinterpret_cast<const bf16x8*>(W + (int64_t)(hid0 + 16 * t + fr) * K + k0 + fk);
#pragma unroll
      for (int p = 0; p < 4; ++p)
        b[p] = *reinterpret_cast<const bf16x8*>(&act[(16 * p + fr) * ld + k0 + fk]);
#pragma unroll
      for (int t = 0; t < HT; ++t)
#pragma unroll
        for (int p = 0; p < 4; ++p) acc[t][p] = mfma1(a[t], b[p], acc[t][p]);
    }
  };
  // h = bf16(silu(acc + bias)) into hs[row][hid]
  auto to_hidden = [&](const float* __restrict__ bias) {
#pragma unroll
    for (int t = 0; t < HT; ++t) {
      const int h = hid0 + 16 * t + 4 * (lane >> 4);
      const f4 bv = *reinterpret_cast<const f4*>(bias + h);
#pragma unroll
      for (int p = 0; p < 4; ++p)
        *reinterpret_cast<bf16x4*>(&hs[(16 * p + fr) * HLD + h]) =
            to_bf16x4(silu(acc[t][p][0] + bv[0]), silu(acc[t][p][1] + bv[1]),
                      silu(acc[t][p][2] + bv[2]), silu(acc[t][p][3] + bv[3]));
    }
  };
  layer(W1, xs, XLD, m);
  to_hidden(b1);
  __syncthreads();
  layer(W2, hs, HLD, H);
  __syncthreads();   // every wave has read all of h1
  to_hidden(b2);
  __syncthreads();
  // layer 3: tile q = (o, p) of the m x 64 output, o < MT, p < 4
  for (int q = wave; q < MT * 4; q += INW) {
    const int o = q / 4, p = q % 4;
    f4 c = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < H; k0 += 32) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(W3 + (int64_t)(16 * o + fr) * H + k0 + fk);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(&hs[(16 * p + fr) * HLD + k0 + fk]);
      c = mfma1(a, b, c);
    }
    const int row = 16 * p + fr, out0 = 16 * o + 4 * (lane >> 4);
    if (row < rows) {
      const f4 xv = *reinterpret_cast<const f4*>(x + (r0 + row) * m + out0);
      const f4 bv = *reinterpret_cast<const f4*>(b3 + out0);
      *reinterpret_cast<f4*>(y + (r0 + row) * m + out0) = xv + (c + bv);
    }
  }
}

// FP32 -> bf16 (nearest, ties to even)
__global__ void round_bf16_kernel(const float* src, __bf16* dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT)
    dst[e] = (__bf16)src[e];
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
  __bf16* Pb = nullptr;      // bf16 copy of the parameters (inference), made on first use
  int pb_step = -1;          // the training step it was rounded at
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

int thcsox_mlp_forward_bf16(thcsox_mlp_t q, const float* x_dev, float* y_dev, int64_t batch) {
  clear_error();
  if (q == nullptr || batch < 0) return set_error(THCSOX_EINVAL, "bad argument");
  const int HT = q->H / 128, MT = q->m / 16;
  if (q->H % 128 != 0 || (HT != 1 && HT != 2 && HT != 4) || q->m % 16 != 0 ||
      (MT != 2 && MT != 4))
    return set_error(THCSOX_EINVAL, "bf16 inference needs m in {32, 64} and H in {128, 256, 512}");
  if (batch == 0) return 0;
  if (x_dev == nullptr || y_dev == nullptr) return set_error(THCSOX_EINVAL, "NULL argument");
  if (q->Pb == nullptr) {
    void* v = nullptr;
    hipError_t e = hipMalloc(&v, sizeof(__bf16) * (size_t)q->np);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return set_error(THCSOX_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    q->allocs.push_back(v);
    q->Pb = static_cast<__bf16*>(v);
  }
  if (q->pb_step != q->step) {
    round_bf16_kernel<<<blocks_for(q->np), NT, 0, q->stream>>>(q->P, q->Pb, q->np);
    MTRY(hipGetLastError());
    q->pb_step = q->step;
  }
  const int64_t nblk = (batch + IRB - 1) / IRB;
  if (nblk > 0x7fffffffLL) return set_error(THCSOX_EINVAL, "batch too large");
  const __bf16 *W1 = q->Pb + q->oW1, *W2 = q->Pb + q->oW2, *W3 = q->Pb + q->oW3;
  const float *b1 = q->P + q->ob1, *b2 = q->P + q->ob2, *b3 = q->P + q->ob3;
  auto go = [&](auto kernel) {
    kernel<<<(unsigned)nblk, INTH, 0, q->stream>>>(x_dev, y_dev, batch, W1, b1, W2, b2, W3, b3);
  };
  if (MT == 4) {
    if (HT == 4) go(mlp_infer_bf16_kernel<4, 4>);
    else if (HT == 2) go(mlp_infer_bf16_kernel<2, 4>);
    else go(mlp_infer_bf16_kernel<1, 4>);
  } else {
    if (HT == 4) go(mlp_infer_bf16_kernel<4, 2>);
    else if (HT == 2) go(mlp_infer_bf16_kernel<2, 2>);
    else go(mlp_infer_bf16_kernel<1, 2>);
  }
  MTRY(hipGetLastError());
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
