// Elementwise steps of the GF2 direct (bubble) self-energy in THC form:
//   Pi_QS = Gt_QS Gbt_SQ (the polarisation on the interpolation grid),
//   H = W o Gt (W = V Pi V), then Sigma = X H X^T by the back-projection.
#include "direct.hpp"

namespace thcsox {
namespace {

constexpr int PT = 32;   // transpose tile edge
constexpr int NT = 256;

// one 32 x 32 tile (Q block, S block) of one tau point; Gbt is read as the
// transposed tile through LDS so both reads and the write are coalesced
__global__ __launch_bounds__(NT) void bubble_pi_kernel(const double* __restrict__ Gt,
                                                       const double* __restrict__ Gbt,
                                                       double* __restrict__ Pi, int naux) {
  __shared__ double t[PT][PT + 1];
  const int64_t off = (int64_t)blockIdx.z * naux * naux;
  const int q0 = blockIdx.y * PT, s0 = blockIdx.x * PT;
  const int tx = threadIdx.x % PT, ty = threadIdx.x / PT;   // 32 x 8
  for (int r = ty; r < PT; r += NT / PT) {
    const int S = s0 + r, Q = q0 + tx;   // Gbt[S][Q], coalesced in Q
    t[r][tx] = (S < naux && Q < naux) ? Gbt[off + (int64_t)S * naux + Q] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < PT; r += NT / PT) {
    const int Q = q0 + r, S = s0 + tx;   // Pi[Q][S], coalesced in S
    if (Q < naux && S < naux)
      Pi[off + (int64_t)Q * naux + S] = Gt[off + (int64_t)Q * naux + S] * t[tx][r];
  }
}

__global__ __launch_bounds__(NT) void hadamard64_kernel(const double* W, const double* __restrict__ Gt,
                                                        double* H, int64_t len) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < len; i += (int64_t)gridDim.x * NT)
    H[i] = W[i] * Gt[i];
}

}  // namespace

hipError_t bubble_pi(const double* Gt, const double* Gbt, double* Pi, int naux, int nb,
                     hipStream_t s) {
  if (naux <= 0 || nb <= 0) return hipSuccess;
  const unsigned nt = (unsigned)((naux + PT - 1) / PT);
  bubble_pi_kernel<<<dim3(nt, nt, nb), NT, 0, s>>>(Gt, Gbt, Pi, naux);
  return hipGetLastError();
}

hipError_t hadamard64(const double* W, const double* Gt, double* H, int64_t len, hipStream_t s) {
  if (len <= 0) return hipSuccess;
  const int64_t b = (len + NT - 1) / NT;
  hadamard64_kernel<<<(unsigned)(b > 8192 ? 8192 : b), NT, 0, s>>>(W, Gt, H, len);
  return hipGetLastError();
}

}  // namespace thcsox
