// Elementwise kernels of the GF2 direct (bubble) term; host launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace thcsox {

// Pi[b][Q][S] = Gt[b][Q][S] * Gbt[b][S][Q] for b < nb (naux x naux blocks,
// consecutive blocks aa = naux^2 apart).
hipError_t bubble_pi(const double* Gt, const double* Gbt, double* Pi, int naux, int nb,
                     hipStream_t s);
// H[i] = W[i] * Gt[i], i < len (H may alias W).
hipError_t hadamard64(const double* W, const double* Gt, double* H, int64_t len, hipStream_t s);

}  // namespace thcsox
