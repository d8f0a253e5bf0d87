// Launchers of the projector kernels (projector.hip) and of the fused
// back-projection epilogues (mocca.hip).
#pragma once

#include "kernels.h"

namespace osscir {

// p[c][l] = sum_k X_{l,k} f[c][k], c < nch (chunks of up to 3 channels).
hipError_t launch_forward(const ScanDesc &sd, const float *f, int nch, float *p, hipStream_t st);

// b[c][k] = sum_l X_{l,k} q[c][l] (chunks of 9, 6, 3, 2 or 1 channels).
hipError_t launch_back(const ScanDesc &sd, const float *q, int nch, float *b, hipStream_t st);

}  // namespace osscir
