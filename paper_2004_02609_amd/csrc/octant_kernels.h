// Kernels of the compressed Toeplitz cache (setup_kernels.hip): the Toeplitz octant of
// one pair filled from the panel integrals, and a pair's circulant embedding read from
// its octant.
#pragma once
#include "mvp_kernels.h"

namespace vc {

// Toeplitz octant of one pair: D[a] non-negative offsets per axis (k_fill_octant)
struct OctArgs {
  int alpha, beta, want;
  int D[3];
};
hipError_t launch_fill_octant(double* T, const OctArgs& a, const double* gl_nodes, hipStream_t st);
hipError_t launch_embed_octant(double* C, const double* T, const FillArgs& a, const OctArgs& o, hipStream_t st);

}  // namespace vc
