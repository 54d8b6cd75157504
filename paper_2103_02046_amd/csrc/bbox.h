// Bounding-box partials of the particle positions (exact float64 min/max),
// shared by the push and the gather that fuses the next push into itself.
#pragma once

#include "common.h"

namespace p3m {

// Adds a position to the running box; a non-finite coordinate sets bad.
__device__ inline void bbox_accumulate(const double* xi, double (&lo)[3], double (&hi)[3], int& bad) {
  for (int d = 0; d < 3; ++d) {
    const double v = xi[d];
    if (!isfinite(v)) {
      bad = 1;
      continue;
    }
    lo[d] = fmin(lo[d], v);
    hi[d] = fmax(hi[d], v);
  }
}

// Block reduction of the box (every thread of the block calls it): wave
// shuffles, then one value per wave in LDS. part holds [6][nblk]: the three
// minima, then the three maxima, one column per block.
__device__ inline void bbox_block_store(double (&lo)[3], double (&hi)[3], double* part, int nblk) {
  __shared__ double s[6][kThreads / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int d = 0; d < 3; ++d) {
    for (int off = 32; off > 0; off >>= 1) {
      lo[d] = fmin(lo[d], __shfl_xor(lo[d], off));
      hi[d] = fmax(hi[d], __shfl_xor(hi[d], off));
    }
    if (lane == 0) {
      s[d][w] = lo[d];
      s[3 + d][w] = hi[d];
    }
  }
  __syncthreads();
  if (t < 6) {
    double v = s[t][0];
    for (int k = 1; k < kThreads / 64; ++k) v = t < 3 ? fmin(v, s[t][k]) : fmax(v, s[t][k]);
    part[t * nblk + blockIdx.x] = v;
  }
}

}  // namespace p3m
