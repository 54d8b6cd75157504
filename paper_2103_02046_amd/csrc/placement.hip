// Mesh placement over the bunch and the leapfrog push.
//
// Placement: the paper fixes the mesh as nodes x_k = k h on [0, L]
// (Sec. 2.4.2) and leaves open where the bunch sits. Each evaluation here
// centres the mesh on the bounding box of the positions and, when the box
// is wider than the nodes an assignment stencil may use, zooms h and r_c by
// a common s >= 1 (the split parameter by 1/s). Bounding boxes are exact
// float64 min/max reductions.
//
// Push: kick-drift-kick leapfrog, the variational integrator of
// Sec. 2.4.3 (eq. leapfrog) applied to the P3M Lagrangian (Sec. 2.5).
#include "bbox.h"
#include "launch.h"

namespace p3m {

namespace {

constexpr int kBboxItems = 4;

__global__ void __launch_bounds__(kThreads) k_bbox(int64_t n, const double* __restrict__ x,
                                                   double* __restrict__ part, int nblk,
                                                   int* __restrict__ status) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads)
    bbox_accumulate(x + 3 * i, lo, hi, bad);
  if (bad) atomicOr(status, kBitNonFinite);
  bbox_block_store(lo, hi, part, nblk);
}

__global__ void __launch_bounds__(kThreads) k_kick_drift_bbox(
    int64_t n, double* __restrict__ x, double* __restrict__ p, const double* __restrict__ f,
    double half_dt, double dt_over_m, double* __restrict__ part, int nblk, int* __restrict__ status) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
    double xi[3];
    for (int d = 0; d < 3; ++d) {
      double pd = p[3 * i + d] + half_dt * f[3 * i + d];
      p[3 * i + d] = pd;
      xi[d] = x[3 * i + d] + dt_over_m * pd;
      x[3 * i + d] = xi[d];
    }
    bbox_accumulate(xi, lo, hi, bad);
  }
  if (bad) atomicOr(status, kBitNonFinite);
  bbox_block_store(lo, hi, part, nblk);
}

__global__ void k_kick(int64_t n, double* __restrict__ p, const double* __restrict__ f, double half_dt) {
  int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (i < 3 * n) p[i] += half_dt * f[i];
}

// One block of kFinThreads reduces the [6][nblk] box partials. Each thread
// issues the loads of up to kFinItems columns before it reduces them, so
// the few thousand partials of a gather-sized grid take one round trip per
// batch rather than one per column.
constexpr int kFinThreads = 1024;
constexpr int kFinItems = 4;

__global__ void __launch_bounds__(kFinThreads) k_place_finalize(int nblk, const double* __restrict__ part,
                                                                Geo geo, const double* __restrict__ place_in,
                                                                Place* __restrict__ out,
                                                                double* __restrict__ place_out,
                                                                int* __restrict__ status) {
  __shared__ double s[6][kFinThreads / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b0 = 0; b0 < nblk; b0 += kFinItems * kFinThreads) {
    double v[kFinItems][6];
#pragma unroll
    for (int k = 0; k < kFinItems; ++k) {
      const int b = b0 + k * kFinThreads + t;
#pragma unroll
      for (int d = 0; d < 6; ++d) v[k][d] = b < nblk ? part[d * nblk + b] : (d < 3 ? INFINITY : -INFINITY);
    }
#pragma unroll
    for (int k = 0; k < kFinItems; ++k)
      for (int d = 0; d < 3; ++d) {
        lo[d] = fmin(lo[d], v[k][d]);
        hi[d] = fmax(hi[d], v[k][3 + d]);
      }
  }
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
    double r = s[t][0];
    for (int k = 1; k < kFinThreads / 64; ++k) r = t < 3 ? fmin(r, s[t][k]) : fmax(r, s[t][k]);
    s[t][0] = r;
  }
  __syncthreads();
  if (t != 0) return;
  double x0[3], zoom;
  if (place_in) {
    for (int d = 0; d < 3; ++d) x0[d] = place_in[d];
    zoom = place_in[3];
    if (!(zoom >= 1.0) || !isfinite(zoom)) { zoom = 1.0; atomicOr(status, kBitDomain); }
    // a replayed placement must still hold every stencil
    for (int d = 0; d < 3; ++d) {
      const double usable = usable_nodes(geo, d);
      double hp = zoom * geo.h[d];
      double c = (double)(geo.grid[d] - 1) * 0.5;
      double ulo = (s[d][0] - x0[d]) / hp, uhi = (s[3 + d][0] - x0[d]) / hp;
      if (!(ulo >= c - 0.5 * usable && uhi <= c + 0.5 * usable)) atomicOr(status, kBitDomain);
    }
  } else {
    zoom = 1.0;
    for (int d = 0; d < 3; ++d) {
      double a = s[d][0], b = s[3 + d][0];
      if (!(a <= b)) { a = 0.0; b = 0.0; }  // no finite position on this axis
      const double usable = usable_nodes(geo, d);
      double need = (b - a) * (1.0 + 1e-6) / (usable * geo.h[d]);
      if (need > zoom) zoom = need;
    }
    if (zoom > 1.0 && !geo.zoom) atomicOr(status, kBitDomain);
    for (int d = 0; d < 3; ++d) {
      double a = s[d][0], b = s[3 + d][0];
      if (!(a <= b)) { a = 0.0; b = 0.0; }
      double hp = zoom * geo.h[d];
      double c = 0.5 * (a + b);
      x0[d] = c - 0.5 * (double)(geo.grid[d] - 1) * hp;
    }
  }
  Place P;
  for (int d = 0; d < 3; ++d) {
    P.x0[d] = x0[d];
    P.inv_hp[d] = 1.0 / (zoom * geo.h[d]);
    P.inv_cell[d] = 1.0 / (zoom * geo.cu[d] * geo.rc);
  }
  P.s = zoom;
  P.inv_lu = 1.0 / (zoom * geo.rc);
  P.fscale = geo.ke_q2 * P.inv_lu * P.inv_lu;
  P.phiscale = P.inv_lu;
  P.pad[0] = P.pad[1] = P.pad[2] = 0.0;
  *out = P;
  if (place_out) {
    for (int d = 0; d < 3; ++d) place_out[d] = x0[d];
    place_out[3] = zoom;
  }
}

}  // namespace

int bbox_blocks(int64_t n) {
  int64_t b = (n + (int64_t)kThreads * kBboxItems - 1) / ((int64_t)kThreads * kBboxItems);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

void launch_bbox(int64_t n, const double* x, double* part, int nblk, int* status, hipStream_t st) {
  k_bbox<<<nblk, kThreads, 0, st>>>(n, x, part, nblk, status);
}

void launch_kick_drift_bbox(int64_t n, double* x, double* p, const double* f, double dt,
                            double inv_m, double* part, int nblk, int* status, hipStream_t st) {
  k_kick_drift_bbox<<<nblk, kThreads, 0, st>>>(n, x, p, f, 0.5 * dt, dt * inv_m, part, nblk, status);
}

void launch_kick(int64_t n, double* p, const double* f, double dt, hipStream_t st) {
  if (n == 0) return;
  int64_t blocks = (3 * n + kThreads - 1) / kThreads;
  k_kick<<<(unsigned)blocks, kThreads, 0, st>>>(n, p, f, 0.5 * dt);
}

void launch_place_finalize(int nblk, const double* part, const Geo& geo, const double* place_in,
                           Place* out, double* place_out, int* status, hipStream_t st) {
  k_place_finalize<<<1, kFinThreads, 0, st>>>(nblk, part, geo, place_in, out, place_out, status);
}

}  // namespace p3m
