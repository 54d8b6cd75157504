// Short-range (PP) pair forces inside the cutoff, summed directly.
//
// For every ordered pair (i, j), j != i, with 0 < rho < 1 (rho = r / Lu, so
// the cutoff is 1 in these units):
//   F_i += w_i w_j [erfc(kappa rho)/rho + (2 kappa/sqrt(pi)) exp(-kappa^2 rho^2)]
//          (x_i - x_j) / rho^2
// which is minus the gradient of the erfc part of the Ewald split of the
// Coulomb kernel (Sec. 2.2, eq. ewald_split; Sec. 1, eq. summation_short;
// Sec. 2.5, eq. eom_p3m_coord second term). Coincident particles (rho = 0,
// the particle itself included) contribute nothing.
//
// float form: erfc(x) = exp(-x^2) t P(t), t = 1/(1 + x/2), with the polynomial
// fitted in this repository (fit_erfcx.py; relative error < 2e-7 in float),
// the exp(-x^2) shared with the second term; per-particle sums are Kahan
// compensated. double form: the device library's erfc and exp.
#include "erfcx_fit.h"
#include "launch.h"

namespace p3m {

namespace {

constexpr double kTwoOverSqrtPi = 1.12837916709551257390;
constexpr float kLog2e = 1.44269504088896340736f;

struct Kahan3 {
  float s[3] = {0.f, 0.f, 0.f};
  float c[3] = {0.f, 0.f, 0.f};
  __device__ __forceinline__ void add(int d, float v) {
    float y = v - c[d];
    float t = s[d] + y;
    c[d] = (t - s[d]) - y;
    s[d] = t;
  }
};

__device__ __forceinline__ float erfcx_poly(float t) {
  float acc = (float)p3m_erfcx_coef[P3M_ERFCX_DEG];
#pragma unroll
  for (int k = P3M_ERFCX_DEG - 1; k >= 0; --k) acc = fmaf(acc, t, (float)p3m_erfcx_coef[k]);
  return acc;
}

// Scalar g(rho) w_j with F = g d; float.
__device__ __forceinline__ float pair_scalar(float r2, float wj, float kappa, float c2k, float* epair) {
  float rinv = __builtin_amdgcn_rsqf(r2);
  float r = r2 * rinv;
  float x = kappa * r;
  float e = __builtin_amdgcn_exp2f(-x * x * kLog2e);
  float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
  float erfc_x = e * t * erfcx_poly(t);
  if (epair) *epair = erfc_x * rinv * wj;
  return (erfc_x * rinv + c2k * e) * (rinv * rinv) * wj;
}

__device__ __forceinline__ double pair_scalar(double r2, double wj, double kappa, double c2k, double* epair) {
  double r = sqrt(r2);
  double x = kappa * r;
  double e = exp(-x * x);
  double ec = erfc(x);
  if (epair) *epair = ec / r * wj;
  return (ec / r + c2k * e) / r2 * wj;
}

template <typename R>
struct Acc3;
template <>
struct Acc3<float> {
  Kahan3 k;
  __device__ __forceinline__ void add(float gx, float gy, float gz) { k.add(0, gx); k.add(1, gy); k.add(2, gz); }
  __device__ __forceinline__ float get(int d) const { return k.s[d]; }
};
template <>
struct Acc3<double> {
  double s[3] = {0, 0, 0};
  __device__ __forceinline__ void add(double gx, double gy, double gz) { s[0] += gx; s[1] += gy; s[2] += gz; }
  __device__ __forceinline__ double get(int d) const { return s[d]; }
};

template <typename R, bool ENERGY>
__global__ void __launch_bounds__(kThreads) k_pp(int64_t n, const PPRec<R>* __restrict__ rec,
                                                 const uint32_t* __restrict__ keys,
                                                 const int* __restrict__ cs, Geo geo,
                                                 PPRec<R>* __restrict__ out, double* __restrict__ energy) {
  const int64_t j = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  double e_acc = 0.0;
  int pairs = 0;
  if (j < n) {
    const PPRec<R> me = rec[j];
    const uint32_t key = keys[j];
    const int nx = geo.ncell[0], ny = geo.ncell[1], nz = geo.ncell[2];
    const int cx = (int)(key % (uint32_t)nx);
    const int cy = (int)((key / (uint32_t)nx) % (uint32_t)ny);
    const int cz = (int)(key / ((uint32_t)nx * (uint32_t)ny));
    const R kappa = (R)geo.kappa;
    const R c2k = (R)(kTwoOverSqrtPi * geo.kappa);
    const R cux = (R)geo.cu[0], cuy = (R)geo.cu[1], cuz = (R)geo.cu[2];
    Acc3<R> acc;
    for (int dz = -1; dz <= 1; ++dz) {
      const int z = cz + dz;
      if (z < 0 || z >= nz) continue;
      for (int dy = -1; dy <= 1; ++dy) {
        const int y = cy + dy;
        if (y < 0 || y >= ny) continue;
        const int rowc = (z * ny + y) * nx;
        // offsets of the neighbour cell corner relative to the own one
        const R oy = me.y - (R)dy * cuy;
        const R oz = me.z - (R)dz * cuz;
        for (int dx = -1; dx <= 1; ++dx) {
          const int xx = cx + dx;
          if (xx < 0 || xx >= nx) continue;
          const R ox = me.x - (R)dx * cux;
          const int b = cs[rowc + xx], e = cs[rowc + xx + 1];
          for (int k = b; k < e; ++k) {
            const PPRec<R> o = rec[k];
            const R ddx = ox - o.x, ddy = oy - o.y, ddz = oz - o.z;
            const R r2 = ddx * ddx + ddy * ddy + ddz * ddz;
            if (r2 < (R)1 && r2 > (R)0) {
              R ep;
              const R g = pair_scalar(r2, o.w, kappa, c2k, ENERGY ? &ep : nullptr);
              acc.add(g * ddx, g * ddy, g * ddz);
              if (ENERGY) {
                e_acc += (double)ep;
                ++pairs;
              }
            }
          }
        }
      }
    }
    PPRec<R> f;
    f.x = acc.get(0) * me.w;
    f.y = acc.get(1) * me.w;
    f.z = acc.get(2) * me.w;
    f.w = (R)0;
    out[j] = f;
    e_acc *= 0.5 * (double)me.w;   // each unordered pair is met twice
  }
  if (ENERGY) {
    // block reduction, one float64 atomic per block; energy[2] counts pairs
    __shared__ double s[2][kThreads];
    s[0][threadIdx.x] = e_acc;
    s[1][threadIdx.x] = (double)pairs;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        s[0][threadIdx.x] += s[0][threadIdx.x + w];
        s[1][threadIdx.x] += s[1][threadIdx.x + w];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      atomicAdd(energy, s[0][0]);
      atomicAdd(energy + 2, s[1][0]);
    }
  }
}

// (H_PP v)_i = sum_j K_ij (v_i - v_j), K_ij = f I + (f'/r) d d^T, F_ij = w_i w_j f(r) d;
// f(r) = g(r)/r^2, g = erfc(kr)/r + (2k/sqrt(pi)) e^{-k^2 r^2}. Internal units,
// double. The derivative of the pair force of the kernel above.
__global__ void __launch_bounds__(kThreads) k_pp_hvp(int64_t n, const PPRec<double>* __restrict__ rec,
                                                     const uint32_t* __restrict__ keys,
                                                     const int* __restrict__ cs, Geo geo,
                                                     const double* __restrict__ v,
                                                     double* __restrict__ out) {
  const int64_t j = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (j >= n) return;
  const PPRec<double> me = rec[j];
  const double vi[3] = {v[3 * j], v[3 * j + 1], v[3 * j + 2]};
  const uint32_t key = keys[j];
  const int nx = geo.ncell[0], ny = geo.ncell[1], nz = geo.ncell[2];
  const int cx = (int)(key % (uint32_t)nx);
  const int cy = (int)((key / (uint32_t)nx) % (uint32_t)ny);
  const int cz = (int)(key / ((uint32_t)nx * (uint32_t)ny));
  const double k = geo.kappa, c2 = kTwoOverSqrtPi;
  double o3[3] = {0, 0, 0};
  for (int dz = -1; dz <= 1; ++dz) {
    const int z = cz + dz;
    if (z < 0 || z >= nz) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = cy + dy;
      if (y < 0 || y >= ny) continue;
      const int rowc = (z * ny + y) * nx;
      for (int dx = -1; dx <= 1; ++dx) {
        const int xx = cx + dx;
        if (xx < 0 || xx >= nx) continue;
        const double sh[3] = {dx * geo.cu[0], dy * geo.cu[1], dz * geo.cu[2]};
        const int b = cs[rowc + xx], e = cs[rowc + xx + 1];
        for (int q = b; q < e; ++q) {
          const PPRec<double> o = rec[q];
          const double d[3] = {me.x - o.x - sh[0], me.y - o.y - sh[1], me.z - o.z - sh[2]};
          const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          if (!(r2 < 1.0 && r2 > 0.0)) continue;
          const double r = sqrt(r2);
          const double ex = exp(-k * k * r2), ec = erfc(k * r);
          const double g = ec / r + c2 * k * ex;
          const double gp = -ec / r2 - c2 * k * ex / r - 2.0 * c2 * k * k * k * r * ex;
          const double f = g / r2;
          const double fp = gp / r2 - 2.0 * g / (r2 * r);
          const double dv[3] = {vi[0] - v[3 * q], vi[1] - v[3 * q + 1], vi[2] - v[3 * q + 2]};
          const double dd = d[0] * dv[0] + d[1] * dv[1] + d[2] * dv[2];
          const double s = me.w * o.w;
          for (int c = 0; c < 3; ++c) o3[c] += s * (f * dv[c] + fp / r * d[c] * dd);
        }
      }
    }
  }
  out[3 * j] = o3[0];
  out[3 * j + 1] = o3[1];
  out[3 * j + 2] = o3[2];
}

}  // namespace

template <typename R>
void launch_pp(int64_t n, const PPRec<R>* rec, const uint32_t* keys, const int* cell_start,
               const Geo& geo, PPRec<R>* out, double* energy, hipStream_t st) {
  unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
  if (energy)
    k_pp<R, true><<<blocks, kThreads, 0, st>>>(n, rec, keys, cell_start, geo, out, energy);
  else
    k_pp<R, false><<<blocks, kThreads, 0, st>>>(n, rec, keys, cell_start, geo, out, nullptr);
}

void launch_pp_hvp(int64_t n, const PPRec<double>* rec, const uint32_t* keys, const int* cell_start,
                   const Geo& geo, const double* v_sorted, double* out_sorted, hipStream_t st) {
  unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
  k_pp_hvp<<<blocks, kThreads, 0, st>>>(n, rec, keys, cell_start, geo, v_sorted, out_sorted);
}

template void launch_pp<float>(int64_t, const PPRec<float>*, const uint32_t*, const int*, const Geo&,
                               PPRec<float>*, double*, hipStream_t);
template void launch_pp<double>(int64_t, const PPRec<double>*, const uint32_t*, const int*, const Geo&,
                                PPRec<double>*, double*, hipStream_t);

}  // namespace p3m
