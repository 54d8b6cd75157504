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
// float form: erfc(x) = exp(-x^2) t P(t), t = 1/(1 + x/2), with the degree-6
// polynomial fitted in this repository on 0 <= x <= 6 (fit_erfcx.py; relative
// error < 5e-7 in float), the exp(-x^2) shared with the second term. Beyond
// x = 6 (kappa > 6 only) t < 1/4, where |t P(t)| < 0.1, and exp(-x^2) <
// 2.4e-16 leaves both terms of the pair force negligible, so t is not clamped;
// per-particle sums are Kahan compensated. double form: the device
// library's erfc and exp.
#include <type_traits>

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

// Half-precision cutoff test of the float form. Coordinates relative to a
// point O of the group's cell, in cutoff units, are rounded to fp16: T for
// the targets (to nearest), C for the candidates (toward zero), and
// W = fp16(|C|^2 - lim). Products of two fp16 values are exact in float32,
// so v = |T|^2 + W - 2 T.C = |T - C|^2 - lim + (W - (|C|^2 - lim)) costs two
// v_dot2_f32_f16 and the candidate needs 8 bytes of LDS.
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
// clang vectors, not HIP's uint2/uint4 structs: a copy of the struct is read
// member by member (4-byte loads), a vector in a single LDS access. The test
// tile is written as 8-byte and read as 16-byte vectors, so both types may
// alias anything.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4), may_alias));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2), may_alias));

// the fp16 pair in a 32-bit value; taken by value, since clang's
// __builtin_bit_cast of a vector element (c.z) reads the vector's first
// element instead
__device__ __forceinline__ half2v as_half2(uint32_t v) { return __builtin_bit_cast(half2v, v); }

__device__ __forceinline__ uint32_t pack_rtz(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(a, b));
}

// a.lo b.lo + a.hi b.hi + c for fp16 pairs a, b, in the VOP3P form: its
// accumulator is an operand of its own, where the builtin's two-operand
// form ties it to the result and costs a copy of c per call
__device__ __forceinline__ float dot2_acc(uint32_t a, uint32_t b, float c) {
  float r;
  asm("v_dot2_f32_f16 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// A bound on the spacing of fp16 values of magnitude <= x: 2^(e - 11) for
// x < 2^e, and at least the subnormal spacing 2^-24.
__device__ __forceinline__ double ulp16_bound(double x) {
  int e;
  frexp(x, &e);
  return ldexp(1.0, e - 11 > -24 ? e - 11 : -24);
}

// lim of the fp16 test, in cutoff units, for cells of largest edge emax.
// Positions lie in [-1/2, 3/2) edges of their cell's corner and O is half
// an edge from that corner, so targets lie within tmax = emax of O, and a
// candidate within the cutoff of one of them within cmx = tmax + 1. Per
// coordinate T errs by at most uT (half a spacing) and C by uC (a spacing),
// each plus 2^-14 should fp16 subnormals be flushed, so |T - C| <=
// |t - c| + sqrt(3) (uT + uC); W errs by at most uW. A pair inside the
// cutoff therefore gives v < 0 once lim exceeds (1 + sqrt(3) (uT + uC))^2 +
// uW, plus 1e-5 of the largest terms for the float32 sums and conversions
// and the rounding of the hit loop's own test on the exact separation.
__device__ __forceinline__ float fp16_test_lim(double emax) {
  const double flush = ldexp(1.0, -14);
  const double tmax = emax * (1.0 + 1e-6), cmx = tmax + 1.0;
  const double uT = 0.5 * ulp16_bound(tmax) + flush, uC = ulp16_bound(cmx) + flush;
  const double uW = ulp16_bound(fmax(1.1, (cmx + uC) * (cmx + uC))) + flush;
  const double d = sqrt(3.0) * (uT + uC);
  return (float)(1.0 + 2.0 * d + d * d + uW + 1e-5 * fmax(1.0, 3.0 * cmx * cmx));
}

__device__ __forceinline__ float erfcx_poly(float t) {
  float acc = (float)p3m_erfcx_coef[P3M_ERFCX_DEG];
#pragma unroll
  for (int k = P3M_ERFCX_DEG - 1; k >= 0; --k) acc = fmaf(acc, t, (float)p3m_erfcx_coef[k]);
  return acc;
}

// Constants of the pair kernel in units of the cutoff.
template <typename R>
struct PairK {
  R kappa, c2k;     // kappa = a r_c, 2 kappa / sqrt(pi)
  R half_kappa;     // kappa / 2
  R ek;             // -kappa^2 log2(e)
};

// Scalar g(rho) w_j with F = g d; float. With x = kappa rho, e = exp(-x^2)
// and erfc(x) = e t P(t): g = (e / rho^2) (t P(t) / rho + 2 kappa/sqrt(pi)).
__device__ __forceinline__ float pair_scalar(float r2, float wj, const PairK<float>& K, float* epair) {
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float r = r2 * rinv;
  const float t = __builtin_amdgcn_rcpf(fmaf(K.half_kappa, r, 1.0f));
  const float e = __builtin_amdgcn_exp2f(K.ek * r2);
  const float tp = t * erfcx_poly(t);
  if (epair) *epair = e * tp * rinv * wj;
  return (e * (rinv * rinv)) * fmaf(tp, rinv, K.c2k) * wj;
}

__device__ __forceinline__ double pair_scalar(double r2, double wj, const PairK<double>& K, double* epair) {
  const double kappa = K.kappa, c2k = K.c2k;
  const double rinv = 1.0 / sqrt(r2);   // one reciprocal; the quotients are products with it
  const double x = kappa * r2 * rinv;
  const double e = exp(-x * x);
  const double ec = erfc(x);
  if (epair) *epair = ec * rinv * wj;
  return (ec * rinv + c2k * e) * (rinv * rinv) * wj;
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

// Work groups (kGroupRun particles at most, one cell) come from the cell
// sort. Cells have edges >= r_c / D (D = Geo::pp_div, 1 or 2), so the
// candidates of every particle of a group lie in (2D+1)^2 contiguous
// ranges: cells cx-D .. cx+D of the (2D+1) x (2D+1) neighbouring rows (a
// row of cells is contiguous in the sorted order); consecutive groups of
// one class (cells of at least kDenseCell particles first, then the others)
// are spatial neighbours. Halving the cells (D = 2) cuts the candidate volume
// from 27 to 125/8 cutoff cubes, for dense bunches whose half-size cells
// still fill the groups.

// (m << 1) | sign(v): one v_alignbit_b32 for float; the sign of a double is
// the top bit of its high word.
__device__ __forceinline__ uint32_t mask_shift_in(uint32_t m, float v) {
  return __builtin_amdgcn_alignbit(m, __float_as_uint(v), 31u);
}
__device__ __forceinline__ uint32_t mask_shift_in(uint32_t m, double v) {
  return __builtin_amdgcn_alignbit(m, (uint32_t)(__double_as_longlong(v) >> 32), 31u);
}

template <typename R>
struct Vec4;
template <>
struct Vec4<float> { using T = float4; };
template <>
struct Vec4<double> { using T = double4; };

constexpr int kWaveGroups = 4;           // groups per wave (16 lanes each)
constexpr int kRun = 2;                  // consecutive candidates read together
constexpr int kTileK = 64;               // candidates per group per tile
constexpr int kPerLane = kTileK / 16;    // candidates each lane stages per tile
constexpr int kXcdRun = 32;              // consecutive waves of groups given to one XCD

// Pair forces of four groups in one wave (lanes 16q .. 16q+15 hold the
// targets of group q).
// The candidates of a group are the concatenation of its row ranges, L of
// them, read in runs of kRun = 2 consecutive ones (32 contiguous bytes).
// With S = ceil(L / 64) tiles, tile t holds runs t, t+S, ..., t+31S: an evenly
// spread sample of the whole neighbourhood, so the hits of a tile spread
// evenly over the group's targets. Consecutive sorted particles sit in one
// small cell, so a run's candidates are all near a target or all far from
// it; short runs keep the hits per lane per tile close to their mean, which
// is what the lanes of a wave wait for in the hit loop (runs of 8, 4 and 2:
// PP 96.4, 91.9 and 89.1 ms on the 2^25-particle core/halo bunch). Per tile:
//   1. each group stages its 64 candidates in LDS (loaded one tile ahead);
//   2. each lane tests its group's 64 candidates against its target, with
//      positions relative to the group's cell (a few cell edges at most;
//      float form: fp16 coordinates and two v_dot2_f32_f16 per candidate
//      under a bounded margin, double form: the expanded square in double):
//      a 64-bit hit mask;
//   3. each lane evaluates its own hits from the exact separation: in the
//      float form the difference of fixed-point positions relative to a
//      point of the group's cell (cell offsets are whole multiples of the
//      cell edge in units, fix_edge), an integer rounded once to float; a
//      candidate's offset along the row comes from the x code in its
//      record, the row's offsets from its range; in the double form
//      cell-local positions plus cell-corner offsets (exact multiples of the
//      cell edge). The tile sum is added to the per-particle total with
//      Kahan compensation (float form).
// The pair kernel runs one wave per work-group, so its syncs order only
// that wave's LDS accesses: LDS operations of a wave complete in order, and
// fences against compiler motion suffice (no s_barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// HVP: the pair part of the Hessian-vector product in place of the force,
// (H_PP v)_i = sum_j K_ij (v_i - v_j) with K_ij = w_i w_j [f I + (f'/r) d d^T],
// the derivative of the pair force F_ij = w_i w_j f d; f = g / r^2,
// g = erfc(kr)/r + (2k/sqrt(pi)) e^{-k^2 r^2} (internal units). v and hv_out
// are sorted [n][3] float64. float form: the separation from the fixed-point
// records (residuals included), the Jacobian in float with the same erfc fit
// as the force, Kahan-compensated per-particle sums.
template <typename R, bool ENERGY, bool PACKED, bool HVP, int DIV>
__global__ void __launch_bounds__(64) k_pp(const int2* __restrict__ desc, const int* __restrict__ counter, int gcap,
                                           const PPPos<R>* __restrict__ rec, const uint32_t* __restrict__ keys,
                                           const int* __restrict__ cs, Geo geo, PPRec<R>* __restrict__ out,
                                           double* __restrict__ energy, const double* __restrict__ hv_in = nullptr,
                                           double* __restrict__ hv_out = nullptr,
                                           unsigned long long* __restrict__ wclock = nullptr) {
  using V4 = typename Vec4<R>::T;
  static_assert(!HVP || !ENERGY, "HVP: no energy");
  // per-group tiles padded by one element so the four groups' broadcast
  // reads fall in different LDS banks
  constexpr int TS = kTileK + 1;
  constexpr int NT = kWaveGroups * TS;
  // the float form's fp16 test tile: pairs of candidates read as 16 bytes,
  // groups 66 slots (132 dwords) apart, so their reads start 4 banks apart
  constexpr int TSH = kTileK + 2;
  constexpr bool kFix = std::is_same<R, float>::value;
  // PACKED: float records whose weight slot holds position residuals (all weights 1)
  static_assert(kFix || !PACKED, "residual packing is a float-form layout");
  __shared__ V4 tile[kFix ? 1 : NT];        // double: group-relative x, y, z and |c|^2 - lim (cutoff test)
  __shared__ u32x4 tileh[kFix ? kWaveGroups * TSH / 2 : 1];   // float: fp16 (Cx, Cy), (Cz, W) per candidate
  __shared__ int4 tfix[kFix ? NT : 1];      // float: fixed-point x, y, z from the group's corner; weight bits
  __shared__ V4 tloc[kFix ? 1 : NT];        // double: cell-local x, y, z and the charge weight
  __shared__ V4 toff[kFix ? 1 : NT];        // double: cell-corner offset from the group's first cell
  __shared__ V4 tvel[HVP ? NT : 1];         // HVP: the candidates' v (in R)
  // neighbourhood of a group's cell: DIV cells on each side along each axis
  // (cells of edge >= r_c / DIV), as NR row ranges of W cells
  constexpr int W = 2 * DIV + 1;
  constexpr int NR = W * W;
  constexpr int RPL = (NR + 15) / 16;   // row ranges per lane of a group
  __shared__ int rstart[kWaveGroups][NR], rpre[kWaveGroups][NR + 1];
  __shared__ int2 royz[kFix ? kWaveGroups : 1][kFix ? NR : 1];   // float: the rows' y, z offsets in units
  __shared__ int gtot[kWaveGroups];
  // Work-group b runs on XCD b % 8 (round-robin dealing). Runs of kXcdRun
  // consecutive waves of groups (spatial neighbours, which share candidates)
  // go to one XCD, so its L2 serves their shared candidates once; the runs
  // are dealt to the XCDs in turn, which keeps dense and sparse regions
  // spread over all of them.
  // dense-cell groups at desc[0 ..), the others at desc[gcap - 1 - i]
  const int ndense = counter[0], ngroups = ndense + counter[1];
  const int nwaves = (ngroups + kWaveGroups - 1) / kWaveGroups;
  const int xcd = (int)(blockIdx.x % kXcds), k = (int)(blockIdx.x / kXcds);
  const int wave = ((k / kXcdRun) * kXcds + xcd) * kXcdRun + k % kXcdRun;
  if (wave >= nwaves) return;
  const int gbase = wave * kWaveGroups;
  // load-balance record (profiling only): the wave's start and end on the
  // constant 100 MHz real-time clock
  const unsigned long long t_start = wclock ? __builtin_amdgcn_s_memrealtime() : 0ull;
  const int lane = threadIdx.x, q = lane >> 4, ql = lane & 15;
  const int gid = gbase + q;
  const bool gvalid = gid < ngroups;
  int2 gd = make_int2(0, 0);
  if (gvalid) gd = desc[gid < ndense ? gid : gcap - 1 - (gid - ndense)];
  const int nx = geo.ncell[0], ny = geo.ncell[1], nz = geo.ncell[2];
  const R cux = (R)geo.cu[0], cuy = (R)geo.cu[1], cuz = (R)geo.cu[2];
  const int kex = fix_edge(geo.cu, 0), key_ = fix_edge(geo.cu, 1), kez = fix_edge(geo.cu, 2);
  // float form: fixed-point positions relative to O, (kex/2, key/2, kez/2)
  // units from the group cell's corner; the offset is common to targets and
  // candidates, so the hit loop's integer separations do not change
  const int hx = kex >> 1, hy = key_ >> 1, hz = kez >> 1;
  const R fu = (R)fix_unit(geo.cu);
  int cx0 = 0, cy = 0, cz = 0;
  if (gvalid) {
    const uint32_t k0 = keys[gd.x];
    cx0 = (int)(k0 % (uint32_t)nx);
    cy = (int)((k0 / (uint32_t)nx) % (uint32_t)ny);
    cz = (int)(k0 / ((uint32_t)nx * (uint32_t)ny));
  }
  // NR candidate ranges per group, range r = (dy + DIV) + W (dz + DIV) on
  // lane r % 16 of the group's quarter: cells cx0-DIV .. cx0+DIV of the row
  // (cy+dy, cz+dz); their lengths' prefix (in range order) in rpre
  const int cx0c = cx0 & 7;   // float form: the group's cell x index mod 8 (the records' x code)
  int lens[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int r = ql + 16 * u;
    int b = 0, e = 0;
    if (r < NR) {
      const int dy = r % W - DIV, dz = r / W - DIV;
      const int y = cy + dy, z = cz + dz;
      if (gvalid && y >= 0 && y < ny && z >= 0 && z < nz) {
        const int row = (z * ny + y) * nx;
        const int xlo = cx0 > DIV ? cx0 - DIV : 0, xhi = cx0 + DIV < nx ? cx0 + DIV : nx - 1;
        b = cs[row + xlo];
        e = cs[row + xhi + 1];
      }
      rstart[q][r] = b;
      if constexpr (kFix) royz[q][r] = make_int2(dy * key_ - hy, dz * kez - hz);
    }
    lens[u] = e - b;
  }
  int tot = 0;
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    int inc = lens[u];
    for (int off = 1; off < 16; off <<= 1) {
      const int v = __shfl_up(inc, off, 16);
      if (ql >= off) inc += v;
    }
    if (ql + 16 * u < NR) rpre[q][ql + 16 * u + 1] = tot + inc;
    tot += __shfl(inc, 15, 16);
  }
  if (ql == 0) {
    rpre[q][0] = 0;
    gtot[q] = tot;
  }
  wave_sync();
  // the target of this lane
  const bool active = gvalid && ql < gd.y;
  R lx = 0, ly = 0, lz = 0, tw = 0;
  int ix = 0, iy = 0, iz = 0;
  int tres = 0;   // float form, packed records: the target's position residuals
  double vi[3] = {0.0, 0.0, 0.0};   // HVP: the target's v
  if (active) {
    // every target of a group is in the group's cell (cell offset 0)
    const int j = gd.x + ql;
    const PPPos<R> me = rec[j];
    if constexpr (kFix) {
      ix = (me.x & kFixMask) - (kFixBias + hx);
      iy = me.y - hy;
      iz = me.z - hz;
      tres = __float_as_int(me.w);
    } else {
      lx = me.x;
      ly = me.y;
      lz = me.z;
    }
    tw = PACKED ? (R)1 : rec_w(me, geo);
    if constexpr (HVP)
      for (int d = 0; d < 3; ++d) vi[d] = hv_in[3 * j + d];
  }
  // cutoff test: r^2 - lim = (|t|^2 + (|c|^2 - lim)) - 2 t.c with lim =
  // 1 + margin. double: the margin covers the rounding of the expanded form
  // for positions within DIV + 1 cell edges of the group's corner
  // (|c|^2 <= 3 (DIV + 1)^2 cu^2); float: the fp16 form above
  const double cmax = fmax(geo.cu[0], fmax(geo.cu[1], geo.cu[2]));
  const R lim = kFix ? (R)fp16_test_lim(cmax) : (R)(1.0 + 1e-5 * fmax(1.0, (DIV + 1) * (DIV + 1) * cmax * cmax));
  R t2x = 0, t2y = 0, t2z = 0, tt = 0;
  uint32_t tP = 0u, tQ = 0u;   // float: fp16 (-2 Tx, -2 Ty) and (-2 Tz, 1)
  if constexpr (kFix) {
    const _Float16 hx_ = (_Float16)((R)ix * fu), hy_ = (_Float16)((R)iy * fu), hz_ = (_Float16)((R)iz * fu);
    tP = __builtin_bit_cast(uint32_t, half2v{(_Float16)-2 * hx_, (_Float16)-2 * hy_});
    tQ = __builtin_bit_cast(uint32_t, half2v{(_Float16)-2 * hz_, (_Float16)1});
    tt = (float)hx_ * (float)hx_ + (float)hy_ * (float)hy_ + (float)hz_ * (float)hz_;
  } else {
    const R tx = active ? lx : (R)1e18;
    t2x = (R)-2 * tx;
    t2y = (R)-2 * ly;
    t2z = (R)-2 * lz;
    tt = tx * tx + ly * ly + lz * lz;
  }
  const int L = gtot[q];
  const int S = (L + kTileK - 1) / kTileK;
  const int nt = max(max((gtot[0] + kTileK - 1) / kTileK, (gtot[1] + kTileK - 1) / kTileK),
                     max((gtot[2] + kTileK - 1) / kTileK, (gtot[3] + kTileK - 1) / kTileK));
  // slot s = 16h + ql of tile t holds candidate ((s/kRun) S + t) kRun +
  // s%kRun; it advances by kRun per tile and its row range index monotonically
  int cq[kPerLane], cr[kPerLane];
#pragma unroll
  for (int h = 0; h < kPerLane; ++h) {
    const int slot = 16 * h + ql;
    cq[h] = (slot / kRun) * S * kRun + slot % kRun;
    int r = 0;
#pragma unroll
    for (int k = 1; k < NR; ++k) r += (cq[h] >= rpre[q][k]) ? 1 : 0;
    cr[h] = r;
  }
  PPPos<R> nx_o[kPerLane] = {};
  int nx_c[kFix ? 1 : kPerLane];   // double form: the candidate's cell x offset
  bool nx_ok[kPerLane];
  double nx_v[HVP ? kPerLane : 1][3];
  // The loads are unconditional (a slot past the group's candidates reads
  // the group's first particle, a valid index), so they stay in flight
  // across the tests and hit loop of the current tile.
  auto fetch = [&](int t) {
#pragma unroll
    for (int h = 0; h < kPerLane; ++h) {
      const int qi = cq[h] + kRun * t;
      nx_ok[h] = t < S && qi < L;
      if (nx_ok[h])
        while (qi >= rpre[q][cr[h] + 1]) ++cr[h];
      const int k = nx_ok[h] ? rstart[q][cr[h]] + (qi - rpre[q][cr[h]]) : gd.x;
      nx_o[h] = rec[k];
      if constexpr (!kFix) nx_c[h] = (int)(keys[k] % (uint32_t)nx) - cx0;
      if constexpr (HVP)
        for (int d = 0; d < 3; ++d) nx_v[h][d] = hv_in[3 * k + d];
    }
  };
  fetch(0);
  // Float form: the pair function takes r^2 in fixed-point units squared,
  // its constants scaled by the unit u (kappa u, 2 kappa u / sqrt(pi),
  // -kappa^2 u^2 log2 e), so no hit multiplies by u^2. Its value is then
  // g / u^3, and the sums are scaled back once per particle (1 / u^2 for
  // the force, whose separations are in units; 1 / u for the potential).
  const double fud = kFix ? fix_unit(geo.cu) : 1.0;
  PairK<R> pk;
  pk.kappa = (R)(geo.kappa * fud);
  pk.c2k = (R)(kTwoOverSqrtPi * geo.kappa * fud);
  pk.half_kappa = (R)(0.5 * geo.kappa * fud);
  pk.ek = (R)(-geo.kappa * geo.kappa * fud * fud * 1.44269504088896340736);
  const R rlim = (R)(1.0 / (fud * fud));   // the cutoff, in the units of r2
  Acc3<R> acc;
  double e_acc = 0.0;
  int pairs = 0;
  for (int t = 0; t < nt; ++t) {
    // 1. stage the prefetched candidates
#pragma unroll
    for (int h = 0; h < kPerLane; ++h) {
      V4 c{(R)1e18, (R)0, (R)0, (R)1e30};
      if constexpr (kFix) {
        // computed for every slot (a slot past the group's candidates holds
        // a stale record) and then, past them, replaced by C = 0, W = +inf,
        // which no cutoff test passes
        // the candidate's cell offset along the row from the x codes (mod 8,
        // |offset| <= DIV), its row's y, z offsets from the range
        const int raw = nx_o[h].x;
        const int dxc = (int)__builtin_amdgcn_sbfe((unsigned)((int)((unsigned)raw >> kXCodeShift) - cx0c), 0, 3);
        const int2 oyz = royz[q][cr[h]];
        const int4 fx = make_int4((raw & kFixMask) - (kFixBias + hx) + dxc * kex, nx_o[h].y + oyz.x,
                                  nx_o[h].z + oyz.y, __float_as_int(nx_o[h].w));
        // C: the float coordinates cut to fp16's 11 significant bits (toward
        // zero, exact in the packing below), so that W is |C|^2 - lim
        const float rx = __uint_as_float(__float_as_uint((R)fx.x * fu) & 0xffffe000u);
        const float ry = __uint_as_float(__float_as_uint((R)fx.y * fu) & 0xffffe000u);
        const float rz = __uint_as_float(__float_as_uint((R)fx.z * fu) & 0xffffe000u);
        const float w = fmaf(rx, rx, fmaf(ry, ry, fmaf(rz, rz, -lim)));
        reinterpret_cast<u32x2*>(tileh)[TSH * q + 16 * h + ql] =
            nx_ok[h] ? u32x2{pack_rtz(rx, ry), pack_rtz(rz, w)} : u32x2{0u, 0x7c000000u};
        tfix[TS * q + 16 * h + ql] = fx;
      } else {
        V4 cl{(R)0, (R)0, (R)0, (R)0}, co{(R)0, (R)0, (R)0, (R)0};
        const int dy = cr[h] % W - DIV, dz = cr[h] / W - DIV;
        if (nx_ok[h]) {
          cl = V4{nx_o[h].x, nx_o[h].y, nx_o[h].z, nx_o[h].w};
          co = V4{(R)nx_c[h] * cux, (R)dy * cuy, (R)dz * cuz, (R)0};
          c.x = cl.x + co.x;
          c.y = cl.y + co.y;
          c.z = cl.z + co.z;
          c.w = c.x * c.x + c.y * c.y + c.z * c.z - lim;
        }
        tloc[TS * q + 16 * h + ql] = cl;
        toff[TS * q + 16 * h + ql] = co;
      }
      if constexpr (HVP)
        tvel[TS * q + 16 * h + ql] = nx_ok[h] ? V4{(R)nx_v[h][0], (R)nx_v[h][1], (R)nx_v[h][2], (R)0}
                                              : V4{(R)0, (R)0, (R)0, (R)0};
      if constexpr (!kFix) tile[TS * q + 16 * h + ql] = c;
    }
    wave_sync();
    fetch(t + 1);
    // 2. hit masks (group-relative positions). The sign bit of r2 - lim is
    //    shifted into the mask (alignbit: m = (m << 1) | (bits >> 31)), so
    //    candidate k of a half-tile ends at bit 31 - k. The test is a little
    //    generous; the evaluation below repeats it exactly on the precise
    //    separation.
    uint32_t m0 = 0u, m1 = 0u;
    if constexpr (kFix) {
      // one 16-byte read per two candidates: (Cx, Cy), (Cz, W) of candidates
      // 2k and 2k + 1
      const u32x4* hq = tileh + (TSH / 2) * q;
      const half2v P = as_half2(tP);
#pragma unroll 4
      for (int k = 0; k < 16; ++k) {
        const u32x4 c = hq[k];
        m0 = mask_shift_in(m0, __builtin_amdgcn_fdot2(P, as_half2(c.x), dot2_acc(tQ, c.y, tt), false));
        m0 = mask_shift_in(m0, __builtin_amdgcn_fdot2(P, as_half2(c.z), dot2_acc(tQ, c.w, tt), false));
      }
#pragma unroll 4
      for (int k = 16; k < 32; ++k) {
        const u32x4 c = hq[k];
        m1 = mask_shift_in(m1, __builtin_amdgcn_fdot2(P, as_half2(c.x), dot2_acc(tQ, c.y, tt), false));
        m1 = mask_shift_in(m1, __builtin_amdgcn_fdot2(P, as_half2(c.z), dot2_acc(tQ, c.w, tt), false));
      }
    } else {
      const V4* tq = tile + TS * q;
#pragma unroll 4
      for (int k = 0; k < 32; ++k) {
        const V4 c = tq[k];
        const R v = fma(t2z, c.z, fma(t2y, c.y, fma(t2x, c.x, tt + c.w)));
        m0 = mask_shift_in(m0, v);
      }
#pragma unroll 4
      for (int k = 0; k < 32; ++k) {
        const V4 c = tq[32 + k];
        const R v = fma(t2z, c.z, fma(t2y, c.y, fma(t2x, c.x, tt + c.w)));
        m1 = mask_shift_in(m1, v);
      }
    }
    if (!active) m0 = m1 = 0u;
    // 3. own hits (the particle itself and coincident ones give r2 = 0).
    //    The masks hold candidate k of a half-tile at bit 31 - k; reversed
    //    once per tile into one 64-bit word, bit k is candidate k, and the
    //    lowest set bit is taken and cleared each round. Float form:
    //    separations and r2 in fixed-point units (the pair constants carry
    //    the unit), scaled back in the sums at the end.
    R sx = 0, sy = 0, sz = 0;
    uint64_t hm = ((uint64_t)__builtin_bitreverse32(m1) << 32) | __builtin_bitreverse32(m0);
    while (hm) {
      const int k = (int)__builtin_ctzll(hm);
      hm &= hm - 1;
      R dx, dy, dz, wj, r2;
      if constexpr (kFix) {
        const int4 cf = tfix[TS * q + k];
        dx = (R)(ix - cf.x);
        dy = (R)(iy - cf.y);
        dz = (R)(iz - cf.z);
        R d2 = dx * dx + dy * dy + dz * dz;
        if constexpr (PACKED) {
          wj = (R)1;
          if (d2 < kCloseUnits2) {
            // a close pair: add the difference of the sub-unit residuals
            const R s = (R)1 / (R)(1 << kResBits);
            dx += (R)(res_field(tres, 0) - res_field(cf.w, 0)) * s;
            dy += (R)(res_field(tres, 1) - res_field(cf.w, 1)) * s;
            dz += (R)(res_field(tres, 2) - res_field(cf.w, 2)) * s;
            d2 = dx * dx + dy * dy + dz * dz;
          }
        } else {
          wj = __int_as_float(cf.w);
        }
        r2 = d2;
      } else {
        const V4 cl = tloc[TS * q + k];
        const V4 co = toff[TS * q + k];
        dx = (lx - cl.x) - co.x;
        dy = (ly - cl.y) - co.y;
        dz = (lz - cl.z) - co.z;
        wj = cl.w;
        r2 = dx * dx + dy * dy + dz * dz;
      }
      if constexpr (HVP && kFix) {
        if (r2 > (R)0 && r2 < rlim) {
          // float: in the cutoff unit (rho = r fu), t = 1/(1 + kappa rho/2),
          // erfc = e t P(t) with e = exp(-kappa^2 rho^2), as in the force
          const V4 vj = tvel[TS * q + k];
          const float fuf = (float)fud;
          const float dx_ = dx * fuf, dy_ = dy * fuf, dz_ = dz * fuf;
          const float s2 = dx_ * dx_ + dy_ * dy_ + dz_ * dz_;
          const float rinv = __builtin_amdgcn_rsqf(s2);
          const float r = s2 * rinv, rinv2 = rinv * rinv;
          const float kap = (float)geo.kappa, c2k = (float)(kTwoOverSqrtPi * geo.kappa);
          const float t = __builtin_amdgcn_rcpf(fmaf(0.5f * kap, r, 1.0f));
          const float ex = __builtin_amdgcn_exp2f(-kap * kap * kLog2e * s2);
          const float ec = ex * t * erfcx_poly(t);
          const float g = fmaf(ec, rinv, c2k * ex);
          const float gp = -ec * rinv2 - c2k * ex * rinv - 2.0f * c2k * kap * kap * r * ex;
          const float f = g * rinv2;
          const float fp_r = (gp - 2.0f * g * rinv) * rinv2 * rinv;
          const float dvx = (float)vi[0] - vj.x, dvy = (float)vi[1] - vj.y, dvz = (float)vi[2] - vj.z;
          const float dd = dx_ * dvx + dy_ * dvy + dz_ * dvz;
          sx += wj * (f * dvx + fp_r * dx_ * dd);
          sy += wj * (f * dvy + fp_r * dy_ * dd);
          sz += wj * (f * dvz + fp_r * dz_ * dd);
        }
      } else if constexpr (HVP) {
        if (r2 > (R)0 && r2 < rlim) {
          // the pair Jacobian applied to v_i - v_j, one reciprocal per pair
          const V4 vj = tvel[TS * q + k];
          const double dvx = vi[0] - vj.x, dvy = vi[1] - vj.y, dvz = vi[2] - vj.z;
          const double dd = dx * dvx + dy * dvy + dz * dvz;
          const double kap = geo.kappa, c2k = kTwoOverSqrtPi * kap;
          const double rinv = 1.0 / sqrt(r2);
          const double r = r2 * rinv, rinv2 = rinv * rinv;
          const double ex = exp(-kap * kap * r2), ec = erfc(kap * r);
          const double g = ec * rinv + c2k * ex;
          const double gp = -ec * rinv2 - c2k * ex * rinv - 2.0 * c2k * kap * kap * r * ex;
          const double f = g * rinv2;
          const double fp_r = (gp - 2.0 * g * rinv) * rinv2 * rinv;
          sx += wj * (f * dvx + fp_r * dx * dd);
          sy += wj * (f * dvy + fp_r * dy * dd);
          sz += wj * (f * dvz + fp_r * dz * dd);
        }
      } else if (r2 > (R)0 && r2 < rlim) {
        R ep;
        const R g = pair_scalar(r2, wj, pk, ENERGY ? &ep : nullptr);
        sx += g * dx;
        sy += g * dy;
        sz += g * dz;
        if (ENERGY) {
          e_acc += (double)ep;
          ++pairs;
        }
      }
    }
    acc.add(sx, sy, sz);
    wave_sync();
  }
  if (HVP && active) {
    for (int d = 0; d < 3; ++d) hv_out[3 * (gd.x + ql) + d] = (double)acc.get(d) * (double)tw;
  } else if (active) {
    const R unit = (R)(1.0 / (fud * fud));   // separations in units: g u^-3 times d u
    PPRec<R> f;
    f.x = acc.get(0) * (tw * unit);
    f.y = acc.get(1) * (tw * unit);
    f.z = acc.get(2) * (tw * unit);
    f.w = (R)0;
    out[gd.x + ql] = f;
  }
  if (wclock && threadIdx.x == 0) {
    wclock[2 * wave] = t_start;
    wclock[2 * wave + 1] = __builtin_amdgcn_s_memrealtime();
  }
  if (ENERGY) {
    e_acc *= 0.5 * (double)tw / fud;   // each unordered pair is met twice
    for (int off = 32; off > 0; off >>= 1) {
      e_acc += __shfl_xor(e_acc, off);
      pairs += __shfl_xor(pairs, off);
    }
    if (lane == 0) {
      atomicAdd(energy, e_acc);
      atomicAdd(energy + 2, (double)pairs);
    }
  }
}

}  // namespace

int pp_group_bound(int64_t n, const Geo& geo) {
  // runs of <= 16 particles of one cell: at most n/16 full runs plus one
  // partial run per cell, and never more than n
  long long b = n / kGroupRun + geo.ncells + 1;
  if (b > n + 1) b = n + 1;
  return (int)b;
}

// Work-groups of the pair kernel: the bound on its waves, rounded up to
// whole rounds of kXcdRun waves on each of the 8 XCDs (every wave index
// below the bound is then some work-group's under the XCD mapping).
unsigned pp_blocks(int64_t n, const Geo& geo) {
  const long long waves = (pp_group_bound(n, geo) + kWaveGroups - 1) / kWaveGroups;
  const long long round = (long long)kXcds * kXcdRun;
  return (unsigned)((waves + round - 1) / round * round);
}

template <typename R>
constexpr bool kPackable = std::is_same<R, float>::value;

template <typename R, int DIV>
void launch_pp_div(unsigned blocks, int gcap, const PPPos<R>* rec, const uint32_t* keys, const int* cell_start,
                   const Geo& geo, const int2* desc, int* counter, PPRec<R>* out, double* energy,
                   hipStream_t st, unsigned long long* wclock) {
  const bool packed = std::is_same<R, float>::value && geo.wpacked;
  if (energy && packed)
    k_pp<R, true, kPackable<R>, false, DIV><<<blocks, 64, 0, st>>>(desc, counter, gcap, rec, keys, cell_start, geo, out,
                                                                   energy);
  else if (energy)
    k_pp<R, true, false, false, DIV><<<blocks, 64, 0, st>>>(desc, counter, gcap, rec, keys, cell_start, geo, out, energy);
  else if (packed)
    k_pp<R, false, kPackable<R>, false, DIV><<<blocks, 64, 0, st>>>(desc, counter, gcap, rec, keys, cell_start, geo, out,
                                                                    nullptr, nullptr, nullptr, wclock);
  else
    k_pp<R, false, false, false, DIV><<<blocks, 64, 0, st>>>(desc, counter, gcap, rec, keys, cell_start, geo, out,
                                                             nullptr, nullptr, nullptr, wclock);
}

template <typename R>
void launch_pp(int64_t n, const PPPos<R>* rec, const uint32_t* keys, const int* cell_start,
               const Geo& geo, const int2* desc, int* counter, PPRec<R>* out, double* energy,
               hipStream_t st, unsigned long long* wclock) {
  // one wave per quad of groups; waves beyond the groups built leave at once
  const unsigned blocks = pp_blocks(n, geo);
  const int gcap = pp_group_bound(n, geo);
  if (geo.pp_div == 2)
    launch_pp_div<R, 2>(blocks, gcap, rec, keys, cell_start, geo, desc, counter, out, energy, st, wclock);
  else
    launch_pp_div<R, 1>(blocks, gcap, rec, keys, cell_start, geo, desc, counter, out, energy, st, wclock);
}

template <typename R, int DIV>
void launch_pp_hvp_div(unsigned blocks, int gcap, const PPPos<R>* rec, const uint32_t* keys, const int* cell_start,
                       const Geo& geo, const int2* desc, int* counter, const double* v_sorted,
                       double* out_sorted, hipStream_t st) {
  const bool packed = std::is_same<R, float>::value && geo.wpacked;
  if (packed)
    k_pp<R, false, kPackable<R>, true, DIV><<<blocks, 64, 0, st>>>(desc, counter, gcap, rec, keys, cell_start, geo,
                                                                   nullptr, nullptr, v_sorted, out_sorted);
  else
    k_pp<R, false, false, true, DIV><<<blocks, 64, 0, st>>>(desc, counter, gcap, rec, keys, cell_start, geo, nullptr,
                                                            nullptr, v_sorted, out_sorted);
}

template <typename R>
void launch_pp_hvp(int64_t n, const PPPos<R>* rec, const uint32_t* keys, const int* cell_start,
                   const Geo& geo, const int2* desc, int* counter, const double* v_sorted, double* out_sorted,
                   hipStream_t st) {
  // the tiled pair kernel in its Hessian-vector mode, over the cell sort's groups
  const unsigned blocks = pp_blocks(n, geo);
  const int gcap = pp_group_bound(n, geo);
  if (geo.pp_div == 2)
    launch_pp_hvp_div<R, 2>(blocks, gcap, rec, keys, cell_start, geo, desc, counter, v_sorted, out_sorted, st);
  else
    launch_pp_hvp_div<R, 1>(blocks, gcap, rec, keys, cell_start, geo, desc, counter, v_sorted, out_sorted, st);
}
template void launch_pp_hvp<float>(int64_t, const PPPos<float>*, const uint32_t*, const int*, const Geo&,
                                   const int2*, int*, const double*, double*, hipStream_t);
template void launch_pp_hvp<double>(int64_t, const PPPos<double>*, const uint32_t*, const int*, const Geo&,
                                    const int2*, int*, const double*, double*, hipStream_t);

template void launch_pp<float>(int64_t, const PPPos<float>*, const uint32_t*, const int*, const Geo&,
                               const int2*, int*, PPRec<float>*, double*, hipStream_t, unsigned long long*);
template void launch_pp<double>(int64_t, const PPPos<double>*, const uint32_t*, const int*, const Geo&,
                                const int2*, int*, PPRec<double>*, double*, hipStream_t, unsigned long long*);

}  // namespace p3m
