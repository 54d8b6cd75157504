// Internal definitions shared by the HIP sources of libp3m (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace p3m {

// Error bits of the device status word.
constexpr int kBitDomain = 1;     // a particle outside the mesh with zoom off
constexpr int kBitNonFinite = 2;  // a non-finite position

constexpr int kThreads = 256;     // block size of the particle kernels
// PP work groups: runs of at most kGroupRun consecutive sorted particles of
// one cell (built by the cell sort, read by the PP kernel). Groups of cells
// of at least kDenseCell particles come first, in cell order, from the front
// of the group array; the others follow, in cell order, stored from its back
// (index cap - 1 - i): the long waves of dense regions start first and the
// short ones fill the end of the launch, while neighbours stay adjacent.
constexpr int kGroupRun = 16;
constexpr int kDenseCell = 2 * kGroupRun;
constexpr int kXcds = 8;          // MI355X: work-groups are dealt round-robin to 8 XCDs

// Placement of one evaluation, written on the device by the finalize kernel.
// Lengths inside the kernels are measured in the unit Lu = s * r_c, in which
// the cutoff is 1, the Ewald parameter is kappa = a * r_c and the PP cell and
// mesh spacings are zoom-invariant constants; physical forces are the
// internal ones times fscale = k_e q^2 / Lu^2.
struct Place {
  double x0[3];        // position of mesh node 0 (m)
  double s;            // zoom
  double inv_hp[3];    // 1 / (s h_d)
  double inv_lu;       // 1 / (s r_c)
  double inv_cell[3];  // 1 / (s c_d), c_d = PP cell edge at zoom 1
  double fscale;       // k_e q^2 / (s r_c)^2
  double phiscale;     // 1 / (s r_c): internal potential -> 1/m
  double pad[3];
};
static_assert(sizeof(Place) == 16 * sizeof(double), "Place layout");

// Mesh kernel tables (the values of p3m_opts.influence).
constexpr int kInfluenceSampled = 0;
constexpr int kInfluenceOptimal = 1;
constexpr int kInfluencePrincipal = 2;
constexpr int kInfluenceLattice = 3;

// Row stride (in k_x) of the half spectrum and of the z pass's copy of the
// kernel table: N_x + 1 values padded to a multiple of 16, so that the
// 16-wide rows of the strided y and z passes are whole cache lines.
__host__ __device__ inline int spec_stride(int nx) { return (nx + 1 + 15) & ~15; }

// Zoom-invariant geometry, passed by value.
struct Geo {
  int grid[3];         // mesh nodes per axis
  int ncell[3];        // PP cells per axis
  long long ncells;    // product of ncell
  double h[3];         // mesh spacing at zoom 1 (m)
  double rc;           // cutoff at zoom 1 (m)
  double hu[3];        // h_d / r_c
  double cu[3];        // c_d / r_c (PP cell edge in units of the cutoff)
  double kappa;        // a * r_c
  double ke_q2;        // k_e q^2
  int order;           // 1 CIC, 2 TSC
  int zoom;            // 1 zoom on
  int gather;          // 0 variational, 1 momentum-conserving (mesh E by central differences)
  int cathode;         // 1: grounded plane z = zc (image charges on the mesh)
  int influence;       // mesh kernel table: kInfluence*
  int wpacked;         // per call: float records carry position residuals, weights all 1
  int mdiff;           // float mesh in the difference form (three difference meshes, no phi)
  int pp_div;          // PP cells per cutoff along each axis (1 or 2): cell edge >= r_c / pp_div
  double zc;           // plane position (m)
};

// Nodes the bunch may span so that every assignment stencil lies on the mesh
// (N-1 for CIC, N-2 for TSC), less the outer node layer on each side when
// the gather differences the potential across the stencil's nodes.
__host__ __device__ inline double usable_nodes(const Geo& g, int d) {
  return (double)((g.order == 1 ? g.grid[d] - 1 : g.grid[d] - 2) - (g.gather ? 2 : 0));
}

template <typename T>
struct C2 {
  T x, y;
};

template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ C2<T> cconj(C2<T> a) { return {a.x, -a.y}; }
// multiply by -i
template <typename T>
__device__ __forceinline__ C2<T> cmul_mi(C2<T> a) { return {a.y, -a.x}; }

// Sorted particle records.
template <typename R> struct PPRec;              // per-particle vector + weight (PP force output)
template <> struct alignas(16) PPRec<float> { float x, y, z, w; };
template <> struct alignas(32) PPRec<double> { double x, y, z, w; };

// Position in the own PP cell + weight. float form: fixed point in one
// unit for all axes, fix_unit = (largest cell edge) / 2^kFixBits Lu; the
// cell edge of axis d is the integer fix_edge(d) units, so separations of
// particles in neighbouring cells are exact integers (rounded once, to
// float, after the subtraction). The x slot holds the position plus
// kFixBias in its low 29 bits and the cell's x index modulo 8 in its top
// three (kXCodeShift), from which the pair kernel reads a candidate's cell
// offset along its row of cells (|offset| <= 2). double form: offset from
// the cell corner in units of Lu.
constexpr int kFixBits = 28;
constexpr int kFixBias = 1 << 27;                        // x slot: position + bias in [0, 2^29)
constexpr int kXCodeShift = 29;                          // bits 29..31: cell x index mod 8
constexpr int kFixMask = (1 << kXCodeShift) - 1;
struct alignas(16) PPFix { int x, y, z; float w; };
template <typename R> struct PPPosOf { using type = PPRec<R>; };
template <> struct PPPosOf<float> { using type = PPFix; };
template <typename R> using PPPos = typename PPPosOf<R>::type;

// Sub-unit residuals of a float record. A fixed-point position rounds the
// position to the unit, so a separation of d units is good to about 1/d:
// for the closest pairs (a few thousand units) that is 1e-4. When every
// weight is 1 (Geo::wpacked), the weight slot holds the residual u - rint(u)
// of each axis instead, in units of 2^-kResBits, as three signed 10-bit fields;
// pairs closer than kCloseUnits add them back.
constexpr int kResBits = 10;
constexpr float kCloseUnits2 = 70368744177664.0f;   // (2^23 units)^2: beyond, rounding is below float's
__host__ __device__ inline float rec_w(const PPFix& r, const Geo& g) { return g.wpacked ? 1.0f : r.w; }
template <typename R>
__host__ __device__ inline R rec_w(const PPRec<R>& r, const Geo&) { return r.w; }
// Weight of sorted particle j read from its record only when the records
// carry weights (a uniform branch: residual-carrying records are not read).
__device__ __forceinline__ float rec_weight(const PPFix* pp, int64_t j, const Geo& g) {
  if (g.wpacked) return 1.0f;
  return pp[j].w;
}
template <typename R>
__device__ __forceinline__ R rec_weight(const PPRec<R>* pp, int64_t j, const Geo&) { return pp[j].w; }
// Residual field f (0..2) of a packed weight slot, sign-extended. The bit
// field builtin is typed unsigned; the cast keeps the field difference signed.
__device__ __forceinline__ int res_field(int v, int f) {
  return (int)__builtin_amdgcn_sbfe(v, 10 * f, 10);
}

__host__ __device__ inline double fix_unit(const double cu[3]) {
  const double m = cu[0] > cu[1] ? (cu[0] > cu[2] ? cu[0] : cu[2]) : (cu[1] > cu[2] ? cu[1] : cu[2]);
  return m / (double)(1 << kFixBits);
}
__host__ __device__ inline int fix_edge(const double cu[3], int d) { return (int)rint(cu[d] / fix_unit(cu)); }

template <typename R> struct MeshRec;            // stencil origin node + fractional offsets
template <> struct alignas(16) MeshRec<float> { float fx, fy, fz; int base; };
template <> struct alignas(32) MeshRec<double> { double fx, fy, fz; long long base; };

__host__ __device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Floor of a double clamped to [lo, hi] in floating point first, so NaN and
// huge values map into range before the integer conversion.
__device__ __forceinline__ int floor_clamp(double v, int lo, int hi) {
  double f = floor(v);
  f = fmax(f, (double)lo);
  f = fmin(f, (double)hi);
  return (int)f;
}

}  // namespace p3m
