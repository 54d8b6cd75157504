// Charge assignment to the mesh and force interpolation back to particles.
//
// Assignment weight of node m for a particle at mesh coordinate u is the
// cardinal B-spline b_p(u - m) per axis (Sec. 2.4.2, eq.
// interpolation_splines_b0: b1, cloud-in-cell; b2, triangular-shaped cloud,
// is the next step of the same recursion):
//   CIC, f = u - floor(u):        w = (1 - f, f)              w' = (-1, 1)
//   TSC, d = u - round(u):        w = ((1/2-d)^2/2, 3/4-d^2, (1/2+d)^2/2)
//                                 w' = (-(1/2-d), -2d, 1/2+d)  w'' = (1, -2, 1)
// Deposit: Q_m = sum_i w_i W_m(x_i)             (Sec. 2.5, eq. eom_p3m_poiss_L)
// Gather:  F_i = -w_i sum_m phi_m grad W_m(x_i) (Sec. 2.5, eq. eom_p3m_coord),
//          the weight gradient read as a finite difference of phi at the
//          nearest nodes (the remark after eq. eom_p3m_coord).
// Lengths are in the unit Lu = s r_c, so grad = (1/hu_d) d/du with hu = h/r_c.
#include <climits>

#include "bbox.h"
#include "launch.h"

namespace p3m {

namespace {

template <typename R, int ORDER>
struct Stencil {
  static constexpr int N = ORDER + 1;
  R w[3][N], dw[3][N];
  __device__ __forceinline__ Stencil(R fx, R fy, R fz) {
    const R f[3] = {fx, fy, fz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (ORDER == 1) {
        w[d][0] = (R)1 - f[d];
        w[d][1] = f[d];
        dw[d][0] = (R)-1;
        dw[d][1] = (R)1;
      } else {
        const R a = (R)0.5 - f[d], b = (R)0.5 + f[d];
        w[d][0] = (R)0.5 * a * a;
        w[d][1] = (R)0.75 - f[d] * f[d];
        w[d][N - 1] = (R)0.5 * b * b;
        dw[d][0] = -a;
        dw[d][1] = (R)-2 * f[d];
        dw[d][N - 1] = b;
      }
    }
  }
};

// Deposit. A block takes 2048 consecutive sorted particles; sorted by PP
// cell they usually cover a small box of nodes. The block accumulates their
// weights in an LDS tile of that box in 64-bit fixed point (integer LDS
// atomics: exact, order-independent, and far cheaper than float LDS
// atomics), then adds the nonzero nodes to the mesh with one float atomic
// each, consecutive lanes on consecutive nodes. A box larger than the tile
// is covered in pieces (z-slabs, or y-bands of one plane), each a pass over
// the block's particles; past kMaxPieces (very sparse bunches) each particle
// adds its weights to the mesh directly, one particle's nodes on as many
// lanes. The fixed-point unit is 2^-s of the
// block's largest |charge weight| with s chosen so that 2048 contributions
// cannot overflow: a node value keeps 50 bits below that weight.
constexpr int kDepItems = 4;
constexpr int kDepThreads = 512;   // 8 waves beside a 64 KB tile
constexpr int kDepChunk = kDepThreads * kDepItems;
constexpr int kTileNodes = 8192;     // 64 KB of int64
constexpr int kMaxPieces = 16;

__device__ __forceinline__ int wave_min(int v) {
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ double wave_maxd(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Nearest integer (ties to even) of |v| < 2^51: adding 1.5 * 2^52 leaves the
// rounded value in the low bits of the sum. A product passed in may fuse
// with the addition into one fma, which rounds the exact product once.
__device__ __forceinline__ long long fix_round(double v) {
  return __double_as_longlong(v + 6755399441055744.0) - 0x4338000000000000ll;
}

// Stencil origin of a sorted particle from its mesh record.
template <typename R>
__device__ __forceinline__ void unpack_base(const MeshRec<R>& m, int nx, unsigned nxy, int b[3]) {
  const unsigned base = (unsigned)m.base;   // < 2^30: at most 1024 nodes per axis
  const unsigned bz = base / nxy, rem = base - bz * nxy;
  const unsigned by = rem / (unsigned)nx;
  b[0] = (int)(rem - by * (unsigned)nx);
  b[1] = (int)by;
  b[2] = (int)bz;
}

// GRAD: the derivative of the deposit along v (sorted [n][3], float64),
// R_m = sum_j w_j grad W_m(x_j) . v_j, in place of the charge. Its values
// are bounded by |w_j| sum_d |v_jd| / (h_d / r_c) (|W| <= 1, |W'| <= 1),
// which takes the place of |w_j| in the fixed-point unit.
template <typename R, typename M, int ORDER, bool GRAD>
__global__ void __launch_bounds__(kDepThreads) k_deposit(int64_t n, const PPPos<R>* __restrict__ pp,
                                                      const MeshRec<R>* __restrict__ mesh, Geo geo,
                                                      const double* __restrict__ v, M* __restrict__ Q) {
  constexpr int NS = ORDER + 1;
  __shared__ long long tile[kTileNodes];
  __shared__ int red[6];
  __shared__ double qred[kDepThreads / 64];
  const int t = threadIdx.x;
  const int nx = geo.grid[0], ny = geo.grid[1];
  const unsigned nxy = (unsigned)nx * (unsigned)ny;
  const int64_t j0 = (int64_t)blockIdx.x * kDepChunk;
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
  double qmax = 0.0;
#pragma unroll
  for (int it = 0; it < kDepItems; ++it) {
    const int64_t j = j0 + it * kDepThreads + t;
    if (j < n) {
      int b[3];
      unpack_base(mesh[j], nx, nxy, b);
      double qa = fabs((double)rec_weight(pp, j, geo));
      if constexpr (GRAD)
        qa *= fabs(v[3 * j]) / geo.hu[0] + fabs(v[3 * j + 1]) / geo.hu[1] + fabs(v[3 * j + 2]) / geo.hu[2];
      qmax = fmax(qmax, qa);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lo[d] = min(lo[d], b[d]);
        hi[d] = max(hi[d], b[d]);
      }
    }
  }
  if (t < 6) red[t] = t < 3 ? INT_MAX : INT_MIN;
  __syncthreads();
  for (int d = 0; d < 3; ++d) {
    const int a = wave_min(lo[d]), c = wave_max(hi[d]);
    if ((t & 63) == 0) {
      atomicMin(&red[d], a);
      atomicMax(&red[3 + d], c);
    }
  }
  qmax = wave_maxd(qmax);
  if ((t & 63) == 0) qred[t >> 6] = qmax;
  __syncthreads();
  qmax = qred[0];
  for (int k = 1; k < kDepThreads / 64; ++k) qmax = fmax(qmax, qred[k]);
  if (red[0] == INT_MAX || qmax == 0.0) return;   // nothing to add (uniform across the block)
  const int o0 = red[0], o1 = red[1], o2 = red[2];
  const int e0 = red[3] - o0 + NS, e1 = red[4] - o1 + NS, e2 = red[5] - o2 + NS;
  const long long plane = (long long)e0 * e1;
  int hz, hy;
  if (plane <= kTileNodes) {
    hz = (int)(kTileNodes / plane);
    hy = e1;
  } else {
    hz = 1;
    hy = kTileNodes / e0;   // e0 <= 1026 < kTileNodes
  }
  const long long pieces = (long long)((e2 + hz - 1) / hz) * ((e1 + hy - 1) / hy);
  if (pieces <= kMaxPieces) {
    // unit 2^-s, s = 50 - ex with qmax < 2^(ex+1): every contribution
    // (weights <= 1) is below 2^51 units, as fix_round needs, and the 2048
    // particles of a block sum to below 2^62 at any node
    const int ex = ilogb(qmax);
    const double toFix = ldexp(1.0, 50 - ex), fromFix = ldexp(1.0, ex - 50);
    for (int pz = 0; pz < e2; pz += hz) {
      const int pe2 = min(hz, e2 - pz);
      for (int py = 0; py < e1; py += hy) {
        const int pe1 = min(hy, e1 - py);
        const int pvol = e0 * pe1 * pe2;
        for (int e = t; e < pvol; e += kDepThreads) tile[e] = 0;
        __syncthreads();
#pragma unroll 1
        for (int it = 0; it < kDepItems; ++it) {
          const int64_t j = j0 + it * kDepThreads + t;
          if (j >= n) continue;
          const MeshRec<R> m = mesh[j];
          const R q = rec_weight(pp, j, geo);
          int b[3];
          unpack_base(m, nx, nxy, b);
          const int rx = b[0] - o0, ry = b[1] - o1 - py, rz = b[2] - o2 - pz;
          if (rz >= pe2 || rz + NS <= 0 || ry >= pe1 || ry + NS <= 0) continue;
          const Stencil<R, ORDER> S(m.fx, m.fy, m.fz);
          double wx[NS], vd[3] = {0.0, 0.0, 0.0};
#pragma unroll
          for (int a = 0; a < NS; ++a) wx[a] = (double)S.w[0][a];
          if constexpr (GRAD)
            for (int d = 0; d < 3; ++d) vd[d] = v[3 * j + d] / geo.hu[d];
#pragma unroll
          for (int c = 0; c < NS; ++c) {
            const int z = rz + c;
            if ((unsigned)z >= (unsigned)pe2) continue;
#pragma unroll
            for (int bb = 0; bb < NS; ++bb) {
              const int y = ry + bb;
              if ((unsigned)y >= (unsigned)pe1) continue;
              unsigned long long* row = reinterpret_cast<unsigned long long*>(tile) + (z * pe1 + y) * e0 + rx;
              if constexpr (GRAD) {
                // q (W'_x W_y W_z v_x + W_x (W'_y W_z v_y + W_y W'_z v_z)) along the row
                const double A = (double)q * S.w[1][bb] * S.w[2][c] * vd[0] * toFix;
                const double B = (double)q * (S.dw[1][bb] * S.w[2][c] * vd[1] + S.w[1][bb] * S.dw[2][c] * vd[2]) * toFix;
#pragma unroll
                for (int a = 0; a < NS; ++a)
                  atomicAdd(row + a, (unsigned long long)fix_round(fma((double)S.dw[0][a], A, wx[a] * B)));
              } else {
                const double wyz = (double)(q * S.w[1][bb] * S.w[2][c]) * toFix;
#pragma unroll
                for (int a = 0; a < NS; ++a) atomicAdd(row + a, (unsigned long long)fix_round(wyz * wx[a]));
              }
            }
          }
        }
        __syncthreads();
        for (int e = t; e < pvol; e += kDepThreads) {
          const long long v = tile[e];
          if (v != 0) {
            const int ex0 = e % e0, ey = (e / e0) % pe1, ez = e / (e0 * pe1);
            atomicAdd(Q + ((long long)(o2 + pz + ez) * ny + (o1 + py + ey)) * nx + (o0 + ex0),
                      (M)((double)v * fromFix));
          }
        }
        __syncthreads();
      }
    }
  } else if constexpr (!GRAD) {
    // Direct atomics with one particle's NS^3 nodes on NS^3 lanes of the
    // wave (two TSC or eight CIC particles per instruction): an instruction
    // then touches about ten cache lines (rows of NS consecutive nodes)
    // instead of one line per lane, and the direct blocks of a sparse halo
    // run about three times faster than with one particle per lane. Each
    // lane loads one record of the wave's 64 particles (coalesced); the
    // loop takes them from their lanes by shuffles, so it waits on no load.
    constexpr int NN = NS * NS * NS, PPI = 64 / NN;
    const int lane = t & 63, sub = lane / NN, node = lane - sub * NN;
    const int a = node % NS, bb = (node / NS) % NS, c = node / (NS * NS);
#pragma unroll 1
    for (int it = 0; it < kDepItems; ++it) {
      const int64_t jw = j0 + it * kDepThreads + (t & ~63);   // the wave's 64 particles
      const int64_t jl = jw + lane;
      MeshRec<R> mine{};
      R qmine = (R)0;
      if (jl < n) {
        mine = mesh[jl];
        qmine = rec_weight(pp, jl, geo);
      }
#pragma unroll 1
      for (int p0 = 0; p0 < 64; p0 += PPI) {
        const int src = min(p0 + sub, 63);   // every lane takes part in the shuffles
        MeshRec<R> m;
        m.fx = __shfl(mine.fx, src);
        m.fy = __shfl(mine.fy, src);
        m.fz = __shfl(mine.fz, src);
        m.base = __shfl(mine.base, src);
        const R q = __shfl(qmine, src);
        if (sub >= PPI || jw + p0 + sub >= n) continue;
        int b[3];
        unpack_base(m, nx, nxy, b);
        const Stencil<R, ORDER> S(m.fx, m.fy, m.fz);
        // this lane's weights, selected by value (no dynamic register index)
        const R wa = a == 0 ? S.w[0][0] : (a == 1 ? S.w[0][1] : S.w[0][NS - 1]);
        const R wb = bb == 0 ? S.w[1][0] : (bb == 1 ? S.w[1][1] : S.w[1][NS - 1]);
        const R wc = c == 0 ? S.w[2][0] : (c == 1 ? S.w[2][1] : S.w[2][NS - 1]);
        atomicAdd(Q + ((long long)(b[2] + c) * ny + (b[1] + bb)) * nx + b[0] + a, (M)(q * wb * wc * wa));
      }
    }
  } else {
#pragma unroll 1
    for (int it = 0; it < kDepItems; ++it) {
      const int64_t j = j0 + it * kDepThreads + t;
      if (j >= n) continue;
      const MeshRec<R> m = mesh[j];
      const R q = rec_weight(pp, j, geo);
      int b[3];
      unpack_base(m, nx, nxy, b);
      const Stencil<R, ORDER> S(m.fx, m.fy, m.fz);
      double vd[3] = {0.0, 0.0, 0.0};
      if constexpr (GRAD)
        for (int d = 0; d < 3; ++d) vd[d] = v[3 * j + d] / geo.hu[d];
#pragma unroll
      for (int c = 0; c < NS; ++c)
#pragma unroll
        for (int bb = 0; bb < NS; ++bb) {
          M* row = Q + ((long long)(b[2] + c) * ny + (b[1] + bb)) * nx + b[0];
          if constexpr (GRAD) {
            const double A = (double)q * S.w[1][bb] * S.w[2][c] * vd[0];
            const double B = (double)q * (S.dw[1][bb] * S.w[2][c] * vd[1] + S.w[1][bb] * S.dw[2][c] * vd[2]);
#pragma unroll
            for (int a = 0; a < NS; ++a) atomicAdd(row + a, (M)(S.dw[0][a] * A + S.w[0][a] * B));
          } else {
            const R wyz = q * S.w[1][bb] * S.w[2][c];
#pragma unroll
            for (int a = 0; a < NS; ++a) atomicAdd(row + a, (M)(wyz * S.w[0][a]));
          }
        }
    }
  }
}

// The stencil sums run in the mesh precision M (the potential differences
// that make the force are small against the potential itself).
// MODE 0, variational: g_d = sum_m phi_m dW_m/du_d.
// MODE 2, variational from the difference meshes D_d phi_m = phi_{m+e_d} -
// phi_m (phi holds the three, one after the other): by the B-spline identity
// b_p'(t) = b_{p-1}(t + 1/2) - b_{p-1}(t - 1/2), the same g_d is
// sum_m D_d phi_m b_{p-1}(u_d - m_d - 1/2) prod_{e != d} b_p(u_e - m_e), with
// b_0 = 1 on the base node (CIC) and b_1 = (1/2 - f, 1/2 + f) on the nodes
// c - 1, c (TSC, f = u - c). No potential (energy) in this mode.
// MODE 1, momentum-conserving: the mesh field by central differences,
// E_{m,d} = -(phi_{m+e_d} - phi_{m-e_d}) / (2 h_d), interpolated with W; on
// the nodes this is g_d = sum_n phi_n (W(n - e_d) - W(n + e_d)) / 2 over the
// stencil widened by one node on each side (inside the mesh: the placement
// keeps stencils off the outer node layer in this mode).
template <typename R, typename M, int ORDER, int MODE>
__global__ void __launch_bounds__(kThreads) k_gather(int64_t n, const PPPos<R>* __restrict__ pp,
                                                     const MeshRec<R>* __restrict__ mesh,
                                                     const PPRec<R>* __restrict__ fpp,
                                                     const uint32_t* __restrict__ perm, Geo geo,
                                                     const Place* __restrict__ pl,
                                                     const M* __restrict__ phi, GatherOut out,
                                                     double* __restrict__ energy) {
  const int64_t j = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  double e_acc = 0.0;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int bad = 0;
  if (j < n) {
    const MeshRec<R> m = mesh[j];
    const R q = rec_weight(pp, j, geo);
    Stencil<M, ORDER> S((M)m.fx, (M)m.fy, (M)m.fz);
    const int nx = geo.grid[0];
    const long long nxy = (long long)nx * geo.grid[1];
    M g[3] = {0, 0, 0};
    M pot = 0;
    if constexpr (MODE == 2) {
      const long long nodes = nxy * geo.grid[2];
      const M f[3] = {(M)m.fx, (M)m.fy, (M)m.fz};
      // weights of b_{p-1} on the axis differenced: one node (CIC) or two (TSC)
      constexpr int ND = ORDER;
      M wd[3][ND];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if constexpr (ORDER == 1) {
          wd[d][0] = (M)1;
        } else {
          wd[d][0] = (M)0.5 - f[d];
          wd[d][ND - 1] = (M)0.5 + f[d];
        }
      }
      // x difference: ND nodes along x, S.N along y and z
      {
        const M* D = phi;
#pragma unroll
        for (int c = 0; c < S.N; ++c)
#pragma unroll
          for (int b = 0; b < S.N; ++b) {
            const M* row = D + m.base + c * nxy + (long long)b * nx;
            M sx = 0;
#pragma unroll
            for (int a = 0; a < ND; ++a) sx += row[a] * wd[0][a];
            g[0] += sx * S.w[1][b] * S.w[2][c];
          }
      }
      {
        const M* D = phi + nodes;
#pragma unroll
        for (int c = 0; c < S.N; ++c)
#pragma unroll
          for (int b = 0; b < ND; ++b) {
            const M* row = D + m.base + c * nxy + (long long)b * nx;
            M sx = 0;
#pragma unroll
            for (int a = 0; a < S.N; ++a) sx += row[a] * S.w[0][a];
            g[1] += sx * wd[1][b] * S.w[2][c];
          }
      }
      {
        const M* D = phi + 2 * nodes;
#pragma unroll
        for (int c = 0; c < ND; ++c)
#pragma unroll
          for (int b = 0; b < S.N; ++b) {
            const M* row = D + m.base + c * nxy + (long long)b * nx;
            M sx = 0;
#pragma unroll
            for (int a = 0; a < S.N; ++a) sx += row[a] * S.w[0][a];
            g[2] += sx * S.w[1][b] * wd[2][c];
          }
      }
    } else if constexpr (MODE == 0) {
#pragma unroll
      for (int c = 0; c < S.N; ++c)
#pragma unroll
        for (int b = 0; b < S.N; ++b) {
          const M* row = phi + m.base + c * nxy + (long long)b * nx;
          M sx = 0, sdx = 0;
#pragma unroll
          for (int a = 0; a < S.N; ++a) {
            const M v = row[a];
            sx += v * S.w[0][a];
            sdx += v * S.dw[0][a];
          }
          g[0] += sdx * S.w[1][b] * S.w[2][c];
          g[1] += sx * S.dw[1][b] * S.w[2][c];
          g[2] += sx * S.w[1][b] * S.dw[2][c];
          pot += sx * S.w[1][b] * S.w[2][c];
        }
    } else {
      constexpr int NE = ORDER + 3;   // widened stencil
      M we[3][NE], ge[3][NE];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int i = 0; i < NE; ++i) we[d][i] = (i >= 1 && i <= S.N) ? S.w[d][i - 1] : (M)0;
#pragma unroll
        for (int i = 0; i < NE; ++i)
          ge[d][i] = (M)0.5 * ((i >= 1 ? we[d][i - 1] : (M)0) - (i + 1 < NE ? we[d][i + 1] : (M)0));
      }
      const M* corner = phi + (m.base - 1 - nx - nxy);
#pragma unroll
      for (int c = 0; c < NE; ++c)
#pragma unroll
        for (int b = 0; b < NE; ++b) {
          const M* row = corner + c * nxy + (long long)b * nx;
          M sw = 0, sg = 0;
#pragma unroll
          for (int a = 0; a < NE; ++a) {
            const M v = row[a];
            sw += v * we[0][a];
            sg += v * ge[0][a];
          }
          g[0] += sg * we[1][b] * we[2][c];
          g[1] += sw * ge[1][b] * we[2][c];
          g[2] += sw * we[1][b] * ge[2][c];
          pot += sw * we[1][b] * we[2][c];
        }
    }
    const double fs = pl->fscale;
    const uint32_t i = out.sorted ? (uint32_t)j : perm[j];
    double fpm[3], fp[3] = {0, 0, 0}, ft[3];
    const PPRec<R> a = fpp[j];
    fp[0] = (double)a.x;
    fp[1] = (double)a.y;
    fp[2] = (double)a.z;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      fpm[d] = -(double)q * (double)g[d] / geo.hu[d];
      ft[d] = fs * (fp[d] + fpm[d]);
    }
    if (out.f)
      for (int d = 0; d < 3; ++d) out.f[3 * i + d] = ft[d];
    if (out.f_pp)
      for (int d = 0; d < 3; ++d) out.f_pp[3 * i + d] = fs * fp[d];
    if (out.f_pm)
      for (int d = 0; d < 3; ++d) out.f_pm[3 * i + d] = fs * fpm[d];
    if (out.p) {
      // the kick(s) and, fused, the next step's drift (leapfrog, Sec. 2.4.3
      // eq. leapfrog), moving the state into this order on the way
      const uint32_t src = out.p_src ? perm[j] : i;
      const double* ps = out.p_src ? out.p_src : out.p;
      double pd[3];
      for (int d = 0; d < 3; ++d) {
        pd[d] = ps[3 * src + d] + out.half_dt * ft[d];
        out.p[3 * i + d] = pd[d];
      }
      if (out.x) {
        const double* xs = out.x_src ? out.x_src : out.x;
        const uint32_t xsrc = out.x_src ? perm[j] : i;
        const double drift = out.part ? out.dt_over_m : 0.0;
        double xi[3];
        for (int d = 0; d < 3; ++d) {
          xi[d] = xs[3 * xsrc + d] + drift * pd[d];
          out.x[3 * i + d] = xi[d];
        }
        if (out.part) bbox_accumulate(xi, lo, hi, bad);
      }
    }
    e_acc = 0.5 * (double)q * (double)pot;
  }
  if (out.part) {   // uniform: every thread of the block reduces the box
    if (bad) atomicOr(out.status, kBitNonFinite);
    bbox_block_store(lo, hi, out.part, (int)gridDim.x);
  }
  if (energy) {
    __shared__ double s[kThreads];
    s[threadIdx.x] = e_acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(energy, s[0]);
  }
}

// out_i = (fscale/Lu) [hpp_i - w_i (sum_m psi_m grad W_m(x_i) + sum_m phi_m (grad grad W_m(x_i)) v_i)]
// in caller order: the PM part of the Hessian-vector product plus the PP part.
template <int ORDER>
__global__ void __launch_bounds__(kThreads) k_gather_hvp(
    int64_t n, const PPRec<double>* __restrict__ pp, const MeshRec<double>* __restrict__ mesh,
    const double* __restrict__ hpp, const double* __restrict__ v, const uint32_t* __restrict__ perm,
    Geo geo, const Place* __restrict__ pl, const double* __restrict__ phi,
    const double* __restrict__ psi, double* __restrict__ out) {
  const int64_t j = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (j >= n) return;
  const MeshRec<double> m = mesh[j];
  const double q = pp[j].w;
  Stencil<double, ORDER> S(m.fx, m.fy, m.fz);
  double d2[3][S.N];
  for (int d = 0; d < 3; ++d)
    for (int a = 0; a < S.N; ++a) d2[d][a] = ORDER == 1 ? 0.0 : (a == 1 ? -2.0 : 1.0);
  const int nx = geo.grid[0];
  const long long nxy = (long long)nx * geo.grid[1];
  double gpsi[3] = {0, 0, 0};
  double hess[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int c = 0; c < S.N; ++c)
    for (int b = 0; b < S.N; ++b)
      for (int a = 0; a < S.N; ++a) {
        const long long node = m.base + c * nxy + (long long)b * nx + a;
        const double ps = psi[node], ph = phi[node];
        const double W[3] = {S.w[0][a], S.w[1][b], S.w[2][c]};
        const double D[3] = {S.dw[0][a], S.dw[1][b], S.dw[2][c]};
        const double E[3] = {d2[0][a], d2[1][b], d2[2][c]};
        gpsi[0] += ps * D[0] * W[1] * W[2];
        gpsi[1] += ps * W[0] * D[1] * W[2];
        gpsi[2] += ps * W[0] * W[1] * D[2];
        for (int p = 0; p < 3; ++p)
          for (int r = 0; r < 3; ++r) {
            double prod = 1.0;
            for (int e = 0; e < 3; ++e) {
              if (p == r && e == p) prod *= E[e];
              else if (e == p || e == r) prod *= D[e];
              else prod *= W[e];
            }
            hess[p][r] += ph * prod;
          }
      }
  const double vj[3] = {v[3 * j], v[3 * j + 1], v[3 * j + 2]};
  const double scale = pl->fscale * pl->inv_lu;
  const uint32_t i = perm[j];
  for (int p = 0; p < 3; ++p) {
    double acc = gpsi[p] / geo.hu[p];
    for (int r = 0; r < 3; ++r) acc += hess[p][r] * vj[r] / (geo.hu[p] * geo.hu[r]);
    out[3 * i + p] = scale * (hpp[3 * j + p] - q * acc);
  }
}

template <typename R>
__global__ void k_mesh_export(long long count, const R* __restrict__ src, const Place* __restrict__ pl,
                              int scale_phi, double* __restrict__ out) {
  long long k = blockIdx.x * (long long)kThreads + threadIdx.x;
  if (k >= count) return;
  double v = (double)src[k];
  out[k] = scale_phi ? v * pl->phiscale : v;
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

template <typename R, typename M>
void launch_deposit(int64_t n, const PPPos<R>* pp, const MeshRec<R>* mesh, const Geo& geo, M* Q,
                    hipStream_t st) {
  launch_fill(Q, (size_t)geo.grid[0] * geo.grid[1] * geo.grid[2] * sizeof(M), st);
  const unsigned blocks = (unsigned)((n + kDepChunk - 1) / kDepChunk);
  if (blocks == 0) return;
  if (geo.order == 1)
    k_deposit<R, M, 1, false><<<blocks, kDepThreads, 0, st>>>(n, pp, mesh, geo, nullptr, Q);
  else
    k_deposit<R, M, 2, false><<<blocks, kDepThreads, 0, st>>>(n, pp, mesh, geo, nullptr, Q);
}

int gather_blocks(int64_t n) { return (int)blocks_for(n); }

template <typename R, typename M>
void launch_gather(int64_t n, const PPPos<R>* pp, const MeshRec<R>* mesh, const PPRec<R>* fpp,
                   const uint32_t* perm, const Geo& geo, const Place* pl, const M* phi,
                   GatherOut out, double* energy, hipStream_t st) {
#define P3M_GATHER(O, G) \
  k_gather<R, M, O, G><<<blocks_for(n), kThreads, 0, st>>>(n, pp, mesh, fpp, perm, geo, pl, phi, out, energy)
  if (geo.gather == 0 && geo.mdiff && !energy) {
    if (geo.order == 1) P3M_GATHER(1, 2);
    else P3M_GATHER(2, 2);
  } else if (geo.gather == 0) {
    if (geo.order == 1) P3M_GATHER(1, 0);
    else P3M_GATHER(2, 0);
  } else {
    if (geo.order == 1) P3M_GATHER(1, 1);
    else P3M_GATHER(2, 1);
  }
#undef P3M_GATHER
}

void launch_deposit_grad(int64_t n, const PPRec<double>* pp, const MeshRec<double>* mesh,
                         const double* v_sorted, const Geo& geo, double* Rm, hipStream_t st) {
  // the tiled, fixed-point deposit with the gradient's node values (Rm is
  // cleared by the caller)
  const unsigned blocks = (unsigned)((n + kDepChunk - 1) / kDepChunk);
  if (blocks == 0) return;
  if (geo.order == 1)
    k_deposit<double, double, 1, true><<<blocks, kDepThreads, 0, st>>>(n, pp, mesh, geo, v_sorted, Rm);
  else
    k_deposit<double, double, 2, true><<<blocks, kDepThreads, 0, st>>>(n, pp, mesh, geo, v_sorted, Rm);
}

void launch_gather_hvp(int64_t n, const PPRec<double>* pp, const MeshRec<double>* mesh,
                       const double* hpp_sorted, const double* v_sorted, const uint32_t* perm,
                       const Geo& geo, const Place* pl, const double* phi, const double* psi,
                       double* out, hipStream_t st) {
  if (geo.order == 1)
    k_gather_hvp<1><<<blocks_for(n), kThreads, 0, st>>>(n, pp, mesh, hpp_sorted, v_sorted, perm, geo, pl,
                                                        phi, psi, out);
  else
    k_gather_hvp<2><<<blocks_for(n), kThreads, 0, st>>>(n, pp, mesh, hpp_sorted, v_sorted, perm, geo, pl,
                                                        phi, psi, out);
}

template <typename R>
void launch_mesh_export(const Geo& geo, const R* src, const Place* pl, int scale_phi, double* out,
                        hipStream_t st) {
  long long count = (long long)geo.grid[0] * geo.grid[1] * geo.grid[2];
  k_mesh_export<R><<<blocks_for(count), kThreads, 0, st>>>(count, src, pl, scale_phi, out);
}

#define P3M_MESH_INST(R, M)                                                                        \
  template void launch_deposit<R, M>(int64_t, const PPPos<R>*, const MeshRec<R>*, const Geo&, M*,        \
                                     hipStream_t);                                                        \
  template void launch_gather<R, M>(int64_t, const PPPos<R>*, const MeshRec<R>*, const PPRec<R>*,          \
                                    const uint32_t*, const Geo&, const Place*, const M*, GatherOut,       \
                                    double*, hipStream_t);
P3M_MESH_INST(float, float)
P3M_MESH_INST(float, double)
P3M_MESH_INST(double, double)
#undef P3M_MESH_INST
template void launch_mesh_export<float>(const Geo&, const float*, const Place*, int, double*, hipStream_t);
template void launch_mesh_export<double>(const Geo&, const double*, const Place*, int, double*, hipStream_t);

}  // namespace p3m
