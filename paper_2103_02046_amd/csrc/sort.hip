// Linked cells on the device: PP-cell key per particle, a counting sort by
// cell (per-cell counts, their prefix sum as the cell starts, and a scatter),
// the PP work groups, and the reorder of the particles into sorted records.
//
// The paper sums the short-range force over particles "close to" each
// particle (Sec. 1, eq. summation_short) inside the cutoff; cells of edge
// >= r_c make the 27 neighbouring cells a superset of that neighbourhood.
// The cell edge is c_d = (N_d - 1) h_d / n_d with n_d = floor((N_d-1) h_d / r_c),
// so the cell grid covers exactly the mesh span and zoom leaves n_d unchanged.
#include <type_traits>

#include "launch.h"

namespace p3m {

namespace {

constexpr int kWaves = kThreads / 64;

// Exclusive scans of C values per thread over the block's 256 threads: a
// shuffle scan inside each wave, then the wave totals through LDS (two
// barriers for all C). excl[c] is the thread's exclusive prefix, total[c]
// the block total.
template <int C>
__device__ inline void block_exclusive_scan(const int (&v)[C], int (&excl)[C], int (&total)[C]) {
  __shared__ int wsum[C][kWaves];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int incl[C];
#pragma unroll
  for (int c = 0; c < C; ++c) incl[c] = v[c];
#pragma unroll
  for (int off = 1; off < 64; off <<= 1)
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int u = __shfl_up(incl[c], off);
      if (lane >= off) incl[c] += u;
    }
  if (lane == 63)
#pragma unroll
    for (int c = 0; c < C; ++c) wsum[c][w] = incl[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < C; ++c) {
    int before = 0, all = 0;
    for (int k = 0; k < kWaves; ++k) {
      const int x = wsum[c][k];
      before += k < w ? x : 0;
      all += x;
    }
    excl[c] = before + incl[c] - v[c];
    total[c] = all;
  }
  __syncthreads();   // wsum is free for the next call
}

// ---- counting sort by cell ------------------------------------------------
// Keys stepped in cell order arrive in runs of equal cells. Within a wave
// (valid lanes form a prefix) the first lane of each run of equal
// consecutive keys is its head: *head_lane is the head of this lane's run,
// *len the run's length (meaningful at heads).
__device__ __forceinline__ void wave_runs(bool valid, uint32_t key, int lane, int* head_lane, int* len) {
  const uint32_t prev = __shfl_up(key, 1);
  const bool head = valid && (lane == 0 || prev != key);
  const unsigned long long heads = __ballot(head);
  const int nvalid = __popcll(__ballot(valid));
  const unsigned long long upto = heads & ((2ull << lane) - 1ull);   // heads at or below this lane
  *head_lane = upto ? 63 - (int)__builtin_clzll(upto) : 0;
  const unsigned long long after = lane == 63 ? 0ull : heads & (~0ull << (lane + 1));
  *len = (after ? (int)__builtin_ctzll(after) : nvalid) - lane;
}

// Cell key of every particle, in the input order, and the number of
// particles per cell (ccount starts at zero; the start kernel re-zeroes it).
// Block 0 also clears the super-block totals of the start prefix.
__global__ void __launch_bounds__(kThreads) k_cell_keys(int64_t n, const double* __restrict__ x,
                                                        const Place* __restrict__ pl, Geo geo,
                                                        uint32_t* __restrict__ keys, int* __restrict__ ccount,
                                                        int* __restrict__ stot, int nstot) {
  if (blockIdx.x == 0)
    for (int e = threadIdx.x; e < nstot; e += kThreads) stot[e] = 0;
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = i < n;
  uint32_t key = 0;
  if (valid) {
    const Place P = *pl;
    int c[3];
    for (int d = 0; d < 3; ++d)
      c[d] = floor_clamp((x[3 * i + d] - P.x0[d]) * P.inv_cell[d], 0, geo.ncell[d] - 1);
    key = (uint32_t)(((long long)c[2] * geo.ncell[1] + c[1]) * geo.ncell[0] + c[0]);
    keys[i] = key;
  }
  int hl, len;
  wave_runs(valid, key, lane, &hl, &len);
  if (valid && hl == lane) atomicAdd(&ccount[key], len);
}

constexpr int kCellItems = 2;                        // cells per thread in the start scan
constexpr int kCellTile = kThreads * kCellItems;     // 512 cells per block
constexpr int kSuper = 64;                           // blocks per super-block of the start prefix
constexpr int kDirectPrefix = 2048;                  // above this many blocks, super-block totals

// Particles, dense-cell groups and other groups (runs of <= 16 of one
// cell) per block of cells, and on large grids their sums per super-block of
// kSuper blocks (stot, cleared by the key kernel); kTotals values each.
constexpr int kTotals = kCellTotals;

__device__ __forceinline__ void cell_groups(int v, int& dense, int& sparse) {
  const int g = (v + kGroupRun - 1) / kGroupRun;
  if (v >= kDenseCell) dense += g;
  else sparse += g;
}

__global__ void __launch_bounds__(kThreads) k_cell_totals(const int* __restrict__ ccount, long long ncells,
                                                          int* __restrict__ btot, int* __restrict__ stot,
                                                          bool super_prefix) {
  const long long c0 = blockIdx.x * (long long)kCellTile + (long long)threadIdx.x * kCellItems;
  int s = 0, gd = 0, gsp = 0;
#pragma unroll
  for (int k = 0; k < kCellItems; ++k) {
    if (c0 + k < ncells) {
      const int v = ccount[c0 + k];
      s += v;
      cell_groups(v, gd, gsp);
    }
  }
  const int val[kTotals] = {s, gd, gsp};
  int excl[kTotals], tot[kTotals];
  block_exclusive_scan<kTotals>(val, excl, tot);
  if (threadIdx.x == 0) {
    for (int c = 0; c < kTotals; ++c) {
      btot[kTotals * blockIdx.x + c] = tot[c];
      if (super_prefix) atomicAdd(&stot[kTotals * (blockIdx.x / kSuper) + c], tot[c]);
    }
  }
}

// Cell starts (exclusive prefix of the counts), the scatter's fill pointers,
// and the PP work groups: dense-cell groups in cell order from the front of
// desc, the others in cell order from its back (desc[cap - 1 - i]). A
// block's offsets are the sums of the block totals before it. Up to
// kDirectPrefix blocks each block adds them all; above, it adds the
// super-block totals before its super-block and the block totals before it
// inside its super-block (at most kSuper - 1), so the work stays linear in
// the number of blocks. ccount is cleared for the next sort; the last block
// stores cell_start[ncells] and the numbers of dense and other groups
// (counter[0], counter[1]).
__global__ void __launch_bounds__(kThreads) k_cell_starts(int* __restrict__ ccount, long long ncells,
                                                          const int* __restrict__ btot,
                                                          const int* __restrict__ stot, bool super_prefix,
                                                          int* __restrict__ cell_start, int* __restrict__ cfill,
                                                          int2* __restrict__ desc, int cap,
                                                          int* __restrict__ counter) {
  __shared__ int red[kTotals][kWaves];
  const int t = threadIdx.x;
  const int sb = super_prefix ? (int)blockIdx.x / kSuper : 0, first = sb * kSuper;
  int pre[kTotals] = {0, 0, 0};
  for (int q = t; q < sb; q += kThreads)
    for (int c = 0; c < kTotals; ++c) pre[c] += stot[kTotals * q + c];
  for (int q = first + t; q < (int)blockIdx.x; q += kThreads)
    for (int c = 0; c < kTotals; ++c) pre[c] += btot[kTotals * q + c];
  for (int c = 0; c < kTotals; ++c) {
    for (int off = 32; off > 0; off >>= 1) pre[c] += __shfl_xor(pre[c], off);
    if ((t & 63) == 0) red[c][t >> 6] = pre[c];
  }
  __syncthreads();
  int P = 0, GD = 0, GS = 0;
  for (int w = 0; w < kWaves; ++w) {
    P += red[0][w];
    GD += red[1][w];
    GS += red[2][w];
  }
  const long long c0 = blockIdx.x * (long long)kCellTile + (long long)t * kCellItems;
  int v[kCellItems];
  int s = 0, gd = 0, gsp = 0;
#pragma unroll
  for (int k = 0; k < kCellItems; ++k) {
    v[k] = c0 + k < ncells ? ccount[c0 + k] : 0;
    s += v[k];
    cell_groups(v[k], gd, gsp);
  }
  const int val[kTotals] = {s, gd, gsp};
  int excl[kTotals], tot[kTotals];
  block_exclusive_scan<kTotals>(val, excl, tot);
  int start = P + excl[0];
  int g = GD + excl[1];
  int h = GS + excl[2];
#pragma unroll
  for (int k = 0; k < kCellItems; ++k) {
    if (c0 + k < ncells) {
      cell_start[c0 + k] = start;
      cfill[c0 + k] = start;
      ccount[c0 + k] = 0;
      const bool dense = v[k] >= kDenseCell;
      for (int j = 0; j < v[k]; j += kGroupRun)
        desc[dense ? g++ : cap - 1 - h++] = make_int2(start + j, min(kGroupRun, v[k] - j));
      start += v[k];
    }
  }
  if (blockIdx.x == gridDim.x - 1 && t == kThreads - 1) {
    cell_start[ncells] = start;
    counter[0] = g;
    counter[1] = h;
  }
}

// Sorted position of every particle: one atomic per run of equal keys on
// the cell's fill pointer, the run's lanes in input order after it. Runs of
// one cell land in the order their atomics arrive, so the order inside a
// cell may differ between runs of the program (the sums over a cell are
// then added in another order, a difference at rounding level).
__global__ void __launch_bounds__(kThreads) k_cell_scatter(int64_t n, const uint32_t* __restrict__ keys_in,
                                                           int* __restrict__ cfill, uint32_t* __restrict__ keys_out,
                                                           uint32_t* __restrict__ perm) {
  const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = i < n;
  const uint32_t key = valid ? keys_in[i] : 0u;
  int hl, len;
  wave_runs(valid, key, lane, &hl, &len);
  int base = 0;
  if (valid && hl == lane) base = atomicAdd(&cfill[key], len);
  base = __shfl(base, hl);
  if (valid) {
    const int dst = base + (lane - hl);
    keys_out[dst] = key;
    perm[dst] = (uint32_t)i;
  }
}

template <typename R>
__device__ __forceinline__ PPPos<R> make_pos(const double* loc, const double* cu, int cx, double w, bool packed);
template <>
__device__ __forceinline__ PPPos<double> make_pos<double>(const double* loc, const double*, int, double w, bool) {
  return PPPos<double>{loc[0], loc[1], loc[2], w};
}
// Nearest fixed-point value. Inside the mesh a particle lies in [0, 1] cell
// edges of its cell's corner; one outside it (reported as a domain error)
// is clamped to [-1/2, 3/2) edges. An edge is at most 2^kFixBits = 2^28
// units, so the position plus the bias 2^27 lies in [0, 2^29) and the x
// slot holds (v + kFixBias) | (cx mod 8) << kXCodeShift; every PP
// separation, cell offsets of up to two edges included, stays below 2^31.
// packed (every weight 1): the weight slot holds the residuals u - rint(u),
// rounded to 2^-kResBits units, as three 10-bit fields (x lowest).
template <>
__device__ __forceinline__ PPPos<float> make_pos<float>(const double* loc, const double* cu, int cx, double w,
                                                        bool packed) {
  const double unit = fix_unit(cu);
  int v[3];
  unsigned res = 0;
  for (int d = 0; d < 3; ++d) {
    const double e = (double)fix_edge(cu, d);
    double u = loc[d] / unit;
    u = fmin(fmax(u, -0.5 * e), 1.4999999 * e);
    v[d] = (int)rint(u);
    const int r = min(max((int)rint((u - v[d]) * (1 << kResBits)), -511), 511);
    res |= ((unsigned)r & 1023u) << (10 * d);
  }
  v[0] = (int)(((unsigned)(v[0] + kFixBias) & (unsigned)kFixMask) | (((unsigned)cx & 7u) << kXCodeShift));
  return PPFix{v[0], v[1], v[2], packed ? __uint_as_float(res) : (float)w};
}

template <typename R>
__global__ void __launch_bounds__(kThreads) k_reorder(
    int64_t n, const double* __restrict__ x, const double* __restrict__ qw,
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ keys,
    const Place* __restrict__ pl, Geo geo, PPPos<R>* __restrict__ pp, MeshRec<R>* __restrict__ mesh,
    int* __restrict__ status, Carry carry) {
  int64_t j = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (j >= n) return;
  const Place P = *pl;
  const uint32_t i = perm[j];
  const uint32_t key = keys[j];
  const int c[3] = {(int)(key % (uint32_t)geo.ncell[0]),
                    (int)((key / (uint32_t)geo.ncell[0]) % (uint32_t)geo.ncell[1]),
                    (int)(key / ((uint32_t)geo.ncell[0] * (uint32_t)geo.ncell[1]))};
  double xi[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
  const double w = qw ? qw[i] : 1.0;
  if (carry.x_out) {
    for (int d = 0; d < 3; ++d) carry.x_out[3 * j + d] = xi[d];
    for (int d = 0; d < 3; ++d) carry.p_out[3 * j + d] = carry.p_in[3 * i + d];
  }
  if (carry.id_out) {
    carry.id_out[j] = carry.id_in ? carry.id_in[i] : i;
    if (qw) carry.qw_out[j] = w;
  }
  // PP record: offset from the own cell corner, formed in float64 before
  // rounding. double form: units of Lu from the corner c cu. float form:
  // from the corner at the whole number c fix_edge of fixed-point units (the
  // pair kernel adds cell offsets as such whole numbers), so that every
  // separation, across cells too, is the exact difference of the global
  // fixed-point positions.
  double loc[3];
  const double unit = fix_unit(geo.cu);
  for (int d = 0; d < 3; ++d) {
    const double corner = std::is_same<R, float>::value ? c[d] * (double)fix_edge(geo.cu, d) * unit
                                                        : c[d] * geo.cu[d];
    loc[d] = (xi[d] - P.x0[d]) * P.inv_lu - corner;
  }
  pp[j] = make_pos<R>(loc, geo.cu, c[0], w, geo.wpacked != 0);
  // Mesh record: stencil origin and fractional offset (Sec. 2.4.2 B-splines).
  // CIC: base floor(u), offset u - base in [0, 1).
  // TSC: centre floor(u + 1/2), offset u - centre in [-1/2, 1/2), base centre - 1.
  int b[3];
  double f[3];
  bool out = false;
  for (int d = 0; d < 3; ++d) {
    double u = (xi[d] - P.x0[d]) * P.inv_hp[d];
    const int mg = geo.gather ? 1 : 0;   // stencil kept off the outer node layer
    if (geo.order == 1) {
      double fl = floor(u);
      b[d] = floor_clamp(u, mg, geo.grid[d] - 2 - mg);
      out |= (double)b[d] != fl;
      f[d] = u - (double)b[d];
    } else {
      double fl = floor(u + 0.5);
      int cc = floor_clamp(u + 0.5, 1 + mg, geo.grid[d] - 2 - mg);
      out |= (double)cc != fl;
      f[d] = u - (double)cc;
      b[d] = cc - 1;
    }
  }
  if (out) atomicOr(status, kBitDomain);
  MeshRec<R> m;
  m.fx = (R)f[0];
  m.fy = (R)f[1];
  m.fz = (R)f[2];
  m.base = ((b[2] * geo.grid[1]) + b[1]) * geo.grid[0] + b[0];
  mesh[j] = m;
}

__global__ void __launch_bounds__(kThreads) k_unpermute(int64_t n, const double* __restrict__ xs,
                                                        const double* __restrict__ ps,
                                                        const double* __restrict__ fs,
                                                        const uint32_t* __restrict__ id, double* __restrict__ x,
                                                        double* __restrict__ p, double* __restrict__ f) {
  int64_t j = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (j >= n) return;
  const uint32_t i = id[j];
  for (int d = 0; d < 3; ++d) {
    x[3 * i + d] = xs[3 * j + d];
    p[3 * i + d] = ps[3 * j + d];
    f[3 * i + d] = fs[3 * j + d];
  }
}

template <typename R>
__global__ void k_sort_vector(int64_t n, const double* __restrict__ v, const uint32_t* __restrict__ perm,
                              R* __restrict__ out) {
  int64_t j = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (j >= n) return;
  uint32_t i = perm[j];
  out[3 * j] = (R)v[3 * i];
  out[3 * j + 1] = (R)v[3 * i + 1];
  out[3 * j + 2] = (R)v[3 * i + 2];
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

int cell_blocks(long long ncells) { return (int)((ncells + kCellTile - 1) / kCellTile); }

int cell_supers(long long ncells) { return (cell_blocks(ncells) + kSuper - 1) / kSuper; }

void launch_cell_sort(int64_t n, const double* x, const Place* pl, const Geo& geo, SortBufs& b, int2* desc,
                      uint32_t** keys, uint32_t** perm, hipStream_t st) {
  const int nbc = cell_blocks(geo.ncells);
  const bool sup = nbc > kDirectPrefix;
  k_cell_keys<<<blocks_for(n), kThreads, 0, st>>>(n, x, pl, geo, b.keys_in, b.ccount, b.stot,
                                                  sup ? kTotals * cell_supers(geo.ncells) : 0);
  k_cell_totals<<<nbc, kThreads, 0, st>>>(b.ccount, geo.ncells, b.btot, b.stot, sup);
  k_cell_starts<<<nbc, kThreads, 0, st>>>(b.ccount, geo.ncells, b.btot, b.stot, sup, b.cell_start, b.cfill,
                                          desc, pp_group_bound(n, geo), b.counter);
  k_cell_scatter<<<blocks_for(n), kThreads, 0, st>>>(n, b.keys_in, b.cfill, b.keys, b.perm);
  *keys = b.keys;
  *perm = b.perm;
}

template <typename R>
void launch_reorder(int64_t n, const double* x, const double* qw, const uint32_t* perm,
                    const uint32_t* keys, const Place* pl, const Geo& geo, PPPos<R>* pp,
                    MeshRec<R>* mesh, int* status, const Carry& carry, hipStream_t st) {
  k_reorder<R><<<blocks_for(n), kThreads, 0, st>>>(n, x, qw, perm, keys, pl, geo, pp, mesh, status, carry);
}

void launch_unpermute(int64_t n, const double* xs, const double* ps, const double* fs, const uint32_t* id,
                      double* x, double* p, double* f, hipStream_t st) {
  if (n > 0) k_unpermute<<<blocks_for(n), kThreads, 0, st>>>(n, xs, ps, fs, id, x, p, f);
}

template <typename R>
void launch_sort_vector(int64_t n, const double* v, const uint32_t* perm, R* out, hipStream_t st) {
  k_sort_vector<R><<<blocks_for(n), kThreads, 0, st>>>(n, v, perm, out);
}

template void launch_reorder<float>(int64_t, const double*, const double*, const uint32_t*,
                                    const uint32_t*, const Place*, const Geo&, PPPos<float>*,
                                    MeshRec<float>*, int*, const Carry&, hipStream_t);
template void launch_reorder<double>(int64_t, const double*, const double*, const uint32_t*,
                                     const uint32_t*, const Place*, const Geo&, PPPos<double>*,
                                     MeshRec<double>*, int*, const Carry&, hipStream_t);
template void launch_sort_vector<float>(int64_t, const double*, const uint32_t*, float*, hipStream_t);
template void launch_sort_vector<double>(int64_t, const double*, const uint32_t*, double*, hipStream_t);

}  // namespace p3m
