// Linked cells on the device: PP-cell key per particle, a stable LSD radix
// sort of (key, index) with digits of up to 11 bits, the start of every cell in the
// sorted order, and the reorder of the particles into sorted records.
//
// The paper sums the short-range force over particles "close to" each
// particle (Sec. 1, eq. summation_short) inside the cutoff; cells of edge
// >= r_c make the 27 neighbouring cells a superset of that neighbourhood.
// The cell edge is c_d = (N_d - 1) h_d / n_d with n_d = floor((N_d-1) h_d / r_c),
// so the cell grid covers exactly the mesh span and zoom leaves n_d unchanged.
#include "launch.h"

namespace p3m {

namespace {

constexpr int kItems = 8;                  // keys per thread in a radix tile
constexpr int kTile = kThreads * kItems;   // 2048 keys per block
constexpr int kWaves = kThreads / 64;

__global__ void __launch_bounds__(kThreads) k_keys(int64_t n, const double* __restrict__ x,
                                                   const Place* __restrict__ pl, Geo geo,
                                                   uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals,
                                                   int* __restrict__ ghist, int nhist,
                                                   int* __restrict__ counter, int* __restrict__ counts,
                                                   int64_t ncounts) {
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < nhist; k += kThreads) ghist[k] = 0;
    if (threadIdx.x < 2) counter[threadIdx.x] = 0;
  }
  int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  // the per-block digit counts of every pass start at zero (the count
  // kernels write only the digits present in their tile)
  for (int64_t e = i; e < ncounts; e += (int64_t)gridDim.x * kThreads) counts[e] = 0;
  if (i >= n) return;
  const Place P = *pl;
  int c[3];
  for (int d = 0; d < 3; ++d)
    c[d] = floor_clamp((x[3 * i + d] - P.x0[d]) * P.inv_cell[d], 0, geo.ncell[d] - 1);
  keys[i] = (uint32_t)(((long long)c[2] * geo.ncell[1] + c[1]) * geo.ncell[0] + c[0]);
  vals[i] = (uint32_t)i;
}

// Digits of db <= 11 bits (nbins = 2^db <= kMaxBins): keys of at most 22
// bits, the usual case, take two passes.
constexpr int kMaxBins = 2048;

__global__ void __launch_bounds__(kThreads) k_radix_count(int64_t n, const uint32_t* __restrict__ keys,
                                                          int shift, int nbins, int* __restrict__ counts,
                                                          int* __restrict__ ghist, int nb) {
  __shared__ int h[kMaxBins];
  for (int d = threadIdx.x; d < nbins; d += kThreads) h[d] = 0;
  __syncthreads();
  const uint32_t mask = (uint32_t)nbins - 1u;
  const int lane = threadIdx.x & 63;
  int64_t base = (int64_t)blockIdx.x * kTile;
  // Keys stepped in cell order arrive in runs of equal digits: the first lane
  // of each run within the wave adds the run's length (valid lanes form a
  // prefix of the wave; equal digits in separate runs simply add separately).
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + k * kThreads + threadIdx.x;
    const bool valid = i < n;
    const int d = valid ? (int)((keys[i] >> shift) & mask) : -1;
    const int prev = __shfl_up(d, 1);
    const bool head = valid && (lane == 0 || prev != d);
    const unsigned long long heads = __ballot(head);
    const int nvalid = __popcll(__ballot(valid));
    if (head) {
      const unsigned long long after = lane == 63 ? 0ull : heads & (~0ull << (lane + 1));
      const int next = after ? (int)__builtin_ctzll(after) : nvalid;
      atomicAdd(&h[d], next - lane);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < nbins; d += kThreads) {
    const int c = h[d];
    if (c) {
      counts[(int64_t)d * nb + blockIdx.x] = c;
      atomicAdd(&ghist[d], c);
    }
  }
}

// Exclusive scan of 256 values held one per thread; returns the thread's
// exclusive prefix and writes the block total to *total.
__device__ inline int block_exclusive_scan(int v, int* total) {
  __shared__ int s[kThreads];
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    int add = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  int incl = s[t];
  *total = s[kThreads - 1];
  __syncthreads();
  return incl - v;
}

// One block per digit: offsets[d][b] = (keys with a smaller digit) + (keys of
// digit d in blocks before b). counts is overwritten with the offsets. The
// first term is the sum of the digit histogram below d, formed by each block.
__global__ void __launch_bounds__(kThreads) k_radix_scan(int* __restrict__ counts,
                                                         const int* __restrict__ ghist, int nb) {
  const int d = blockIdx.x, t = threadIdx.x;
  if (ghist[d] == 0) return;   // no key has this digit: its offsets are never read
  int below = 0;
  for (int q = t; q < d; q += kThreads) below += ghist[q];
  int total;
  (void)block_exclusive_scan(below, &total);
  int carry = total;
  int* row = counts + (int64_t)d * nb;
  for (int b0 = 0; b0 < nb; b0 += kThreads) {
    int v = (b0 + t < nb) ? row[b0 + t] : 0;
    int ex = block_exclusive_scan(v, &total);
    if (b0 + t < nb) row[b0 + t] = carry + ex;
    carry += total;
  }
}

// Stable scatter of one tile: keys keep their order within a digit. Per
// round of 256 keys, each wave ranks its lanes by matching the digit bit by
// bit (ballots); the first lane of each digit run in a wave records the
// run's length for the waves after it, adds it to the digit's running count
// and clears its entry, so the per-wave counts never need a full clear.
__global__ void __launch_bounds__(kThreads) k_radix_scatter(
    int64_t n, const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, int shift, int db,
    const int* __restrict__ offsets, int nb) {
  __shared__ int run[kMaxBins];
  __shared__ int base[kMaxBins];
  __shared__ int wcnt[kWaves][kMaxBins];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nbins = 1 << db;
  // a digit's offset is fetched when the digit first occurs in the tile (a
  // tile of sorted keys holds few digits; two waves may fetch the same one)
  for (int d = t; d < nbins; d += kThreads) {
    run[d] = 0;
    base[d] = -1;
    for (int q = 0; q < kWaves; ++q) wcnt[q][d] = 0;
  }
  __syncthreads();
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t mask = (uint32_t)nbins - 1u;
  int64_t tile = (int64_t)blockIdx.x * kTile;
  for (int k = 0; k < kItems; ++k) {
    int64_t i = tile + k * kThreads + t;
    const bool valid = i < n;
    uint32_t key = valid ? kin[i] : 0u;
    uint32_t val = valid ? vin[i] : 0u;
    const int d = (int)((key >> shift) & mask);
    unsigned long long peers = __ballot(valid);
    for (int bit = 0; bit < db; ++bit) {
      const bool b = (d >> bit) & 1;
      unsigned long long m = __ballot(b);
      peers &= b ? m : ~m;
    }
    const int rank = __popcll(peers & lt);
    const int cnt = __popcll(peers);
    if (valid && rank == 0) {
      wcnt[w][d] = cnt;
      if (base[d] < 0) base[d] = offsets[(int64_t)d * nb + blockIdx.x];
    }
    __syncthreads();
    if (valid) {
      int pos = base[d] + run[d] + rank;
      for (int q = 0; q < w; ++q) pos += wcnt[q][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    if (valid && rank == 0) {
      atomicAdd(&run[d], cnt);
      wcnt[w][d] = 0;
    }
    __syncthreads();
  }
}

// cell_start[c] = first sorted index with key >= c, for c in [0, ncells]:
// one thread per cell, binary search in the sorted keys.
__global__ void k_cell_start(int64_t n, const uint32_t* __restrict__ keys, int* __restrict__ cs,
                             long long ncells) {
  const long long c = blockIdx.x * (long long)kThreads + threadIdx.x;
  if (c > ncells) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((long long)keys[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  cs[c] = (int)lo;
}

template <typename R>
__device__ __forceinline__ PPPos<R> make_pos(const double* loc, const double* cu, double w, bool packed);
template <>
__device__ __forceinline__ PPPos<double> make_pos<double>(const double* loc, const double*, double w, bool) {
  return PPPos<double>{loc[0], loc[1], loc[2], w};
}
// Nearest fixed-point value. Inside the mesh a particle lies in [0, 1] cell
// edges of its cell's corner; one outside it (reported as a domain error)
// is clamped to [-1/2, 3/2) edges, which keeps every PP separation, cell
// offsets included, below 2^31 units (an edge is at most 2^29 units).
// packed (every weight 1): the weight slot holds the residuals u - rint(u),
// rounded to 2^-kResBits units, as three 10-bit fields (x lowest).
template <>
__device__ __forceinline__ PPPos<float> make_pos<float>(const double* loc, const double* cu, double w,
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
    carry.id_out[j] = carry.id_in ? carry.id_in[i] : i;
    if (qw) carry.qw_out[j] = w;
  }
  // PP record: offset from the own cell corner, formed in float64 before
  // rounding (units of Lu, or fixed point of the cell edge).
  double loc[3];
  for (int d = 0; d < 3; ++d) loc[d] = (xi[d] - P.x0[d]) * P.inv_lu - c[d] * geo.cu[d];
  pp[j] = make_pos<R>(loc, geo.cu, w, geo.wpacked != 0);
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

static int key_bits(long long ncells) {
  int bits = 1;
  while ((1ll << bits) < ncells) ++bits;
  return bits;
}

int sort_passes(long long ncells) { return (key_bits(ncells) + 10) / 11; }

static int digit_bits(long long ncells) {
  const int bits = key_bits(ncells), passes = sort_passes(ncells);
  return (bits + passes - 1) / passes;
}

int sort_blocks(int64_t n) { return (int)((n + kTile - 1) / kTile); }

void launch_cell_sort(int64_t n, const double* x, const Place* pl, const Geo& geo, SortBufs& b,
                      uint32_t** keys, uint32_t** perm, hipStream_t st) {
  const int passes = sort_passes(geo.ncells);
  const int db = digit_bits(geo.ncells), nbins = 1 << db;
  const int nb = sort_blocks(n);
  const int64_t per_pass = (int64_t)nbins * nb;
  k_keys<<<blocks_for(n), kThreads, 0, st>>>(n, x, pl, geo, b.keys_a, b.vals_a, b.ghist, passes * nbins,
                                             b.counter, b.counts, passes * per_pass);
  uint32_t *ka = b.keys_a, *va = b.vals_a, *kb = b.keys_b, *vb = b.vals_b;
  for (int p = 0; p < passes; ++p) {
    int* gh = b.ghist + p * nbins;
    int* cnt = b.counts + p * per_pass;
    k_radix_count<<<nb, kThreads, 0, st>>>(n, ka, db * p, nbins, cnt, gh, nb);
    k_radix_scan<<<nbins, kThreads, 0, st>>>(cnt, gh, nb);
    k_radix_scatter<<<nb, kThreads, 0, st>>>(n, ka, va, kb, vb, db * p, db, cnt, nb);
    uint32_t* tk = ka; ka = kb; kb = tk;
    uint32_t* tv = va; va = vb; vb = tv;
  }
  k_cell_start<<<blocks_for(geo.ncells + 1), kThreads, 0, st>>>(n, ka, b.cell_start, geo.ncells);
  *keys = ka;
  *perm = va;
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
