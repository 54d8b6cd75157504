// Float64 reductions for the observables of a bunch (momentum, kinetic
// energy, centroid, rms sizes, normalised rms emittances), and a plain fill
// kernel used instead of memset so every clear is an ordinary kernel.
//
// acc layout (doubles):
//   mode 0: [0..2] sum p_d, [3] sum |p|^2, [4..6] sum x_d, [7] sum w
//   mode 1 (about the means n^-1 acc[0..2], n^-1 acc[4..6]):
//           [16..18] sum dx_d^2, [19..21] sum dp_d^2, [22..24] sum dx_d dp_d
#include "launch.h"

namespace p3m {

namespace {

constexpr int kQ = 9;

__global__ void __launch_bounds__(kThreads) k_moments(int64_t n, const double* __restrict__ x,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ qw,
                                                      double* __restrict__ acc, int mode) {
  double v[kQ];
  for (int k = 0; k < kQ; ++k) v[k] = 0.0;
  double mx[3], mp[3];
  if (mode == 1) {
    const double inv = n > 0 ? 1.0 / (double)n : 0.0;
    for (int d = 0; d < 3; ++d) { mp[d] = acc[d] * inv; mx[d] = acc[4 + d] * inv; }
  }
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    if (mode == 0) {
      for (int d = 0; d < 3; ++d) {
        const double pd = p[3 * i + d];
        v[d] += pd;
        v[3] += pd * pd;
        v[4 + d] += x[3 * i + d];
      }
      v[7] += qw ? qw[i] : 1.0;
    } else {
      for (int d = 0; d < 3; ++d) {
        const double dx = x[3 * i + d] - mx[d], dp = p[3 * i + d] - mp[d];
        v[d] += dx * dx;
        v[3 + d] += dp * dp;
        v[6 + d] += dx * dp;
      }
    }
  }
  __shared__ double s[kQ][kThreads];
  for (int k = 0; k < kQ; ++k) s[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < kQ; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
  if ((int)threadIdx.x < kQ) {
    const int dst = mode == 0 ? (int)threadIdx.x : 16 + (int)threadIdx.x;
    if (mode == 0 && threadIdx.x == 8) return;
    atomicAdd(acc + dst, s[threadIdx.x][0]);
  }
}

// Zero `words` 32-bit words: 16-byte stores over the 16-byte-aligned body,
// the few words before and after it one at a time.
__global__ void k_fill(uint32_t* __restrict__ p, long long words, long long head, long long quads) {
  const long long k0 = blockIdx.x * (long long)kThreads + threadIdx.x;
  const long long tail = words - head - 4 * quads;
  if (k0 < head) p[k0] = 0u;
  if (k0 < tail) p[head + 4 * quads + k0] = 0u;
  uint4* q = reinterpret_cast<uint4*>(p + head);
  for (long long k = k0; k < quads; k += (long long)gridDim.x * kThreads) q[k] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

void launch_moments(int64_t n, const double* x, const double* p, const double* qw, double* acc,
                    int mode, hipStream_t st) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  k_moments<<<(unsigned)b, kThreads, 0, st>>>(n, x, p, qw, acc, mode);
}

void launch_fill(void* ptr, size_t bytes, hipStream_t st) {
  const long long words = (long long)(bytes / 4);
  if (words == 0) return;
  long long head = (long long)(((16 - ((uintptr_t)ptr & 15)) & 15) / 4);
  if (head > words) head = words;
  const long long quads = (words - head) / 4;
  long long b = (quads + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  k_fill<<<(unsigned)b, kThreads, 0, st>>>((uint32_t*)ptr, words, head, quads);
}

}  // namespace p3m
