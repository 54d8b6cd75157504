// Open-boundary convolution phi = G (x) Q on the mesh by FFT on the doubled
// mesh (zero padding), and the Fourier table of G.
//
// The long-range potential is the finite convolution of the mesh charge with
// the long-range kernel (Sec. 3, eq. phi_L); with free-space boundaries
// (Sec. 2.1, eq. free_gf) and the Gaussian screening of Sec. 2.2 folded into
// the kernel, G(delta) = erf(kappa rho)/rho sampled at the node offsets,
// G(0) = 2 kappa / sqrt(pi). The charge occupies N nodes per axis, so every
// offset that matters lies in [-(N-1), N-1] and a cyclic convolution on 2N
// nodes per axis reproduces the aperiodic one exactly.
//
// Passes (L_d = 2 N_d; forward transforms e^{-2 pi i k n / L}):
//   x: real lines of N_x charges, two lines packed as one complex line,
//      zero-padded to L_x, split into two half spectra (k_x = 0..N_x);
//   y: for every (z < N_z, k_x): N_y inputs, L_y outputs;
//   z: for every (k_y, k_x): N_z inputs -> L_z -> times the real, even Ghat
//      -> inverse -> keep z < N_z  (the full spectrum never reaches memory);
//   y inverse: keep y < N_y;  x inverse: two half spectra -> two real lines.
// Each line is transformed in LDS by a Stockham radix-16 (then 8, 4 or 2) FFT;
// a block holds B lines side by side (point-major), so the strided y and z
// passes read and write rows of B consecutive k_x values. Spectrum rows are
// spec_stride(N_x) long (N_x + 1 padded to a multiple of 16), so those rows
// start on cache-line boundaries; the padding is never read.
// The inverse is conj(FFT(conj(.))); 1/(L_x L_y L_z) is folded into Ghat.
#include <cmath>
#include <type_traits>
#include <vector>

#include "launch.h"

namespace p3m {

namespace {

constexpr int kFftThreads = 256;
constexpr int kLdsBytes = 32768;

template <typename T, int L>
struct Cfg {
  static constexpr int raw = kLdsBytes / (L * (int)sizeof(C2<T>));
  static constexpr int B = raw < 1 ? 1 : raw;   // lines per block (power of two)
  // blocks of the strided y and z passes whose B-wide rows share one 128-byte line
  static constexpr int share = 128 / (int)sizeof(C2<T>) / B;
  static constexpr int G = share < 1 ? 1 : share;
};

// Block order of the strided y and z passes. Logical block l = row * nchp +
// chunk takes the B values k_x = chunk * B .. of one row of lines; nchp is
// the chunk count rounded up to a multiple of G, so the G chunks of one
// 128-byte line are G consecutive logical blocks. Work-groups are dealt to
// the XCDs round-robin, so those G blocks are placed kXcds slots apart in
// runs of G * kXcds: they run on one XCD at about the same time and its L2
// fetches each line once, not once per chunk (at 1024-point float lines
// B = 4 and G = 4). Returns false for the padding blocks.
template <int G>
__device__ __forceinline__ bool line_block(int nch, long long nrows, int& row, int& kx0, int B) {
  const long long hb = blockIdx.x;
  const int j = (int)(hb % (G * kXcds));
  const long long l = hb - j + (long long)(j % kXcds) * G + j / kXcds;
  const int nchp = (nch + G - 1) / G * G;
  const long long r = l / nchp;
  const int c = (int)(l - r * nchp);
  row = (int)r;
  kx0 = c * B;
  return r < nrows && c < nch;
}

template <typename T, int L>
unsigned line_grid(long long nrows, int K) {
  constexpr int B = Cfg<T, L>::B, G = Cfg<T, L>::G;
  const long long nchp = ((K + B - 1) / B + G - 1) / G * G;
  const long long run = (long long)G * kXcds;
  return (unsigned)((nrows * nchp + run - 1) / run * run);
}

template <typename T>
__device__ __forceinline__ void dft2(C2<T>* v) {
  C2<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T>
__device__ __forceinline__ void dft4(C2<T>* v) {
  C2<T> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  C2<T> a2 = cadd(v[1], v[3]), a3 = cmul_mi(csub(v[1], v[3]));
  v[0] = cadd(a0, a2);
  v[2] = csub(a0, a2);
  v[1] = cadd(a1, a3);
  v[3] = csub(a1, a3);
}

template <typename T>
__device__ __forceinline__ void dft8(C2<T>* v) {
  C2<T> e[4] = {v[0], v[2], v[4], v[6]};
  C2<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4(e);
  dft4(o);
  const T c = (T)0.70710678118654752440;
  // multiply o[k] by e^{-2 pi i k / 8}
  C2<T> o1 = {c * (o[1].x + o[1].y), c * (o[1].y - o[1].x)};
  C2<T> o2 = cmul_mi(o[2]);
  C2<T> o3 = {c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y)};
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

// 16 points as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2; DFTs over n1, twiddles
// w16^(n2 k1), DFTs over n2.
template <typename T>
__device__ __forceinline__ void dft16(C2<T>* v) {
  C2<T> y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    C2<T> a[4] = {v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]};
    dft4(a);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = a[k1];
  }
  const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;
  const T h = (T)0.70710678118654752440;
  // w16^j = (cos(2 pi j / 16), -sin(2 pi j / 16)) for j = n2 k1
  y[1][1] = cmul(y[1][1], C2<T>{c1, -s1});
  y[1][2] = cmul(y[1][2], C2<T>{h, -h});
  y[1][3] = cmul(y[1][3], C2<T>{s1, -c1});
  y[2][1] = cmul(y[2][1], C2<T>{h, -h});
  y[2][2] = cmul_mi(y[2][2]);
  y[2][3] = cmul(y[2][3], C2<T>{-h, -h});
  y[3][1] = cmul(y[3][1], C2<T>{s1, -c1});
  y[3][2] = cmul(y[3][2], C2<T>{-h, -h});
  y[3][3] = cmul(y[3][3], C2<T>{-c1, s1});
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    C2<T> b[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
    dft4(b);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
  }
}

template <typename T, int R>
__device__ __forceinline__ void dftR(C2<T>* v) {
  if constexpr (R == 16) dft16(v);
  else if constexpr (R == 8) dft8(v);
  else if constexpr (R == 4) dft4(v);
  else if constexpr (R == 2) dft2(v);
}

// One Stockham stage: radix R, Ns = product of the radices already applied.
// Element j + r L/R of every line is read, twiddled by w_{Ns R}^{r (j mod Ns)},
// transformed, and written to (j / Ns) Ns R + (j mod Ns) + r Ns.
template <typename T, int L, int B, int Ns, int R>
__device__ __forceinline__ void fft_stage(C2<T>* s, const C2<T>* __restrict__ tw) {
  constexpr int NBF = B * (L / R);
  constexpr int PER = (NBF + kFftThreads - 1) / kFftThreads;
  C2<T> v[PER][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int it = 0; it < PER; ++it) {
    const int t = tid + it * kFftThreads;
    if (NBF % kFftThreads == 0 || t < NBF) {
      const int b = t % B, jj = t / B;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = s[(jj + r * (L / R)) * B + b];
      if constexpr (Ns > 1) {
        const int k = jj % Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) v[it][r] = cmul(v[it][r], tw[r * k * (L / (Ns * R))]);
      }
      dftR<T, R>(v[it]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < PER; ++it) {
    const int t = tid + it * kFftThreads;
    if (NBF % kFftThreads == 0 || t < NBF) {
      const int b = t % B, jj = t / B;
      const int k = jj % Ns;
      const int base = (jj / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) s[(base + r * Ns) * B + b] = v[it][r];
    }
  }
  __syncthreads();
}

template <typename T, int L, int B, int Ns = 1>
__device__ __forceinline__ void fft_lines(C2<T>* s, const C2<T>* __restrict__ tw) {
  if constexpr (Ns < L) {
    constexpr int rem = L / Ns;
    constexpr int R = rem >= 16 ? 16 : rem >= 8 ? 8 : rem;
    fft_stage<T, L, B, Ns, R>(s, tw);
    fft_lines<T, L, B, Ns * R>(s, tw);
  }
}

// ---- x pass, forward: two real rows -> one complex line -> two half spectra
template <typename T, int L>
__global__ void __launch_bounds__(kFftThreads) k_fft_x_fwd(Geo geo, const T* __restrict__ Q,
                                                           C2<T>* __restrict__ S,
                                                           const C2<T>* __restrict__ tw) {
  constexpr int B = Cfg<T, L>::B;
  constexpr int N = L / 2, K = N + 1, KS = (K + 15) & ~15;
  __shared__ C2<T> s[L * B];
  const int ny = geo.grid[1];
  const long long rows = (long long)ny * geo.grid[2];
  const long long row0 = (long long)blockIdx.x * (2 * B);
  for (int e = threadIdx.x; e < L * B; e += kFftThreads) s[e] = C2<T>{(T)0, (T)0};
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * B * N; e += kFftThreads) {
    const int r = e / N, p = e % N;
    const long long gr = row0 + r;
    if (gr < rows) {
      T v = Q[gr * N + p];
      if (r & 1) s[p * B + (r >> 1)].y = v;
      else s[p * B + (r >> 1)].x = v;
    }
  }
  __syncthreads();
  fft_lines<T, L, B>(s, tw);
  for (int e = threadIdx.x; e < 2 * B * K; e += kFftThreads) {
    const int r = e / K, k = e % K;
    const long long gr = row0 + r;
    if (gr >= rows) continue;
    const int l = r >> 1;
    const C2<T> z = s[k * B + l], zm = s[((L - k) & (L - 1)) * B + l];
    C2<T> o;
    if (r & 1) o = C2<T>{(T)0.5 * (z.y + zm.y), (T)-0.5 * (z.x - zm.x)};   // (Z - conj Zm) / 2i
    else o = C2<T>{(T)0.5 * (z.x + zm.x), (T)0.5 * (z.y - zm.y)};          // (Z + conj Zm) / 2
    const long long z_ = gr / ny, y = gr % ny;
    S[(z_ * 2 * ny + y) * KS + k] = o;
  }
}

// ---- y pass: lines over y for fixed (z, kx); INV: inverse, keep y < N_y
// DIFF (inverse only, difference form of the mesh): the line is also
// multiplied by dy(k_y) = e^{2 pi i k_y / L} - 1 and inverse-transformed into
// S3 (same layout), the forward difference along y.
template <typename T, int L, bool INV, bool DIFF = false>
__global__ void __launch_bounds__(kFftThreads) k_fft_y(Geo geo, C2<T>* __restrict__ S,
                                                       const C2<T>* __restrict__ tw,
                                                       C2<T>* __restrict__ S3 = nullptr,
                                                       const C2<T>* __restrict__ dy = nullptr) {
  static_assert(INV || !DIFF, "the difference form acts on the inverse pass");
  constexpr int B = Cfg<T, L>::B;
  constexpr int N = L / 2;
  constexpr int PER = (L * B + kFftThreads - 1) / kFftThreads;
  __shared__ C2<T> s[L * B];
  const int K = geo.grid[0] + 1, KS = spec_stride(geo.grid[0]);
  int z, kx0;
  if (!line_block<Cfg<T, L>::G>((K + B - 1) / B, geo.grid[2], z, kx0, B)) return;
  C2<T>* base = S + (long long)z * L * KS;
  const int nin = INV ? L : N;
  C2<T> hold[DIFF ? PER : 1];
#pragma unroll
  for (int it = 0; it < PER; ++it) {
    const int e = threadIdx.x + it * kFftThreads;
    if (e < L * B) {
      const int p = e / B, b = e % B;
      C2<T> v{(T)0, (T)0};
      if (p < nin && kx0 + b < K) v = base[(long long)p * KS + kx0 + b];
      if (INV) v.y = -v.y;
      s[e] = v;
      if constexpr (DIFF) hold[it] = v;
    }
  }
  __syncthreads();
  fft_lines<T, L, B>(s, tw);
  const int nout = INV ? N : L;
  for (int e = threadIdx.x; e < nout * B; e += kFftThreads) {
    const int p = e / B, b = e % B;
    if (kx0 + b < K) {
      C2<T> v = s[e];
      if (INV) v.y = -v.y;
      base[(long long)p * KS + kx0 + b] = v;
    }
  }
  if constexpr (DIFF) {
    __syncthreads();
    // the loaded values are conj(S): conj(S dy) = conj(S) conj(dy)
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int e = threadIdx.x + it * kFftThreads;
      if (e < L * B) s[e] = cmul(hold[it], cconj(dy[e / B]));
    }
    __syncthreads();
    fft_lines<T, L, B>(s, tw);
    C2<T>* base3 = S3 + (long long)z * L * KS;
    for (int e = threadIdx.x; e < N * B; e += kFftThreads) {
      const int p = e / B, b = e % B;
      if (kx0 + b < K) {
        C2<T> v = s[e];
        base3[(long long)p * KS + kx0 + b] = C2<T>{v.x, -v.y};
      }
    }
  }
}

// ---- z pass: forward, times Ghat, inverse, keep z < N_z
// DIFF (difference form of the mesh): the product Ghat Z is also multiplied
// by dz(k_z) = e^{2 pi i k_z / L} - 1 and inverse-transformed into S2, the
// spectrum of the forward difference phi_{m+e_z} - phi_m along z.
template <typename T, int L, bool IMG, bool DIFF = false>
__global__ void __launch_bounds__(kFftThreads) k_fft_z(Geo geo, C2<T>* __restrict__ S,
                                                       const T* __restrict__ gz,
                                                       const C2<double>* __restrict__ gimg,
                                                       const C2<T>* __restrict__ tw,
                                                       C2<T>* __restrict__ S2 = nullptr,
                                                       const C2<T>* __restrict__ dz = nullptr) {
  static_assert(!(IMG && DIFF), "the difference form is built for open boundaries");
  constexpr int B = Cfg<T, L>::B;
  constexpr int N = L / 2;
  __shared__ C2<T> s[L * B];
  const int K = geo.grid[0] + 1, KS = spec_stride(geo.grid[0]);
  const int ly = 2 * geo.grid[1];
  int ky, kx0;
  if (!line_block<Cfg<T, L>::G>((K + B - 1) / B, ly, ky, kx0, B)) return;
  const long long zstride = (long long)ly * KS;
  C2<T>* base = S + (long long)ky * KS;
  for (int e = threadIdx.x; e < L * B; e += kFftThreads) {
    const int p = e / B, b = e % B;
    C2<T> v{(T)0, (T)0};
    if (p < N && kx0 + b < K) v = base[p * zstride + kx0 + b];
    s[e] = v;
  }
  __syncthreads();
  fft_lines<T, L, B>(s, tw);
  const int kyp = ky <= geo.grid[1] ? ky : ly - ky;
  const long long gplane = (long long)(geo.grid[1] + 1) * K;    // image table
  const long long gplane_s = (long long)(geo.grid[1] + 1) * KS;
  constexpr int PER = (L * B + kFftThreads - 1) / kFftThreads;
  if constexpr (DIFF) {
    // keep conj(g Z) in registers for the second inverse
    C2<T> hold[PER];
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int e = threadIdx.x + it * kFftThreads;
      if (e < L * B) {
        const int kz = e / B, b = e % B;
        const int kzp = kz <= N ? kz : L - kz;
        const int kx = kx0 + b < K ? kx0 + b : K - 1;
        const T g = gz[kzp * gplane_s + (long long)kyp * KS + kx];
        const C2<T> v = s[e];
        hold[it] = C2<T>{g * v.x, -(g * v.y)};
        s[e] = hold[it];
      }
    }
    __syncthreads();
    fft_lines<T, L, B>(s, tw);
    for (int e = threadIdx.x; e < N * B; e += kFftThreads) {
      const int p = e / B, b = e % B;
      if (kx0 + b < K) {
        C2<T> v = s[e];
        base[p * zstride + kx0 + b] = C2<T>{v.x, -v.y};
      }
    }
    __syncthreads();
    // conj(g Z dz) = conj(g Z) conj(dz)
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int e = threadIdx.x + it * kFftThreads;
      if (e < L * B) s[e] = cmul(hold[it], cconj(dz[e / B]));
    }
    __syncthreads();
    fft_lines<T, L, B>(s, tw);
    C2<T>* base2 = S2 + (long long)ky * KS;
    for (int e = threadIdx.x; e < N * B; e += kFftThreads) {
      const int p = e / B, b = e % B;
      if (kx0 + b < K) {
        C2<T> v = s[e];
        base2[p * zstride + kx0 + b] = C2<T>{v.x, -v.y};
      }
    }
    return;
  }
  if constexpr (!IMG) {
    for (int e = threadIdx.x; e < L * B; e += kFftThreads) {
      const int kz = e / B, b = e % B;
      const int kzp = kz <= N ? kz : L - kz;
      const int kx = kx0 + b < K ? kx0 + b : K - 1;   // a block may span more than a row
      const T g = gz[kzp * gplane_s + (long long)kyp * KS + kx];
      C2<T> v = s[e];
      s[e] = C2<T>{g * v.x, -(g * v.y)};   // conj(g Z): input of the inverse
    }
  } else {
    // grounded plane: minus the image term, Gs(k) Z(kx, ky, -kz) (the reflected
    // charge's spectrum), Gs the shifted kernel's table with phase and scale
    C2<T> nv[PER];
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int e = threadIdx.x + it * kFftThreads;
      if (e < L * B) {
        const int kz = e / B, b = e % B;
        const int kzp = kz <= N ? kz : L - kz;
        const int kzm = kz == 0 ? 0 : L - kz;
        const int kx = kx0 + b < K ? kx0 + b : K - 1;
        const T g = gz[kzp * gplane_s + (long long)kyp * KS + kx];
        const C2<double> gd = gimg[(long long)kz * gplane + (long long)kyp * K + kx];
        const C2<T> gs{(T)gd.x, (T)gd.y};
        const C2<T> v = s[e], vm = s[kzm * B + b];
        const T zr = g * v.x - (gs.x * vm.x - gs.y * vm.y);
        const T zi = g * v.y - (gs.x * vm.y + gs.y * vm.x);
        nv[it] = C2<T>{zr, -zi};
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int e = threadIdx.x + it * kFftThreads;
      if (e < L * B) s[e] = nv[it];
    }
  }
  __syncthreads();
  fft_lines<T, L, B>(s, tw);
  for (int e = threadIdx.x; e < N * B; e += kFftThreads) {
    const int p = e / B, b = e % B;
    if (kx0 + b < K) {
      C2<T> v = s[e];
      base[p * zstride + kx0 + b] = C2<T>{v.x, -v.y};
    }
  }
}

// ---- float lines of 256 points held in registers (y and z passes) ------------
// 256 = 16 x 16: with n = r + 16 m and k = k1 + 16 k2,
//   X[k] = sum_r w16^(r k2) w256^(r k1) sum_m x[r + 16 m] w16^(m k1).
// Thread t of a block takes line b = t % 16 (16 consecutive k_x) and index
// r = t / 16: it loads x[r + 16 m] straight from memory, transforms over m,
// twiddles, and passes the values through LDS (one transpose) to the thread
// that transforms over r, which then holds X[q + 16 k2] for its q = t / 16.
// That is again the input layout of a transform, so the z pass multiplies
// by the kernel table and starts the inverse in registers. Two LDS passes per
// line instead of one per radix stage plus the staging in and out.
constexpr int kRegL = 256;

__device__ __forceinline__ void reg_first_half(C2<float>* v, int r, const C2<float>* __restrict__ tw,
                                               C2<float>* s, int b) {
  dft16(v);
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], tw[r * k1]);
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) s[(k1 * 16 + r) * 16 + b] = v[k1];
}

__device__ __forceinline__ void reg_second_half(C2<float>* v, int q, const C2<float>* s, int b) {
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = s[(q * 16 + r) * 16 + b];
  dft16(v);
}

// y pass on 256-point float lines: forward (N inputs, all outputs) or inverse
// (all inputs, N outputs kept), conjugating around the forward transform.
template <bool INV>
__global__ void __launch_bounds__(kFftThreads) k_fft_y_reg(Geo geo, C2<float>* __restrict__ S,
                                                           const C2<float>* __restrict__ tw) {
  constexpr int L = kRegL, N = L / 2;
  __shared__ C2<float> s[L * 16];
  const int K = geo.grid[0] + 1, KS = spec_stride(geo.grid[0]);
  const int nch = (K + 15) / 16;
  const int z = blockIdx.x / nch, kx0 = (blockIdx.x % nch) * 16;
  const int b = threadIdx.x & 15, r = threadIdx.x >> 4;
  const bool valid = kx0 + b < K;
  C2<float>* base = S + (long long)z * L * KS + kx0 + b;
  C2<float> v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int p = r + 16 * m;
    C2<float> x{0.f, 0.f};
    if (valid && (INV || p < N)) x = base[(long long)p * KS];
    if (INV) x.y = -x.y;
    v[m] = x;
  }
  reg_first_half(v, r, tw, s, b);
  __syncthreads();
  reg_second_half(v, r, s, b);
  if (valid) {
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) {
      const int p = r + 16 * k2;
      if (INV && p >= N) continue;
      C2<float> x = v[k2];
      if (INV) x.y = -x.y;
      base[(long long)p * KS] = x;
    }
  }
}

// z pass on 256-point float lines, free space: forward, times the kernel
// table, inverse, keep z < N.
//
// Block order: the kernel table is float, so a block's 16 k_x values are half
// a 128-byte line, and rows k_y and 2 N_y - k_y read the same table row. The
// four blocks of one table line (two k_x chunks of a row and of its mirror)
// take slots kXcds apart in a run of 4 kXcds, so that they run on one XCD at
// about the same time and its L2 fetches the line once; slots with no row or
// chunk (self-mirrored rows 0 and N_y, an odd last chunk) end at once.
__host__ __device__ inline int z_reg_groups(const Geo& g) {
  return (g.grid[1] + 1) * ((g.grid[0] + 1 + 31) / 32);
}
__global__ void __launch_bounds__(kFftThreads) k_fft_z_reg(Geo geo, C2<float>* __restrict__ S,
                                                           const float* __restrict__ gz,
                                                           const C2<float>* __restrict__ tw) {
  constexpr int L = kRegL, N = L / 2;
  __shared__ C2<float> s[L * 16];
  const int K = geo.grid[0] + 1, KS = spec_stride(geo.grid[0]);
  const int ly = 2 * geo.grid[1];
  const int nch = (K + 15) / 16, ncp = (nch + 1) / 2;
  const int slot = (int)blockIdx.x;
  const int grp = (slot / (4 * kXcds)) * kXcds + slot % kXcds;
  const int member = (slot / kXcds) % 4;
  const int rg = grp / ncp, c = 2 * (grp % ncp) + (member >> 1);
  if (rg > geo.grid[1] || c >= nch) return;   // whole block: no barrier passed yet
  if ((member & 1) && (rg == 0 || rg == geo.grid[1])) return;
  const int ky = (member & 1) ? ly - rg : rg, kx0 = c * 16;
  const int b = threadIdx.x & 15, q = threadIdx.x >> 4;
  const int kx = kx0 + b;
  const bool valid = kx < K;
  const long long zstride = (long long)ly * KS;
  C2<float>* base = S + (long long)ky * KS + kx;
  C2<float> v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int p = q + 16 * m;
    v[m] = (valid && p < N) ? base[p * zstride] : C2<float>{0.f, 0.f};
  }
  // the kernel table at this thread's frequencies kz = q + 16 k2 (after the
  // forward transform), loaded now so that its latency overlaps the transform
  const float* grow = gz + (long long)rg * KS + (valid ? kx : K - 1);
  const long long gplane_s = (long long)(geo.grid[1] + 1) * KS;
  float g[16];
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) {
    const int kz = q + 16 * k2;
    g[k2] = grow[(kz <= N ? kz : L - kz) * gplane_s];
  }
  reg_first_half(v, q, tw, s, b);
  __syncthreads();
  reg_second_half(v, q, s, b);
  // v[k2] = Z(kz): conj(Ghat Z) is the inverse's input
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) v[k2] = C2<float>{g[k2] * v[k2].x, -(g[k2] * v[k2].y)};
  __syncthreads();   // every thread has read its column of s
  reg_first_half(v, q, tw, s, b);
  __syncthreads();
  reg_second_half(v, q, s, b);
  if (valid) {
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {   // z = q + 16 k2 < N
      const C2<float> x = v[k2];
      base[(long long)(q + 16 * k2) * zstride] = C2<float>{x.x, -x.y};
    }
  }
}

// ---- float lines of 1024 points held in registers (y and z passes) -----------
// 1024 = 16 x 16 x 4, w = e^{-2 pi i / 1024}. With n = r + 64 m (r < 64,
// m < 16), r = p + 4 q (p < 4, q < 16) and k = k1 + 16 c + 256 d (k1, c < 16,
// d < 4):
//   X[k] = sum_p w4^(p d) w^(16 p c) sum_q w16^(q c) [w^(r k1) sum_m x[r + 64 m] w16^(m k1)].
// A block of 256 threads holds B = 4 lines (b = t % 4, consecutive k_x):
//   phase A, thread (b, r = t / 4): its 16 points x[r + 64 m], a DFT-16 over m,
//     twiddles w^(r k1); LDS transpose;
//   phase B, thread (b, p = (t / 4) % 4, k1 = t / 16): a DFT-16 over q,
//     twiddles w^(16 p c); LDS transpose;
//   phase C, thread (b, c4 = (t / 4) % 4, k1): DFT-4s over p, after which it
//     holds X[k1 + 16 (4 c4 + j) + 256 d] for j, d < 4 at v[4 j + d].
// The transposed network takes that layout back: with the same index
// splitting read the other way, Z[r + 64 m] = sum_{k1} w16^(k1 m) w^(k1 r)
// sum_c w16^(c q) w^(16 c p) sum_d w4^(d p) y[k1 + 16 c + 256 d] is a forward
// transform from the C layout to the A layout (DFT-4s in registers, two LDS
// transposes, DFT-16s), so a line multiplied in the C layout goes straight
// into the inverse. The LDS rows of one k1 are kPad1k entries apart, so the
// four k1 of a wave's reads fall in different banks.
constexpr int kReg1k = 1024;
constexpr int kPad1k = 4 * 64 + 16;

__device__ __forceinline__ void fwd1k(C2<float>* v, C2<float>* s, const C2<float>* __restrict__ tw) {
  const int t = threadIdx.x, b = t & 3;
  {
    const int r = t >> 2;
    dft16(v);
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], tw[r * k1]);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) s[k1 * kPad1k + 4 * r + b] = v[k1];
  }
  __syncthreads();
  const int p = (t >> 2) & 3, k1 = t >> 4;
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = s[k1 * kPad1k + 4 * (p + 4 * q) + b];
  dft16(v);
#pragma unroll
  for (int c = 1; c < 16; ++c) v[c] = cmul(v[c], tw[16 * p * c]);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 16; ++c) s[k1 * kPad1k + ((c & 3) * 4 + p) * 16 + (c >> 2) * 4 + b] = v[c];
  __syncthreads();
  const int c4 = p;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    C2<float> u[4];
#pragma unroll
    for (int pp = 0; pp < 4; ++pp) u[pp] = s[k1 * kPad1k + (j * 4 + pp) * 16 + c4 * 4 + b];
    dft4(u);
#pragma unroll
    for (int d = 0; d < 4; ++d) v[4 * j + d] = u[d];
  }
}

// The transposed network: v[4 j + d] = y[k1 + 16 (4 c4 + j) + 256 d] on entry
// (C layout), v[m] = Z[r + 64 m] on return (A layout), Z the forward
// transform of y. The caller syncs before it if s was being read.
__device__ __forceinline__ void fwd1k_t(C2<float>* v, C2<float>* s, const C2<float>* __restrict__ tw) {
  const int t = threadIdx.x, b = t & 3, c4 = (t >> 2) & 3, k1 = t >> 4;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    C2<float> u[4] = {v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]};
    dft4(u);   // over d, output index p
    const int c = 4 * c4 + j;
#pragma unroll
    for (int pp = 0; pp < 4; ++pp) {
      const C2<float> x = pp ? cmul(u[pp], tw[16 * c * pp]) : u[0];
      s[k1 * kPad1k + (j * 4 + pp) * 16 + c4 * 4 + b] = x;
    }
  }
  __syncthreads();
  const int p = c4;
#pragma unroll
  for (int c = 0; c < 16; ++c) v[c] = s[k1 * kPad1k + ((c & 3) * 4 + p) * 16 + (c >> 2) * 4 + b];
  dft16(v);   // over c, output index q
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = k1 * (p + 4 * q);
    if (q || p) v[q] = cmul(v[q], tw[e]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) s[k1 * kPad1k + 4 * (p + 4 * q) + b] = v[q];
  __syncthreads();
  const int r = t >> 2;
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) v[kk] = s[kk * kPad1k + 4 * r + b];
  dft16(v);   // over k1, output index m
}

// Frequency held at v[e] in the C layout: k1 + 16 (4 c4 + j) + 256 d, e = 4 j + d.
__device__ __forceinline__ int c1k_freq(int e) {
  const int t = threadIdx.x;
  return (t >> 4) + 16 * (4 * ((t >> 2) & 3) + (e >> 2)) + 256 * (e & 3);
}

// z pass on 1024-point float lines, free space: forward (N = 512 inputs),
// times the kernel table, inverse, keep z < N; DIFF: also the inverse of the
// product times dz(k_z) = e^{2 pi i k_z / L} - 1 into S2 (the z difference).
// Block order as k_fft_z (line_block, 4 k_x per block).
template <bool DIFF>
__global__ void __launch_bounds__(kFftThreads) k_fft_z_1k(Geo geo, C2<float>* __restrict__ S,
                                                          const float* __restrict__ gz,
                                                          const C2<float>* __restrict__ tw,
                                                          C2<float>* __restrict__ S2,
                                                          const C2<float>* __restrict__ dz) {
  constexpr int L = kReg1k, N = L / 2, B = 4;
  __shared__ C2<float> s[16 * kPad1k];
  const int K = geo.grid[0] + 1, KS = spec_stride(geo.grid[0]);
  const int ly = 2 * geo.grid[1];
  int ky, kx0;
  if (!line_block<Cfg<float, L>::G>((K + B - 1) / B, ly, ky, kx0, B)) return;
  const int t = threadIdx.x, b = t & 3, r = t >> 2;
  const int kx = kx0 + b;
  const bool valid = kx < K;
  const long long zstride = (long long)ly * KS;
  C2<float>* base = S + (long long)ky * KS + kx;
  C2<float> v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m)
    v[m] = (m < 8 && valid) ? base[(long long)(r + 64 * m) * zstride] : C2<float>{0.f, 0.f};
  // the kernel table at this thread's frequencies, loaded before the transform
  const int kyp = ky <= geo.grid[1] ? ky : ly - ky;
  const long long gplane_s = (long long)(geo.grid[1] + 1) * KS;
  const float* grow = gz + (long long)kyp * KS + (valid ? kx : K - 1);
  float g[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int kz = c1k_freq(e);
    g[e] = grow[(kz <= N ? kz : L - kz) * gplane_s];
  }
  fwd1k(v, s, tw);
  // conj(Ghat Z): the input of the inverse
#pragma unroll
  for (int e = 0; e < 16; ++e) v[e] = C2<float>{g[e] * v[e].x, -(g[e] * v[e].y)};
  C2<float> hold[DIFF ? 16 : 1];
  if constexpr (DIFF) {
#pragma unroll
    for (int e = 0; e < 16; ++e) hold[e] = v[e];
  }
  __syncthreads();   // phase C's reads of s are done
  fwd1k_t(v, s, tw);
  if (valid) {
#pragma unroll
    for (int m = 0; m < 8; ++m) base[(long long)(r + 64 * m) * zstride] = C2<float>{v[m].x, -v[m].y};
  }
  if constexpr (DIFF) {
    // conj(g Z dz) = conj(g Z) conj(dz)
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = cmul(hold[e], cconj(dz[c1k_freq(e)]));
    __syncthreads();
    fwd1k_t(v, s, tw);
    if (valid) {
      C2<float>* base2 = S2 + (long long)ky * KS + kx;
#pragma unroll
      for (int m = 0; m < 8; ++m) base2[(long long)(r + 64 * m) * zstride] = C2<float>{v[m].x, -v[m].y};
    }
  }
}

// y pass on 1024-point float lines: forward (N inputs, all outputs, C-layout
// stores) or inverse (all inputs loaded in the C layout, N outputs kept),
// conjugating around the transposed network; DIFF (inverse only): also the
// inverse of the line times dy(k_y) into S3 (the y difference).
template <bool INV, bool DIFF>
__global__ void __launch_bounds__(kFftThreads) k_fft_y_1k(Geo geo, C2<float>* __restrict__ S,
                                                          const C2<float>* __restrict__ tw,
                                                          C2<float>* __restrict__ S3,
                                                          const C2<float>* __restrict__ dy) {
  static_assert(INV || !DIFF, "the difference form acts on the inverse pass");
  constexpr int L = kReg1k, B = 4;
  __shared__ C2<float> s[16 * kPad1k];
  const int K = geo.grid[0] + 1, KS = spec_stride(geo.grid[0]);
  int z, kx0;
  if (!line_block<Cfg<float, L>::G>((K + B - 1) / B, geo.grid[2], z, kx0, B)) return;
  const int t = threadIdx.x, b = t & 3, r = t >> 2;
  const int kx = kx0 + b;
  const bool valid = kx < K;
  C2<float>* base = S + (long long)z * L * KS + kx;
  C2<float> v[16];
  if constexpr (!INV) {
#pragma unroll
    for (int m = 0; m < 16; ++m)
      v[m] = (m < 8 && valid) ? base[(long long)(r + 64 * m) * KS] : C2<float>{0.f, 0.f};
    fwd1k(v, s, tw);
    if (valid) {
#pragma unroll
      for (int e = 0; e < 16; ++e) base[(long long)c1k_freq(e) * KS] = v[e];
    }
  } else {
    // conj of the spectrum in the C layout
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      C2<float> x = valid ? base[(long long)c1k_freq(e) * KS] : C2<float>{0.f, 0.f};
      v[e] = C2<float>{x.x, -x.y};
    }
    C2<float> hold[DIFF ? 16 : 1];
    if constexpr (DIFF) {
#pragma unroll
      for (int e = 0; e < 16; ++e) hold[e] = v[e];
    }
    fwd1k_t(v, s, tw);
    if (valid) {
#pragma unroll
      for (int m = 0; m < 8; ++m) base[(long long)(r + 64 * m) * KS] = C2<float>{v[m].x, -v[m].y};
    }
    if constexpr (DIFF) {
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = cmul(hold[e], cconj(dy[c1k_freq(e)]));
      __syncthreads();
      fwd1k_t(v, s, tw);
      if (valid) {
        C2<float>* base3 = S3 + (long long)z * L * KS + kx;
#pragma unroll
        for (int m = 0; m < 8; ++m) base3[(long long)(r + 64 * m) * KS] = C2<float>{v[m].x, -v[m].y};
      }
    }
  }
}

// x passes on 256-point float lines (two real rows of N = 128 per complex
// line): the same 16 x 16 transform, with the lanes of a line along the
// row (index fastest) so that loads and stores run along rows. The LDS rows
// are 17 long so that the transposed reads do not share banks.
constexpr int kXPad = 17;

__global__ void __launch_bounds__(kFftThreads) k_fft_x_fwd_reg(Geo geo, const float* __restrict__ Q,
                                                               C2<float>* __restrict__ S,
                                                               const C2<float>* __restrict__ tw) {
  constexpr int L = kRegL, N = L / 2, K = N + 1, KS = (K + 15) & ~15;
  __shared__ C2<float> s[16 * 16 * kXPad];
  const int ny = geo.grid[1];
  const long long rows = (long long)ny * geo.grid[2];
  const int r = threadIdx.x & 15, b = threadIdx.x >> 4;
  const long long ra = (long long)blockIdx.x * 32 + 2 * b, rc = ra + 1;
  C2<float> v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    v[m] = C2<float>{0.f, 0.f};
    if (m < 8) {
      const int p = r + 16 * m;
      if (ra < rows) v[m].x = Q[ra * N + p];
      if (rc < rows) v[m].y = Q[rc * N + p];
    }
  }
  dft16(v);
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], tw[r * k1]);
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) s[(b * 16 + k1) * kXPad + r] = v[k1];
  __syncthreads();
  const int q = r;   // this thread now transforms over r for k1 = q
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = s[(b * 16 + q) * kXPad + j];
  dft16(v);          // v[k2] = Z(q + 16 k2)
  __syncthreads();
  C2<float>* zs = s + b * L;   // natural order, for Z(L - k)
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) zs[q + 16 * k2] = v[k2];
  __syncthreads();
#pragma unroll
  for (int k2 = 0; k2 < 9; ++k2) {
    const int k = q + 16 * k2;
    if (k > N) continue;
    const C2<float> z = v[k2], zm = zs[(L - k) & (L - 1)];
    if (ra < rows)   // (Z + conj Zm) / 2
      S[((ra / ny) * 2 * ny + ra % ny) * KS + k] = C2<float>{0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y)};
    if (rc < rows)   // (Z - conj Zm) / 2i
      S[((rc / ny) * 2 * ny + rc % ny) * KS + k] = C2<float>{0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x)};
  }
}

__global__ void __launch_bounds__(kFftThreads) k_fft_x_inv_reg(Geo geo, const C2<float>* __restrict__ S,
                                                               float* __restrict__ phi,
                                                               const C2<float>* __restrict__ tw) {
  constexpr int L = kRegL, N = L / 2, K = N + 1, KS = (K + 15) & ~15;
  __shared__ C2<float> s[16 * 16 * kXPad];
  const int ny = geo.grid[1];
  const long long rows = (long long)ny * geo.grid[2];
  const int r = threadIdx.x & 15, b = threadIdx.x >> 4;
  const long long ra = (long long)blockIdx.x * 32 + 2 * b, rc = ra + 1;
  const C2<float>* A = S + ((ra / ny) * 2 * ny + ra % ny) * KS;
  const C2<float>* C = S + ((rc / ny) * 2 * ny + rc % ny) * KS;
  // conj(Z_n), Z = A + i C the packed line: Z_n from (A_n, C_n) for n <= N,
  // from conj(A_{L-n}) + i conj(C_{L-n}) above
  C2<float> v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int n = r + 16 * m;
    const int k = n <= N ? n : L - n;
    C2<float> a{0.f, 0.f}, c{0.f, 0.f};
    if (ra < rows) a = A[k];
    if (rc < rows) c = C[k];
    v[m] = n <= N ? C2<float>{a.x - c.y, -(a.y + c.x)} : C2<float>{a.x + c.y, a.y - c.x};
  }
  dft16(v);
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], tw[r * k1]);
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) s[(b * 16 + k1) * kXPad + r] = v[k1];
  __syncthreads();
  const int q = r;
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = s[(b * 16 + q) * kXPad + j];
  dft16(v);          // v[k2] = conj of the inverse at n = q + 16 k2
#pragma unroll
  for (int k2 = 0; k2 < 8; ++k2) {   // n < N
    const int n = q + 16 * k2;
    if (ra < rows) phi[ra * N + n] = v[k2].x;
    if (rc < rows) phi[rc * N + n] = -v[k2].y;
  }
}

// ---- x pass, inverse: two half spectra -> one complex line -> two real rows
// dx (difference form of the mesh, may be null): both half spectra are first
// multiplied by dx(k_x) = e^{2 pi i k_x / L} - 1, giving the forward
// difference along x.
template <typename T, int L>
__global__ void __launch_bounds__(kFftThreads) k_fft_x_inv(Geo geo, const C2<T>* __restrict__ S,
                                                           T* __restrict__ phi,
                                                           const C2<T>* __restrict__ tw,
                                                           const C2<T>* __restrict__ dx = nullptr) {
  constexpr int B = Cfg<T, L>::B;
  constexpr int N = L / 2, K = N + 1, KS = (K + 15) & ~15;
  __shared__ C2<T> s[L * B];
  const int ny = geo.grid[1];
  const long long rows = (long long)ny * geo.grid[2];
  const long long row0 = (long long)blockIdx.x * (2 * B);
  for (int e = threadIdx.x; e < B * K; e += kFftThreads) {
    const int l = e / K, k = e % K;
    const long long ga = row0 + 2 * l, gc = ga + 1;
    C2<T> A{(T)0, (T)0}, C{(T)0, (T)0};
    if (ga < rows) A = S[((ga / ny) * 2 * ny + ga % ny) * KS + k];
    if (gc < rows) C = S[((gc / ny) * 2 * ny + gc % ny) * KS + k];
    if (dx) {
      const C2<T> f = dx[k];
      A = cmul(A, f);
      C = cmul(C, f);
    }
    // Z_k = A_k + i C_k ; stored conjugated (input of the inverse)
    s[k * B + l] = C2<T>{A.x - C.y, -(A.y + C.x)};
    if (k > 0 && k < N) s[(L - k) * B + l] = C2<T>{A.x + C.y, -(C.x - A.y)};
  }
  __syncthreads();
  fft_lines<T, L, B>(s, tw);
  for (int e = threadIdx.x; e < 2 * B * N; e += kFftThreads) {
    const int r = e / N, p = e % N;
    const long long gr = row0 + r;
    if (gr >= rows) continue;
    const C2<T> v = s[p * B + (r >> 1)];
    phi[gr * N + p] = (r & 1) ? -v.y : v.x;
  }
}

// ---- Fourier table of the sampled kernel (float64) -------------------------

__global__ void k_green_sample(Geo geo, double* __restrict__ g) {
  const int kx = geo.grid[0] + 1, ky = geo.grid[1] + 1, kz = geo.grid[2] + 1;
  const long long total = (long long)kx * ky * kz;
  const long long e = blockIdx.x * (long long)kThreads + threadIdx.x;
  if (e >= total) return;
  const int ix = (int)(e % kx), iy = (int)((e / kx) % ky), iz = (int)(e / ((long long)kx * ky));
  const double rx = ix * geo.hu[0], ry = iy * geo.hu[1], rz = iz * geo.hu[2];
  const double rho = sqrt(rx * rx + ry * ry + rz * rz);
  g[e] = rho == 0.0 ? 1.12837916709551257390 * geo.kappa : erf(geo.kappa * rho) / rho;
}

// Even extension to 2N points, transformed along one axis: a cosine sum
//   out[k] = sum_{d=0}^{N} c_d in[d] cos(pi k d / N),  c_0 = c_N = 1, else 2.
__global__ void k_green_dct(int axis, Geo geo, const double* __restrict__ in, double* __restrict__ out,
                            const double* __restrict__ cosv, double scale) {
  const int kx = geo.grid[0] + 1, ky = geo.grid[1] + 1, kz = geo.grid[2] + 1;
  const long long total = (long long)kx * ky * kz;
  const long long e = blockIdx.x * (long long)kThreads + threadIdx.x;
  if (e >= total) return;
  const int ext[3] = {kx, ky, kz};
  const long long stride[3] = {1, kx, (long long)kx * ky};
  const int n = geo.grid[axis];
  const int idx[3] = {(int)(e % kx), (int)((e / kx) % ky), (int)(e / ((long long)kx * ky))};
  const int k = idx[axis];
  const long long line = e - (long long)k * stride[axis];
  double acc = 0.0;
  for (int d = 0; d <= n; ++d) {
    const double c = (d == 0 || d == n) ? 1.0 : 2.0;
    acc += c * in[line + d * stride[axis]] * cosv[((long long)k * d) % (2 * n)];
  }
  out[e] = acc * scale;
  (void)ext;
}

// ---- Fourier table of the image term (grounded plane z = zc), float64 ------
// With the charge reflected in z (node k -> N_z - 1 - k) the mirror images of
// the nodes sit at z-offset delta_z h_z + D from the field nodes,
// D = (N_z - 1) h_z + 2 (z0 - zc): the image potential is the aperiodic
// convolution of the reflected charge with G shifted by D in z (the shifted
// Green's function of Sec. 3.1, eq. GreenFunc_planar_cathode with the mirror
// map of eq. symmetry_planar_cathode). The kernel is even in x and y, so its
// table keeps k_x, k_y in [0, N]; in z it is complex over all 2 N_z
// frequencies. The reflection becomes Z(k_z) -> e^{-2 pi i k_z (N_z-1)/L_z}
// Z(-k_z), whose phase is folded in here with the 1/(L_x L_y L_z) of the
// inverse. Built per evaluation (D follows the placement), in internal units.

// x: sample and transform lines over x for every (y offset, z slot); keep
// the real part (even input) for k_x in [0, N_x].
template <int L>
__global__ void __launch_bounds__(kFftThreads) k_gimg_x(Geo geo, const Place* __restrict__ pl,
                                                        double* __restrict__ t1,
                                                        const C2<double>* __restrict__ tw) {
  constexpr int B = Cfg<double, L>::B;
  constexpr int N = L / 2;
  __shared__ C2<double> s[L * B];
  const int ny1 = geo.grid[1] + 1, nz = geo.grid[2], lz = 2 * nz;
  const long long lines = (long long)ny1 * lz;
  const long long l0 = (long long)blockIdx.x * B;
  const double du = (nz - 1) * geo.hu[2] + 2.0 * (pl->x0[2] - geo.zc) * pl->inv_lu;
  const double g0 = 1.12837916709551257390 * geo.kappa;
  for (int e = threadIdx.x; e < L * B; e += kFftThreads) {
    const int p = e / B, b = e % B;
    const long long line = l0 + b;
    double v = 0.0;
    if (line < lines) {
      const int iy = (int)(line % ny1), jz = (int)(line / ny1);
      if (jz != nz) {   // slot nz (offset +-N_z) is never reached by a node pair
        const int dx = p <= N ? p : L - p;
        const int dz = jz < nz ? jz : jz - lz;
        const double rx = dx * geo.hu[0], ry = iy * geo.hu[1], rz = dz * geo.hu[2] + du;
        const double rho = sqrt(rx * rx + ry * ry + rz * rz);
        v = rho == 0.0 ? g0 : erf(geo.kappa * rho) / rho;
      }
    }
    s[e] = C2<double>{v, 0.0};
  }
  __syncthreads();
  fft_lines<double, L, B>(s, tw);
  for (int e = threadIdx.x; e < (N + 1) * B; e += kFftThreads) {
    const int k = e / B, b = e % B;
    const long long line = l0 + b;
    if (line < lines) t1[line * (N + 1) + k] = s[k * B + b].x;
  }
}

// y: even lines over y for every (k_x, z slot); real part for k_y in [0, N_y].
template <int L>
__global__ void __launch_bounds__(kFftThreads) k_gimg_y(Geo geo, const double* __restrict__ t1,
                                                        double* __restrict__ t2,
                                                        const C2<double>* __restrict__ tw) {
  constexpr int B = Cfg<double, L>::B;
  constexpr int N = L / 2;
  __shared__ C2<double> s[L * B];
  const int K = geo.grid[0] + 1, ny1 = N + 1;
  const int nch = (K + B - 1) / B;
  const int jz = blockIdx.x / nch, kx0 = (blockIdx.x % nch) * B;
  for (int e = threadIdx.x; e < L * B; e += kFftThreads) {
    const int p = e / B, b = e % B;
    const int iy = p <= N ? p : L - p;
    double v = 0.0;
    if (kx0 + b < K) v = t1[((long long)jz * ny1 + iy) * K + kx0 + b];
    s[e] = C2<double>{v, 0.0};
  }
  __syncthreads();
  fft_lines<double, L, B>(s, tw);
  for (int e = threadIdx.x; e < ny1 * B; e += kFftThreads) {
    const int k = e / B, b = e % B;
    if (kx0 + b < K) t2[((long long)jz * ny1 + k) * K + kx0 + b] = s[k * B + b].x;
  }
}

// z: complex lines over all z slots for every (k_x, k_y); phase and scale.
template <int L>
__global__ void __launch_bounds__(kFftThreads) k_gimg_z(Geo geo, const double* __restrict__ t2,
                                                        C2<double>* __restrict__ gimg,
                                                        const C2<double>* __restrict__ tw) {
  constexpr int B = Cfg<double, L>::B;
  __shared__ C2<double> s[L * B];
  const int K = geo.grid[0] + 1, ny1 = geo.grid[1] + 1, nz = geo.grid[2];
  const int nch = (K + B - 1) / B;
  const int ky = blockIdx.x / nch, kx0 = (blockIdx.x % nch) * B;
  for (int e = threadIdx.x; e < L * B; e += kFftThreads) {
    const int p = e / B, b = e % B;
    double v = 0.0;
    if (kx0 + b < K) v = t2[((long long)p * ny1 + ky) * K + kx0 + b];
    s[e] = C2<double>{v, 0.0};
  }
  __syncthreads();
  fft_lines<double, L, B>(s, tw);
  const double scale = 1.0 / (8.0 * (double)geo.grid[0] * geo.grid[1] * nz);
  for (int e = threadIdx.x; e < L * B; e += kFftThreads) {
    const int k = e / B, b = e % B;
    if (kx0 + b < K) {
      const C2<double> ph = tw[((long long)k * (nz - 1)) % L];   // e^{-2 pi i k (N_z - 1) / L}
      const C2<double> v = cmul(s[e], ph);
      gimg[((long long)k * ny1 + ky) * K + kx0 + b] = C2<double>{v.x * scale, v.y * scale};
    }
  }
}

// ---- optimal influence function (Sec. 3.1.2, eq. Ghfinal) ---------------------
// For point particles with the Gaussian screening in the reference kernel,
// (R gamma)(k) = 4 pi exp(-k^2 / (4 kappa^2)) / k^2, and the assignment
// U(k) = prod_d sinc(k_d h_d / 2)^(p+1):
//   optimal (mode 1): G = sum_m U^2(k_m) (R gamma)(k_m) / [sum_m U^2(k_m)]^2,
//                     k_m = k - 2 pi m / h, |m_d| <= 2;
//   principal (mode 2): the m = 0 term, (R gamma)(k) / U^2(k).
// The table gets (G - (R gamma)(k)) / (h_x h_y h_z) added to the transform of
// the sampled kernel: the difference is finite at k = 0 and short-ranged, so
// the mesh kernel becomes the optimum near the origin while its erf(kappa r)/r
// tail, which the zero-padded open boundary relies on, is kept. Octant
// entries (the table is even in each k_d); the k = 0 entry is the limit along
// k_x. Internal units (lengths in r_c).
__device__ __forceinline__ double sinc_pow(double kh, int p1) {
  const double x = 0.5 * kh;
  const double s = x == 0.0 ? 1.0 : sin(x) / x;
  double r = s;
  for (int i = 1; i < p1; ++i) r *= s;
  return r;
}

__device__ __forceinline__ double rgamma(double kx, double ky, double kz, double kappa) {
  const double k2 = kx * kx + ky * ky + kz * kz;
  return 4.0 * M_PI * exp(-k2 / (4.0 * kappa * kappa)) / k2;
}

__global__ void k_green_influence(Geo geo, int mode, double* __restrict__ ghat, double scale) {
  const int nx1 = geo.grid[0] + 1, ny1 = geo.grid[1] + 1, nz1 = geo.grid[2] + 1;
  const long long total = (long long)nx1 * ny1 * nz1;
  const long long e = blockIdx.x * (long long)kThreads + threadIdx.x;
  if (e >= total) return;
  const int i[3] = {(int)(e % nx1), (int)((e / nx1) % ny1), (int)(e / ((long long)nx1 * ny1))};
  double k[3];
  for (int d = 0; d < 3; ++d) k[d] = M_PI * i[d] / (geo.grid[d] * geo.hu[d]);
  if (e == 0) k[0] = 1e-3 * M_PI / (geo.grid[0] * geo.hu[0]);
  const int p1 = geo.order + 1;
  const double h[3] = {geo.hu[0], geo.hu[1], geo.hu[2]};
  double G;
  if (mode == 2) {
    double u2 = 1.0;
    for (int d = 0; d < 3; ++d) {
      const double u = sinc_pow(k[d] * h[d], p1);
      u2 *= u * u;
    }
    G = rgamma(k[0], k[1], k[2], geo.kappa) / u2;
  } else {
    constexpr int M = 2;
    double num = 0.0, den[3] = {0.0, 0.0, 0.0};
    double u2a[3][2 * M + 1];
    for (int d = 0; d < 3; ++d)
      for (int m = -M; m <= M; ++m) {
        const double u = sinc_pow((k[d] - 2.0 * M_PI * m / h[d]) * h[d], p1);
        u2a[d][m + M] = u * u;
        den[d] += u * u;
      }
    for (int mz = -M; mz <= M; ++mz)
      for (int my = -M; my <= M; ++my)
        for (int mx = -M; mx <= M; ++mx) {
          const double u2 = u2a[0][mx + M] * u2a[1][my + M] * u2a[2][mz + M];
          num += u2 * rgamma(k[0] - 2.0 * M_PI * mx / h[0], k[1] - 2.0 * M_PI * my / h[1],
                             k[2] - 2.0 * M_PI * mz / h[2], geo.kappa);
        }
    const double dd = den[0] * den[1] * den[2];
    G = num / (dd * dd);
  }
  const double corr = (G - rgamma(k[0], k[1], k[2], geo.kappa)) / (h[0] * h[1] * h[2]);
  ghat[e] += corr * scale;
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

template <typename T, int L>
void run_x_fwd(const Geo& g, const T* Q, C2<T>* S, const C2<T>* tw, hipStream_t st) {
  constexpr int B = Cfg<T, L>::B;
  long long rows = (long long)g.grid[1] * g.grid[2];
  if constexpr (std::is_same<T, float>::value && L == kRegL) {
    k_fft_x_fwd_reg<<<(unsigned)((rows + 31) / 32), kFftThreads, 0, st>>>(g, Q, S, tw);
    return;
  }
  unsigned blocks = (unsigned)((rows + 2 * B - 1) / (2 * B));
  k_fft_x_fwd<T, L><<<blocks, kFftThreads, 0, st>>>(g, Q, S, tw);
}
template <typename T, int L>
void run_x_inv(const Geo& g, const C2<T>* S, T* phi, const C2<T>* tw, hipStream_t st) {
  constexpr int B = Cfg<T, L>::B;
  long long rows = (long long)g.grid[1] * g.grid[2];
  if constexpr (std::is_same<T, float>::value && L == kRegL) {
    k_fft_x_inv_reg<<<(unsigned)((rows + 31) / 32), kFftThreads, 0, st>>>(g, S, phi, tw);
    return;
  }
  unsigned blocks = (unsigned)((rows + 2 * B - 1) / (2 * B));
  k_fft_x_inv<T, L><<<blocks, kFftThreads, 0, st>>>(g, S, phi, tw);
}
template <typename T, int L, bool INV>
void run_y(const Geo& g, C2<T>* S, const C2<T>* tw, hipStream_t st) {
  constexpr int B = Cfg<T, L>::B;
  int K = g.grid[0] + 1;
  if constexpr (std::is_same<T, float>::value && L == kRegL) {
    static_assert(B == 16, "register lines take 16 k_x per block");
    k_fft_y_reg<INV><<<(unsigned)(g.grid[2] * ((K + 15) / 16)), kFftThreads, 0, st>>>(g, S, tw);
    return;
  }
  if constexpr (std::is_same<T, float>::value && L == kReg1k) {
    static_assert(B == 4, "1024-point register lines take 4 k_x per block");
    k_fft_y_1k<INV, false><<<line_grid<T, L>(g.grid[2], K), kFftThreads, 0, st>>>(g, S, tw, nullptr, nullptr);
    return;
  }
  k_fft_y<T, L, INV><<<line_grid<T, L>(g.grid[2], K), kFftThreads, 0, st>>>(g, S, tw);
}
template <typename T, int L>
void run_z(const Geo& g, C2<T>* S, const T* gz, const C2<double>* gimg, const C2<T>* tw,
           hipStream_t st) {
  int K = g.grid[0] + 1;
  const unsigned blocks = line_grid<T, L>(2 * g.grid[1], K);
  if constexpr (std::is_same<T, float>::value && L == kRegL) {
    if (!gimg) {
      const unsigned slots = (unsigned)((z_reg_groups(g) + kXcds - 1) / kXcds * 4 * kXcds);
      k_fft_z_reg<<<slots, kFftThreads, 0, st>>>(g, S, gz, tw);
      return;
    }
  }
  if constexpr (std::is_same<T, float>::value && L == kReg1k) {
    if (!gimg) {
      k_fft_z_1k<false><<<blocks, kFftThreads, 0, st>>>(g, S, gz, tw, nullptr, nullptr);
      return;
    }
  }
  if (gimg)
    k_fft_z<T, L, true><<<blocks, kFftThreads, 0, st>>>(g, S, gz, gimg, tw);
  else
    k_fft_z<T, L, false><<<blocks, kFftThreads, 0, st>>>(g, S, gz, nullptr, tw);
}

// The z pass's copy of the kernel table: float64 octant [N_z+1][N_y+1][N_x+1]
// -> mesh precision with rows of spec_stride(N_x), zero in the padding.
template <typename R>
__global__ void k_green_pack(Geo geo, const double* __restrict__ ghat, R* __restrict__ gz) {
  const int K = geo.grid[0] + 1, KS = spec_stride(geo.grid[0]);
  const long long rows = (long long)(geo.grid[1] + 1) * (geo.grid[2] + 1);
  const long long e = blockIdx.x * (long long)kThreads + threadIdx.x;
  if (e >= rows * KS) return;
  const long long row = e / KS;
  const int kx = (int)(e % KS);
  gz[e] = kx < K ? (R)ghat[row * K + kx] : (R)0;
}

#define P3M_FFT_SWITCH(L_, CALL) \
  switch (L_) {                  \
    case 8: CALL(8); break;      \
    case 16: CALL(16); break;    \
    case 32: CALL(32); break;    \
    case 64: CALL(64); break;    \
    case 128: CALL(128); break;  \
    case 256: CALL(256); break;  \
    case 512: CALL(512); break;  \
    case 1024: CALL(1024); break;\
    case 2048: CALL(2048); break;\
    default: break;              \
  }

}  // namespace

bool fft_supported(int nodes) {
  return nodes >= 4 && nodes <= 1024 && (nodes & (nodes - 1)) == 0;
}

size_t spectrum_elems(const Geo& g) {
  return (size_t)g.grid[2] * 2 * g.grid[1] * spec_stride(g.grid[0]);
}

size_t green_pack_elems(const Geo& g) {
  return (size_t)(g.grid[2] + 1) * (g.grid[1] + 1) * spec_stride(g.grid[0]);
}

template <typename R>
void launch_green_pack(const Geo& g, const double* ghat, R* gz, hipStream_t st) {
  k_green_pack<R><<<blocks_for((long long)green_pack_elems(g)), kThreads, 0, st>>>(g, ghat, gz);
}

template <typename R>
void launch_convolve(const Geo& g, const R* Q, C2<R>* S, const R* gz, const C2<double>* gimg,
                     const C2<R>* tw[3], R* phi, hipStream_t st) {
  const int Lx = 2 * g.grid[0], Ly = 2 * g.grid[1], Lz = 2 * g.grid[2];
#define XF(L) run_x_fwd<R, L>(g, Q, S, tw[0], st)
#define YF(L) run_y<R, L, false>(g, S, tw[1], st)
#define ZZ(L) run_z<R, L>(g, S, gz, gimg, tw[2], st)
#define YI(L) run_y<R, L, true>(g, S, tw[1], st)
#define XI(L) run_x_inv<R, L>(g, S, phi, tw[0], st)
  P3M_FFT_SWITCH(Lx, XF)
  P3M_FFT_SWITCH(Ly, YF)
  P3M_FFT_SWITCH(Lz, ZZ)
  P3M_FFT_SWITCH(Ly, YI)
  P3M_FFT_SWITCH(Lx, XI)
#undef XF
#undef YF
#undef ZZ
#undef YI
#undef XI
}

// Difference form (float meshes wider than the register lines): the three
// forward differences D_d phi_m = phi_{m+e_d} - phi_m come out of the same
// spectrum times (e^{2 pi i k_d / L_d} - 1), so their rounding follows the
// differences, not the potential. Passes: x and y forward as above; z with
// the second inverse into S2 (z difference); y inverse with the second
// inverse into S3 (y difference) and a plain y inverse of S2; then x inverse
// of S times dx (x difference), of S3 and of S2; phi itself only on request.
template <typename R>
void launch_convolve_diff(const Geo& g, const R* Q, C2<R>* S, C2<R>* S2, C2<R>* S3, const R* gz,
                          const C2<R>* tw[3], const C2<R>* dtab[3], R* dphi, R* phi, hipStream_t st) {
  const int Lx = 2 * g.grid[0], Ly = 2 * g.grid[1], Lz = 2 * g.grid[2];
  const long long nodes = (long long)g.grid[0] * g.grid[1] * g.grid[2];
  const int K = g.grid[0] + 1;
  const long long rows = (long long)g.grid[1] * g.grid[2];
#define XF(L) run_x_fwd<R, L>(g, Q, S, tw[0], st)
#define YF(L) run_y<R, L, false>(g, S, tw[1], st)
#define ZD(L)                                                                                \
  do {                                                                                       \
    const unsigned nb = line_grid<R, L>(2 * g.grid[1], K);                                   \
    if constexpr (std::is_same<R, float>::value && L == kReg1k)                              \
      k_fft_z_1k<true><<<nb, kFftThreads, 0, st>>>(g, S, gz, tw[2], S2, dtab[2]);           \
    else                                                                                     \
      k_fft_z<R, L, false, true><<<nb, kFftThreads, 0, st>>>(g, S, gz, nullptr, tw[2], S2, dtab[2]); \
  } while (0)
#define YD(L)                                                                                \
  do {                                                                                       \
    const unsigned nb = line_grid<R, L>(g.grid[2], K);                                       \
    if constexpr (std::is_same<R, float>::value && L == kReg1k) {                            \
      k_fft_y_1k<true, true><<<nb, kFftThreads, 0, st>>>(g, S, tw[1], S3, dtab[1]);          \
      k_fft_y_1k<true, false><<<nb, kFftThreads, 0, st>>>(g, S2, tw[1], nullptr, nullptr);   \
    } else {                                                                                 \
      k_fft_y<R, L, true, true><<<nb, kFftThreads, 0, st>>>(g, S, tw[1], S3, dtab[1]);       \
      k_fft_y<R, L, true, false><<<nb, kFftThreads, 0, st>>>(g, S2, tw[1]);                  \
    }                                                                                        \
  } while (0)
#define XD(L)                                                                                \
  do {                                                                                       \
    const unsigned nb = (unsigned)((rows + 2 * Cfg<R, L>::B - 1) / (2 * Cfg<R, L>::B));      \
    k_fft_x_inv<R, L><<<nb, kFftThreads, 0, st>>>(g, S, dphi, tw[0], dtab[0]);               \
    k_fft_x_inv<R, L><<<nb, kFftThreads, 0, st>>>(g, S3, dphi + nodes, tw[0]);               \
    k_fft_x_inv<R, L><<<nb, kFftThreads, 0, st>>>(g, S2, dphi + 2 * nodes, tw[0]);           \
    if (phi) k_fft_x_inv<R, L><<<nb, kFftThreads, 0, st>>>(g, S, phi, tw[0]);                \
  } while (0)
  P3M_FFT_SWITCH(Lx, XF)
  P3M_FFT_SWITCH(Ly, YF)
  P3M_FFT_SWITCH(Lz, ZD)
  P3M_FFT_SWITCH(Ly, YD)
  P3M_FFT_SWITCH(Lx, XD)
#undef XF
#undef YF
#undef ZD
#undef YD
#undef XD
}

// The potential from the spectrum S left by launch_convolve_diff (the x
// inverse of its y-inverted lines), for a caller that asks for phi later.
template <typename R>
void launch_phi_from_diff(const Geo& g, const C2<R>* S, const C2<R>* tw_x, R* phi, hipStream_t st) {
  const int Lx = 2 * g.grid[0];
  const long long rows = (long long)g.grid[1] * g.grid[2];
#define XP(L)                                                                                \
  k_fft_x_inv<R, L><<<(unsigned)((rows + 2 * Cfg<R, L>::B - 1) / (2 * Cfg<R, L>::B)), kFftThreads, 0, \
                      st>>>(g, S, phi, tw_x)
  P3M_FFT_SWITCH(Lx, XP)
#undef XP
}

// Factors e^{2 pi i k / L} - 1 = (-2 sin^2(pi k / L), sin(2 pi k / L)) for
// k = 0 .. L-1, from float64 (no cancellation in the real part).
template <typename R>
void make_diff_factors(int L, C2<R>* out) {
  for (int k = 0; k < L; ++k) {
    const double h = std::sin(M_PI * (double)k / (double)L);
    out[k] = C2<R>{(R)(-2.0 * h * h), (R)std::sin(2.0 * M_PI * (double)k / (double)L)};
  }
}

template <typename R>
void make_twiddles(int L, C2<R>* out) {
  for (int k = 0; k < L; ++k) {
    const double a = -2.0 * M_PI * (double)k / (double)L;
    out[k] = C2<R>{(R)std::cos(a), (R)std::sin(a)};
  }
}

hipError_t build_green_table(const Geo& g, double* table, double* scratch, double* const cosv[3],
                             hipStream_t st) {
  const long long total = (long long)(g.grid[0] + 1) * (g.grid[1] + 1) * (g.grid[2] + 1);
  const double scale = 1.0 / (8.0 * g.grid[0] * g.grid[1] * g.grid[2]);
  if (g.influence == kInfluenceLattice) {
    const hipError_t e = build_lattice_kernel(g, scratch, st);
    if (e != hipSuccess) return e;
  } else {
    k_green_sample<<<blocks_for(total), kThreads, 0, st>>>(g, scratch);
  }
  k_green_dct<<<blocks_for(total), kThreads, 0, st>>>(0, g, scratch, table, cosv[0], 1.0);
  k_green_dct<<<blocks_for(total), kThreads, 0, st>>>(1, g, table, scratch, cosv[1], 1.0);
  k_green_dct<<<blocks_for(total), kThreads, 0, st>>>(2, g, scratch, table, cosv[2], scale);
  if (g.influence == kInfluenceOptimal || g.influence == kInfluencePrincipal)
    k_green_influence<<<blocks_for(total), kThreads, 0, st>>>(g, g.influence, table, scale);
  return hipGetLastError();
}

size_t image_table_elems(const Geo& g) {
  return (size_t)(g.grid[0] + 1) * (g.grid[1] + 1) * (2 * (size_t)g.grid[2]);
}

void build_image_table(const Geo& g, const Place* pl, double* t1, double* t2, C2<double>* gimg,
                       const C2<double>* const tw[3], hipStream_t st) {
  const int Lx = 2 * g.grid[0], Ly = 2 * g.grid[1], Lz = 2 * g.grid[2];
  const long long K = g.grid[0] + 1, ny1 = g.grid[1] + 1;
#define GX(L)                                                                                    \
  k_gimg_x<L><<<(unsigned)((ny1 * Lz + Cfg<double, L>::B - 1) / Cfg<double, L>::B), kFftThreads, 0, \
                st>>>(g, pl, t1, tw[0])
#define GY(L)                                                                                 \
  k_gimg_y<L><<<(unsigned)(Lz * ((K + Cfg<double, L>::B - 1) / Cfg<double, L>::B)), kFftThreads, 0, \
                st>>>(g, t1, t2, tw[1])
#define GZ(L)                                                                                  \
  k_gimg_z<L><<<(unsigned)(ny1 * ((K + Cfg<double, L>::B - 1) / Cfg<double, L>::B)), kFftThreads, 0, \
                st>>>(g, t2, gimg, tw[2])
  P3M_FFT_SWITCH(Lx, GX)
  P3M_FFT_SWITCH(Ly, GY)
  P3M_FFT_SWITCH(Lz, GZ)
#undef GX
#undef GY
#undef GZ
}

template void launch_convolve<float>(const Geo&, const float*, C2<float>*, const float*, const C2<double>*,
                                     const C2<float>*[3], float*, hipStream_t);
template void launch_convolve<double>(const Geo&, const double*, C2<double>*, const double*, const C2<double>*,
                                      const C2<double>*[3], double*, hipStream_t);
template void launch_convolve_diff<float>(const Geo&, const float*, C2<float>*, C2<float>*, C2<float>*,
                                          const float*, const C2<float>* [3], const C2<float>* [3], float*,
                                          float*, hipStream_t);
template void launch_phi_from_diff<float>(const Geo&, const C2<float>*, const C2<float>*, float*, hipStream_t);
template void make_diff_factors<float>(int, C2<float>*);
template void launch_green_pack<float>(const Geo&, const double*, float*, hipStream_t);
template void launch_green_pack<double>(const Geo&, const double*, double*, hipStream_t);
template void make_twiddles<float>(int, C2<float>*);
template void make_twiddles<double>(int, C2<double>*);

}  // namespace p3m
