// Mesh kernel of the lattice form (p3m_opts.influence = P3M_INFLUENCE_LATTICE),
// float64, on the octant of node offsets 0 <= n_d <= N_d, in internal units
// (spacings hu, screening kappa): the free-space Green's function of the
// 7-point discrete Laplacian L = -sum_d D_d / h_d^2 (the second differences of
// Sec. 2.4.2, eq. 1d_ddiff, summed as in eq. 3dim_second_order_fin_diff_tensor;
// the lattice Green's function of Sec. 3, eq. def_G_L), normalised so that
// L G = delta / (h_x h_y h_z), convolved with the Gaussian screening charge
// per cell g = prod_d g_d, g_d(m) = [erf(a (m+1/2) h_d) - erf(a (m-1/2) h_d)]/2,
// and scaled by 4 pi: K -> 1/rho far away, like the sampled erf(kappa rho)/rho.
//
// With 1/L = int_0^inf exp(-t L) dt the kernel separates per axis:
//   K(n) = (4 pi / V) int_0^inf prod_d F_d(n_d, t) dt,
//   F_d(n, t) = (1/pi) int_0^pi ghat_d(theta) exp(-4 (t / h_d^2) sin^2(theta/2)) cos(n theta) dtheta,
// ghat_d(theta) = g_d(0) + 2 sum_m g_d(m) cos(m theta). The theta integral is
// Gauss-Legendre on [0, theta_max], theta_max = min(pi, 14 / sqrt(2 t / h_d^2))
// (past it the integrand is below e^-98 of its peak). The t integral is the
// trapezoid rule in ln t (step <= 1/4) over [1e-14 h_min^2, 1e10 h_max^2],
// with the Gaussian asymptote of each factor,
//   A_d(n, t) = h_d exp(-(n h_d)^2 / (4 (t + c))) / sqrt(4 pi (t + c)),  c = h_max^2,
// subtracted under the integral, so the integrand decays at both ends, and
// its exact integral erf(rho / (2 sqrt(c))) / rho added back.
#include <algorithm>
#include <cmath>
#include <vector>

#include "launch.h"

namespace p3m {

namespace {

constexpr double kTauLo = 1e-14;   // lower end of t, units of h_min^2
constexpr double kTauHi = 1e10;    // upper end of t, units of h_max^2
constexpr double kMaxStepLn = 0.25;
constexpr double kThetaCut = 14.0;
constexpr double kCellTol = 1e-18;
constexpr int kMaxCells = 256;

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_J.
void gauss_legendre(int J, std::vector<double>& x, std::vector<double>& w) {
  x.assign(J, 0.0);
  w.assign(J, 0.0);
  for (int i = 0; i < (J + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (J + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= J; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = J * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= J; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = J * (z * p1 - p0) / (z * z - 1.0);
    x[i] = -z;
    x[J - 1 - i] = z;
    w[i] = w[J - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Screening charge per cell along one axis, m = 0..M (the tail through erfc);
// empty if the cloud spans more than kMaxCells cells.
std::vector<double> cell_weights(double h, double a) {
  std::vector<double> g;
  g.push_back(std::erf(0.5 * a * h));
  for (int m = 1; m < kMaxCells; ++m) {
    const double v = 0.5 * (std::erfc(a * (m - 0.5) * h) - std::erfc(a * (m + 0.5) * h));
    g.push_back(v);
    if (v < kCellTol) return g;
  }
  return {};
}

struct AxisTab {
  int n1;              // N_d + 1 offsets
  int J;               // Gauss-Legendre nodes
  int M;               // cell weights g(0..M)
  double h;
  const double* glx;   // [J]
  const double* glw;   // [J]
  const double* g;     // [M + 1]
  double* F;           // [nt][n1]
  double* A;           // [nt][n1]
};
struct LatticeArgs {
  AxisTab ax[3];
  const double* tau;   // [nt]
  const double* wt;    // [nt] trapezoid weight in ln t, times t
  double c;
};

// One block per (t node, axis): the quadrature weights of the theta integral
// in LDS, then F_d(n, t) and A_d(n, t) for every offset n. The t weight is
// folded into axis 0.
__global__ void __launch_bounds__(256) k_lattice_factor(LatticeArgs args) {
  extern __shared__ double lds[];
  const int t = blockIdx.x, d = blockIdx.y;
  const AxisTab& T = args.ax[d];
  double* th = lds;
  double* cw = lds + T.J;
  const double tau = args.tau[t];
  const double z = 2.0 * tau / (T.h * T.h);
  const double tmax = fmin(M_PI, kThetaCut / sqrt(z));
  for (int j = threadIdx.x; j < T.J; j += blockDim.x) {
    const double theta = 0.5 * tmax * (T.glx[j] + 1.0);
    double gh = T.g[0];
    for (int m = 1; m <= T.M; ++m) gh += 2.0 * T.g[m] * cos(m * theta);
    const double sh = sin(0.5 * theta);
    th[j] = theta;
    cw[j] = 0.5 * tmax * T.glw[j] * gh * exp(-2.0 * z * sh * sh) * (1.0 / M_PI);
  }
  __syncthreads();
  const double scale = d == 0 ? args.wt[t] : 1.0;
  const double tc = tau + args.c;
  const double an = T.h / sqrt(4.0 * M_PI * tc);
  for (int n = threadIdx.x; n < T.n1; n += blockDim.x) {
    double f = 0.0;
    for (int j = 0; j < T.J; ++j) f += cw[j] * cos(n * th[j]);
    const double x = n * T.h;
    T.F[(size_t)t * T.n1 + n] = scale * f;
    T.A[(size_t)t * T.n1 + n] = scale * an * exp(-x * x / (4.0 * tc));
  }
}

// One thread per octant entry: the t sum of the factor products minus the
// asymptote's, plus the asymptote's exact integral.
__global__ void __launch_bounds__(256) k_lattice_sum(LatticeArgs args, int nt, double* __restrict__ out) {
  const int nx1 = args.ax[0].n1, ny1 = args.ax[1].n1, nz1 = args.ax[2].n1;
  const long long total = (long long)nx1 * ny1 * nz1;
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int ix = (int)(e % nx1), iy = (int)((e / nx1) % ny1), iz = (int)(e / ((long long)nx1 * ny1));
  double acc = 0.0;
  for (int t = 0; t < nt; ++t) {
    const double f = args.ax[0].F[(size_t)t * nx1 + ix] * args.ax[1].F[(size_t)t * ny1 + iy] *
                     args.ax[2].F[(size_t)t * nz1 + iz];
    const double a = args.ax[0].A[(size_t)t * nx1 + ix] * args.ax[1].A[(size_t)t * ny1 + iy] *
                     args.ax[2].A[(size_t)t * nz1 + iz];
    acc += f - a;
  }
  const double V = args.ax[0].h * args.ax[1].h * args.ax[2].h;
  const double rx = ix * args.ax[0].h, ry = iy * args.ax[1].h, rz = iz * args.ax[2].h;
  const double rho = sqrt(rx * rx + ry * ry + rz * rz);
  const double sc = 2.0 * sqrt(args.c);
  const double tail = rho > 0.0 ? erf(rho / sc) / rho : 1.0 / sqrt(M_PI * args.c);
  out[e] = 4.0 * M_PI / V * acc + tail;
}

}  // namespace

hipError_t build_lattice_kernel(const Geo& geo, double* out, hipStream_t st) {
  double hmin = geo.hu[0], hmax = geo.hu[0];
  for (int d = 1; d < 3; ++d) {
    hmin = std::min(hmin, geo.hu[d]);
    hmax = std::max(hmax, geo.hu[d]);
  }
  const double ulo = std::log(kTauLo * hmin * hmin), uhi = std::log(kTauHi * hmax * hmax);
  const int nt = (int)std::ceil((uhi - ulo) / kMaxStepLn) + 1;
  const double du = (uhi - ulo) / (nt - 1);
  std::vector<double> tau(nt), wt(nt);
  for (int t = 0; t < nt; ++t) {
    tau[t] = std::exp(ulo + du * t);
    wt[t] = (t == 0 || t == nt - 1 ? 0.5 * du : du) * tau[t];
  }
  // host tables: per axis GL nodes, weights and cell weights; sizes of F, A
  std::vector<double> host;
  size_t off_glx[3], off_glw[3], off_g[3], off_F[3], off_A[3];
  int J[3], M[3], jmax = 0;
  std::vector<double> gx, gw;
  for (int d = 0; d < 3; ++d) {
    const std::vector<double> g = cell_weights(geo.hu[d], geo.kappa);
    if (g.empty()) return hipErrorInvalidValue;
    M[d] = (int)g.size() - 1;
    J[d] = 2 * (geo.grid[d] + M[d]) + 64;
    jmax = std::max(jmax, J[d]);
    gauss_legendre(J[d], gx, gw);
    off_glx[d] = host.size();
    host.insert(host.end(), gx.begin(), gx.end());
    off_glw[d] = host.size();
    host.insert(host.end(), gw.begin(), gw.end());
    off_g[d] = host.size();
    host.insert(host.end(), g.begin(), g.end());
  }
  const size_t off_tau = host.size();
  host.insert(host.end(), tau.begin(), tau.end());
  const size_t off_wt = host.size();
  host.insert(host.end(), wt.begin(), wt.end());
  size_t total = host.size();
  for (int d = 0; d < 3; ++d) {
    off_F[d] = total;
    total += (size_t)nt * (geo.grid[d] + 1);
    off_A[d] = total;
    total += (size_t)nt * (geo.grid[d] + 1);
  }
  const size_t lds = 2 * (size_t)jmax * sizeof(double);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  double* buf = nullptr;
  hipError_t e = hipMalloc(&buf, total * sizeof(double));
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(buf, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, st);
  LatticeArgs args{};
  for (int d = 0; d < 3; ++d) {
    AxisTab& T = args.ax[d];
    T.n1 = geo.grid[d] + 1;
    T.J = J[d];
    T.M = M[d];
    T.h = geo.hu[d];
    T.glx = buf + off_glx[d];
    T.glw = buf + off_glw[d];
    T.g = buf + off_g[d];
    T.F = buf + off_F[d];
    T.A = buf + off_A[d];
  }
  args.tau = buf + off_tau;
  args.wt = buf + off_wt;
  args.c = hmax * hmax;
  if (e == hipSuccess) {
    k_lattice_factor<<<dim3(nt, 3), 256, lds, st>>>(args);
    const long long oct = (long long)(geo.grid[0] + 1) * (geo.grid[1] + 1) * (geo.grid[2] + 1);
    k_lattice_sum<<<(unsigned)((oct + 255) / 256), 256, 0, st>>>(args, nt, out);
    e = hipGetLastError();
  }
  // the host vector and the device tables must outlive the launches
  const hipError_t es = hipStreamSynchronize(st);
  const hipError_t ef = hipFree(buf);
  return e != hipSuccess ? e : (es != hipSuccess ? es : ef);
}

}  // namespace p3m
