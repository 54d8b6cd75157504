// Host-side launchers of the libp3m kernels (internal).
#pragma once

#include "common.h"

namespace p3m {

// ---- placement and push (placement.hip) -----------------------------------
int bbox_blocks(int64_t n);
void launch_bbox(int64_t n, const double* x, double* part, int nblk, int* status, hipStream_t st);
void launch_kick_drift_bbox(int64_t n, double* x, double* p, const double* f, double dt,
                            double inv_m, double* part, int nblk, int* status, hipStream_t st);
void launch_kick(int64_t n, double* p, const double* f, double dt, hipStream_t st);
void launch_place_finalize(int nblk, const double* part, const Geo& geo, const double* place_in,
                           Place* out, double* place_out, int* status, hipStream_t st);

// ---- linked cells (sort.hip) ----------------------------------------------
struct SortBufs {
  uint32_t *keys_in, *keys, *perm;   // [n]: keys in input order; sorted keys and input index
  int* ccount;      // [ncells] particles per cell, zero between sorts
  int* cfill;       // [ncells] the scatter's fill pointers
  int* btot;        // [kCellTotals cell_blocks] particles, dense-cell and other groups per block of cells
  int* stot;        // [kCellTotals cell_supers] their sums per super-block
  int* cell_start;  // [ncells + 1]
  int* counter;     // [0] PP groups of dense cells, [1] other PP groups
};
constexpr int kCellTotals = 3;
int cell_blocks(long long ncells);
int cell_supers(long long ncells);
// Counting sort of the particles by PP cell: keys, cell starts and the PP
// work groups (desc of pp_group_bound(n, geo) entries, counter[0..1]); on
// return *keys/*perm point at the sorted key and input index arrays.
void launch_cell_sort(int64_t n, const double* x, const Place* pl, const Geo& geo, SortBufs& b, int2* desc,
                      uint32_t** keys, uint32_t** perm, hipStream_t st);
// Stepping in cell order: the reorder can also move the particle state into
// the new order (x_out NULL: x and p are not moved; id_out NULL: neither are
// the caller indices and weights).
struct Carry {
  double* x_out = nullptr;           // x[perm[j]]
  const double* p_in = nullptr;      // momenta, in the order of x
  double* p_out = nullptr;           // p_in[perm[j]]
  const uint32_t* id_in = nullptr;   // caller index of each particle of x (NULL: the identity)
  uint32_t* id_out = nullptr;        // id_in[perm[j]]
  double* qw_out = nullptr;          // qw[perm[j]] (when qw is given)
};
template <typename R>
void launch_reorder(int64_t n, const double* x, const double* qw, const uint32_t* perm,
                    const uint32_t* keys, const Place* pl, const Geo& geo, PPPos<R>* pp,
                    MeshRec<R>* mesh, int* status, const Carry& carry, hipStream_t st);
// Back to caller order: x[id[j]] = xs[j], p[id[j]] = ps[j], f[id[j]] = fs[j].
void launch_unpermute(int64_t n, const double* xs, const double* ps, const double* fs, const uint32_t* id,
                      double* x, double* p, double* f, hipStream_t st);
template <typename R>
void launch_sort_vector(int64_t n, const double* v, const uint32_t* perm, R* out, hipStream_t st);

// ---- pair forces (pp.hip) ------------------------------------------------
// Upper bound of the number of PP work groups (runs of <= kGroupRun particles of one cell).
int pp_group_bound(int64_t n, const Geo& geo);
// wclock (may be null; profiling): each wave of the force kernel (no
// energy) writes its start and end on the 100 MHz real-time clock at
// [2 w], [2 w + 1], w its wave index (fewer than pp_blocks(n, geo)).
unsigned pp_blocks(int64_t n, const Geo& geo);
template <typename R>
void launch_pp(int64_t n, const PPPos<R>* rec, const uint32_t* keys, const int* cell_start,
               const Geo& geo, const int2* desc, int* counter, PPRec<R>* out, double* energy,
               hipStream_t st, unsigned long long* wclock = nullptr);
template <typename R>
void launch_pp_hvp(int64_t n, const PPPos<R>* rec, const uint32_t* keys,
                   const int* cell_start, const Geo& geo, const int2* desc, int* counter,
                   const double* v_sorted, double* out_sorted, hipStream_t st);

// ---- mesh assignment (mesh.hip) --------------------------------------------
// Deposit into a mesh of type M (float or double) from records of type R in
// PP-cell order; clears Q first.
template <typename R, typename M>
void launch_deposit(int64_t n, const PPPos<R>* pp, const MeshRec<R>* mesh, const Geo& geo, M* Q,
                    hipStream_t st);
// Gather modes: write the total force, the two parts, or (step) total + half kick.
struct GatherOut {
  double* f;        // total, caller order (may be NULL)
  double* f_pp;     // PP part, caller order (may be NULL)
  double* f_pm;     // PM part, caller order (may be NULL)
  double* p;        // momenta to kick by half_dt * f (may be NULL)
  double half_dt;
  bool sorted = false;   // all of the above in cell order instead of caller order
  // State moved into the sorted order (sorted outputs only): with p_src, p
  // = p_src[perm[j]] + half_dt f, and x (when given) = x_src[perm[j]] (x
  // in place when x_src is NULL). Fused push (part given): x also drifts by
  // dt_over_m p, and the block partials of the new bounding box go to part
  // ([6][gather_blocks(n)]); a non-finite position sets the status bit.
  const double* p_src = nullptr;
  const double* x_src = nullptr;
  double* x = nullptr;
  double dt_over_m = 0.0;
  double* part = nullptr;
  int* status = nullptr;
};
// Blocks of the gather launch (the column count of its box partials).
int gather_blocks(int64_t n);
template <typename R, typename M>
void launch_gather(int64_t n, const PPPos<R>* pp, const MeshRec<R>* mesh, const PPRec<R>* fpp,
                   const uint32_t* perm, const Geo& geo, const Place* pl, const M* phi,
                   GatherOut out, double* energy, hipStream_t st);
void launch_deposit_grad(int64_t n, const PPRec<double>* pp, const MeshRec<double>* mesh,
                         const double* v_sorted, const Geo& geo, double* R, hipStream_t st);
void launch_gather_hvp(int64_t n, const PPRec<double>* pp, const MeshRec<double>* mesh,
                       const double* hpp_sorted, const double* v_sorted, const uint32_t* perm,
                       const Geo& geo, const Place* pl, const double* phi, const double* psi,
                       double* out, hipStream_t st);
template <typename R>
void launch_mesh_export(const Geo& geo, const R* src, const Place* pl, int scale_phi, double* out,
                        hipStream_t st);

// ---- open-boundary convolution (fft.hip) ------------------------------------
bool fft_supported(int nodes);
// Spectrum buffer: complex, grid[2] x 2 grid[1] x (grid[0] + 1).
size_t spectrum_elems(const Geo& geo);
// Elements of the z pass's padded copy of the kernel table, and its build.
size_t green_pack_elems(const Geo& geo);
template <typename R>
void launch_green_pack(const Geo& geo, const double* ghat, R* gz, hipStream_t st);
// phi = G (x) Q on the mesh (internal units); with gimg (the image table of a
// grounded plane) minus the image term.
template <typename R>
void launch_convolve(const Geo& geo, const R* Q, C2<R>* spec, const R* gz, const C2<double>* gimg,
                     const C2<R>* tw[3], R* phi, hipStream_t st);
// Difference form of the convolution (float meshes): the three forward
// differences of phi, dphi[d * nodes + m] = phi_{m+e_d} - phi_m (m_d < N_d - 1
// meaningful), from the spectrum times (e^{2 pi i k_d / L_d} - 1); S2 and S3
// are two more spectrum buffers; dtab[d] the factors of make_diff_factors
// (2 grid[d] entries); phi (may be null) the potential as well. S is left
// holding the y-inverted lines, from which launch_phi_from_diff gives phi.
template <typename R>
void launch_convolve_diff(const Geo& geo, const R* Q, C2<R>* S, C2<R>* S2, C2<R>* S3, const R* gz,
                          const C2<R>* tw[3], const C2<R>* dtab[3], R* dphi, R* phi, hipStream_t st);
template <typename R>
void launch_phi_from_diff(const Geo& geo, const C2<R>* S, const C2<R>* tw_x, R* phi, hipStream_t st);
template <typename R>
void make_diff_factors(int L, C2<R>* host_out);
// Image table of the grounded plane z = geo.zc for the placement *pl:
// complex, [2 grid[2]][grid[1] + 1][grid[0] + 1]; t1, t2 float64 scratch of
// image_table_elems each; tw float64 twiddles of the three doubled lengths.
size_t image_table_elems(const Geo& geo);
void build_image_table(const Geo& geo, const Place* pl, double* t1, double* t2, C2<double>* gimg,
                       const C2<double>* const tw[3], hipStream_t st);
template <typename R>
void make_twiddles(int L, C2<R>* host_out);
// Fourier transform of the sampled kernel erf(kappa rho)/rho on the doubled
// mesh, divided by the number of doubled-mesh nodes: (grid+1)^3 float64
// octant [kz][ky][kx]. scratch holds 2 (grid+1)^3 doubles.
// Lattice-form kernel on the octant of offsets into out (float64, internal units).
hipError_t build_lattice_kernel(const Geo& geo, double* out, hipStream_t st);
hipError_t build_green_table(const Geo& geo, double* table, double* scratch, double* const cosv[3],
                       hipStream_t st);

// ---- reductions (diag.hip) ------------------------------------------------
// acc[0..15] += first moments (mode 0) or centred second moments about the
// means held in acc[16..] (mode 1); see diag.hip for the layout.
void launch_moments(int64_t n, const double* x, const double* p, const double* qw, double* acc,
                    int mode, hipStream_t st);
void launch_fill(void* ptr, size_t bytes, hipStream_t st);

}  // namespace p3m
