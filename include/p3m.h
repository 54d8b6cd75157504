/*
 * p3m.h -- C ABI of the MI355X P3M space-charge library (libp3m.so).
 *
 * The library evaluates the P3M force of Wyssling & Adelmann (arXiv
 * 2103.02046) on a bunch of equal-mass macro-particles and advances it with
 * the leapfrog integrator, all in hand-written HIP kernels for gfx950:
 *
 *   F_i = F_i^PP + F_i^PM                              (Sec. 2.5, eq. eom_p3m_coord)
 *   F_i^PP = sum_{j != i, r_ij < r_c'} k_e q^2 w_i w_j
 *            [erfc(a' r)/r + (2a'/sqrt(pi)) e^{-a'^2 r^2}] (x_i - x_j)/r^2
 *                                       (Sec. 1, eq. summation_short with the
 *                                        erfc part of eq. ewald_split, Sec. 2.2)
 *   Q_m    = sum_i w_i prod_d b_p(u_{i,d} - m_d)     (Sec. 2.4.2, B-spline assignment,
 *                                                      eq. interpolation_splines_b0)
 *   phi_m  = sum_m' G(m - m') Q_m',  G = erf(a' r)/r sampled on the mesh,
 *            aperiodic (open boundaries by zero padding to a doubled mesh)
 *                                       (Sec. 3, eq. phi_L with eq. free_gf)
 *   F_i^PM = -k_e q^2 w_i sum_m phi_m grad b(u_i - m) (Sec. 2.5, eq. eom_p3m_coord)
 *   leapfrog (kick-drift-kick)          (Sec. 2.4.3, eq. leapfrog)
 *
 * Placement: every evaluation centres the mesh (nodes x0 + k h') on the
 * bounding box of the positions. When the box is wider than the nodes an
 * assignment stencil may use (grid-1 for CIC, grid-2 for TSC), a common zoom
 * s >= 1 scales h' = s h and r_c' = s r_c and divides the split parameter,
 * a' = a / s (with zoom disabled this is the P3M_EDOMAIN error instead).
 *
 * Conventions for every call:
 *   - particle arrays are DEVICE pointers, row-major [n][3] float64, in the
 *     caller's particle order, owned by the caller; the library never keeps
 *     them after the call returns;
 *   - `stream` is a hipStream_t (NULL = the default stream); all work is
 *     enqueued on it and calls return without synchronising unless stated;
 *     one context must be used by one stream at a time;
 *   - errors in the arguments are returned at once; errors that depend on
 *     the data (non-finite or out-of-mesh positions) are raised in a device
 *     status word and returned by the next p3m_status_sync;
 *   - p3m_last_error gives a message for the last failing call.
 */
#ifndef P3M_H
#define P3M_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct p3m_ctx p3m_ctx;
typedef int32_t p3m_status;

#define P3M_OK          0
#define P3M_EINVAL     (-1)   /* bad argument                                   */
#define P3M_ENOMEM     (-2)   /* device allocation failed                       */
#define P3M_EHIP       (-3)   /* a HIP runtime call failed                      */
#define P3M_ESTATE     (-4)   /* call not valid in the context's state          */
#define P3M_EDOMAIN    (-5)   /* a particle left the mesh with zoom disabled    */
#define P3M_ENONFINITE (-6)   /* a position was NaN or infinite                 */

#define P3M_FP64   0          /* every stage in float64                         */
#define P3M_FP32C  1          /* pair forces and FFT in float32 with Kahan-     */
                              /* compensated pair sums; float64 Green's table,  */
                              /* positions, momenta and reductions              */

/* Mesh precision of the P3M_FP32C form (the P3M_FP64 form is float64
 * throughout). The mesh force is a difference of node potentials, so a
 * float32 potential carries a relative force error of about 6e-8 times the
 * bunch extent in cells: below 1e-5 up to ~150 cells. On a float32 mesh
 * with an axis of more than P3M_MESH_AUTO_F32_MAX nodes the transform
 * therefore delivers the three forward differences phi_{m+e_d} - phi_m
 * instead of phi (the spectrum times e^{2 pi i k_d / L_d} - 1), and the
 * gather uses the B-spline identity b_p' (t) = b_{p-1}(t + 1/2) -
 * b_{p-1}(t - 1/2): the same force, with rounding relative to the
 * differences (the "difference form"; the variational gather in free space).
 * AUTO: float32 (in the difference form above P3M_MESH_AUTO_F32_MAX nodes);
 * float64 above that size for the momentum-conserving gather or the
 * grounded plane. F32 forces float32 (the difference form where it
 * applies), F64 float64 (charge, transform and potential; pair forces stay
 * float32). p3m_info reports the mesh precision in use. */
#define P3M_MESH_AUTO 0
#define P3M_MESH_F32  1
#define P3M_MESH_F64  2
#define P3M_MESH_AUTO_F32_MAX 128

/* Mesh force at the particles (p3m_opts.gather).
 * VARIATIONAL: F_i = -w_i sum_m phi_m grad W_m(x_i), minus the gradient of
 *   the discrete energy (Sec. 2.5, eq. eom_p3m_coord, first term).
 * MOMENTUM: the mesh field by central differences,
 *   E_m = -(phi_{m+e_d} - phi_{m-e_d}) / (2 h_d), interpolated with the
 *   assignment weights, F_i = w_i sum_m W_m(x_i) E_m: a reading of the
 *   remark after that equation (the weight gradient as a finite difference
 *   of the potential). The total mesh force and the self-force vanish; the
 *   force is not the gradient of an energy. The placement keeps every
 *   stencil off the outer node layer (usable span 2 nodes shorter). */
#define P3M_GATHER_VARIATIONAL 0
#define P3M_GATHER_MOMENTUM    1

/* Boundary of the long-range (mesh) problem (p3m_opts.boundary).
 * OPEN: free space (Sec. 2.1, eq. free_gf), by zero padding.
 * CATHODE: a grounded plane z = cathode_z (Sec. 3.1): the mesh kernel of
 *   every node charge is taken together with that of its mirror image of
 *   opposite sign (eq. GreenFunc_planar_cathode, mirror map eq.
 *   symmetry_planar_cathode), computed with the shifted Green's function of
 *   that section so the gap to the images is never meshed. The pair (PP)
 *   part stays free-space, as in the section's scheme: a particle closer
 *   than r_c/2 to the plane misses the short-range part of its images. The
 *   bunch is assumed on one side of the plane. Costs one extra table build
 *   (three float64 FFT passes) per evaluation. */
#define P3M_BOUNDARY_OPEN    0
#define P3M_BOUNDARY_CATHODE 1

/* Fourier table of the mesh kernel (p3m_opts.influence), built at create.
 * SAMPLED: erf(a r)/r sampled at the node offsets, no deconvolution.
 * OPTIMAL: the optimal influence function of Sec. 3.1.2 (eq. Ghfinal) for
 *   point particles, sum_m U^2(k_m) (R gamma)(k_m) / [sum_m U^2(k_m)]^2 with
 *   U the B-spline's transform and |m_d| <= 2, which minimises the mean
 *   square error of the mesh potential; PRINCIPAL: its m = 0 form
 *   (R gamma)/U^2. Either enters as (G - R gamma)/V added to the sampled
 *   kernel's table, which changes the kernel near the origin only and keeps
 *   the open boundary. Lowers the potential error for CIC and TSC and the
 *   force error for TSC. Free space only (P3M_EINVAL with the cathode). */
#define P3M_INFLUENCE_SAMPLED   0
#define P3M_INFLUENCE_OPTIMAL   1
#define P3M_INFLUENCE_PRINCIPAL 2
/* LATTICE: the paper's literal discrete field equation. The mesh potential
 * solves the 7-point discrete Poisson equation of the free lattice: the
 * second differences D_d of Sec. 2.4.2 (eq. 1d_ddiff), divided by h_d^2 and
 * summed as in eq. 3dim_second_order_fin_diff_tensor, with the Green's
 * function of Sec. 3 (eq. def_G_L). The source is the deposited charge
 * convolved with the Gaussian screening's charge per cell,
 * [erf(a (m+1/2) h) - erf(a (m-1/2) h)]/2 per axis. The kernel tends to
 * erf(a r)/r at second order in a h, and to 1/r far away. Built at create
 * from a one-dimensional integral representation of the lattice Green's
 * function, to about 1e-13. Free space only. P3M_EINVAL when the screening
 * cloud spans more than 256 cells. */
#define P3M_INFLUENCE_LATTICE   3

#define P3M_CIC 1             /* linear B-spline b1 (2 nodes per axis)          */
#define P3M_TSC 2             /* quadratic B-spline b2 (3 nodes per axis)       */

/* Placement record of one evaluation: x0[3] (position of mesh node 0, m) and
 * the zoom s. Used to record placements in a forward run and replay them. */
#define P3M_PLACEMENT_DOUBLES 4

typedef struct {
    int32_t order;      /* P3M_CIC or P3M_TSC                               [TSC]  */
    int32_t precision;  /* P3M_FP64 or P3M_FP32C                            [FP64] */
    int32_t zoom;       /* 1: zoom the mesh to fit the bunch; 0: EDOMAIN    [1]    */
    int32_t gather;     /* P3M_GATHER_VARIATIONAL or _MOMENTUM     [VARIATIONAL]  */
    int32_t mesh_precision; /* P3M_MESH_AUTO, _F32 or _F64 (P3M_FP32C only) [AUTO] */
    int32_t pp_cell_div; /* PP cells per cutoff along each axis: 1 (edge >= r_c,
                            27 neighbour cells) or 2 (edge >= r_c/2, 125 half-size
                            cells: 125/8 instead of 27 cutoff cubes of candidates
                            per particle, for dense bunches); 0 means 1       [0]  */
    double ke;          /* Coulomb constant 1/(4 pi eps0)     [8.9875517923e9]    */
    double q;           /* macro-particle charge, C                        [1.0]  */
    double m;           /* macro-particle mass, kg                         [1.0]  */
    int32_t boundary;   /* P3M_BOUNDARY_OPEN or _CATHODE                   [OPEN] */
    int32_t influence;  /* P3M_INFLUENCE_SAMPLED, _OPTIMAL, _PRINCIPAL or _LATTICE [SAMPLED] */
    double cathode_z;   /* plane position for P3M_BOUNDARY_CATHODE, m       [0.0]  */
} p3m_opts;

/* Fill *opts with the defaults shown in brackets above. */
p3m_status p3m_default_opts(p3m_opts *opts);

/*
 * Create a context for a grid[0] x grid[1] x grid[2] vertex mesh with spacing
 * h[3] (m), PP cutoff r_cut (m) and Ewald split parameter `split` (1/m; 0
 * means the whole Coulomb force is summed pairwise inside r_cut and the mesh
 * part vanishes). Grid sizes must be powers of two in [4, 1024].
 * Builds the Fourier transform of the sampled erf(a r)/r kernel on the
 * doubled mesh in float64 (once; zoom rescales it exactly by 1/s).
 * *out receives the context; the caller frees it with p3m_destroy.
 * Errors: P3M_EINVAL (sizes, non-positive h or r_cut, negative split, bad
 * opts), P3M_ENOMEM, P3M_EHIP.
 */
p3m_status p3m_create(p3m_ctx **out, const int32_t grid[3], const double h[3],
                      double r_cut, double split, const p3m_opts *opts);

/*
 * Total P3M force on n particles at positions x[n][3] (device, m).
 * qw[n] (device, may be NULL = all 1) are dimensionless charge weights: the
 * charge of particle i is q * qw[i]. Writes f[n][3] (device, N) in caller
 * order. n may be 0 (no work). Device buffers grow on demand (this call may
 * allocate when n exceeds every earlier n).
 * Errors: P3M_EINVAL (n < 0, NULL x or f), P3M_ENOMEM, P3M_EHIP; data
 * errors via p3m_status_sync.
 */
p3m_status p3m_forces(p3m_ctx *ctx, int64_t n, const double *x, const double *qw,
                      double *f, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * force as p3m_forces, computed by the same kernels, with every per-call
 * work buffer (cell keys, permutation, PP work groups, particle records,
 * pair forces) in a static device array of P3M_NOALLOC_SCRATCH_BYTES per GPU
 * instead of context buffers; the mesh buffers are the context's, allocated
 * by p3m_create. This call allocates and frees nothing. The work buffers
 * take 12 bytes per particle plus 48 (P3M_FP32C) or 96 (P3M_FP64) for the
 * records and 8 per PP work group (n/16 plus the PP cells); above the array
 * the call returns P3M_EINVAL (about 1.1 million particles in P3M_FP32C on a
 * 128^3 mesh, 0.6 million in P3M_FP64). The array is shared by every call on
 * one GPU, whatever the context or stream, and keeps the last call's
 * contents (every call overwrites what it reads): calls that overlap on one
 * GPU race. Each GPU the library runs on holds its array until the process
 * ends. Errors as p3m_forces (no P3M_ENOMEM).
 */
#define P3M_NOALLOC_SCRATCH_BYTES (64u << 20)
p3m_status p3m_forces_noalloc(p3m_ctx *ctx, int64_t n, const double *x, const double *qw,
                              double *f, void *stream);

/*
 * As p3m_forces, with the two parts written separately (either may be NULL)
 * and an optional fixed placement: if place_in (device, P3M_PLACEMENT_DOUBLES
 * float64) is not NULL the mesh is placed there instead of on the bounding
 * box; if place_out (device) is not NULL the placement used is written there.
 */
p3m_status p3m_forces_ex(p3m_ctx *ctx, int64_t n, const double *x, const double *qw,
                         double *f_pp, double *f_pm, const double *place_in,
                         double *place_out, void *stream);

/*
 * Advance (x, p) (device [n][3] float64, m and kg m/s, updated in place) by
 * nsteps kick-drift-kick leapfrog steps of dt seconds:
 *   p += dt/2 F(x);  x += dt p / m;  p += dt/2 F(x).
 * The force at the starting x is evaluated first unless `reuse_force` is 1
 * and the previous p3m_step on this context ended at this same x (the
 * context caches that force; any other call clears the cache).
 * If place_replay (device) is not NULL it holds (nsteps+1) placement
 * records used instead of the bounding-box placement: record 0 for the start
 * position, record k for the end of step k (a recorded run replayed exactly).
 * With reuse_force, record 0 is not read (the cached force stands for it).
 * If place_record (device) is not NULL it receives the (nsteps+1) placements
 * used, in the same order; it needs a fresh start force (P3M_EINVAL with
 * reuse_force).
 * Errors: as p3m_forces; P3M_ESTATE if reuse_force is asked with no cache.
 */
p3m_status p3m_step(p3m_ctx *ctx, int64_t n, double *x, double *p, const double *qw,
                    double dt, int32_t nsteps, int32_t reuse_force, const double *place_replay,
                    double *place_record, void *stream);

/*
 * Hessian-vector product of the P3M potential: out = H v, H = dF/dx at x with
 * the placement fixed at place (device, P3M_PLACEMENT_DOUBLES; NULL = the
 * bounding-box placement of x). H is symmetric because F = -grad U, so this
 * is also the vector-Jacobian product. v and out are device [n][3] float64.
 * Precision: the mesh part (the weight-gradient deposit of v, the
 * convolution and the gather with the weights' first and second derivatives)
 * runs in float64 in both forms, since its second differences of the
 * potential would lose float32's digits; the pair Jacobian runs in float64
 * (P3M_FP64) or in float32 with compensated sums (P3M_FP32C, about 1e-6 of
 * the float64 product). This is the derivative of the force at a frozen
 * placement (the placement is a function of the bounding box, which the
 * derivative does not follow), allocates the float64 mesh on first use, and
 * P3M_ESTATE with the momentum-conserving gather (its force has no potential).
 */
p3m_status p3m_hvp(p3m_ctx *ctx, int64_t n, const double *x, const double *qw,
                   const double *v, const double *place, double *out, void *stream);

/*
 * Adjoint of one leapfrog step (x_n, p_n) -> (x_np1, p_np1) of length dt
 * (Hessian-vector products of the precision described at p3m_hvp),
 * with the placements recorded in the forward run (place_n, place_np1,
 * device). Given the gradients xbar_np1, pbar_np1 of a scalar objective with
 * respect to (x_np1, p_np1), writes those with respect to (x_n, p_n):
 *   xb = xbar_np1 + dt/2 H(x_np1) pbar_np1;  pb = pbar_np1 + dt/m xb;
 *   xbar_n = xb + dt/2 H(x_n) pb;  pbar_n = pb.
 * All arrays device [n][3] float64; outputs may alias the inputs.
 * P3M_ESTATE with the momentum-conserving gather.
 */
p3m_status p3m_backward(p3m_ctx *ctx, int64_t n, const double *x_n, const double *x_np1,
                        const double *qw, const double *xbar_np1, const double *pbar_np1,
                        double *xbar_n, double *pbar_n, double dt, const double *place_n,
                        const double *place_np1, void *stream);

/*
 * Adjoint of nsteps leapfrog steps at once (the same steps as p3m_backward).
 * xs (device, [nsteps+1][n][3]) holds the positions x_0 .. x_nsteps of the
 * forward run and places (device, [nsteps+1][P3M_PLACEMENT_DOUBLES]) its
 * placements. xbar, pbar (device [n][3]) hold the gradients with respect to
 * (x_nsteps, p_nsteps) on entry and with respect to (x_0, p_0) on return.
 * The product H(x_k) pbar_k that ends the step k+1 -> k also begins the step
 * k -> k-1, so it is formed once: nsteps + 1 Hessian-vector products in all,
 * not 2 nsteps. nsteps = 0 leaves xbar, pbar unchanged.
 * P3M_EINVAL for nsteps < 0 or missing arrays; P3M_ESTATE with the
 * momentum-conserving gather.
 */
p3m_status p3m_backward_steps(p3m_ctx *ctx, int64_t n, int32_t nsteps, const double *xs,
                              const double *qw, double *xbar, double *pbar, double dt,
                              const double *places, void *stream);

typedef struct {
    double momentum[3];   /* sum_i p_i                                   kg m/s */
    double kinetic;       /* sum_i |p_i|^2 / (2m)                        J      */
    double u_pp;          /* sum_{i<j, r<r_c'} k_e q^2 w_i w_j erfc(a'r)/r  J   */
    double u_pm;          /* k_e q^2 sum_m Q_m phi_m / 2                  J      */
    double mean[3];       /* centroid                                    m      */
    double rms[3];        /* rms size per axis                           m      */
    double emit_n[3];     /* normalised rms emittance per axis, m rad:
                             sqrt(<dx^2><dp^2> - <dx dp>^2) / (m c)            */
    double zoom;          /* s of this evaluation                               */
    double charge;        /* sum_i w_i                                          */
    double pairs;         /* ordered pairs (i, j), j != i, with 0 < r < r_c'    */
} p3m_diag;

/*
 * Observables of (x, p) in float64 reductions (the energies use a fresh force
 * evaluation at x). Synchronises `stream`; *out is host memory.
 */
p3m_status p3m_diagnostics(p3m_ctx *ctx, int64_t n, const double *x, const double *p,
                           const double *qw, p3m_diag *out, void *stream);

/*
 * Copy the mesh of the last evaluation into out (device, float64,
 * [grid[2]][grid[1]][grid[0]], x fastest): which = 0 the charge Q (units of
 * q), which = 1 the potential phi (1/m; the physical potential is k_e q phi).
 */
p3m_status p3m_mesh(p3m_ctx *ctx, int32_t which, double *out, void *stream);

/* Stage timing with HIP events recorded on the calling stream around every
 * selected stage of every evaluation, for at most max_records stage launches:
 *   0 push + placement, 1 linked-cell sort and PP work groups, 2 reorder,
 *   3 PP pair forces (the pair kernel alone), 4 deposit, 5 FFT convolution
 *   (five passes), 6 gather.
 * Bit 7 instead records, for the load balance of the pair kernel, the start
 * and end of each of its waves (a wave takes up to 4 work groups of up to 16
 * particles of one cell) in every force evaluation of up to the largest n
 * evaluated before this call; p3m_profile_pp_waves returns those of the last.
 * stage_mask selects the stages (bit s for stage s; 0x7f all, nonzero). An
 * event pair costs about 2 us of idle GPU between the kernels it separates,
 * so a throughput measurement times only the stages it needs.
 * p3m_profile_end synchronises `stream`, writes the summed milliseconds and
 * the number of timed launches per stage (arrays of 8, host) and stops.
 * P3M_EINVAL for max_records < 1 or a mask outside 0x01..0xff. */
p3m_status p3m_profile_begin(p3m_ctx *ctx, int32_t max_records, int32_t stage_mask);
p3m_status p3m_profile_end(p3m_ctx *ctx, double ms[8], int64_t launches[8], void *stream);

/* The pair-kernel waves of the last force evaluation recorded under bit 7
 * of p3m_profile_begin: *count (host) receives the number of waves, out
 * (host, [cap][2]) the start and end of the first min(count, cap) waves in
 * microseconds from the earliest start (100 MHz device clock). Synchronises
 * `stream`. P3M_ESTATE if no evaluation recorded its waves. */
p3m_status p3m_profile_pp_waves(p3m_ctx *ctx, int64_t cap, double *out, int64_t *count, void *stream);

/* Synchronise `stream`, return and clear the device status word
 * (P3M_OK, P3M_EDOMAIN or P3M_ENONFINITE). */
p3m_status p3m_status_sync(p3m_ctx *ctx, void *stream);

/* Host info: out[0] the bits of the mesh arithmetic the context uses
 * (charge, transform and potential: 64, or 32 for a float32 mesh), out[1..4]
 * the PP cells (total, x, y, z), out[5..7] the padded FFT extents (x, y, z). */
p3m_status p3m_info(const p3m_ctx *ctx, int64_t out[8]);

/* Message of the last failing call on ctx (never NULL). */
const char *p3m_last_error(const p3m_ctx *ctx);

/* Free the context and every device buffer it owns. NULL is a no-op. */
void p3m_destroy(p3m_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* P3M_H */
