// C ABI of libp3m: context, device buffers and the order of the kernels of
// one P3M force evaluation, leapfrog step and adjoint step.
//
//   placement (bbox) -> cell keys -> counting sort by cell (cell starts and
//   PP work groups) -> reorder -> PP pair forces -> deposit -> FFT
//   convolution -> gather (+ kick, state move and the next drift)
//
// Everything is enqueued on the caller's stream; the host never waits for
// the device inside p3m_forces / p3m_step / p3m_hvp / p3m_backward(_steps).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "p3m.h"
#include "launch.h"

using namespace p3m;

namespace {

constexpr double kCLight = 299792458.0;

template <typename R>
struct Engine {
  // per-particle
  PPPos<R>* pp = nullptr;
  MeshRec<R>* mesh = nullptr;
  PPRec<R>* fpp = nullptr;
  // mesh
  R* Q = nullptr;
  R* phi = nullptr;
  C2<R>* spec = nullptr;
  R* gz = nullptr;              // kernel table in this precision, padded rows (z pass)
  C2<R>* tw[3] = {nullptr, nullptr, nullptr};
  // difference form of a float mesh: two more spectra, the three difference
  // meshes and the difference factors per axis
  C2<R>* spec2 = nullptr;
  C2<R>* spec3 = nullptr;
  R* dphi = nullptr;
  C2<R>* dtab[3] = {nullptr, nullptr, nullptr};
  bool phi_current = false;     // phi holds the potential of the last evaluation
  int64_t cap = 0;
  bool mesh_ready = false;
};

}  // namespace

struct p3m_ctx {
  Geo geo{};
  p3m_opts opts{};
  std::string err;
  int64_t cap = 0;
  // sort
  SortBufs sb{};
  int2* groups = nullptr;       // PP work groups
  int sort_nb_cap = 0;
  // placement, status, small scratch
  Place* place = nullptr;
  int* status = nullptr;
  double* bbox_part = nullptr;  // [6][bbox_slots] bounding-box partials
  int bbox_slots = 1024;
  double* acc = nullptr;        // 64 doubles of reduction scratch
  double* ghat = nullptr;
  // grounded plane: image table (rebuilt per evaluation), scratch, twiddles
  C2<double>* gimg = nullptr;
  double *gimg_t1 = nullptr, *gimg_t2 = nullptr;
  C2<double>* tw64[3] = {nullptr, nullptr, nullptr};
  // step
  double* fcache = nullptr;     // [cap][3]
  // state stepped in cell order (double-buffered), its caller indices, and
  // the force in that order
  double *xs[2] = {nullptr, nullptr}, *ps[2] = {nullptr, nullptr}, *qs[2] = {nullptr, nullptr};
  uint32_t* ids[2] = {nullptr, nullptr};
  double* fs = nullptr;
  bool force_cached = false;
  const double* cached_x = nullptr;
  int64_t cached_n = -1;
  // adjoint scratch (float64)
  double *v_sorted = nullptr, *hpp = nullptr, *hv = nullptr, *xb = nullptr, *pb = nullptr;
  double *Rm = nullptr, *psi = nullptr;
  Engine<float> e32;
  Engine<double> e64;
  uint32_t* keys = nullptr;     // sorted keys of the last evaluation
  uint32_t* perm = nullptr;     // sorted -> caller index of the last evaluation
  int device = 0;               // the GPU the context's buffers live on
  int last_precision = -1;      // mesh precision of the last evaluation
  bool mesh64 = false;          // float32 particle path with a float64 mesh
  // stage timing
  bool prof_on = false;
  int prof_mask = 0;            // stages timed (bit s: stage s); bit 7: pair-kernel wave clocks
  unsigned long long* wclock = nullptr;   // [2 wclock_cap] start/end of each pair-kernel wave
  int64_t wclock_cap = 0;
  bool wclock_valid = false;    // the last evaluation recorded its pair kernel's waves
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_stage;
  int prof_next = 0;
};

// Work buffers of p3m_forces_noalloc: one static array per GPU (each device
// holds its own copy of a __device__ variable), found on the host through
// hipGetSymbolAddress once per device. In host code `scratch` is only a
// stand-in for the symbol; kernels get the address kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[P3M_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on `dev` (must be the current device the first
// time), or nullptr with the HIP error in *err.
void* scratch_for(int dev, hipError_t* err) {
  *err = hipSuccess;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}

size_t mesh_nodes(const Geo& g) { return (size_t)g.grid[0] * g.grid[1] * g.grid[2]; }

p3m_status fail(p3m_ctx* c, p3m_status code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, e_ == hipErrorOutOfMemory ? P3M_ENOMEM : P3M_EHIP,             \
                  std::string(#call) + ": " + hipGetErrorString(e_));                 \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, count * sizeof(T));
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

template <typename R>
p3m_status engine_mesh_alloc(p3m_ctx* ctx, Engine<R>& E) {
  if (E.mesh_ready) return P3M_OK;
  const Geo& g = ctx->geo;
  HIPCHK(dalloc(&E.Q, mesh_nodes(g)));
  HIPCHK(dalloc(&E.phi, mesh_nodes(g)));
  HIPCHK(dalloc(&E.spec, spectrum_elems(g)));
  HIPCHK(dalloc(&E.gz, green_pack_elems(g)));
  launch_green_pack<R>(g, ctx->ghat, E.gz, nullptr);
  HIPCHK(hipStreamSynchronize(nullptr));
  HIPCHK(hipMemset(E.Q, 0, mesh_nodes(g) * sizeof(R)));
  for (int d = 0; d < 3; ++d) {
    const int L = 2 * g.grid[d];
    std::vector<C2<R>> h(L);
    make_twiddles<R>(L, h.data());
    HIPCHK(dalloc(&E.tw[d], (size_t)L));
    HIPCHK(hipMemcpy(E.tw[d], h.data(), L * sizeof(C2<R>), hipMemcpyHostToDevice));
  }
  if constexpr (std::is_same<R, float>::value) {
    if (g.mdiff) {
      HIPCHK(dalloc(&E.spec2, spectrum_elems(g)));
      HIPCHK(dalloc(&E.spec3, spectrum_elems(g)));
      HIPCHK(dalloc(&E.dphi, 3 * mesh_nodes(g)));
      for (int d = 0; d < 3; ++d) {
        const int L = 2 * g.grid[d];
        std::vector<C2<R>> h(L);
        make_diff_factors<R>(L, h.data());
        HIPCHK(dalloc(&E.dtab[d], (size_t)L));
        HIPCHK(hipMemcpy(E.dtab[d], h.data(), L * sizeof(C2<R>), hipMemcpyHostToDevice));
      }
    }
  }
  E.mesh_ready = true;
  return P3M_OK;
}

template <typename R>
p3m_status engine_particles(p3m_ctx* ctx, Engine<R>& E, int64_t n) {
  if (n <= E.cap) return P3M_OK;
  dfree(E.pp);
  dfree(E.mesh);
  dfree(E.fpp);
  E.cap = 0;
  HIPCHK(dalloc(&E.pp, (size_t)n));
  HIPCHK(dalloc(&E.mesh, (size_t)n));
  HIPCHK(dalloc(&E.fpp, (size_t)n));
  E.cap = n;
  return P3M_OK;
}

template <typename R>
void engine_free(Engine<R>& E) {
  dfree(E.pp);
  dfree(E.mesh);
  dfree(E.fpp);
  dfree(E.Q);
  dfree(E.phi);
  dfree(E.spec);
  dfree(E.gz);
  dfree(E.spec2);
  dfree(E.spec3);
  dfree(E.dphi);
  for (int d = 0; d < 3; ++d) dfree(E.tw[d]);
  for (int d = 0; d < 3; ++d) dfree(E.dtab[d]);
  E.cap = 0;
  E.mesh_ready = false;
}

void free_state(p3m_ctx* ctx) {
  for (int b = 0; b < 2; ++b) {
    dfree(ctx->xs[b]);
    dfree(ctx->ps[b]);
    dfree(ctx->qs[b]);
    dfree(ctx->ids[b]);
  }
  dfree(ctx->fs);
}

// Buffers of the cell-ordered step state, at the current capacity.
p3m_status ensure_state(p3m_ctx* ctx, bool weights) {
  if (!ctx->fs) {
    for (int b = 0; b < 2; ++b) {
      HIPCHK(dalloc(&ctx->xs[b], (size_t)3 * ctx->cap));
      HIPCHK(dalloc(&ctx->ps[b], (size_t)3 * ctx->cap));
      HIPCHK(dalloc(&ctx->ids[b], (size_t)ctx->cap));
    }
    HIPCHK(dalloc(&ctx->fs, (size_t)3 * ctx->cap));
  }
  if (weights && !ctx->qs[0]) {
    HIPCHK(dalloc(&ctx->qs[0], (size_t)ctx->cap));
    HIPCHK(dalloc(&ctx->qs[1], (size_t)ctx->cap));
  }
  return P3M_OK;
}

p3m_status ensure_capacity(p3m_ctx* ctx, int64_t n) {
  if (n > 0xffffffffll / 2) return fail(ctx, P3M_EINVAL, "n exceeds the 32-bit particle index range");
  if (n <= ctx->cap) return P3M_OK;
  dfree(ctx->sb.keys_in);
  dfree(ctx->sb.keys);
  dfree(ctx->sb.perm);
  dfree(ctx->groups);
  dfree(ctx->fcache);
  free_state(ctx);
  dfree(ctx->v_sorted);
  dfree(ctx->hpp);
  dfree(ctx->hv);
  dfree(ctx->xb);
  dfree(ctx->pb);
  ctx->cap = 0;
  ctx->force_cached = false;
  HIPCHK(dalloc(&ctx->sb.keys_in, (size_t)n));
  HIPCHK(dalloc(&ctx->sb.keys, (size_t)n));
  HIPCHK(dalloc(&ctx->sb.perm, (size_t)n));
  HIPCHK(dalloc(&ctx->groups, (size_t)pp_group_bound(n, ctx->geo)));
  HIPCHK(dalloc(&ctx->fcache, (size_t)3 * n));
  if (gather_blocks(n) > ctx->bbox_slots) {   // the gather's fused push writes one column per block
    dfree(ctx->bbox_part);
    ctx->bbox_slots = 0;
    HIPCHK(dalloc(&ctx->bbox_part, (size_t)6 * gather_blocks(n)));
    ctx->bbox_slots = gather_blocks(n);
  }
  ctx->cap = n;
  return P3M_OK;
}

p3m_status ensure_adjoint(p3m_ctx* ctx, int64_t n) {
  if (!ctx->v_sorted) {
    HIPCHK(dalloc(&ctx->v_sorted, (size_t)3 * ctx->cap));
    HIPCHK(dalloc(&ctx->hpp, (size_t)3 * ctx->cap));
    HIPCHK(dalloc(&ctx->hv, (size_t)3 * ctx->cap));
    HIPCHK(dalloc(&ctx->xb, (size_t)3 * ctx->cap));
    HIPCHK(dalloc(&ctx->pb, (size_t)3 * ctx->cap));
  }
  if (!ctx->Rm) {
    HIPCHK(dalloc(&ctx->Rm, mesh_nodes(ctx->geo)));
    HIPCHK(dalloc(&ctx->psi, mesh_nodes(ctx->geo)));
  }
  (void)n;
  return P3M_OK;
}

// Stage timing: record an event pair around a group of launches.
struct StageTimer {
  p3m_ctx* c;
  hipStream_t st;
  int slot = -1;
  StageTimer(p3m_ctx* ctx, int stage, hipStream_t s) : c(ctx), st(s) {
    if (c->prof_on && ((c->prof_mask >> stage) & 1) && c->prof_next < (int)c->prof_stage.size()) {
      slot = c->prof_next++;
      c->prof_stage[slot] = stage;
      (void)hipEventRecord(c->prof_ev[2 * slot], st);
    }
  }
  ~StageTimer() {
    if (slot >= 0) (void)hipEventRecord(c->prof_ev[2 * slot + 1], st);
  }
};

// Placement from the bounding box of x (or from place_in), into ctx->place.
void place(p3m_ctx* ctx, int64_t n, const double* x, const double* place_in, double* place_out,
           hipStream_t st) {
  StageTimer t(ctx, 0, st);
  const int nb = bbox_blocks(n);
  launch_bbox(n, x, ctx->bbox_part, nb, ctx->status, st);
  launch_place_finalize(nb, ctx->bbox_part, ctx->geo, place_in, ctx->place, place_out, ctx->status, st);
}

// Image table for the current placement (grounded plane only); returns the
// table to hand to the convolution, or nullptr for free space.
const C2<double>* image_table(p3m_ctx* ctx, hipStream_t st) {
  if (!ctx->geo.cathode) return nullptr;
  const C2<double>* tw[3] = {ctx->tw64[0], ctx->tw64[1], ctx->tw64[2]};
  build_image_table(ctx->geo, ctx->place, ctx->gimg_t1, ctx->gimg_t2, ctx->gimg, tw, st);
  return ctx->gimg;
}

// Everything after the placement: linked cells, PP, mesh, gather. Particle
// records in R, the mesh (charge, transform, potential) of engine EM in M.
template <typename R, typename M>
p3m_status evaluate(p3m_ctx* ctx, Engine<R>& E, Engine<M>& EM, int64_t n, const double* x,
                    const double* qw, GatherOut out, double* e_pp, double* e_pm, const Carry& carry,
                    hipStream_t st) {
  p3m_status s;
  if ((s = engine_mesh_alloc(ctx, EM)) != P3M_OK) return s;
  if ((s = engine_particles(ctx, E, n)) != P3M_OK) return s;
  // float records of a call without weights carry the position residuals
  Geo g = ctx->geo;
  g.wpacked = (std::is_same<R, float>::value && !qw) ? 1 : 0;
  if constexpr (!std::is_same<M, float>::value) g.mdiff = 0;
  {
    StageTimer t(ctx, 1, st);
    launch_cell_sort(n, x, ctx->place, g, ctx->sb, ctx->groups, &ctx->keys, &ctx->perm, st);
  }
  {
    StageTimer t(ctx, 2, st);
    launch_reorder<R>(n, x, qw, ctx->perm, ctx->keys, ctx->place, g, E.pp, E.mesh, ctx->status, carry, st);
  }
  {
    StageTimer t(ctx, 3, st);
    unsigned long long* wc = nullptr;
    if (ctx->prof_on && (ctx->prof_mask & 0x80) && !e_pp && (int64_t)pp_blocks(n, g) <= ctx->wclock_cap)
      wc = ctx->wclock;
    launch_pp<R>(n, E.pp, ctx->keys, ctx->sb.cell_start, g, ctx->groups, ctx->sb.counter, E.fpp, e_pp, st, wc);
    if (wc) ctx->wclock_valid = true;
  }
  {
    StageTimer t(ctx, 4, st);
    launch_deposit<R, M>(n, E.pp, E.mesh, g, EM.Q, st);
  }
  // difference form: the gather reads the three difference meshes, and phi is
  // formed only when the mesh energy is asked for
  bool diff = false;
  if constexpr (std::is_same<M, float>::value) diff = g.mdiff != 0;
  {
    StageTimer t(ctx, 5, st);
    const C2<M>* tw[3] = {EM.tw[0], EM.tw[1], EM.tw[2]};
    if (diff) {
      if constexpr (std::is_same<M, float>::value) {
        const C2<M>* dt[3] = {EM.dtab[0], EM.dtab[1], EM.dtab[2]};
        launch_convolve_diff<M>(g, EM.Q, EM.spec, EM.spec2, EM.spec3, EM.gz, tw, dt, EM.dphi,
                                e_pm ? EM.phi : nullptr, st);
      }
    } else {
      launch_convolve<M>(g, EM.Q, EM.spec, EM.gz, image_table(ctx, st), tw, EM.phi, st);
    }
    EM.phi_current = !diff || e_pm != nullptr;
  }
  {
    StageTimer t(ctx, 6, st);
    const M* field = (diff && !e_pm) ? EM.dphi : EM.phi;
    launch_gather<R, M>(n, E.pp, E.mesh, E.fpp, ctx->perm, g, ctx->place, field, out, e_pm, st);
  }
  ctx->last_precision = sizeof(M) == 4 ? P3M_FP32C : P3M_FP64;
  return P3M_OK;
}

p3m_status evaluate_any(p3m_ctx* ctx, int64_t n, const double* x, const double* qw, GatherOut out,
                        double* e_pp, double* e_pm, hipStream_t st, const Carry& carry = Carry{}) {
  if (ctx->opts.precision == P3M_FP32C) {
    if (ctx->mesh64)
      return evaluate<float, double>(ctx, ctx->e32, ctx->e64, n, x, qw, out, e_pp, e_pm, carry, st);
    return evaluate<float, float>(ctx, ctx->e32, ctx->e32, n, x, qw, out, e_pp, e_pm, carry, st);
  }
  return evaluate<double, double>(ctx, ctx->e64, ctx->e64, n, x, qw, out, e_pp, e_pm, carry, st);
}

p3m_status check_last(p3m_ctx* ctx) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, P3M_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return P3M_OK;
}

// H v at x (placement fixed at ctx->place), into out (caller order). The mesh
// part runs in float64 (the second differences of the potential that its
// Hessian term takes would lose float32's digits); the pair part in float64,
// or for a float-compensated context in float32 from the float records
// (compensated sums).
p3m_status hvp_core(p3m_ctx* ctx, int64_t n, const double* x, const double* qw, const double* v,
                    double* out, hipStream_t st) {
  p3m_status s;
  Engine<double>& E = ctx->e64;
  if ((s = engine_mesh_alloc(ctx, E)) != P3M_OK) return s;
  if ((s = engine_particles(ctx, E, n)) != P3M_OK) return s;
  if ((s = ensure_adjoint(ctx, n)) != P3M_OK) return s;
  const bool pp32 = ctx->opts.precision == P3M_FP32C;
  if (pp32 && (s = engine_particles(ctx, ctx->e32, n)) != P3M_OK) return s;
  const Geo& g = ctx->geo;
  launch_cell_sort(n, x, ctx->place, g, ctx->sb, ctx->groups, &ctx->keys, &ctx->perm, st);
  launch_reorder<double>(n, x, qw, ctx->perm, ctx->keys, ctx->place, g, E.pp, E.mesh, ctx->status, Carry{}, st);
  launch_sort_vector<double>(n, v, ctx->perm, ctx->v_sorted, st);
  if (pp32) {
    Geo gf = g;
    gf.wpacked = qw ? 0 : 1;
    launch_reorder<float>(n, x, qw, ctx->perm, ctx->keys, ctx->place, gf, ctx->e32.pp, ctx->e32.mesh,
                          ctx->status, Carry{}, st);
    launch_pp_hvp<float>(n, ctx->e32.pp, ctx->keys, ctx->sb.cell_start, gf, ctx->groups, ctx->sb.counter,
                         ctx->v_sorted, ctx->hpp, st);
  } else {
    launch_pp_hvp<double>(n, E.pp, ctx->keys, ctx->sb.cell_start, g, ctx->groups, ctx->sb.counter,
                          ctx->v_sorted, ctx->hpp, st);
  }
  const C2<double>* tw[3] = {E.tw[0], E.tw[1], E.tw[2]};
  launch_deposit<double, double>(n, E.pp, E.mesh, g, E.Q, st);
  const C2<double>* gimg = image_table(ctx, st);
  launch_convolve<double>(g, E.Q, E.spec, E.gz, gimg, tw, E.phi, st);
  launch_fill(ctx->Rm, mesh_nodes(g) * sizeof(double), st);
  launch_deposit_grad(n, E.pp, E.mesh, ctx->v_sorted, g, ctx->Rm, st);
  launch_convolve<double>(g, ctx->Rm, E.spec, E.gz, gimg, tw, ctx->psi, st);
  launch_gather_hvp(n, E.pp, E.mesh, ctx->hpp, ctx->v_sorted, ctx->perm, g, ctx->place, E.phi, ctx->psi,
                    out, st);
  ctx->last_precision = -1;
  return P3M_OK;
}

}  // namespace

namespace {

// Layout of the noalloc work buffers for n particles with records in R:
// sort keys in input order, sorted keys, permutation, PP work groups, PP
// positions, mesh records and PP forces, each at a 256-byte boundary.
template <typename R>
struct NoallocLayout {
  size_t keys_in, keys, perm, groups, pp, mesh, fpp, total;
  NoallocLayout(int64_t n, const Geo& g) {
    size_t off = 0;
    auto take = [&off](size_t bytes) {
      const size_t at = off;
      off += (bytes + 255) & ~(size_t)255;
      return at;
    };
    keys_in = take((size_t)n * sizeof(uint32_t));
    keys = take((size_t)n * sizeof(uint32_t));
    perm = take((size_t)n * sizeof(uint32_t));
    groups = take((size_t)pp_group_bound(n, g) * sizeof(int2));
    pp = take((size_t)n * sizeof(PPPos<R>));
    mesh = take((size_t)n * sizeof(MeshRec<R>));
    fpp = take((size_t)n * sizeof(PPRec<R>));
    total = off;
  }
};

template <typename R, typename M>
p3m_status forces_noalloc(p3m_ctx* ctx, Engine<M>& EM, int64_t n, const double* x, const double* qw,
                          double* f, unsigned char* base, hipStream_t st) {
  const NoallocLayout<R> lay(n, ctx->geo);
  if (lay.total > (size_t)P3M_NOALLOC_SCRATCH_BYTES)
    return fail(ctx, P3M_EINVAL,
                "p3m_forces_noalloc: " + std::to_string(n) + " particles need " + std::to_string(lay.total) +
                    " bytes of work buffers, above the static " + std::to_string(P3M_NOALLOC_SCRATCH_BYTES));
  if (!EM.mesh_ready) return fail(ctx, P3M_ESTATE, "p3m_forces_noalloc: mesh buffers missing");
  // particle records in the static array; the context's cell-sort tables,
  // placement and mesh as allocated by p3m_create
  Engine<R> E;
  E.pp = reinterpret_cast<PPPos<R>*>(base + lay.pp);
  E.mesh = reinterpret_cast<MeshRec<R>*>(base + lay.mesh);
  E.fpp = reinterpret_cast<PPRec<R>*>(base + lay.fpp);
  E.cap = n;
  E.mesh_ready = true;   // never used for the mesh: EM is
  const SortBufs saved = ctx->sb;
  int2* saved_groups = ctx->groups;
  ctx->sb.keys_in = reinterpret_cast<uint32_t*>(base + lay.keys_in);
  ctx->sb.keys = reinterpret_cast<uint32_t*>(base + lay.keys);
  ctx->sb.perm = reinterpret_cast<uint32_t*>(base + lay.perm);
  ctx->groups = reinterpret_cast<int2*>(base + lay.groups);
  place(ctx, n, x, nullptr, nullptr, st);
  GatherOut out{f, nullptr, nullptr, nullptr, 0.0};
  const p3m_status s = evaluate<R, M>(ctx, E, EM, n, x, qw, out, nullptr, nullptr, Carry{}, st);
  ctx->sb = saved;
  ctx->groups = saved_groups;
  ctx->keys = nullptr;
  ctx->perm = nullptr;
  return s;
}

}  // namespace

extern "C" {

p3m_status p3m_default_opts(p3m_opts* o) {
  if (!o) return P3M_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->order = P3M_TSC;
  o->precision = P3M_FP64;
  o->zoom = 1;
  o->ke = 8.9875517923e9;
  o->q = 1.0;
  o->m = 1.0;
  return P3M_OK;
}

p3m_status p3m_create(p3m_ctx** out, const int32_t grid[3], const double h[3], double r_cut,
                      double split, const p3m_opts* opts) {
  if (!out || !grid || !h) return P3M_EINVAL;
  *out = nullptr;
  p3m_opts o;
  if (opts) o = *opts;
  else p3m_default_opts(&o);
  if (o.order != P3M_CIC && o.order != P3M_TSC) return P3M_EINVAL;
  if (o.gather != P3M_GATHER_VARIATIONAL && o.gather != P3M_GATHER_MOMENTUM) return P3M_EINVAL;
  if (o.pp_cell_div < 0 || o.pp_cell_div > 2) return P3M_EINVAL;
  if (o.influence < P3M_INFLUENCE_SAMPLED || o.influence > P3M_INFLUENCE_LATTICE) return P3M_EINVAL;
  if (o.influence != P3M_INFLUENCE_SAMPLED && o.boundary == P3M_BOUNDARY_CATHODE) return P3M_EINVAL;
  if (o.boundary != P3M_BOUNDARY_OPEN && o.boundary != P3M_BOUNDARY_CATHODE) return P3M_EINVAL;
  if (o.boundary == P3M_BOUNDARY_CATHODE && !std::isfinite(o.cathode_z)) return P3M_EINVAL;
  if (o.precision != P3M_FP64 && o.precision != P3M_FP32C) return P3M_EINVAL;
  if (o.mesh_precision != P3M_MESH_AUTO && o.mesh_precision != P3M_MESH_F32 &&
      o.mesh_precision != P3M_MESH_F64)
    return P3M_EINVAL;
  if (!(o.m > 0) || !std::isfinite(o.ke) || !std::isfinite(o.q)) return P3M_EINVAL;
  if (!(r_cut > 0) || !std::isfinite(r_cut) || !(split >= 0) || !std::isfinite(split)) return P3M_EINVAL;
  for (int d = 0; d < 3; ++d) {
    if (!fft_supported(grid[d])) return P3M_EINVAL;
    if (!(h[d] > 0) || !std::isfinite(h[d])) return P3M_EINVAL;
  }
  p3m_ctx* ctx = new (std::nothrow) p3m_ctx();
  if (!ctx) return P3M_ENOMEM;
  ctx->opts = o;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return P3M_EHIP;
  }
  // float mesh wider than P3M_MESH_AUTO_F32_MAX nodes on some axis: the
  // difference form for the variational gather in free space, else (AUTO)
  // a float64 mesh
  const bool wide = grid[0] > P3M_MESH_AUTO_F32_MAX || grid[1] > P3M_MESH_AUTO_F32_MAX ||
                    grid[2] > P3M_MESH_AUTO_F32_MAX;
  const bool diff_ok = o.gather == P3M_GATHER_VARIATIONAL && o.boundary == P3M_BOUNDARY_OPEN;
  if (o.precision == P3M_FP32C)
    ctx->mesh64 = o.mesh_precision == P3M_MESH_F64 ||
                  (o.mesh_precision == P3M_MESH_AUTO && wide && !diff_ok);
  Geo& g = ctx->geo;
  g.mdiff = (o.precision == P3M_FP32C && !ctx->mesh64 && wide && diff_ok) ? 1 : 0;
  g.rc = r_cut;
  g.kappa = split * r_cut;
  g.ke_q2 = o.ke * o.q * o.q;
  g.order = o.order;
  g.zoom = o.zoom ? 1 : 0;
  g.gather = o.gather == P3M_GATHER_MOMENTUM ? 1 : 0;
  g.cathode = o.boundary == P3M_BOUNDARY_CATHODE ? 1 : 0;
  g.zc = g.cathode ? o.cathode_z : 0.0;
  g.influence = o.influence;
  g.pp_div = o.pp_cell_div == 2 ? 2 : 1;
  g.ncells = 1;
  for (int d = 0; d < 3; ++d) {
    g.grid[d] = grid[d];
    g.h[d] = h[d];
    g.hu[d] = h[d] / r_cut;
    // PP cells of edge >= r_c / pp_div covering the mesh span exactly
    const double span = (grid[d] - 1) * h[d];
    long long nc = (long long)std::floor(span * g.pp_div / r_cut);
    if (nc < 1) nc = 1;
    if (nc > 4096) nc = 4096;
    g.ncell[d] = (int)nc;
    g.cu[d] = span / (double)nc / r_cut;
    g.ncells *= nc;
  }
  bool roomy = true;
  for (int d = 0; d < 3; ++d) roomy = roomy && usable_nodes(g, d) >= 1.0;
  if (g.ncells > (1ll << 31) - 2 || !roomy) {
    delete ctx;
    return P3M_EINVAL;
  }
  auto bail = [&](p3m_status s) {
    p3m_destroy(ctx);
    return s;
  };
  hipStream_t st = 0;
  if (dalloc(&ctx->place, 1) != hipSuccess || dalloc(&ctx->status, 1) != hipSuccess ||
      dalloc(&ctx->bbox_part, 6 * 1024) != hipSuccess || dalloc(&ctx->acc, 64) != hipSuccess ||
      dalloc(&ctx->sb.counter, 2) != hipSuccess || dalloc(&ctx->sb.cell_start, (size_t)g.ncells + 1) != hipSuccess ||
      dalloc(&ctx->sb.ccount, (size_t)g.ncells) != hipSuccess || dalloc(&ctx->sb.cfill, (size_t)g.ncells) != hipSuccess ||
      dalloc(&ctx->sb.btot, (size_t)kCellTotals * cell_blocks(g.ncells)) != hipSuccess ||
      dalloc(&ctx->sb.stot, (size_t)kCellTotals * cell_supers(g.ncells)) != hipSuccess)
    return bail(P3M_ENOMEM);
  // the per-cell counts start at zero; each sort leaves them at zero
  if (hipMemset(ctx->sb.ccount, 0, (size_t)g.ncells * sizeof(int)) != hipSuccess) return bail(P3M_EHIP);
  if (hipMemset(ctx->status, 0, sizeof(int)) != hipSuccess) return bail(P3M_EHIP);
  // Fourier table of the mesh kernel (float64), built once.
  const size_t oct = (size_t)(grid[0] + 1) * (grid[1] + 1) * (grid[2] + 1);
  double* scratch = nullptr;
  double* cosv[3] = {nullptr, nullptr, nullptr};
  if (dalloc(&ctx->ghat, oct) != hipSuccess || dalloc(&scratch, oct) != hipSuccess) {
    dfree(scratch);
    return bail(P3M_ENOMEM);
  }
  for (int d = 0; d < 3; ++d) {
    const int n2 = 2 * grid[d];
    std::vector<double> c(n2);
    for (int m = 0; m < n2; ++m) c[m] = std::cos(M_PI * (double)m / (double)grid[d]);
    if (dalloc(&cosv[d], (size_t)n2) != hipSuccess ||
        hipMemcpy(cosv[d], c.data(), n2 * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      for (int k = 0; k <= d; ++k) dfree(cosv[k]);
      dfree(scratch);
      return bail(P3M_ENOMEM);
    }
  }
  hipError_t e = build_green_table(g, ctx->ghat, scratch, cosv, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  else (void)hipStreamSynchronize(st);
  for (int d = 0; d < 3; ++d) dfree(cosv[d]);
  dfree(scratch);
  // the lattice table refuses a screening cloud wider than its cell-weight table
  if (e == hipErrorInvalidValue) return bail(P3M_EINVAL);
  if (e != hipSuccess) return bail(P3M_EHIP);
  if (g.cathode) {
    const size_t ne = image_table_elems(g);
    if (dalloc(&ctx->gimg, ne) != hipSuccess || dalloc(&ctx->gimg_t1, ne) != hipSuccess ||
        dalloc(&ctx->gimg_t2, ne) != hipSuccess)
      return bail(P3M_ENOMEM);
    for (int d = 0; d < 3; ++d) {
      const int L = 2 * grid[d];
      std::vector<C2<double>> h(L);
      make_twiddles<double>(L, h.data());
      if (dalloc(&ctx->tw64[d], (size_t)L) != hipSuccess ||
          hipMemcpy(ctx->tw64[d], h.data(), L * sizeof(C2<double>), hipMemcpyHostToDevice) != hipSuccess)
        return bail(P3M_ENOMEM);
    }
  }
  // the mesh buffers of the engine this precision evaluates with, allocated
  // now (p3m_forces_noalloc allocates nothing), and the scratch symbol of
  // this device resolved once
  {
    p3m_status ms = P3M_OK;
    if (o.precision == P3M_FP32C && !ctx->mesh64) ms = engine_mesh_alloc(ctx, ctx->e32);
    else ms = engine_mesh_alloc(ctx, ctx->e64);
    if (ms != P3M_OK) return bail(ms);
    hipError_t se;
    if (!scratch_for(ctx->device, &se)) return bail(P3M_EHIP);
  }
  *out = ctx;
  return P3M_OK;
}

p3m_status p3m_forces_ex(p3m_ctx* ctx, int64_t n, const double* x, const double* qw, double* f_pp,
                         double* f_pm, const double* place_in, double* place_out, void* stream) {
  if (!ctx) return P3M_EINVAL;
  if (n < 0 || (n > 0 && !x)) return fail(ctx, P3M_EINVAL, "bad particle arguments");
  ctx->force_cached = false;
  if (n == 0) return P3M_OK;
  hipStream_t st = (hipStream_t)stream;
  p3m_status s;
  if ((s = ensure_capacity(ctx, n)) != P3M_OK) return s;
  place(ctx, n, x, place_in, place_out, st);
  GatherOut out{nullptr, f_pp, f_pm, nullptr, 0.0};
  if ((s = evaluate_any(ctx, n, x, qw, out, nullptr, nullptr, st)) != P3M_OK) return s;
  return check_last(ctx);
}

p3m_status p3m_forces(p3m_ctx* ctx, int64_t n, const double* x, const double* qw, double* f, void* stream) {
  if (!ctx) return P3M_EINVAL;
  if (n < 0 || (n > 0 && (!x || !f))) return fail(ctx, P3M_EINVAL, "bad particle arguments");
  ctx->force_cached = false;
  if (n == 0) return P3M_OK;
  hipStream_t st = (hipStream_t)stream;
  p3m_status s;
  if ((s = ensure_capacity(ctx, n)) != P3M_OK) return s;
  place(ctx, n, x, nullptr, nullptr, st);
  GatherOut out{f, nullptr, nullptr, nullptr, 0.0};
  if ((s = evaluate_any(ctx, n, x, qw, out, nullptr, nullptr, st)) != P3M_OK) return s;
  return check_last(ctx);
}

p3m_status p3m_forces_noalloc(p3m_ctx* ctx, int64_t n, const double* x, const double* qw, double* f,
                              void* stream) {
  if (!ctx) return P3M_EINVAL;
  if (n < 0 || (n > 0 && (!x || !f))) return fail(ctx, P3M_EINVAL, "bad particle arguments");
  if (n > 0xffffffffll / 2) return fail(ctx, P3M_EINVAL, "n exceeds the 32-bit particle index range");
  ctx->force_cached = false;
  if (n == 0) return P3M_OK;
  hipError_t se;
  unsigned char* base = static_cast<unsigned char*>(scratch_for(ctx->device, &se));
  if (!base) return fail(ctx, P3M_EHIP, std::string("scratch symbol: ") + hipGetErrorString(se));
  hipStream_t st = (hipStream_t)stream;
  p3m_status s;
  if (ctx->opts.precision == P3M_FP32C) {
    if (ctx->mesh64) s = forces_noalloc<float, double>(ctx, ctx->e64, n, x, qw, f, base, st);
    else s = forces_noalloc<float, float>(ctx, ctx->e32, n, x, qw, f, base, st);
  } else {
    s = forces_noalloc<double, double>(ctx, ctx->e64, n, x, qw, f, base, st);
  }
  if (s != P3M_OK) return s;
  return check_last(ctx);
}

p3m_status p3m_step(p3m_ctx* ctx, int64_t n, double* x, double* p, const double* qw, double dt,
                    int32_t nsteps, int32_t reuse_force, const double* place_replay,
                    double* place_record, void* stream) {
  if (!ctx) return P3M_EINVAL;
  if (n < 0 || nsteps < 0 || !std::isfinite(dt) || (n > 0 && (!x || !p)))
    return fail(ctx, P3M_EINVAL, "bad step arguments");
  if (n == 0) return P3M_OK;
  hipStream_t st = (hipStream_t)stream;
  p3m_status s;
  if ((s = ensure_capacity(ctx, n)) != P3M_OK) return s;
  if (reuse_force) {
    if (!ctx->force_cached || ctx->cached_x != x || ctx->cached_n != n)
      return fail(ctx, P3M_ESTATE, "no cached force for these positions");
    // a replay skips record 0 (the cached force stands for it); a record
    // would leave record 0 unwritten
    if (place_record) return fail(ctx, P3M_EINVAL, "placement record needs a fresh start force");
  }
  // The state is stepped in the cell order of the latest force evaluation:
  // each reorder moves x, p, the caller indices and the weights into the new
  // order, so that the push, the gather's writes and the next sort stream
  // through memory instead of scattering to caller order every step. One
  // scatter at the end restores caller order. Placement (min/max) and the
  // fixed-point deposit do not depend on the order; the PP sums do only
  // through rounding.
  // Every gather moves x and p into its evaluation's order (read through
  // the permutation from the previous order) with the closing kick; every
  // gather but the last of the call also applies the next step's kick and
  // drift and stores the box partials of the new positions, so the step
  // needs no separate push pass. The reorder carries the caller indices and
  // weights.
  if ((s = ensure_state(ctx, qw != nullptr)) != P3M_OK) return s;
  const double inv_m = 1.0 / ctx->opts.m;
  auto move_state = [&](GatherOut& o, const double* x_src, const double* p_src, int to, double kick, bool push) {
    o.p = ctx->ps[to];
    o.p_src = p_src;
    o.x = ctx->xs[to];
    o.x_src = x_src;
    o.half_dt = kick;
    o.dt_over_m = dt * inv_m;
    o.part = push ? ctx->bbox_part : nullptr;
    o.status = ctx->status;
  };
  int cur = 0;
  bool sorted = false;
  bool pushed = false;   // the last gather applied the kick and drift of the step to come
  if (!reuse_force) {
    place(ctx, n, x, place_replay, place_record, st);
    Carry c;
    c.id_out = ctx->ids[0];
    c.qw_out = ctx->qs[0];
    GatherOut out{ctx->fs, nullptr, nullptr, nullptr, 0.0, true};
    pushed = nsteps > 0;
    move_state(out, x, p, 0, pushed ? 0.5 * dt : 0.0, pushed);
    if ((s = evaluate_any(ctx, n, x, qw, out, nullptr, nullptr, st, c)) != P3M_OK) return s;
    sorted = true;
  }
  const int nb = bbox_blocks(n);
  for (int k = 0; k < nsteps; ++k) {
    const size_t off = (size_t)P3M_PLACEMENT_DOUBLES * (k + 1);
    double* xk = sorted ? ctx->xs[cur] : x;
    double* pk = sorted ? ctx->ps[cur] : p;
    const double* qk = sorted ? (qw ? ctx->qs[cur] : nullptr) : qw;
    {
      StageTimer t(ctx, 0, st);
      if (!pushed)
        launch_kick_drift_bbox(n, xk, pk, sorted ? ctx->fs : ctx->fcache, dt, inv_m, ctx->bbox_part, nb,
                               ctx->status, st);
      launch_place_finalize(pushed ? gather_blocks(n) : nb, ctx->bbox_part, ctx->geo,
                            place_replay ? place_replay + off : nullptr, ctx->place,
                            place_record ? place_record + off : nullptr, ctx->status, st);
    }
    const int nxt = sorted ? 1 - cur : 0;
    Carry c;
    c.id_in = sorted ? ctx->ids[cur] : nullptr;
    c.id_out = ctx->ids[nxt];
    c.qw_out = ctx->qs[nxt];
    GatherOut out{ctx->fs, nullptr, nullptr, nullptr, 0.0, true};
    pushed = k + 1 < nsteps;
    // this step's closing half kick, and the next step's half kick when fused
    move_state(out, xk, pk, nxt, pushed ? dt : 0.5 * dt, pushed);
    if ((s = evaluate_any(ctx, n, xk, qk, out, nullptr, nullptr, st, c)) != P3M_OK) return s;
    cur = nxt;
    sorted = true;
  }
  if (sorted) {
    StageTimer t(ctx, 2, st);
    launch_unpermute(n, ctx->xs[cur], ctx->ps[cur], ctx->fs, ctx->ids[cur], x, p, ctx->fcache, st);
  }
  ctx->force_cached = true;
  ctx->cached_x = x;
  ctx->cached_n = n;
  return check_last(ctx);
}

p3m_status p3m_hvp(p3m_ctx* ctx, int64_t n, const double* x, const double* qw, const double* v,
                   const double* place_in, double* out, void* stream) {
  if (!ctx) return P3M_EINVAL;
  if (n < 0 || (n > 0 && (!x || !v || !out))) return fail(ctx, P3M_EINVAL, "bad hvp arguments");
  if (ctx->geo.gather) return fail(ctx, P3M_ESTATE, "the Hessian is that of the variational force");
  ctx->force_cached = false;
  if (n == 0) return P3M_OK;
  hipStream_t st = (hipStream_t)stream;
  p3m_status s;
  if ((s = ensure_capacity(ctx, n)) != P3M_OK) return s;
  place(ctx, n, x, place_in, nullptr, st);
  if ((s = hvp_core(ctx, n, x, qw, v, out, st)) != P3M_OK) return s;
  return check_last(ctx);
}

p3m_status p3m_backward(p3m_ctx* ctx, int64_t n, const double* x_n, const double* x_np1, const double* qw,
                        const double* xbar_np1, const double* pbar_np1, double* xbar_n, double* pbar_n,
                        double dt, const double* place_n, const double* place_np1, void* stream) {
  if (!ctx) return P3M_EINVAL;
  if (n < 0 || !std::isfinite(dt) ||
      (n > 0 && (!x_n || !x_np1 || !xbar_np1 || !pbar_np1 || !xbar_n || !pbar_n)))
    return fail(ctx, P3M_EINVAL, "bad backward arguments");
  if (ctx->geo.gather) return fail(ctx, P3M_ESTATE, "the adjoint is that of the variational force");
  ctx->force_cached = false;
  if (n == 0) return P3M_OK;
  hipStream_t st = (hipStream_t)stream;
  p3m_status s;
  if ((s = ensure_capacity(ctx, n)) != P3M_OK) return s;
  if ((s = ensure_adjoint(ctx, n)) != P3M_OK) return s;
  const size_t bytes = (size_t)3 * n * sizeof(double);
  // xb = xbar_np1 + dt/2 H(x_np1) pbar_np1
  place(ctx, n, x_np1, place_np1, nullptr, st);
  if ((s = hvp_core(ctx, n, x_np1, qw, pbar_np1, ctx->hv, st)) != P3M_OK) return s;
  HIPCHK(hipMemcpyAsync(ctx->xb, xbar_np1, bytes, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->pb, pbar_np1, bytes, hipMemcpyDeviceToDevice, st));
  launch_kick(n, ctx->xb, ctx->hv, dt, st);                  // xb += dt/2 hv
  // pb += dt/m xb  (a kick with 'force' xb and step 2 dt/m)
  launch_kick(n, ctx->pb, ctx->xb, 2.0 * dt / ctx->opts.m, st);
  // xbar_n = xb + dt/2 H(x_n) pb
  place(ctx, n, x_n, place_n, nullptr, st);
  if ((s = hvp_core(ctx, n, x_n, qw, ctx->pb, ctx->hv, st)) != P3M_OK) return s;
  launch_kick(n, ctx->xb, ctx->hv, dt, st);
  HIPCHK(hipMemcpyAsync(xbar_n, ctx->xb, bytes, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(pbar_n, ctx->pb, bytes, hipMemcpyDeviceToDevice, st));
  return check_last(ctx);
}

p3m_status p3m_backward_steps(p3m_ctx* ctx, int64_t n, int32_t nsteps, const double* xs, const double* qw,
                              double* xbar, double* pbar, double dt, const double* places, void* stream) {
  if (!ctx) return P3M_EINVAL;
  if (n < 0 || nsteps < 0 || !std::isfinite(dt) || (n > 0 && nsteps > 0 && (!xs || !xbar || !pbar || !places)))
    return fail(ctx, P3M_EINVAL, "bad backward arguments");
  if (ctx->geo.gather) return fail(ctx, P3M_ESTATE, "the adjoint is that of the variational force");
  ctx->force_cached = false;
  if (n == 0 || nsteps == 0) return P3M_OK;
  hipStream_t st = (hipStream_t)stream;
  p3m_status s;
  if ((s = ensure_capacity(ctx, n)) != P3M_OK) return s;
  if ((s = ensure_adjoint(ctx, n)) != P3M_OK) return s;
  const size_t stride = (size_t)3 * n;
  auto xk = [&](int k) { return xs + (size_t)k * stride; };
  auto pk = [&](int k) { return places + (size_t)k * P3M_PLACEMENT_DOUBLES; };
  // hv = H(x_N) pbar_N; then per step k+1 -> k:
  //   xbar += dt/2 hv;  pbar += dt/m xbar;  hv = H(x_k) pbar;  xbar += dt/2 hv
  place(ctx, n, xk(nsteps), pk(nsteps), nullptr, st);
  if ((s = hvp_core(ctx, n, xk(nsteps), qw, pbar, ctx->hv, st)) != P3M_OK) return s;
  for (int k = nsteps - 1; k >= 0; --k) {
    launch_kick(n, xbar, ctx->hv, dt, st);
    launch_kick(n, pbar, xbar, 2.0 * dt / ctx->opts.m, st);
    place(ctx, n, xk(k), pk(k), nullptr, st);
    if ((s = hvp_core(ctx, n, xk(k), qw, pbar, ctx->hv, st)) != P3M_OK) return s;
    launch_kick(n, xbar, ctx->hv, dt, st);
  }
  return check_last(ctx);
}

p3m_status p3m_diagnostics(p3m_ctx* ctx, int64_t n, const double* x, const double* p, const double* qw,
                           p3m_diag* out, void* stream) {
  if (!ctx || !out) return P3M_EINVAL;
  if (n < 1 || !x || !p) return fail(ctx, P3M_EINVAL, "bad diagnostics arguments");
  ctx->force_cached = false;
  hipStream_t st = (hipStream_t)stream;
  p3m_status s;
  if ((s = ensure_capacity(ctx, n)) != P3M_OK) return s;
  launch_fill(ctx->acc, 64 * sizeof(double), st);
  place(ctx, n, x, nullptr, nullptr, st);
  GatherOut go{nullptr, nullptr, nullptr, nullptr, 0.0};
  // acc[40] pair energy, acc[41] mesh energy, acc[42] pair count
  if ((s = evaluate_any(ctx, n, x, qw, go, ctx->acc + 40, ctx->acc + 41, st)) != P3M_OK) return s;
  launch_moments(n, x, p, qw, ctx->acc, 0, st);
  launch_moments(n, x, p, qw, ctx->acc, 1, st);
  double h[64];
  Place P;
  HIPCHK(hipMemcpyAsync(h, ctx->acc, sizeof(h), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&P, ctx->place, sizeof(P), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double inv_n = 1.0 / (double)n;
  const double m = ctx->opts.m;
  for (int d = 0; d < 3; ++d) {
    out->momentum[d] = h[d];
    out->mean[d] = h[4 + d] * inv_n;
    const double sxx = h[16 + d] * inv_n, spp = h[19 + d] * inv_n, sxp = h[22 + d] * inv_n;
    out->rms[d] = std::sqrt(sxx);
    const double e2 = sxx * spp - sxp * sxp;
    out->emit_n[d] = std::sqrt(e2 > 0 ? e2 : 0.0) / (m * kCLight);
  }
  out->kinetic = h[3] / (2.0 * m);
  // energies: internal units times k_e q^2 / Lu
  const double escale = ctx->geo.ke_q2 * P.inv_lu;
  out->u_pp = h[40] * escale;
  out->u_pm = h[41] * escale;
  out->zoom = P.s;
  out->charge = h[7];
  out->pairs = h[42];
  return P3M_OK;
}

p3m_status p3m_mesh(p3m_ctx* ctx, int32_t which, double* out, void* stream) {
  if (!ctx || !out || (which != 0 && which != 1)) return P3M_EINVAL;
  if (ctx->last_precision < 0) return fail(ctx, P3M_ESTATE, "no force evaluation yet");
  hipStream_t st = (hipStream_t)stream;
  if (ctx->last_precision == P3M_FP32C) {
    Engine<float>& E = ctx->e32;
    if (which == 1 && !E.phi_current) {
      // difference form: phi from the spectrum the last evaluation left
      launch_phi_from_diff<float>(ctx->geo, E.spec, E.tw[0], E.phi, st);
      E.phi_current = true;
    }
    launch_mesh_export<float>(ctx->geo, which ? E.phi : E.Q, ctx->place, which, out, st);
  } else
    launch_mesh_export<double>(ctx->geo, which ? ctx->e64.phi : ctx->e64.Q, ctx->place, which, out, st);
  return check_last(ctx);
}

p3m_status p3m_profile_begin(p3m_ctx* ctx, int32_t max_records, int32_t stage_mask) {
  if (!ctx || max_records < 1 || (stage_mask & ~0xff) || !stage_mask) return P3M_EINVAL;
  ctx->prof_mask = stage_mask;
  if (stage_mask & 0x80) {
    // wave clocks of the pair kernel, for the largest n evaluated so far
    const int64_t need = 2 * (int64_t)pp_blocks(ctx->cap > 0 ? ctx->cap : 1, ctx->geo);
    if (need > ctx->wclock_cap) {
      dfree(ctx->wclock);
      ctx->wclock_cap = 0;
      HIPCHK(dalloc(&ctx->wclock, (size_t)need));
      ctx->wclock_cap = need / 2;
    }
    ctx->wclock_valid = false;
  }
  for (auto& e : ctx->prof_ev) (void)hipEventDestroy(e);
  ctx->prof_ev.assign(2 * (size_t)max_records, nullptr);
  for (auto& e : ctx->prof_ev) HIPCHK(hipEventCreate(&e));
  ctx->prof_stage.assign(max_records, -1);
  ctx->prof_next = 0;
  ctx->prof_on = true;
  return P3M_OK;
}

p3m_status p3m_profile_end(p3m_ctx* ctx, double ms[8], int64_t launches[8], void* stream) {
  if (!ctx || !ms || !launches) return P3M_EINVAL;
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  for (int k = 0; k < 8; ++k) { ms[k] = 0.0; launches[k] = 0; }
  for (int s = 0; s < ctx->prof_next; ++s) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, ctx->prof_ev[2 * s], ctx->prof_ev[2 * s + 1]));
    ms[ctx->prof_stage[s]] += t;
    launches[ctx->prof_stage[s]] += 1;
  }
  ctx->prof_on = false;
  ctx->prof_next = 0;
  return P3M_OK;
}

p3m_status p3m_profile_pp_waves(p3m_ctx* ctx, int64_t cap, double* out, int64_t* count, void* stream) {
  if (!ctx || cap < 0 || (cap > 0 && !out) || !count) return P3M_EINVAL;
  if (!ctx->wclock_valid) return fail(ctx, P3M_ESTATE, "no pair-kernel waves recorded");
  hipStream_t st = (hipStream_t)stream;
  int cnt[2] = {0, 0};   // dense-cell and other PP groups
  HIPCHK(hipMemcpyAsync(cnt, ctx->sb.counter, sizeof(cnt), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const int64_t groups = (int64_t)cnt[0] + cnt[1];
  const int64_t waves = (groups + 3) / 4;
  *count = waves;
  const int64_t m = waves < cap ? waves : cap;
  if (m > 0) {
    std::vector<unsigned long long> h(2 * (size_t)m);
    HIPCHK(hipMemcpy(h.data(), ctx->wclock, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    unsigned long long t0 = h[0];
    for (int64_t k = 0; k < m; ++k) t0 = h[2 * k] < t0 ? h[2 * k] : t0;
    for (int64_t k = 0; k < 2 * m; ++k) out[k] = (double)(h[k] - t0) * 0.01;   // 100 MHz ticks -> us
  }
  return P3M_OK;
}

p3m_status p3m_status_sync(p3m_ctx* ctx, void* stream) {
  if (!ctx) return P3M_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, ctx->status, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (h) {
    launch_fill(ctx->status, sizeof(int), st);
    HIPCHK(hipStreamSynchronize(st));
  }
  if (h & kBitNonFinite) return fail(ctx, P3M_ENONFINITE, "non-finite particle position");
  if (h & kBitDomain) return fail(ctx, P3M_EDOMAIN, "particle outside the mesh (zoom disabled or replayed placement)");
  return P3M_OK;
}

p3m_status p3m_info(const p3m_ctx* ctx, int64_t out[8]) {
  if (!ctx || !out) return P3M_EINVAL;
  // bits of the mesh arithmetic (charge, transform, potential) of this context
  out[0] = (ctx->opts.precision == P3M_FP64 || ctx->mesh64) ? 64 : 32;
  out[1] = ctx->geo.ncells;
  out[2] = ctx->geo.ncell[0];
  out[3] = ctx->geo.ncell[1];
  out[4] = ctx->geo.ncell[2];
  out[5] = 2 * ctx->geo.grid[0];
  out[6] = 2 * ctx->geo.grid[1];
  out[7] = 2 * ctx->geo.grid[2];
  return P3M_OK;
}

const char* p3m_last_error(const p3m_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

void p3m_destroy(p3m_ctx* ctx) {
  if (!ctx) return;
  for (auto& e : ctx->prof_ev) (void)hipEventDestroy(e);
  engine_free(ctx->e32);
  engine_free(ctx->e64);
  dfree(ctx->sb.keys_in);
  dfree(ctx->sb.keys);
  dfree(ctx->sb.perm);
  dfree(ctx->sb.ccount);
  dfree(ctx->sb.cfill);
  dfree(ctx->sb.btot);
  dfree(ctx->sb.stot);
  dfree(ctx->sb.counter);
  dfree(ctx->groups);
  dfree(ctx->sb.cell_start);
  dfree(ctx->place);
  dfree(ctx->status);
  dfree(ctx->bbox_part);
  dfree(ctx->acc);
  dfree(ctx->ghat);
  dfree(ctx->gimg);
  dfree(ctx->gimg_t1);
  dfree(ctx->gimg_t2);
  for (int d = 0; d < 3; ++d) dfree(ctx->tw64[d]);
  dfree(ctx->fcache);
  dfree(ctx->wclock);
  free_state(ctx);
  dfree(ctx->v_sorted);
  dfree(ctx->hpp);
  dfree(ctx->hv);
  dfree(ctx->xb);
  dfree(ctx->pb);
  dfree(ctx->Rm);
  dfree(ctx->psi);
  delete ctx;
}

}  // extern "C"
