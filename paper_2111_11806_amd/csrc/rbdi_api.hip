// rbdi_api.hip -- host side of librbdi: the C ABI declared in include/rbdi.h.
// Validates arguments, owns device buffers, and enqueues the kernels of
// rbdi_kernels.hpp on the handle's stream. Instantiated for the systems
// (dimension, materials, elastoplastic) and precisions the library supports.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rbdi.h"
#include "rbdi_batch.hpp"
#include "rbdi_mlp.hpp"

using namespace rbdi;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_OK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) return fail(RBDI_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

struct Ops;

}  // namespace

struct rbdi_handle {
  rbdi_desc desc;
  Params P;
  int nf = 0;
  int elem = 8;            // bytes per stored value
  void* U[3] = {nullptr, nullptr, nullptr};
  void* D = nullptr;
  void* D2 = nullptr;  // 3D: the y sweep's part of the operator (the z sweep's is in D)
  double* stage_buf = nullptr;  // FP64 staging for API transfers (nf * ncell)
  SeedTask* tasks = nullptr;    // seeding tasks of the rigid band
  int task_cap = 0;
  int par = 0;                  // parity of the next step
  bool cfl_valid = false;       // CFL partials of the current state are in cflpart
  double* cflpart = nullptr;    // CFL partials (one per block of their producer)
  int part_cap = 0;
  DevScalars* sc = nullptr;
  double* part = nullptr;       // reduction partials
  double* red_out = nullptr;    // reduction results (device)
  hipStream_t stream = nullptr;
  bool have_mat[kMaxMat] = {false, false};
  bool have_state = false;
  bool band_valid = false;
  bool dynamic_r = false;
  double t_host = 0.0;
  const Ops* ops = nullptr;
  rbdi_batch* owner = nullptr;  // batch that steps this instance, if any
  rbdi_mlp* mlp = nullptr;      // surrogate closure of the elastoplastic sources, if set
  long long enqueued = 0;       // steps enqueued by this handle
  int x_waves = 0;              // x-sweep wavefronts per block (0: the library's rule)
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev;   // start/stop pairs
  std::vector<int> ev_cls;      // class of each recorded pair
  size_t ev_used = 0;
};

namespace {

// Event pair for the next launch of class cls when kernel timing is on.
bool timing_pair(rbdi_handle* h, int cls, hipEvent_t& e0, hipEvent_t& e1) {
  if (!h->timing || cls < 0) return false;
  if (h->ev_used * 2 + 2 > h->ev.size()) {
    for (int k = 0; k < 256; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return false;
      h->ev.push_back(e);
    }
  }
  const size_t slot = h->ev_used++;
  if (h->ev_cls.size() < h->ev_used) h->ev_cls.resize(h->ev_used);
  h->ev_cls[slot] = cls;
  e0 = h->ev[2 * slot];
  e1 = h->ev[2 * slot + 1];
  return true;
}

// Launch on the handle's stream. With kernel timing on, the event pair is
// part of the dispatch itself (hipExtLaunchKernelGGL), so the elapsed time is
// the kernel's own duration.
template <typename F, typename... Args>
void launch(rbdi_handle* h, int cls, F kernel, dim3 g, dim3 b, unsigned shm, Args... args) {
  hipEvent_t e0, e1;
  if (timing_pair(h, cls, e0, e1)) hipExtLaunchKernelGGL(kernel, g, b, shm, h->stream, e0, e1, 0, args...);
  else hipLaunchKernelGGL(kernel, g, b, shm, h->stream, args...);
}

}  // namespace

struct rbdi_mlp {
  __bf16* blob = nullptr;   // padded BF16 operands (see MlpDev)
  float* bias = nullptr;    // kBiasN
  float* master = nullptr;  // FP32 parameters, flat layout
  float* m1 = nullptr;      // Adam moments
  float* m2 = nullptr;
  float* sum = nullptr;     // kNParam + 1 (gradient + loss)
  double tau_max = 1.0;
  int step = 0;
};

namespace {

MlpDev mlp_dev(const rbdi_mlp* m) {
  MlpDev d;
  const __bf16* b = m->blob;
  d.W1 = b;
  d.W2 = b + kW1n;
  d.W3 = d.W2 + kW2n;
  d.W4 = d.W3 + kW3n;
  d.W2T = d.W4 + kW4n;
  d.W3T = d.W2T + kW2Tn;
  d.W4T = d.W3T + kW3Tn;
  d.b1 = m->bias;
  d.b2 = m->bias + 64;
  d.b3 = m->bias + 128;
  d.b4 = m->bias + 192;
  d.tau_max = m->tau_max;
  return d;
}

struct Ops {
  void (*prim_to_state)(rbdi_handle*, const double*);
  void (*state_to_prim)(rbdi_handle*, double*);
  void (*state_to_f64)(rbdi_handle*, double*, int);
  void (*f64_to_state)(rbdi_handle*, const double*);
  void (*r_from_sdf)(rbdi_handle*, const double*, double);
  void (*band)(rbdi_handle*, const StepArgs&);
  void (*seed)(rbdi_handle*, const StepArgs&);
  void (*stages)(rbdi_handle*, const StepArgs&);
  void (*cfl)(rbdi_handle*);
  void (*force)(rbdi_handle*, const double*);
  void (*totals)(rbdi_handle*);
  int (*part_blocks)(const Params&);
  void (*unit)(rbdi_handle*, int, int, const double*, const double*, double*, int);
  void (*rhs)(rbdi_handle*, int);
  void (*replay)(rbdi_handle*, int);
};

inline unsigned blocks_for(long long n, int t) { return (unsigned)((n + t - 1) / t); }

template <class S, typename T>
struct Impl {
  static T* u(rbdi_handle* h, int k) { return static_cast<T*>(h->U[k]); }

  static void prim_to_state(rbdi_handle* h, const double* W) {
    hipLaunchKernelGGL((k_prim_to_state<S, T>), dim3(blocks_for(h->P.ncell, 256)), dim3(256), 0, h->stream, h->P,
                       W, u(h, 0));
  }
  static void state_to_prim(rbdi_handle* h, double* W) {
    hipLaunchKernelGGL((k_state_to_prim<S, T>), dim3(blocks_for(h->P.ncell, 256)), dim3(256), 0, h->stream, h->P,
                       (const T*)u(h, 0), W);
  }
  static void state_to_f64(rbdi_handle* h, double* out, int add_B) {
    hipLaunchKernelGGL((k_state_to_f64<S, T>), dim3(blocks_for(h->P.ncell, 256)), dim3(256), 0, h->stream, h->P,
                       (const T*)u(h, 0), out, add_B);
  }
  static void f64_to_state(rbdi_handle* h, const double* in) {
    hipLaunchKernelGGL((k_f64_to_state<S, T>), dim3(blocks_for(h->P.ncell, 256)), dim3(256), 0, h->stream, h->P,
                       in, u(h, 0));
  }
  static void r_from_sdf(rbdi_handle* h, const double* sdf, double inv_w) {
    hipLaunchKernelGGL((k_r_from_sdf<S, T>), dim3(blocks_for(h->P.ncell, 256)), dim3(256), 0, h->stream, h->P,
                       sdf, inv_w, u(h, 0));
  }
  static void band(rbdi_handle* h, const StepArgs& A) {
    hipLaunchKernelGGL(k_band_reset, dim3(1), dim3(1), 0, h->stream, h->sc, A);
    launch(h, 4, k_band<S, T>, dim3(blocks_for(h->P.ncell, 256)), dim3(256), 0, h->P, (const T*)u(h, 0), h->tasks,
           h->task_cap, h->sc, A);
  }
  // Launches with more than one rigid body take the kernels that test the
  // ownership boxes (rigid_velocity<true>); the others leave that code out.
  static bool multi(const rbdi_handle* h) { return h->P.nbody > 1; }
  static void seed(rbdi_handle* h, const StepArgs& A) {
    if (multi(h))
      launch(h, 3, k_seed<S, T, true>, dim3(256), dim3(256), 0, h->P, u(h, 0), (const SeedTask*)h->tasks,
             h->task_cap, h->sc, A);
    else
      launch(h, 3, k_seed<S, T, false>, dim3(256), dim3(256), 0, h->P, u(h, 0), (const SeedTask*)h->tasks,
             h->task_cap, h->sc, A);
  }
  // Wavefronts per x-sweep block: 1 in 1D and for the elastoplastic systems
  // (their blocks hold LDS per wavefront and nothing per block, so a block of
  // one leaves no wavefront idle: on the 256-cell rows of the 256^3 copper
  // grid, 5 segments, an FP64 x sweep takes 4.8 ms as 5 blocks of 1, 5.1 ms
  // as 3 blocks of 2, 7.6 ms as 2 blocks of 4); otherwise 4 or 2, whichever
  // leaves fewer idle wavefronts at the end of a row (4 on ties; measured on
  // the 1024-cell rows of the shock/cylinder grid: 18 segments run 1.4%
  // faster per step as 9 blocks of 2 than as 5 blocks of 4).
  static int x_wpb(const rbdi_handle* h) {
    if (S::D == 1) return 1;
    if (h->x_waves > 0) return h->x_waves;  // rbdi_set_x_waves / rbdi_autotune
    if (S::S) return 1;
    const int nseg = (h->P.n[0] + kOut - 1) / kOut;
    const int idle4 = (nseg + 3) / 4 * 4 - nseg, idle2 = (nseg + 1) / 2 * 2 - nseg;
    return idle2 < idle4 ? 2 : 4;
  }
  static dim3 x_grid(const rbdi_handle* h) {
    const Params& P = h->P;
    const unsigned nseg = (unsigned)((P.n[0] + kOut - 1) / kOut);
    const unsigned w = (unsigned)x_wpb(h);
    return dim3((nseg + w - 1) / w, (unsigned)P.n[1], (unsigned)P.n[2]);
  }
  template <bool MB>
  static void sweep_x_mb(rbdi_handle* h, const T* Uin, const T* U0, T* Uout, const StepArgs& A, double b, int stage) {
    if constexpr (S::S) {
      if (h->P.surr) {  // the surrogate sources inside the final sweep
        launch(h, 0, k_sweep_x_surr<S, T, MB>, x_grid(h), dim3(kWave * x_wpb(h)),
               (unsigned)(x_wpb(h) * sizeof(XSurrLds<S, T>)), h->P, Uin, U0,
               (const T*)h->D, (const T*)h->D2, Uout, h->sc, h->cflpart, A, b, stage, mlp_dev(h->mlp));
        return;
      }
    }
    launch(h, 0, k_sweep_x<S, T, MB>, x_grid(h), dim3(kWave * x_wpb(h)), x_sweep_lds<S, T>(x_wpb(h)), h->P, Uin,
           U0, (const T*)h->D, (const T*)h->D2, Uout,
           h->sc, h->cflpart, A, b, stage);
  }
  static void sweep_x(rbdi_handle* h, const T* Uin, const T* U0, T* Uout, const StepArgs& A, double b, int stage) {
    if (multi(h)) sweep_x_mb<true>(h, Uin, U0, Uout, A, b, stage);
    else sweep_x_mb<false>(h, Uin, U0, Uout, A, b, stage);
  }
  // dst: the accumulator (D, or in 3D D2 for the y sweep)
  template <int DIR, int MODE, bool REDUCE>
  static void sweep_t(rbdi_handle* h, const T* Uin, const StepArgs& A, void* dst) {
    const Params& P = h->P;
    constexpr int TC = tile_cols<S, T>();
    const unsigned nseg = (unsigned)((P.n[DIR] + kOut - 1) / kOut);
    const unsigned gx = (unsigned)((P.n[0] + TC - 1) / TC);
    const dim3 grid = DIR == 1 ? dim3(gx, nseg, (unsigned)P.n[2]) : dim3(gx, (unsigned)P.n[1], nseg);
    if (multi(h))
      launch(h, DIR, k_sweep_tile<S, T, DIR, MODE, REDUCE, true>, grid, dim3(kTileThreads), 0, P, Uin,
             static_cast<T*>(dst), h->sc, (const double*)h->cflpart, A);
    else
      launch(h, DIR, k_sweep_tile<S, T, DIR, MODE, REDUCE, false>, grid, dim3(kTileThreads), 0, P, Uin,
             static_cast<T*>(dst), h->sc, (const double*)h->cflpart, A);
  }
  static void stages(rbdi_handle* h, const StepArgs& A) {
    const double bc[3] = {1.0, 0.25, 2.0 / 3.0};
    const int in_[3] = {0, 1, 2}, out_[3] = {1, 2, 0};
    if constexpr (S::D == 1) launch(h, 5, k_reduce_dt, dim3(1), dim3(256), 0, h->sc, (const double*)h->cflpart, A);
    for (int s = 0; s < 3; ++s) {
      const T* Uin = u(h, in_[s]);
      const T* U0 = u(h, 0);
      T* Uout = u(h, out_[s]);
      if constexpr (S::D == 3) {
        if (s == 0) sweep_t<2, 0, true>(h, Uin, A, h->D);
        else sweep_t<2, 0, false>(h, Uin, A, h->D);
        sweep_t<1, 0, false>(h, Uin, A, h->D2);
      } else if constexpr (S::D == 2) {
        if (s == 0) sweep_t<1, 0, true>(h, Uin, A, h->D);
        else sweep_t<1, 0, false>(h, Uin, A, h->D);
      }
      sweep_x(h, Uin, U0, Uout, A, bc[s], s);
    }
  }
  static void cfl(rbdi_handle* h) {
    if (multi(h))
      launch(h, 5, k_cfl<S, T, true>, dim3(kRedBlocks), dim3(kRedThreads), 0, h->P, (const T*)u(h, 0), h->sc,
             h->par, h->cflpart);
    else
      launch(h, 5, k_cfl<S, T, false>, dim3(kRedBlocks), dim3(kRedThreads), 0, h->P, (const T*)u(h, 0), h->sc,
             h->par, h->cflpart);
  }
  static void force(rbdi_handle* h, const double* c) {
    hipLaunchKernelGGL((k_force_partial<S, T>), dim3(kRedBlocks), dim3(kRedThreads), 0, h->stream, h->P,
                       (const T*)u(h, 0), c[0], c[1], c[2], h->part);
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(kRedThreads), 0, h->stream, (const double*)h->part, kRedBlocks, 6,
                       h->red_out);
  }
  static void totals(rbdi_handle* h) {
    hipLaunchKernelGGL((k_totals_partial<S, T>), dim3(kRedBlocks), dim3(kRedThreads), 0, h->stream, h->P,
                       (const T*)u(h, 0), h->part);
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(kRedThreads), 0, h->stream, (const double*)h->part, kRedBlocks,
                       2 * S::NF, h->red_out);
  }
  // capacity for the CFL partials of any x-sweep block size up to kMaxWPB
  // wavefronts (a batch may choose another than the default)
  static int part_blocks(const Params& P) {
    const long long nseg = (P.n[0] + kOut - 1) / kOut;
    const long long segs = (nseg + kMaxWPB - 1) / kMaxWPB * kMaxWPB;
    return (int)std::max<long long>(segs * P.n[1] * P.n[2], kRedBlocks);
  }
  // D(U^n) into U[1] (rigid mask from r), for diagnostics
  static void rhs(rbdi_handle* h, int dirmask) {
    StepArgs A{};
    A.par = h->par;
    A.rhs_only = 1 | ((~dirmask & 7) << 1);
    const T* U0 = u(h, 0);
    if constexpr (S::D == 3) {
      sweep_t<2, 0, false>(h, U0, A, h->D);
      sweep_t<1, 0, false>(h, U0, A, h->D2);
    } else if constexpr (S::D == 2) {
      sweep_t<1, 0, false>(h, U0, A, h->D);
    }
    sweep_x(h, U0, U0, u(h, 1), A, 1.0, 0);
  }
  // One launch of a sweep of the middle RK stage of the last step, on that
  // step's buffers (inputs U(1), U^n, D; outputs D or U(2), which the next
  // step rewrites before reading): cls 0 x sweep, 1 y sweep, 2 z sweep.
  static void replay(rbdi_handle* h, int cls) {
    StepArgs A{};
    A.par = h->par ^ 1;
    const T* U1 = u(h, 1);
    if (cls == 0) sweep_x(h, U1, u(h, 0), u(h, 2), A, 0.25, 1);
    if constexpr (S::D >= 2)
      if (cls == 1) sweep_t<1, 0, false>(h, U1, A, S::D == 3 ? h->D2 : h->D);
    if constexpr (S::D == 3)
      if (cls == 2) sweep_t<2, 0, false>(h, U1, A, h->D);
  }
  // what: 0 face flux (dir), 1 closure, 2 solid sources
  static void unit(rbdi_handle* h, int what, int dir, const double* a, const double* b, double* out, int n) {
    const dim3 g((unsigned)((n + 63) / 64)), t(64);
    if (what == 0) {
      if (dir == 0) hipLaunchKernelGGL((k_unit_flux<S, T, 0>), g, t, 0, h->stream, h->P, a, b, out, n);
      else if (dir == 1 && S::D > 1) hipLaunchKernelGGL((k_unit_flux<S, T, (S::D > 1 ? 1 : 0)>), g, t, 0, h->stream, h->P, a, b, out, n);
      else if (dir == 2 && S::D > 2) hipLaunchKernelGGL((k_unit_flux<S, T, (S::D > 2 ? 2 : 0)>), g, t, 0, h->stream, h->P, a, b, out, n);
    } else if (what == 1) {
      hipLaunchKernelGGL((k_unit_closure<S, T>), g, t, 0, h->stream, h->P, a, out, n);
    } else {
      hipLaunchKernelGGL((k_unit_sources<S, T>), g, t, 0, h->stream, h->P, out, n);
    }
  }
  static const Ops* ops() {
    static const Ops o = {prim_to_state, state_to_prim, state_to_f64, f64_to_state, r_from_sdf, band, seed,
                          stages, cfl, force, totals, part_blocks, unit, rhs, replay};
    return &o;
  }
};

template <typename T>
const Ops* pick(int dim, int nmat, int solid) {
  if (!solid) {
    if (dim == 1 && nmat == 1) return Impl<Sys<1, 1, false>, T>::ops();
    if (dim == 1 && nmat == 2) return Impl<Sys<1, 2, false>, T>::ops();
    if (dim == 2 && nmat == 1) return Impl<Sys<2, 1, false>, T>::ops();
    if (dim == 2 && nmat == 2) return Impl<Sys<2, 2, false>, T>::ops();
    if (dim == 3 && nmat == 1) return Impl<Sys<3, 1, false>, T>::ops();
    if (dim == 3 && nmat == 2) return Impl<Sys<3, 2, false>, T>::ops();
  } else {
    if (dim == 1 && nmat == 2) return Impl<Sys<1, 2, true>, T>::ops();
    if (dim == 2 && nmat == 2) return Impl<Sys<2, 2, true>, T>::ops();
    if (dim == 3 && nmat == 2) return Impl<Sys<3, 2, true>, T>::ops();
  }
  return nullptr;
}

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RBDI_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return RBDI_OK;
}

void free_all(rbdi_handle* h) {
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
  for (auto& p : h->U)
    if (p) { (void)hipFree(p); p = nullptr; }
  void* ptrs[] = {h->D, h->D2, h->stage_buf, h->tasks, h->sc, h->part, h->red_out, h->cflpart};
  h->mlp = nullptr;
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  h->D = nullptr; h->D2 = nullptr; h->stage_buf = nullptr; h->tasks = nullptr; h->sc = nullptr; h->part = nullptr; h->red_out = nullptr;
  h->cflpart = nullptr;
}

}  // namespace

// Members of a batch are stepped and configured by the batch only.
static int free_member(const rbdi_handle* h) {
  if (h->owner) return fail(RBDI_ERR_NOT_READY, "the instance belongs to a batch");
  return RBDI_OK;
}

extern "C" {

RBDI_API const char* rbdi_last_error(void) { return g_err.c_str(); }

RBDI_API int rbdi_create(const rbdi_desc* d, rbdi_handle** out) {
  if (!d || !out) return fail(RBDI_ERR_BAD_ARG, "null desc or out");
  *out = nullptr;
  if (d->dim < 1 || d->dim > 3) return fail(RBDI_ERR_BAD_ARG, "dim must be 1..3");
  if (d->nmat < 1 || d->nmat > kMaxMat) return fail(RBDI_ERR_BAD_ARG, "nmat must be 1..2");
  if (d->precision != RBDI_FP64 && d->precision != RBDI_FP32) return fail(RBDI_ERR_BAD_ARG, "bad precision");
  long long ncell = 1;
  for (int a = 0; a < 3; ++a) {
    const int na = a < d->dim ? d->n[a] : 1;
    if (na < 1 || (a >= d->dim && d->n[a] != 1)) return fail(RBDI_ERR_BAD_ARG, "bad grid size");
    if (a < d->dim && !(d->dx[a] > 0.0)) return fail(RBDI_ERR_BAD_ARG, "dx must be positive");
    ncell *= na;
  }
  if (ncell >= (1LL << 31)) return fail(RBDI_ERR_BAD_ARG, "too many cells for 32-bit band indices");
  for (int q = 0; q < 6; ++q) {
    if (d->bc[q] < 0 || d->bc[q] > 3) return fail(RBDI_ERR_BAD_ARG, "bad boundary condition");
    if (q / 2 < d->dim && d->bc[q] == RBDI_BC_REFLECTIVE && d->n[q / 2] < kHalo)
      return fail(RBDI_ERR_BAD_ARG, "reflective boundary needs at least 3 cells");
    if (q / 2 < d->dim && (d->bc[q] == RBDI_BC_PERIODIC) != (d->bc[q ^ 1] == RBDI_BC_PERIODIC))
      return fail(RBDI_ERR_BAD_ARG, "periodic boundaries must be paired");
  }
  if (d->recon < 0 || d->recon > 1 || d->riemann < 0 || d->riemann > 1 || d->seed < 0 || d->seed > 2 ||
      d->probe < 0 || d->probe > 1 || d->normal < 0 || d->normal > 1)
    return fail(RBDI_ERR_BAD_ARG, "bad scheme option");
  if (d->normal == RBDI_NORMAL_ELVIRA && d->dim != 2) return fail(RBDI_ERR_BAD_ARG, "ELVIRA normals are 2D only");
  if (d->recon == RBDI_RECON_BVD_THINC && !(d->thinc_beta > 0.0)) return fail(RBDI_ERR_BAD_ARG, "thinc_beta must be > 0");
  if (d->riemann == RBDI_RIEMANN_HLLC_LM && !(d->lm_mach > 0.0)) return fail(RBDI_ERR_BAD_ARG, "lm_mach must be > 0");
  const Ops* ops = d->precision == RBDI_FP64 ? pick<double>(d->dim, d->nmat, d->solid)
                                             : pick<float>(d->dim, d->nmat, d->solid);
  if (!ops) return fail(RBDI_ERR_UNSUPPORTED, "no kernels for this (dim, nmat, solid) combination");

  rbdi_handle* h = new rbdi_handle();
  h->desc = *d;
  h->ops = ops;
  h->nf = 2 * d->nmat + d->dim + 1 + (d->solid ? 10 : 0);
  h->elem = d->precision == RBDI_FP64 ? 8 : 4;
  Params& P = h->P;
  std::memset(&P, 0, sizeof(P));
  P.dim = d->dim;
  P.dmin = 1e300;
  for (int a = 0; a < 3; ++a) {
    P.n[a] = a < d->dim ? d->n[a] : 1;
    P.dx[a] = a < d->dim ? d->dx[a] : 1.0;
    P.inv_dx[a] = 1.0 / P.dx[a];
    P.x0[a] = d->origin[a];
    if (a < d->dim) P.dmin = std::fmin(P.dmin, P.dx[a]);
  }
  P.st[0] = 1;
  P.st[1] = P.n[0];
  P.st[2] = (long long)P.n[0] * P.n[1];
  P.ncell = ncell;
  P.fs = (ncell + 63) / 64 * 64;
  for (int q = 0; q < 6; ++q) P.bc[q] = q / 2 < d->dim ? d->bc[q] : RBDI_BC_TRANSMISSIVE;
  P.recon = d->recon;
  P.riemann = d->riemann;
  P.seed = d->seed;
  P.probe = d->probe;
  P.normal = d->normal;
  P.plastic = d->plastic;
  P.beta = d->thinc_beta;
  P.cosh_b = std::cosh(d->thinc_beta);
  P.inv_sinh_b = 1.0 / std::sinh(d->thinc_beta);
  P.tanh_b = std::tanh(d->thinc_beta);
  P.lm_mach = d->lm_mach;
  P.solid_phase = -1;
  {
    double f = 1.0;
    for (int k = 0; k < 14; ++k) {
      if (k > 0) f *= (double)k;
      P.exc[k] = 1.0 / f;
    }
    const long double ln2 = 0.6931471805599453094172321214581766L;
    P.ln2_hi = std::ldexp(std::floor(std::ldexp((double)ln2, 32)), -32);  // k * ln2_hi exact for |k| < 2^20
    P.ln2_lo = (double)(ln2 - (long double)P.ln2_hi);
    P.inv_ln2 = (double)(1.0L / ln2);
  }

  const size_t state_bytes = (size_t)P.fs * h->nf * h->elem;
  hipError_t e = hipSuccess;
  for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipMalloc(&h->U[k], state_bytes);
  if (e == hipSuccess) e = hipMalloc(&h->D, state_bytes);
  if (e == hipSuccess && d->dim == 3) e = hipMalloc(&h->D2, state_bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&h->stage_buf, (size_t)ncell * h->nf * sizeof(double));
  h->task_cap = (int)std::max<long long>(4096, ncell / 4);
  if (e == hipSuccess) e = hipMalloc((void**)&h->tasks, (size_t)h->task_cap * sizeof(SeedTask));
  if (e == hipSuccess) e = hipMalloc((void**)&h->sc, sizeof(DevScalars));
  if (e == hipSuccess) e = hipMalloc((void**)&h->part, sizeof(double) * kRedBlocks * 2 * kMaxF);
  if (e == hipSuccess) e = hipMalloc((void**)&h->red_out, sizeof(double) * 2 * kMaxF);
  h->part_cap = ops->part_blocks(P);
  if (e == hipSuccess) e = hipMalloc((void**)&h->cflpart, sizeof(double) * h->part_cap);
  if (e != hipSuccess) {
    free_all(h);
    delete h;
    return fail(e == hipErrorOutOfMemory ? RBDI_ERR_OOM : RBDI_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  DevScalars zero{};
  zero.first_bad = -1;
  P.r_static = 1;
  P.nbody = 1;  // one body at rest until a motion is set
  e = hipMemcpy(h->sc, &zero, sizeof(zero), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(h->U[0], 0, state_bytes);
  if (e != hipSuccess) {
    free_all(h);
    delete h;
    return fail(RBDI_ERR_HIP, std::string("init: ") + hipGetErrorString(e));
  }
  *out = h;
  return RBDI_OK;
}

RBDI_API int rbdi_destroy(rbdi_handle* h) {
  if (!h) return fail(RBDI_ERR_BAD_ARG, "null handle");
  (void)hipStreamSynchronize(h->stream);
  free_all(h);
  delete h;
  return RBDI_OK;
}

RBDI_API int rbdi_nfields(const rbdi_handle* h) { return h ? h->nf : RBDI_ERR_BAD_ARG; }

RBDI_API int rbdi_set_stream(rbdi_handle* h, void* s) {
  if (!h) return fail(RBDI_ERR_BAD_ARG, "null handle");
  if (free_member(h)) return RBDI_ERR_NOT_READY;
  h->stream = static_cast<hipStream_t>(s);
  return RBDI_OK;
}

RBDI_API int rbdi_set_material(rbdi_handle* h, int l, const rbdi_eos* e) {
  if (!h || !e) return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (free_member(h)) return RBDI_ERR_NOT_READY;
  if (l < 0 || l >= h->desc.nmat) return fail(RBDI_ERR_BAD_ARG, "material index out of range");
  MatDev m{};
  m.kind = e->kind;
  if (e->kind == RBDI_EOS_IDEAL || e->kind == RBDI_EOS_STIFFENED) {
    if (!(e->gamma > 1.0)) return fail(RBDI_ERR_BAD_ARG, "gamma must be > 1");
    const double pinf = e->kind == RBDI_EOS_STIFFENED ? e->pinf : 0.0;
    if (!(pinf >= 0.0)) return fail(RBDI_ERR_BAD_ARG, "pinf must be >= 0");
    m.gamma = e->gamma;
    m.pinf = pinf;
    m.Gam = e->gamma - 1.0;
    m.invGam = 1.0 / m.Gam;
    m.Bfl = e->gamma * pinf / m.Gam;
    m.gGam = e->gamma / m.Gam;
  } else if (e->kind == RBDI_EOS_ROMENSKII) {
    if (!h->desc.solid) return fail(RBDI_ERR_BAD_ARG, "Romenskii material needs desc.solid = 1");
    if (!(e->rho0 > 0.0) || !(e->K0 >= 0.0) || !(e->G0 >= 0.0) || !(e->alpha > 0.0) || !(e->Gamma0 > 0.0) ||
        !(e->sigma_y >= 0.0))
      return fail(RBDI_ERR_BAD_ARG, "bad Romenskii parameters");
    m.rho0 = e->rho0;
    m.invrho0 = 1.0 / e->rho0;
    m.K0 = e->K0;
    m.G0 = e->G0;
    m.alpha = e->alpha;
    m.beta = e->beta;
    m.kc = e->K0 / (2.0 * e->alpha * e->alpha);
    // small integer exponents are evaluated by multiplication on the device
    m.ialpha = (e->alpha == std::floor(e->alpha) && e->alpha >= 1.0 && e->alpha <= 8.0) ? (int)e->alpha : 0;
    const double b1 = e->beta + 1.0;
    m.ibeta1 = (b1 == std::floor(b1) && b1 >= 1.0 && b1 <= 8.0) ? (int)b1 : 0;
    m.Gam = e->Gamma0;
    m.invGam = 1.0 / e->Gamma0;
    m.sigY = e->sigma_y;
    if (h->P.solid_phase < 0 || h->P.solid_phase == l) h->P.solid_phase = l;
  } else {
    return fail(RBDI_ERR_BAD_ARG, "unknown EOS kind");
  }
  h->P.mat[l] = m;
  h->have_mat[l] = true;
  h->P.stiff = 0;
  for (int k = 0; k < kMaxMat; ++k)
    if (h->P.mat[k].Bfl != 0.0) h->P.stiff = 1;
  return RBDI_OK;
}

static int ready_materials(rbdi_handle* h) {
  for (int l = 0; l < h->desc.nmat; ++l)
    if (!h->have_mat[l]) return fail(RBDI_ERR_NOT_READY, "set every material first");
  if (h->desc.solid && h->P.solid_phase < 0) return fail(RBDI_ERR_NOT_READY, "solid system needs a Romenskii material");
  return RBDI_OK;
}

RBDI_API int rbdi_set_bc_state(rbdi_handle* h, int face, const double* W) {
  if (!h || !W) return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (free_member(h)) return RBDI_ERR_NOT_READY;
  if (face < 0 || face > 5) return fail(RBDI_ERR_BAD_ARG, "face must be 0..5");
  for (int q = 0; q < h->nf; ++q) {
    if (!std::isfinite(W[q])) return fail(RBDI_ERR_BAD_ARG, "non-finite boundary state");
    h->P.bcW[face][q] = W[q];
  }
  return RBDI_OK;
}

RBDI_API int rbdi_set_face_modifier(rbdi_handle* h, int mode, const double* Wgap) {
  if (!h) return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (free_member(h)) return RBDI_ERR_NOT_READY;
  if (mode != 0 && mode != 1) return fail(RBDI_ERR_BAD_ARG, "face modifier mode must be 0 or 1");
  if (mode == 1 && !h->desc.solid) return fail(RBDI_ERR_BAD_ARG, "the face modifier needs an elastoplastic system");
  if (mode == 1 && !Wgap) return fail(RBDI_ERR_BAD_ARG, "null gap state");
  if (mode == 1)
    for (int q = 0; q < h->nf; ++q) {
      if (!std::isfinite(Wgap[q])) return fail(RBDI_ERR_BAD_ARG, "non-finite gap state");
      h->P.gapW[q] = Wgap[q];
    }
  h->P.face_mod = mode;
  return RBDI_OK;
}

static int stage_in(rbdi_handle* h, const double* src, int on_device) {
  const size_t bytes = (size_t)h->P.ncell * h->nf * sizeof(double);
  HIP_OK(hipMemcpyAsync(h->stage_buf, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        h->stream));
  return RBDI_OK;
}

RBDI_API int rbdi_set_state_prim(rbdi_handle* h, const double* W, int on_device) {
  if (!h || !W) return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (free_member(h)) return RBDI_ERR_NOT_READY;
  int rc = ready_materials(h);
  if (rc) return rc;
  rc = stage_in(h, W, on_device);
  if (rc) return rc;
  h->ops->prim_to_state(h, h->stage_buf);
  h->have_state = true;
  h->band_valid = false;
  h->cfl_valid = false;
  HIP_OK(hipStreamSynchronize(h->stream));
  return check_launch();
}

RBDI_API int rbdi_set_state_cons(rbdi_handle* h, const double* U, int on_device) {
  if (!h || !U) return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (free_member(h)) return RBDI_ERR_NOT_READY;
  int rc = ready_materials(h);
  if (rc) return rc;
  rc = stage_in(h, U, on_device);
  if (rc) return rc;
  h->ops->f64_to_state(h, h->stage_buf);
  h->have_state = true;
  h->band_valid = false;
  h->cfl_valid = false;
  HIP_OK(hipStreamSynchronize(h->stream));
  return check_launch();
}

static int stage_out(rbdi_handle* h, double* dst, int on_device) {
  const size_t bytes = (size_t)h->P.ncell * h->nf * sizeof(double);
  HIP_OK(hipMemcpyAsync(dst, h->stage_buf, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  return check_launch();
}

RBDI_API int rbdi_get_state_prim(rbdi_handle* h, double* W, int on_device) {
  if (!h || !W) return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (!h->have_state) return fail(RBDI_ERR_NOT_READY, "no state set");
  h->ops->state_to_prim(h, h->stage_buf);
  return stage_out(h, W, on_device);
}

RBDI_API int rbdi_get_state_cons(rbdi_handle* h, double* U, int on_device) {
  if (!h || !U) return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (!h->have_state) return fail(RBDI_ERR_NOT_READY, "no state set");
  h->ops->state_to_f64(h, h->stage_buf, 1);
  return stage_out(h, U, on_device);
}

RBDI_API int rbdi_set_rigid_sdf(rbdi_handle* h, const double* sdf, int on_device, double width, const double v[3],
                                const double omega[3], const double center[3]) {
  if (!h || !sdf || !v || !omega || !center) return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (free_member(h)) return RBDI_ERR_NOT_READY;
  if (!(width > 0.0)) return fail(RBDI_ERR_BAD_ARG, "width must be > 0");
  if (!h->have_state) return fail(RBDI_ERR_NOT_READY, "set the state before the rigid field");
  const size_t bytes = (size_t)h->P.ncell * sizeof(double);
  HIP_OK(hipMemcpyAsync(h->stage_buf, sdf, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        h->stream));
  h->ops->r_from_sdf(h, h->stage_buf, 1.0 / (width * h->P.dmin));
  int rc = rbdi_set_rigid_motion(h, v, omega, center);
  if (rc) return rc;
  h->band_valid = false;
  h->cfl_valid = false;
  HIP_OK(hipStreamSynchronize(h->stream));
  return check_launch();
}

__global__ void k_set_motion_time(DevScalars* sc, int par) { sc->t_motion = sc->t[par]; }

static_assert(RBDI_MAX_BODIES == kMaxBody, "the body table of the header and of the kernels differ");

RBDI_API int rbdi_set_rigid_bodies(rbdi_handle* h, int nbody, const double* v, const double* omega,
                                   const double* center, const double* box_lo, const double* box_hi) {
  if (!h || !v || !omega || !center || (nbody > 1 && (!box_lo || !box_hi)))
    return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (nbody < 1 || nbody > kMaxBody) return fail(RBDI_ERR_BAD_ARG, "nbody must be 1.." + std::to_string(kMaxBody));
  if (free_member(h)) return RBDI_ERR_NOT_READY;
  for (int k = 0; k < nbody; ++k)
    for (int a = 0; a < 3; ++a) {
      if (!std::isfinite(v[3 * k + a]) || !std::isfinite(omega[3 * k + a]) || !std::isfinite(center[3 * k + a]))
        return fail(RBDI_ERR_BAD_ARG, "non-finite rigid motion");
      if (k > 0 && (std::isnan(box_lo[3 * k + a]) || std::isnan(box_hi[3 * k + a])))
        return fail(RBDI_ERR_BAD_ARG, "NaN ownership box");
    }
  bool moving = false;
  h->P.nbody = nbody;
  for (int k = 0; k < kMaxBody; ++k)
    for (int a = 0; a < 3; ++a) {
      const bool on = k < nbody;
      h->P.vr[k][a] = on ? v[3 * k + a] : 0.0;
      h->P.om[k][a] = on ? omega[3 * k + a] : 0.0;
      h->P.ctr[k][a] = on ? center[3 * k + a] : 0.0;
      h->P.blo[k][a] = (on && k > 0) ? box_lo[3 * k + a] : -HUGE_VAL;
      h->P.bhi[k][a] = (on && k > 0) ? box_hi[3 * k + a] : HUGE_VAL;
      moving = moving || (on && (v[3 * k + a] != 0.0 || omega[3 * k + a] != 0.0));
    }
  h->dynamic_r = moving;
  h->P.r_static = moving ? 0 : 1;
  h->cfl_valid = false;
  hipLaunchKernelGGL(k_set_motion_time, dim3(1), dim3(1), 0, h->stream, h->sc, h->par);
  return check_launch();
}

RBDI_API int rbdi_set_rigid_motion(rbdi_handle* h, const double v[3], const double omega[3], const double center[3]) {
  return rbdi_set_rigid_bodies(h, 1, v, omega, center, nullptr, nullptr);
}

// One step: (CFL minimum if stale) -> band (once for a static body) ->
// seeding -> three stages of sweeps. The first kernel of the step does the
// step bookkeeping on the device.
static void enqueue_step(rbdi_handle* h, double dt_fixed, double cfl, double t_end) {
  if (dt_fixed <= 0.0 && !h->cfl_valid) h->ops->cfl(h);
  StepArgs A{};
  A.par = h->par;
  A.cfl = cfl;
  A.t_end = t_end;
  A.dt_fixed = dt_fixed;
  if (h->P.seed != RBDI_SEED_NONE) {
    if (!h->band_valid || h->dynamic_r) {
      h->ops->band(h, A);
      h->band_valid = true;
    }
    h->ops->seed(h, A);
  }
  h->ops->stages(h, A);
  h->par ^= 1;
  h->cfl_valid = true;
  h->enqueued += 1;
}

RBDI_API int rbdi_step(rbdi_handle* h, double dt) {
  if (!h) return fail(RBDI_ERR_BAD_ARG, "null handle");
  if (free_member(h)) return RBDI_ERR_NOT_READY;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RBDI_ERR_BAD_ARG, "dt must be positive and finite");
  if (!h->have_state) return fail(RBDI_ERR_NOT_READY, "no state set");
  enqueue_step(h, dt, 0.0, 0.0);
  return check_launch();
}

RBDI_API int rbdi_compute_dt(rbdi_handle* h, double cfl, double* dt) {
  if (!h || !dt) return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (!(cfl > 0.0)) return fail(RBDI_ERR_BAD_ARG, "cfl must be > 0");
  if (!h->have_state) return fail(RBDI_ERR_NOT_READY, "no state set");
  if (!h->cfl_valid) {
    h->ops->cfl(h);
    h->cfl_valid = true;
  }
  hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(256), 0, h->stream, (const double*)h->cflpart,
                     (const DevScalars*)h->sc, h->red_out);
  double m = 0.0;
  HIP_OK(hipMemcpyAsync(&m, h->red_out, sizeof(m), hipMemcpyDeviceToHost, h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  int rc = check_launch();
  if (rc) return rc;
  *dt = m > 0.0 ? cfl / m : 0.0;
  if (!std::isfinite(*dt) || !(*dt > 0.0)) return fail(RBDI_ERR_NONPHYSICAL, "no finite CFL time step");
  return RBDI_OK;
}

RBDI_API int rbdi_advance(rbdi_handle* h, double cfl, int nsteps, double t_end) {
  if (!h) return fail(RBDI_ERR_BAD_ARG, "null handle");
  if (free_member(h)) return RBDI_ERR_NOT_READY;
  if (!(cfl > 0.0) || nsteps < 0) return fail(RBDI_ERR_BAD_ARG, "cfl must be > 0 and nsteps >= 0");
  if (!h->have_state) return fail(RBDI_ERR_NOT_READY, "no state set");
  for (int s = 0; s < nsteps; ++s) enqueue_step(h, 0.0, cfl, t_end);
  return check_launch();
}

RBDI_API int rbdi_unit_eval(rbdi_handle* h, int what, int dir, const double* a, const double* b, double* out,
                           int n) {
  if (!h || !a || !out || n < 0 || what < 0 || what > 2) return fail(RBDI_ERR_BAD_ARG, "bad unit_eval argument");
  if (what == 0 && (!b || dir < 0 || dir >= h->desc.dim)) return fail(RBDI_ERR_BAD_ARG, "bad flux direction");
  if (n == 0) return RBDI_OK;
  const int nf = h->nf, nt = nf - 1;
  const size_t in_n = (size_t)n * nf;
  const size_t out_n = (size_t)n * (what == 0 ? nt + 4 : (what == 1 ? nf + 10 : nf));
  double *da = nullptr, *db = nullptr, *dout = nullptr;
  HIP_OK(hipMalloc(&da, in_n * sizeof(double)));
  HIP_OK(hipMalloc(&db, in_n * sizeof(double)));
  HIP_OK(hipMalloc(&dout, out_n * sizeof(double)));
  HIP_OK(hipMemcpyAsync(da, a, in_n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  if (what == 0) HIP_OK(hipMemcpyAsync(db, b, in_n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  if (what == 2) HIP_OK(hipMemcpyAsync(dout, a, in_n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  h->ops->unit(h, what, dir, da, db, dout, n);
  HIP_OK(hipMemcpyAsync(out, dout, out_n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  int rc = check_launch();
  (void)hipFree(da);
  (void)hipFree(db);
  (void)hipFree(dout);
  return rc;
}

RBDI_API int rbdi_eval_rhs(rbdi_handle* h, int dirmask, double* D) {
  if (!h || !D) return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (!h->have_state) return fail(RBDI_ERR_NOT_READY, "no state set");
  h->ops->rhs(h, dirmask);
  // D sits in state buffer 1; convert it through the staging buffer
  std::swap(h->U[0], h->U[1]);
  h->ops->state_to_f64(h, h->stage_buf, 0);
  std::swap(h->U[0], h->U[1]);
  const size_t bytes = (size_t)h->P.ncell * h->nf * sizeof(double);
  HIP_OK(hipMemcpyAsync(D, h->stage_buf, bytes, hipMemcpyDeviceToHost, h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  return check_launch();
}

RBDI_API int rbdi_set_kernel_timing(rbdi_handle* h, int enable) {
  if (!h) return fail(RBDI_ERR_BAD_ARG, "null handle");
  h->timing = enable != 0;
  return RBDI_OK;
}

RBDI_API int rbdi_kernel_times(rbdi_handle* h, double* ms, long long* launches) {
  if (!h || !ms || !launches) return fail(RBDI_ERR_BAD_ARG, "null argument");
  HIP_OK(hipStreamSynchronize(h->stream));
  for (size_t k = 0; k < h->ev_used; ++k) {
    float e = 0.0f;
    HIP_OK(hipEventElapsedTime(&e, h->ev[2 * k], h->ev[2 * k + 1]));
    const int c = h->ev_cls[k];
    ms[c] += e;
    launches[c] += 1;
  }
  h->ev_used = 0;
  return RBDI_OK;
}

RBDI_API int rbdi_kernel_replay(rbdi_handle* h, int cls, int reps, double* us) {
  if (!h || !us || reps < 1 || cls < 0 || cls > 2) return fail(RBDI_ERR_BAD_ARG, "bad kernel_replay argument");
  if (cls >= h->desc.dim) return fail(RBDI_ERR_BAD_ARG, "no sweep along that direction");
  if (h->owner || h->enqueued < 1) return fail(RBDI_ERR_NOT_READY, "replay needs a step of this handle first");
  const bool was = h->timing;
  h->timing = false;
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  h->ops->replay(h, cls);
  HIP_OK(hipEventRecord(e0, h->stream));
  for (int r = 0; r < reps; ++r) h->ops->replay(h, cls);
  HIP_OK(hipEventRecord(e1, h->stream));
  HIP_OK(hipEventSynchronize(e1));
  h->timing = was;
  float ms = 0.0f;
  HIP_OK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *us = 1e3 * ms / reps;
  return check_launch();
}

RBDI_API int rbdi_set_x_waves(rbdi_handle* h, int waves) {
  if (!h) return fail(RBDI_ERR_BAD_ARG, "null handle");
  if (free_member(h)) return RBDI_ERR_NOT_READY;
  if (waves != 0 && waves != 1 && waves != 2 && waves != 4) return fail(RBDI_ERR_BAD_ARG, "x waves must be 0, 1, 2 or 4");
  if (h->desc.dim == 1 && waves > 1) return fail(RBDI_ERR_BAD_ARG, "1D x sweeps run one wavefront per block");
  h->x_waves = waves;
  return RBDI_OK;
}

RBDI_API int rbdi_autotune(rbdi_handle* h, double cfl, int nsteps, int* best, double* us) {
  if (!h || !best || !us || nsteps < 1 || !(cfl > 0.0)) return fail(RBDI_ERR_BAD_ARG, "bad autotune argument");
  if (free_member(h)) return RBDI_ERR_NOT_READY;
  if (!h->have_state) return fail(RBDI_ERR_NOT_READY, "no state set");
  // everything a step changes that a later step reads: the state (U^n and
  // the buffer order), the device scalars, the CFL partials, and the
  // host-side step bookkeeping
  const size_t state_bytes = (size_t)h->P.fs * h->nf * h->elem;
  const size_t part_bytes = sizeof(double) * (size_t)h->part_cap;
  char* save = nullptr;
  HIP_OK(hipMalloc((void**)&save, state_bytes + part_bytes + sizeof(DevScalars)));
  void* const u_order[3] = {h->U[0], h->U[1], h->U[2]};
  const int par = h->par, x0 = h->x_waves;
  const bool cfl_valid = h->cfl_valid, band_valid = h->band_valid, timing = h->timing;
  const long long enq = h->enqueued;
  int rc = RBDI_OK;
  auto copy = [&](bool out) -> int {
    char* p = save;
    void* dst[3] = {p, p + state_bytes, p + state_bytes + part_bytes};
    void* src[3] = {h->U[0], h->cflpart, h->sc};
    const size_t sz[3] = {state_bytes, part_bytes, sizeof(DevScalars)};
    for (int k = 0; k < 3; ++k)
      if (hipMemcpyAsync(out ? dst[k] : src[k], out ? src[k] : dst[k], sz[k], hipMemcpyDeviceToDevice, h->stream) !=
          hipSuccess)
        return fail(RBDI_ERR_HIP, "autotune state copy");
    return RBDI_OK;
  };
  rc = copy(true);
  const int cands[3] = {1, 2, 4};
  const int ncand = h->desc.dim == 1 ? 1 : 3;
  double best_us = 0.0;
  int best_w = 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = fail(RBDI_ERR_HIP, "autotune events");
  h->timing = false;
  for (int c = 0; c < ncand && !rc; ++c) {
    h->x_waves = h->desc.dim == 1 ? 0 : cands[c];
    if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = fail(RBDI_ERR_HIP, "autotune event"); break; }
    for (int s = 0; s < nsteps; ++s) enqueue_step(h, 0.0, cfl, 0.0);
    if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      rc = fail(RBDI_ERR_HIP, "autotune timing");
      break;
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double t = 1e3 * ms / nsteps;
    if (c == 0 || t < best_us) { best_us = t; best_w = h->desc.dim == 1 ? 1 : cands[c]; }
    // back to the state before the call
    for (int k = 0; k < 3; ++k) h->U[k] = u_order[k];
    h->par = par;
    h->cfl_valid = cfl_valid;
    h->band_valid = band_valid;
    h->enqueued = enq;
    if (!rc) rc = copy(false);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  h->timing = timing;
  if (hipStreamSynchronize(h->stream) != hipSuccess && !rc) rc = fail(RBDI_ERR_HIP, "autotune sync");
  (void)hipFree(save);
  if (rc) {
    h->x_waves = x0;
    return rc;
  }
  h->x_waves = h->desc.dim == 1 ? 0 : best_w;
  *best = best_w;
  *us = best_us;
  return check_launch();
}

RBDI_API int rbdi_status(rbdi_handle* h, rbdi_stats* st) {
  if (!h || !st) return fail(RBDI_ERR_BAD_ARG, "null argument");
  DevScalars s{};
  HIP_OK(hipMemcpyAsync(&s, h->sc, sizeof(s), hipMemcpyDeviceToHost, h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  st->steps = s.steps;
  st->t = s.t[h->par];
  st->last_dt = s.last_dt;
  st->band_cells = (long long)s.band_count + s.band_fail;
  st->seeded = s.seeded;
  st->probe_fail = s.band_fail;
  st->nonphysical = s.nonphys;
  st->first_bad = s.nonphys ? s.first_bad : -1;
  st->surr_net = s.surr_net;
  st->surr_exact = s.surr_exact;
  int rc = check_launch();
  if (rc) return rc;
  if (s.nonphys) return fail(RBDI_ERR_NONPHYSICAL, "a cell left the admissible set");
  if (s.band_count > h->task_cap) return fail(RBDI_ERR_OOM, "rigid band exceeds the seeding task capacity");
  return RBDI_OK;
}

RBDI_API int rbdi_rigid_force(rbdi_handle* h, const double center[3], double F[3], double T[3]) {
  if (!h || !center || !F || !T) return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (!h->have_state) return fail(RBDI_ERR_NOT_READY, "no state set");
  h->ops->force(h, center);
  double out[6];
  HIP_OK(hipMemcpyAsync(out, h->red_out, sizeof(out), hipMemcpyDeviceToHost, h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  for (int a = 0; a < 3; ++a) { F[a] = out[a]; T[a] = out[3 + a]; }
  return check_launch();
}

RBDI_API int rbdi_conserved_totals(rbdi_handle* h, double* out) {
  if (!h || !out) return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (!h->have_state) return fail(RBDI_ERR_NOT_READY, "no state set");
  h->ops->totals(h);
  HIP_OK(hipMemcpyAsync(out, h->red_out, sizeof(double) * 2 * h->nf, hipMemcpyDeviceToHost, h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  return check_launch();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched instances
// ---------------------------------------------------------------------------

namespace {

struct BatchOps;

}  // namespace

struct rbdi_batch {
  std::vector<rbdi_handle*> m;
  const BatchOps* ops = nullptr;
  int dim = 0, nf = 0, elem = 8;
  hipStream_t stream = nullptr;
  void* inst = nullptr;          // BatchInst<T>[count] (device)
  BatchItem* items = nullptr;    // seed | x | y | z item lists (device)
  size_t item_cap = 0;
  int n_seed = 0, n_x = 0, n_y = 0, n_z = 0;
  int off_x = 0, off_y = 0, off_z = 0;
  double* dtfix = nullptr;       // per-member fixed dt (device)
  double* dtfix_host = nullptr;  // pinned staging of dtfix
  int flip = 0;
  rbdi_tuning tune{};
};

namespace {

int lds_ok(const rbdi_batch* b, int tc) { return (size_t)b->nf * tc * kRS * b->elem <= 65536; }

struct BatchOps {
  void (*fill)(rbdi_batch*, const std::vector<int>& ntask, std::vector<unsigned char>&);
  void (*seed)(rbdi_batch*, const BatchArgs&, int grid);
  // which: 0 first sweep of the step (reduces dt), 1 first sweep of a later
  // stage, 2 second sweep (3D: y after z, accumulating)
  void (*tile)(rbdi_batch*, int dir, int which, const BatchArgs&, int grid, int tc);
  void (*xsweep)(rbdi_batch*, const BatchArgs&, int grid, int wpb);
};

template <class S, typename T>
struct BImpl {
  static void fill(rbdi_batch* b, const std::vector<int>& ntask, std::vector<unsigned char>& out) {
    out.assign(sizeof(BatchInst<T>) * b->m.size(), 0);
    BatchInst<T>* t = reinterpret_cast<BatchInst<T>*>(out.data());
    for (size_t i = 0; i < b->m.size(); ++i) {
      rbdi_handle* h = b->m[i];
      BatchInst<T> bi{};
      bi.P = h->P;
      for (int k = 0; k < 3; ++k) bi.U[k] = static_cast<T*>(h->U[k]);
      bi.D = static_cast<T*>(h->D);
      bi.sc = h->sc;
      bi.cflpart = h->cflpart;
      bi.tasks = h->tasks;
      bi.ntask = ntask[i];
      bi.par0 = h->par;
      std::memcpy(&t[i], &bi, sizeof(bi));
    }
  }
  static void seed(rbdi_batch* b, const BatchArgs& B, int grid) {
    hipLaunchKernelGGL((kb_seed<S, T>), dim3(grid), dim3(256), 0, b->stream, (const BatchInst<T>*)b->inst,
                       (const BatchItem*)b->items, B);
  }
  template <int DIR, int MODE, bool REDUCE>
  static void tile_l(rbdi_batch* b, const BatchArgs& B, int grid, int tc, const BatchItem* items) {
    const size_t lds = (size_t)S::NF * tc * kRS * sizeof(T);
    hipLaunchKernelGGL((kb_sweep_tile<S, T, DIR, MODE, REDUCE>), dim3(grid), dim3(kTileThreads), lds, b->stream,
                       (const BatchInst<T>*)b->inst, items, B, tc);
  }
  static void tile(rbdi_batch* b, int dir, int which, const BatchArgs& B, int grid, int tc) {
    const BatchItem* it = b->items + (dir == 1 ? b->off_y : b->off_z);
    if constexpr (S::D == 3) {
      if (dir == 2 && which == 0) tile_l<2, 0, true>(b, B, grid, tc, it);
      else if (dir == 2) tile_l<2, 0, false>(b, B, grid, tc, it);
      else tile_l<1, 1, false>(b, B, grid, tc, it);
    } else {
      if (which == 0) tile_l<1, 0, true>(b, B, grid, tc, it);
      else tile_l<1, 0, false>(b, B, grid, tc, it);
    }
  }
  static void xsweep(rbdi_batch* b, const BatchArgs& B, int grid, int wpb) {
    hipLaunchKernelGGL((kb_sweep_x<S, T>), dim3(grid), dim3(kWave * wpb), 0, b->stream,
                       (const BatchInst<T>*)b->inst, (const BatchItem*)(b->items + b->off_x), B);
  }
  static const BatchOps* ops() {
    static const BatchOps o = {fill, seed, tile, xsweep};
    return &o;
  }
};

template <typename T>
const BatchOps* pick_batch(int dim, int nmat, int solid) {
  if (solid) return nullptr;
  if (dim == 2 && nmat == 1) return BImpl<Sys<2, 1, false>, T>::ops();
  if (dim == 2 && nmat == 2) return BImpl<Sys<2, 2, false>, T>::ops();
  if (dim == 3 && nmat == 1) return BImpl<Sys<3, 1, false>, T>::ops();
  if (dim == 3 && nmat == 2) return BImpl<Sys<3, 2, false>, T>::ops();
  return nullptr;
}

// Tile lists of the current tuning, members in order of decreasing size (the
// largest instances' tiles are taken first by a persistent grid).
int batch_build_items(rbdi_batch* b, const std::vector<int>& ntask) {
  std::vector<int> order(b->m.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return b->m[a]->P.ncell > b->m[c]->P.ncell; });
  std::vector<BatchItem> seed, xs, ys, zs;
  const int wpb = b->tune.x_waves, tc = b->tune.tile_cols;
  for (int i : order) {
    const Params& P = b->m[i]->P;
    for (int t0 = 0; t0 < ntask[i]; t0 += 256) seed.push_back(BatchItem{i, t0, 0, 0, 0, {0, 0}});
    const int gx = ((P.n[0] + kOut - 1) / kOut + wpb - 1) / wpb, gy = P.n[1], gz = P.n[2];
    for (int z = 0; z < gz; ++z)
      for (int y = 0; y < gy; ++y)
        for (int x = 0; x < gx; ++x)
          xs.push_back(BatchItem{i, x, y, z, ((long long)z * gy + y) * gx + x, {0, 0}});
    const int tx = (P.n[0] + tc - 1) / tc;
    const int sy = (P.n[1] + kOut - 1) / kOut;
    for (int z = 0; z < P.n[2]; ++z)
      for (int y = 0; y < sy; ++y)
        for (int x = 0; x < tx; ++x) ys.push_back(BatchItem{i, x, y, z, 0, {0, 0}});
    if (b->dim == 3) {
      const int sz = (P.n[2] + kOut - 1) / kOut;
      for (int z = 0; z < sz; ++z)
        for (int y = 0; y < P.n[1]; ++y)
          for (int x = 0; x < tx; ++x) zs.push_back(BatchItem{i, x, y, z, 0, {0, 0}});
    }
  }
  b->n_seed = (int)seed.size();
  b->n_x = (int)xs.size();
  b->n_y = (int)ys.size();
  b->n_z = (int)zs.size();
  b->off_x = b->n_seed;
  b->off_y = b->off_x + b->n_x;
  b->off_z = b->off_y + b->n_y;
  const size_t total = (size_t)b->off_z + b->n_z;
  std::vector<BatchItem> all;
  all.reserve(total);
  all.insert(all.end(), seed.begin(), seed.end());
  all.insert(all.end(), xs.begin(), xs.end());
  all.insert(all.end(), ys.begin(), ys.end());
  all.insert(all.end(), zs.begin(), zs.end());
  HIP_OK(hipStreamSynchronize(b->stream));
  if (total > b->item_cap) {
    if (b->items) (void)hipFree(b->items);
    b->items = nullptr;
    b->item_cap = 0;
    HIP_OK(hipMalloc((void**)&b->items, total * sizeof(BatchItem)));
    b->item_cap = total;
  }
  if (total) HIP_OK(hipMemcpy(b->items, all.data(), total * sizeof(BatchItem), hipMemcpyHostToDevice));
  return RBDI_OK;
}

int batch_ntask(rbdi_batch* b, std::vector<int>& ntask) {
  ntask.assign(b->m.size(), 0);
  for (size_t i = 0; i < b->m.size(); ++i) {
    rbdi_handle* h = b->m[i];
    if (h->P.seed == RBDI_SEED_NONE) continue;
    DevScalars s{};
    HIP_OK(hipMemcpy(&s, h->sc, sizeof(s), hipMemcpyDeviceToHost));
    if (s.band_count > h->task_cap) return fail(RBDI_ERR_OOM, "rigid band exceeds the seeding task capacity");
    ntask[i] = s.band_count;
  }
  return RBDI_OK;
}

int batch_tables(rbdi_batch* b) {
  std::vector<int> ntask;
  int rc = batch_ntask(b, ntask);
  if (rc) return rc;
  std::vector<unsigned char> tab;
  b->ops->fill(b, ntask, tab);
  HIP_OK(hipStreamSynchronize(b->stream));
  if (!b->inst) HIP_OK(hipMalloc(&b->inst, tab.size()));
  HIP_OK(hipMemcpy(b->inst, tab.data(), tab.size(), hipMemcpyHostToDevice));
  b->flip = 0;
  return batch_build_items(b, ntask);
}

int check_tuning(const rbdi_batch* b, const rbdi_tuning& t) {
  if (t.x_waves != 1 && t.x_waves != 2 && t.x_waves != 4) return fail(RBDI_ERR_BAD_ARG, "x_waves must be 1, 2 or 4");
  if (t.tile_cols != 4 && t.tile_cols != 8 && t.tile_cols != 16 && t.tile_cols != 32)
    return fail(RBDI_ERR_BAD_ARG, "tile_cols must be 4, 8, 16 or 32");
  if (!lds_ok(b, t.tile_cols)) return fail(RBDI_ERR_BAD_ARG, "tile_cols exceeds 64 KiB of LDS for this system");
  if (t.x_blocks < 0 || t.t_blocks < 0 || t.x_blocks > (1 << 20) || t.t_blocks > (1 << 20))
    return fail(RBDI_ERR_BAD_ARG, "bad persistent grid size");
  return RBDI_OK;
}

inline int grid_of(int blocks, int nitems) { return blocks > 0 ? std::min(blocks, nitems) : nitems; }

void batch_enqueue_step(rbdi_batch* b, double cfl, double t_end, bool fixed) {
  BatchArgs B{};
  B.flip = b->flip;
  B.cfl = cfl;
  B.t_end = t_end;
  B.dtfix = fixed ? b->dtfix : nullptr;
  if (b->n_seed) {
    B.nitems = b->n_seed;
    B.xcd = 0;
    b->ops->seed(b, B, b->n_seed);
  }
  const double bc[3] = {1.0, 0.25, 2.0 / 3.0};
  const int in_[3] = {0, 1, 2}, out_[3] = {1, 2, 0};
  for (int s = 0; s < 3; ++s) {
    B.in = in_[s];
    B.out = out_[s];
    B.stage = s;
    B.bcoef = bc[s];
    B.xcd = b->tune.t_xcd;
    if (b->dim == 3) {
      B.nitems = b->n_z;
      b->ops->tile(b, 2, s == 0 ? 0 : 1, B, grid_of(b->tune.t_blocks, b->n_z), b->tune.tile_cols);
      B.nitems = b->n_y;
      b->ops->tile(b, 1, 2, B, grid_of(b->tune.t_blocks, b->n_y), b->tune.tile_cols);
    } else {
      B.nitems = b->n_y;
      b->ops->tile(b, 1, s == 0 ? 0 : 1, B, grid_of(b->tune.t_blocks, b->n_y), b->tune.tile_cols);
    }
    B.nitems = b->n_x;
    B.xcd = b->tune.x_xcd;
    b->ops->xsweep(b, B, grid_of(b->tune.x_blocks, b->n_x), b->tune.x_waves);
  }
  b->flip ^= 1;
  for (rbdi_handle* h : b->m) {
    h->par ^= 1;
    h->cfl_valid = true;
  }
}

void batch_free(rbdi_batch* b) {
  if (b->inst) (void)hipFree(b->inst);
  if (b->items) (void)hipFree(b->items);
  if (b->dtfix) (void)hipFree(b->dtfix);
  if (b->dtfix_host) (void)hipHostFree(b->dtfix_host);
  b->inst = nullptr;
  b->items = nullptr;
  b->dtfix = nullptr;
  b->dtfix_host = nullptr;
}

}  // namespace

extern "C" {

RBDI_API int rbdi_batch_create(int count, rbdi_handle* const* members, rbdi_batch** out) {
  if (!members || !out || count < 1) return fail(RBDI_ERR_BAD_ARG, "need count >= 1 members and out");
  *out = nullptr;
  const rbdi_handle* h0 = members[0];
  if (!h0) return fail(RBDI_ERR_BAD_ARG, "null member");
  for (int i = 0; i < count; ++i) {
    const rbdi_handle* h = members[i];
    if (!h) return fail(RBDI_ERR_BAD_ARG, "null member");
    for (int j = 0; j < i; ++j)
      if (members[j] == h) return fail(RBDI_ERR_BAD_ARG, "a member appears twice");
    if (h->desc.dim != h0->desc.dim || h->desc.nmat != h0->desc.nmat || h->desc.solid != h0->desc.solid ||
        h->desc.precision != h0->desc.precision)
      return fail(RBDI_ERR_BAD_ARG, "members must share dim, nmat, solid and precision");
    if (h->owner) return fail(RBDI_ERR_NOT_READY, "a member already belongs to a batch");
    if (!h->have_state) return fail(RBDI_ERR_NOT_READY, "a member has no state");
    if (h->dynamic_r) return fail(RBDI_ERR_UNSUPPORTED, "batched members must have static bodies");
  }
  const BatchOps* ops = h0->desc.precision == RBDI_FP64
                            ? pick_batch<double>(h0->desc.dim, h0->desc.nmat, h0->desc.solid)
                            : pick_batch<float>(h0->desc.dim, h0->desc.nmat, h0->desc.solid);
  if (!ops) return fail(RBDI_ERR_UNSUPPORTED, "batches support 2D/3D fluid systems");
  rbdi_batch* b = new rbdi_batch();
  b->m.assign(members, members + count);
  b->ops = ops;
  b->dim = h0->desc.dim;
  b->nf = h0->nf;
  b->elem = h0->elem;
  b->stream = h0->stream;
  b->tune.x_waves = kWPB;
  b->tune.tile_cols = b->elem == 8 ? 16 : 32;
  while (!lds_ok(b, b->tune.tile_cols)) b->tune.tile_cols /= 2;
  if (b->tune.tile_cols < 4) {
    delete b;
    return fail(RBDI_ERR_UNSUPPORTED, "system too wide for an LDS tile");
  }
  // members on the batch stream; static bands and CFL partials ready
  for (rbdi_handle* h : b->m) {
    h->stream = b->stream;
    if (h->P.seed != RBDI_SEED_NONE && !h->band_valid) {
      StepArgs A{};
      A.par = h->par;
      h->ops->band(h, A);
      h->band_valid = true;
    }
    if (!h->cfl_valid) {
      h->ops->cfl(h);
      h->cfl_valid = true;
    }
  }
  hipError_t e = hipMalloc((void**)&b->dtfix, sizeof(double) * count);
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->dtfix_host, sizeof(double) * count);
  if (e != hipSuccess) {
    batch_free(b);
    delete b;
    return fail(RBDI_ERR_OOM, std::string("batch allocation: ") + hipGetErrorString(e));
  }
  int rc = check_launch();
  if (!rc) rc = batch_tables(b);
  if (rc) {
    batch_free(b);
    delete b;
    return rc;
  }
  for (rbdi_handle* h : b->m) h->owner = b;
  *out = b;
  return RBDI_OK;
}

RBDI_API int rbdi_batch_destroy(rbdi_batch* b) {
  if (!b) return fail(RBDI_ERR_BAD_ARG, "null batch");
  (void)hipStreamSynchronize(b->stream);
  for (rbdi_handle* h : b->m) h->owner = nullptr;
  batch_free(b);
  delete b;
  return RBDI_OK;
}

RBDI_API int rbdi_batch_set_stream(rbdi_batch* b, void* s) {
  if (!b) return fail(RBDI_ERR_BAD_ARG, "null batch");
  b->stream = static_cast<hipStream_t>(s);
  for (rbdi_handle* h : b->m) h->stream = b->stream;
  return RBDI_OK;
}

RBDI_API int rbdi_batch_set_tuning(rbdi_batch* b, const rbdi_tuning* t) {
  if (!b || !t) return fail(RBDI_ERR_BAD_ARG, "null argument");
  int rc = check_tuning(b, *t);
  if (rc) return rc;
  const bool relist = t->x_waves != b->tune.x_waves || t->tile_cols != b->tune.tile_cols;
  b->tune = *t;
  if (!relist) return RBDI_OK;
  std::vector<int> ntask;
  rc = batch_ntask(b, ntask);
  if (rc) return rc;
  return batch_build_items(b, ntask);
}

RBDI_API int rbdi_batch_get_tuning(const rbdi_batch* b, rbdi_tuning* t) {
  if (!b || !t) return fail(RBDI_ERR_BAD_ARG, "null argument");
  *t = b->tune;
  return RBDI_OK;
}

RBDI_API int rbdi_batch_step(rbdi_batch* b, double cfl, const double* dts) {
  if (!b) return fail(RBDI_ERR_BAD_ARG, "null batch");
  const int n = (int)b->m.size();
  bool need_cfl = dts == nullptr;
  if (dts)
    for (int i = 0; i < n; ++i) {
      if (!std::isfinite(dts[i])) return fail(RBDI_ERR_BAD_ARG, "non-finite dt");
      need_cfl = need_cfl || !(dts[i] > 0.0);
    }
  if (need_cfl && !(cfl > 0.0)) return fail(RBDI_ERR_BAD_ARG, "cfl must be > 0 for CFL steps");
  if (dts) {
    HIP_OK(hipStreamSynchronize(b->stream));  // the previous upload has been consumed
    std::memcpy(b->dtfix_host, dts, sizeof(double) * n);
    HIP_OK(hipMemcpyAsync(b->dtfix, b->dtfix_host, sizeof(double) * n, hipMemcpyHostToDevice, b->stream));
  }
  batch_enqueue_step(b, cfl, 0.0, dts != nullptr);
  return check_launch();
}

RBDI_API int rbdi_batch_advance(rbdi_batch* b, double cfl, int nsteps, double t_end) {
  if (!b) return fail(RBDI_ERR_BAD_ARG, "null batch");
  if (!(cfl > 0.0) || nsteps < 0) return fail(RBDI_ERR_BAD_ARG, "cfl must be > 0 and nsteps >= 0");
  for (int s = 0; s < nsteps; ++s) batch_enqueue_step(b, cfl, t_end, false);
  return check_launch();
}

RBDI_API int rbdi_batch_autotune(rbdi_batch* b, int reps, rbdi_tuning* best) {
  if (!b || reps < 1) return fail(RBDI_ERR_BAD_ARG, "null batch or reps < 1");
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  rbdi_tuning cur = b->tune;
  // the operator of the current state: tile sweeps into D, x sweep into the
  // stage buffer U[1]; nothing a step reads before writing it
  BatchArgs B{};
  B.flip = b->flip;
  B.cfl = 1.0;
  B.in = 0;
  B.out = 1;
  B.stage = 0;
  B.bcoef = 1.0;
  B.rhs_only = 1;
  const int grids[4] = {0, 512, 1024, 2048};
  auto time_it = [&](auto&& launch, double& us) -> int {
    launch();
    HIP_OK(hipEventRecord(e0, b->stream));
    for (int r = 0; r < reps; ++r) launch();
    HIP_OK(hipEventRecord(e1, b->stream));
    HIP_OK(hipEventSynchronize(e1));
    int rc = check_launch();
    if (rc) return rc;
    float ms = 0.0f;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    us = 1e3 * ms / reps;
    return RBDI_OK;
  };
  std::vector<int> ntask;
  int rc = batch_ntask(b, ntask);
  double best_t = 1e300, best_x = 1e300;
  rbdi_tuning bt = cur;
  // y/z sweeps: tile width x grid x XCD ranges
  for (int tc : {4, 8, 16, 32}) {
    if (rc || !lds_ok(b, tc)) continue;
    b->tune.tile_cols = tc;
    rc = batch_build_items(b, ntask);
    for (int g : grids)
      for (int xcd = 0; xcd < (g ? 2 : 1) && !rc; ++xcd) {
        double us = 0.0;
        rc = time_it(
            [&]() {
              B.xcd = xcd;
              if (b->dim == 3) {
                B.nitems = b->n_z;
                b->ops->tile(b, 2, 1, B, grid_of(g, b->n_z), tc);
                B.nitems = b->n_y;
                b->ops->tile(b, 1, 2, B, grid_of(g, b->n_y), tc);
              } else {
                B.nitems = b->n_y;
                b->ops->tile(b, 1, 1, B, grid_of(g, b->n_y), tc);
              }
            },
            us);
        if (!rc && us < best_t) {
          best_t = us;
          bt.tile_cols = tc;
          bt.t_blocks = g;
          bt.t_xcd = xcd;
        }
      }
  }
  for (int wpb : {1, 2, 4}) {
    if (rc) break;
    b->tune.x_waves = wpb;
    rc = batch_build_items(b, ntask);
    for (int g : grids)
      for (int xcd = 0; xcd < (g ? 2 : 1) && !rc; ++xcd) {
        double us = 0.0;
        rc = time_it(
            [&]() {
              B.xcd = xcd;
              B.nitems = b->n_x;
              b->ops->xsweep(b, B, grid_of(g, b->n_x), wpb);
            },
            us);
        if (!rc && us < best_x) {
          best_x = us;
          bt.x_waves = wpb;
          bt.x_blocks = g;
          bt.x_xcd = xcd;
        }
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    b->tune = cur;
    (void)batch_build_items(b, ntask);
    return rc;
  }
  bt.x_us = best_x;
  bt.t_us = best_t;
  b->tune = bt;
  rc = batch_build_items(b, ntask);
  if (rc) return rc;
  if (best) *best = bt;
  return RBDI_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Surrogate network (training, inference) and its use in the step
// ---------------------------------------------------------------------------

namespace {

// Partial gradient rows of rbdi_mlp_grad_noalloc: one row (kNParam gradients
// + the loss) per 64-sample block, kNoAllocRows rows, in a fixed device array
// (9.4 MB) that each GPU the library runs on holds until the process ends.
// Host code never passes `scratch` itself to a kernel (on the host the name
// stands for a host-side shadow, not a device address): it uses the address
// hipGetSymbolAddress returns for the current device, resolved once per
// device and kept in g_scratch.
constexpr int kNoAllocRows = RBDI_MLP_GRAD_NOALLOC_MAX / 64;
static __device__ __align__(256) float scratch[(size_t)kNoAllocRows * (kNParam + 1)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch[kMaxDevices] = {};

// Device address of the current device's scratch array (resolved on the
// first call on that device).
int scratch_address(float** out) {
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(RBDI_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(RBDI_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = static_cast<float*>(p);
  }
  *out = g_scratch[dev];
  return RBDI_OK;
}

void mlp_free(rbdi_mlp* m) {
  void* ptrs[] = {m->blob, m->bias, m->master, m->m1, m->m2, m->sum};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  m->blob = nullptr; m->bias = nullptr; m->master = nullptr; m->m1 = nullptr; m->m2 = nullptr; m->sum = nullptr;
}

// Device copy of n x w host floats (caller frees).
template <typename X>
int upload(const X* src, size_t n, X** dst) {
  *dst = nullptr;
  if (n == 0) return RBDI_OK;
  HIP_OK(hipMalloc((void**)dst, n * sizeof(X)));
  HIP_OK(hipMemcpy(*dst, src, n * sizeof(X), hipMemcpyHostToDevice));
  return RBDI_OK;
}

}  // namespace

extern "C" {

RBDI_API int rbdi_mlp_create(rbdi_mlp** out) {
  if (!out) return fail(RBDI_ERR_BAD_ARG, "null out");
  rbdi_mlp* m = new rbdi_mlp();
  hipError_t e = hipMalloc((void**)&m->blob, sizeof(__bf16) * kBlobBf16);
  if (e == hipSuccess) e = hipMalloc((void**)&m->bias, sizeof(float) * kBiasN);
  if (e == hipSuccess) e = hipMalloc((void**)&m->master, sizeof(float) * kNParam);
  if (e == hipSuccess) e = hipMalloc((void**)&m->m1, sizeof(float) * kNParam);
  if (e == hipSuccess) e = hipMalloc((void**)&m->m2, sizeof(float) * kNParam);
  if (e == hipSuccess) e = hipMalloc((void**)&m->sum, sizeof(float) * (kNParam + 1));
  if (e == hipSuccess) e = hipMemset(m->blob, 0, sizeof(__bf16) * kBlobBf16);
  if (e == hipSuccess) e = hipMemset(m->bias, 0, sizeof(float) * kBiasN);
  if (e == hipSuccess) e = hipMemset(m->master, 0, sizeof(float) * kNParam);
  if (e == hipSuccess) e = hipMemset(m->m1, 0, sizeof(float) * kNParam);
  if (e == hipSuccess) e = hipMemset(m->m2, 0, sizeof(float) * kNParam);
  if (e != hipSuccess) {
    mlp_free(m);
    delete m;
    return fail(RBDI_ERR_OOM, std::string("mlp allocation: ") + hipGetErrorString(e));
  }
  // set-up of rbdi_mlp_grad_noalloc on this device
  float* sp = nullptr;
  if (const int rc = scratch_address(&sp)) {
    mlp_free(m);
    delete m;
    return rc;
  }
  *out = m;
  return RBDI_OK;
}

RBDI_API int rbdi_mlp_destroy(rbdi_mlp* m) {
  if (!m) return fail(RBDI_ERR_BAD_ARG, "null network");
  (void)hipDeviceSynchronize();
  mlp_free(m);
  delete m;
  return RBDI_OK;
}

RBDI_API int rbdi_mlp_set_params(rbdi_mlp* m, const float* params, double tau_max) {
  if (!m || !params) return fail(RBDI_ERR_BAD_ARG, "null argument");
  if (!(tau_max > 0.0) || !(tau_max < 1.0)) return fail(RBDI_ERR_BAD_ARG, "tau_max must be in (0, 1)");
  for (int p = 0; p < kNParam; ++p)
    if (!std::isfinite(params[p])) return fail(RBDI_ERR_BAD_ARG, "non-finite parameter");
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipMemcpy(m->master, params, sizeof(float) * kNParam, hipMemcpyHostToDevice));
  HIP_OK(hipMemset(m->m1, 0, sizeof(float) * kNParam));
  HIP_OK(hipMemset(m->m2, 0, sizeof(float) * kNParam));
  m->tau_max = tau_max;
  m->step = 0;
  hipLaunchKernelGGL(k_mlp_sync, dim3((kNParam + 255) / 256), dim3(256), 0, nullptr, (const float*)m->master,
                     m->blob, m->bias);
  HIP_OK(hipDeviceSynchronize());
  return check_launch();
}

RBDI_API int rbdi_mlp_get_params(rbdi_mlp* m, float* params, double* tau_max) {
  if (!m || !params) return fail(RBDI_ERR_BAD_ARG, "null argument");
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipMemcpy(params, m->master, sizeof(float) * kNParam, hipMemcpyDeviceToHost));
  if (tau_max) *tau_max = m->tau_max;
  return RBDI_OK;
}

RBDI_API int rbdi_mlp_forward(rbdi_mlp* m, const float* z, int n, float* y) {
  if (!m || !z || !y || n < 0) return fail(RBDI_ERR_BAD_ARG, "bad mlp_forward argument");
  if (n == 0) return RBDI_OK;
  float *dz = nullptr, *dy = nullptr;
  int rc = upload(z, (size_t)n * 6, &dz);
  if (!rc && hipMalloc((void**)&dy, sizeof(float) * 6 * (size_t)n) != hipSuccess) rc = fail(RBDI_ERR_OOM, "mlp_forward");
  if (!rc) {
    hipLaunchKernelGGL(k_mlp_infer, dim3((n + 255) / 256), dim3(256), 0, nullptr, mlp_dev(m), (const float*)dz, dy, n);
    if (hipMemcpy(y, dy, sizeof(float) * 6 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) rc = fail(RBDI_ERR_HIP, "mlp_forward copy");
    if (!rc) rc = check_launch();
  }
  if (dz) (void)hipFree(dz);
  if (dy) (void)hipFree(dy);
  return rc;
}

RBDI_API int rbdi_mlp_grad(rbdi_mlp* m, const float* z, const float* t, int n, float* grad, float* loss) {
  if (!m || !z || !t || !grad || !loss || n < 1) return fail(RBDI_ERR_BAD_ARG, "bad mlp_grad argument");
  const int nb = (n + 63) / 64;
  float *dz = nullptr, *dt = nullptr, *part = nullptr;
  int rc = upload(z, (size_t)n * 6, &dz);
  if (!rc) rc = upload(t, (size_t)n * 6, &dt);
  if (!rc && hipMalloc((void**)&part, sizeof(float) * (size_t)nb * (kNParam + 1)) != hipSuccess) rc = fail(RBDI_ERR_OOM, "mlp_grad");
  if (!rc) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(64), 0, nullptr, mlp_dev(m), (const float*)dz, (const float*)dt,
                       0LL, n, n, part);
    hipLaunchKernelGGL(k_mlp_sum, dim3((kNParam + 256) / 256), dim3(256), 0, nullptr, (const float*)part, nb, m->sum,
                       m->sum + kNParam);
    std::vector<float> h(kNParam + 1);
    if (hipMemcpy(h.data(), m->sum, sizeof(float) * (kNParam + 1), hipMemcpyDeviceToHost) != hipSuccess)
      rc = fail(RBDI_ERR_HIP, "mlp_grad copy");
    if (!rc) rc = check_launch();
    if (!rc) {
      std::memcpy(grad, h.data(), sizeof(float) * kNParam);
      *loss = h[kNParam];
    }
  }
  if (dz) (void)hipFree(dz);
  if (dt) (void)hipFree(dt);
  if (part) (void)hipFree(part);
  return rc;
}

RBDI_API int rbdi_mlp_grad_noalloc(rbdi_mlp* m, const float* z, const float* t, int n, float* grad, float* loss,
                                   void* hip_stream) {
  if (!m || !z || !t || !grad || !loss) return fail(RBDI_ERR_BAD_ARG, "null mlp_grad_noalloc argument");
  if (n < 1 || n > RBDI_MLP_GRAD_NOALLOC_MAX)
    return fail(RBDI_ERR_BAD_ARG, "mlp_grad_noalloc: n = " + std::to_string(n) + " outside [1, " +
                                      std::to_string(RBDI_MLP_GRAD_NOALLOC_MAX) + "]");
  float* part = nullptr;
  if (const int rc = scratch_address(&part)) return rc;
  const hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int nb = (n + 63) / 64;
  // every block writes its whole partial row: nothing to clear
  hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(64), 0, st, mlp_dev(m), z, t, 0LL, n, n, part);
  hipLaunchKernelGGL(k_mlp_sum, dim3((kNParam + 256) / 256), dim3(256), 0, st, (const float*)part, nb, grad, loss);
  return check_launch();
}

RBDI_API int rbdi_mlp_train(rbdi_mlp* m, const float* z, const float* t, int n, int batch, int iters, float lr,
                            float* losses) {
  if (!m || !z || !t || n < 1 || batch < 64 || iters < 0 || !(lr > 0.0f))
    return fail(RBDI_ERR_BAD_ARG, "bad mlp_train argument");
  if (batch % 64) return fail(RBDI_ERR_BAD_ARG, "batch must be a multiple of 64");
  const int nb = batch / 64;
  float *dz = nullptr, *dt = nullptr, *part = nullptr, *dl = nullptr;
  int rc = upload(z, (size_t)n * 6, &dz);
  if (!rc) rc = upload(t, (size_t)n * 6, &dt);
  if (!rc && hipMalloc((void**)&part, sizeof(float) * (size_t)nb * (kNParam + 1)) != hipSuccess) rc = fail(RBDI_ERR_OOM, "mlp_train");
  if (!rc && hipMalloc((void**)&dl, sizeof(float) * std::max(iters, 1)) != hipSuccess) rc = fail(RBDI_ERR_OOM, "mlp_train");
  long long start = 0;
  for (int it = 0; it < iters && !rc; ++it) {
    // consecutive slices of the (caller-shuffled) samples, cyclically
    if (start >= n) start = 0;
    const int cnt = (int)std::min<long long>(batch, n - start);
    const int nbi = (cnt + 63) / 64;
    hipLaunchKernelGGL(k_mlp_grad, dim3(nbi), dim3(64), 0, nullptr, mlp_dev(m), (const float*)dz, (const float*)dt,
                       start, cnt, cnt, part);
    AdamArgs a;
    a.lr = lr * 0.5f * (1.0f + cosf(3.14159265f * (float)it / (float)iters));
    a.beta1 = 0.9f;
    a.beta2 = 0.999f;
    a.eps = 1e-8f;
    a.step = ++m->step;
    hipLaunchKernelGGL(k_mlp_adam, dim3((kNParam + 256) / 256), dim3(256), 0, nullptr, (const float*)part, nbi,
                       m->master, m->m1, m->m2, m->blob, m->bias, a, dl + it);
    start += cnt;
  }
  if (!rc) rc = check_launch();
  if (!rc && losses && iters > 0 &&
      hipMemcpy(losses, dl, sizeof(float) * iters, hipMemcpyDeviceToHost) != hipSuccess)
    rc = fail(RBDI_ERR_HIP, "mlp_train copy");
  if (!rc && hipDeviceSynchronize() != hipSuccess) rc = fail(RBDI_ERR_HIP, "mlp_train sync");
  if (dz) (void)hipFree(dz);
  if (dt) (void)hipFree(dt);
  if (part) (void)hipFree(part);
  if (dl) (void)hipFree(dl);
  return rc;
}

RBDI_API int rbdi_mlp_data(const double* V, int n, double tau_max, float* z, float* t) {
  if (!V || !z || !t || n < 0 || !(tau_max > 0.0)) return fail(RBDI_ERR_BAD_ARG, "bad mlp_data argument");
  if (n == 0) return RBDI_OK;
  double* dV = nullptr;
  float *dz = nullptr, *dt = nullptr;
  int rc = upload(V, (size_t)n * 9, &dV);
  if (!rc && (hipMalloc((void**)&dz, sizeof(float) * 6 * (size_t)n) != hipSuccess ||
              hipMalloc((void**)&dt, sizeof(float) * 6 * (size_t)n) != hipSuccess))
    rc = fail(RBDI_ERR_OOM, "mlp_data");
  if (!rc) {
    hipLaunchKernelGGL(k_mlp_data, dim3((n + 255) / 256), dim3(256), 0, nullptr, (const double*)dV, n, tau_max, dz, dt);
    if (hipMemcpy(z, dz, sizeof(float) * 6 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(t, dt, sizeof(float) * 6 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess)
      rc = fail(RBDI_ERR_HIP, "mlp_data copy");
    if (!rc) rc = check_launch();
  }
  if (dV) (void)hipFree(dV);
  if (dz) (void)hipFree(dz);
  if (dt) (void)hipFree(dt);
  return rc;
}

RBDI_API int rbdi_set_surrogate(rbdi_handle* h, rbdi_mlp* m) {
  if (!h) return fail(RBDI_ERR_BAD_ARG, "null handle");
  if (free_member(h)) return RBDI_ERR_NOT_READY;
  if (m && !h->desc.solid) return fail(RBDI_ERR_UNSUPPORTED, "the surrogate closes the elastoplastic system only");
  h->mlp = m;
  h->P.surr = m ? 1 : 0;
  return RBDI_OK;
}

}  // extern "C"
