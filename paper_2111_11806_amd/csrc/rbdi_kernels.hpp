// rbdi_kernels.hpp -- gfx950 kernels of the diffuse-interface rigid-body
// step (arXiv 2111.11806): direction sweeps of the semi-discrete operator with
// the SSP-RK3 combine fused into the last sweep (Sec. 3.1), rigid-band
// compaction and interface seeding (Sec. 3.2), the CFL reduction (Sec. 3),
// FP64 force/torque and conservation reductions, and state conversions.
//
// Storage: structure of arrays over interior cells, field q at base + q*fs,
// cell (i,j,k) at i + j*nx + k*nx*ny. Domain ghost cells are not stored:
// a load outside the domain maps to its boundary source on the fly.
//
// Sweep mapping: one wavefront (64 lanes) owns 64 consecutive cells along the
// sweep direction, of which the middle 58 are updated (3-cell halo each
// side, the width of the MUSCL-BVD-THINC stencil). Neighbour values travel by
// cross-lane shuffles: each cell's closure, reconstruction candidates and
// face flux are computed once.
#pragma once

#include "rbdi_physics.hpp"

namespace rbdi {

constexpr int kWave = 64;
constexpr int kOut = 58;       // cells updated per wavefront
constexpr int kHalo = 3;
constexpr int kWPB = 4;        // wavefronts per block in 2D/3D x sweeps (default)
constexpr int kMaxWPB = 4;     // largest x-sweep block (partial capacity)
constexpr int kTileThreads = 256;  // block size of the y/z tile sweeps

// Device-resident scalars of one instance. Per-step values live in two
// slots indexed by the parity of the step: during step n (parity p) slot p
// holds t_n and, once the first sweep of the step has reduced the CFL
// partials, dt_n; that reduction also writes t_{n+1} into slot p^1, which
// nothing else reads during step n.
struct DevScalars {
  double t[2];        // time at the start of the step of each parity
  double dtv[2];      // dt of the step of each parity
  double t_motion;    // time at which the rigid centre was set
  double last_dt;
  long long steps;
  long long seeded;
  long long first_bad;
  int nonphys;
  int band_count;     // seeding tasks of the current band
  int band_fail;      // band cells without a valid probe
  int npart;          // CFL partials written by their last producer
  long long surr_net;    // plastic-return cells closed by the surrogate
  long long surr_exact;  // ... by the exact closure (outside its envelope / flagged)
};

// Host-side arguments of one step.
struct StepArgs {
  int par;          // parity of the step
  double cfl;       // CFL number (device dt)
  double t_end;     // clip time (<= 0: none)
  double dt_fixed;  // > 0: use this dt instead of the CFL value
  int rhs_only;     // bit 0: the final sweep stores D(U_in) itself; bits 1-3:
                    // directions x, y, z left out of it (diagnostics)
};

// A step at or after t_end does no work.
__device__ inline bool step_done(const DevScalars* sc, const StepArgs& a) {
  if (a.dt_fixed > 0.0 || !(a.t_end > 0.0)) return false;
  return !(a.t_end - sc->t[a.par] > 1e-14 * a.t_end);
}

// dt of the step: the fixed value, or cfl divided by the maximum of the CFL
// partials (max over fluid cells and directions of max(|u_d| + c, |v_r,d|) /
// dx_d), clipped at t_end; 0 (no work) once t_end is reached or when no
// fluid cell exists. Run by one whole block (a max is exact and order
// independent), which also does the step bookkeeping.
__device__ inline void reduce_dt(DevScalars* sc, const double* __restrict__ part, const StepArgs& a) {
  __shared__ double sh[16];
  double m = 0.0;
  if (!(a.dt_fixed > 0.0)) {
    const int np = sc->npart;
    for (int q = threadIdx.x; q < np; q += blockDim.x) m = fmax(m, part[q]);
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) m = fmax(m, sh[q]);
    double dt = a.dt_fixed > 0.0 ? a.dt_fixed : (m > 0.0 ? a.cfl / m : 0.0);
    if (step_done(sc, a)) dt = 0.0;
    else if (a.t_end > 0.0 && !(a.dt_fixed > 0.0) && dt > a.t_end - sc->t[a.par]) dt = a.t_end - sc->t[a.par];
    if (!(dt < 1e299)) dt = 0.0;
    sc->dtv[a.par] = dt;
    sc->t[a.par ^ 1] = sc->t[a.par] + dt;
    if (dt > 0.0) {
      sc->steps += 1;
      sc->last_dt = dt;
    }
  }
}

// Single-block reduction kernel (used when no sweep precedes the one that
// needs dt: 1D systems).
__global__ void k_reduce_dt(DevScalars* sc, const double* __restrict__ part, StepArgs a) { reduce_dt(sc, part, a); }

// Neighbour exchange along the wavefront by DPP whole-wave shifts (a VALU
// move instead of an LDS permute): shup gives lane i the value of lane i-1,
// shdn that of lane i+1. With Z the end lanes read zero (bound_ctrl), so the
// move needs no copy of an old value into its destination; otherwise they
// keep their own value. Lanes 0 and 63 are halo lanes: with the 3-lane halo
// no updated lane depends on what they read (every loop of the per-cell
// arithmetic has a fixed trip bound, and no address depends on the data).
// Measured: Z takes 2.6% off a 2D single-gas step; the 18-field
// elastoplastic sweeps run 8% slower with it (register allocation), so they
// keep the copying form.
template <bool Z>
__device__ inline int dpp_shr1(int v) {
  if constexpr (Z) return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
  else return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false);
}
template <bool Z>
__device__ inline int dpp_shl1(int v) {
  if constexpr (Z) return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true);
  else return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false);
}

template <bool Z>
__device__ inline float shup(float v) { return __builtin_bit_cast(float, dpp_shr1<Z>(__builtin_bit_cast(int, v))); }
template <bool Z>
__device__ inline float shdn(float v) { return __builtin_bit_cast(float, dpp_shl1<Z>(__builtin_bit_cast(int, v))); }
template <bool Z>
__device__ inline double shup(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_shr1<Z>((int)(b & 0xffffffffLL)), hi = dpp_shr1<Z>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
template <bool Z>
__device__ inline double shdn(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_shl1<Z>((int)(b & 0xffffffffLL)), hi = dpp_shl1<Z>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Keeps a value's computation where it stands in the program: an empty asm
// that reads and writes the register. Without it the compiler sinks every
// field's BVD selection to the end of the unrolled per-field loop, so all
// fields' candidates and shifted neighbour faces stay live at once (18
// fields: 256 registers and 74 spilled per lane, against 126 with it).
template <typename T>
__device__ inline void pin(T& x) {
  asm volatile("" : "+v"(x));
}

__device__ inline long long cell_index(const Params& P, int i, int j, int k) {
  return (long long)i * P.st[0] + (long long)j * P.st[1] + (long long)k * P.st[2];
}

// Boundary mapping of a position along direction d. Returns 0 (use the source
// cell as is), 1 (mirror: negate the normal velocity and the normal-
// tangential stretch components) or 2 (Dirichlet state of the face).
__device__ inline int ghost_map(const Params& P, int d, int pos, int& src, int& face) {
  const int n = P.n[d];
  if (pos >= 0 && pos < n) { src = pos; face = -1; return 0; }
  const int side = pos < 0 ? 0 : 1;
  face = 2 * d + side;
  switch (P.bc[face]) {
    case BC_REFLECTIVE: src = side ? 2 * n - 1 - pos : -1 - pos; return 1;
    case BC_PERIODIC: src = ((pos % n) + n) % n; return 0;
    case BC_DIRICHLET: src = 0; return 2;
    default: src = side ? n - 1 : 0; return 0;
  }
}

template <class S, typename T>
__device__ inline void load_cons(const Params& P, const T* __restrict__ U, long long c, T* Uc) {
#pragma unroll
  for (int q = 0; q < S::NF; ++q) Uc[q] = U[q * P.fs + c];
}

// Primitive state at (i,j,k) where the coordinate along DIR may lie in the
// ghost range.
template <class S, typename T, int DIR>
__device__ inline void load_prim(const Params& P, const T* __restrict__ U, int i, int j, int k, T* W) {
  int p[3] = {i, j, k};
  int src, face;
  const int mode = ghost_map(P, DIR, p[DIR], src, face);
  if (mode == 2) {
#pragma unroll
    for (int q = 0; q < S::NF; ++q) W[q] = (T)P.bcW[face][q];
    return;
  }
  p[DIR] = src;
  T Uc[S::NF];
  load_cons<S>(P, U, cell_index(P, p[0], p[1], p[2]), Uc);
  cons_to_prim<S>(P, Uc, W);
  if (mode == 1) {
    W[S::wU(DIR)] = -W[S::wU(DIR)];
    if constexpr (S::S) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          if ((a == DIR) != (b == DIR)) W[S::wV(a, b)] = -W[S::wV(a, b)];
    }
  }
}

// r at a face-neighbour of an interior cell (ghosts by the boundary map).
template <class S, typename T>
__device__ inline double r_at(const Params& P, const T* __restrict__ U, int i, int j, int k, int d, int off) {
  int p[3] = {i, j, k};
  int src, face;
  const int mode = ghost_map(P, d, p[d] + off, src, face);
  if (mode == 2) return P.bcW[face][S::R];
  p[d] = src;
  return (double)U[S::R * P.fs + cell_index(P, p[0], p[1], p[2])];
}

// ---------------------------------------------------------------------------
// Direction sweeps of one RK stage.
// ---------------------------------------------------------------------------

// CFL signal rate of one cell: max_d max(|u_d| + c, |v_r,d|) / dx_d
// (dt = cfl / max over fluid cells; mixture sound speed of Sec. 2.2). With
// adm, also whether the cell's state is admissible: positive phasic
// densities, volume fractions in [0,1], a positive mixture sound speed
// squared (a phase present only in trace may sit outside its own
// admissible range, as trace air inside water under tension), a finite rate.
template <class S, typename T, bool MB = false>
__device__ inline double cfl_rate(const Params& P, const T* Uc, const double* x, double tc, bool* adm = nullptr) {
  T W[S::NF];
  double J2 = 0.0;
  cons_to_prim<S>(P, Uc, W, nullptr, &J2);
  double phi[kMaxMat], rl[kMaxMat], c2, G, sY;
  phases_w<S>(W, phi, rl);
  mix_c2_G<S>(P, phi, rl, J2, (double)W[S::wP], c2, G, sY);
  if (adm) {
    bool ok = c2 > 0.0;
#pragma unroll
    for (int l = 0; l < S::N; ++l) ok = ok && rl[l] > 0.0 && phi[l] >= 0.0 && phi[l] <= 1.0;
    *adm = ok;
  }
  const double cs = sqrt(c2);
  double v[3];
  rigid_velocity<MB>(P, x, tc, v);
  double m = 0.0;
#pragma unroll
  for (int d = 0; d < S::D; ++d) m = fmax(m, fmax(fabs((double)W[S::wU(d)]) + cs, fabs(v[d])) * P.inv_dx[d]);
  if (adm) *adm = *adm && isfinite(m);
  return m;
}

// The per-cell work of a sweep along DIR on a wavefront whose lanes hold 64
// consecutive cells (lane order = position order): MUSCL-BVD-THINC of every
// primitive (Sec. 3.1; r skipped when it never changes, its flux being zero
// then), first-order fallback of inadmissible cells, HLLC at the face to
// the right of each cell, the upwind r flux, and this direction's part of
// D = (F_+ - F_-)/dx - s_non-con (Sec. 3.1) for the cell. All lanes execute
// it (cross-lane shuffles); only lanes 3..60 get a complete d.
template <class S, typename T, int DIR, bool MB = false>
__device__ inline void sweep_core(const Params& P, const T* W, int pos, const int* pc, double tc, T* d) {
  constexpr bool Z = !S::S;  // zero-filling shifts (see dpp_shr1)
  T sL[S::NF], sR[S::NF];
#pragma unroll
  for (int q = 0; q < S::NF; ++q) {
    if (q == S::R && P.r_static) { sL[q] = W[q]; sR[q] = W[q]; continue; }
    const T wm = shup<Z>(W[q]), wp = shdn<Z>(W[q]);
    const Cand<T> c = candidates(P, wm, W[q], wp);
    const T lmR = shup<Z>(c.mR), ltR = shup<Z>(c.tR);
    const T rmL = shdn<Z>(c.mL), rtL = shdn<Z>(c.tL);
    bvd(P, lmR, ltR, c, rmL, rtL, sL[q], sR[q]);
  }
  // first-order fallback; skipped by the whole wavefront when no lane needs
  // it (the common case) instead of selects on every lane (1.3% off a 2D
  // FP64 step)
  const bool bad = !admissible<S>(P, sL) || !admissible<S>(P, sR);
  if (__any(bad)) {
#pragma unroll
    for (int q = 0; q < S::NF; ++q) {
      sL[q] = bad ? W[q] : sL[q];
      sR[q] = bad ? W[q] : sR[q];
    }
  }
  // face pos+1/2: left state = this cell's right face, right state = the
  // next cell's left face
  T WR[S::NF];
#pragma unroll
  for (int q = 0; q < S::NF; ++q) WR[q] = shdn<Z>(sL[q]);
  T F[S::NT], us, Vs[3] = {T(0), T(0), T(0)};
  hllc<S, DIR>(P, sR, WR, F, us, Vs);
  T vf = T(0), rfl = T(0);
  if (!P.r_static) {
    double xf[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xf[a] = a < S::D ? P.x0[a] + (pc[a] + 0.5) * P.dx[a] : 0.0;
    xf[DIR] = P.x0[DIR] + (pos + 1) * P.dx[DIR];
    double v[3];
    rigid_velocity<MB>(P, xf, tc, v);
    vf = (T)v[DIR];
    rfl = vf > T(0) ? sR[S::R] * vf : (vf < T(0) ? WR[S::R] * vf : T(0));
  }
  // the left face of this cell is the previous lane's right face
  T Fm[S::NT];
#pragma unroll
  for (int q = 0; q < S::NT; ++q) Fm[q] = shup<Z>(F[q]);
  const T usm = shup<Z>(us), vfm = shup<Z>(vf), rflm = shup<Z>(rfl);
  T Vsm[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) Vsm[b] = shup<Z>(Vs[b]);
  const T inv = (T)P.inv_dx[DIR];
#pragma unroll
  for (int q = 0; q < S::NT; ++q) d[q] = (F[q] - Fm[q]) * inv;
  const T du = us - usm;
#pragma unroll
  for (int l = 0; l < S::N - 1; ++l) d[S::cPHI(l)] -= W[S::wPHI(l)] * du * inv;
  if (P.stiff) {  // the energy slot holds E~ = rho E - B(phi)
    double phi[kMaxMat], rl[kMaxMat];
    phases_w<S>(W, phi, rl);
    d[S::cE] += (T)(mix_B<S>(P, phi) * (double)(du * inv));
  }
  if constexpr (S::S) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T ua = a < S::D ? W[S::wU(a)] : T(0);
#pragma unroll
      for (int b = 0; b < 3; ++b)
        d[S::cV(a, b)] -= (T(2.0 / 3.0) * W[S::wV(a, b)] * du - ua * (Vs[b] - Vsm[b])) * inv;
    }
  }
  d[S::R] = ((rfl - rflm) - W[S::R] * (vf - vfm)) * inv;
}

// Dimensions whose elastoplastic sweeps carry the void-opening face modifier.
#ifndef RBDI_FACE_MOD_DIMS
#define RBDI_FACE_MOD_DIMS 3
#endif
constexpr int kFaceModDims = RBDI_FACE_MOD_DIMS;

// Void-opening face modifier (Sec. 3.2, end) on the face states of a face
// whose two cells lie on either side of the rigid surface,
// (0.5 - r_L)(0.5 - r_R) < 0, taken as one cell rigid (r > 0.5) and the other
// not, a cell with r = 0.5 being a material cell as everywhere else (cross;
// real_left: the material cell is the left one). The rigid side's state becomes the mirror image of the material
// side's (normal velocity reflected about the rigid velocity, Vbar conjugated
// by the reflection): an exact wall. Where the normal traction on that wall's
// contact (from the left state of the fan) is tensile, the solid is let go:
// the rigid side becomes the gap gas (P.gapW, moving with the body's normal
// velocity, at rest tangentially), which flows into the opening gap. r keeps
// its face values (its flux is formed apart).
template <class S, int DIR, bool MB, typename T>
__device__ inline void face_modifier(const Params& P, int pos, const int* pc, double tc, bool cross, bool real_left,
                                     T* sR, T* WR) {
  double v[3] = {0.0, 0.0, 0.0};
  if (!P.r_static) {
    double xf[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xf[a] = a < S::D ? P.x0[a] + (pc[a] + 0.5) * P.dx[a] : 0.0;
    xf[DIR] = P.x0[DIR] + (pos + 1) * P.dx[DIR];
    rigid_velocity<MB>(P, xf, tc, v);
  }
  const T vd = (T)v[DIR];
#pragma unroll
  for (int q = 0; q < S::R; ++q) {
    const T re = real_left ? sR[q] : WR[q];
    T m = re;
    if (q == S::wU(DIR)) m = T(2) * vd - re;
    if constexpr (S::S) {
      if (q >= S::wV(0, 0) && q < S::wEP) {
        const int a = (q - S::wV(0, 0)) / 3, b = (q - S::wV(0, 0)) % 3;
        if ((a == DIR) != (b == DIR)) m = -re;
      }
    }
    WR[q] = (cross && real_left) ? m : WR[q];
    sR[q] = (cross && !real_left) ? m : sR[q];
  }
  HllcFace<S, DIR, T> f;
  f.init(P, sR, WR);
  const bool open = cross && (f.L.P + f.L.rho * (f.SL - f.L.un) * (f.Ss - f.L.un)) < 0.0;
  if (__any(open)) {
#pragma unroll
    for (int q = 0; q < S::R; ++q) {
      T g = (T)P.gapW[q];
#pragma unroll
      for (int a = 0; a < S::D; ++a)
        if (q == S::wU(a)) g = a == DIR ? vd : T(0);
      WR[q] = (open && real_left) ? g : WR[q];
      sR[q] = (open && !real_left) ? g : sR[q];
    }
  }
}

// sweep_core for the elastoplastic system, with the same results: the face
// solver's wave data are built once, then each field's flux, its difference
// with the left neighbour's and its non-conservative terms are formed one
// field at a time and handed to put(q, d_q) (all lanes call put; only lanes
// 3..60 carry a complete d). The flux and update arrays of sweep_core are
// never held in registers, which keeps these 18-field sweeps within two
// wavefronts' register budget per SIMD.
template <class S, typename T, int DIR, bool MB, class Put>
__device__ inline void sweep_core_streamed(const Params& P, const T* W, int pos, const int* pc, double tc, Put&& put) {
  constexpr bool Z = false;
  T sL[S::NF], sR[S::NF];
#pragma unroll
  for (int q = 0; q < S::NF; ++q) {
    if (q == S::R && P.r_static) { sL[q] = W[q]; sR[q] = W[q]; continue; }
    const T wm = shup<Z>(W[q]), wp = shdn<Z>(W[q]);
    const Cand<T> c = candidates(P, wm, W[q], wp);
    const T lmR = shup<Z>(c.mR), ltR = shup<Z>(c.tR);
    const T rmL = shdn<Z>(c.mL), rtL = shdn<Z>(c.tL);
    bvd(P, lmR, ltR, c, rmL, rtL, sL[q], sR[q]);
    pin(sL[q]);
    pin(sR[q]);
  }
  const bool bad = !admissible<S>(P, sL) || !admissible<S>(P, sR);
  if (__any(bad)) {
#pragma unroll
    for (int q = 0; q < S::NF; ++q) {
      sL[q] = bad ? W[q] : sL[q];
      sR[q] = bad ? W[q] : sR[q];
    }
  }
  T WR[S::NF];
#pragma unroll
  for (int q = 0; q < S::NF; ++q) WR[q] = shdn<Z>(sL[q]);
  if constexpr (kFaceModDims >= S::D) {
    if (P.face_mod) {  // uniform over the grid
      const T rn = shdn<Z>(W[S::R]);
      const bool rig = W[S::R] > T(0.5);
      const bool cross = rig != (rn > T(0.5));
      if (__any(cross)) face_modifier<S, DIR, MB>(P, pos, pc, tc, cross, !rig, sR, WR);
    }
  }
  HllcFace<S, DIR, T> face;
  face.init(P, sR, WR);
  const T us = (T)face.ustar();
  T Vs[3] = {T(0), T(0), T(0)};
  if constexpr (S::S) {
#pragma unroll
    for (int b = 0; b < 3; ++b) Vs[b] = (T)face.vstar(sR, WR, b);
  }
  T vf = T(0), rfl = T(0);
  if (!P.r_static) {
    double xf[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xf[a] = a < S::D ? P.x0[a] + (pc[a] + 0.5) * P.dx[a] : 0.0;
    xf[DIR] = P.x0[DIR] + (pos + 1) * P.dx[DIR];
    double v[3];
    rigid_velocity<MB>(P, xf, tc, v);
    vf = (T)v[DIR];
    rfl = vf > T(0) ? sR[S::R] * vf : (vf < T(0) ? WR[S::R] * vf : T(0));
  }
  const T inv = (T)P.inv_dx[DIR];
  const T du = us - shup<Z>(us);
  T dV[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) dV[b] = Vs[b] - shup<Z>(Vs[b]);
  double Bm = 0.0;
  if (P.stiff) {
    double phi[kMaxMat], rl[kMaxMat];
    phases_w<S>(W, phi, rl);
    Bm = mix_B<S>(P, phi);
  }
#pragma unroll
  for (int q = 0; q < S::NT; ++q) {
    const T F = (T)face.flux(sR, WR, q);
    T d = (F - shup<Z>(F)) * inv;
    if (q >= S::cPHI(0) && q < S::cPHI(0) + S::N - 1) d -= W[S::wPHI(q - S::cPHI(0))] * du * inv;
    if (q == S::cE && P.stiff) d += (T)(Bm * (double)(du * inv));
    if constexpr (S::S) {
      if (q >= S::cV(0, 0) && q < S::cEP) {
        const int a = (q - S::cV(0, 0)) / 3, b = (q - S::cV(0, 0)) % 3;
        const T ua = a < S::D ? W[S::wU(a)] : T(0);
        d -= (T(2.0 / 3.0) * W[S::wV(a, b)] * du - ua * dV[b]) * inv;
      }
    }
    put(q, d);
  }
  put(S::R, ((rfl - shup<Z>(rfl)) - W[S::R] * (vf - shup<Z>(vf))) * inv);
}

// Mirror / Dirichlet treatment of a primitive loaded for a ghost position.
template <class S, typename T, int DIR>
__device__ inline void ghost_fix(const Params& P, int mode, int face, T* W) {
  if (mode == 2) {
#pragma unroll
    for (int q = 0; q < S::NF; ++q) W[q] = (T)P.bcW[face][q];
  } else if (mode == 1) {
    W[S::wU(DIR)] = -W[S::wU(DIR)];
    if constexpr (S::S) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          if ((a == DIR) != (b == DIR)) W[S::wV(a, b)] = -W[S::wV(a, b)];
    }
  }
}

// Final sweep (along x, coalesced): total D, RK combine
// U_out = U^n + b (U_in - dt D - U^n) (b = 1, 1/4, 2/3; Sec. 3.1), rigid
// freeze (Sec. 3.1), solid sources, admissibility flag; in the third stage
// also one CFL partial per wavefront for the next step.
template <class S>
constexpr int sweep_max_threads() { return 256; }

// No-op per-cell sources (systems without a stretch tensor).
struct NoSources {
  template <class S, typename T>
  __device__ void operator()(const Params&, T*, bool) const {}
};

// The exact elastoplastic sources of one cell (det(Vbar) renormalisation and
// the plastic return), applied by each lane to its own updated cell.
struct ExactSources {
  template <class S, typename T>
  __device__ void operator()(const Params& P, T* Un, bool act) const {
    if constexpr (S::S) {
      if (act) solid_sources<S>(P, Un);
    }
  }
};

// The final x sweep of a stage. xw: this wavefront's LDS slots of the
// streamed d (elastoplastic systems; NF x 64 values of T); xu: its slots of
// the d-independent part of the RK combine (NF x 64 FP64 values; the same
// systems). Dacc2: the second operator part (3D: the y sweep's), or null
// where Dacc holds the whole y/z operator. src(P, Un, act) applies
// the per-cell sources to the updated state Un; every lane of the wavefront
// calls it (act: the lane holds an updated non-rigid cell), so a source step
// may work across the wavefront (the surrogate's matrix instructions).
template <class S, typename T, class Src = ExactSources, bool MB = false>
__device__ __forceinline__ void sweep_x_body(const Params& P, const T* __restrict__ Uin, const T* __restrict__ U0,
                                             const T* __restrict__ Dacc, const T* __restrict__ Dacc2,
                                             T* __restrict__ Uout,
                                             DevScalars* __restrict__ sc, double* __restrict__ cflpart,
                                             const StepArgs& A, double bcoef, int stage, int bx, int by, int bz,
                                             long long blin, int wpb, int nparts, T* xw = nullptr, double* xu = nullptr,
                                             const Src& src = Src()) {
  const double dt = A.rhs_only ? 1.0 : sc->dtv[A.par];
  if (dt == 0.0) return;  // uniform over the grid
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  // the wavefronts of a block take consecutive segments of one row, so the
  // cache lines shared by neighbouring segments are fetched once
  const int seg = bx * wpb + wave, j = by, k = bz;
  const size_t part_slot = (size_t)blin * wpb + wave;
  if (stage == 2 && blin == 0 && threadIdx.x == 0) sc->npart = nparts;
  if (seg * kOut >= P.n[0]) {  // whole wavefront beyond the row
    if (stage == 2 && lane == 0) cflpart[part_slot] = 0.0;
    return;
  }
  const int nd = P.n[0];
  const int pos = seg * kOut - kHalo + lane;
  const int posl = pos < nd + kHalo ? pos : nd + kHalo - 1;
  const int pc[3] = {posl, j, k};
  const double tc = sc->t[A.par] - sc->t_motion;
  const bool outlane0 = lane >= kHalo && lane < kHalo + kOut && pos < nd;
  const long long c0 = outlane0 ? cell_index(P, pos, j, k) : 0;
  bool rigid0 = false;
  T W[S::NF], Uc[S::NF];  // Uc: this lane's U_in, reused by the combine
  {
    int src, face;
    const int mode = ghost_map(P, 0, posl, src, face);
    if (mode != 2) {
      load_cons<S>(P, Uin, cell_index(P, src, j, k), Uc);
      if constexpr (S::S) {
        // the part of the RK combine that does not depend on d, formed now
        // and kept in FP64 in this lane's own LDS slots (read back by the
        // same lane: no barrier): U^n + b (U_in - U^n), U^n in rigid cells;
        // the FP32 path then rounds the stage result once. U^n is loaded
        // right behind U_in by every lane, in every stage, in one batch:
        // lanes outside the output range read cell 0 and their slots are
        // never read back, and the first stage (b = 1), whose input is U^n
        // itself, reads the lines U_in's loads have just fetched. Loads
        // guarded per lane or per stage measured several times slower: the
        // guard made each one wait for the one before or for all of U_in.
        T u0v[S::NF];
#pragma unroll
        for (int q = 0; q < S::NF; ++q) u0v[q] = U0[q * P.fs + c0];
        rigid0 = outlane0 && !A.rhs_only && (double)u0v[S::R] > 0.5;
#pragma unroll
        for (int q = 0; q < S::NF; ++q) {
          const double u0 = (double)u0v[q];
          xu[q * kWave + lane] = (rigid0 && q != S::R) ? u0 : u0 + bcoef * ((double)Uc[q] - u0);
        }
      }
      cons_to_prim<S>(P, Uc, W);
    }
    ghost_fix<S, T, 0>(P, mode, face, W);
  }
  T dpre[S::NF];
  if (S::S && S::D == 3 && Dacc2 && !A.rhs_only) {  // all lanes, as U^n
#pragma unroll
    for (int q = 0; q < S::NF; ++q) dpre[q] = Dacc[q * P.fs + c0] + Dacc2[q * P.fs + c0];
  }
  T d[S::NF];
  if constexpr (S::S) {
    // streamed: this lane's d goes through its own LDS slots (no other lane
    // reads them)
    T* my = xw + lane;
    sweep_core_streamed<S, T, 0, MB>(P, W, pos, pc, tc, [&](int q, T v) { my[q * kWave] = v; });
#pragma unroll
    for (int q = 0; q < S::NF; ++q) d[q] = my[q * kWave];
  } else {
    sweep_core<S, T, 0, MB>(P, W, pos, pc, tc, d);
  }
  if (A.rhs_only & 2) {
#pragma unroll
    for (int q = 0; q < S::NF; ++q) d[q] = T(0);
  }
  const bool outlane = lane >= kHalo && lane < kHalo + kOut && pos < nd;
  const long long c = outlane ? cell_index(P, pos, j, k) : 0;
  // gas: U^n for the combine (its r row in the first stage) is loaded here,
  // beside D, in one batch; loads inside the combine's per-field selects
  // waited for each field in turn
  T u0v[S::NF];
  if constexpr (!S::S) {
    if (outlane && !A.rhs_only) {
      u0v[S::R] = U0[S::R * P.fs + c];
      if (stage != 0) {  // uniform over the grid
#pragma unroll
        for (int q = 0; q < S::NF; ++q)
          if (q != S::R) u0v[q] = U0[q * P.fs + c];
      }
    }
  }
  if (outlane && S::D > 1) {
    // with a static body r's operator is zero and the y/z sweeps do not
    // store its row of D: the loaded value is discarded by a select (a
    // branch around the loads measured slower than the bytes it saves).
    // In 3D the z and y sweeps leave their parts in D and D2 (a y sweep
    // that added into D read it back first); both are added here in the
    // order d_z + d_y + d_x.
    if (S::S && S::D == 3 && Dacc2 && !A.rhs_only) {
#pragma unroll
      for (int q = 0; q < S::NF; ++q) d[q] = (q == S::R && P.r_static) ? d[q] : dpre[q] + d[q];
    } else if (S::D == 3 && Dacc2) {
#pragma unroll
      for (int q = 0; q < S::NF; ++q) {
        const T dq = Dacc[q * P.fs + c] + Dacc2[q * P.fs + c];
        d[q] = (q == S::R && P.r_static) ? d[q] : dq + d[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < S::NF; ++q) {
        const T dq = Dacc[q * P.fs + c];
        d[q] = (q == S::R && P.r_static) ? d[q] : dq + d[q];
      }
    }
  }
  if (A.rhs_only) {  // uniform over the grid
    if (outlane) {
#pragma unroll
      for (int q = 0; q < S::NF; ++q) Uout[q * P.fs + c] = d[q];
    }
    return;
  }
  T Un[S::NF];
  bool rigid = false;
  if (outlane) {
    const T dtt = (T)dt;
    const T b = (T)bcoef;
    if constexpr (S::S) {
      rigid = rigid0;
      const double coef = stage == 0 ? dt : bcoef * dt;
#pragma unroll
      for (int q = 0; q < S::NF; ++q) {
        const double w = xu[q * kWave + lane];
        Un[q] = (T)((rigid && q != S::R) ? w : w - coef * (double)d[q]);
      }
    } else {
      rigid = (double)u0v[S::R] > 0.5;
#pragma unroll
      for (int q = 0; q < S::NF; ++q) {
        // an output lane is an interior cell: U_in is its own load
        const T ui = Uc[q];
        const T ust = ui - dtt * d[q];
        if (stage == 0) {
          Un[q] = (rigid && q != S::R) ? ui : ust;
        } else {
          const T u0 = u0v[q];
          Un[q] = (rigid && q != S::R) ? u0 : u0 + b * (ust - u0);
        }
      }
    }
  }
  src.template operator()<S, T>(P, Un, outlane && !rigid);
  double rate = 0.0;
  if (outlane) {
    bool ok = true;
#pragma unroll
    for (int l = 0; l < S::N; ++l) ok = ok && (Un[S::cA(l)] > T(0));
    ok = ok && isfinite((double)Un[S::cE]);
    if (!ok) {
      if (atomicExch(&sc->nonphys, 1) == 0) sc->first_bad = c;
    }
#pragma unroll
    for (int q = 0; q < S::NF; ++q) Uout[q * P.fs + c] = Un[q];
    if (stage == 2 && !((double)Un[S::R] > 0.5)) {
      double x[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < S::D; ++a) x[a] = P.x0[a] + (pc[a] + 0.5) * P.dx[a];
      x[0] = P.x0[0] + (pos + 0.5) * P.dx[0];
      bool adm;
      rate = cfl_rate<S, T, MB>(P, Un, x, tc + dt, &adm);
      // the full admissibility test of the step's result (the closure is
      // at hand here); the earlier stages test positivity and finiteness
      if (!adm && atomicExch(&sc->nonphys, 1) == 0) sc->first_bad = c;
    }
  }
  if (stage == 2) {
    for (int o = 32; o > 0; o >>= 1) rate = fmax(rate, __shfl_xor(rate, o));
    if (lane == 0) cflpart[part_slot] = rate;
  }
}

// Occupancy requests (waves per SIMD) of the single-gas sweep kernels: the
// sweeps are latency-bound chains of FP64 operations, so more resident
// wavefronts hide more of each chain, as long as the register budget does
// not force spills (measured on the 2D x sweep: four, 128 registers without
// spills, beats five with spills and six; the LDS tile holds the y/z sweeps
// at three). Other systems: the compiler's choice (1 = no request).
// XCD-aware block order: workgroups are dispatched round-robin over the 8
// XCDs by flat id, and each XCD has its own L2. The blocks that one XCD runs
// (flat ids = its index mod 8) take a contiguous run of the grid's blocks in
// x-fastest order instead of every eighth one, so neighbouring blocks whose
// loads share cache lines (tile rows of TC values, 32-128 bytes; x-sweep
// segments overlapping by their halos) run on the same L2 at about the same
// time. Returns the block's logical linear index.
__device__ inline int xcd_block(int& bx, int& by, int& bz) {
  const int gx = (int)gridDim.x, gy = (int)gridDim.y;
  const int n = gx * gy * (int)gridDim.z;
  const int b = (int)blockIdx.x + gx * ((int)blockIdx.y + gy * (int)blockIdx.z);
  const int xcd = b & 7, q = n >> 3, r = n & 7;
  const int l = xcd * q + (xcd < r ? xcd : r) + (b >> 3);
  bx = l % gx;
  by = (l / gx) % gy;
  bz = l / (gx * gy);
  return l;
}

// Dynamic LDS of a launch (bytes given at the launch), as an array of T.
template <typename T>
__device__ inline T* dyn_lds() {
  extern __shared__ __align__(16) unsigned char rbdi_dyn_lds[];
  return reinterpret_cast<T*>(rbdi_dyn_lds);
}

// LDS bytes of an x-sweep block of wpb wavefronts: the elastoplastic sweeps
// stage each wavefront's streamed d (nfields x 64 values of T) and the
// d-independent part of its RK combine (nfields x 64 FP64 values).
template <class S, typename T>
constexpr unsigned x_sweep_lds(int wpb) {
  return S::S ? (unsigned)(wpb * S::NF * kWave * (sizeof(T) + sizeof(double))) : 0u;
}

template <class S>
constexpr int x_sweep_waves() { return S::S ? 2 : S::N != 1 ? 1 : 4; }
template <class S>
constexpr int tile_sweep_waves() { return S::S ? 2 : S::N != 1 ? 1 : 3; }

template <class S, typename T, bool MB = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(x_sweep_waves<S>()))) void k_sweep_x(Params P, const T* __restrict__ Uin, const T* __restrict__ U0,
                                                const T* __restrict__ Dacc, const T* __restrict__ Dacc2,
                                                T* __restrict__ Uout,
                                                DevScalars* __restrict__ sc, double* __restrict__ cflpart,
                                                StepArgs A, double bcoef, int stage) {
  const int wpb = blockDim.x / kWave;
  int bx, by, bz;
  const long long blin = xcd_block(bx, by, bz);
  const int nparts = (int)(gridDim.x * gridDim.y * gridDim.z) * wpb;
  if constexpr (S::S) {
    // per-wavefront staging of the streamed d, sized by the launch for the
    // block's wavefronts (a static size for the largest block would hold
    // LDS that 1- and 2-wavefront blocks never use and cap their occupancy)
    unsigned char* base = dyn_lds<unsigned char>() + (threadIdx.x / kWave) * x_sweep_lds<S, T>(1);
    T* xd = reinterpret_cast<T*>(base);
    double* xu = reinterpret_cast<double*>(base + S::NF * kWave * sizeof(T));
    sweep_x_body<S, T, ExactSources, MB>(P, Uin, U0, Dacc, Dacc2, Uout, sc, cflpart, A, bcoef, stage, bx, by, bz, blin,
                                         wpb, nparts, xd, xu);
  } else {
    sweep_x_body<S, T, ExactSources, MB>(P, Uin, U0, Dacc, Dacc2, Uout, sc, cflpart, A, bcoef, stage, bx, by, bz, blin,
                                         wpb, nparts);
  }
}

// Sweeps along y and z (not final): a block stages a tile of kTC columns x
// 64 positions along DIR of U_in in LDS with coalesced loads (rows of kTC
// consecutive x), each wavefront then runs the sweep on one column at a time
// with lanes along DIR, writes its d back into the tile column, and the block
// stores the tile coalesced into D (MODE 0: D = d; MODE 1: D += d).
// REDUCE: the first sweep of a step; its block (0,0,0) also reduces the CFL
// partials into the step's dt (this sweep itself does not use dt).
constexpr int kRS = 65;  // LDS stride of a tile column (padded)

#ifndef RBDI_TC
#define RBDI_TC 16
#endif
// Columns of a y/z tile: the widest of 16, 8, 4 whose tile fits the LDS
// budget: 80 KB (two blocks per CU in its 160 KB) for FP32 and for the FP64
// elastoplastic systems, 48 KB for the FP64 fluid ones. Wider tiles load
// and store longer rows (TC consecutive x values) but give each wavefront
// more columns in sequence, which costs registers across the column loop:
// on the 256^3 copper grid the FP64 elastoplastic y + z sweeps take 5.25 ms
// at 8 columns (64-byte rows) against 5.66 at 4.
template <class S, typename T>
constexpr int tile_lds_budget() { return (sizeof(T) == 8 && !S::S ? 48 : 80) * 1024; }
template <class S, typename T>
constexpr int tile_cols() {
  return (S::NF * RBDI_TC * kRS * (int)sizeof(T) <= tile_lds_budget<S, T>()) ? RBDI_TC
       : (S::NF * 8 * kRS * (int)sizeof(T) <= tile_lds_budget<S, T>()) ? 8 : 4;
}

template <class S, typename T, int DIR, int MODE, bool REDUCE, bool MB = false>
__device__ __forceinline__ void sweep_tile_body(const Params& P, const T* __restrict__ Uin, T* __restrict__ Dacc,
                                                DevScalars* __restrict__ sc, const double* __restrict__ cflpart,
                                                const StepArgs& A, int bx, int by, int bz, T* tile,
                                                int TC) {
  if constexpr (REDUCE) {
    if (bx == 0 && by == 0 && bz == 0) reduce_dt(sc, cflpart, A);
    if (step_done(sc, A)) return;  // uniform over the grid
  } else {
    if (!A.rhs_only && sc->dtv[A.par] == 0.0) return;  // uniform over the grid
  }
  const int x0 = bx * TC;
  int seg, j, k;
  if (DIR == 1) { seg = by; k = bz; j = 0; }
  else { j = by; seg = bz; k = 0; }
  const int nd = P.n[DIR];
  const int base = seg * kOut - kHalo;
  // Tile load: each thread owns TC * kWave / kTileThreads cells; the loads of
  // a group of them are all issued before the first LDS write, so their
  // latencies overlap (a group holds at most about 24 values).
  constexpr int kG = 24 / S::NF > 0 ? 24 / S::NF : 1;
  const int nper = TC * kWave / kTileThreads;
  for (int it0 = 0; it0 < nper; it0 += kG) {
    T v[kG][S::NF];
    int dst[kG];
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      dst[g] = -1;
      const int e = threadIdx.x + (it0 + g) * kTileThreads;
      const int c = e % TC, r = e / TC;
      const int x = x0 + c;
      const int pos = base + r;
      const int posl = pos < nd + kHalo ? pos : nd + kHalo - 1;
      int src = 0, face;
      if (it0 + g < nper && x < P.n[0] && ghost_map(P, DIR, posl, src, face) != 2) {
        int p3[3] = {x, j, k};
        p3[DIR] = src;
        const long long cell = cell_index(P, p3[0], p3[1], p3[2]);
#pragma unroll
        for (int q = 0; q < S::NF; ++q) v[g][q] = Uin[q * P.fs + cell];
        dst[g] = c * kRS + r;
      }
    }
#pragma unroll
    for (int g = 0; g < kG; ++g)
      if (dst[g] >= 0) {
#pragma unroll
        for (int q = 0; q < S::NF; ++q) tile[q * TC * kRS + dst[g]] = v[g][q];
      }
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const double tc = sc->t[A.par] - sc->t_motion;
  // one column at a time (unrolled, two columns' sweeps would interleave and
  // double the register demand)
#pragma unroll 1
  for (int c = wave; c < TC; c += kTileThreads / kWave) {
    const int x = x0 + c;
    if (x >= P.n[0]) break;  // uniform in the wavefront
    const int pos = base + lane;
    const int posl = pos < nd + kHalo ? pos : nd + kHalo - 1;
    int pc[3] = {x, j, k};
    pc[DIR] = posl;
    T W[S::NF];
    int src, face;
    const int mode = ghost_map(P, DIR, posl, src, face);
    if (mode != 2) {
      T Uc[S::NF];
#pragma unroll
      for (int q = 0; q < S::NF; ++q) Uc[q] = tile[(q * TC + c) * kRS + lane];
      cons_to_prim<S>(P, Uc, W);
    }
    ghost_fix<S, T, DIR>(P, mode, face, W);
    const bool outlane = lane >= kHalo && lane < kHalo + kOut && pos < nd;
    const bool zero = (A.rhs_only & (2 << DIR)) != 0;
    if constexpr (S::S) {
      // streamed: each field's d goes straight into this lane's slot of the
      // tile column (its U_in there was consumed by the closure above; the
      // slots of halo lanes and of positions beyond the domain are written
      // too, and never read: the store below takes the output rows only)
      sweep_core_streamed<S, T, DIR, MB>(P, W, pos, pc, tc, [&](int q, T v) {
        tile[(q * TC + c) * kRS + lane] = zero ? T(0) : v;
      });
    } else {
      T d[S::NF];
      sweep_core<S, T, DIR, MB>(P, W, pos, pc, tc, d);
      if (zero) {
#pragma unroll
        for (int q = 0; q < S::NF; ++q) d[q] = T(0);
      }
      if (outlane) {
#pragma unroll
        for (int q = 0; q < S::NF; ++q) tile[(q * TC + c) * kRS + lane] = d[q];
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TC * kWave; e += kTileThreads) {
    const int c = e % TC, r = e / TC;
    const int x = x0 + c;
    const int pos = base + r;
    if (x >= P.n[0] || r < kHalo || r >= kHalo + kOut || pos >= nd) continue;
    int p3[3] = {x, j, k};
    p3[DIR] = pos;
    const long long cell = cell_index(P, p3[0], p3[1], p3[2]);
#pragma unroll
    for (int q = 0; q < S::NF; ++q) {
      if (q == S::R && P.r_static) continue;  // zero; the x sweep ignores this row
      const T v = tile[(q * TC + c) * kRS + r];
      if (MODE == 0) Dacc[q * P.fs + cell] = v;
      else Dacc[q * P.fs + cell] += v;
    }
  }
}


template <class S, typename T, int DIR, int MODE, bool REDUCE, bool MB = false>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(tile_sweep_waves<S>()))) void k_sweep_tile(Params P, const T* __restrict__ Uin, T* __restrict__ Dacc,
                                                   DevScalars* __restrict__ sc, const double* __restrict__ cflpart,
                                                   StepArgs A) {
  constexpr int TC = tile_cols<S, T>();
  __shared__ T tile[S::NF * TC * kRS];
  int bx, by, bz;
  xcd_block(bx, by, bz);
  sweep_tile_body<S, T, DIR, MODE, REDUCE, MB>(P, Uin, Dacc, sc, cflpart, A, bx, by, bz, tile, TC);
}

// ---------------------------------------------------------------------------
// Rigid band (rigid cells with a nonzero r gradient) and seeding (Sec. 3.2)
// ---------------------------------------------------------------------------

__device__ inline void decode(const Params& P, long long c, int& i, int& j, int& k) {
  i = (int)(c % P.n[0]);
  j = (int)((c / P.n[0]) % P.n[1]);
  k = (int)(c / ((long long)P.n[0] * P.n[1]));
}

// Youngs normal (Sec. 3.3): n = -grad r / |grad r| with central differences.
template <class S, typename T>
__device__ inline bool youngs_normal(const Params& P, const T* __restrict__ U, int i, int j, int k, double n[3]) {
  double g[3] = {0.0, 0.0, 0.0}, m2 = 0.0;
#pragma unroll
  for (int d = 0; d < S::D; ++d) {
    g[d] = (r_at<S>(P, U, i, j, k, d, 1) - r_at<S>(P, U, i, j, k, d, -1)) / (2.0 * P.dx[d]);
    m2 += g[d] * g[d];
  }
  const double mag = sqrt(m2);
  if (!(mag * P.dmin > 1e-12)) return false;
#pragma unroll
  for (int d = 0; d < 3; ++d) n[d] = d < S::D ? -g[d] / mag : 0.0;
  return true;
}

// ELVIRA (Sec. 3.3, after Pilliod and Puckett), 2D.
//
// r at (i+a, j+b) for |a|, |b| <= 1 with ghost positions mapped as the
// domain ghost layers are filled: along y first (a Dirichlet face gives its
// state), then along x within the source row.
template <class S, typename T>
__device__ inline double r_block(const Params& P, const T* __restrict__ U, int i, int j, int k) {
  int sj, sx, face;
  const int my = ghost_map(P, 1, j, sj, face);
  if (my == 2) return P.bcW[face][S::R];
  const int mx = ghost_map(P, 0, i, sx, face);
  if (mx == 2) return P.bcW[face][S::R];
  return (double)U[S::R * P.fs + cell_index(P, sx, sj, k)];
}

// Fraction of a cell of sides hx, hy lying on the side n.p <= beta of the
// line with unit normal n (p measured from the cell centre): with
// c1 <= c2 the two projections |n_x| hx, |n_y| hy and s = beta + (c1+c2)/2
// the distance from the lowest corner, the cut is a triangle (s < c1), a
// trapezoid (s <= c2) or the complement of a triangle.
__device__ inline double cut_fraction(double nx, double ny, double hx, double hy, double beta) {
  double c1 = fabs(nx) * hx, c2 = fabs(ny) * hy;
  if (c1 > c2) { const double t = c1; c1 = c2; c2 = t; }
  const double s = beta + 0.5 * (c1 + c2);
  if (s <= 0.0) return 0.0;
  if (s >= c1 + c2) return 1.0;
  if (s < c1) return s * s / (2.0 * c1 * c2);
  if (s <= c2) return (s - 0.5 * c1) / c2;
  const double t = c1 + c2 - s;
  return 1.0 - t * t / (2.0 * c1 * c2);
}

// Inverse of cut_fraction in beta for 0 < f < 1.
__device__ inline double cut_offset(double nx, double ny, double hx, double hy, double f) {
  double c1 = fabs(nx) * hx, c2 = fabs(ny) * hy;
  if (c1 > c2) { const double t = c1; c1 = c2; c2 = t; }
  const double f1 = 0.5 * c1 / c2;  // fraction at s = c1
  double s;
  if (f <= f1) s = sqrt(2.0 * c1 * c2 * f);
  else if (f <= 1.0 - f1) s = f * c2 + 0.5 * c1;
  else s = c1 + c2 - sqrt(2.0 * c1 * c2 * (1.0 - f));
  return s - 0.5 * (c1 + c2);
}

// Candidates: the interface as a graph over x (slopes from the backward,
// central and forward differences of the column sums of r) and over y (row
// sums); the body lies on the side given by the sign of the opposite sums
// (rows bottom vs top, columns left vs right), a family with sign zero is
// left out. Each candidate line cuts the centre cell at its fraction; the
// one whose nine cell fractions differ least from r in the sum of squares is
// taken (the first on ties). Returns false where the centre fraction is not
// strictly between 0 and 1 or no family exists.
template <class S, typename T>
__device__ inline bool elvira_normal(const Params& P, const T* __restrict__ U, int i, int j, int k, double n[3]) {
  double f[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) f[a][b] = r_block<S>(P, U, i + a - 1, j + b - 1, k);
  const double fc = f[1][1];
  if (!(fc > 0.0 && fc < 1.0)) return false;
  const double hx = P.dx[0], hy = P.dx[1];
  double H[3], Wr[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) H[a] = hy * (f[a][0] + f[a][1] + f[a][2]);
#pragma unroll
  for (int b = 0; b < 3; ++b) Wr[b] = hx * (f[0][b] + f[1][b] + f[2][b]);
  const double sy = Wr[2] > Wr[0] ? 1.0 : (Wr[2] < Wr[0] ? -1.0 : 0.0);
  const double sx = H[2] > H[0] ? 1.0 : (H[2] < H[0] ? -1.0 : 0.0);
  double best = 0.0;
  bool found = false;
  for (int c = 0; c < 6; ++c) {
    const bool colf = c < 3;
    const double sg = colf ? sy : sx;
    if (sg == 0.0) continue;
    const double* A = colf ? H : Wr;
    const double h = colf ? hx : hy;
    const int m = c % 3;
    const double sl = m == 0 ? (A[1] - A[0]) / h : (m == 1 ? (A[2] - A[0]) / (2.0 * h) : (A[2] - A[1]) / h);
    const double vx = colf ? -sl : -sg, vy = colf ? -sg : -sl;
    const double mag = sqrt(vx * vx + vy * vy);
    const double nx = vx / mag, ny = vy / mag;
    const double beta = cut_offset(nx, ny, hx, hy, fc);
    double err = 0.0;
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
      for (int b = -1; b <= 1; ++b) {
        const double e = cut_fraction(nx, ny, hx, hy, beta - nx * a * hx - ny * b * hy) - f[a + 1][b + 1];
        err += e * e;
      }
    if (!found || err < best) {
      best = err;
      found = true;
      n[0] = nx;
      n[1] = ny;
      n[2] = 0.0;
    }
  }
  return found;
}

// Normal of a rigid cell for seeding: ELVIRA in 2D when selected and
// defined, otherwise Youngs.
template <class S, typename T>
__device__ inline bool band_normal(const Params& P, const T* __restrict__ U, int i, int j, int k, double n[3]) {
  if constexpr (S::D == 2) {
    if (P.normal == NORMAL_ELVIRA && elvira_normal<S>(P, U, i, j, k, n)) return true;
  }
  return youngs_normal<S>(P, U, i, j, k, n);
}

// Seeding geometry of one rigid cell (Sec. 3.2 steps 1-2): outward normal,
// probe along n at 1, 1.5, ..., 4 dx (or the fixed 1.5 dx); the first point
// whose enclosing cells with a nonzero interpolation weight are all interior
// with r <= 0.5 is used. A point between the outermost cell centres and a
// domain face is moved, along that axis, onto the outermost centre, so that
// a probe running along a wall does not switch between valid and invalid
// with the sign of a rounding error. It depends on r only, so for a static
// body it is computed once and reused by every step.
struct SeedTask {
  int c;          // linear index of the rigid cell
  int lo[3];      // lower corner of the interpolation support
  double w[3];    // multilinear weights
  double n[3];    // outward normal
};

template <class S, typename T>
__device__ inline bool probe_ok(const Params& P, const T* __restrict__ U, const int* lo, const double* w) {
  bool ok = true;
#pragma unroll
  for (int cb = 0; cb < (1 << S::D); ++cb) {
    int cp[3] = {0, 0, 0};
    bool used = true, inside = true;
#pragma unroll
    for (int a = 0; a < S::D; ++a) {
      const int bit = (cb >> a) & 1;
      if (bit && w[a] == 0.0) used = false;
      cp[a] = lo[a] + bit;
      inside = inside && cp[a] >= 0 && cp[a] < P.n[a];
    }
    if (used) {
      if (!inside) ok = false;
      else if (!((double)U[S::R * P.fs + cell_index(P, cp[0], cp[1], cp[2])] <= 0.5)) ok = false;
    }
  }
  return ok;
}

template <class S, typename T>
__global__ __launch_bounds__(256) void k_band(Params P, const T* __restrict__ U, SeedTask* __restrict__ tasks,
                                             int cap, DevScalars* __restrict__ sc, StepArgs A) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (step_done(sc, A)) return;
  if (c >= P.ncell) return;
  if (!((double)U[S::R * P.fs + c] > 0.5)) return;
  int pi[3];
  decode(P, c, pi[0], pi[1], pi[2]);
  double n[3];
  if (!band_normal<S>(P, U, pi[0], pi[1], pi[2], n)) return;
  const int nprobe = P.probe == PROBE_FIXED ? 1 : 7;
  int best = -1;
  int blo[3] = {0, 0, 0};
  double bw[3] = {0.0, 0.0, 0.0};
  // all probe distances are tested independently (their loads overlap);
  // the first valid one wins
#pragma unroll
  for (int pr = 0; pr < 7; ++pr) {
    if (pr < nprobe) {
      const double dist = P.probe == PROBE_FIXED ? 1.5 : 1.0 + 0.5 * pr;
      int lo[3] = {0, 0, 0};
      double w[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < S::D; ++a) {
        double xi = pi[a] + dist * n[a] * (P.dmin / P.dx[a]);
        const double last = (double)(P.n[a] - 1);
        xi = (xi < 0.0 && xi >= -0.5) ? 0.0 : xi;
        xi = (xi > last && xi <= last + 0.5) ? last : xi;
        lo[a] = (int)floor(xi);
        w[a] = xi - lo[a];
      }
      if (probe_ok<S>(P, U, lo, w) && best < 0) {
        best = pr;
#pragma unroll
        for (int a = 0; a < 3; ++a) { blo[a] = lo[a]; bw[a] = w[a]; }
      }
    }
  }
  if (best < 0) {
    atomicAdd(&sc->band_fail, 1);
    return;
  }
  const int slot = atomicAdd(&sc->band_count, 1);
  if (slot >= cap) return;  // reported by rbdi_status
  SeedTask t;
  t.c = (int)c;
#pragma unroll
  for (int a = 0; a < 3; ++a) { t.lo[a] = blo[a]; t.w[a] = bw[a]; t.n[a] = n[a]; }
  tasks[slot] = t;
}

__global__ void k_band_reset(DevScalars* sc, StepArgs A) {
  if (step_done(sc, A)) return;
  sc->band_count = 0;
  sc->band_fail = 0;
}

// Seeding states (Sec. 3.2 steps 3-5): multilinear interpolation of the
// primitives at the probe (nested linear interpolations), mirror state,
// optional Riemann star state, written to the thermodynamic fields of the
// rigid cell. Support cells are never rigid, so no thread reads a cell that
// another one writes.
template <class S, typename T, bool MB = false>
__device__ __forceinline__ void seed_one(const Params& P, T* __restrict__ U, const SeedTask& t, double tc) {
  double Wc[1 << S::D][S::NF];
#pragma unroll
  for (int cb = 0; cb < (1 << S::D); ++cb) {
    int cp[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < S::D; ++a) {
      const int bit = (cb >> a) & 1;
      cp[a] = t.lo[a] + ((bit && t.w[a] != 0.0) ? 1 : 0);
    }
    T Uc[S::NF], Wt[S::NF];
    load_cons<S>(P, U, cell_index(P, cp[0], cp[1], cp[2]), Uc);
    cons_to_prim<S>(P, Uc, Wt);
#pragma unroll
    for (int q = 0; q < S::NF; ++q) Wc[cb][q] = (double)Wt[q];
  }
  int m = 1 << S::D;
#pragma unroll
  for (int a = 0; a < S::D; ++a) {
    m >>= 1;
#pragma unroll
    for (int cb = 0; cb < m; ++cb)
#pragma unroll
      for (int q = 0; q < S::NF; ++q)
        Wc[cb][q] = Wc[2 * cb][q] + t.w[a] * (Wc[2 * cb + 1][q] - Wc[2 * cb][q]);
  }
  int pi[3];
  decode(P, t.c, pi[0], pi[1], pi[2]);
  double xc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < S::D; ++a) xc[a] = P.x0[a] + (pi[a] + 0.5) * P.dx[a];
  double v[3];
  rigid_velocity<MB>(P, xc, tc, v);
  double Wm[S::NF], Wg[S::NF];
  mirror<S>(Wc[0], t.n, v, Wm);
  if (P.seed == SEED_RIEMANN) riemann_seed<S>(P, Wm, Wc[0], t.n, Wg);
  else {
#pragma unroll
    for (int q = 0; q < S::NF; ++q) Wg[q] = Wm[q];
  }
  T Wt[S::NF], Ug[S::NF];
#pragma unroll
  for (int q = 0; q < S::NF; ++q) Wt[q] = (T)Wg[q];
  Wt[S::R] = U[S::R * P.fs + t.c];
  prim_to_cons<S>(P, Wt, Ug);
#pragma unroll
  for (int q = 0; q < S::NT; ++q) U[q * P.fs + t.c] = Ug[q];
}

// Sum of an int over the wavefront; lane 0 adds it to a counter (one atomic
// per wavefront instead of one per lane).
__device__ inline void wave_count_add(long long* counter, int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd((unsigned long long*)counter, (unsigned long long)v);
}

template <class S, typename T, bool MB = false>
__global__ __launch_bounds__(256) void k_seed(Params P, T* __restrict__ U, const SeedTask* __restrict__ tasks,
                                             int cap, DevScalars* __restrict__ sc, StepArgs A) {
  if (step_done(sc, A)) return;
  const int nb = sc->band_count < cap ? sc->band_count : cap;
  const double tc = sc->t[A.par] - sc->t_motion;
  int nseed = 0;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
    seed_one<S, T, MB>(P, U, tasks[b], tc);
    ++nseed;
  }
  wave_count_add(&sc->seeded, nseed);
}

// ---------------------------------------------------------------------------
// Reductions (fixed grid, fixed-order trees: deterministic)
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

template <typename T>
__device__ inline T block_min(T v, T* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) v = fmin(v, sh[q]);
    sh[0] = v;
  }
  __syncthreads();
  v = sh[0];
  __syncthreads();
  return v;
}

// Fixed-order block sum of one double per thread (pairwise tree in LDS).
__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// CFL partials (one per block) of the current state, for a state that did
// not come from a step; the first sweep of the next step reduces them.
template <class S, typename T, bool MB = false>
__global__ __launch_bounds__(kRedThreads) void k_cfl(Params P, const T* __restrict__ U,
                                                    DevScalars* __restrict__ sc, int par,
                                                    double* __restrict__ part) {
  __shared__ double sh[kRedThreads / 64];
  double m = 0.0;
  const double tc = sc->t[par] - sc->t_motion;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < P.ncell;
       c += (long long)gridDim.x * blockDim.x) {
    if ((double)U[S::R * P.fs + c] > 0.5) continue;
    T Uc[S::NF];
    load_cons<S>(P, U, c, Uc);
    int pi[3];
    decode(P, c, pi[0], pi[1], pi[2]);
    double x[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < S::D; ++a) x[a] = P.x0[a] + (pi[a] + 0.5) * P.dx[a];
    m = fmax(m, cfl_rate<S, T, MB>(P, Uc, x, tc));
  }
  m = -block_min(-m, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->npart = gridDim.x;
}

// Maximum of the valid CFL partials (for rbdi_compute_dt).
__global__ void k_max_partials(const double* __restrict__ part, const DevScalars* __restrict__ sc,
                               double* __restrict__ out) {
  __shared__ double sh[4];
  const int n = sc->npart;
  double m = 0.0;
  for (int q = threadIdx.x; q < n; q += blockDim.x) m = fmax(m, part[q]);
  m = -block_min(-m, sh);
  if (threadIdx.x == 0) *out = m;
}

// Force and torque: per cell f = -sigma . grad_h r dV, torque (x - c) x f.
template <class S, typename T>
__global__ __launch_bounds__(kRedThreads) void k_force_partial(Params P, const T* __restrict__ U, double cx,
                                                              double cy, double cz, double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  double dV = 1.0;
  for (int d = 0; d < S::D; ++d) dV *= P.dx[d];
  const double ctr[3] = {cx, cy, cz};
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < P.ncell;
       c += (long long)gridDim.x * blockDim.x) {
    int pi[3];
    decode(P, c, pi[0], pi[1], pi[2]);
    double g[3] = {0.0, 0.0, 0.0};
    bool any = false;
#pragma unroll
    for (int d = 0; d < S::D; ++d) {
      g[d] = (r_at<S>(P, U, pi[0], pi[1], pi[2], d, 1) - r_at<S>(P, U, pi[0], pi[1], pi[2], d, -1)) /
             (2.0 * P.dx[d]);
      any = any || g[d] != 0.0;
    }
    if (!any) continue;
    T Uc[S::NF], W[S::NF];
    load_cons<S>(P, U, c, Uc);
    double H[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, J2 = 0.0;
    cons_to_prim<S>(P, Uc, W, H, &J2);
    double G = 0.0;
    if constexpr (S::S) {
      double phi[kMaxMat], rl[kMaxMat], c2, sY;
      phases_w<S>(W, phi, rl);
      mix_c2_G<S>(P, phi, rl, J2, (double)W[S::wP], c2, G, sY);
    }
    const double p = (double)W[S::wP];
    double f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double sig = (a == b ? -p : 0.0) + 2.0 * G * H[3 * a + b];
        s -= sig * g[b];
      }
      f[a] = s * dV;
    }
    double xr[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < S::D; ++a) xr[a] = P.x0[a] + (pi[a] + 0.5) * P.dx[a] - ctr[a];
    acc[0] += f[0];
    acc[1] += f[1];
    acc[2] += f[2];
    acc[3] += xr[1] * f[2] - xr[2] * f[1];
    acc[4] += xr[2] * f[0] - xr[0] * f[2];
    acc[5] += xr[0] * f[1] - xr[1] * f[0];
  }
  for (int q = 0; q < 6; ++q) {
    const double s = block_sum(acc[q], sh);
    if (threadIdx.x == 0) part[q * gridDim.x + blockIdx.x] = s;
  }
}

// Totals of every field (all cells, non-rigid cells), times dV.
template <class S, typename T>
__global__ __launch_bounds__(kRedThreads) void k_totals_partial(Params P, const T* __restrict__ U,
                                                               double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  double all[S::NF], flu[S::NF];
#pragma unroll
  for (int q = 0; q < S::NF; ++q) { all[q] = 0.0; flu[q] = 0.0; }
  double dV = 1.0;
  for (int d = 0; d < S::D; ++d) dV *= P.dx[d];
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < P.ncell;
       c += (long long)gridDim.x * blockDim.x) {
    const bool rig = (double)U[S::R * P.fs + c] > 0.5;
    T Uc[S::NF];
    load_cons<S>(P, U, c, Uc);
    const double Bc = mix_B_cons<S>(P, Uc);
#pragma unroll
    for (int q = 0; q < S::NF; ++q) {
      const double v = ((double)Uc[q] + (q == S::cE ? Bc : 0.0)) * dV;
      all[q] += v;
      flu[q] += rig ? 0.0 : v;
    }
  }
  for (int q = 0; q < S::NF; ++q) {
    double s = block_sum(all[q], sh);
    if (threadIdx.x == 0) part[q * gridDim.x + blockIdx.x] = s;
    s = block_sum(flu[q], sh);
    if (threadIdx.x == 0) part[(S::NF + q) * gridDim.x + blockIdx.x] = s;
  }
}

// Final fixed-order sum of nq rows of nparts partials.
__global__ void k_sum_rows(const double* __restrict__ part, int nparts, int nq, double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  for (int q = 0; q < nq; ++q) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) v += part[q * nparts + b];
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) out[q] = s;
  }
}

// ---------------------------------------------------------------------------
// Conversions and initialisation
// ---------------------------------------------------------------------------

template <class S, typename T>
__global__ void k_prim_to_state(Params P, const double* __restrict__ Win, T* __restrict__ U) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.ncell) return;
  T W[S::NF], Uc[S::NF];
#pragma unroll
  for (int q = 0; q < S::NF; ++q) W[q] = (T)Win[q * P.ncell + c];
  prim_to_cons<S>(P, W, Uc);
#pragma unroll
  for (int q = 0; q < S::NF; ++q) U[q * P.fs + c] = Uc[q];
}

template <class S, typename T>
__global__ void k_state_to_prim(Params P, const T* __restrict__ U, double* __restrict__ Wout) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.ncell) return;
  T Uc[S::NF], W[S::NF];
  load_cons<S>(P, U, c, Uc);
  cons_to_prim<S>(P, Uc, W);
#pragma unroll
  for (int q = 0; q < S::NF; ++q) Wout[q * P.ncell + c] = (double)W[q];
}

template <class S, typename T>
__global__ void k_state_to_f64(Params P, const T* __restrict__ U, double* __restrict__ out, int add_B) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.ncell) return;
  T Uc[S::NF];
  load_cons<S>(P, U, c, Uc);
#pragma unroll
  for (int q = 0; q < S::NF; ++q) out[q * P.ncell + c] = (double)Uc[q];
  if (add_B) out[S::cE * P.ncell + c] += mix_B_cons<S>(P, Uc);  // rho E = E~ + B(phi)
}

template <class S, typename T>
__global__ void k_f64_to_state(Params P, const double* __restrict__ in, T* __restrict__ U) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.ncell) return;
  double Ud[S::NF];
#pragma unroll
  for (int q = 0; q < S::NF; ++q) Ud[q] = in[q * P.ncell + c];
  Ud[S::cE] -= mix_B_cons<S>(P, Ud);  // E~ = rho E - B(phi)
#pragma unroll
  for (int q = 0; q < S::NF; ++q) U[q * P.fs + c] = (T)Ud[q];
}

// r = (1 - tanh(sdf / (width dx_min))) / 2 (bodies as a diffuse scalar field).
template <class S, typename T>
__global__ void k_r_from_sdf(Params P, const double* __restrict__ sdf, double inv_w, T* __restrict__ U) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.ncell) return;
  U[S::R * P.fs + c] = (T)(0.5 * (1.0 - tanh(sdf[c] * inv_w)));
}

// ---------------------------------------------------------------------------
// Unit-level kernels (parity checks of single device functions)
// ---------------------------------------------------------------------------

// Face flux of (WL, WR) along DIR: out = {F[NT], u*, Vbar*_{DIR,0..2}}.
template <class S, typename T, int DIR>
__global__ void k_unit_flux(Params P, const double* __restrict__ WL, const double* __restrict__ WR,
                            double* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T L[S::NF], R[S::NF], F[S::NT], us, Vs[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int q = 0; q < S::NF; ++q) { L[q] = (T)WL[i * S::NF + q]; R[q] = (T)WR[i * S::NF + q]; }
  hllc<S, DIR>(P, L, R, F, us, Vs);
  double* o = out + (size_t)i * (S::NT + 4);
#pragma unroll
  for (int q = 0; q < S::NT; ++q) o[q] = (double)F[q];
  // flux of rho E = flux of E~ + B_N (unit-field flux) + sum_l (B_l - B_N) F(phi_l)
  const double BN = P.mat[S::N - 1].Bfl;
  o[S::cE] += BN * (double)us;
#pragma unroll
  for (int l = 0; l < S::N - 1; ++l) o[S::cE] += (P.mat[l].Bfl - BN) * (double)F[S::cPHI(l)];
  o[S::NT] = (double)us;
  for (int b = 0; b < 3; ++b) o[S::NT + 1 + b] = (double)Vs[b];
}

// Closure of conserved states: out = {W[NF], c2, sigma (9)}.
template <class S, typename T>
__global__ void k_unit_closure(Params P, const double* __restrict__ U, double* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T Uc[S::NF], W[S::NF];
#pragma unroll
  for (int q = 0; q < S::NF; ++q) Uc[q] = (T)U[i * S::NF + q];
  Uc[S::cE] = (T)(U[i * S::NF + S::cE] - mix_B_cons<S>(P, U + (size_t)i * S::NF));
  double H[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, J2 = 0.0;
  cons_to_prim<S>(P, Uc, W, H, &J2);
  double phi[kMaxMat], rl[kMaxMat], c2, G, sY;
  phases_w<S>(W, phi, rl);
  mix_c2_G<S>(P, phi, rl, J2, (double)W[S::wP], c2, G, sY);
  double* o = out + (size_t)i * (S::NF + 10);
#pragma unroll
  for (int q = 0; q < S::NF; ++q) o[q] = (double)W[q];
  o[S::NF] = c2;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) o[S::NF + 1 + 3 * a + b] = (a == b ? -(double)W[S::wP] : 0.0) + 2.0 * G * H[3 * a + b];
}

// Per-stage solid sources of conserved states, in place.
template <class S, typename T>
__global__ void k_unit_sources(Params P, double* __restrict__ U, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T Uc[S::NF];
#pragma unroll
  for (int q = 0; q < S::NF; ++q) Uc[q] = (T)U[i * S::NF + q];
  const double B = mix_B_cons<S>(P, U + (size_t)i * S::NF);
  Uc[S::cE] = (T)(U[i * S::NF + S::cE] - B);
  if constexpr (S::S) solid_sources<S>(P, Uc);
#pragma unroll
  for (int q = 0; q < S::NF; ++q) U[i * S::NF + q] = (double)Uc[q];
  U[i * S::NF + S::cE] = (double)Uc[S::cE] + B;
}

}  // namespace rbdi
