// rbdi_physics.hpp -- device physics of the diffuse-interface rigid-body
// method (arXiv 2111.11806) for gfx950: field layout, mixture closure,
// MUSCL-BVD-THINC candidates, HLLC / HLLC-LM flux, mirror and Riemann
// seeding states, stretch-tensor algebra and the plastic return.
//
// Everything here is per cell or per face and lives in registers; the
// kernels that move data are in rbdi_kernels.hpp.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace rbdi {

constexpr int kMaxF = 20;
constexpr int kMaxMat = 2;
constexpr int kMaxBody = 4;  // rigid bodies with their own motions

enum { EOS_IDEAL = 0, EOS_STIFFENED = 1, EOS_ROMENSKII = 2 };
enum { BC_TRANSMISSIVE = 0, BC_REFLECTIVE = 1, BC_DIRICHLET = 2, BC_PERIODIC = 3 };
enum { REC_MUSCL = 0, REC_BVD_THINC = 1 };
enum { RS_HLLC = 0, RS_HLLC_LM = 1 };
enum { SEED_ORIGINAL = 0, SEED_RIEMANN = 1, SEED_NONE = 2 };
enum { PROBE_STEPOUT = 0, PROBE_FIXED = 1 };
enum { NORMAL_YOUNGS = 0, NORMAL_ELVIRA = 1 };

// Reciprocal from the hardware estimate refined by two Newton steps (FP64;
// within an ulp or two of 1/x), or the single-precision hardware
// reciprocal. Used only where x is finite and nonzero.
__device__ inline double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Material constants in the form the device closure uses.
struct MatDev {
  int kind;
  double gamma, pinf;
  double Gam, invGam;   // Gruneisen coefficient and its inverse
  double Bfl;           // fluids: rho e_ref - p_ref / Gamma = gamma p_inf / Gamma
  double rho0, invrho0, K0, G0, alpha, beta, kc;  // Romenskii, kc = K0 / (2 alpha^2)
  int ialpha, ibeta1;   // alpha and beta + 1 when they are integers in [1, 8], else 0
  double sigY;
  double gGam;          // fluids: gamma / Gamma (sound-speed weight)
};

// Launch-invariant parameters of one instance (passed by value).
struct Params {
  int dim;
  int n[3];
  long long st[3];        // element strides of x, y, z
  long long fs;           // element stride between fields
  long long ncell;        // interior cells
  double dx[3], inv_dx[3], x0[3], dmin;
  int bc[6];
  int recon, riemann, seed, probe, plastic;
  int normal;
  double cosh_b, inv_sinh_b, tanh_b, beta;
  double lm_mach;
  double exc[14];         // 1/k!, k = 0..13 (exponential series, kept in scalar registers)
  double ln2_hi, ln2_lo, inv_ln2;
  int solid_phase;
  int r_static;           // rigid velocity identically zero: r never changes
  int stiff;              // some phase has a stiffening energy (B(phi) != 0)
  int surr;               // elastoplastic sources with the surrogate network
                          // (the final sweep's variant with the network)
  MatDev mat[kMaxMat];
  // Rigid motions v + omega x (x - c): body 0 everywhere, except where a
  // point lies in the ownership box of a body 1..nbody-1 (first match); the
  // centres and boxes are those of the time the motions were set and move
  // with each body's translation.
  int nbody;
  double vr[kMaxBody][3], om[kMaxBody][3], ctr[kMaxBody][3];
  double blo[kMaxBody][3], bhi[kMaxBody][3];
  double bcW[6][kMaxF];   // Dirichlet primitive states per face
  // void-opening face modifier at solid-rigid faces (elastoplastic systems):
  // on/off, and the primitive state of the gas that fills an opening gap
  int face_mod;
  double gapW[kMaxF];
};

// Compile-time field layout of the reduced-equation multi-material system
// (Sec. 2.1.1, 2.4):
//   U = (phi_l rho_l [N], rho u [D], rho E, phi_l [N-1], Vbar [9], a_s eps_p, r)
//   W = (phi_l [N-1], rho_l [N], u [D], p, Vbar [9], eps_p, r)
template <int DIM_, int NMAT_, bool SOLID_>
struct Sys {
  static constexpr int D = DIM_;
  static constexpr int N = NMAT_;
  static constexpr bool S = SOLID_;
  static constexpr int NF = 2 * N + D + 1 + (S ? 10 : 0);
  static constexpr int NT = NF - 1;  // thermodynamic fields
  static constexpr int R = NF - 1;
  __host__ __device__ static constexpr int cA(int l) { return l; }
  __host__ __device__ static constexpr int cM(int a) { return N + a; }
  static constexpr int cE = N + D;
  __host__ __device__ static constexpr int cPHI(int l) { return N + D + 1 + l; }
  __host__ __device__ static constexpr int cV(int a, int b) { return 2 * N + D + 3 * a + b; }
  static constexpr int cEP = 2 * N + D + 9;
  __host__ __device__ static constexpr int wPHI(int l) { return l; }
  __host__ __device__ static constexpr int wRHO(int l) { return N - 1 + l; }
  __host__ __device__ static constexpr int wU(int a) { return 2 * N - 1 + a; }
  static constexpr int wP = 2 * N - 1 + D;
  __host__ __device__ static constexpr int wV(int a, int b) { return 2 * N + D + 3 * a + b; }
  static constexpr int wEP = 2 * N + D + 9;
};

// Element k of a small per-thread array, k known only at run time (the
// solid phase), by a chain of selects: indexing such an array with a run-time
// value would place the whole array in scratch memory.
template <int N, typename T>
__device__ inline T pick(const T* a, int k) {
  T v = a[0];
#pragma unroll
  for (int l = 1; l < N; ++l) v = (k == l) ? a[l] : v;
  return v;
}

// ---------------------------------------------------------------------------
// Small 3x3 algebra (stretch tensor)
// ---------------------------------------------------------------------------

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations with a fixed
// maximum number of sweeps and an early exit once the off-diagonal part is
// below roundoff of the diagonal.
template <typename T>
__device__ inline void jacobi3(T A[3][3], T Q[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Q[i][j] = (i == j) ? T(1) : T(0);
  for (int sweep = 0; sweep < 12; ++sweep) {
    const T off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const T dg = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= T(1e-34) * dg || off == T(0)) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0;
      const int q = pq == 0 ? 1 : 2;
      const T apq = A[p][q];
      if (apq == T(0)) continue;
      const T th = (A[q][q] - A[p][p]) / (T(2) * apq);
      const T t = (th >= T(0) ? T(1) : T(-1)) / (fabs(th) + sqrt(th * th + T(1)));
      const T c = T(1) / sqrt(t * t + T(1));
      const T s = t * c;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T akp = A[k][p], akq = A[k][q];
        A[k][p] = c * akp - s * akq;
        A[k][q] = s * akp + c * akq;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T apk = A[p][k], aqk = A[q][k];
        A[p][k] = c * apk - s * aqk;
        A[q][k] = s * apk + c * aqk;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T qkp = Q[k][p], qkq = Q[k][q];
        Q[k][p] = c * qkp - s * qkq;
        Q[k][q] = s * qkp + c * qkq;
      }
    }
  }
}

// Isotropic matrix functions without an eigen-decomposition. For a
// symmetric 3x3 matrix A with principal invariants i1, i2, i3, the
// Cayley-Hamilton theorem A^3 = i1 A^2 - i2 A + i3 I keeps every power in the
// span of I, A, A^2: if A^k = al I + be A + ga A^2 then
// A^(k+1) = ga i3 I + (al - ga i2) A + (be + ga i1) A^2. A power series
// f(A) = sum_k w_k A^k is therefore c0 I + c1 A + c2 A^2 with the sums of
// w_k (al, be, ga). Used for ln(I + X) and exp(A) at small |X|, |A|, where
// the series converge fast; the same functions by eigen-decomposition remain
// the fallback for large arguments.
struct SymM {
  double a00, a11, a22, a01, a02, a12;
};

__device__ inline SymM sym_sq(const SymM& x) {
  SymM q;
  q.a00 = x.a00 * x.a00 + x.a01 * x.a01 + x.a02 * x.a02;
  q.a11 = x.a01 * x.a01 + x.a11 * x.a11 + x.a12 * x.a12;
  q.a22 = x.a02 * x.a02 + x.a12 * x.a12 + x.a22 * x.a22;
  q.a01 = x.a00 * x.a01 + x.a01 * x.a11 + x.a02 * x.a12;
  q.a02 = x.a00 * x.a02 + x.a01 * x.a12 + x.a02 * x.a22;
  q.a12 = x.a01 * x.a02 + x.a11 * x.a12 + x.a12 * x.a22;
  return q;
}

// Power series coefficients: w_k for k >= 1 from a table (terms until the
// k-th term is below 1e-17 of the first), returns (c0, c1, c2) for
// sum_{k>=1} w_k A^k; t = Frobenius norm of A (bounds its spectral radius),
// first = |w_1| t, the scale of the leading term.
template <int KMAX, typename WF>
__device__ inline void ch_series(const SymM& A, double t, WF wk, double& c0, double& c1, double& c2) {
  const double i1 = A.a00 + A.a11 + A.a22;
  const double t2 = t * t;
  const double i2 = 0.5 * (i1 * i1 - t2);
  const double i3 = A.a00 * (A.a11 * A.a22 - A.a12 * A.a12) - A.a01 * (A.a01 * A.a22 - A.a12 * A.a02) +
                    A.a02 * (A.a01 * A.a12 - A.a11 * A.a02);
  double al = 0.0, be = 1.0, ga = 0.0;
  c0 = 0.0;
  c1 = 0.0;
  c2 = 0.0;
  const double lead = fabs(wk(1)) * t;
  for (int k = 1; k <= KMAX; ++k) {
    const double w = wk(k);
    c0 += w * al;
    c1 += w * be;
    c2 += w * ga;
    const double mag = fabs(w) * (fabs(al) + fabs(be) * t + fabs(ga) * t2);
    if (k > 1 && mag <= 1e-17 * lead) break;
    const double nal = ga * i3, nbe = al - ga * i2, nga = be + ga * i1;
    al = nal;
    be = nbe;
    ga = nga;
  }
}

__device__ inline double log_w(int k) { return (k & 1 ? 0.5 : -0.5) / (double)k; }

// Hencky strain H = (1/2) ln(Vbar Vbar^T) (equals ln Vbar for a symmetric
// stretch; Sec. 2.1.2) and J2 = H:H, by eigen-decomposition.
template <typename T>
__device__ __forceinline__ void hencky3_eig(const T V[9], T H[9], T& J2) {
  T b[3][3], Q[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      b[i][j] = V[3 * i] * V[3 * j] + V[3 * i + 1] * V[3 * j + 1] + V[3 * i + 2] * V[3 * j + 2];
  jacobi3(b, Q);
  T h[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) h[k] = T(0.5) * log(b[k][k]);
  J2 = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T v = Q[i][0] * h[0] * Q[j][0] + Q[i][1] * h[1] * Q[j][1] + Q[i][2] * h[2] * Q[j][2];
      H[3 * i + j] = v;
      J2 += v * v;
    }
}

// The same H and J2: for |X| <= 0.3 (X = Vbar Vbar^T - I) by the series of
// (1/2) ln(I + X), otherwise by eigen-decomposition.
template <typename T>
__device__ inline void hencky3(const T V[9], T H[9], T& J2) {
  SymM X;
  X.a00 = (double)(V[0] * V[0] + V[1] * V[1] + V[2] * V[2]) - 1.0;
  X.a11 = (double)(V[3] * V[3] + V[4] * V[4] + V[5] * V[5]) - 1.0;
  X.a22 = (double)(V[6] * V[6] + V[7] * V[7] + V[8] * V[8]) - 1.0;
  X.a01 = (double)(V[0] * V[3] + V[1] * V[4] + V[2] * V[5]);
  X.a02 = (double)(V[0] * V[6] + V[1] * V[7] + V[2] * V[8]);
  X.a12 = (double)(V[3] * V[6] + V[4] * V[7] + V[5] * V[8]);
  const SymM X2 = sym_sq(X);
  const double t2 = X2.a00 + X2.a11 + X2.a22;
  if (!(t2 <= 0.09)) {
    hencky3_eig(V, H, J2);
    return;
  }
  double c0, c1, c2;
  ch_series<64>(X, sqrt(t2), log_w, c0, c1, c2);
  const double h00 = c0 + c1 * X.a00 + c2 * X2.a00, h11 = c0 + c1 * X.a11 + c2 * X2.a11;
  const double h22 = c0 + c1 * X.a22 + c2 * X2.a22, h01 = c1 * X.a01 + c2 * X2.a01;
  const double h02 = c1 * X.a02 + c2 * X2.a02, h12 = c1 * X.a12 + c2 * X2.a12;
  H[0] = (T)h00; H[1] = (T)h01; H[2] = (T)h02;
  H[3] = (T)h01; H[4] = (T)h11; H[5] = (T)h12;
  H[6] = (T)h02; H[7] = (T)h12; H[8] = (T)h22;
  J2 = (T)(h00 * h00 + h11 * h11 + h22 * h22 + 2.0 * (h01 * h01 + h02 * h02 + h12 * h12));
}

// ---------------------------------------------------------------------------
// Closure (Sec. 2.1.2 Mie-Gruneisen form, Sec. 2.1.3 EOS, Sec. 2.2 mixture)
// ---------------------------------------------------------------------------

// Per-phase reference terms: B = rho e_ref - p_ref / Gamma (enters the
// isobaric pressure inversion), the phase sound speed squared, and the shear
// modulus. Fluids (ideal / stiffened): B = gamma p_inf / Gamma, c^2 =
// gamma (p + p_inf) / rho, G = 0. Romenskii: x = rho/rho0, y = x^alpha,
// G = G0 x^(beta+1), rho e_ref = kc (y-1)^2 + G J2,
// p_ref = kc (y-1)((2 alpha - 1) y + 1) + beta G J2,
// a^2 = (Gamma + 1)(p - p_ref)/rho + dp_ref/drho, c^2 = a^2 + 4 G / (3 rho).
struct PhaseOut {
  double B, c2, G;
};

// x^k for 1 <= k <= 8 by repeated multiplication (k = 0: pow(x, e)).
__device__ inline double pow_small(double x, int k, double e) {
  if (k == 0) return pow(x, e);
  double r = x;
  for (int i = 1; i < k; ++i) r *= x;
  return r;
}

__device__ inline void romenskii_ref(const MatDev& m, double rho, double J2, double& rhoe_ref,
                                     double& p_ref, double& dpref, double& G) {
  const double x = rho * m.invrho0;
  const double y = pow_small(x, m.ialpha, m.alpha);
  G = m.G0 * pow_small(x, m.ibeta1, m.beta + 1.0);
  const double ym = y - 1.0;
  rhoe_ref = m.kc * ym * ym + G * J2;
  p_ref = m.kc * ym * ((2.0 * m.alpha - 1.0) * y + 1.0) + m.beta * G * J2;
  dpref = (m.K0 / m.alpha) * ((2.0 * m.alpha - 1.0) * y - m.alpha + 1.0) * y / rho +
          m.beta * (m.beta + 1.0) * G * J2 / rho;
}

// Mixture pressure from rho e (FP64 in every precision):
// p = [rho e - sum phi_l B_l] / sum(phi_l / Gamma_l).
template <class S>
__device__ inline double mix_pressure(const Params& P, const double* phi, const double* rho, double J2,
                                      double rhoe_t) {
  if constexpr (S::N == 1 && !S::S) return rhoe_t * P.mat[0].Gam;
  double num = rhoe_t, den = 0.0;
#pragma unroll
  for (int l = 0; l < S::N; ++l) {
    const MatDev& m = P.mat[l];
    if (S::S && m.kind == EOS_ROMENSKII) {
      double er, pr, dp, G;
      romenskii_ref(m, rho[l], J2, er, pr, dp, G);
      num -= phi[l] * (er - pr * m.invGam);
    }
    den += phi[l] * m.invGam;
  }
  return num * frcp(den);
}

// rho e from p (the same isobaric relation solved for rho e).
template <class S>
__device__ inline double mix_rhoe(const Params& P, const double* phi, const double* rho, double J2, double p) {
  double s = 0.0, den = 0.0;
#pragma unroll
  for (int l = 0; l < S::N; ++l) {
    const MatDev& m = P.mat[l];
    if (S::S && m.kind == EOS_ROMENSKII) {
      double er, pr, dp, G;
      romenskii_ref(m, rho[l], J2, er, pr, dp, G);
      s += phi[l] * (er - pr * m.invGam);
    }
    den += phi[l] * m.invGam;
  }
  return p * den + s;
}

// Stiffening energy of the mixture, B(phi) = sum_l phi_l gamma_l p_inf,l /
// (gamma_l - 1) over the fluid phases. The state stores E~ = rho E - B(phi)
// in place of rho E: for stiffened gases rho E carries the large constant
// part B, and E~ (of the size of p) keeps the pressure inversion and the
// energy fluxes free of cancellation in any precision. Since phi* = chi phi
// and the unit field's star value is chi, the HLLC flux of E~ has the form of
// that of rho E with E replaced by E~, and
// E~_t + div((E~ + P) u) = -B(phi) div(u*) (with div(u*) the divergence of
// the unit field's flux, the one the volume fractions use).
template <class S>
__device__ inline double mix_B(const Params& P, const double* phi) {
  double b = 0.0;
#pragma unroll
  for (int l = 0; l < S::N; ++l) b += phi[l] * P.mat[l].Bfl;
  return b;
}

// B(phi) from the stored volume fractions of a conserved state.
template <class S, typename T>
__device__ inline double mix_B_cons(const Params& P, const T* U) {
  double phi[kMaxMat], s = 0.0;
#pragma unroll
  for (int l = 0; l < S::N - 1; ++l) {
    phi[l] = (double)U[S::cPHI(l)];
    s += phi[l];
  }
  phi[S::N - 1] = 1.0 - s;
  return mix_B<S>(P, phi);
}

// Mixture sound speed squared (Sec. 2.2, mass-fraction weighted over
// sum phi/Gamma), shear modulus (Sec. 2.2) and yield stress (same weights).
template <class S>
__device__ inline void mix_c2_G(const Params& P, const double* phi, const double* rho, double J2, double p,
                                double& c2, double& G, double& sigY) {
  if constexpr (!S::S) {
    // fluids: Y_l c_l^2 = phi_l gamma_l (p + p_inf,l) / rho
    G = 0.0;
    sigY = 0.0;
    if constexpr (S::N == 1) {
      c2 = P.mat[0].gamma * (p + P.mat[0].pinf) * frcp(rho[0]);
    } else {
      double num = 0.0, den = 0.0, rhom = 0.0;
#pragma unroll
      for (int l = 0; l < S::N; ++l) {
        num += phi[l] * P.mat[l].gGam * (p + P.mat[l].pinf);
        den += phi[l] * P.mat[l].invGam;
        rhom += phi[l] * rho[l];
      }
      c2 = num * frcp(rhom * den);
    }
    return;
  }
  double rhom = 0.0;
#pragma unroll
  for (int l = 0; l < S::N; ++l) rhom += phi[l] * rho[l];
  double nc = 0.0, nG = 0.0, nY = 0.0, den = 0.0;
#pragma unroll
  for (int l = 0; l < S::N; ++l) {
    const MatDev& m = P.mat[l];
    double cl2, Gl = 0.0;
    if (S::S && m.kind == EOS_ROMENSKII) {
      double er, pr, dp;
      romenskii_ref(m, rho[l], J2, er, pr, dp, Gl);
      cl2 = (m.Gam + 1.0) * (p - pr) / rho[l] + dp + (4.0 / 3.0) * Gl / rho[l];
    } else {
      cl2 = m.gamma * (p + m.pinf) / rho[l];
    }
    nc += phi[l] * rho[l] * cl2 * m.invGam;
    nG += phi[l] * Gl * m.invGam;
    nY += phi[l] * m.sigY * m.invGam;
    den += phi[l] * m.invGam;
  }
  const double inv = 1.0 / den;
  c2 = nc / rhom * inv;
  G = nG * inv;
  sigY = nY * inv;
}

// Face-state thermodynamics in one pass over the phases (one Romenskii
// reference-curve evaluation per phase): mixture c^2, shear modulus, yield
// stress (as mix_c2_G) and rho e from p (as mix_rhoe).
template <class S>
__device__ inline void mix_state(const Params& P, const double* phi, const double* rho, double J2, double p,
                                 double& c2, double& G, double& sigY, double& rhoe) {
  if constexpr (!S::S) {
    mix_c2_G<S>(P, phi, rho, J2, p, c2, G, sigY);
    rhoe = mix_rhoe<S>(P, phi, rho, J2, p);
    return;
  }
  double rhom = 0.0;
#pragma unroll
  for (int l = 0; l < S::N; ++l) rhom += phi[l] * rho[l];
  double nc = 0.0, nG = 0.0, nY = 0.0, den = 0.0, s = 0.0;
#pragma unroll
  for (int l = 0; l < S::N; ++l) {
    const MatDev& m = P.mat[l];
    double cl2, Gl = 0.0;
    const double ir = frcp(rho[l]);
    if (m.kind == EOS_ROMENSKII) {
      double er, pr, dp;
      romenskii_ref(m, rho[l], J2, er, pr, dp, Gl);
      cl2 = ((m.Gam + 1.0) * (p - pr) + (4.0 / 3.0) * Gl) * ir + dp;
      s += phi[l] * (er - pr * m.invGam);
    } else {
      cl2 = m.gamma * (p + m.pinf) * ir;
    }
    nc += phi[l] * rho[l] * cl2 * m.invGam;
    nG += phi[l] * Gl * m.invGam;
    nY += phi[l] * m.sigY * m.invGam;
    den += phi[l] * m.invGam;
  }
  const double inv = frcp(den);
  c2 = nc * frcp(rhom) * inv;
  G = nG * inv;
  sigY = nY * inv;
  rhoe = p * den + s;
}

// Volume fractions and phasic densities of a primitive vector.
template <class S, typename T>
__device__ inline void phases_w(const T* W, double* phi, double* rho) {
  double s = 0.0;
#pragma unroll
  for (int l = 0; l < S::N - 1; ++l) {
    phi[l] = (double)W[S::wPHI(l)];
    s += phi[l];
  }
  phi[S::N - 1] = 1.0 - s;
#pragma unroll
  for (int l = 0; l < S::N; ++l) rho[l] = (double)W[S::wRHO(l)];
}

// Conserved -> primitive (Sec. 2.2); the energy slot holds E~ = rho E -
// B(phi). For the elastoplastic system the Hencky strain of Vbar is also
// returned (J2, H).
template <class S, typename T>
__device__ inline void cons_to_prim(const Params& P, const T* U, T* W, double* Hout = nullptr,
                                    double* J2out = nullptr) {
  double rho = 0.0;
#pragma unroll
  for (int l = 0; l < S::N; ++l) rho += (double)U[S::cA(l)];
  double phi[kMaxMat], rl[kMaxMat];
  double s = 0.0;
#pragma unroll
  for (int l = 0; l < S::N - 1; ++l) {
    phi[l] = (double)U[S::cPHI(l)];
    s += phi[l];
  }
  phi[S::N - 1] = 1.0 - s;
  if constexpr (S::N == 1) {
    rl[0] = (double)U[S::cA(0)];
  } else {
#pragma unroll
    for (int l = 0; l < S::N; ++l) rl[l] = (double)U[S::cA(l)] * frcp(phi[l]);
  }
  const double inv = frcp(rho);
  double ke = 0.0;
#pragma unroll
  for (int a = 0; a < S::D; ++a) {
    const double u = (double)U[S::cM(a)] * inv;
    W[S::wU(a)] = (T)u;
    ke += u * (double)U[S::cM(a)];
  }
  const double rhoe = (double)U[S::cE] - 0.5 * ke;
  double J2 = 0.0;
  if constexpr (S::S) {
    double V[9], H[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      V[q] = (double)U[S::cV(0, 0) + q];
      W[S::wV(0, 0) + q] = U[S::cV(0, 0) + q];
    }
    hencky3(V, H, J2);
    if (Hout) {
#pragma unroll
      for (int q = 0; q < 9; ++q) Hout[q] = H[q];
    }
    const int sp = P.solid_phase;
    W[S::wEP] = (T)((double)U[S::cEP] / (double)pick<S::N>(U + S::cA(0), sp));
  }
  if (J2out) *J2out = J2;
#pragma unroll
  for (int l = 0; l < S::N - 1; ++l) W[S::wPHI(l)] = U[S::cPHI(l)];
#pragma unroll
  for (int l = 0; l < S::N; ++l) W[S::wRHO(l)] = (T)rl[l];
  W[S::wP] = (T)mix_pressure<S>(P, phi, rl, J2, rhoe);
  W[S::R] = U[S::R];
}

// Primitive -> conserved. Returns J2 (and H) of the stretch when solid.
template <class S, typename T>
__device__ inline void prim_to_cons(const Params& P, const T* W, T* U, double* Hout = nullptr) {
  double phi[kMaxMat], rl[kMaxMat];
  phases_w<S>(W, phi, rl);
  double rho = 0.0;
#pragma unroll
  for (int l = 0; l < S::N; ++l) {
    const double a = phi[l] * rl[l];
    U[S::cA(l)] = (T)a;
    rho += a;
  }
  double ke = 0.0;
#pragma unroll
  for (int a = 0; a < S::D; ++a) {
    const double u = (double)W[S::wU(a)];
    U[S::cM(a)] = (T)(rho * u);
    ke += rho * u * u;
  }
  double J2 = 0.0;
  if constexpr (S::S) {
    double V[9], H[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      V[q] = (double)W[S::wV(0, 0) + q];
      U[S::cV(0, 0) + q] = W[S::wV(0, 0) + q];
    }
    hencky3(V, H, J2);
    if (Hout) {
#pragma unroll
      for (int q = 0; q < 9; ++q) Hout[q] = H[q];
    }
    const int sp = P.solid_phase;
    U[S::cEP] = (T)(pick<S::N>(phi, sp) * pick<S::N>(rl, sp) * (double)W[S::wEP]);
  }
  U[S::cE] = (T)(mix_rhoe<S>(P, phi, rl, J2, (double)W[S::wP]) + 0.5 * ke);
#pragma unroll
  for (int l = 0; l < S::N - 1; ++l) U[S::cPHI(l)] = W[S::wPHI(l)];
  U[S::R] = W[S::R];
}

// Admissibility of a reconstructed primitive state (positive phasic
// densities, volume fractions in [0,1], p + p_inf > 0 for fluid phases).
template <class S, typename T>
__device__ inline bool admissible(const Params& P, const T* W) {
  double phi[kMaxMat], rl[kMaxMat];
  phases_w<S>(W, phi, rl);
  const double p = (double)W[S::wP];
  bool ok = true;
#pragma unroll
  for (int l = 0; l < S::N; ++l) {
    ok = ok && (rl[l] > 0.0) && (phi[l] >= 0.0) && (phi[l] <= 1.0);
    if (P.mat[l].kind != EOS_ROMENSKII) ok = ok && (p + P.mat[l].pinf > 0.0);
  }
  return ok;
}

// ---------------------------------------------------------------------------
// Reconstruction (Sec. 3.1: MUSCL on primitives, THINC, BVD selection)
// ---------------------------------------------------------------------------

// Candidates of one variable in one cell: {MUSCL left, MUSCL right, THINC
// left, THINC right}. van Leer slope; THINC where the cell is strictly
// monotone, with the closed-form face values of the tanh profile whose cell
// average is the cell value.
template <typename T>
struct Cand {
  T mL, mR, tL, tR;
};

// exp(x) in FP64 for the THINC argument: x = k ln2 + r (Cody-Waite split of
// ln2, |r| <= ln2/2), the Taylor series of exp(r) to r^13 (truncation below
// 5e-18), scaled by 2^k. The series coefficients come from the launch
// parameters, i.e. scalar registers, instead of being rebuilt in vector
// registers for every inlined call.
__device__ inline double exp_thinc(const Params& P, double x) {
  const double k = rint(x * P.inv_ln2);
  double r = fma(-k, P.ln2_hi, x);
  r = fma(-k, P.ln2_lo, r);
  double p = P.exc[13];
#pragma unroll
  for (int j = 12; j >= 0; --j) p = fma(p, r, P.exc[j]);
  return ldexp(p, (int)k);
}
__device__ inline float exp_thinc(const Params&, float x) { return expf(x); }

template <typename T>
__device__ inline Cand<T> candidates(const Params& P, T qm, T q0, T qp) {
  Cand<T> c;
  const T a = qp - q0, b = q0 - qm;
  const T ab = a * b;
  T half_slope = T(0);
  if (ab > T(0)) half_slope = ab * frcp(a + b);
  c.mL = q0 - half_slope;
  c.mR = q0 + half_slope;
  c.tL = c.mL;
  c.tR = c.mR;
  if (P.recon == REC_BVD_THINC && ab > T(0)) {
    const T qmin = qm < qp ? qm : qp;
    const T dq = fabs(qp - qm);
    const T th = qp > qm ? T(1) : T(-1);
    const T C = (q0 - qmin) * frcp(dq);
    const T e = exp_thinc(P, th * T(P.beta) * (T(2) * C - T(1)));
    const T tt = (T(P.cosh_b) - e) * T(P.inv_sinh_b);
    const T tb = T(P.tanh_b);
    const T hd = T(0.5) * dq;
    c.tL = qmin + hd * (T(1) - th * tt);
    c.tR = qmin + hd * (T(1) + th * (tb - tt) * frcp(T(1) - tb * tt));
  }
  return c;
}

// BVD (Sec. 3.1): THINC faces when their total boundary variation against
// the neighbours' faces of the same scheme is strictly smaller.
template <typename T>
__device__ inline void bvd(const Params& P, T lmR, T ltR, const Cand<T>& c0, T rmL, T rtL, T& qL, T& qR) {
  const T tbm = fabs(lmR - c0.mL) + fabs(c0.mR - rmL);
  const T tbt = fabs(ltR - c0.tL) + fabs(c0.tR - rtL);
  const bool thinc = (P.recon == REC_BVD_THINC) && (tbt < tbm);
  qL = thinc ? c0.tL : c0.mL;
  qR = thinc ? c0.tR : c0.mR;
}

// ---------------------------------------------------------------------------
// Riemann solver (Sec. 3.1 HLLC; Sec. 4.3 HLLC-LM)
// ---------------------------------------------------------------------------

// Side data of a face state along direction d.
template <class S>
struct SideState {
  double rho, un, P, c, E;   // density, normal velocity, normal traction, sound speed, rho E
  double u[3];
  double sig[3];             // sigma_{a d}, tension positive
  double phi[kMaxMat], rl[kMaxMat];
  double H[9];
};

template <class S, int DIR, typename T>
__device__ inline void side_state(const Params& P, const T* W, SideState<S>& s) {
  phases_w<S>(W, s.phi, s.rl);
  s.rho = 0.0;
#pragma unroll
  for (int l = 0; l < S::N; ++l) s.rho += s.phi[l] * s.rl[l];
  double ke = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    s.u[a] = a < S::D ? (double)W[S::wU(a)] : 0.0;
    ke += s.u[a] * s.u[a];
  }
  s.un = s.u[DIR];
  const double p = (double)W[S::wP];
  double J2 = 0.0;
  if constexpr (S::S) {
    double V[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) V[q] = (double)W[S::wV(0, 0) + q];
    hencky3(V, s.H, J2);
  }
  double c2, G, sY, rhoe;
  mix_state<S>(P, s.phi, s.rl, J2, p, c2, G, sY, rhoe);
  s.c = sqrt(c2);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double sg = (a == DIR) ? -p : 0.0;
    if constexpr (S::S) sg += 2.0 * G * s.H[3 * a + DIR];
    s.sig[a] = sg;
  }
  s.P = -s.sig[DIR];
  s.E = rhoe + 0.5 * s.rho * ke;
}

// Conserved value, physical flux and star value of field q on one side.
// chi = (S_K - u_K)/(S_K - S*); star: mass-like fields * chi, normal
// momentum rho* S*, tangential rho* u_t, energy chi [E + (S*-u)(rho S* +
// P/(S-u))], phi * chi, Vbar rows scaled by chi^(-2/3) (normal) and
// chi^(1/3) (tangential).
template <class S, int DIR, typename T>
__device__ inline void field_terms(const T* W, const SideState<S>& s, int q, int sp, double Sk, double Ss,
                                   double chi, double cn, double ct, double& u, double& f, double& us) {
  const double un = s.un;
  if (q < S::N) {  // phi_l rho_l
    u = s.phi[q] * s.rl[q];
    f = u * un;
    us = chi * u;
  } else if (q < S::N + S::D) {  // momentum
    const int a = q - S::N;
    u = s.rho * s.u[a];
    f = u * un - s.sig[a];
    us = chi * s.rho * (a == DIR ? Ss : s.u[a]);
  } else if (q == S::cE) {
    u = s.E;
    double work = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) work += s.u[a] * s.sig[a];
    f = s.E * un - work;
    us = chi * (s.E + (Ss - un) * (s.rho * Ss + s.P * frcp(Sk - un)));
  } else if (q < S::cE + S::N) {  // phi_l
    u = (double)W[S::wPHI(q - S::cE - 1)];
    f = u * un;
    us = chi * u;
  } else if (S::S && q < S::cEP) {  // Vbar_ab
    const int ab = q - S::cV(0, 0);
    const int a = ab / 3, b = ab % 3;
    u = (double)W[S::wV(0, 0) + ab];
    f = u * un - (double)W[S::wV(DIR, b)] * s.u[a];
    us = (a == DIR ? cn : ct) * u;
  } else {  // phi_s rho_s eps_p
    u = pick<S::N>(s.phi, sp) * pick<S::N>(s.rl, sp) * (double)W[S::wEP];
    f = u * un;
    us = chi * u;
  }
}

// sin(x) for x in [0, pi/2] by its Taylor series to x^23 in Horner form
// (truncation below 4e-18 on the interval; no range reduction needed).
__device__ inline double sin_quadrant(double x) {
  const double x2 = x * x;
  double p = -1.0 / 25852016738884976640000.0;  // -1/23!
  p = fma(p, x2, 1.0 / 51090942171709440000.0);   // 1/21!
  p = fma(p, x2, -1.0 / 121645100408832000.0);    // -1/19!
  p = fma(p, x2, 1.0 / 355687428096000.0);        // 1/17!
  p = fma(p, x2, -1.0 / 1307674368000.0);         // -1/15!
  p = fma(p, x2, 1.0 / 6227020800.0);             // 1/13!
  p = fma(p, x2, -1.0 / 39916800.0);              // -1/11!
  p = fma(p, x2, 1.0 / 362880.0);                 // 1/9!
  p = fma(p, x2, -1.0 / 5040.0);                  // -1/7!
  p = fma(p, x2, 1.0 / 120.0);                    // 1/5!
  p = fma(p, x2, -1.0 / 6.0);                     // -1/3!
  return fma(p * x2, x, x);
}

// Toro's HLLC flux from side K (the side whose fan region holds x/t = 0):
// F = F_K, or with star = true F_K + S_K (U*_K - U_K).
template <class S, int DIR, typename T>
__device__ inline void toro_side(const T* WK, const SideState<S>& K, int sp, double Sk, double Ss, bool star, T* F,
                                 T& ustar, T* Vstar) {
  const double chi = star ? (Sk - K.un) * frcp(Sk - Ss) : 1.0;
  double cn = 1.0, ct = 1.0;
  if constexpr (S::S) {
    if (star) { ct = cbrt(chi); cn = 1.0 / (ct * ct); }
  }
#pragma unroll
  for (int q = 0; q < S::NT; ++q) {
    double u, f, us;
    field_terms<S, DIR>(WK, K, q, sp, Sk, Ss, chi, cn, ct, u, f, us);
    F[q] = (T)(star ? f + Sk * (us - u) : f);
  }
  ustar = (T)(star ? K.un + Sk * (chi - 1.0) : K.un);
  if constexpr (S::S) {
#pragma unroll
    for (int b = 0; b < 3; ++b) Vstar[b] = (T)((double)WK[S::wV(DIR, b)] * (star ? cn : 1.0));
  }
}

// HLLC flux along DIR. Outputs the thermodynamic flux F[NT], the wall
// velocity u* (the flux formula applied to the unit field, star value chi),
// and the wall stretch row Vbar*_{DIR,:} (Godunov value at x/t = 0).
// Davis wave speeds; HLLC-LM: central form with the acoustic terms scaled by
// sin(min(1, Ma/Ma_lim) pi/2), Ma from the normal velocities.
template <class S, int DIR, typename T>
__device__ inline void hllc(const Params& P, const T* WL, const T* WR, T* F, T& ustar, T* Vstar) {
  SideState<S> L, R;
  side_state<S, DIR>(P, WL, L);
  side_state<S, DIR>(P, WR, R);
  const double SL = fmin(L.un - L.c, R.un - R.c);
  const double SR = fmax(L.un + L.c, R.un + R.c);
  const double mL = L.rho * (SL - L.un), mR = R.rho * (SR - R.un);
  const double Ss = (R.P - L.P + L.un * mL - R.un * mR) * frcp(mL - mR);
  const int sp = P.solid_phase < 0 ? 0 : P.solid_phase;
  // central form: HLLC-LM, and always for the elastoplastic system, whose
  // star states do not satisfy the jump condition of the tangential traction
  // across the contact (the central form has no jump at S* = 0)
  if ((P.riemann == RS_HLLC_LM || S::S) && SL < 0.0 && SR > 0.0) {
    const double chiL = (SL - L.un) * frcp(SL - Ss), chiR = (SR - R.un) * frcp(SR - Ss);
    double cnL = 1, ctL = 1, cnR = 1, ctR = 1;
    if constexpr (S::S) {
      ctL = cbrt(chiL); cnL = 1.0 / (ctL * ctL);
      ctR = cbrt(chiR); cnR = 1.0 / (ctR * ctR);
    }
    // acoustic scaling sin(min(1, Ma/Ma_lim) pi/2) of HLLC-LM; 1 once either
    // side reaches the limit
    double ph = 1.0;
    if (P.riemann == RS_HLLC_LM && !(fabs(L.un) >= P.lm_mach * L.c || fabs(R.un) >= P.lm_mach * R.c)) {
      const double Ma = fmax(fabs(L.un) * frcp(L.c), fabs(R.un) * frcp(R.c));
      ph = sin_quadrant(fmin(1.0, Ma / P.lm_mach) * (M_PI * 0.5));
    }
    const double aS = fabs(Ss);
#pragma unroll
    for (int q = 0; q < S::NT; ++q) {
      double uL, fL, usL, uR, fR, usR;
      field_terms<S, DIR>(WL, L, q, sp, SL, Ss, chiL, cnL, ctL, uL, fL, usL);
      field_terms<S, DIR>(WR, R, q, sp, SR, Ss, chiR, cnR, ctR, uR, fR, usR);
      F[q] = (T)(0.5 * (fL + fR) + 0.5 * (ph * SL * (usL - uL) + aS * (usL - usR) + ph * SR * (usR - uR)));
    }
    ustar = (T)(0.5 * (L.un + R.un) + 0.5 * (ph * SL * (chiL - 1.0) + aS * (chiL - chiR) + ph * SR * (chiR - 1.0)));
    if constexpr (S::S) {
      // star states weighted by the contact's position in the fan
      const double w = (Ss - SL) * frcp(SR - SL);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double vl = (double)WL[S::wV(DIR, b)] * cnL, vr = (double)WR[S::wV(DIR, b)] * cnR;
        Vstar[b] = (T)(vr + w * (vl - vr));
      }
    }
    return;
  }
  // Toro HLLC: the side K whose fan region contains x/t = 0 (both sides are
  // spelled out, so that no array or state is selected by reference at run
  // time: such a selection would place them in scratch memory).
  if (SL >= 0.0 || Ss >= 0.0) toro_side<S, DIR>(WL, L, sp, SL, Ss, !(SL >= 0.0), F, ustar, Vstar);
  else toro_side<S, DIR>(WR, R, sp, SR, Ss, SR > 0.0, F, ustar, Vstar);
}

// The same HLLC / HLLC-LM face in a form that yields one field's flux at a
// time: init() builds both side states and the wave data (speeds, S*, chi,
// the LM factor and which part of the fan holds x/t = 0); flux(q), ustar()
// and vstar() then give what hllc() gives, with the same arithmetic, without
// a flux array held in registers. Used by the sweeps of the elastoplastic
// system, whose 18 fields otherwise need more registers than a wavefront
// can hold without spilling.
enum { FAN_LEFT = 0, FAN_RIGHT = 1, FAN_CENTRAL = 2, FAN_STAR_L = 3, FAN_STAR_R = 4 };

template <class S, int DIR, typename T>
struct HllcFace {
  SideState<S> L, R;
  double SL, SR, Ss, chiL, chiR, cnL, ctL, cnR, ctR, ph, aS;
  int mode, sp;

  __device__ inline void init(const Params& P, const T* WL, const T* WR) {
    side_state<S, DIR>(P, WL, L);
    side_state<S, DIR>(P, WR, R);
    SL = fmin(L.un - L.c, R.un - R.c);
    SR = fmax(L.un + L.c, R.un + R.c);
    const double mL = L.rho * (SL - L.un), mR = R.rho * (SR - R.un);
    Ss = (R.P - L.P + L.un * mL - R.un * mR) * frcp(mL - mR);
    sp = P.solid_phase < 0 ? 0 : P.solid_phase;
    if ((P.riemann == RS_HLLC_LM || S::S) && SL < 0.0 && SR > 0.0) mode = FAN_CENTRAL;
    else if (SL >= 0.0) mode = FAN_LEFT;
    else if (Ss >= 0.0) mode = FAN_STAR_L;
    else if (SR > 0.0) mode = FAN_STAR_R;
    else mode = FAN_RIGHT;
    chiL = (SL - L.un) * frcp(SL - Ss);
    chiR = (SR - R.un) * frcp(SR - Ss);
    cnL = ctL = cnR = ctR = 1.0;
    if constexpr (S::S) {
      ctL = cbrt(chiL); cnL = 1.0 / (ctL * ctL);
      ctR = cbrt(chiR); cnR = 1.0 / (ctR * ctR);
    }
    ph = 1.0;
    if (mode == FAN_CENTRAL && P.riemann == RS_HLLC_LM &&
        !(fabs(L.un) >= P.lm_mach * L.c || fabs(R.un) >= P.lm_mach * R.c)) {
      const double Ma = fmax(fabs(L.un) * frcp(L.c), fabs(R.un) * frcp(R.c));
      ph = sin_quadrant(fmin(1.0, Ma / P.lm_mach) * (M_PI * 0.5));
    }
    aS = fabs(Ss);
  }

  // flux of thermodynamic field q
  __device__ inline double flux(const T* WL, const T* WR, int q) const {
    double uL, fL, usL, uR, fR, usR;
    field_terms<S, DIR>(WL, L, q, sp, SL, Ss, chiL, cnL, ctL, uL, fL, usL);
    field_terms<S, DIR>(WR, R, q, sp, SR, Ss, chiR, cnR, ctR, uR, fR, usR);
    const double fc = 0.5 * (fL + fR) + 0.5 * (ph * SL * (usL - uL) + aS * (usL - usR) + ph * SR * (usR - uR));
    const double fsl = fL + SL * (usL - uL), fsr = fR + SR * (usR - uR);
    return mode == FAN_CENTRAL ? fc : mode == FAN_LEFT ? fL : mode == FAN_RIGHT ? fR : mode == FAN_STAR_L ? fsl : fsr;
  }

  // wall velocity (the flux formula applied to the unit field)
  __device__ inline double ustar() const {
    const double uc = 0.5 * (L.un + R.un) + 0.5 * (ph * SL * (chiL - 1.0) + aS * (chiL - chiR) + ph * SR * (chiR - 1.0));
    return mode == FAN_CENTRAL ? uc : mode == FAN_LEFT ? L.un : mode == FAN_RIGHT ? R.un
         : mode == FAN_STAR_L ? L.un + SL * (chiL - 1.0) : R.un + SR * (chiR - 1.0);
  }

  // wall stretch row Vbar*_{DIR,b}
  __device__ inline double vstar(const T* WL, const T* WR, int b) const {
    const double vl = (double)WL[S::wV(DIR, b)], vr = (double)WR[S::wV(DIR, b)];
    const double w = (Ss - SL) * frcp(SR - SL);
    const double vc = vr * cnR + w * (vl * cnL - vr * cnR);
    return mode == FAN_CENTRAL ? vc : mode == FAN_LEFT ? vl : mode == FAN_RIGHT ? vr
         : mode == FAN_STAR_L ? vl * cnL : vr * cnR;
  }
};

// ---------------------------------------------------------------------------
// Rigid-body velocity and seeding states (Sec. 2.3, Sec. 3.2)
// ---------------------------------------------------------------------------

// Rigid velocity of body B at point x, tc after the motion was set: the
// body's centre has moved by v tc since, which is evaluated as x - v tc
// against the centre of that time.
template <int B>
__device__ inline void body_velocity(const Params& P, const double x[3], double tc, double v[3]) {
  const double xs0 = x[0] - P.vr[B][0] * tc, xs1 = x[1] - P.vr[B][1] * tc, xs2 = x[2] - P.vr[B][2] * tc;
  const double d0 = xs0 - P.ctr[B][0], d1 = xs1 - P.ctr[B][1], d2 = xs2 - P.ctr[B][2];
  v[0] = P.vr[B][0] + P.om[B][1] * d2 - P.om[B][2] * d1;
  v[1] = P.vr[B][1] + P.om[B][2] * d0 - P.om[B][0] * d2;
  v[2] = P.vr[B][2] + P.om[B][0] * d1 - P.om[B][1] * d0;
}

template <int B>
__device__ inline bool body_owns(const Params& P, const double x[3], double tc) {
  const double xs0 = x[0] - P.vr[B][0] * tc, xs1 = x[1] - P.vr[B][1] * tc, xs2 = x[2] - P.vr[B][2] * tc;
  return (xs0 >= P.blo[B][0]) & (xs0 < P.bhi[B][0]) & (xs1 >= P.blo[B][1]) & (xs1 < P.bhi[B][1]) &
         (xs2 >= P.blo[B][2]) & (xs2 < P.bhi[B][2]);
}

// Body B's claim on x: its velocity replaces v where no earlier body has
// claimed x and x lies in B's ownership box. Both candidates are computed and
// selected, without branches: branches that differ only in the body's
// offsets into the launch parameters get merged into one load through a
// chosen address, which copies the parameters to scratch memory.
template <int B>
__device__ inline void claim_body(const Params& P, const double x[3], double tc, double v[3], bool& taken) {
  double w[3];
  body_velocity<B>(P, x, tc, w);
  const bool own = !taken && B < P.nbody && body_owns<B>(P, x, tc);
  v[0] = own ? w[0] : v[0];
  v[1] = own ? w[1] : v[1];
  v[2] = own ? w[2] : v[2];
  taken = taken || own;
}

// Rigid velocity at point x (Sec. 2.3: v_r = v + omega x (x - c) of the body
// that owns x: the first body 1.. whose ownership box holds x, else body 0).
// MB = false: body 0 only, for launches with one body (the claims cost the
// sweeps registers even where the run-time test skips them).
template <bool MB>
__device__ inline void rigid_velocity(const Params& P, const double x[3], double tc, double v[3]) {
  static_assert(kMaxBody == 4, "one claim per body");
  body_velocity<0>(P, x, tc, v);
  if (MB && P.nbody > 1) {
    bool taken = false;
    claim_body<1>(P, x, tc, v, taken);
    claim_body<2>(P, x, tc, v, taken);
    claim_body<3>(P, x, tc, v, taken);
  }
}

// Mirror state of the seeding routine, as the Householder reflection
// P = I - 2 n n^T (rotation-independent form of rotate, reflect the normal
// velocity and the normal-tangential stretch components, rotate back):
// u' = P u + 2 (v_r . n) n, Vbar' = P Vbar P, scalars unchanged.
template <class S>
__device__ inline void mirror(const double* Wi, const double n[3], const double v[3], double* Wm) {
#pragma unroll
  for (int q = 0; q < S::NF; ++q) Wm[q] = Wi[q];
  double un = 0.0, vn = 0.0;
#pragma unroll
  for (int a = 0; a < S::D; ++a) { un += Wi[S::wU(a)] * n[a]; vn += v[a] * n[a]; }
#pragma unroll
  for (int a = 0; a < S::D; ++a) Wm[S::wU(a)] = Wi[S::wU(a)] - 2.0 * un * n[a] + 2.0 * vn * n[a];
  if constexpr (S::S) {
    // P V P = V - 2 n (n^T V) - 2 (V n) n^T + 4 (n^T V n) n n^T
    double nV[3], Vn[3], nVn = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      nV[b] = n[0] * Wi[S::wV(0, b)] + n[1] * Wi[S::wV(1, b)] + n[2] * Wi[S::wV(2, b)];
      Vn[b] = Wi[S::wV(b, 0)] * n[0] + Wi[S::wV(b, 1)] * n[1] + Wi[S::wV(b, 2)] * n[2];
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) nVn += nV[b] * n[b];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        Wm[S::wV(a, b)] = Wi[S::wV(a, b)] - 2.0 * n[a] * nV[b] - 2.0 * Vn[a] * n[b] + 4.0 * nVn * n[a] * n[b];
  }
}

// Riemann-problem seeding state: HLLC right star state of (mirror, interp)
// along n, in primitive form (phasic densities * chi_R, normal velocity S*,
// p* = p_R + rho_R (S_R - u_R)(S* - u_R), Vbar* = D Vbar_R with the
// uniaxial stretch D along n; other fields from the interpolated state).
template <class S>
__device__ inline void riemann_seed(const Params& P, const double* Wm, const double* Wi, const double n[3],
                                    double* Wo) {
  double phL[kMaxMat], rL[kMaxMat], phR[kMaxMat], rR[kMaxMat];
  phases_w<S>(Wm, phL, rL);
  phases_w<S>(Wi, phR, rR);
  double rhoL = 0.0, rhoR = 0.0;
#pragma unroll
  for (int l = 0; l < S::N; ++l) { rhoL += phL[l] * rL[l]; rhoR += phR[l] * rR[l]; }
  double uL = 0.0, uR = 0.0;
#pragma unroll
  for (int a = 0; a < S::D; ++a) { uL += Wm[S::wU(a)] * n[a]; uR += Wi[S::wU(a)] * n[a]; }
  double J2L = 0.0, J2R = 0.0, HL[9], HR[9];
  if constexpr (S::S) {
    hencky3(Wm + S::wV(0, 0), HL, J2L);
    hencky3(Wi + S::wV(0, 0), HR, J2R);
  }
  double c2L, GL, yL, c2R, GR, yR;
  mix_c2_G<S>(P, phL, rL, J2L, Wm[S::wP], c2L, GL, yL);
  mix_c2_G<S>(P, phR, rR, J2R, Wi[S::wP], c2R, GR, yR);
  double PL = Wm[S::wP], PR = Wi[S::wP];
  if constexpr (S::S) {
    double nHnL = 0.0, nHnR = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) { nHnL += n[a] * HL[3 * a + b] * n[b]; nHnR += n[a] * HR[3 * a + b] * n[b]; }
    PL -= 2.0 * GL * nHnL;
    PR -= 2.0 * GR * nHnR;
  }
  const double cL = sqrt(c2L), cR = sqrt(c2R);
  const double SL = fmin(uL - cL, uR - cR);
  const double SR = fmax(uL + cL, uR + cR);
  const double mL = rhoL * (SL - uL), mR = rhoR * (SR - uR);
  const double Ss = (PR - PL + uL * mL - uR * mR) / (mL - mR);
  const double chi = (SR - uR) / (SR - Ss);
#pragma unroll
  for (int q = 0; q < S::NF; ++q) Wo[q] = Wi[q];
#pragma unroll
  for (int l = 0; l < S::N; ++l) Wo[S::wRHO(l)] = Wi[S::wRHO(l)] * chi;
#pragma unroll
  for (int a = 0; a < S::D; ++a) Wo[S::wU(a)] = Wi[S::wU(a)] + (Ss - uR) * n[a];
  Wo[S::wP] = Wi[S::wP] + rhoR * (SR - uR) * (Ss - uR);
  if constexpr (S::S) {
    const double ct = cbrt(chi), cn = 1.0 / (ct * ct);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double Dak = (a == k ? ct : 0.0) + (cn - ct) * n[a] * n[k];
          s += Dak * Wi[S::wV(k, b)];
        }
        Wo[S::wV(a, b)] = s;
      }
  }
}

// ---------------------------------------------------------------------------
// Per-stage sources of the elastoplastic system: unit-determinant
// renormalisation of Vbar and perfect-plasticity radial return in Hencky
// space (sigma_eq = sqrt(6) G |H| scaled back to the mixture yield stress
// through Vbar <- exp((s-1) H) Vbar; eps_p grows by sqrt(2/3)(1-s)|H|;
// rho E unchanged).
// ---------------------------------------------------------------------------
__device__ inline double exp_w(int k) {
  double f = 1.0;
  for (int j = 2; j <= k; ++j) f *= (double)j;
  return 1.0 / f;
}

// E = exp(a H) for symmetric H: by eigen-decomposition.
__device__ __forceinline__ void plastic_exp_eig(double a, const double* H, double* E) {
  double A[3][3], Q[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = a * H[3 * i + j];
  jacobi3(A, Q);
  double ev[3];
  for (int k = 0; k < 3; ++k) ev[k] = exp(A[k][k]);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) E[3 * i + j] = Q[i][0] * ev[0] * Q[j][0] + Q[i][1] * ev[1] * Q[j][1] + Q[i][2] * ev[2] * Q[j][2];
}

// E = exp(a H): the exponential series for |a H| <= 1, else by
// eigen-decomposition.
__device__ inline void plastic_exp(double a, const double* H, double* E) {
  SymM A;
  A.a00 = a * H[0]; A.a11 = a * H[4]; A.a22 = a * H[8];
  A.a01 = a * H[1]; A.a02 = a * H[2]; A.a12 = a * H[5];
  const SymM A2 = sym_sq(A);
  const double t2 = A2.a00 + A2.a11 + A2.a22;
  if (!(t2 <= 1.0)) {
    plastic_exp_eig(a, H, E);
    return;
  }
  double c0, c1, c2;
  ch_series<40>(A, sqrt(t2), exp_w, c0, c1, c2);
  c0 += 1.0;  // the k = 0 term
  E[0] = c0 + c1 * A.a00 + c2 * A2.a00;
  E[4] = c0 + c1 * A.a11 + c2 * A2.a11;
  E[8] = c0 + c1 * A.a22 + c2 * A2.a22;
  E[1] = E[3] = c1 * A.a01 + c2 * A2.a01;
  E[2] = E[6] = c1 * A.a02 + c2 * A2.a02;
  E[5] = E[7] = c1 * A.a12 + c2 * A2.a12;
}

// Whether the radial return may act on a cell: false when it provably does
// not. For X = Vbar Vbar^T - I with tau = |X|_F < 1 every eigenvalue x of X
// has |x| <= tau and |ln(1 + x)| <= |x| / (1 - |x|), so the Hencky strain
// obeys |H|_F <= tau / (2 (1 - tau)); with the mixture G and yield stress
// (neither depends on the strain) sigma_eq = sqrt(6) G |H|_F then stays at
// or below sqrt(6) G tau / (2 (1 - tau)). When that bound (1% margin for
// rounding) is at most sigma_Y, or sigma_Y = 0, the return is not applied,
// exactly as the full test would decide, so the cell skips the closure.
template <class S, typename T>
__device__ inline bool may_yield(const Params& P, const T* U, const double* V) {
  double phi[kMaxMat], s = 0.0;
#pragma unroll
  for (int l = 0; l < S::N - 1; ++l) {
    phi[l] = (double)U[S::cPHI(l)];
    s += phi[l];
  }
  phi[S::N - 1] = 1.0 - s;
  double nG = 0.0, nY = 0.0, den = 0.0;
#pragma unroll
  for (int l = 0; l < S::N; ++l) {
    const MatDev& m = P.mat[l];
    if (m.kind == EOS_ROMENSKII) {
      const double rho = (double)U[S::cA(l)] / phi[l];
      nG += phi[l] * m.G0 * pow_small(rho * m.invrho0, m.ibeta1, m.beta + 1.0) * m.invGam;
    }
    nY += phi[l] * m.sigY * m.invGam;
    den += phi[l] * m.invGam;
  }
  if (!(nY > 0.0)) return false;  // sigma_Y = 0: no return
  const double x00 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2] - 1.0;
  const double x11 = V[3] * V[3] + V[4] * V[4] + V[5] * V[5] - 1.0;
  const double x22 = V[6] * V[6] + V[7] * V[7] + V[8] * V[8] - 1.0;
  const double x01 = V[0] * V[3] + V[1] * V[4] + V[2] * V[5];
  const double x02 = V[0] * V[6] + V[1] * V[7] + V[2] * V[8];
  const double x12 = V[3] * V[6] + V[4] * V[7] + V[5] * V[8];
  const double tau = sqrt(x00 * x00 + x11 * x11 + x22 * x22 + 2.0 * (x01 * x01 + x02 * x02 + x12 * x12));
  if (!(tau < 0.5)) return true;
  // sqrt(6) G tau / (2 (1 - tau)) > sigma_Y, both sides times den > 0
  return 1.01 * 2.449489742783178 * nG * tau > 2.0 * (1.0 - tau) * nY;
}

template <class S, typename T>
__device__ inline void solid_sources(const Params& P, T* U) {
  double V[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) V[q] = (double)U[S::cV(0, 0) + q];
  const double det = V[0] * (V[4] * V[8] - V[5] * V[7]) - V[1] * (V[3] * V[8] - V[5] * V[6]) +
                     V[2] * (V[3] * V[7] - V[4] * V[6]);
  const double sc = 1.0 / cbrt(det);
#pragma unroll
  for (int q = 0; q < 9; ++q) V[q] *= sc;
  if (P.plastic && may_yield<S>(P, U, V)) {
    T Ut[S::NF], Wt[S::NF];
#pragma unroll
    for (int q = 0; q < S::NF; ++q) Ut[q] = U[q];
#pragma unroll
    for (int q = 0; q < 9; ++q) Ut[S::cV(0, 0) + q] = (T)V[q];
    double H[9], J2;
    cons_to_prim<S>(P, Ut, Wt, H, &J2);
    double phi[kMaxMat], rl[kMaxMat];
    phases_w<S>(Wt, phi, rl);
    double c2, G, sY;
    mix_c2_G<S>(P, phi, rl, J2, (double)Wt[S::wP], c2, G, sY);
    const double Hn = sqrt(J2);
    const double seq = 2.449489742783178 * G * Hn;
    if (sY > 0.0 && seq > sY) {
      const double s = sY / seq;
      // exp((s-1) H)
      double X[9], Vn[9];
      plastic_exp(s - 1.0, H, X);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Vn[3 * a + b] = X[3 * a] * V[b] + X[3 * a + 1] * V[3 + b] + X[3 * a + 2] * V[6 + b];
#pragma unroll
      for (int q = 0; q < 9; ++q) V[q] = Vn[q];
      const int sp = P.solid_phase;
      const double as = pick<S::N>(phi, sp) * pick<S::N>(rl, sp);
      U[S::cEP] = (T)((double)U[S::cEP] + as * 0.816496580927726 * (1.0 - s) * Hn);
    }
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) U[S::cV(0, 0) + q] = (T)V[q];
}

}  // namespace rbdi
