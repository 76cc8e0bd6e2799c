// rbdi_oracle.cpp -- plain, slow, FP64 CPU oracle of the diffuse-interface
// rigid-body finite-volume step of Wallis, Barton & Nikiforakis, "A unified
// diffuse interface method for the interaction of rigid bodies with
// elastoplastic solids and multi-phase mixtures" (arXiv 2111.11806).
//
// TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg
// of the benchmark load this library. The product library (librbdi) never
// links, includes or calls it, and it shares no code with the HIP path.
//
// Each routine names the passage of the paper it follows. Where the paper is
// silent, garbled or defers to a work that is not reproduced in it, the
// reading taken is stated at the routine as "Reading:".
//
// Parity status of each part (what pins it) is listed in the header of
// oracle/__init__.py.
//
// Build: g++ -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fast-math).

#include <omp.h>
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#define ORC_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr int kMaxMat = 3;
constexpr int kMaxBodies = 4;  // rigid bodies with their own motion
constexpr int kMaxF = 32;

enum { EOS_IDEAL = 0, EOS_STIFFENED = 1, EOS_ROMENSKII = 2 };
enum { BC_TRANSMISSIVE = 0, BC_REFLECTIVE = 1, BC_DIRICHLET = 2, BC_PERIODIC = 3 };
enum { REC_MUSCL = 0, REC_BVD_THINC = 1 };
enum { RS_HLLC = 0, RS_HLLC_LM = 1 };
enum { SEED_ORIGINAL = 0, SEED_RIEMANN = 1, SEED_NONE = 2 };
enum { PROBE_STEPOUT = 0, PROBE_FIXED = 1 };
enum { NORMAL_YOUNGS = 0, NORMAL_ELVIRA = 1 };

struct Material {
  int kind = EOS_IDEAL;
  double gamma = 1.4, pinf = 0.0;                          // ideal / stiffened gas
  double rho0 = 1, K0 = 0, G0 = 0, alpha = 1, beta = 0, Gamma0 = 1;  // Romenskii
  double sigY = 0;                                         // perfect plasticity
};

// Field layout of the conserved vector U and the primitive vector W of the
// reduced-equation multi-material system (Sec. 2.1.1 and Sec. 2.3-2.4).
//   U = (phi_l rho_l [N], rho u [dim], rho E, phi_l [N-1], V [9], a_s eps_p, r)
//   W = (phi_l [N-1], rho_l [N], u [dim], p, V [9], eps_p, r)
// V and eps_p are present only for the elastoplastic system.
struct Layout {
  int dim = 1, nmat = 1, solid = 0, n = 0;
  void init(int d, int nm, int s) {
    dim = d; nmat = nm; solid = s;
    n = 2 * nmat + dim + 1 + (solid ? 10 : 0);
  }
  int A(int l) const { return l; }
  int M(int a) const { return nmat + a; }
  int E() const { return nmat + dim; }
  int PHI(int l) const { return nmat + dim + 1 + l; }
  int V(int a, int b) const { return 2 * nmat + dim + 3 * a + b; }
  int EP() const { return 2 * nmat + dim + 9; }
  int R() const { return n - 1; }
  int wPHI(int l) const { return l; }
  int wRHO(int l) const { return nmat - 1 + l; }
  int wU(int a) const { return 2 * nmat - 1 + a; }
  int wP() const { return 2 * nmat - 1 + dim; }
  int wV(int a, int b) const { return 2 * nmat + dim + 3 * a + b; }
  int wEP() const { return 2 * nmat + dim + 9; }
  int wR() const { return n - 1; }
};

// ---------------------------------------------------------------------------
// Small linear algebra
// ---------------------------------------------------------------------------

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix, iterated until
// the off-diagonal part is negligible: A = Q diag(lam) Q^T, Q's columns are
// the eigenvectors.
void sym_eig3(const double Ain[3][3], double lam[3], double Q[3][3]) {
  double A[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) { A[i][j] = Ain[i][j]; Q[i][j] = (i == j) ? 1.0 : 0.0; }
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    double diag = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-34 * diag || off == 0.0) break;
    for (int p = 0; p < 2; ++p) {
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {  // A <- A J
          double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {  // A <- J^T A
          double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {  // Q <- Q J
          double qkp = Q[k][p], qkq = Q[k][q];
          Q[k][p] = c * qkp - s * qkq;
          Q[k][q] = s * qkp + c * qkq;
        }
      }
    }
  }
  for (int i = 0; i < 3; ++i) lam[i] = A[i][i];
}

// Hencky strain of the elastic stretch (Sec. 2.1.2): dev H = ln Vbar. The
// stored Vbar need not stay symmetric under its evolution equation, so the
// strain is taken from the left Cauchy-Green tensor b = Vbar Vbar^T:
// H = (1/2) ln b, which equals ln Vbar when Vbar is symmetric positive.
void hencky(const double V[3][3], double H[3][3]) {
  double b[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += V[i][k] * V[j][k];
      b[i][j] = s;
    }
  double lam[3], Q[3][3];
  sym_eig3(b, lam, Q);
  double hl[3];
  for (int k = 0; k < 3; ++k) hl[k] = 0.5 * std::log(lam[k]);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += Q[i][k] * hl[k] * Q[j][k];
      H[i][j] = s;
    }
}

// exp of a symmetric 3x3 matrix by eigen-decomposition (used by the plastic
// return, which rescales the Hencky strain).
void sym_exp(const double S[3][3], double X[3][3]) {
  double lam[3], Q[3][3];
  sym_eig3(S, lam, Q);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += Q[i][k] * std::exp(lam[k]) * Q[j][k];
      X[i][j] = s;
    }
}

double det3(const double A[3][3]) {
  return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
         A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
         A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

// ---------------------------------------------------------------------------
// Thermodynamics (Sec. 2.1.2 Thermodynamics, Sec. 2.1.3 Closure Models)
// ---------------------------------------------------------------------------

// Reference curves of the Mie-Gruneisen form p = p_ref + rho Gamma (e - e_ref)
// (Sec. 2.1.2, Mie-Gruneisen equation) for one phase at phasic density rho and
// shear-strain invariant J2 = tr(dev H dev H^T).
struct PhaseRef {
  double rhoe_ref;   // rho * e_ref
  double p_ref;      // rho^2 d e_ref / d rho
  double Gam;        // Gruneisen coefficient
  double dGam_drho;  // its density derivative (zero for every EOS used here)
  double dpref_drho; // d p_ref / d rho
  double rho_deref;  // rho * d e_ref / d rho  (= p_ref / rho)
  double G;          // shear modulus
};

PhaseRef phase_ref(const Material& m, double rho, double J2) {
  PhaseRef r{};
  if (m.kind == EOS_IDEAL) {
    // Ideal gas (Sec. 2.1.3): p_ref = e_ref = 0, gamma = Gamma + 1.
    r.Gam = m.gamma - 1.0;
  } else if (m.kind == EOS_STIFFENED) {
    // Stiffened gas expressed through the Mie-Gruneisen reference curves.
    // Reading (the paper names no stiffened gas): e_ref = p_inf / rho and
    // p_ref = -p_inf, which satisfy p_ref = rho^2 de_ref/drho and give
    // p = (gamma - 1) rho e - gamma p_inf.
    r.Gam = m.gamma - 1.0;
    r.rhoe_ref = m.pinf;
    r.p_ref = -m.pinf;
    r.rho_deref = -m.pinf / rho;
  } else {
    // Romenskii EOS (Sec. 2.1.3): Gamma = Gamma0,
    // e_ref = K0/(2 rho alpha^2) ((rho/rho0)^alpha - 1)^2 + G(rho) J2 / rho,
    // G(rho) = G0 (rho/rho0)^(beta+1), p_ref = rho^2 d e_ref / d rho.
    const double x = rho / m.rho0;
    const double y = std::pow(x, m.alpha);
    const double G = m.G0 * std::pow(x, m.beta + 1.0);
    const double k = m.K0 / (2.0 * m.alpha * m.alpha);
    r.Gam = m.Gamma0;
    r.G = G;
    r.rhoe_ref = k * (y - 1.0) * (y - 1.0) + G * J2;
    // rho^2 de_ref/drho, differentiated term by term at fixed J2.
    r.p_ref = k * (y - 1.0) * ((2.0 * m.alpha - 1.0) * y + 1.0) + m.beta * G * J2;
    r.rho_deref = r.p_ref / rho;
    r.dpref_drho = (m.K0 / m.alpha) * ((2.0 * m.alpha - 1.0) * y - m.alpha + 1.0) * y / rho +
                   m.beta * (m.beta + 1.0) * G * J2 / rho;
  }
  return r;
}

// Squared phase sound speed, c^2 ~ a^2 + (4/3) b^2 with a^2 the isentropic
// derivative written in terms of the reference curves and b^2 = G / rho
// (Sec. 2.1.2, sound-speed approximation).
double phase_c2(const PhaseRef& r, double rho, double p) {
  const double a2 = r.Gam * p / rho + (p - r.p_ref) * (1.0 / rho + r.dGam_drho) +
                    (r.dpref_drho - r.Gam * r.rho_deref);
  return a2 + (4.0 / 3.0) * r.G / rho;
}

struct Oracle;

struct CellThermo {
  double rho, p, c2, G, sigY;
  double H[3][3];
  double J2;
  double sigma[3][3];  // Cauchy stress, tension positive
};

// ---------------------------------------------------------------------------
// The oracle instance
// ---------------------------------------------------------------------------
struct Oracle {
  Layout L;
  int dim = 1, n[3] = {1, 1, 1}, ng = 3, N[3] = {1, 1, 1}, g[3] = {0, 0, 0};
  double dx[3] = {1, 1, 1}, x0[3] = {0, 0, 0};
  int bc[6] = {0, 0, 0, 0, 0, 0};
  std::vector<double> bcU[6];
  int recon = REC_BVD_THINC, riemann = RS_HLLC, seed = SEED_ORIGINAL, probe = PROBE_STEPOUT;
  int normal = NORMAL_YOUNGS;
  int plastic = 1;
  double beta_thinc = 1.6;
  double lm_mach = 0.1;
  // Void-opening face modifier at solid-rigid faces (Sec. 3.2, end): off by
  // default; when on, gap_W is the primitive state of the gas that fills an
  // opening gap.
  int face_mod = 0;
  double gap_W[kMaxF] = {};
  int nmat = 1, solid_phase = -1;
  Material mat[kMaxMat];
  // Rigid motions: body 0 moves every point no other body claims; body
  // k >= 1 claims the points of its ownership box [lo, hi). Centres and boxes
  // are those of the start of the current step.
  int nbody = 1;
  double vr[kMaxBodies][3] = {}, om[kMaxBodies][3] = {}, ctr[kMaxBodies][3] = {};
  double box_lo[kMaxBodies][3] = {}, box_hi[kMaxBodies][3] = {};
  double t = 0;
  size_t ncell = 0;   // cells including ghosts
  std::vector<double> U;  // [L.n][ncell]
  // diagnostics
  long probe_fail = 0, seeded = 0, fallback = 0;

  size_t idx(int i, int j, int k) const {
    return ((size_t)(k + g[2]) * N[1] + (size_t)(j + g[1])) * N[0] + (size_t)(i + g[0]);
  }
  double* f(int q) { return U.data() + (size_t)q * ncell; }
  const double* f(int q) const { return U.data() + (size_t)q * ncell; }
  size_t stride(int d) const { return d == 0 ? 1 : (d == 1 ? (size_t)N[0] : (size_t)N[0] * N[1]); }
  double cell_volume() const {
    double v = 1;
    for (int d = 0; d < dim; ++d) v *= dx[d];
    return v;
  }
  double xc(int d, int i) const { return x0[d] + (i + 0.5) * dx[d]; }
  double nint() const { return (double)n[0] * n[1] * n[2]; }

  // ---- closure (Sec. 2.2 Mixture Rules) -----------------------------------

  void phases_from_prim(const double* W, double* phi, double* rho) const {
    double s = 0;
    for (int l = 0; l < nmat - 1; ++l) { phi[l] = W[L.wPHI(l)]; s += phi[l]; }
    phi[nmat - 1] = 1.0 - s;  // volume fractions sum to one (Sec. 2.2)
    for (int l = 0; l < nmat; ++l) rho[l] = W[L.wRHO(l)];
  }

  void stretch_from(const double* X, int base, double V[3][3]) const {
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) V[a][b] = X[base + 3 * a + b];
  }

  // Mixture pressure-independent parts of the closure at given phase state.
  // Returns the mixture pressure from rho e by the isobaric inversion
  // (Sec. 2.2): p = [rho e - sum phi_l (rho_l e_ref,l - p_ref,l/Gamma_l)] /
  //                 sum (phi_l / Gamma_l).
  double mixture_pressure(const double* phi, const double* rho, double J2, double rhoe) const {
    double num = rhoe, den = 0;
    for (int l = 0; l < nmat; ++l) {
      PhaseRef r = phase_ref(mat[l], rho[l], J2);
      num -= phi[l] * (r.rhoe_ref - r.p_ref / r.Gam);
      den += phi[l] / r.Gam;
    }
    return num / den;
  }

  // The inverse: rho e at given p (the same isobaric relation solved for rho e).
  double mixture_rhoe(const double* phi, const double* rho, double J2, double p) const {
    double s = 0, den = 0;
    for (int l = 0; l < nmat; ++l) {
      PhaseRef r = phase_ref(mat[l], rho[l], J2);
      s += phi[l] * (r.rhoe_ref - r.p_ref / r.Gam);
      den += phi[l] / r.Gam;
    }
    return p * den + s;
  }

  // Thermodynamic state of a primitive vector: mixture density, sound speed
  // (Sec. 2.2, sound-speed mixture rule), shear modulus (Sec. 2.2, shear
  // modulus mixture rule), Hencky strain and total stress
  // sigma = -p I + 2 G dev H (Sec. 2.2 total stress).
  // Reading: the paper prints sigma = p I + dev sigma, which contradicts its
  // own fluxes rho u u - sigma and sigma = -p delta of the reduced system;
  // the tension-positive sign is used. The sound-speed mixture rule is taken
  // with the mass fraction Y_l alone (the extra phi_l in the printed rule is
  // read as a typesetting slip; both agree in pure cells).
  void thermo_from_prim(const double* W, CellThermo& th) const {
    double phi[kMaxMat], rho[kMaxMat];
    phases_from_prim(W, phi, rho);
    th.rho = 0;
    for (int l = 0; l < nmat; ++l) th.rho += phi[l] * rho[l];
    th.p = W[L.wP()];
    std::memset(th.H, 0, sizeof(th.H));
    th.J2 = 0;
    if (L.solid) {
      double V[3][3];
      stretch_from(W, L.wV(0, 0), V);
      hencky(V, th.H);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) th.J2 += th.H[a][b] * th.H[a][b];
    }
    double num_c = 0, num_G = 0, num_Y = 0, den = 0;
    for (int l = 0; l < nmat; ++l) {
      PhaseRef r = phase_ref(mat[l], rho[l], th.J2);
      const double Yl = phi[l] * rho[l] / th.rho;
      num_c += Yl * phase_c2(r, rho[l], th.p) / r.Gam;
      num_G += phi[l] * r.G / r.Gam;
      num_Y += phi[l] * mat[l].sigY / r.Gam;
      den += phi[l] / r.Gam;
    }
    th.c2 = num_c / den;
    th.G = num_G / den;
    th.sigY = num_Y / den;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        th.sigma[a][b] = (a == b ? -th.p : 0.0) + 2.0 * th.G * th.H[a][b];
  }

  // Conserved -> primitive (Sec. 2.2): rho = sum phi_l rho_l, rho e = rho E -
  // rho |u|^2 / 2, then the isobaric pressure inversion.
  void cons_to_prim(const double* Uc, double* W) const {
    double phi[kMaxMat], rho[kMaxMat];
    double s = 0;
    for (int l = 0; l < nmat - 1; ++l) { phi[l] = Uc[L.PHI(l)]; s += phi[l]; }
    phi[nmat - 1] = 1.0 - s;
    double rhom = 0;
    for (int l = 0; l < nmat; ++l) { rho[l] = Uc[L.A(l)] / phi[l]; rhom += Uc[L.A(l)]; }
    double u[3] = {0, 0, 0}, ke = 0;
    for (int a = 0; a < dim; ++a) { u[a] = Uc[L.M(a)] / rhom; ke += u[a] * Uc[L.M(a)]; }
    const double rhoe = Uc[L.E()] - 0.5 * ke;
    double J2 = 0;
    if (L.solid) {
      double V[3][3], H[3][3];
      stretch_from(Uc, L.V(0, 0), V);
      hencky(V, H);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) J2 += H[a][b] * H[a][b];
      for (int q = 0; q < 9; ++q) W[L.wV(0, 0) + q] = Uc[L.V(0, 0) + q];
      const double as = phi[solid_phase] * rho[solid_phase];
      W[L.wEP()] = Uc[L.EP()] / as;
    }
    for (int l = 0; l < nmat - 1; ++l) W[L.wPHI(l)] = phi[l];
    for (int l = 0; l < nmat; ++l) W[L.wRHO(l)] = rho[l];
    for (int a = 0; a < dim; ++a) W[L.wU(a)] = u[a];
    W[L.wP()] = mixture_pressure(phi, rho, J2, rhoe);
    W[L.wR()] = Uc[L.R()];
  }

  void prim_to_cons(const double* W, double* Uc) const {
    double phi[kMaxMat], rho[kMaxMat];
    phases_from_prim(W, phi, rho);
    double rhom = 0;
    for (int l = 0; l < nmat; ++l) { Uc[L.A(l)] = phi[l] * rho[l]; rhom += phi[l] * rho[l]; }
    double ke = 0;
    for (int a = 0; a < dim; ++a) {
      Uc[L.M(a)] = rhom * W[L.wU(a)];
      ke += rhom * W[L.wU(a)] * W[L.wU(a)];
    }
    double J2 = 0;
    if (L.solid) {
      double V[3][3], H[3][3];
      stretch_from(W, L.wV(0, 0), V);
      hencky(V, H);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) J2 += H[a][b] * H[a][b];
      for (int q = 0; q < 9; ++q) Uc[L.V(0, 0) + q] = W[L.wV(0, 0) + q];
      Uc[L.EP()] = phi[solid_phase] * rho[solid_phase] * W[L.wEP()];
    }
    Uc[L.E()] = mixture_rhoe(phi, rho, J2, W[L.wP()]) + 0.5 * ke;
    for (int l = 0; l < nmat - 1; ++l) Uc[L.PHI(l)] = phi[l];
    Uc[L.R()] = W[L.wR()];
  }

  // Admissibility of a reconstructed primitive state. Reading (the paper
  // gives no positivity treatment): phase densities positive, every volume
  // fraction in [0,1], and p + p_inf > 0 for every fluid phase.
  bool admissible(const double* W) const {
    double phi[kMaxMat], rho[kMaxMat];
    phases_from_prim(W, phi, rho);
    for (int l = 0; l < nmat; ++l) {
      if (!(rho[l] > 0.0)) return false;
      if (!(phi[l] >= 0.0 && phi[l] <= 1.0)) return false;
      if (mat[l].kind != EOS_ROMENSKII) {
        const double pinf = mat[l].kind == EOS_STIFFENED ? mat[l].pinf : 0.0;
        if (!(W[L.wP()] + pinf > 0.0)) return false;
      }
    }
    return true;
  }

  // Rigid-body velocity field v_r(x) = v + omega x (x - c), imposed and
  // one-way (Sec. 2.3), of the body that owns x. Reading: the centre is taken
  // at the start of the step.
  int owner(const double x[3]) const {
    for (int k = 1; k < nbody; ++k) {
      bool in = true;
      for (int a = 0; a < 3; ++a) in = in && x[a] >= box_lo[k][a] && x[a] < box_hi[k][a];
      if (in) return k;
    }
    return 0;
  }
  void rigid_velocity(const double x[3], double v[3]) const {
    const int k = owner(x);
    const double d[3] = {x[0] - ctr[k][0], x[1] - ctr[k][1], x[2] - ctr[k][2]};
    v[0] = vr[k][0] + om[k][1] * d[2] - om[k][2] * d[1];
    v[1] = vr[k][1] + om[k][2] * d[0] - om[k][0] * d[2];
    v[2] = vr[k][2] + om[k][0] * d[1] - om[k][1] * d[0];
  }
  void set_one_body(const double* v, const double* omega, const double* center) {
    nbody = 1;
    for (int a = 0; a < 3; ++a) { vr[0][a] = v[a]; om[0][a] = omega[a]; ctr[0][a] = center[a]; }
  }

  // ---- ghost cells ---------------------------------------------------------
  // Domain boundary conditions (per-configuration; the paper states only the
  // kind per test). Transmissive copies the edge cell; reflective mirrors the
  // cells and negates the normal momentum and conjugates Vbar by the axis
  // reflection; Dirichlet sets a fixed state; periodic wraps.
  void fill_ghosts(std::vector<double>& X) const {
    auto F = [&](int q) { return X.data() + (size_t)q * ncell; };
    for (int d = 0; d < dim; ++d) {
      // ranges: dims < d over full extent (ghosts included), dims > d interior
      int lo[3], hi[3];
      for (int e = 0; e < 3; ++e) {
        if (e >= dim) { lo[e] = 0; hi[e] = 1; }
        else if (e < d) { lo[e] = -g[e]; hi[e] = n[e] + g[e]; }
        else { lo[e] = 0; hi[e] = n[e]; }
      }
      lo[d] = 0; hi[d] = 1;
      for (int k = lo[2]; k < hi[2]; ++k)
        for (int j = lo[1]; j < hi[1]; ++j)
          for (int i = lo[0]; i < hi[0]; ++i) {
            int p[3] = {i, j, k};
            for (int side = 0; side < 2; ++side) {
              const int type = bc[2 * d + side];
              for (int gi = 0; gi < ng; ++gi) {
                int gp[3] = {p[0], p[1], p[2]}, sp[3] = {p[0], p[1], p[2]};
                gp[d] = side == 0 ? -1 - gi : n[d] + gi;
                bool mirror = false;
                if (type == BC_TRANSMISSIVE) sp[d] = side == 0 ? 0 : n[d] - 1;
                else if (type == BC_REFLECTIVE) { sp[d] = side == 0 ? gi : n[d] - 1 - gi; mirror = true; }
                else if (type == BC_PERIODIC) sp[d] = side == 0 ? n[d] - 1 - gi : gi;
                const size_t gc = idx(gp[0], gp[1], gp[2]);
                if (type == BC_DIRICHLET) {
                  for (int q = 0; q < L.n; ++q) F(q)[gc] = bcU[2 * d + side][q];
                  continue;
                }
                const size_t sc = idx(sp[0], sp[1], sp[2]);
                for (int q = 0; q < L.n; ++q) F(q)[gc] = F(q)[sc];
                if (mirror) {
                  F(L.M(d))[gc] = -F(L.M(d))[sc];
                  if (L.solid)
                    for (int a = 0; a < 3; ++a)
                      for (int b = 0; b < 3; ++b)
                        if ((a == d) != (b == d)) F(L.V(a, b))[gc] = -F(L.V(a, b))[sc];
                }
              }
            }
          }
    }
  }

  void prim_all(const std::vector<double>& X, std::vector<double>& Wf) const {
    Wf.assign((size_t)L.n * ncell, 0.0);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)ncell; ++c) {
      double Uc[kMaxF], W[kMaxF];
      for (int q = 0; q < L.n; ++q) Uc[q] = X[(size_t)q * ncell + c];
      cons_to_prim(Uc, W);
      for (int q = 0; q < L.n; ++q) Wf[(size_t)q * ncell + c] = W[q];
    }
  }

  // ---- reconstruction (Sec. 3.1) ------------------------------------------
  // Piecewise-linear MUSCL candidate and THINC candidate of one primitive
  // variable in one cell, from the cell and its two neighbours along the
  // sweep. out = {MUSCL left face, MUSCL right face, THINC left, THINC right}.
  // Reading (limiter, beta and the THINC switch are not given): van Leer
  // limiter; THINC where the cell is strictly monotone, with steepness beta.
  // The THINC face values are the exact face values of
  //   q(X) = q_min + dq/2 (1 + theta tanh(beta (X - Xc))), X in [0,1],
  // whose cell average equals the cell value; Xc is solved in closed form
  // from the cell average (tanh integrates to a log of cosh).
  void candidates(double qm, double q0, double qp, double out[4]) const {
    const double a = qp - q0, b = q0 - qm;
    double slope = 0.0;
    if (a * b > 0.0) slope = 2.0 * a * b / (a + b);
    out[0] = q0 - 0.5 * slope;
    out[1] = q0 + 0.5 * slope;
    out[2] = out[0];
    out[3] = out[1];
    if (recon == REC_BVD_THINC && a * b > 0.0) {
      const double beta = beta_thinc;
      const double qmin = std::min(qm, qp);
      const double dq = std::fabs(qp - qm);
      const double theta = qp > qm ? 1.0 : -1.0;
      const double C = (q0 - qmin) / dq;
      // tanh(beta Xc) from the cell-average condition
      const double T = (std::cosh(beta) - std::exp(theta * beta * (2.0 * C - 1.0))) / std::sinh(beta);
      const double tb = std::tanh(beta);
      out[2] = qmin + 0.5 * dq * (1.0 - theta * T);
      out[3] = qmin + 0.5 * dq * (1.0 + theta * (tb - T) / (1.0 - tb * T));
    }
  }

  // MUSCL-BVD-THINC selection (Sec. 3.1): a cell takes its THINC faces only
  // when their total boundary variation, measured against the neighbours'
  // faces of the same scheme, is strictly lower than MUSCL's.
  // cm, c0, cp: candidates of the left neighbour, the cell, the right one.
  void bvd_select(const double cm[4], const double c0[4], const double cp[4], double& ql,
                  double& qr) const {
    if (recon != REC_BVD_THINC) { ql = c0[0]; qr = c0[1]; return; }
    const double tbv_m = std::fabs(cm[1] - c0[0]) + std::fabs(c0[1] - cp[0]);
    const double tbv_t = std::fabs(cm[3] - c0[2]) + std::fabs(c0[3] - cp[2]);
    if (tbv_t < tbv_m) { ql = c0[2]; qr = c0[3]; }
    else { ql = c0[0]; qr = c0[1]; }
  }

  // ---- Riemann solver (Sec. 3.1; HLLC-LM in Sec. 4.3) ----------------------
  // Physical flux along direction d of the thermodynamic part of U (all
  // conserved fields except r), Sec. 2.1.1 and the compact form of Sec. 3.
  void phys_flux(const double* W, const double* Uc, const CellThermo& th, int d, double* F) const {
    const double ud = W[L.wU(d)];
    double u[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) u[a] = W[L.wU(a)];
    for (int l = 0; l < nmat; ++l) F[L.A(l)] = Uc[L.A(l)] * ud;
    for (int a = 0; a < dim; ++a) F[L.M(a)] = Uc[L.M(a)] * ud - th.sigma[a][d];
    double work = 0;
    for (int a = 0; a < 3; ++a) work += u[a] * th.sigma[a][d];
    F[L.E()] = Uc[L.E()] * ud - work;
    for (int l = 0; l < nmat - 1; ++l) F[L.PHI(l)] = Uc[L.PHI(l)] * ud;
    if (L.solid) {
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) F[L.V(a, b)] = Uc[L.V(a, b)] * ud - Uc[L.V(d, b)] * u[a];
      F[L.EP()] = Uc[L.EP()] * ud;
    }
  }

  // Star state of side K (HLLC, Toro). chi = (S_K - u_K)/(S_K - S*).
  // Mass-like fields scale by chi; normal momentum rho* S*, tangential
  // rho* u_t; energy chi [E + (S* - u)(rho S* + P/(S - u))]; P = -sigma_dd.
  // Reading (the multi-material star state is deferred to other work):
  // phi* = chi phi, which makes the phi flux equal to phi times the wall
  // velocity u* (the same formula applied to the unit field), and Vbar* =
  // D Vbar with D scaling the normal row by chi^(-2/3) and the tangential rows
  // by chi^(1/3) (a uniaxial compression by chi that keeps det Vbar).
  void star_state(const double* W, const double* Uc, const CellThermo& th, int d, double S,
                  double Sstar, double* Us, double& chi_out) const {
    const double ud = W[L.wU(d)];
    const double chi = (S - ud) / (S - Sstar);
    chi_out = chi;
    const double P = -th.sigma[d][d];
    double rhos = 0;
    for (int l = 0; l < nmat; ++l) { Us[L.A(l)] = chi * Uc[L.A(l)]; rhos += Us[L.A(l)]; }
    for (int a = 0; a < dim; ++a) Us[L.M(a)] = (a == d) ? rhos * Sstar : rhos * W[L.wU(a)];
    Us[L.E()] = chi * (Uc[L.E()] + (Sstar - ud) * (th.rho * Sstar + P / (S - ud)));
    for (int l = 0; l < nmat - 1; ++l) Us[L.PHI(l)] = chi * Uc[L.PHI(l)];
    if (L.solid) {
      const double cn = std::pow(chi, -2.0 / 3.0), ct = std::cbrt(chi);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Us[L.V(a, b)] = (a == d ? cn : ct) * Uc[L.V(a, b)];
      Us[L.EP()] = chi * Uc[L.EP()];
    }
  }

  // HLLC flux (Toro) with Davis wave-speed estimates, optionally in the
  // low-Mach form HLLC-LM. Returns the flux of the thermodynamic fields, the
  // wall velocity u* (the same flux formula applied to the unit field, whose
  // star value is chi) and the wall stretch row Vbar*_{d,:} (the Godunov state
  // at x/t = 0 of the HLLC fan).
  // Reading (wave speeds and the LM constants are not printed): Davis
  // S_L = min(uL - cL, uR - cR), S_R = max(uL + cL, uR + cR); HLLC-LM uses
  // the central form with the acoustic terms scaled by
  // phi = sin(min(1, Ma/0.1) pi/2), Ma = max(|uL|/cL, |uR|/cR) (normal
  // velocity components).
  void hllc(const double* WL, const double* WR, int d, double* Fo, double& ustar,
            double Vstar[3], double* pstar = nullptr) const {
    const int nt = L.n - 1;  // thermodynamic fields (r excluded)
    double UL[kMaxF], UR[kMaxF], FL[kMaxF], FR[kMaxF], UsL[kMaxF], UsR[kMaxF];
    prim_to_cons(WL, UL);
    prim_to_cons(WR, UR);
    CellThermo tl, tr;
    thermo_from_prim(WL, tl);
    thermo_from_prim(WR, tr);
    phys_flux(WL, UL, tl, d, FL);
    phys_flux(WR, UR, tr, d, FR);
    const double uL = WL[L.wU(d)], uR = WR[L.wU(d)];
    const double cL = std::sqrt(tl.c2), cR = std::sqrt(tr.c2);
    const double PL = -tl.sigma[d][d], PR = -tr.sigma[d][d];
    const double SL = std::min(uL - cL, uR - cR);
    const double SR = std::max(uL + cL, uR + cR);
    const double Ss = (PR - PL + tl.rho * uL * (SL - uL) - tr.rho * uR * (SR - uR)) /
                      (tl.rho * (SL - uL) - tr.rho * (SR - uR));
    // normal traction (compression positive) on the contact of the fan
    if (pstar) *pstar = PL + tl.rho * (SL - uL) * (Ss - uL);
    double chiL, chiR;
    star_state(WL, UL, tl, d, SL, Ss, UsL, chiL);
    star_state(WR, UR, tr, d, SR, Ss, UsR, chiR);
    double VL[3], VR[3], VsL[3], VsR[3];
    for (int b = 0; b < 3; ++b) {
      VL[b] = L.solid ? UL[L.V(d, b)] : 0.0;
      VR[b] = L.solid ? UR[L.V(d, b)] : 0.0;
      VsL[b] = L.solid ? UsL[L.V(d, b)] : 0.0;
      VsR[b] = L.solid ? UsR[L.V(d, b)] : 0.0;
    }
    // Wall value of the stretch row: its state at x/t = 0 of the HLLC fan
    // outside the star region; inside it, the star states weighted by the
    // position of the contact in the fan, w = (S* - S_L)/(S_R - S_L), which
    // is continuous in S* (the two star states differ across the contact).
    for (int b = 0; b < 3; ++b) {
      if (SL >= 0.0) Vstar[b] = VL[b];
      else if (SR <= 0.0) Vstar[b] = VR[b];
      else Vstar[b] = VsR[b] + (Ss - SL) / (SR - SL) * (VsL[b] - VsR[b]);
    }
    // Reading (the paper's solid solver is HLLD, not given here): for the
    // elastoplastic system the star states carry only the normal traction, so
    // the Rankine-Hugoniot condition across the contact fails for the
    // tangential traction and its work; the star-region flux is then taken
    // in the central form (1/2)(F*_L + F*_R) + (1/2)|S*|(U*_L - U*_R), which
    // equals Toro's flux where that condition holds and has no jump at S* = 0.
    if (riemann == RS_HLLC_LM || L.solid) {
      if (SL >= 0.0) { for (int q = 0; q < nt; ++q) Fo[q] = FL[q]; ustar = uL; return; }
      if (SR <= 0.0) { for (int q = 0; q < nt; ++q) Fo[q] = FR[q]; ustar = uR; return; }
      double ph = 1.0;
      if (riemann == RS_HLLC_LM) {
        const double Ma = std::max(std::fabs(uL) / cL, std::fabs(uR) / cR);
        ph = std::sin(std::min(1.0, Ma / lm_mach) * M_PI * 0.5);
      }
      const double aS = std::fabs(Ss);
      for (int q = 0; q < nt; ++q)
        Fo[q] = 0.5 * (FL[q] + FR[q]) +
                0.5 * (ph * SL * (UsL[q] - UL[q]) + aS * (UsL[q] - UsR[q]) + ph * SR * (UsR[q] - UR[q]));
      ustar = 0.5 * (uL + uR) +
              0.5 * (ph * SL * (chiL - 1.0) + aS * (chiL - chiR) + ph * SR * (chiR - 1.0));
      return;
    }
    if (SL >= 0.0) {
      for (int q = 0; q < nt; ++q) Fo[q] = FL[q];
      ustar = uL;
    } else if (Ss >= 0.0) {
      for (int q = 0; q < nt; ++q) Fo[q] = FL[q] + SL * (UsL[q] - UL[q]);
      ustar = uL + SL * (chiL - 1.0);
    } else if (SR > 0.0) {
      for (int q = 0; q < nt; ++q) Fo[q] = FR[q] + SR * (UsR[q] - UR[q]);
      ustar = uR + SR * (chiR - 1.0);
    } else {
      for (int q = 0; q < nt; ++q) Fo[q] = FR[q];
      ustar = uR;
    }
  }

  // Void-opening face modifier (Sec. 3.2, end): applied at a face whose two
  // cells lie on either side of the rigid surface, (0.5 - r_L)(0.5 - r_R) < 0,
  // read as "one cell rigid (r > 0.5), the other not": a cell with r exactly
  // 0.5 is a material cell, as in the rest of the method (with the strict
  // product it would shield the wall from the modifier).
  // Reading (the modifier is defined in other work): the face sees the
  // material cell's face state against its mirror image about the face
  // (normal velocity reflected about the rigid velocity, Vbar conjugated by
  // the reflection), i.e. an exact wall; where the normal traction on that
  // wall's contact is tensile the solid is let go: the rigid side is replaced
  // by the gap gas (gap_W, moving with the body's normal velocity, at rest
  // tangentially), which then flows into the opening gap. real: the material
  // side's face state; real_left: it lies left of the face.
  void wall_face(const double* real, bool real_left, int d, const double v[3], double* Fo, double& ust,
                 double vst[3]) const {
    double nrm[3] = {0, 0, 0}, m[kMaxF];
    nrm[d] = 1.0;
    mirror_state(real, nrm, v, m);
    double ps;
    if (real_left) hllc(real, m, d, Fo, ust, vst, &ps);
    else hllc(m, real, d, Fo, ust, vst, &ps);
    if (!(ps < 0.0)) return;
    double gW[kMaxF];
    for (int q = 0; q < L.n; ++q) gW[q] = gap_W[q];
    for (int a = 0; a < dim; ++a) gW[L.wU(a)] = (a == d) ? v[d] : 0.0;
    gW[L.wR()] = m[L.wR()];
    if (real_left) hllc(real, gW, d, Fo, ust, vst);
    else hllc(gW, real, d, Fo, ust, vst);
  }

  // ---- semi-discrete operator (Sec. 3.1, spatial operator D_ijk) ----------
  // D = sum_d (F_{+1/2} - F_{-1/2}) / dx_d - s_non-con, fluxes from
  // successive sweeps of each direction, summed (spatially unsplit).
  // Non-conservative terms (Sec. 3.1): for r, r_i (v_{+} - v_{-}); for phi,
  // phi_i (u*_{+} - u*_{-}); for Vbar_ab, (2/3) Vbar_ab (u*_{+} - u*_{-})
  // - u_a (Vbar*_{db,+} - Vbar*_{db,-}); all over dx_d.
  // Fluxes of r: upwind on the sign of the rigid velocity at the face, with
  // the reconstructed face values of r (Sec. 3.1).
  // Cells with r > 0.5 at the start of the step keep their thermodynamic
  // state (Sec. 3.1: not updated in rigid cells); only r is updated there.
  int dirmask = 7;  // diagnostics: directions included in D
  void rhs(const std::vector<double>& Uin, const std::vector<unsigned char>& rigid,
           std::vector<double>& D) {
    std::vector<double> X = Uin;
    fill_ghosts(X);
    std::vector<double> Wf;
    prim_all(X, Wf);
    D.assign((size_t)L.n * ncell, 0.0);
    const int nv = L.n;
    long nfb = 0;
    for (int d = 0; d < dim; ++d) {
      if (!((dirmask >> d) & 1)) continue;
      const size_t st = stride(d);
      // pencils along d: iterate over the interior of the other dimensions
      int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
      for (int e = 0; e < dim; ++e) { lo[e] = 0; hi[e] = n[e]; }
      hi[d] = 1;
      std::vector<std::array<int, 3>> pencils;
      for (int k = lo[2]; k < hi[2]; ++k)
        for (int j = lo[1]; j < hi[1]; ++j)
          for (int i = lo[0]; i < hi[0]; ++i) pencils.push_back({i, j, k});
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : nfb)
      for (long pi = 0; pi < (long)pencils.size(); ++pi) {
        const int nd = n[d];
        const int np = nd + 4;  // cells -2 .. nd+1 need candidates
        std::vector<double> cand((size_t)np * nv * 4);
        std::vector<double> selL((size_t)(nd + 2) * nv), selR((size_t)(nd + 2) * nv);
        int p0[3] = {pencils[pi][0], pencils[pi][1], pencils[pi][2]};
        p0[d] = 0;
        const size_t base = idx(p0[0], p0[1], p0[2]);
        auto Wat = [&](int q, int i) { return Wf[(size_t)q * ncell + base + (long)i * (long)st]; };
        for (int i = -2; i <= nd + 1; ++i)
          for (int q = 0; q < nv; ++q)
            candidates(Wat(q, i - 1), Wat(q, i), Wat(q, i + 1), &cand[((size_t)(i + 2) * nv + q) * 4]);
        for (int i = -1; i <= nd; ++i) {
          double wl[kMaxF], wr[kMaxF];
          for (int q = 0; q < nv; ++q)
            bvd_select(&cand[((size_t)(i + 1) * nv + q) * 4], &cand[((size_t)(i + 2) * nv + q) * 4],
                       &cand[((size_t)(i + 3) * nv + q) * 4], wl[q], wr[q]);
          // Reading (no positivity treatment is given): a cell whose selected
          // faces are inadmissible falls back to first order.
          if (!admissible(wl) || !admissible(wr)) {
            for (int q = 0; q < nv; ++q) { wl[q] = Wat(q, i); wr[q] = wl[q]; }
            if (i >= 0 && i < nd) ++nfb;
          }
          for (int q = 0; q < nv; ++q) {
            selL[(size_t)(i + 1) * nv + q] = wl[q];
            selR[(size_t)(i + 1) * nv + q] = wr[q];
          }
        }
        // faces i+1/2 for i = -1 .. nd-1
        const int nt = nv - 1;
        std::vector<double> Ff((size_t)(nd + 1) * nt), us(nd + 1), vface(nd + 1), rfl(nd + 1),
            Vs((size_t)(nd + 1) * 3);
        for (int i = -1; i <= nd - 1; ++i) {
          const double* wl = &selR[(size_t)(i + 1) * nv];  // right face of cell i
          const double* wr = &selL[(size_t)(i + 2) * nv];  // left face of cell i+1
          double xf[3];
          for (int e = 0; e < 3; ++e) xf[e] = (e < dim) ? xc(e, p0[e]) : 0.0;
          xf[d] = x0[d] + (i + 1) * dx[d];
          double v[3];
          rigid_velocity(xf, v);
          double Fo[kMaxF], ust, vst[3];
          const double rci = Wat(L.wR(), i), rcj = Wat(L.wR(), i + 1);
          if (face_mod && ((rci > 0.5) != (rcj > 0.5)))
            wall_face(rci > 0.5 ? wr : wl, !(rci > 0.5), d, v, Fo, ust, vst);
          else
            hllc(wl, wr, d, Fo, ust, vst);
          for (int q = 0; q < nt; ++q) Ff[(size_t)(i + 1) * nt + q] = Fo[q];
          us[i + 1] = ust;
          for (int b = 0; b < 3; ++b) Vs[(size_t)(i + 1) * 3 + b] = vst[b];
          const double vd = v[d];
          vface[i + 1] = vd;
          const double rL = wl[L.wR()], rR = wr[L.wR()];
          rfl[i + 1] = vd > 0.0 ? rL * vd : (vd < 0.0 ? rR * vd : 0.0);
        }
        for (int i = 0; i < nd; ++i) {
          const size_t c = base + (size_t)i * st;
          const double inv = 1.0 / dx[d];
          // r: conservative upwind flux minus r_i (v_+ - v_-)
          D[(size_t)L.R() * ncell + c] +=
              ((rfl[i + 1] - rfl[i]) - Wat(L.wR(), i) * (vface[i + 1] - vface[i])) * inv;
          if (rigid[c]) continue;
          for (int q = 0; q < nt; ++q)
            D[(size_t)q * ncell + c] += (Ff[(size_t)(i + 1) * nt + q] - Ff[(size_t)i * nt + q]) * inv;
          const double du = us[i + 1] - us[i];
          for (int l = 0; l < nmat - 1; ++l)
            D[(size_t)L.PHI(l) * ncell + c] -= Wat(L.wPHI(l), i) * du * inv;
          if (L.solid) {
            for (int a = 0; a < 3; ++a) {
              const double ua = a < dim ? Wat(L.wU(a), i) : 0.0;
              for (int b = 0; b < 3; ++b) {
                const double dV = Vs[(size_t)(i + 1) * 3 + b] - Vs[(size_t)i * 3 + b];
                D[(size_t)L.V(a, b) * ncell + c] -=
                    ((2.0 / 3.0) * Wat(L.wV(a, b), i) * du - ua * dV) * inv;
              }
            }
          }
        }
      }
    }
    fallback += nfb;
  }

  // ---- per-stage source updates for the elastoplastic system --------------
  // Reading (the plastic update is deferred to other work): after each stage
  // Vbar is renormalised to unit determinant, then perfect plasticity is
  // applied as a radial return in Hencky space: with sigma_eq = sqrt(6) G |H|
  // above the (Gamma-weighted) mixture yield stress, H is scaled by
  // s = sigma_Y / sigma_eq through Vbar <- exp((s-1) H) Vbar, and the
  // equivalent plastic strain grows by sqrt(2/3)(1-s)|H| (Sec. 2.1.1, plastic
  // source; Sec. 4.5 and 4.6, ideal plasticity). rho E is unchanged.
  void solid_sources(double* Uc) const {
    double V[3][3];
    stretch_from(Uc, L.V(0, 0), V);
    const double det = det3(V);
    const double sc = 1.0 / std::cbrt(det);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) V[a][b] *= sc;
    if (plastic) {
      double W[kMaxF];
      for (int q = 0; q < 9; ++q) Uc[L.V(0, 0) + q] = V[q / 3][q % 3];
      cons_to_prim(Uc, W);
      CellThermo th;
      thermo_from_prim(W, th);
      const double Hn = std::sqrt(th.J2);
      const double seq = std::sqrt(6.0) * th.G * Hn;
      if (th.sigY > 0.0 && seq > th.sigY) {
        const double s = th.sigY / seq;
        double S[3][3], X[3][3], Vn[3][3];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) S[a][b] = (s - 1.0) * th.H[a][b];
        sym_exp(S, X);
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += X[a][k] * V[k][b];
            Vn[a][b] = acc;
          }
        std::memcpy(V, Vn, sizeof(V));
        double phi[kMaxMat], rho[kMaxMat];
        phases_from_prim(W, phi, rho);
        const double as = phi[solid_phase] * rho[solid_phase];
        Uc[L.EP()] += as * std::sqrt(2.0 / 3.0) * (1.0 - s) * Hn;
      }
    }
    for (int q = 0; q < 9; ++q) Uc[L.V(0, 0) + q] = V[q / 3][q % 3];
  }

  // ---- ELVIRA normal (Sec. 3.3; Pilliod and Puckett's second-order method) --

  // Fraction of the cell [-hx/2,hx/2] x [-hy/2,hy/2] on the side n.p <= beta
  // of a straight line: the cell rectangle is clipped by the half-plane and
  // the area of the clipped polygon is taken by the shoelace formula.
  static double cut_fraction(const double nv[2], double hx, double hy, double beta) {
    const double px[4] = {-0.5 * hx, 0.5 * hx, 0.5 * hx, -0.5 * hx};
    const double py[4] = {-0.5 * hy, -0.5 * hy, 0.5 * hy, 0.5 * hy};
    double qx[8], qy[8];
    int m = 0;
    for (int e = 0; e < 4; ++e) {
      const int f = (e + 1) % 4;
      const double se = nv[0] * px[e] + nv[1] * py[e] - beta;
      const double sf = nv[0] * px[f] + nv[1] * py[f] - beta;
      if (se <= 0.0) { qx[m] = px[e]; qy[m] = py[e]; ++m; }
      if ((se < 0.0 && sf > 0.0) || (se > 0.0 && sf < 0.0)) {
        const double t = se / (se - sf);
        qx[m] = px[e] + t * (px[f] - px[e]);
        qy[m] = py[e] + t * (py[f] - py[e]);
        ++m;
      }
    }
    double a2 = 0.0;
    for (int e = 0; e < m; ++e) {
      const int f = (e + 1) % m;
      a2 += qx[e] * qy[f] - qx[f] * qy[e];
    }
    return 0.5 * std::fabs(a2) / (hx * hy);
  }

  // The line offset beta whose cut fraction is frac (0 < frac < 1), by
  // bisection on the nondecreasing cut_fraction.
  static double cut_offset(const double nv[2], double hx, double hy, double frac) {
    double hi = 0.5 * (std::fabs(nv[0]) * hx + std::fabs(nv[1]) * hy), lo = -hi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (!(mid > lo && mid < hi)) break;
      if (cut_fraction(nv, hx, hy, mid) < frac) lo = mid;
      else hi = mid;
    }
    return 0.5 * (lo + hi);
  }

  // ELVIRA on the 3x3 block f[a+1][b+1] = r(i+a, j+b) of a rigid cell.
  // Candidate lines: the interface as a graph over x, with slopes from the
  // backward, central and forward differences of the column sums, and as a
  // graph over y from the row sums. Readings: the body lies on the side of
  // each family given by the sign of the opposite block sums (the bottom vs
  // top rows for graphs over x, the left vs right columns for graphs over
  // y); a family whose sign is zero is left out. Each candidate line is
  // placed so that it cuts the centre cell at its own fraction, and the one
  // whose fractions in the nine cells differ least from f in the sum of
  // squares wins (first in the order above on ties). The outward normal
  // points away from the body. Returns false when f(centre) is not strictly
  // between 0 and 1 or no family is defined.
  static bool elvira_normal(const double f[3][3], double hx, double hy, double nout[2]) {
    const double fc = f[1][1];
    if (!(fc > 0.0 && fc < 1.0)) return false;
    double H[3], Wr[3];
    for (int a = 0; a < 3; ++a) H[a] = hy * (f[a][0] + f[a][1] + f[a][2]);
    for (int b = 0; b < 3; ++b) Wr[b] = hx * (f[0][b] + f[1][b] + f[2][b]);
    const double sy = Wr[2] > Wr[0] ? 1.0 : (Wr[2] < Wr[0] ? -1.0 : 0.0);
    const double sx = H[2] > H[0] ? 1.0 : (H[2] < H[0] ? -1.0 : 0.0);
    double cand[6][2];
    int nc = 0;
    if (sy != 0.0) {
      const double sl[3] = {(H[1] - H[0]) / hx, (H[2] - H[0]) / (2.0 * hx), (H[2] - H[1]) / hx};
      for (int c = 0; c < 3; ++c) { cand[nc][0] = -sl[c]; cand[nc][1] = -sy; ++nc; }
    }
    if (sx != 0.0) {
      const double sl[3] = {(Wr[1] - Wr[0]) / hy, (Wr[2] - Wr[0]) / (2.0 * hy), (Wr[2] - Wr[1]) / hy};
      for (int c = 0; c < 3; ++c) { cand[nc][0] = -sx; cand[nc][1] = -sl[c]; ++nc; }
    }
    if (nc == 0) return false;
    double best = 0.0;
    int ib = -1;
    for (int c = 0; c < nc; ++c) {
      const double mag = std::sqrt(cand[c][0] * cand[c][0] + cand[c][1] * cand[c][1]);
      const double nv[2] = {cand[c][0] / mag, cand[c][1] / mag};
      const double beta = cut_offset(nv, hx, hy, fc);
      double err = 0.0;
      for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b) {
          const double e = cut_fraction(nv, hx, hy, beta - nv[0] * a * hx - nv[1] * b * hy) - f[a + 1][b + 1];
          err += e * e;
        }
      if (ib < 0 || err < best) { best = err; ib = c; nout[0] = nv[0]; nout[1] = nv[1]; }
    }
    return true;
  }

  // ---- rigid-body interface seeding (Sec. 3.2, the seeding routine) --------

  // Normal of the rigid cell (i,j,k) (Sec. 3.3): ELVIRA in 2D when selected
  // and defined (a fraction strictly between 0 and 1 and at least one
  // candidate family), otherwise Youngs. Ghost values come from the filled
  // ghost layers (corners included).
  bool normal_at(const std::vector<double>& X, int i, int j, int k, double nrm[3]) const {
    const double* r = X.data() + (size_t)L.R() * ncell;
    if (normal == NORMAL_ELVIRA && dim == 2) {
      double f[3][3], n2[2];
      for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b) f[a + 1][b + 1] = r[idx(i + a, j + b, k)];
      if (elvira_normal(f, dx[0], dx[1], n2)) {
        nrm[0] = n2[0]; nrm[1] = n2[1]; nrm[2] = 0.0;
        return true;
      }
    }
    return youngs_at(X, i, j, k, nrm);
  }

  // Youngs normal (Sec. 3.3): n = -grad r / |grad r| with central
  // differences. Returns false where the gradient vanishes.
  bool youngs_at(const std::vector<double>& X, int i, int j, int k, double nrm[3]) const {
    const double* r = X.data() + (size_t)L.R() * ncell;
    const size_t c = idx(i, j, k);
    double gr[3] = {0, 0, 0}, mag = 0;
    for (int d = 0; d < dim; ++d) {
      gr[d] = (r[c + stride(d)] - r[c - stride(d)]) / (2.0 * dx[d]);
      mag += gr[d] * gr[d];
    }
    mag = std::sqrt(mag);
    double dmin = dx[0];
    for (int d = 1; d < dim; ++d) dmin = std::min(dmin, dx[d]);
    if (!(mag * dmin > 1e-12)) return false;
    for (int d = 0; d < 3; ++d) nrm[d] = d < dim ? -gr[d] / mag : 0.0;
    return true;
  }

  // Mirror state (seeding steps 3-4): in the frame whose x axis is n, the
  // normal velocity is reflected and the rigid normal velocity added twice;
  // the shear components Vbar_{xy}, Vbar_{xz}, Vbar_{yx}, Vbar_{zx} are
  // reflected; scalars are unchanged. The rotation R of the paper is not
  // needed: rotate-reflect-rotate back equals the Householder reflection
  // P = I - 2 n n^T for any R with R n = x: u' = P u + 2 (v_r . n) n and
  // Vbar' = P Vbar P.
  void mirror_state(const double* Win, const double nrm[3], const double v[3], double* Wout) const {
    for (int q = 0; q < L.n; ++q) Wout[q] = Win[q];
    double u[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) u[a] = Win[L.wU(a)];
    double un = 0, vn = 0;
    for (int a = 0; a < 3; ++a) { un += u[a] * nrm[a]; vn += v[a] * nrm[a]; }
    for (int a = 0; a < dim; ++a) Wout[L.wU(a)] = u[a] - 2.0 * un * nrm[a] + 2.0 * vn * nrm[a];
    if (L.solid) {
      double P[3][3], V[3][3], T[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) P[a][b] = (a == b ? 1.0 : 0.0) - 2.0 * nrm[a] * nrm[b];
      stretch_from(Win, L.wV(0, 0), V);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double s = 0;
          for (int k = 0; k < 3; ++k) s += P[a][k] * V[k][b];
          T[a][b] = s;
        }
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double s = 0;
          for (int k = 0; k < 3; ++k) s += T[a][k] * P[k][b];
          Wout[L.wV(a, b)] = s;
        }
    }
  }

  // Riemann-problem based seeding (step 5, second option): the HLLC star state
  // on the right of the problem (left = mirror state, right = interpolated
  // state) along n. Reading: the star state is taken in primitive form,
  // phasic densities times chi_R, normal velocity S*, tangential velocity,
  // volume fractions and plastic strain from the right state, pressure
  // p* = p_R + rho_R (S_R - u_R)(S* - u_R), and Vbar* = D Vbar_R with the
  // uniaxial stretch D along n used by the flux.
  void riemann_star_right(const double* Wm, const double* Wi, const double nrm[3], double* Wout) const {
    CellThermo tl, tr;
    thermo_from_prim(Wm, tl);
    thermo_from_prim(Wi, tr);
    double uL = 0, uR = 0;
    for (int a = 0; a < dim; ++a) { uL += Wm[L.wU(a)] * nrm[a]; uR += Wi[L.wU(a)] * nrm[a]; }
    double PL = 0, PR = 0;  // normal traction -n.sigma.n
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) { PL -= nrm[a] * tl.sigma[a][b] * nrm[b]; PR -= nrm[a] * tr.sigma[a][b] * nrm[b]; }
    const double cL = std::sqrt(tl.c2), cR = std::sqrt(tr.c2);
    const double SL = std::min(uL - cL, uR - cR);
    const double SR = std::max(uL + cL, uR + cR);
    const double Ss = (PR - PL + tl.rho * uL * (SL - uL) - tr.rho * uR * (SR - uR)) /
                      (tl.rho * (SL - uL) - tr.rho * (SR - uR));
    const double chi = (SR - uR) / (SR - Ss);
    for (int q = 0; q < L.n; ++q) Wout[q] = Wi[q];
    for (int l = 0; l < nmat; ++l) Wout[L.wRHO(l)] = Wi[L.wRHO(l)] * chi;
    for (int a = 0; a < dim; ++a) Wout[L.wU(a)] = Wi[L.wU(a)] + (Ss - uR) * nrm[a];
    Wout[L.wP()] = Wi[L.wP()] + tr.rho * (SR - uR) * (Ss - uR);
    if (L.solid) {
      const double cn = std::pow(chi, -2.0 / 3.0), ct = std::cbrt(chi);
      double Dm[3][3], V[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Dm[a][b] = (a == b ? ct : 0.0) + (cn - ct) * nrm[a] * nrm[b];
      stretch_from(Wi, L.wV(0, 0), V);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double s = 0;
          for (int k = 0; k < 3; ++k) s += Dm[a][k] * V[k][b];
          Wout[L.wV(a, b)] = s;
        }
    }
  }

  // Seeding (Sec. 3.2), once per time step before the hyperbolic update, on
  // every rigid cell (r > 0.5):
  //  1. outward normal n (Youngs, or ELVIRA in 2D);
  //  2. probe along n. Reading: step-out distances 1, 1.5, ..., 4 dx (or the
  //     fixed 1.5 dx probe); a probe point is valid when every enclosing cell
  //     centre that carries a nonzero interpolation weight is an interior cell
  //     with r <= 0.5; the first valid point is used; primitive variables are
  //     interpolated multilinearly; no valid point -> no action. A point in
  //     the half cell between the outermost cell centres and a domain face
  //     takes, along that axis, the outermost centre's coordinate (the
  //     boundary cell's state extends to the face): without it a probe that
  //     runs along a wall through the first row of centres would flip
  //     between valid and invalid with the sign of a rounding error;
  //  3-4. mirror state (mirror_state);
  //  5. original: the mirror state replaces the cell state; Riemann: the HLLC
  //     right star state of (mirror, interpolated) replaces it.
  // r itself is never changed by seeding. Valid support cells are never
  // rigid, so the in-place order does not matter.
  void do_seed() {
    if (seed == SEED_NONE) return;
    fill_ghosts(U);
    const double* r = f(L.R());
    double dmin = dx[0];
    for (int d = 1; d < dim; ++d) dmin = std::min(dmin, dx[d]);
    long nfail = 0, nseed = 0;
    // primitive values are read only from non-rigid interior cells, which the
    // loop never writes
    std::vector<double> Wf;
    prim_all(U, Wf);
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nfail, nseed)
    for (long lin = 0; lin < (long)nint(); ++lin) {
      const int i = (int)(lin % n[0]);
      const int j = (int)((lin / n[0]) % n[1]);
      const int k = (int)(lin / ((long)n[0] * n[1]));
      const size_t c = idx(i, j, k);
      if (!(r[c] > 0.5)) continue;
      double nrm[3];
      if (!normal_at(U, i, j, k, nrm)) continue;
      const int nprobe = probe == PROBE_FIXED ? 1 : 7;
      bool found = false;
      double Wint[kMaxF];
      for (int pI = 0; pI < nprobe && !found; ++pI) {
        const double dist = probe == PROBE_FIXED ? 1.5 : 1.0 + 0.5 * pI;
        const int pos[3] = {i, j, k};
        int lo[3] = {0, 0, 0};
        double w[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) {
          double xi = pos[a] + dist * nrm[a] * (dmin / dx[a]);
          if (xi < 0.0 && xi >= -0.5) xi = 0.0;
          if (xi > n[a] - 1 && xi <= n[a] - 0.5) xi = n[a] - 1;
          lo[a] = (int)std::floor(xi);
          w[a] = xi - lo[a];
        }
        bool ok = true;
        const int ncorner = 1 << dim;
        for (int cb = 0; cb < ncorner && ok; ++cb) {
          int cp[3] = {0, 0, 0};
          bool used = true;
          for (int a = 0; a < dim; ++a) {
            const int bit = (cb >> a) & 1;
            if (bit && w[a] == 0.0) used = false;
            cp[a] = lo[a] + bit;
          }
          if (!used) continue;
          for (int a = 0; a < dim; ++a)
            if (cp[a] < 0 || cp[a] >= n[a]) ok = false;
          if (!ok) break;
          if (!(r[idx(cp[0], cp[1], cp[2])] <= 0.5)) ok = false;
        }
        if (!ok) continue;
        // multilinear interpolation as nested linear interpolations
        for (int q = 0; q < L.n; ++q) {
          double vals[8];
          for (int cb = 0; cb < ncorner; ++cb) {
            int cp[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) {
              const int bit = (cb >> a) & 1;
              cp[a] = lo[a] + ((bit && w[a] != 0.0) ? 1 : 0);
            }
            vals[cb] = Wf[(size_t)q * ncell + idx(cp[0], cp[1], cp[2])];
          }
          int m = ncorner;
          for (int a = 0; a < dim; ++a) {
            m >>= 1;
            for (int cb = 0; cb < m; ++cb) vals[cb] = vals[2 * cb] + w[a] * (vals[2 * cb + 1] - vals[2 * cb]);
          }
          Wint[q] = vals[0];
        }
        found = true;
      }
      if (!found) { ++nfail; continue; }
      double xcell[3] = {0, 0, 0};
      const int pos[3] = {i, j, k};
      for (int a = 0; a < dim; ++a) xcell[a] = xc(a, pos[a]);
      double v[3];
      rigid_velocity(xcell, v);
      double Wm[kMaxF], Wg[kMaxF], Ug[kMaxF];
      mirror_state(Wint, nrm, v, Wm);
      if (seed == SEED_RIEMANN) riemann_star_right(Wm, Wint, nrm, Wg);
      else for (int q = 0; q < L.n; ++q) Wg[q] = Wm[q];
      Wg[L.wR()] = r[c];
      prim_to_cons(Wg, Ug);
      for (int q = 0; q < L.n - 1; ++q) U[(size_t)q * ncell + c] = Ug[q];
      ++nseed;
    }
    probe_fail += nfail;
    seeded += nseed;
  }

  // ---- one time step (Sec. 3.1 SSP-RK3 and Sec. 3.2 seeding) -------------
  void step(double dt) {
    do_seed();
    const size_t nc = ncell;
    std::vector<unsigned char> rigid(nc, 0);
    {
      const double* r = f(L.R());
      for (long lin = 0; lin < (long)nint(); ++lin) {
        const int i = (int)(lin % n[0]);
        const int j = (int)((lin / n[0]) % n[1]);
        const int k = (int)(lin / ((long)n[0] * n[1]));
        const size_t c = idx(i, j, k);
        rigid[c] = r[c] > 0.5;
      }
    }
    const std::vector<double> U0 = U;
    std::vector<double> Uk = U, D;
    // U(1) = U^n - dt D(U^n); U(2) = U(1) - dt D(U(1)); U(3) = 3/4 U^n + 1/4 U(2);
    // U(4) = U(3) - dt D(U(3)); U^{n+1} = 1/3 U^n + 2/3 U(4).
    // The convex combinations a U^n + b U(k) (a + b = 1) are evaluated as
    // U^n + b (U(k) - U^n), which returns U^n exactly when U(k) = U^n.
    const double a_k[3] = {1.0, 0.25, 2.0 / 3.0};
    for (int s = 0; s < 3; ++s) {
      rhs(Uk, rigid, D);
      std::vector<double> Un(U.size(), 0.0);
#pragma omp parallel for schedule(static)
      for (long lin = 0; lin < (long)nint(); ++lin) {
        const int i = (int)(lin % n[0]);
        const int j = (int)((lin / n[0]) % n[1]);
        const int k = (int)(lin / ((long)n[0] * n[1]));
        const size_t c = idx(i, j, k);
        double Uc[kMaxF];
        for (int q = 0; q < L.n; ++q) {
          const size_t o = (size_t)q * nc + c;
          const double ustage = Uk[o] - dt * D[o];
          Uc[q] = s == 0 ? ustage : U0[o] + a_k[s] * (ustage - U0[o]);
          if (rigid[c] && q != L.R()) Uc[q] = U0[o];
        }
        if (L.solid && !rigid[c]) solid_sources(Uc);
        for (int q = 0; q < L.n; ++q) Un[(size_t)q * nc + c] = Uc[q];
      }
      Uk.swap(Un);
    }
    U.swap(Uk);
    t += dt;
  }

  // ---- CFL time step (Sec. 3: a fraction of the global maximum allowable
  // step). Reading: dt = CFL min over non-rigid cells and directions of
  // dx_d / max(|u_d| + c, |v_r,d|).
  double compute_dt(double cfl) {
    double m = 1e300;
    const double* r = f(L.R());
#pragma omp parallel for reduction(min : m)
    for (long lin = 0; lin < (long)nint(); ++lin) {
      const int i = (int)(lin % n[0]);
      const int j = (int)((lin / n[0]) % n[1]);
      const int k = (int)(lin / ((long)n[0] * n[1]));
      const size_t c = idx(i, j, k);
      if (r[c] > 0.5) continue;
      double Uc[kMaxF], W[kMaxF];
      for (int q = 0; q < L.n; ++q) Uc[q] = U[(size_t)q * ncell + c];
      cons_to_prim(Uc, W);
      CellThermo th;
      thermo_from_prim(W, th);
      const double cs = std::sqrt(th.c2);
      double xcell[3] = {0, 0, 0};
      const int pos[3] = {i, j, k};
      for (int a = 0; a < dim; ++a) xcell[a] = xc(a, pos[a]);
      double v[3];
      rigid_velocity(xcell, v);
      for (int d = 0; d < dim; ++d) {
        const double s = std::max(std::fabs(W[L.wU(d)]) + cs, std::fabs(v[d]));
        m = std::min(m, dx[d] / s);
      }
    }
    return cfl * m;
  }
};

// Pairwise (cascade) summation of a sequence, FP64.
double pairwise_sum(const double* a, size_t n) {
  if (n <= 8) {
    double s = 0;
    for (size_t i = 0; i < n; ++i) s += a[i];
    return s;
  }
  const size_t h = n / 2;
  return pairwise_sum(a, h) + pairwise_sum(a + h, n - h);
}

thread_local std::string g_err;

}  // namespace

// ===========================================================================
// C interface (ctypes)
// ===========================================================================

struct orc_desc {
  int dim, nx, ny, nz;
  double dx[3], origin[3];
  int nmat, solid;
  int bc[6];
  int recon, riemann, seed, probe, plastic;
  double thinc_beta, lm_mach;
  int normal;
};

ORC_API const char* orc_last_error() { return g_err.c_str(); }

// Number of OpenMP threads of the oracle's loops (timing of the baseline).
ORC_API void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
ORC_API int orc_get_threads() { return omp_get_max_threads(); }

ORC_API void* orc_create(const orc_desc* d) {
  if (!d || d->dim < 1 || d->dim > 3 || d->nmat < 1 || d->nmat > kMaxMat) { g_err = "bad desc"; return nullptr; }
  Oracle* o = new Oracle();
  o->dim = d->dim;
  o->n[0] = d->nx; o->n[1] = d->dim > 1 ? d->ny : 1; o->n[2] = d->dim > 2 ? d->nz : 1;
  for (int a = 0; a < 3; ++a) {
    o->dx[a] = d->dx[a];
    o->x0[a] = d->origin[a];
    o->g[a] = a < d->dim ? o->ng : 0;
    o->N[a] = o->n[a] + 2 * o->g[a];
  }
  o->nmat = d->nmat;
  o->L.init(d->dim, d->nmat, d->solid);
  for (int q = 0; q < 6; ++q) { o->bc[q] = d->bc[q]; o->bcU[q].assign(o->L.n, 0.0); }
  o->recon = d->recon; o->riemann = d->riemann; o->seed = d->seed; o->probe = d->probe;
  o->plastic = d->plastic;
  o->beta_thinc = d->thinc_beta; o->lm_mach = d->lm_mach;
  o->normal = d->normal;
  o->ncell = (size_t)o->N[0] * o->N[1] * o->N[2];
  o->U.assign((size_t)o->L.n * o->ncell, 0.0);
  return o;
}

ORC_API void orc_destroy(void* h) { delete static_cast<Oracle*>(h); }

ORC_API int orc_nfields(void* h) { return static_cast<Oracle*>(h)->L.n; }

ORC_API int orc_set_material(void* h, int l, int kind, const double* p) {
  Oracle* o = static_cast<Oracle*>(h);
  if (l < 0 || l >= o->nmat) return -1;
  Material m;
  m.kind = kind;
  if (kind == EOS_IDEAL) { m.gamma = p[0]; }
  else if (kind == EOS_STIFFENED) { m.gamma = p[0]; m.pinf = p[1]; }
  else { m.rho0 = p[0]; m.K0 = p[1]; m.G0 = p[2]; m.alpha = p[3]; m.beta = p[4]; m.Gamma0 = p[5]; m.sigY = p[6]; }
  o->mat[l] = m;
  if (kind == EOS_ROMENSKII && o->solid_phase < 0) o->solid_phase = l;
  return 0;
}

ORC_API int orc_set_bc_state(void* h, int face, const double* W) {
  Oracle* o = static_cast<Oracle*>(h);
  double Uc[kMaxF];
  o->prim_to_cons(W, Uc);
  for (int q = 0; q < o->L.n; ++q) o->bcU[face][q] = Uc[q];
  return 0;
}

// W: [nfields][nz][ny][nx] interior primitives.
ORC_API int orc_set_state_prim(void* h, const double* W) {
  Oracle* o = static_cast<Oracle*>(h);
  const size_t ni = (size_t)o->nint();
  for (size_t lin = 0; lin < ni; ++lin) {
    const int i = (int)(lin % o->n[0]);
    const int j = (int)((lin / o->n[0]) % o->n[1]);
    const int k = (int)(lin / ((size_t)o->n[0] * o->n[1]));
    double Wc[kMaxF], Uc[kMaxF];
    for (int q = 0; q < o->L.n; ++q) Wc[q] = W[(size_t)q * ni + lin];
    o->prim_to_cons(Wc, Uc);
    const size_t c = o->idx(i, j, k);
    for (int q = 0; q < o->L.n; ++q) o->U[(size_t)q * o->ncell + c] = Uc[q];
  }
  return 0;
}

ORC_API int orc_get_state_prim(void* h, double* W) {
  Oracle* o = static_cast<Oracle*>(h);
  const size_t ni = (size_t)o->nint();
  for (size_t lin = 0; lin < ni; ++lin) {
    const int i = (int)(lin % o->n[0]);
    const int j = (int)((lin / o->n[0]) % o->n[1]);
    const int k = (int)(lin / ((size_t)o->n[0] * o->n[1]));
    double Wc[kMaxF], Uc[kMaxF];
    const size_t c = o->idx(i, j, k);
    for (int q = 0; q < o->L.n; ++q) Uc[q] = o->U[(size_t)q * o->ncell + c];
    o->cons_to_prim(Uc, Wc);
    for (int q = 0; q < o->L.n; ++q) W[(size_t)q * ni + lin] = Wc[q];
  }
  return 0;
}

ORC_API int orc_get_state_cons(void* h, double* Uo) {
  Oracle* o = static_cast<Oracle*>(h);
  const size_t ni = (size_t)o->nint();
  for (size_t lin = 0; lin < ni; ++lin) {
    const int i = (int)(lin % o->n[0]);
    const int j = (int)((lin / o->n[0]) % o->n[1]);
    const int k = (int)(lin / ((size_t)o->n[0] * o->n[1]));
    const size_t c = o->idx(i, j, k);
    for (int q = 0; q < o->L.n; ++q) Uo[(size_t)q * ni + lin] = o->U[(size_t)q * o->ncell + c];
  }
  return 0;
}

ORC_API int orc_set_state_cons(void* h, const double* Ui) {
  Oracle* o = static_cast<Oracle*>(h);
  const size_t ni = (size_t)o->nint();
  for (size_t lin = 0; lin < ni; ++lin) {
    const int i = (int)(lin % o->n[0]);
    const int j = (int)((lin / o->n[0]) % o->n[1]);
    const int k = (int)(lin / ((size_t)o->n[0] * o->n[1]));
    const size_t c = o->idx(i, j, k);
    for (int q = 0; q < o->L.n; ++q) o->U[(size_t)q * o->ncell + c] = Ui[(size_t)q * ni + lin];
  }
  return 0;
}

// Rigid volume fraction from a signed distance (negative inside the body):
// r = (1 - tanh(d / (width dx_min))) / 2. Reading: the paper obtains r from
// a cut-cell volume of an STL surface (Sec. 4.8); a tanh profile of the signed
// distance replaces it here.
ORC_API int orc_set_rigid_sdf(void* h, const double* sdf, double width, const double* v,
                              const double* omega, const double* center) {
  Oracle* o = static_cast<Oracle*>(h);
  double dmin = o->dx[0];
  for (int d = 1; d < o->dim; ++d) dmin = std::min(dmin, o->dx[d]);
  const size_t ni = (size_t)o->nint();
  double* r = o->f(o->L.R());
  for (size_t lin = 0; lin < ni; ++lin) {
    const int i = (int)(lin % o->n[0]);
    const int j = (int)((lin / o->n[0]) % o->n[1]);
    const int k = (int)(lin / ((size_t)o->n[0] * o->n[1]));
    r[o->idx(i, j, k)] = 0.5 * (1.0 - std::tanh(sdf[lin] / (width * dmin)));
  }
  o->set_one_body(v, omega, center);
  return 0;
}

ORC_API int orc_set_rigid_motion(void* h, const double* v, const double* omega, const double* center) {
  static_cast<Oracle*>(h)->set_one_body(v, omega, center);
  return 0;
}

// Several rigid bodies in one r field (the extrusion test of Sec. 4.5: a
// moving piston and a static wedge): nbody x 3 motions, and for bodies
// 1..nbody-1 their ownership boxes [lo, hi) (row 0 unused). Returns -1 for
// nbody outside 1..kMaxBodies.
ORC_API int orc_set_rigid_bodies(void* h, int nbody, const double* v, const double* omega, const double* center,
                                 const double* lo, const double* hi) {
  Oracle* o = static_cast<Oracle*>(h);
  if (nbody < 1 || nbody > kMaxBodies) return -1;
  o->nbody = nbody;
  for (int k = 0; k < nbody; ++k)
    for (int a = 0; a < 3; ++a) {
      o->vr[k][a] = v[3 * k + a];
      o->om[k][a] = omega[3 * k + a];
      o->ctr[k][a] = center[3 * k + a];
      o->box_lo[k][a] = k > 0 ? lo[3 * k + a] : 0.0;
      o->box_hi[k][a] = k > 0 ? hi[3 * k + a] : 0.0;
    }
  return 0;
}

// Void-opening face modifier: mode 0 off (default), 1 on; Wgap: primitive
// state of the gas that fills an opening gap (its velocity and r are set per
// face). Returns -1 for another mode or a fluid system.
ORC_API int orc_set_face_mod(void* h, int mode, const double* Wgap) {
  Oracle* o = static_cast<Oracle*>(h);
  if (mode != 0 && mode != 1) return -1;
  if (mode == 1 && !o->L.solid) return -1;  // elastoplastic systems only
  o->face_mod = mode;
  if (Wgap)
    for (int q = 0; q < o->L.n; ++q) o->gap_W[q] = Wgap[q];
  return 0;
}

ORC_API double orc_compute_dt(void* h, double cfl) { return static_cast<Oracle*>(h)->compute_dt(cfl); }

ORC_API int orc_step(void* h, double dt) {
  Oracle* o = static_cast<Oracle*>(h);
  o->step(dt);
  // each body's centre and ownership box move with its translational velocity
  for (int k = 0; k < o->nbody; ++k)
    for (int a = 0; a < 3; ++a) {
      o->ctr[k][a] += o->vr[k][a] * dt;
      o->box_lo[k][a] += o->vr[k][a] * dt;
      o->box_hi[k][a] += o->vr[k][a] * dt;
    }
  return 0;
}

ORC_API int orc_seed(void* h) { static_cast<Oracle*>(h)->do_seed(); return 0; }

// The semi-discrete operator D(U) of the current state (no seeding), rigid
// mask from the current r: out [nfields][interior cells].
ORC_API int orc_rhs(void* h, double* out, int dirmask) {
  Oracle* o = static_cast<Oracle*>(h);
  o->dirmask = dirmask;
  std::vector<unsigned char> rigid(o->ncell, 0);
  const double* r = o->f(o->L.R());
  for (size_t c = 0; c < o->ncell; ++c) rigid[c] = r[c] > 0.5;
  std::vector<double> D;
  o->rhs(o->U, rigid, D);
  const size_t ni = (size_t)o->nint();
  for (size_t lin = 0; lin < ni; ++lin) {
    const int i = (int)(lin % o->n[0]);
    const int j = (int)((lin / o->n[0]) % o->n[1]);
    const int k = (int)(lin / ((size_t)o->n[0] * o->n[1]));
    const size_t c = o->idx(i, j, k);
    for (int q = 0; q < o->L.n; ++q) out[(size_t)q * ni + lin] = D[(size_t)q * o->ncell + c];
  }
  o->dirmask = 7;
  return 0;
}

ORC_API double orc_time(void* h) { return static_cast<Oracle*>(h)->t; }

ORC_API void orc_stats(void* h, long* out) {
  Oracle* o = static_cast<Oracle*>(h);
  out[0] = o->seeded; out[1] = o->probe_fail; out[2] = o->fallback;
}

// Force and torque exerted by the material on the rigid body, FP64.
// Reading (the paper's bodies are one-way and it defines no load): the
// diffuse-surface integral F = sum_i (-sigma_i . grad_h r_i) dV and
// T = sum_i (x_i - c) x (-sigma_i . grad_h r_i) dV over interior cells, on the
// stored state (rigid cells hold their seeded states), central differences.
ORC_API int orc_rigid_force(void* h, const double* center, double* F, double* T) {
  Oracle* o = static_cast<Oracle*>(h);
  std::vector<double> X = o->U;
  o->fill_ghosts(X);
  const size_t ni = (size_t)o->nint();
  std::vector<double> terms[6];
  for (auto& t : terms) t.assign(ni, 0.0);
  const double dV = o->cell_volume();
  const double* r = X.data() + (size_t)o->L.R() * o->ncell;
#pragma omp parallel for schedule(static)
  for (long lin = 0; lin < (long)ni; ++lin) {
    const int i = (int)(lin % o->n[0]);
    const int j = (int)((lin / o->n[0]) % o->n[1]);
    const int k = (int)(lin / ((long)o->n[0] * o->n[1]));
    const size_t c = o->idx(i, j, k);
    double gr[3] = {0, 0, 0};
    bool any = false;
    for (int d = 0; d < o->dim; ++d) {
      gr[d] = (r[c + o->stride(d)] - r[c - o->stride(d)]) / (2.0 * o->dx[d]);
      if (gr[d] != 0.0) any = true;
    }
    if (!any) continue;
    double Uc[kMaxF], W[kMaxF];
    for (int q = 0; q < o->L.n; ++q) Uc[q] = X[(size_t)q * o->ncell + c];
    o->cons_to_prim(Uc, W);
    CellThermo th;
    o->thermo_from_prim(W, th);
    double fc[3];
    for (int a = 0; a < 3; ++a) {
      double s = 0;
      for (int b = 0; b < 3; ++b) s -= th.sigma[a][b] * gr[b];
      fc[a] = s * dV;
    }
    const int pos[3] = {i, j, k};
    double xr[3] = {0, 0, 0};
    for (int a = 0; a < o->dim; ++a) xr[a] = o->xc(a, pos[a]) - center[a];
    for (int a = 0; a < 3; ++a) terms[a][lin] = fc[a];
    terms[3][lin] = xr[1] * fc[2] - xr[2] * fc[1];
    terms[4][lin] = xr[2] * fc[0] - xr[0] * fc[2];
    terms[5][lin] = xr[0] * fc[1] - xr[1] * fc[0];
  }
  for (int a = 0; a < 3; ++a) {
    F[a] = pairwise_sum(terms[a].data(), ni);
    T[a] = pairwise_sum(terms[3 + a].data(), ni);
  }
  return 0;
}

// Totals of every conserved field times the cell volume: out[0..n) over all
// interior cells, out[n..2n) over non-rigid (r <= 0.5) cells.
ORC_API int orc_conserved_totals(void* h, double* out) {
  Oracle* o = static_cast<Oracle*>(h);
  const size_t ni = (size_t)o->nint();
  const double dV = o->cell_volume();
  std::vector<double> a(ni), b(ni);
  const double* r = o->f(o->L.R());
  for (int q = 0; q < o->L.n; ++q) {
    const double* fq = o->f(q);
    for (size_t lin = 0; lin < ni; ++lin) {
      const int i = (int)(lin % o->n[0]);
      const int j = (int)((lin / o->n[0]) % o->n[1]);
      const int k = (int)(lin / ((size_t)o->n[0] * o->n[1]));
      const size_t c = o->idx(i, j, k);
      a[lin] = fq[c] * dV;
      b[lin] = r[c] > 0.5 ? 0.0 : fq[c] * dV;
    }
    out[q] = pairwise_sum(a.data(), ni);
    out[o->L.n + q] = pairwise_sum(b.data(), ni);
  }
  return 0;
}

// ---- unit-level entry points for the pins ----------------------------------

ORC_API void orc_candidates(void* h, double qm, double q0, double qp, double* out4) {
  static_cast<Oracle*>(h)->candidates(qm, q0, qp, out4);
}

// BVD selection of one cell from the candidates of the left neighbour, the
// cell and the right neighbour (4 values each, as orc_candidates returns).
ORC_API void orc_bvd_select(void* h, const double* cm, const double* c0, const double* cp, double* out2) {
  static_cast<Oracle*>(h)->bvd_select(cm, c0, cp, out2[0], out2[1]);
}

ORC_API void orc_prim_to_cons(void* h, const double* W, double* Uc) { static_cast<Oracle*>(h)->prim_to_cons(W, Uc); }
ORC_API void orc_cons_to_prim(void* h, const double* Uc, double* W) { static_cast<Oracle*>(h)->cons_to_prim(Uc, W); }

// thermo: out = {rho, p, c2, G, sigY, J2, sigma[9], H[9]}
ORC_API void orc_thermo(void* h, const double* W, double* out) {
  CellThermo th;
  static_cast<Oracle*>(h)->thermo_from_prim(W, th);
  out[0] = th.rho; out[1] = th.p; out[2] = th.c2; out[3] = th.G; out[4] = th.sigY; out[5] = th.J2;
  for (int q = 0; q < 9; ++q) { out[6 + q] = th.sigma[q / 3][q % 3]; out[15 + q] = th.H[q / 3][q % 3]; }
}

// flux of the thermodynamic fields at one face: F[n-1], then u*, Vstar[3]
ORC_API void orc_face_flux(void* h, const double* WL, const double* WR, int d, double* out) {
  Oracle* o = static_cast<Oracle*>(h);
  double Fo[kMaxF], us, vs[3];
  o->hllc(WL, WR, d, Fo, us, vs);
  const int nt = o->L.n - 1;
  for (int q = 0; q < nt; ++q) out[q] = Fo[q];
  out[nt] = us;
  for (int b = 0; b < 3; ++b) out[nt + 1 + b] = vs[b];
}

ORC_API void orc_phys_flux(void* h, const double* W, int d, double* F) {
  Oracle* o = static_cast<Oracle*>(h);
  double Uc[kMaxF];
  o->prim_to_cons(W, Uc);
  CellThermo th;
  o->thermo_from_prim(W, th);
  o->phys_flux(W, Uc, th, d, F);
}

ORC_API void orc_mirror_state(void* h, const double* W, const double* nrm, const double* v, double* Wout) {
  static_cast<Oracle*>(h)->mirror_state(W, nrm, v, Wout);
}

ORC_API void orc_riemann_seed_state(void* h, const double* Wm, const double* Wi, const double* nrm, double* Wout) {
  static_cast<Oracle*>(h)->riemann_star_right(Wm, Wi, nrm, Wout);
}

// ELVIRA pieces for the pins: normal of a 3x3 block f9[(a+1)*3 + (b+1)] =
// r(i+a, j+b) (returns 0 where undefined), and the cut fraction of a cell.
ORC_API int orc_elvira_normal(const double* f9, double hx, double hy, double* n2) {
  double f[3][3];
  for (int q = 0; q < 9; ++q) f[q / 3][q % 3] = f9[q];
  return Oracle::elvira_normal(f, hx, hy, n2) ? 1 : 0;
}
ORC_API double orc_cut_fraction(const double* n2, double hx, double hy, double beta) {
  return Oracle::cut_fraction(n2, hx, hy, beta);
}

ORC_API void orc_solid_sources(void* h, double* Uc) { static_cast<Oracle*>(h)->solid_sources(Uc); }

ORC_API void orc_hencky(const double* V9, double* H9) {
  double V[3][3], H[3][3];
  for (int q = 0; q < 9; ++q) V[q / 3][q % 3] = V9[q];
  hencky(V, H);
  for (int q = 0; q < 9; ++q) H9[q] = H[q / 3][q % 3];
}

ORC_API void orc_phase_ref(int kind, const double* p, double rho, double J2, double* out) {
  Material m;
  m.kind = kind;
  if (kind == EOS_IDEAL) m.gamma = p[0];
  else if (kind == EOS_STIFFENED) { m.gamma = p[0]; m.pinf = p[1]; }
  else { m.rho0 = p[0]; m.K0 = p[1]; m.G0 = p[2]; m.alpha = p[3]; m.beta = p[4]; m.Gamma0 = p[5]; m.sigY = p[6]; }
  PhaseRef r = phase_ref(m, rho, J2);
  out[0] = r.rhoe_ref; out[1] = r.p_ref; out[2] = r.Gam; out[3] = r.dpref_drho; out[4] = r.G;
}
