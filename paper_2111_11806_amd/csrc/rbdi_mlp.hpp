// rbdi_mlp.hpp -- the learned surrogate of the elastoplastic closure:
// a 6 -> 64 -> 64 -> 64 -> 6 ReLU network with BF16 weights and FP32
// accumulation, evaluated and trained with gfx950 matrix-core instructions
// (v_mfma_f32_16x16x32_bf16), and the per-stage elastoplastic source pass
// that uses it (not part of the paper: a data-driven replacement of the
// closure step the paper's method performs per cell).
//
// What the network represents. For b = Vbar Vbar^T and X = b - I, the Hencky
// strain H = (1/2) ln b and its square are isotropic functions of X, so by
// the Cayley-Hamilton theorem H = a0 I + a1 X + a2 X^2 and
// H^2 = c0 I + c1 X + c2 X^2 with coefficients that are functions of the
// invariants of X. The series of (1/2) ln(I + X) and (1/4) ln(I + X)^2 up
// to X^3 fix the leading parts of (a, c); the network returns the remainders
// (the terms of order X^4 and up) scaled by kappa tau^p (tau = |X|_F,
// p = 4, 3, 2 for the coefficients of I, X, X^2), so that its error shrinks
// with the strain like the remainder itself. Inputs: tau / tau_max, the
// shape invariants e1/tau, e2/tau^2, e3/tau^3 of X (principal invariants e),
// (tau / tau_max)^2 and (e1/tau)(tau/tau_max).
//
// Matrix-core layout (wave64, 16x16x32 BF16, as used below): the A operand
// (16 x 32) has lane l holding row l%16, k = 8(l/16) .. 8(l/16)+7; the B
// operand (32 x 16) has lane l holding column l%16 and the same k; the
// 16 x 16 FP32 result has lane l holding column l%16, rows 4(l/16) .. +3.
// A layer computes Z^T = W A^T: weights are the A operand (rows = units),
// the activations of 64 samples (one per lane of the wave) are the B
// operand, read from a per-wavefront LDS tile [sample][unit].
#pragma once

#include "rbdi_kernels.hpp"

namespace rbdi {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 6, kMlpHid = 64, kMlpOut = 6;
constexpr int kLdA = 72;  // LDS row stride (bf16) of an activation tile
constexpr double kMlpKappa = 0.125;
constexpr double kTauTiny = 1e-30;  // below: shape features and remainders taken as 0

// Flat FP32 parameter layout (unpadded, row-major [out][in]):
// W1[64][6] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[6][64] b4[6].
constexpr int kOffW1 = 0, kOffB1 = 384, kOffW2 = 448, kOffB2 = 4544, kOffW3 = 4608, kOffB3 = 8704,
              kOffW4 = 8768, kOffB4 = 9152, kNParam = 9158;

// Device copies: BF16 operands in padded layouts, FP32 biases.
struct MlpDev {
  const __bf16* W1;   // [64][32], columns 6.. zero
  const __bf16* W2;   // [64][64]
  const __bf16* W3;   // [64][64]
  const __bf16* W4;   // [16][64], rows 6.. zero
  const __bf16* W2T;  // [64][64] = W2^T
  const __bf16* W3T;  // [64][64] = W3^T
  const __bf16* W4T;  // [64][32] = W4^T, columns 6.. zero
  const float* b1;
  const float* b2;
  const float* b3;
  const float* b4;    // [16], entries 6.. zero
  double tau_max;     // envelope: |X|_F <= tau_max; input scale
};

// Element counts of the padded device arrays (bf16 blob order as above).
constexpr int kW1n = 64 * 32, kW2n = 64 * 64, kW3n = 64 * 64, kW4n = 16 * 64, kW2Tn = 64 * 64, kW3Tn = 64 * 64,
              kW4Tn = 64 * 32;
constexpr int kBlobBf16 = kW1n + kW2n + kW3n + kW4n + kW2Tn + kW3Tn + kW4Tn;
constexpr int kBiasN = 64 + 64 + 64 + 16;

// ---------------------------------------------------------------------------
// Features, decoding and exact targets
// ---------------------------------------------------------------------------

struct StrainInv {
  SymM X, X2;
  double tau, e1, e2, e3;
};

__device__ inline StrainInv strain_invariants(const double V[9]) {
  StrainInv s;
  s.X.a00 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2] - 1.0;
  s.X.a11 = V[3] * V[3] + V[4] * V[4] + V[5] * V[5] - 1.0;
  s.X.a22 = V[6] * V[6] + V[7] * V[7] + V[8] * V[8] - 1.0;
  s.X.a01 = V[0] * V[3] + V[1] * V[4] + V[2] * V[5];
  s.X.a02 = V[0] * V[6] + V[1] * V[7] + V[2] * V[8];
  s.X.a12 = V[3] * V[6] + V[4] * V[7] + V[5] * V[8];
  s.X2 = sym_sq(s.X);
  const double t2 = s.X2.a00 + s.X2.a11 + s.X2.a22;
  s.tau = sqrt(t2);
  s.e1 = s.X.a00 + s.X.a11 + s.X.a22;
  s.e2 = 0.5 * (s.e1 * s.e1 - t2);
  const SymM& X = s.X;
  s.e3 = X.a00 * (X.a11 * X.a22 - X.a12 * X.a12) - X.a01 * (X.a01 * X.a22 - X.a12 * X.a02) +
         X.a02 * (X.a01 * X.a12 - X.a11 * X.a02);
  return s;
}

__device__ inline void mlp_features(const StrainInv& s, double tau_max, float z[6]) {
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (s.tau > kTauTiny) {
    const double it = 1.0 / s.tau;
    s1 = s.e1 * it;
    s2 = s.e2 * it * it;
    s3 = s.e3 * it * it * it;
  }
  const double m = s.tau / tau_max;
  z[0] = (float)m;
  z[1] = (float)s1;
  z[2] = (float)s2;
  z[3] = (float)s3;
  z[4] = (float)(m * m);
  z[5] = (float)(s1 * m);
}

// (a0, a1, a2, c0, c1, c2) from the network outputs.
__device__ inline void mlp_decode(const StrainInv& s, const float y[6], double a[3], double c[3]) {
  const double t2 = s.tau * s.tau, t3 = t2 * s.tau, t4 = t2 * t2;
  a[0] = s.e3 / 6.0 + kMlpKappa * t4 * (double)y[0];
  a[1] = 0.5 - s.e2 / 6.0 + kMlpKappa * t3 * (double)y[1];
  a[2] = -0.25 + s.e1 / 6.0 + kMlpKappa * t2 * (double)y[2];
  c[0] = -0.25 * s.e3 + kMlpKappa * t4 * (double)y[3];
  c[1] = 0.25 * s.e2 + kMlpKappa * t3 * (double)y[4];
  c[2] = 0.25 - 0.25 * s.e1 + kMlpKappa * t2 * (double)y[5];
}

// Exact normalised remainders: the terms k >= 4 of (1/2) ln(I + X) =
// sum_k (-1)^(k+1) X^k / (2k) and (1/4) ln(I + X)^2 =
// sum_{k>=2} (-1)^k H_{k-1} X^k / (2k) (H_n harmonic numbers), each power in
// the I, X, X^2 basis by the Cayley-Hamilton recurrence.
__device__ inline void mlp_targets(const StrainInv& s, float t[6]) {
  double al = 0.0, be = 1.0, ga = 0.0;  // X^1
  double ra[3] = {0.0, 0.0, 0.0}, rc[3] = {0.0, 0.0, 0.0};
  double harm = 1.0;  // H_{k-1} at k = 2
  const double lead = 0.5 * s.tau;
  for (int k = 1; k <= 200; ++k) {
    if (k > 2) harm += 1.0 / (double)(k - 1);
    if (k >= 4) {
      const double wa = (k & 1 ? 0.5 : -0.5) / (double)k;
      const double wc = (k & 1 ? -0.5 : 0.5) * harm / (double)k;
      ra[0] += wa * al; ra[1] += wa * be; ra[2] += wa * ga;
      rc[0] += wc * al; rc[1] += wc * be; rc[2] += wc * ga;
      const double mag = (fabs(al) + fabs(be) * s.tau + fabs(ga) * s.tau * s.tau);
      if (mag <= 1e-18 * lead) break;
    }
    const double nal = ga * s.e3, nbe = al - ga * s.e2, nga = be + ga * s.e1;
    al = nal;
    be = nbe;
    ga = nga;
  }
  const double t2 = s.tau * s.tau, t3 = t2 * s.tau, t4 = t2 * t2;
  const bool ok = s.tau > kTauTiny;
  t[0] = ok ? (float)(ra[0] / (kMlpKappa * t4)) : 0.0f;
  t[1] = ok ? (float)(ra[1] / (kMlpKappa * t3)) : 0.0f;
  t[2] = ok ? (float)(ra[2] / (kMlpKappa * t2)) : 0.0f;
  t[3] = ok ? (float)(rc[0] / (kMlpKappa * t4)) : 0.0f;
  t[4] = ok ? (float)(rc[1] / (kMlpKappa * t3)) : 0.0f;
  t[5] = ok ? (float)(rc[2] / (kMlpKappa * t2)) : 0.0f;
}

// ---------------------------------------------------------------------------
// Wavefront forward pass (inference): 64 samples, one per lane
// ---------------------------------------------------------------------------

struct __align__(16) MlpWaveLds {
  __bf16 act[64 * kLdA];
  float y[64 * 8];
};

__device__ inline bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

// Order LDS writes of some lanes before reads by other lanes of the same
// wavefront.
__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One layer in place on the activation tile: Z^T = W A^T + b, ReLU unless
// the last layer (FP32 result into y[sample][unit], units < 8 kept).
template <int MT, int KT, bool LAST>
__device__ inline void mlp_layer_inplace(const __bf16* __restrict__ W, const float* __restrict__ b, MlpWaveLds* L) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  bf16x8 a[MT][KT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) a[mt][kt] = ld8(W + (mt * 16 + r) * (KT * 32) + kt * 32 + 8 * g);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    floatx4 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      const bf16x8 bb = ld8(L->act + (nt * 16 + r) * kLdA + kt * 32 + 8 * g);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt][kt], bb, acc[mt], 0, 0, 0);
    }
    // every lane of the wavefront has read rows nt*16.. before any is written
    wave_sync_lds();
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int u = mt * 16 + 4 * g + i;
        float v = acc[mt][i] + b[u];
        if (LAST) {
          if (u < 8) L->y[(nt * 16 + r) * 8 + u] = v;
        } else {
          L->act[(nt * 16 + r) * kLdA + u] = (__bf16)fmaxf(v, 0.0f);
        }
      }
    wave_sync_lds();
  }
}

// Forward pass of the wavefront's 64 samples (lane = sample). Every lane of
// the wavefront must call it (matrix instructions use all lanes).
__device__ inline void mlp_wave_forward(const MlpDev& m, MlpWaveLds* L, const float z[6], float y[6]) {
  const int lane = threadIdx.x & 63;
  __bf16* row = L->act + lane * kLdA;
#pragma unroll
  for (int k = 0; k < 32; ++k) row[k] = (__bf16)(k < kMlpIn ? z[k] : 0.0f);
  wave_sync_lds();
  mlp_layer_inplace<4, 1, false>(m.W1, m.b1, L);
  mlp_layer_inplace<4, 2, false>(m.W2, m.b2, L);
  mlp_layer_inplace<4, 2, false>(m.W3, m.b3, L);
  mlp_layer_inplace<1, 2, true>(m.W4, m.b4, L);
  wave_sync_lds();
#pragma unroll
  for (int o = 0; o < kMlpOut; ++o) y[o] = L->y[lane * 8 + o];
}

// Batched inference (tests): z [n][6] -> y [n][6].
__global__ __launch_bounds__(256) void k_mlp_infer(MlpDev m, const float* __restrict__ z, float* __restrict__ y,
                                                  int n) {
  __shared__ MlpWaveLds lds[4];
  const int wave = threadIdx.x >> 6;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float zi[6], yi[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) zi[k] = i < n ? z[i * 6 + k] : 0.0f;
  mlp_wave_forward(m, &lds[wave], zi, yi);
  if (i < n)
#pragma unroll
    for (int k = 0; k < 6; ++k) y[i * 6 + k] = yi[k];
}

// ---------------------------------------------------------------------------
// Training: forward + backward of 64 samples per wavefront (one wavefront
// per block), per-block gradient partials, then a fixed-order reduction and
// the Adam update.
// ---------------------------------------------------------------------------

struct __align__(16) MlpTrainLds {
  __bf16 x0[64 * 40];
  __bf16 a1[64 * kLdA], a2[64 * kLdA], a3[64 * kLdA];
  __bf16 d0[64 * kLdA], d1[64 * kLdA];
  float y[64 * 8];
};

// Z^T = W A^T + b into out (ReLU) or into y (last layer), not in place.
template <int MT, int KT, bool LAST>
__device__ inline void mlp_layer_fwd(const __bf16* __restrict__ W, const float* __restrict__ b,
                                     const __bf16* in, int ldi, __bf16* out, float* y) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(W + (mt * 16 + r) * (KT * 32) + kt * 32 + 8 * g),
                                                      ld8(in + (nt * 16 + r) * ldi + kt * 32 + 8 * g), acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int u = mt * 16 + 4 * g + i;
        const float v = acc[i] + b[u];
        if (LAST) {
          if (u < 8) y[(nt * 16 + r) * 8 + u] = v;
        } else {
          out[(nt * 16 + r) * kLdA + u] = (__bf16)fmaxf(v, 0.0f);
        }
      }
    }
}

// Gather 8 bf16 values p[(k0 + j) * ld] (a column of a [sample][unit] tile).
__device__ inline bf16x8 gather8(const __bf16* p, int ld) {
  bf16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = p[j * ld];
  return v;
}

// dW[u][k] = sum_s delta[s][u] act[s][k] over the 64 samples: MT unit tiles,
// NT input tiles; written (FP32) to gw[u * ldw + k] for u < nu, k < nk.
template <int MT, int NT>
__device__ inline void mlp_dw(const __bf16* delta, const __bf16* act, int lda, float* gw, int ldw, int nu, int nk) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const bf16x8 av = gather8(delta + (ks * 32 + 8 * g) * kLdA + mt * 16 + r, kLdA);
        const bf16x8 bv = gather8(act + (ks * 32 + 8 * g) * lda + nt * 16 + r, lda);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int u = mt * 16 + 4 * g + i, k = nt * 16 + r;
        if (u < nu && k < nk) gw[u * ldw + k] = acc[i];
      }
    }
}

// delta_in[s][k] = (sum_u W[u][k] delta[s][u]) * [act_in[s][k] > 0], with
// WT = W^T ([k][u], KT*32 columns) as the A operand.
template <int MT, int KT>
__device__ inline void mlp_dback(const __bf16* __restrict__ WT, const __bf16* delta, const __bf16* act_in,
                                 __bf16* delta_in) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(WT + (mt * 16 + r) * (KT * 32) + kt * 32 + 8 * g),
                                                      ld8(delta + (nt * 16 + r) * kLdA + kt * 32 + 8 * g), acc, 0,
                                                      0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = mt * 16 + 4 * g + i, s = nt * 16 + r;
        const bool on = (float)act_in[s * kLdA + k] > 0.0f;
        delta_in[s * kLdA + k] = (__bf16)(on ? acc[i] : 0.0f);
      }
    }
}

// Gradient of the mean squared error (over the ntot samples of the batch and
// the 6 outputs) of samples [first + 64 b, first + 64 b + 64) clipped at
// first + count; one partial row (kNParam gradients + the loss) per block.
__global__ __launch_bounds__(64) void k_mlp_grad(MlpDev m, const float* __restrict__ z, const float* __restrict__ t,
                                                long long first, int count, int ntot, float* __restrict__ part) {
  __shared__ MlpTrainLds L;
  const int lane = threadIdx.x;
  const int sidx = blockIdx.x * 64 + lane;
  const bool valid = sidx < count;
  const long long si = first + sidx;
  float zi[6], ti[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    zi[k] = valid ? z[si * 6 + k] : 0.0f;
    ti[k] = valid ? t[si * 6 + k] : 0.0f;
  }
  for (int k = 0; k < 40; ++k) L.x0[lane * 40 + k] = (__bf16)(k < 6 ? zi[k] : 0.0f);
  wave_sync_lds();
  mlp_layer_fwd<4, 1, false>(m.W1, m.b1, L.x0, 40, L.a1, nullptr);
  wave_sync_lds();
  mlp_layer_fwd<4, 2, false>(m.W2, m.b2, L.a1, kLdA, L.a2, nullptr);
  wave_sync_lds();
  mlp_layer_fwd<4, 2, false>(m.W3, m.b3, L.a2, kLdA, L.a3, nullptr);
  wave_sync_lds();
  mlp_layer_fwd<1, 2, true>(m.W4, m.b4, L.a3, kLdA, nullptr, L.y);
  wave_sync_lds();
  // output error: dL/dy = 2 (y - t) / (6 ntot); padded outputs zero
  const float scale = 2.0f / (6.0f * (float)ntot);
  float loss = 0.0f;
  for (int k = 0; k < 32; ++k) {
    float d = 0.0f;
    if (k < 6 && valid) {
      const float e = L.y[lane * 8 + k] - ti[k];
      loss += e * e;
      d = scale * e;
    }
    L.d0[lane * kLdA + k] = (__bf16)d;
  }
  wave_sync_lds();
  float* P = part + (size_t)blockIdx.x * (kNParam + 1);
  // layer 4
  mlp_dw<1, 4>(L.d0, L.a3, kLdA, P + kOffW4, 64, 6, 64);
  if (lane < 6) {
    float s = 0.0f;
    for (int q = 0; q < 64; ++q) s += (float)L.d0[q * kLdA + lane];
    P[kOffB4 + lane] = s;
  }
  mlp_dback<4, 1>(m.W4T, L.d0, L.a3, L.d1);
  wave_sync_lds();
  // layer 3
  mlp_dw<4, 4>(L.d1, L.a2, kLdA, P + kOffW3, 64, 64, 64);
  {
    float s = 0.0f;
    for (int q = 0; q < 64; ++q) s += (float)L.d1[q * kLdA + lane];
    P[kOffB3 + lane] = s;
  }
  mlp_dback<4, 2>(m.W3T, L.d1, L.a2, L.d0);
  wave_sync_lds();
  // layer 2
  mlp_dw<4, 4>(L.d0, L.a1, kLdA, P + kOffW2, 64, 64, 64);
  {
    float s = 0.0f;
    for (int q = 0; q < 64; ++q) s += (float)L.d0[q * kLdA + lane];
    P[kOffB2 + lane] = s;
  }
  mlp_dback<4, 2>(m.W2T, L.d0, L.a1, L.d1);
  wave_sync_lds();
  // layer 1
  mlp_dw<4, 1>(L.d1, L.x0, 40, P + kOffW1, 6, 64, 6);
  {
    float s = 0.0f;
    for (int q = 0; q < 64; ++q) s += (float)L.d1[q * kLdA + lane];
    P[kOffB1 + lane] = s;
  }
  for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o);
  if (lane == 0) P[kNParam] = loss / (6.0f * (float)ntot);
}

// Sum of the per-block partial rows in block order (deterministic).
// Gradients go to grad[0..kNParam), the loss to *loss.
__global__ void k_mlp_sum(const float* __restrict__ part, int nblocks, float* __restrict__ grad,
                          float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kNParam) return;
  float s = 0.0f;
  for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * (kNParam + 1) + p];
  if (p < kNParam) grad[p] = s;
  else *loss = s;
}

// Where parameter p lives in the padded BF16 arrays (W and W^T copies).
struct MlpSlots {
  int w, wt, bias;  // blob index of W, of W^T (-1: none), bias index (-1: none)
};

__host__ __device__ inline MlpSlots mlp_slots(int p) {
  MlpSlots s{-1, -1, -1};
  const int oW2 = kW1n, oW3 = oW2 + kW2n, oW4 = oW3 + kW3n, oW2T = oW4 + kW4n, oW3T = oW2T + kW2Tn,
            oW4T = oW3T + kW3Tn;
  if (p < kOffB1) {
    const int u = p / 6, k = p % 6;
    s.w = u * 32 + k;
  } else if (p < kOffW2) {
    s.bias = p - kOffB1;
  } else if (p < kOffB2) {
    const int q = p - kOffW2, u = q / 64, k = q % 64;
    s.w = oW2 + u * 64 + k;
    s.wt = oW2T + k * 64 + u;
  } else if (p < kOffW3) {
    s.bias = 64 + (p - kOffB2);
  } else if (p < kOffB3) {
    const int q = p - kOffW3, u = q / 64, k = q % 64;
    s.w = oW3 + u * 64 + k;
    s.wt = oW3T + k * 64 + u;
  } else if (p < kOffW4) {
    s.bias = 128 + (p - kOffB3);
  } else if (p < kOffB4) {
    const int q = p - kOffW4, o = q / 64, k = q % 64;
    s.w = oW4 + o * 64 + k;
    s.wt = oW4T + k * 32 + o;
  } else {
    s.bias = 192 + (p - kOffB4);
  }
  return s;
}

// Write parameter p (FP32 master value v) into the device copies.
__device__ inline void mlp_store(__bf16* blob, float* bias, int p, float v) {
  const MlpSlots s = mlp_slots(p);
  if (s.w >= 0) blob[s.w] = (__bf16)v;
  if (s.wt >= 0) blob[s.wt] = (__bf16)v;
  if (s.bias >= 0) bias[s.bias] = v;
}

__global__ void k_mlp_sync(const float* __restrict__ master, __bf16* blob, float* bias) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kNParam) mlp_store(blob, bias, p, master[p]);
}

struct AdamArgs {
  float lr, beta1, beta2, eps;
  int step;  // 1-based
};

// Adam on the summed gradient of nblocks partial rows; also records the
// batch loss at loss_out.
__global__ void k_mlp_adam(const float* __restrict__ part, int nblocks, float* master, float* m1, float* m2,
                           __bf16* blob, float* bias, AdamArgs a, float* loss_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kNParam) return;
  float g = 0.0f;
  for (int b = 0; b < nblocks; ++b) g += part[(size_t)b * (kNParam + 1) + p];
  if (p == kNParam) {
    *loss_out = g;
    return;
  }
  const float mm = a.beta1 * m1[p] + (1.0f - a.beta1) * g;
  const float vv = a.beta2 * m2[p] + (1.0f - a.beta2) * g * g;
  m1[p] = mm;
  m2[p] = vv;
  const float mh = mm / (1.0f - powf(a.beta1, (float)a.step));
  const float vh = vv / (1.0f - powf(a.beta2, (float)a.step));
  const float w = master[p] - a.lr * mh / (sqrtf(vh) + a.eps);
  master[p] = w;
  mlp_store(blob, bias, p, w);
}

// Features and exact targets of n stretch tensors V [n][9] (FP64).
__global__ void k_mlp_data(const double* __restrict__ V, int n, double tau_max, float* __restrict__ z,
                           float* __restrict__ t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v[9];
  for (int q = 0; q < 9; ++q) v[q] = V[(size_t)i * 9 + q];
  const StrainInv s = strain_invariants(v);
  float zi[6], ti[6];
  mlp_features(s, tau_max, zi);
  mlp_targets(s, ti);
  for (int q = 0; q < 6; ++q) {
    z[(size_t)i * 6 + q] = zi[q];
    t[(size_t)i * 6 + q] = ti[q];
  }
}

// ---------------------------------------------------------------------------
// Elastoplastic sources with the surrogate, inside the final sweep of each
// stage (SurrogateSources, called by every lane of the wavefront on its
// updated cell): det(Vbar) renormalisation; H and J2 = H:H from the network
// (the wavefront's 64 cells are one matrix tile) inside the envelope, the
// exact closure outside it or where the error flag is raised; perfect-
// plasticity radial return Vbar <- exp((s-1) H) Vbar with
// eps_p += sqrt(2/3)(1-s)|H|. Error flag: the network's J2 (from its H^2
// coefficients) disagrees with the J2 of its own H by more than 1e-6
// relative, or its H violates the identity tr H = (1/2) ln det(Vbar Vbar^T)
// = 0 of the renormalised stretch by more than 1e-6 |H|.
// ---------------------------------------------------------------------------
struct SurrogateSources {
  MlpDev m;
  MlpWaveLds* L;        // this wavefront's LDS tile
  DevScalars* sc;       // counters of network / exact closures

  template <class S, typename T>
  __device__ void operator()(const Params& P, T* Un, bool act) const {
    if constexpr (S::S) {
      // the tile shares its LDS with the sweep's d, which every lane has read
      wave_sync_lds();
      double V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
      if (act) {
#pragma unroll
        for (int q = 0; q < 9; ++q) V[q] = (double)Un[S::cV(0, 0) + q];
        const double det = V[0] * (V[4] * V[8] - V[5] * V[7]) - V[1] * (V[3] * V[8] - V[5] * V[6]) +
                           V[2] * (V[3] * V[7] - V[4] * V[6]);
        const double scl = 1.0 / cbrt(det);
#pragma unroll
        for (int q = 0; q < 9; ++q) V[q] *= scl;
      }
      // cells that provably do not yield keep V (renormalised) and skip the
      // closure; a wavefront without any other cell skips the network
      const bool ret = act && P.plastic && may_yield<S>(P, Un, V);
      const StrainInv si = strain_invariants(V);
      const bool env = ret && si.tau <= m.tau_max;
      float z[6] = {0, 0, 0, 0, 0, 0}, y[6] = {0, 0, 0, 0, 0, 0};
      if (env) mlp_features(si, m.tau_max, z);
      if (__any(env)) mlp_wave_forward(m, L, z, y);  // every lane of the wavefront
      int used_net = 0, used_exact = 0;
      if (ret) {
        double H[9], J2 = 0.0;
        bool ok = env;
        if (ok) {
          double a[3], cc[3];
          mlp_decode(si, y, a, cc);
          const SymM& X = si.X;
          const SymM& X2 = si.X2;
          const double h00 = a[0] + a[1] * X.a00 + a[2] * X2.a00, h11 = a[0] + a[1] * X.a11 + a[2] * X2.a11;
          const double h22 = a[0] + a[1] * X.a22 + a[2] * X2.a22, h01 = a[1] * X.a01 + a[2] * X2.a01;
          const double h02 = a[1] * X.a02 + a[2] * X2.a02, h12 = a[1] * X.a12 + a[2] * X2.a12;
          H[0] = h00; H[1] = h01; H[2] = h02; H[3] = h01; H[4] = h11; H[5] = h12; H[6] = h02; H[7] = h12; H[8] = h22;
          const double j2h = h00 * h00 + h11 * h11 + h22 * h22 + 2.0 * (h01 * h01 + h02 * h02 + h12 * h12);
          // J2 = tr(H^2) from the network's H^2 coefficients (tr X^2 = tau^2)
          J2 = 3.0 * cc[0] + cc[1] * si.e1 + cc[2] * si.tau * si.tau;
          ok = fabs(J2 - j2h) <= 1e-6 * j2h + 1e-300;
          // tr H = 3 a0 + a1 tr X + a2 tr X^2 must vanish (unit determinant)
          ok = ok && fabs(h00 + h11 + h22) <= 1e-6 * sqrt(j2h) + 1e-300;
          J2 = j2h;
        }
        if (!ok) hencky3(V, H, J2);
        used_net = ok ? 1 : 0;
        used_exact = ok ? 0 : 1;
        // closure terms of the plastic return: phases, pressure, G, yield
        double rho = 0.0;
#pragma unroll
        for (int l = 0; l < S::N; ++l) rho += (double)Un[S::cA(l)];
        double phi[kMaxMat], rl[kMaxMat], sph = 0.0;
#pragma unroll
        for (int l = 0; l < S::N - 1; ++l) {
          phi[l] = (double)Un[S::cPHI(l)];
          sph += phi[l];
        }
        phi[S::N - 1] = 1.0 - sph;
#pragma unroll
        for (int l = 0; l < S::N; ++l) rl[l] = (double)Un[S::cA(l)] / phi[l];
        double ke = 0.0;
#pragma unroll
        for (int a = 0; a < S::D; ++a) ke += (double)Un[S::cM(a)] * (double)Un[S::cM(a)] / rho;
        const double p = mix_pressure<S>(P, phi, rl, J2, (double)Un[S::cE] - 0.5 * ke);
        double c2, G, sY;
        mix_c2_G<S>(P, phi, rl, J2, p, c2, G, sY);
        const double Hn = sqrt(J2);
        const double seq = 2.449489742783178 * G * Hn;
        if (sY > 0.0 && seq > sY) {
          const double s = sY / seq;
          double E[9], Vn[9];
          plastic_exp(s - 1.0, H, E);
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) Vn[3 * a + b] = E[3 * a] * V[b] + E[3 * a + 1] * V[3 + b] + E[3 * a + 2] * V[6 + b];
#pragma unroll
          for (int q = 0; q < 9; ++q) V[q] = Vn[q];
          const int sp = P.solid_phase;
          const double as = pick<S::N>(phi, sp) * pick<S::N>(rl, sp);
          Un[S::cEP] = (T)((double)Un[S::cEP] + as * 0.816496580927726 * (1.0 - s) * Hn);
        }
      }
      if (act) {
#pragma unroll
        for (int q = 0; q < 9; ++q) Un[S::cV(0, 0) + q] = (T)V[q];
      }
      wave_count_add(&sc->surr_net, used_net);
      wave_count_add(&sc->surr_exact, used_exact);
    }
  }
};

// The final x sweep with the surrogate sources. LDS per wavefront: the
// streamed d, then (once d has been read back) the network's tile; and the
// d-independent part of the wavefront's RK combine.
template <class S, typename T>
struct XSurrLds {
  union {
    T d[S::NF * kWave];
    MlpWaveLds mlp;
  };
  double u[S::NF * kWave];  // the d-independent part of the wavefront's RK combine
};

template <class S, typename T, bool MB = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(x_sweep_waves<S>()))) void k_sweep_x_surr(
    Params P, const T* __restrict__ Uin, const T* __restrict__ U0, const T* __restrict__ Dacc,
    const T* __restrict__ Dacc2, T* __restrict__ Uout,
    DevScalars* __restrict__ sc, double* __restrict__ cflpart, StepArgs A, double bcoef, int stage, MlpDev m) {
  XSurrLds<S, T>* lds = dyn_lds<XSurrLds<S, T>>();  // one per wavefront, sized by the launch
  const int wpb = blockDim.x / kWave;
  int bx, by, bz;
  const long long blin = xcd_block(bx, by, bz);
  const int nparts = (int)(gridDim.x * gridDim.y * gridDim.z) * wpb;
  XSurrLds<S, T>* my = &lds[threadIdx.x / kWave];
  SurrogateSources src{m, &my->mlp, sc};
  sweep_x_body<S, T, SurrogateSources, MB>(P, Uin, U0, Dacc, Dacc2, Uout, sc, cflpart, A, bcoef, stage, bx, by, bz, blin,
                                           wpb, nparts, my->d, my->u, src);
}

}  // namespace rbdi
