// stage_kernels.h -- HIP kernels (gfx950) of one explicit finite-volume
// compressible-Euler SSP-RK2 stage over a list of work items.
//
// Method (arXiv 2507.09337, Sec. 6: explicit finite volume with a guard-cell
// halo, 2nd-order Runge-Kutta refreshing guards before each stage; Sec. 5.2:
// ideal-gas gamma-law EOS).  Reconstruction and flux follow the textbook
// methods named in include/hydro.h: PLM on primitives with minmod (or, as
// variants, on the conserved variables with the face states recovered
// afterwards, or on the characteristic variables of the primitive system),
// HLLC with Davis (or, as variants, Einfeldt or PVRS) wave speeds, SSP-RK2
// combine, CFL rate sum_d (|u_d| + c)/dx_d; as a further variant of the FP64
// tile, a gas + radiation EOS in place of the gamma law.
//
// Design for CDNA4 (wave64, 160 KiB LDS per CU, 8 XCDs):
//   * One workgroup = 256 threads = one x-y tile of a block (16x16) or four
//     independent 8x8 tiles (one per wave).  The workgroup marches its tile
//     column through the z planes of the block ("2.5-D"): the z direction
//     lives in registers (a sliding window of primitives per thread, so
//     every z face is computed once by the thread below it), the
//     current plane with its x/y guard ring lives in LDS.
//   * Guard cells are never stored: a tile load gathers them from the linked
//     neighbour block's interior (or wraps / repeats the edge), so HBM holds
//     interior cells only and there is no guard-fill pass.
//   * Loads are struct-of-arrays, one variable per instruction, x-fastest, so
//     a wave reads whole 128-byte lines.
//   * Every x and y face of a plane is one "face job" computed once from LDS
//     and shared by its two cells; the update differences the shared fluxes,
//     so the flux sum telescopes and mass, momentum and energy are conserved
//     to the rounding of the FP64 update.
//   * Primitive recovery (with e = E - rho|v|^2/2, where cancellation
//     happens), the RK combine and the CFL rate are always FP64.  In the mixed
//     variant the recovered primitives are rounded to FP32, reconstruction and
//     HLLC run in FP32 (hardware rcp/rsqrt), and the FP32 face fluxes are
//     widened to FP64 before they are differenced.
//   * The CFL rate of the new state is reduced in the stage-2 epilogue:
//     wave64 shuffles, then one 64-bit atomic max per wave on the bit pattern
//     of a non-negative double.  No MFMA: this is a stencil, not a contraction.
//
// Included by the instantiation units (kernels_inst.hip, built once per
// dimension, precision and stage) and by kernels.hip (rate kernels).
#pragma once
#include <climits>
#include <type_traits>

#include "hydro_internal.h"

namespace hyd {

// ------------------------------------------------------------------------
// FP32 arithmetic of the mixed tile (FP64 uses IEEE division and square root).
// ------------------------------------------------------------------------
template <typename T>
struct Arith;

template <>
struct Arith<float> {  // hardware reciprocal and reciprocal square root (about 1 ulp)
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
  // c = sqrt(g p / r) = g p / sqrt(g p r)
  static __device__ __forceinline__ float sound(float g, float p, float r) {
    float gp = g * p;
    return gp * __builtin_amdgcn_rsqf(gp * r);
  }
};

// minmod: the smaller-magnitude argument when both have the same strict sign,
// else 0.  That is the median of (a, b, 0): both positive gives min(a, b), both
// negative max(a, b), a sign change or a zero gives 0.  Four min/max
// instructions, no compares or selects; the value equals the sign-tested form
// (a zero result may carry either sign, which no later sum or product can see
// except in the sign of a zero).
template <typename T>
__host__ __device__ __forceinline__ T minmod(T a, T b) {
  return fmax(fmin(a, b), fmin(fmax(a, b), T(0)));
}

// PLM face states between w1 and w2 of four consecutive cells.
template <typename T>
__host__ __device__ __forceinline__ void plm(T w0, T w1, T w2, T w3, T &l, T &r) {
  T d01 = w1 - w0, d12 = w2 - w1, d23 = w3 - w2;
  l = w1 + T(0.5) * minmod(d01, d12);
  r = w2 - T(0.5) * minmod(d12, d23);
}

enum { SPEEDS_DAVIS = 0, SPEEDS_EINFELDT = 1, SPEEDS_PVRS = 2 };
// Variables PLM reconstructs.
enum { RECON_PRIMITIVE = 0, RECON_CONSERVED = 1, RECON_CHARACTERISTIC = 2 };
// Equation of state: the gamma law, or gas + radiation (FP64 tile only).
enum { EOS_IDEAL = 0, EOS_GAS_RADIATION = 1 };

// Gas + radiation EOS in units with gas and radiation constants 1:
//   p = rho T + T^4/3,  rho e = rho T/(gamma - 1) + T^4.
// The temperature is the root of a convex increasing quartic, found by
// Newton's method from an upper bound (the smaller of the gas-only and the
// radiation-only temperature): the iterates decrease until one no longer
// does.  First adiabatic exponent of the mixture (Clayton), beta = rho T / p:
//   Gamma1 = beta + (4 - 3 beta)^2 (gamma - 1)/(beta + 12 (gamma - 1)(1 - beta)).
// Plain FP64 in the order of the statement (IEEE division and square root),
// so each result is rounded as in a CPU evaluation of the same formulas.
constexpr double ARAD = 1.0;

__host__ __device__ __forceinline__ double gr_temperature_e(double rho, double rhoe, double gamma) {
#pragma clang fp contract(off)
  const double cv = rho / (gamma - 1.0);
  double T = fmin(rhoe / cv, __builtin_sqrt(__builtin_sqrt(rhoe / ARAD)));
  for (int k = 0; k < 64; ++k) {
    const double T3 = T * T * T;
    const double f = cv * T + ARAD * T3 * T - rhoe;
    const double fp = cv + 4.0 * ARAD * T3;
    const double Tn = T - f / fp;
    if (!(Tn < T)) break;
    T = Tn;
  }
  return T;
}

__host__ __device__ __forceinline__ double gr_temperature_p(double rho, double p) {
#pragma clang fp contract(off)
  double T = fmin(p / rho, __builtin_sqrt(__builtin_sqrt(3.0 * p / ARAD)));
  for (int k = 0; k < 64; ++k) {
    const double T3 = T * T * T;
    const double f = rho * T + ARAD * T3 * T / 3.0 - p;
    const double fp = rho + 4.0 * ARAD * T3 / 3.0;
    const double Tn = T - f / fp;
    if (!(Tn < T)) break;
    T = Tn;
  }
  return T;
}

__host__ __device__ __forceinline__ double gr_gamma1(double rho, double T, double p, double gamma) {
#pragma clang fp contract(off)
  const double beta = rho * T / p;
  const double g1 = gamma - 1.0;
  return beta + (4.0 - 3.0 * beta) * (4.0 - 3.0 * beta) * g1 / (beta + 12.0 * g1 * (1.0 - beta));
}

// Sound speed and internal energy per volume of a primitive state.
template <int EOS>
__host__ __device__ __forceinline__ void thermo_fp64(double r, double p, double g, double &c, double &e) {
#pragma clang fp contract(off)
  if constexpr (EOS == EOS_GAS_RADIATION) {
    const double T = gr_temperature_p(r, p);
    c = __builtin_sqrt(gr_gamma1(r, T, p, g) * p / r);
    e = r * T / (g - 1.0) + ARAD * T * T * T * T;
  } else {
    c = __builtin_sqrt(g * p / r);
    e = p / (g - 1.0);
  }
}

// HLLC flux in the face frame: L, R = (rho, u_normal, u_t1, u_t2, p).  Wave
// speed bounds: Davis, min/max of u -+ c over both sides; or Einfeldt,
// u_bar -+ d_bar with sqrt(rho)-weighted u_bar and d_bar^2 = weighted mean of
// c^2 + s_L s_R / (2 (s_L + s_R)^2) (u_R - u_L)^2 (Toro sec. 10.5.1); or
// pressure-based, u_L - c_L q_L and u_R + c_R q_R with q_K = 1 unless the
// linearised (PVRS) star pressure p* = max(0, (p_L + p_R)/2 - (u_R - u_L)
// rho_bar c_bar / 2) exceeds p_K, then the shock factor
// sqrt(1 + (gamma + 1)/(2 gamma) (p*/p_K - 1)) (Toro sec. 10.5.2).
// The side of the contact is chosen first (left if S_L >= 0 or S* >= 0) and
// only that side's physical flux and star state are formed:
//   F = F_K + S (U*_K - U_K),  S = min(S_L, 0) on the left, max(S_R, 0) on the
// right, which reproduces the four textbook branches (S = 0 gives F_K).
// The star state is written with one reciprocal of (S_K - S*):
//   q = (S_K - u)/(S_K - S*), rho* = rho q,
//   E* = q E + rho* (S* - u) S* + (S* - u) p /(S_K - S*).
// FP32 arithmetic is not contracted by the compiler here: every fused
// multiply-add is written out, so each inlined copy (one per face site)
// rounds alike and identical states give identical fluxes at every site.
template <int SPEEDS>
__device__ __forceinline__ void hllc(const float L[5], const float R[5], float g, float rgm1, float F[5]) {
#pragma clang fp contract(off)
  using A = Arith<float>;
  float SL, SR;
  if constexpr (SPEEDS == SPEEDS_EINFELDT) {
    // Einfeldt: u_bar -+ d_bar with sqrt(rho) weights s_K; c_K^2 = g p_K / rho_K = g p_K (1/s_K)^2
    const float qL = __builtin_amdgcn_rsqf(L[0]), qR = __builtin_amdgcn_rsqf(R[0]);
    const float sL = L[0] * qL, sR = R[0] * qR;
    const float c2L = g * L[4] * qL * qL, c2R = g * R[4] * qR * qR;
    const float is = A::rcp(sL + sR);
    const float ub = __builtin_fmaf(sL, L[1], sR * R[1]) * is;
    const float du = R[1] - L[1];
    const float d2 = __builtin_fmaf(__builtin_fmaf(sL, c2L, sR * c2R), is, 0.5f * sL * sR * is * is * du * du);
    const float d = d2 * __builtin_amdgcn_rsqf(d2);
    SL = ub - d;
    SR = ub + d;
  } else if constexpr (SPEEDS == SPEEDS_PVRS) {
    const float cL = A::sound(g, L[4], L[0]);
    const float cR = A::sound(g, R[4], R[0]);
    // rho_bar c_bar / 2 = (rho_L + rho_R)(c_L + c_R) / 8
    const float ps = fmax(__builtin_fmaf(-0.125f * (R[1] - L[1]) * (L[0] + R[0]), cL + cR, 0.5f * (L[4] + R[4])), 0.0f);
    const float k = __builtin_fmaf(0.5f, A::rcp(g), 0.5f);  // (gamma + 1)/(2 gamma)
    // x_K = 1 + k (p*/p_K - 1) > 1 on the shock branch: q_K = x_K rsqrt(x_K)
    const float xL = __builtin_fmaf(k, __builtin_fmaf(ps, A::rcp(L[4]), -1.0f), 1.0f);
    const float xR = __builtin_fmaf(k, __builtin_fmaf(ps, A::rcp(R[4]), -1.0f), 1.0f);
    const float qL = ps > L[4] ? xL * __builtin_amdgcn_rsqf(xL) : 1.0f;
    const float qR = ps > R[4] ? xR * __builtin_amdgcn_rsqf(xR) : 1.0f;
    SL = __builtin_fmaf(-cL, qL, L[1]);
    SR = __builtin_fmaf(cR, qR, R[1]);
  } else {
    const float cL = A::sound(g, L[4], L[0]);
    const float cR = A::sound(g, R[4], R[0]);
    SL = fmin(L[1] - cL, R[1] - cR);
    SR = fmax(L[1] + cL, R[1] + cR);
  }
  const float aL = L[0] * (SL - L[1]);
  const float aR = R[0] * (SR - R[1]);
  const float Ss = A::div(__builtin_fmaf(-aR, R[1], __builtin_fmaf(aL, L[1], R[4] - L[4])), aL - aR);
  const bool useL = (SL >= 0.0f) || (Ss >= 0.0f);
  const float r = useL ? L[0] : R[0];
  const float u = useL ? L[1] : R[1];
  const float v = useL ? L[2] : R[2];
  const float w = useL ? L[3] : R[3];
  const float p = useL ? L[4] : R[4];
  const float SK = useL ? SL : SR;
  const float S = useL ? fmin(SL, 0.0f) : fmax(SR, 0.0f);
  const float ru = r * u;
  const float E = __builtin_fmaf(p, rgm1, (0.5f * r) * __builtin_fmaf(u, u, __builtin_fmaf(v, v, w * w)));
  const float f0 = ru, f1 = __builtin_fmaf(ru, u, p), f2 = ru * v, f3 = ru * w, f4 = u * (E + p);
  const float inv = A::rcp(SK - Ss);
  const float q = (SK - u) * inv;
  const float a = r * q;
  const float su = Ss - u;
  const float Es = __builtin_fmaf(q, E, __builtin_fmaf(a * su, Ss, su * p * inv));
  const bool star = (S != 0.0f);
  F[0] = star ? __builtin_fmaf(S, a - r, f0) : f0;
  F[1] = star ? __builtin_fmaf(S, __builtin_fmaf(a, Ss, -ru), f1) : f1;
  F[2] = star ? __builtin_fmaf(S, v * (a - r), f2) : f2;
  F[3] = star ? __builtin_fmaf(S, w * (a - r), f3) : f3;
  F[4] = star ? __builtin_fmaf(S, Es - E, f4) : f4;
}

// HLLC in FP64 with the operations in the order of the textbook statement
// (left and right states, Davis, Einfeldt or PVRS speeds, S* from the jump relations, star state
// rho_K (S_K - u)/(S_K - S*) (1, S*, v, w, E/rho + (S* - u)(S* + p/(rho (S_K - u))))),
// no contraction into FMAs.  Division and square root are IEEE-correct on the
// device, so each face flux is rounded exactly as in a plain FP64 CPU
// evaluation of the same formulas.  Only the side K of the contact is formed.
template <int SPEEDS, int EOS = EOS_IDEAL>
__host__ __device__ __forceinline__ void hllc_fp64(const double L[5], const double R[5], double g, double F[5]) {
#pragma clang fp contract(off)
  const double rL = L[0], uL = L[1], vL = L[2], wL = L[3], pL = L[4];
  const double rR = R[0], uR = R[1], vR = R[2], wR = R[3], pR = R[4];
  double cL, cR, eL, eR;  // the ideal-gas energies are not used (E is formed for side K below)
  thermo_fp64<EOS>(rL, pL, g, cL, eL);
  thermo_fp64<EOS>(rR, pR, g, cR, eR);
  double SL, SR;
  if constexpr (SPEEDS == SPEEDS_EINFELDT) {
    const double sL = __builtin_sqrt(rL), sR = __builtin_sqrt(rR);
    const double ubar = (sL * uL + sR * uR) / (sL + sR);
    const double eta2 = 0.5 * sL * sR / ((sL + sR) * (sL + sR));
    const double dbar = __builtin_sqrt((sL * cL * cL + sR * cR * cR) / (sL + sR) + eta2 * (uR - uL) * (uR - uL));
    SL = ubar - dbar;
    SR = ubar + dbar;
  } else if constexpr (SPEEDS == SPEEDS_PVRS) {
    const double rbar = 0.5 * (rL + rR), cbar = 0.5 * (cL + cR);
    const double ps = fmax(0.0, 0.5 * (pL + pR) - 0.5 * (uR - uL) * rbar * cbar);
    const double k = (g + 1.0) / (2.0 * g);
    const double qL = ps <= pL ? 1.0 : __builtin_sqrt(1.0 + k * (ps / pL - 1.0));
    const double qR = ps <= pR ? 1.0 : __builtin_sqrt(1.0 + k * (ps / pR - 1.0));
    SL = uL - cL * qL;
    SR = uR + cR * qR;
  } else {
    SL = fmin(uL - cL, uR - cR);
    SR = fmax(uL + cL, uR + cR);
  }
  const double Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) / (rL * (SL - uL) - rR * (SR - uR));
  const bool useL = (0.0 <= SL) || (0.0 <= Ss);
  const double r = useL ? rL : rR, u = useL ? uL : uR, v = useL ? vL : vR, w = useL ? wL : wR, p = useL ? pL : pR;
  const double SK = useL ? SL : SR;
  const bool star = useL ? !(0.0 <= SL) : (0.0 < SR);
  const double eK = (EOS == EOS_GAS_RADIATION) ? (useL ? eL : eR) : p / (g - 1.0);
  const double E = eK + 0.5 * r * (u * u + v * v + w * w);
  const double FK[5] = {r * u, r * u * u + p, r * u * v, r * u * w, u * (E + p)};
  const double UK[5] = {r, r * u, r * v, r * w, E};
  const double a = r * (SK - u) / (SK - Ss);
  const double Us[5] = {a, a * Ss, a * v, a * w, a * (E / r + (Ss - u) * (Ss + p / (r * (SK - u))))};
#pragma unroll
  for (int k = 0; k < 5; ++k) F[k] = star ? FK[k] + SK * (Us[k] - UK[k]) : FK[k];
}

// Characteristic limiting in FP64 (Toro 2009, ch. 3), in the face frame
// (normal velocity in slot 1): the one-sided differences da, db of cell W
// are split into the amplitudes of the waves u - c, entropy, two shear
// waves, u + c (left eigenvectors at W, impedance rho c):
//   a_- = (d_p - rho c d_u)/(2 c^2), a_0 = d_rho - d_p/c^2, a_t = d_t,
//   a_+ = (d_p + rho c d_u)/(2 c^2);
// each is limited by minmod and the slope rebuilt from the right
// eigenvectors: d_rho = m_- + m_0 + m_+, d_u = (c/rho)(m_+ - m_-),
// d_t = m_t, d_p = c^2 (m_- + m_+).  Operation order of the plain
// statement, no contraction (IEEE division and square root).
__device__ __forceinline__ void char_slope_fp64(const double W[5], const double da[5], const double db[5], double g,
                                                double s[5]) {
#pragma clang fp contract(off)
  const double c = __builtin_sqrt(g * W[4] / W[0]);
  const double rc = W[0] * c, c2 = c * c;
  const double am = minmod((da[4] - rc * da[1]) / (2.0 * c2), (db[4] - rc * db[1]) / (2.0 * c2));
  const double a0 = minmod(da[0] - da[4] / c2, db[0] - db[4] / c2);
  const double at1 = minmod(da[2], db[2]);
  const double at2 = minmod(da[3], db[3]);
  const double ap = minmod((da[4] + rc * da[1]) / (2.0 * c2), (db[4] + rc * db[1]) / (2.0 * c2));
  s[0] = am + a0 + ap;
  s[1] = (c / W[0]) * (ap - am);
  s[2] = at1;
  s[3] = at2;
  s[4] = c2 * (am + ap);
}

// Face states between cells 1 and 2 of four cells w (face frame) with
// characteristic limiting: left W_1 + slope_1/2, right W_2 - slope_2/2.
__device__ __forceinline__ void char_states_fp64(const double (&w)[4][5], double g, double L[5], double R[5]) {
#pragma clang fp contract(off)
  double d01[5], d12[5], d23[5], s1[5], s2[5];
#pragma unroll
  for (int v = 0; v < NVAR; ++v) {
    d01[v] = w[1][v] - w[0][v];
    d12[v] = w[2][v] - w[1][v];
    d23[v] = w[3][v] - w[2][v];
  }
  char_slope_fp64(w[1], d01, d12, g, s1);
  char_slope_fp64(w[2], d12, d23, g, s2);
#pragma unroll
  for (int v = 0; v < NVAR; ++v) {
    L[v] = w[1][v] + 0.5 * s1[v];
    R[v] = w[2][v] - 0.5 * s2[v];
  }
}

// A reconstructed face state is physical: rho > 0, p > 0, all finite.
__device__ __forceinline__ bool state_ok(const double s[5]) {
  const double m = fabs(s[1]) + fabs(s[2]) + fabs(s[3]) + s[4] + s[0];
  return (s[0] > 0.0) && (s[4] > 0.0) && (m < __builtin_huge_val());
}

// FP64 primitive recovery (ideal gas), in the plain evaluation order
// u = m/rho; rho e = E - (m_x u + m_y v + m_z w)/2; p = (gamma-1) rho e.
// Returns false for rho <= 0, p <= 0 or non-finite values.
__host__ __device__ __forceinline__ bool recover(double U0, double U1, double U2, double U3, double U4, double gm1,
                                        double W[5]) {
#pragma clang fp contract(off)
  const double u = U1 / U0, v = U2 / U0, w = U3 / U0;
  const double rhoe = U4 - 0.5 * (U1 * u + U2 * v + U3 * w);
  const double p = gm1 * rhoe;
  W[0] = U0;
  W[1] = u;
  W[2] = v;
  W[3] = w;
  W[4] = p;
  const double s = fabs(u) + fabs(v) + fabs(w) + p + U0;
  return (U0 > 0.0) && (p > 0.0) && (s < __builtin_huge_val());
}

// 1/x in FP64 from the hardware reciprocal estimate refined by two Newton
// steps (about 1 ulp for normal x; no denormal or overflow scaling).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return r;
}

// Faster recovery for the mixed path (one refined reciprocal); its primitives
// are rounded to FP32 right after, while rho e = E - m.u/2 keeps FP64.
__device__ __forceinline__ bool recover_fast(double U0, double U1, double U2, double U3, double U4, double gm1,
                                             double W[5]) {
#pragma clang fp contract(off)
  const double inv = rcp_nr(U0);
  const double u = U1 * inv, v = U2 * inv, w = U3 * inv;
  const double rhoe = __builtin_fma(-0.5, __builtin_fma(U1, u, __builtin_fma(U2, v, U3 * w)), U4);
  const double p = gm1 * rhoe;
  W[0] = U0;
  W[1] = u;
  W[2] = v;
  W[3] = w;
  W[4] = p;
  const double s = fabs(u) + fabs(v) + fabs(w) + p + U0;
  return (U0 > 0.0) && (p > 0.0) && (s < __builtin_huge_val());
}

// Recovery under either EOS (the gamma law is `recover`).  Gas + radiation:
// p from the temperature of rho e = E - m.u/2; a state with rho e <= 0 has
// no temperature and keeps p = rho e, which the check reports.
template <int EOS>
__device__ __forceinline__ bool recover_eos(double U0, double U1, double U2, double U3, double U4, double gamma,
                                            double W[5]) {
#pragma clang fp contract(off)
  if constexpr (EOS == EOS_IDEAL) {
    return recover(U0, U1, U2, U3, U4, gamma - 1.0, W);
  } else {
    const double u = U1 / U0, v = U2 / U0, w = U3 / U0;
    const double rhoe = U4 - 0.5 * (U1 * u + U2 * v + U3 * w);
    double p = rhoe;
    if (rhoe > 0.0) {
      const double T = gr_temperature_e(U0, rhoe, gamma);
      p = U0 * T + ARAD * T * T * T * T / 3.0;
    }
    W[0] = U0;
    W[1] = u;
    W[2] = v;
    W[3] = w;
    W[4] = p;
    const double s = fabs(u) + fabs(v) + fabs(w) + p + U0;
    return (U0 > 0.0) && (p > 0.0) && (s < __builtin_huge_val());
  }
}

template <int EOS>
__device__ __forceinline__ bool load_prim(const double *__restrict__ p, int64_t vs, double gamma, double W[5]) {
  return recover_eos<EOS>(p[0], p[vs], p[2 * vs], p[3 * vs], p[4 * vs], gamma, W);
}

// CFL rate of one cell, sum over active directions of (|u_d| + c)/dx_d.
template <int DIM, int EOS = EOS_IDEAL>
__host__ __device__ __forceinline__ double cell_rate(const double W[5], double gamma, double dx0, double dx1, double dx2) {
#pragma clang fp contract(off)
  double c, e;
  thermo_fp64<EOS>(W[0], W[4], gamma, c, e);
  double lam = 0.0;
  lam += (fabs(W[1]) + c) / dx0;
  lam += (fabs(W[2]) + c) / dx1;
  if (DIM == 3) lam += (fabs(W[3]) + c) / dx2;
  return lam;
}

// CFL rate of one cell on the mixed path, from primitives recovered by
// recover_fast: c = g p / sqrt(g p rho) with the hardware reciprocal square
// root refined by one Newton step, and the reciprocal cell widths rdx_d.
// Both the stage-2 epilogue and the mixed rate kernel use it, so a mixed run
// reduces the same rate whether dt comes from the previous step's stage 2 or
// from a fresh reduction (a run resumed from a saved state repeats the
// uninterrupted run bit for bit).
template <int DIM>
__device__ __forceinline__ double cell_rate_fast(const double W[5], double gamma, double rdx0, double rdx1,
                                                 double rdx2) {
#pragma clang fp contract(off)
  const double gp = gamma * W[4], q = gp * W[0];
  double y = __builtin_amdgcn_rsq(q);
  y = y * __builtin_fma(-0.5 * q * y, y, 1.5);
  const double cs = gp * y;
  double l = __builtin_fma(fabs(W[1]) + cs, rdx0, (fabs(W[2]) + cs) * rdx1);
  if (DIM == 3) l = __builtin_fma(fabs(W[3]) + cs, rdx2, l);
  return l;
}

// Source of an out-of-block cell along one axis: face f's source block and
// the coordinate along the axis inside it.  `c` is -2, -1 (low face) or
// n, n+1 (high face).
__device__ __forceinline__ int guard_coord(const DevBlock *__restrict__ B, int f, int c, int n) {
  const bool high = f & 1;
  if (B->fmode[f]) return high ? n - 1 : 0;    // outflow: edge layer repeated
  return high ? c - n : B->fnax[f] + c;        // wrap: far layers of the source
}

// Element offset of variable 0 and variable stride of cell (x, y, z) of block
// B, at most one coordinate outside the block.
__device__ __forceinline__ void cell_addr(const DevBlock *__restrict__ B, int x, int y, int z, int64_t &off,
                                          int64_t &vs) {
  const int nx = B->n[0], ny = B->n[1], nz = B->n[2];
  if (x < 0 || x >= nx) {
    const int f = x < 0 ? 0 : 1;
    const int xs = guard_coord(B, f, x, nx);
    const int nax = B->fmode[f] ? nx : B->fnax[f];
    off = B->foff[f] + ((int64_t)z * ny + y) * nax + xs;
    vs = B->fmode[f] ? B->ncell : B->fnc[f];
  } else if (y < 0 || y >= ny) {
    const int f = y < 0 ? 2 : 3;
    const int ys = guard_coord(B, f, y, ny);
    const int nay = B->fmode[f] ? ny : B->fnax[f];
    off = B->foff[f] + ((int64_t)z * nay + ys) * nx + x;
    vs = B->fmode[f] ? B->ncell : B->fnc[f];
  } else if (z < 0 || z >= nz) {
    const int f = z < 0 ? 4 : 5;
    const int zs = guard_coord(B, f, z, nz);
    off = B->foff[f] + ((int64_t)zs * ny + y) * nx + x;
    vs = B->fmode[f] ? B->ncell : B->fnc[f];
  } else {
    off = B->off + ((int64_t)z * ny + y) * nx + x;
    vs = B->ncell;
  }
}

template <int TX, int TY>
struct TileGeom {
  static constexpr int NT = TX * TY;           // threads per tile
  static constexpr int PX = TX + 4, PY = TY + 4;
  static constexpr int PP = PX * PY;           // padded plane (corners unused)
  static constexpr int NXF = (TX + 1) * TY;    // x faces of a plane
  static constexpr int NYF = TX * (TY + 1);    // y faces of a plane
  static constexpr int ELEMS = NVAR * (PP + NXF + NYF);
};

template <int TX, int TY, int NSUB, typename T>
constexpr size_t tile_lds_bytes() {
  return (size_t)NSUB * TileGeom<TX, TY>::ELEMS * sizeof(T);
}

// Per-thread geometry of one tile of a work item: the block, the thread's
// column, dt/dx, and the guard cell this thread gathers for every plane.
struct TileCtx {
  int b;
  bool active;
  const DevBlock *Bp;
  int x, y, z0, z1, nz, ncell;
  double dtdx, dtdy, dtdz, dx0, dx1, dx2;
  int64_t plane, boff, cidx;
  int gslot;                 // LDS slot (in a [PY][PX] plane) of this thread's guard cell, -1: none
  int64_t goff, gvs, gps;    // guard source: offset at z = 0, variable stride, z-plane stride
};

// Threads [0, 4TY) gather the x guards (side, layer, row), threads
// [4TY, 4TY+4TX) the y guards; the assignment is fixed for the whole column.
template <int TX, int TY, int DIM>
__device__ __forceinline__ void tile_setup(TileCtx &C, const StageArgs &A, const WorkItem *__restrict__ it, int sub,
                                           int lt, double dt, int PX) {
  const int ti = lt % TX, tj = lt / TX;
  C.b = __builtin_amdgcn_readfirstlane(it->block[sub]);  // uniform across the tile's waves
  C.active = C.b >= 0;
  C.Bp = A.blocks + (C.active ? C.b : 0);
  const int x0 = C.active ? __builtin_amdgcn_readfirstlane(it->x0[sub]) : 0;
  const int y0 = C.active ? __builtin_amdgcn_readfirstlane(it->y0[sub]) : 0;
  C.x = x0 + ti;
  C.y = y0 + tj;
  C.z0 = it->z0;
  C.z1 = it->z1;
  C.dtdx = C.dtdy = C.dtdz = 0.0;
  C.dx0 = C.dx1 = C.dx2 = 1.0;
  int nx = 1, ny = 1;
  C.nz = 1;
  C.ncell = 1;
  C.plane = 1;
  C.boff = 0;
  if (C.active) {
    nx = C.Bp->n[0];
    ny = C.Bp->n[1];
    C.nz = C.Bp->n[2];
    C.ncell = C.Bp->ncell;
    C.boff = C.Bp->off;
    C.plane = (int64_t)nx * ny;
    C.dx0 = C.Bp->dx[0];
    C.dx1 = C.Bp->dx[1];
    C.dx2 = C.Bp->dx[2];
    C.dtdx = dt / C.dx0;
    C.dtdy = dt / C.dx1;
    if (DIM == 3) C.dtdz = dt / C.dx2;
  }
  C.cidx = (int64_t)C.y * nx + C.x;
  C.gslot = -1;
  C.goff = C.gvs = C.gps = 0;
  if (C.active && lt < 4 * (TX + TY)) {
    int gx, gy;
    if (lt < 4 * TY) {
      const int side = lt / (2 * TY), r = lt % (2 * TY), layer = r / TY + 1, row = r % TY;
      gx = side ? TX + layer - 1 : -layer;
      gy = row;
    } else {
      const int l2 = lt - 4 * TY;
      const int side = l2 / (2 * TX), r = l2 % (2 * TX), layer = r / TX + 1, col = r % TX;
      gx = col;
      gy = side ? TY + layer - 1 : -layer;
    }
    C.gslot = (gy + 2) * PX + (gx + 2);
    const int X = x0 + gx, Y = y0 + gy;
    cell_addr(C.Bp, X, Y, 0, C.goff, C.gvs);
    int64_t o1, v1;
    cell_addr(C.Bp, X, Y, DIM == 3 ? 1 : 0, o1, v1);
    C.gps = o1 - C.goff;  // the source block's z-plane stride (same block for every z)
  }
}

// ------------------------------------------------------------------------
// One work item: NSUB tiles of TX x TY cells (one tile per NT threads),
// marched over z planes [z0, z1).
// ------------------------------------------------------------------------
template <int TX, int TY, int NSUB, int DIM, int STAGE, int SPEEDS, int RECON, int EOS>
__device__ __forceinline__ void run_tile(const StageArgs &A, const WorkItem *__restrict__ it, unsigned char *lds,
                                         int slot, double dt, double &lam, int &bad, int &badblk) {
  using T = double;
  using G = TileGeom<TX, TY>;
  constexpr int NT = G::NT, PX = G::PX, PP = G::PP, NXF = G::NXF, NYF = G::NYF;
  static_assert(NT * NSUB == WG, "tile threads must fill the workgroup");
  static_assert(4 * (TX + TY) <= NT, "guard ring must fit the tile's threads");

  const int tid = threadIdx.x;
  // a tile is NT/64 whole waves, so `sub` is wave-uniform: make it scalar
  const int sub = (NSUB == 1) ? 0 : __builtin_amdgcn_readfirstlane(tid / NT);
  const int lt = tid - sub * NT;
  const int ti = lt % TX, tj = lt / TX;
  T *Wp = reinterpret_cast<T *>(lds) + sub * G::ELEMS;  // [5][PY][PX] primitives of the current plane
  T *Fx = Wp + NVAR * PP;                                // [5][TY][TX+1]
  T *Fy = Fx + NVAR * NXF;                               // [5][TY+1][TX]

  TileCtx C;
  tile_setup<TX, TY, DIM>(C, A, it, NSUB == 1 ? slot : sub, lt, dt, PX);
  const int b = C.b;
  const bool active = (NSUB == 1) ? true : C.active;  // a 16x16 item always names a block
  const DevBlock *__restrict__ Bp = C.Bp;
  const int x = C.x, y = C.y, z0 = C.z0, z1 = C.z1;
  const double gamma = A.gamma, gm1 = gamma - 1.0;
  const double dtdx = C.dtdx, dtdy = C.dtdy, dtdz = C.dtdz, dx0 = C.dx0, dx1 = C.dx1, dx2 = C.dx2;
  const int nz = C.nz, ncell = C.ncell;
  const int64_t plane = C.plane, boff = C.boff, cidx = C.cidx;
  const int gslot = C.gslot;
  const int64_t goff = C.goff, gvs = C.gvs, gps = C.gps;

  const double *__restrict__ src = A.src;
  const int64_t own_vs = ncell;
  const double *__restrict__ own = src + boff + cidx;

  // Global loads are issued early and consumed late, as in the mixed tile:
  // own cell of plane j+2 and (stage 2) Un of plane j at the top of the
  // iteration for plane j, the guard cell of plane j+1 right after staging
  // plane j.  The arithmetic and its order are unchanged by the pipeline.
  auto fetch = [&](const double *p, int64_t vs, double (&U)[5]) {
#pragma unroll
    for (int v = 0; v < NVAR; ++v) U[v] = p[v * vs];
  };
  // the variables PLM reconstructs (primitives, or the conserved values
  // themselves); the cell's primitives are recovered either way, as the
  // check for a non-physical cell
  auto prims = [&](const double (&U)[5], T (&W)[5], bool own) {
    double Wd[5];
    if (!recover_eos<EOS>(U[0], U[1], U[2], U[3], U[4], gamma, Wd)) {
      bad = 1;
      if (own) badblk = min(badblk, b);
    }
#pragma unroll
    for (int v = 0; v < NVAR; ++v) W[v] = (RECON == RECON_CONSERVED) ? U[v] : Wd[v];
  };
  // conserved reconstruction: recover a face state (same formulas, FP64),
  // which must be physical too
  auto face_prims = [&](T (&s)[5]) {
    if constexpr (RECON == RECON_CONSERVED) {
      double Wd[5];
      if (!recover(s[0], s[1], s[2], s[3], s[4], gm1, Wd) && active) {
        bad = 1;
        badblk = min(badblk, b);
      }
#pragma unroll
      for (int v = 0; v < NVAR; ++v) s[v] = Wd[v];
    }
  };
  auto fetch_guard = [&](int z, double (&G)[5]) {
    if (gslot >= 0) fetch(src + goff + (int64_t)z * gps, gvs, G);
  };
  auto fetch_un = [&](int z, double (&Un)[5]) {
    if (STAGE == 2 && active) {  // Un is read once, pointwise: streamed in
      const double *p = A.un + boff + (int64_t)z * plane + cidx;
#pragma unroll
      for (int v = 0; v < NVAR; ++v) Un[v] = __builtin_nontemporal_load(&p[v * own_vs]);
    }
  };

  // stage the x/y guard ring and this thread's cell of the plane into LDS
  auto stage_plane = [&](const T (&Wc)[5], const double (&Gr)[5]) {
    if (active) {
#pragma unroll
      for (int v = 0; v < NVAR; ++v) Wp[v * PP + (tj + 2) * PX + (ti + 2)] = Wc[v];
    }
    if (gslot >= 0) {
      T Wg[5];
      prims(Gr, Wg, false);
#pragma unroll
      for (int v = 0; v < NVAR; ++v) Wp[v * PP + gslot] = Wg[v];
    }
  };

  // x and y faces of the plane in LDS, each computed once
  auto plane_faces = [&]() {
    for (int f = lt; f < NXF + NYF; f += NT) {
      const bool isx = f < NXF;
      const int g = isx ? f : f - NXF;
      int base, stride;
      T *out;
      int ostride;
      if (isx) {
        const int row = g / (TX + 1), col = g % (TX + 1);
        base = (row + 2) * PX + col;
        stride = 1;
        out = Fx + row * (TX + 1) + col;
        ostride = NXF;
      } else {
        const int row = g / TX, col = g % TX;
        base = row * PX + (col + 2);
        stride = PX;
        out = Fy + row * TX + col;
        ostride = NYF;
      }
      T Lr[5], Rr[5];
      if constexpr (RECON == RECON_CHARACTERISTIC) {
        T w[4][5];  // the four cells in the face frame
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const T *p = Wp + base + k * stride;
          w[k][0] = p[0];
          w[k][1] = isx ? p[PP] : p[2 * PP];
          w[k][2] = isx ? p[2 * PP] : p[PP];
          w[k][3] = p[3 * PP];
          w[k][4] = p[4 * PP];
        }
        char_states_fp64(w, gamma, Lr, Rr);
        if (!(state_ok(Lr) && state_ok(Rr)) && active) {
          bad = 1;
          badblk = min(badblk, b);
        }
      } else {
        T wl[5], wr[5];
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
          const T *p = Wp + v * PP + base;
          plm(p[0], p[stride], p[2 * stride], p[3 * stride], wl[v], wr[v]);
        }
        face_prims(wl);
        face_prims(wr);
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
          Lr[v] = wl[v];
          Rr[v] = wr[v];
        }
        Lr[1] = isx ? wl[1] : wl[2];
        Lr[2] = isx ? wl[2] : wl[1];
        Rr[1] = isx ? wr[1] : wr[2];
        Rr[2] = isx ? wr[2] : wr[1];
      }
      T Fr[5];
      hllc_fp64<SPEEDS, EOS>(Lr, Rr, gamma, Fr);
      out[0] = Fr[0];
      out[ostride] = isx ? Fr[1] : Fr[2];
      out[2 * ostride] = isx ? Fr[2] : Fr[1];
      out[3 * ostride] = Fr[3];
      out[4 * ostride] = Fr[4];
    }
  };

  // RK stage update of this thread's cell in plane z:
  //   dU = sum over x, y, z of (dt/dx_d)(F_lo - F_hi), FP64, no contraction;
  //   stage 1: U1 = Un + dU;  stage 2: Un+1 = Un/2 + (U1 + dU)/2.
  auto update = [&](int z, const double (&Us)[5], const double (&Un)[5], const T (&fzlo)[5], const T (&fzhi)[5]) {
#pragma clang fp contract(off)
    if (!active) return;
    const int64_t c = (int64_t)z * plane;
    double Unew[5];
#pragma unroll
    for (int v = 0; v < NVAR; ++v) {
      const double fxl = (double)Fx[v * NXF + tj * (TX + 1) + ti];
      const double fxh = (double)Fx[v * NXF + tj * (TX + 1) + ti + 1];
      const double fyl = (double)Fy[v * NYF + tj * TX + ti];
      const double fyh = (double)Fy[v * NYF + (tj + 1) * TX + ti];
      double dU = dtdx * (fxl - fxh);
      dU += dtdy * (fyl - fyh);
      if (DIM == 3) dU += dtdz * ((double)fzlo[v] - (double)fzhi[v]);
      Unew[v] = (STAGE == 1) ? Us[v] + dU : 0.5 * Un[v] + 0.5 * (Us[v] + dU);
      __builtin_nontemporal_store(Unew[v], &A.dst[boff + v * own_vs + c + cidx]);  // streamed out
    }
    if (STAGE == 2) {  // CFL rate of the new state (FP64)
      double W[5];
      if (!recover_eos<EOS>(Unew[0], Unew[1], Unew[2], Unew[3], Unew[4], gamma, W)) {
        bad = 1;
        badblk = min(badblk, b);
      } else {
        lam = fmax(lam, cell_rate<DIM, EOS>(W, gamma, dx0, dx1, dx2));
      }
    }
  };

  double Gr[5] = {0, 0, 0, 0, 0}, Un[5] = {0, 0, 0, 0, 0};
  if (DIM == 2) {
    double U[5] = {1, 0, 0, 0, 1};
    T Wc[5] = {1, 0, 0, 0, 1};
    if (active) fetch(own, own_vs, U);
    fetch_guard(0, Gr);
    fetch_un(0, Un);
    if (active) prims(U, Wc, true);
    stage_plane(Wc, Gr);
    __syncthreads();
    plane_faces();
    __syncthreads();
    const T zero[5] = {0, 0, 0, 0, 0};
    update(0, U, Un, zero, zero);
    return;
  }

  // ---- 3D: z march with a four-plane register window of primitives and a
  // three-plane ring of the conserved source values, so no source cell is
  // read twice.  At iteration j the window holds planes (j-1, j, j+1) and
  // receives j+2; the z face j+1/2 is computed at a single site for every
  // face of the column (the prologue iteration j = z0-1 yields the face z0-1/2).
  T Wa[5] = {1, 0, 0, 0, 1}, Wb[5] = {1, 0, 0, 0, 1}, Wc[5] = {1, 0, 0, 0, 1}, Wd[5] = {1, 0, 0, 0, 1};
  double Ub[5] = {0, 0, 0, 0, 0}, Uc[5] = {0, 0, 0, 0, 0}, Ud[5] = {0, 0, 0, 0, 0};  // planes j, j+1, j+2
  auto fetch_z = [&](int z, double (&U)[5]) {
    if (!active) return;
    int64_t off, vs;
    if (z >= 0 && z < nz) {
      off = boff + (int64_t)z * plane + cidx;
      vs = own_vs;
    } else {
      cell_addr(Bp, x, y, z, off, vs);
    }
    fetch(src + off, vs, U);
  };
  fetch_z(z0 - 2, Ud);
  fetch_z(z0 - 1, Ub);
  fetch_z(z0, Uc);
  fetch_guard(z0, Gr);
  if (active) {
    prims(Ud, Wa, true);
    prims(Ub, Wb, true);
    prims(Uc, Wc, true);
  }
  T fzlo[5] = {0, 0, 0, 0, 0};
  for (int j = z0 - 1; j < z1; ++j) {
    const bool work = j >= z0;
    fetch_z(j + 2, Ud);
    if (work) {
      fetch_un(j, Un);
      stage_plane(Wb, Gr);
      if (j + 1 < z1) fetch_guard(j + 1, Gr);
      __syncthreads();
      plane_faces();
    }
    if (active) prims(Ud, Wd, true);
    T fz[5];
    {
      T Lr[5], Rr[5];
      if constexpr (RECON == RECON_CHARACTERISTIC) {
        const T w[4][5] = {{Wa[0], Wa[3], Wa[2], Wa[1], Wa[4]},
                           {Wb[0], Wb[3], Wb[2], Wb[1], Wb[4]},
                           {Wc[0], Wc[3], Wc[2], Wc[1], Wc[4]},
                           {Wd[0], Wd[3], Wd[2], Wd[1], Wd[4]}};
        char_states_fp64(w, gamma, Lr, Rr);
        if (!(state_ok(Lr) && state_ok(Rr)) && active) {
          bad = 1;
          badblk = min(badblk, b);
        }
      } else {
        T wl[5], wr[5];
#pragma unroll
        for (int v = 0; v < NVAR; ++v) plm(Wa[v], Wb[v], Wc[v], Wd[v], wl[v], wr[v]);
        face_prims(wl);
        face_prims(wr);
        const T l[5] = {wl[0], wl[3], wl[2], wl[1], wl[4]};
        const T r[5] = {wr[0], wr[3], wr[2], wr[1], wr[4]};
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
          Lr[v] = l[v];
          Rr[v] = r[v];
        }
      }
      T Fr[5];
      hllc_fp64<SPEEDS, EOS>(Lr, Rr, gamma, Fr);
      fz[0] = Fr[0];
      fz[1] = Fr[3];
      fz[2] = Fr[2];
      fz[3] = Fr[1];
      fz[4] = Fr[4];
    }
    if (work) {
      __syncthreads();
      update(j, Ub, Un, fzlo, fz);
    }
#pragma unroll
    for (int v = 0; v < NVAR; ++v) {
      fzlo[v] = fz[v];
      Wa[v] = Wb[v];
      Wb[v] = Wc[v];
      Wc[v] = Wd[v];
      Ub[v] = Uc[v];
      Uc[v] = Ud[v];
    }
  }
}

// ------------------------------------------------------------------------
// Mixed-precision tile (FP32 PLM + HLLC).
//
// Per z plane j:  A) stage the plane's primitives and x/y guard ring in LDS;
// B) each face job reads the four primitives along its axis, forms the two
// PLM states of the face and runs HLLC; C) update.  Two barriers per plane.
// The z faces are formed in registers: the z slope of each cell is carried
// down the column (one minmod per cell per plane).
// Face states at cell i along an axis: plus = W_i + D_i/2 (left state of face
// i+1/2), minus = W_i - D_i/2 (right state of face i-1/2), D_i =
// minmod(W_i - W_{i-1}, W_{i+1} - W_i).
// ------------------------------------------------------------------------

// minmod in FP32 as the median of (a, b, 0): one v_med3_f32.
__device__ __forceinline__ float minmod_f(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, 0.0f);
}

// Characteristic limiting in FP32 (the FP64 statement above, with hardware
// reciprocals): slope s of cell W (primitives, x, y, z frame) from its
// one-sided differences da, db, along the axis whose velocity is slot N.
template <int N>
__device__ __forceinline__ void char_slope_f32(const float W[5], const float da[5], const float db[5], float g,
                                               float s[5]) {
#pragma clang fp contract(off)
  const float c = Arith<float>::sound(g, W[4], W[0]);
  const float rc = W[0] * c, c2 = c * c;
  const float ic2 = __builtin_amdgcn_rcpf(c2), h = 0.5f * ic2;  // 1/c^2, 1/(2 c^2)
  const float am = minmod_f(__builtin_fmaf(-rc, da[N], da[4]) * h, __builtin_fmaf(-rc, db[N], db[4]) * h);
  const float ap = minmod_f(__builtin_fmaf(rc, da[N], da[4]) * h, __builtin_fmaf(rc, db[N], db[4]) * h);
  const float a0 = minmod_f(__builtin_fmaf(-ic2, da[4], da[0]), __builtin_fmaf(-ic2, db[4], db[0]));
  s[0] = am + a0 + ap;
  s[4] = c2 * (am + ap);
#pragma unroll
  for (int k = 1; k <= 3; ++k)
    s[k] = (k == N) ? (c * __builtin_amdgcn_rcpf(W[0])) * (ap - am) : minmod_f(da[k], db[k]);
}

// LDS layout of the mixed tile, per variable: the plane's primitives with
// their two-cell x/y guard ring [TX+4 rows][TX+4] (corners unused), then the
// x fluxes (faces 0..TX-1 of each row [row][face], then face TX [row]) and
// the y fluxes [face 0..TX][x].
// A value that is the same on every lane of the wave, kept in scalar
// registers (the compiler cannot see the uniformity through the loads).
__device__ __forceinline__ double wave_uniform(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ int64_t wave_uniform(int64_t x) {
  const int lo = __builtin_amdgcn_readfirstlane((int)x), hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
  return ((int64_t)hi << 32) | (uint32_t)lo;
}

template <int TX>
struct SplitGeom {
  static constexpr int NT = TX * TX;
  static constexpr int PX = TX + 4;
  static constexpr int PP = PX * PX;
  static constexpr int NF = (TX + 1) * TX;  // faces per direction
  static constexpr int OW = 0;
  static constexpr int OFX = OW + NVAR * PP;
  static constexpr int OFY = OFX + NVAR * NF;
  static constexpr int ELEMS = OFY + NVAR * NF;
};

template <int TX, int NSUB, int DIM, int STAGE, int SPEEDS, int RECON>
__device__ __forceinline__ void run_tile_mixed(const StageArgs &A, const WorkItem *__restrict__ it, unsigned char *lds,
                                               int slot, double dt, double &lam, int &bad, int &badblk) {
  // No automatic contraction: the fused operations are written out, so the
  // face code inlined at each face site rounds alike (a uniform state stays
  // fixed bitwise) and the result does not hinge on the compiler's choices.
#pragma clang fp contract(off)
  using G = SplitGeom<TX>;
  constexpr int NT = G::NT, PX = G::PX, PP = G::PP, NF = G::NF;
  static_assert(NT * NSUB == WG, "tile threads must fill the workgroup");
  static_assert(8 * TX <= NT, "guard ring must fit the tile's threads");

  const int tid = threadIdx.x;
  const int sub = (NSUB == 1) ? 0 : __builtin_amdgcn_readfirstlane(tid / NT);
  const int lt = tid - sub * NT;
  const int ti = lt % TX, tj = lt / TX;
  float *L = reinterpret_cast<float *>(lds) + sub * G::ELEMS;

  TileCtx C;
  tile_setup<TX, TX, DIM>(C, A, it, NSUB == 1 ? slot : sub, lt, dt, PX);
  auto uniform_ctx = [&]() {
  if (NSUB == 1) {  // one block per tile: its scalars are wave-uniform
    C.boff = wave_uniform(C.boff);
    C.plane = wave_uniform(C.plane);
    C.ncell = __builtin_amdgcn_readfirstlane(C.ncell);
    C.nz = __builtin_amdgcn_readfirstlane(C.nz);
    C.dtdx = wave_uniform(C.dtdx);
    C.dtdy = wave_uniform(C.dtdy);
    C.dtdz = wave_uniform(C.dtdz);
  }
  };
  uniform_ctx();
  // a 16x16 item always names a block: the flag is a constant there
  const bool active = (NSUB == 1) ? true : C.active;
  const double gamma = A.gamma, gm1 = gamma - 1.0;
  const float g32 = (float)gamma, rgm1 = (float)(1.0 / gm1);
  const double *__restrict__ src = A.src;

  // LDS slot of this thread's cell and of its second x flux
  const int cw = (tj + 2) * PX + (ti + 2);
  const int fx1 = (ti + 1 < TX) ? tj * TX + ti + 1 : TX * TX + tj;

  // Face jobs of this thread, the same for every plane: job 0 is an x face,
  // job 1 a y face, job 2 (threads < 2 TX) one of the TX x and TX y faces
  // left over.  A job names the slot of the first of the four cells along
  // its axis whose primitives give the face's two PLM states, and the slot
  // of its flux.
  static_assert(NF - NT == TX, "one leftover row of faces per direction");
  auto xjob = [&](int f, int &wb, int &o) {  // x face `col` of row `row`: cells col-2 .. col+1
    const int row = f / (TX + 1), col = f % (TX + 1);
    wb = G::OW + (row + 2) * PX + col;
    o = G::OFX + (col < TX ? row * TX + col : TX * TX + row);
  };
  auto yjob = [&](int g, int &wb, int &o) {  // y face `row` of column `col`: cells row-2 .. row+1
    const int row = g / TX, col = g % TX;
    wb = G::OW + row * PX + col + 2;
    o = G::OFY + row * TX + col;
  };
  int jw0, jo0, jw1, jo1, jw2 = 0, jo2 = 0;
  xjob(lt, jw0, jo0);
  yjob(lt, jw1, jo1);
  const bool has2 = lt < 2 * TX, x2 = lt < TX;
  if (has2) {
    if (x2)
      xjob(NT + lt, jw2, jo2);
    else
      yjob(NT + lt - TX, jw2, jo2);
  }

  // Global loads are issued early and consumed late (software pipeline):
  // at the top of the iteration for plane j the thread issues its own cell of
  // plane j+2 (and, in stage 2, Un of plane j); right after staging plane j it
  // issues its guard cell of plane j+1.  Their latency is covered by the LDS
  // phases of plane j.
  auto fetch = [&](const double *p, int64_t vs, double (&U)[5]) {
#pragma unroll
    for (int v = 0; v < NVAR; ++v) U[v] = p[v * vs];
  };
  // the variables PLM reconstructs, rounded to FP32: the primitives, or the
  // conserved values themselves; the cell is recovered in FP64 either way,
  // as the check for a non-physical cell
  auto prims = [&](const double (&U)[5], float (&W)[5], bool own) {
    double Wd[5];
    if (!recover_fast(U[0], U[1], U[2], U[3], U[4], gm1, Wd)) {
      bad = 1;
      if (own) badblk = min(badblk, C.b);
    }
#pragma unroll
    for (int v = 0; v < NVAR; ++v) W[v] = (float)((RECON == RECON_CONSERVED) ? U[v] : Wd[v]);
  };
  // conserved reconstruction: recover a face state in FP32 (the precision of
  // the reconstruction), which must be physical too.  The fused operations are
  // spelled out so that every face site rounds alike (identical states must
  // give identical fluxes for a uniform state to stay fixed bitwise).
  const float gm1f = (float)gm1;
  auto face_prims = [&](float (&s)[5]) {
    if constexpr (RECON == RECON_CONSERVED) {
      const float inv = __builtin_amdgcn_rcpf(s[0]);
      const float u = s[1] * inv, v = s[2] * inv, w = s[3] * inv;
      const float ke = __builtin_fmaf(s[1], u, __builtin_fmaf(s[2], v, s[3] * w));
      const float p = gm1f * __builtin_fmaf(-0.5f, ke, s[4]);
      if (!(s[0] > 0.0f && p > 0.0f) && active) {  // a NaN fails both tests
        bad = 1;
        badblk = min(badblk, C.b);
      }
      s[1] = u;
      s[2] = v;
      s[3] = w;
      s[4] = p;
    }
  };
  auto fetch_guard = [&](int z, double (&G)[5]) {
    if (C.gslot >= 0) fetch(src + C.goff + (int64_t)z * C.gps, C.gvs, G);
  };

  // A) this thread's cell and guard cell of plane z into LDS
  auto stage_plane = [&](const float (&Wc)[5], const double (&Gr)[5]) {
    if (active) {
#pragma unroll
      for (int v = 0; v < NVAR; ++v) L[G::OW + v * PP + cw] = Wc[v];
    }
    if (C.gslot >= 0) {
      float Wg[5];
      prims(Gr, Wg, false);
#pragma unroll
      for (int v = 0; v < NVAR; ++v) L[G::OW + v * PP + C.gslot] = Wg[v];
    }
  };

  // B) one face: the PLM states on both sides from the four cells starting
  // at slot wb with stride st (1 along x, PX along y), then HLLC.  A y face
  // swaps the two in-plane velocity components into the face frame and its
  // flux back.
  auto face = [&](int wb, int st, int o, bool isx) {
    float Lr[5], Rr[5];
    if constexpr (RECON == RECON_CHARACTERISTIC) {
      // the four cells in the face frame (normal velocity in slot 1), then
      // each state from its own cell's characteristic slope
      float w[4][5];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float *q = L + wb + k * st;
        w[k][0] = q[0];
        w[k][1] = isx ? q[PP] : q[2 * PP];
        w[k][2] = isx ? q[2 * PP] : q[PP];
        w[k][3] = q[3 * PP];
        w[k][4] = q[4 * PP];
      }
      float d01[5], d12[5], d23[5], s1[5], s2[5];
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        d01[v] = w[1][v] - w[0][v];
        d12[v] = w[2][v] - w[1][v];
        d23[v] = w[3][v] - w[2][v];
      }
      char_slope_f32<1>(w[1], d01, d12, g32, s1);
      char_slope_f32<1>(w[2], d12, d23, g32, s2);
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        Lr[v] = __builtin_fmaf(0.5f, s1[v], w[1][v]);
        Rr[v] = __builtin_fmaf(-0.5f, s2[v], w[2][v]);
      }
      if (!(Lr[0] > 0.0f && Lr[4] > 0.0f && Rr[0] > 0.0f && Rr[4] > 0.0f) && active) {
        bad = 1;
        badblk = min(badblk, C.b);
      }
    } else {
      float a[5], r[5];
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        const float *w = L + v * PP + wb;
        const float w0 = w[0], w1 = w[st], w2 = w[2 * st], w3 = w[3 * st];
        const float d01 = w1 - w0, d12 = w2 - w1, d23 = w3 - w2;
        a[v] = __builtin_fmaf(0.5f, minmod_f(d01, d12), w1);
        r[v] = __builtin_fmaf(-0.5f, minmod_f(d12, d23), w2);
      }
      face_prims(a);
      face_prims(r);
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        Lr[v] = a[v];
        Rr[v] = r[v];
      }
      Lr[1] = isx ? a[1] : a[2];
      Lr[2] = isx ? a[2] : a[1];
      Rr[1] = isx ? r[1] : r[2];
      Rr[2] = isx ? r[2] : r[1];
    }
    float F[5];
    hllc<SPEEDS>(Lr, Rr, g32, rgm1, F);
    float *q = L + o;
    q[0] = F[0];
    q[NF] = isx ? F[1] : F[2];
    q[2 * NF] = isx ? F[2] : F[1];
    q[3 * NF] = F[3];
    q[4 * NF] = F[4];
  };
  auto faces = [&]() {
    face(jw0, 1, jo0, true);
    face(jw1, PX, jo1, false);
    if (has2) face(jw2, x2 ? 1 : PX, jo2, x2);
  };

  const double rdx0 = wave_uniform(1.0 / C.dx0), rdx1 = wave_uniform(1.0 / C.dx1), rdx2 = wave_uniform(1.0 / C.dx2);
  // C) FP64 update of this thread's cell in plane z (FP32 fluxes widened);
  // Un is the prefetched stage-2 state of the cell
  auto update = [&](int z, const double (&Us)[5], const double (&Un)[5], const float (&fzlo)[5],
                    const float (&fzhi)[5]) {
    if (!active) return;
    const int64_t c = (int64_t)z * C.plane + C.cidx;
    double Unew[5];
#pragma unroll
    for (int v = 0; v < NVAR; ++v) {
      const float *fx = L + G::OFX + v * NF;
      const float *fy = L + G::OFY + v * NF + tj * TX + ti;
      double dU = C.dtdx * ((double)fx[tj * TX + ti] - (double)fx[fx1]);
      dU = __builtin_fma(C.dtdy, (double)fy[0] - (double)fy[TX], dU);
      if (DIM == 3) dU = __builtin_fma(C.dtdz, (double)fzlo[v] - (double)fzhi[v], dU);
      Unew[v] = (STAGE == 1) ? Us[v] + dU : __builtin_fma(0.5, Un[v], 0.5 * (Us[v] + dU));
      // streamed out: the stage result is not read again in this launch, so it
      // must not evict the neighbours' cells that the guard reads hit in L2
      __builtin_nontemporal_store(Unew[v], &(A.dst + C.boff)[(int64_t)v * C.ncell + (int)c]);
    }
    if (STAGE == 2) {  // CFL rate of the new state in FP64
      double W[5];
      if (!recover_fast(Unew[0], Unew[1], Unew[2], Unew[3], Unew[4], gm1, W)) {
        bad = 1;
        badblk = min(badblk, C.b);
      } else {
        lam = fmax(lam, cell_rate_fast<DIM>(W, gamma, rdx0, rdx1, rdx2));
      }
    }
  };
  auto fetch_un = [&](int z, double (&Un)[5]) {
    if (STAGE == 2 && active) {
      const double *__restrict__ ub = A.un + C.boff;
      const int o = z * (int)C.plane + (int)C.cidx;
#pragma unroll
      for (int v = 0; v < NVAR; ++v) Un[v] = __builtin_nontemporal_load(&ub[(int64_t)v * C.ncell + o]);  // read once
    }
  };

  double Gr[5] = {0, 0, 0, 0, 0}, Un[5] = {0, 0, 0, 0, 0};
  if (DIM == 2) {
    double U[5] = {1, 0, 0, 0, 1};
    float Wc[5] = {1, 0, 0, 0, 1};
    if (active) fetch(src + C.boff + C.cidx, C.ncell, U);
    fetch_guard(0, Gr);
    fetch_un(0, Un);
    if (active) prims(U, Wc, true);
    const float zero[5] = {0, 0, 0, 0, 0};
    stage_plane(Wc, Gr);
    __syncthreads();
    faces();
    __syncthreads();
    update(0, U, Un, zero, zero);
    return;
  }

  // 3D: window Wb, Wc, Wd = planes j, j+1, j+2; carried z data: zp = plus
  // state of plane j, dlo = W_{j+1} - W_j; ring Ub, Uc, Ud of conserved values.
  float Wa[5] = {1, 0, 0, 0, 1}, Wb[5] = {1, 0, 0, 0, 1}, Wc[5] = {1, 0, 0, 0, 1}, Wd[5] = {1, 0, 0, 0, 1};
  double Ub[5] = {0, 0, 0, 0, 0}, Uc[5] = {0, 0, 0, 0, 0}, Ud[5] = {0, 0, 0, 0, 0};
  // own cells: wave-uniform base per variable, 32-bit lane offset
  auto fetch_z = [&](int z, double (&U)[5]) {
    if (!active) return;
    if (z >= 0 && z < C.nz) {
      const double *__restrict__ sb = src + C.boff;
      const int o = z * (int)C.plane + (int)C.cidx;
#pragma unroll
      for (int v = 0; v < NVAR; ++v) U[v] = sb[(int64_t)v * C.ncell + o];
    } else {
      int64_t off, vs;
      cell_addr(C.Bp, C.x, C.y, z, off, vs);
      fetch(src + off, vs, U);
    }
  };
  // Stage 1 fetches the guard ring two planes ahead (its registers allow
  // the second buffer; stage 2, held to three waves, fetches one ahead).
  constexpr bool G2 = STAGE == 1;
  double Gr2[5] = {0, 0, 0, 0, 0};
  fetch_z(C.z0 - 2, Ud);
  fetch_z(C.z0 - 1, Ub);
  fetch_z(C.z0, Uc);
  fetch_guard(C.z0, Gr);
  if (G2 && C.z0 + 1 < C.z1) fetch_guard(C.z0 + 1, Gr2);
  if (active) {
    prims(Ud, Wa, true);
    prims(Ub, Wb, true);
    prims(Uc, Wc, true);
  }
  float zp[5], dlo[5];
#pragma unroll
  for (int v = 0; v < NVAR; ++v) {
    dlo[v] = Wc[v] - Wb[v];
    zp[v] = __builtin_fmaf(0.5f, minmod_f(Wb[v] - Wa[v], dlo[v]), Wb[v]);
  }
  if constexpr (RECON == RECON_CHARACTERISTIC) {  // plane z0's slope from its own waves
    float da[5], s0[5];
#pragma unroll
    for (int v = 0; v < NVAR; ++v) da[v] = Wb[v] - Wa[v];
    char_slope_f32<3>(Wb, da, dlo, g32, s0);
#pragma unroll
    for (int v = 0; v < NVAR; ++v) zp[v] = __builtin_fmaf(0.5f, s0[v], Wb[v]);
  }
  // z face above plane j: primitives of plane j+2 (loaded one iteration
  // earlier), then the minus state of plane j+1 and HLLC with the carried plus
  // state of plane j
  auto zface = [&](float (&fz)[5]) {
    if (active) prims(Ud, Wd, true);
    float zr[5];
    if constexpr (RECON == RECON_CHARACTERISTIC) {
      float dhi[5], sc[5];
#pragma unroll
      for (int v = 0; v < NVAR; ++v) dhi[v] = Wd[v] - Wc[v];
      char_slope_f32<3>(Wc, dlo, dhi, g32, sc);
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        zr[v] = __builtin_fmaf(-0.5f, sc[v], Wc[v]);
        dlo[v] = dhi[v];
        Wa[v] = __builtin_fmaf(0.5f, sc[v], Wc[v]);  // plus state of plane j+1, carried into zp
      }
      if (!(zp[0] > 0.0f && zp[4] > 0.0f && zr[0] > 0.0f && zr[4] > 0.0f) && active) {
        bad = 1;
        badblk = min(badblk, C.b);
      }
    } else {
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        const float dhi = Wd[v] - Wc[v];
        const float m = minmod_f(dlo[v], dhi);
        zr[v] = __builtin_fmaf(-0.5f, m, Wc[v]);
        dlo[v] = dhi;
        Wa[v] = __builtin_fmaf(0.5f, m, Wc[v]);  // plus state of plane j+1, carried into zp
      }
    }
    float zl[5] = {zp[0], zp[1], zp[2], zp[3], zp[4]};  // zp is carried on as it is
    face_prims(zl);
    face_prims(zr);
    const float Lr[5] = {zl[0], zl[3], zl[2], zl[1], zl[4]};
    const float Rr[5] = {zr[0], zr[3], zr[2], zr[1], zr[4]};
    float F[5];
    hllc<SPEEDS>(Lr, Rr, g32, rgm1, F);
    fz[0] = F[0];
    fz[1] = F[3];
    fz[2] = F[2];
    fz[3] = F[1];
    fz[4] = F[4];
  };
  float fzlo[5];
  auto rotate = [&](const float (&fz)[5]) {
#pragma unroll
    for (int v = 0; v < NVAR; ++v) {
      zp[v] = Wa[v];
      fzlo[v] = fz[v];
      Wb[v] = Wc[v];
      Wc[v] = Wd[v];
      Ub[v] = Uc[v];
      Uc[v] = Ud[v];
    }
  };
  {  // the z face below the first plane
    fetch_z(C.z0 + 1, Ud);
    float fz[5];
    zface(fz);
    rotate(fz);
  }
  // A 16x16 item may be a z-run: slots 1..3 name the blocks above slot 0's,
  // linked along +z.  The plane loop then carries on from one block into the
  // next: planes beyond a block are read through its +z link, which is the
  // next block of the run, so the window already holds that block's first
  // planes -- no new prologue and no z halo read twice.
  int nrun = 1;
  if (NSUB == 1)
    while (nrun < 4 && __builtin_amdgcn_readfirstlane(it->block[nrun]) >= 0) ++nrun;
  for (int s = 0; s < nrun; ++s) {
    if (s > 0) {
      tile_setup<TX, TX, DIM>(C, A, it, s, lt, dt, PX);
      uniform_ctx();
      fetch_guard(C.z0, Gr);  // the new block's guard cells of its first plane(s)
      if (G2 && C.z0 + 1 < C.z1) fetch_guard(C.z0 + 1, Gr2);
    }
    for (int j = C.z0; j < C.z1; ++j) {
      fetch_z(j + 2, Ud);
      fetch_un(j, Un);
      stage_plane(Wb, Gr);
      if constexpr (G2) {
#pragma unroll
        for (int v = 0; v < NVAR; ++v) Gr[v] = Gr2[v];
        if (j + 2 < C.z1) fetch_guard(j + 2, Gr2);
      } else {
        if (j + 1 < C.z1) fetch_guard(j + 1, Gr);
      }
      __syncthreads();
      // x and y faces, then the z face (register work, no LDS), then the
      // leftover faces of job 2: one straight run of independent work
      face(jw0, 1, jo0, true);
      face(jw1, PX, jo1, false);
      float fz[5];
      zface(fz);
      if (has2) face(jw2, x2 ? 1 : PX, jo2, x2);
      __syncthreads();
      update(j, Ub, Un, fzlo, fz);
      rotate(fz);
    }
  }
}

// ------------------------------------------------------------------------
// Wave/workgroup reductions into the accumulator.
// ------------------------------------------------------------------------
__device__ __forceinline__ void flush_acc(DevTime *acc, double lam, int bad, int badblk, bool with_lam) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    lam = fmax(lam, __shfl_xor(lam, o));
    bad |= __shfl_xor(bad, o);
    badblk = min(badblk, __shfl_xor(badblk, o));
  }
  if ((threadIdx.x & 63) == 0) {
    if (with_lam) atomicMax(&acc->lam_bits, (unsigned long long)__double_as_longlong(lam));
    if (bad) {
      atomicOr(&acc->status, 1);
      if (badblk != INT_MAX) atomicMin(&acc->bad_block, badblk);
    }
  }
}

// Workgroups of a dispatch are handed to the 8 XCDs round-robin (workgroup i
// runs on XCD i mod 8), and each XCD has its own L2.  Renumbering so that XCD
// x runs the x-th contiguous span of workgroup indices keeps neighbouring
// blocks (whose interiors are each other's guards) on one L2.  The map is a
// bijection of [0, g) for any g.
__device__ __forceinline__ int xcd_logical(int bid, int g) {
  const int q = g >> 3, r = g & 7, x = bid & 7, l = bid >> 3;
  return x * q + min(x, r) + l;
}

template <int KMASK, bool MIXED>
constexpr size_t stage_lds_bytes() {
  using T = typename std::conditional<MIXED, float, double>::type;
  constexpr size_t a = (KMASK & 1) ? (MIXED ? SplitGeom<16>::ELEMS * sizeof(float) : tile_lds_bytes<16, 16, 1, T>()) : 0;
  constexpr size_t b = (KMASK & 2) ? (MIXED ? 4 * SplitGeom<8>::ELEMS * sizeof(float) : tile_lds_bytes<8, 8, 4, T>()) : 0;
  return a > b ? a : b;
}

// Occupancy: registers bound the mixed tile to three waves per SIMD (its
// 18.9 KiB of LDS would admit more).  Mixed stage 2 holds Un and the CFL rate
// on top of stage 1's registers and would settle at two; it is held to the
// register budget of three waves.  The FP64 16x16 tile's stage 1 (184
// registers, two waves) is held to three waves too: a few spilled dwords,
// measured 4 % faster; its stage 2, and both stages of kernels that also
// carry the 8x8 tile, spill too much at three and keep two.
// OCC > 0 asks instead for at least OCC waves per SIMD (the register budget
// of OCC waves: 2, 3 or 4), a candidate of the autotuner.
template <int DIM, bool MIXED, int STAGE, int KMASK, int SPEEDS, int RECON, int EOS, int OCC = 0>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(
    OCC > 0 ? OCC : (MIXED ? true : (STAGE == 1 && KMASK == 1 && EOS == EOS_IDEAL)) ? 3 : 1)))
void k_stage(StageArgs A) {
  static_assert(EOS == EOS_IDEAL || !MIXED, "the gas + radiation EOS runs on the FP64 tile only");
  __shared__ __attribute__((aligned(16))) unsigned char lds[stage_lds_bytes<KMASK, MIXED>()];
  if (A.reset_time && blockIdx.x == 0 && threadIdx.x == 0) {
    // plain path: this launch precedes the stage-2 launch that accumulates
    A.acc->lam_bits = 0ull;
    A.acc->status = 0;
    A.acc->bad_block = INT_MAX;
  }
  const double dt = A.dt_dev ? A.dt_dev->dt : A.dt;
  // A device time step that is not finite marks a failed step (k_finalize
  // sets it to NaN once a non-physical state was seen): the launch leaves
  // the state alone, so the state keeps the result of the failing step.
  // dt is one value for the whole launch, so every workgroup returns here
  // before its first barrier.
  if (!(__builtin_fabs(dt) <= __DBL_MAX__)) return;
  double lam = 0.0;
  int bad = 0, badblk = INT_MAX;
  const int first = A.xcd_remap ? xcd_logical(blockIdx.x, gridDim.x) : blockIdx.x;
  for (int i = first; i < A.nitems; i += gridDim.x) {
    const WorkItem *it = A.items + i;
    if ((KMASK & 1) && it->kind == KIND_T16) {
      // a 16x16 item is a run of up to four tiles taken one after the other
      // (the same tile of consecutive blocks of a z column: each tile's z
      // halo planes were read moments before by this workgroup, from L2)
      if constexpr (MIXED) {
        run_tile_mixed<16, 1, DIM, STAGE, SPEEDS, RECON>(A, it, lds, 0, dt, lam, bad, badblk);  // marches the whole run
      } else {
        for (int s = 0; s < 4; ++s) {
          if (s > 0) {
            if (__builtin_amdgcn_readfirstlane(it->block[s]) < 0) break;
            __syncthreads();  // LDS is reused by the next tile
          }
          run_tile<16, 16, 1, DIM, STAGE, SPEEDS, RECON, EOS>(A, it, lds, s, dt, lam, bad, badblk);
        }
      }
    } else if (KMASK & 2) {
      if constexpr (MIXED)
        run_tile_mixed<8, 4, DIM, STAGE, SPEEDS, RECON>(A, it, lds, 0, dt, lam, bad, badblk);
      else
        run_tile<8, 8, 4, DIM, STAGE, SPEEDS, RECON, EOS>(A, it, lds, 0, dt, lam, bad, badblk);
    }
    __syncthreads();  // LDS is reused by the next item
  }
  // Stage 1 reports nothing: a bad Un was already reported by the rate
  // reduction that produced dt, and a bad U1 is caught when stage 2 recovers
  // it -- also after a non-physical face state of conserved reconstruction,
  // whose negative pressure turns the face's sound speed, flux and so the
  // cells' U1 into NaN.  (In the plain path stage 1 also clears the
  // accumulator, so it must not race with its own reports.)
  if (STAGE == 2) flush_acc(A.acc, lam, bad, badblk, true);
}

// ------------------------------------------------------------------------
// Fused step of self-periodic 8^3 blocks: both RK stages of a block in one
// workgroup, the block on chip.  The 512 cells' primitives of the current
// stage source sit in LDS (each cell wraps around its own block, so the
// stencil never leaves it); each of the 256 threads owns two cells and keeps
// their Un and U1 in FP64 registers.  Per stage: recover the two cells into
// LDS; barrier; the flux of the low x, y and z face of each owned cell (PLM +
// HLLC from the four cells along the axis, wrapping) into three flux arrays;
// barrier; dU = sum_d (dt/dx_d)(F_lo - F_hi) in x, y, z order.  Stage 2 writes
// Un+1 over Un and reduces the CFL rate of the new state.  A workgroup loops
// over its blocks and loads the next block's Un while it computes the
// current one.  Un is read once and Un+1 written once: 80 algorithmic bytes
// per cell-update instead of the two-launch step's 200 (no first-stage state
// in HBM).  FP64: the oracle's operations in its order (bit-exact); MIXED:
// the mixed tile's FP32 faces, FP64 recovery check, update and rate.  Davis
// bounds, primitive PLM, gamma law.
// rate_only = 1: only the CFL rate of the current state (the dt of a run's
// first step).
// ------------------------------------------------------------------------
template <bool MIXED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MIXED ? 3 : 1))) void k_fused_cube8(FusedArgs A) {
#pragma clang fp contract(off)
  using T = typename std::conditional<MIXED, float, double>::type;
  constexpr int N = 8, NC = N * N * N, NT = 256;
  static_assert(2 * NT == NC, "two cells per thread");
  __shared__ T W[NVAR * NC];
  __shared__ T F[3][NVAR * NC];  // fluxes of the low x, y, z face of each cell
  const double dt = A.rate_only ? 0.0 : (A.dt_dev ? A.dt_dev->dt : A.dt);
  // a failed step (device dt not finite) leaves the state alone, as the stage kernels do
  if (!A.rate_only && !(__builtin_fabs(dt) <= __DBL_MAX__)) return;
  const double gamma = A.gamma, gm1 = gamma - 1.0;
  const float g32 = (float)gamma, rgm1 = (float)(1.0 / gm1);
  double lam = 0.0;
  int bad = 0, badblk = INT_MAX;
  const int tid = threadIdx.x;
  auto recov = [&](const double (&U)[5], double (&Wd)[5]) {
    return MIXED ? recover_fast(U[0], U[1], U[2], U[3], U[4], gm1, Wd)
                 : recover(U[0], U[1], U[2], U[3], U[4], gm1, Wd);
  };
  auto rate = [&](const double (&Wd)[5], const DevBlock &B) {
    return MIXED ? cell_rate_fast<3>(Wd, gamma, 1.0 / B.dx[0], 1.0 / B.dx[1], 1.0 / B.dx[2])
                 : cell_rate<3>(Wd, gamma, B.dx[0], B.dx[1], B.dx[2]);
  };
  // low face of cell c along axis d: the four cells c - 2e_d .. c + e_d
  // (wrapping around the block), rotated into the face frame (normal velocity
  // first, the tangential ones in the order the other kernels use), HLLC, and
  // the flux rotated back
  auto face = [&](int c, int d) {
    const int i = c & 7, j = (c >> 3) & 7, k = c >> 6;
    auto at = [&](int o) {
      const int ii = d == 0 ? (i + o) & 7 : i, jj = d == 1 ? (j + o) & 7 : j, kk = d == 2 ? (k + o) & 7 : k;
      return (kk * N + jj) * N + ii;
    };
    const int c0 = at(-2), c1 = at(-1), c3 = at(1);
    T wl[5], wr[5];
#pragma unroll
    for (int v = 0; v < NVAR; ++v) {
      const T w0 = W[v * NC + c0], w1 = W[v * NC + c1], w2 = W[v * NC + c], w3 = W[v * NC + c3];
      if constexpr (MIXED) {
        const float d01 = w1 - w0, d12 = w2 - w1, d23 = w3 - w2;
        wl[v] = __builtin_fmaf(0.5f, minmod_f(d01, d12), w1);
        wr[v] = __builtin_fmaf(-0.5f, minmod_f(d12, d23), w2);
      } else {
        plm(w0, w1, w2, w3, wl[v], wr[v]);
      }
    }
    const int n = 1 + d, t1 = d == 1 ? 1 : 2, t2 = d == 2 ? 1 : 3;
    const T L[5] = {wl[0], wl[n], wl[t1], wl[t2], wl[4]};
    const T R[5] = {wr[0], wr[n], wr[t1], wr[t2], wr[4]};
    T Fr[5];
    if constexpr (MIXED)
      hllc<SPEEDS_DAVIS>(L, R, g32, rgm1, Fr);
    else
      hllc_fp64<SPEEDS_DAVIS, EOS_IDEAL>(L, R, gamma, Fr);
    T Fo[5];
    Fo[0] = Fr[0];
    Fo[4] = Fr[4];
    Fo[n] = Fr[1];
    Fo[t1] = Fr[2];
    Fo[t2] = Fr[3];
#pragma unroll
    for (int v = 0; v < NVAR; ++v) F[d][v * NC + c] = Fo[v];
  };
  // the cell above c along axis d (wrapping)
  auto up = [&](int c, int d) {
    const int i = c & 7, j = (c >> 3) & 7, k = c >> 6;
    return d == 0 ? (k * N + j) * N + ((i + 1) & 7) : d == 1 ? (k * N + ((j + 1) & 7)) * N + i
                                                             : (((k + 1) & 7) * N + j) * N + i;
  };
  auto load = [&](int q, double (&U)[2][5]) {
    if (q >= A.nblocks) return;
    const double *__restrict__ st = A.state + A.blocks[__builtin_amdgcn_readfirstlane(A.ids[q])].off;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int v = 0; v < NVAR; ++v) U[h][v] = st[v * NC + tid + NT * h];
  };

  const int first = A.xcd_remap ? xcd_logical(blockIdx.x, gridDim.x) : blockIdx.x;
  double Un[2][5] = {}, Unext[2][5] = {};
  load(first, Unext);
  for (int q = first; q < A.nblocks; q += gridDim.x) {
    const int b = __builtin_amdgcn_readfirstlane(A.ids[q]);
    const DevBlock &B = A.blocks[b];
    double *__restrict__ st = A.state + B.off;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int v = 0; v < NVAR; ++v) Un[h][v] = Unext[h][v];
    load(q + gridDim.x, Unext);  // in flight while this block is computed
    if (A.rate_only) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double Wd[5];
        if (!recov(Un[h], Wd)) {
          bad = 1;
          badblk = min(badblk, b);
        } else {
          lam = fmax(lam, rate(Wd, B));
        }
      }
      continue;
    }
    const double dtd[3] = {dt / B.dx[0], dt / B.dx[1], dt / B.dx[2]};
    double Us[2][5];
#pragma unroll
    for (int stage = 1; stage <= 2; ++stage) {
      // the stage source's primitives into LDS (stage 1 reports nothing: a bad
      // Un was reported by the rate reduction that gave dt).  The previous
      // stage's (or block's) last LDS reads were of F, behind a barrier
      // after its last reads of W.
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double Wd[5];
        if (!recov(stage == 1 ? Un[h] : Us[h], Wd) && stage == 2) {
          bad = 1;
          badblk = min(badblk, b);
        }
#pragma unroll
        for (int v = 0; v < NVAR; ++v) W[v * NC + tid + NT * h] = (T)Wd[v];
      }
      __syncthreads();
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        face(tid, d);
        face(tid + NT, d);
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = tid + NT * h;
        const int cx = up(c, 0), cy = up(c, 1), cz = up(c, 2);
#pragma unroll
        for (int v = 0; v < NVAR; ++v) {
          const double fx = (double)F[0][v * NC + c] - (double)F[0][v * NC + cx];
          const double fy = (double)F[1][v * NC + c] - (double)F[1][v * NC + cy];
          const double fz = (double)F[2][v * NC + c] - (double)F[2][v * NC + cz];
          double dU;
          if constexpr (MIXED) {
            dU = __builtin_fma(dtd[2], fz, __builtin_fma(dtd[1], fy, dtd[0] * fx));
          } else {
            dU = dtd[0] * fx;
            dU += dtd[1] * fy;
            dU += dtd[2] * fz;
          }
          if (stage == 1)
            Us[h][v] = Un[h][v] + dU;
          else
            Us[h][v] = MIXED ? __builtin_fma(0.5, Un[h][v], 0.5 * (Us[h][v] + dU))
                             : 0.5 * Un[h][v] + 0.5 * (Us[h][v] + dU);
        }
      }
      // W is rewritten next only after every thread has passed the barrier
      // above, i.e. after every face read of W; F is rewritten only after the
      // next barrier, i.e. after every read of F
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int v = 0; v < NVAR; ++v) __builtin_nontemporal_store(Us[h][v], &st[v * NC + tid + NT * h]);
      double Wd[5];
      if (!recov(Us[h], Wd)) {
        bad = 1;
        badblk = min(badblk, b);
      } else {
        lam = fmax(lam, rate(Wd, B));
      }
    }
  }
  flush_acc(A.acc, lam, bad, badblk, true);
}

// CFL rate of the interior cells of the work list (FP64): in oracle order,
// or (MIXED) with the mixed path's recovery and rate, as its stage 2 reduces
// it.
template <int DIM, int KMASK, int EOS, bool MIXED>
__global__ __launch_bounds__(WG) void k_lambda(StageArgs A) {
  double lam = 0.0;
  int bad = 0, badblk = INT_MAX;
  const int first = A.xcd_remap ? xcd_logical(blockIdx.x, gridDim.x) : blockIdx.x;
  for (int i = first; i < A.nitems; i += gridDim.x) {
    const WorkItem *it = A.items + i;
    const bool t16 = (KMASK & 1) && it->kind == KIND_T16;
    const int TX = t16 ? 16 : 8, NT = t16 ? 256 : 64;
    const int sub = __builtin_amdgcn_readfirstlane(threadIdx.x / NT), lt = threadIdx.x % NT;
    // the tiles of the item: slots 0..3 of a 16x16 run, or this wave's 8x8 tile
    for (int s = 0; s < (t16 ? 4 : 1); ++s) {
      const int slot = t16 ? s : sub;
      const int b = __builtin_amdgcn_readfirstlane(it->block[slot]);
      if (b < 0) break;
      const DevBlock &B = A.blocks[b];
      const int x = __builtin_amdgcn_readfirstlane(it->x0[slot]) + lt % TX;
      const int y = __builtin_amdgcn_readfirstlane(it->y0[slot]) + lt / TX;
      const int64_t plane = (int64_t)B.n[0] * B.n[1];
      const double *p = A.src + B.off + (int64_t)y * B.n[0] + x;
      const int za = DIM == 3 ? it->z0 : 0, zb = DIM == 3 ? it->z1 : 1;
      // unrolled so that the loads of several planes are in flight at once
#pragma unroll 4
      for (int z = za; z < zb; ++z) {
        double W[5];
        if constexpr (MIXED) {
          const double *q = p + z * plane;
          const int64_t vs = B.ncell;
          if (!recover_fast(q[0], q[vs], q[2 * vs], q[3 * vs], q[4 * vs], A.gamma - 1.0, W)) {
            bad = 1;
            badblk = min(badblk, b);
            continue;
          }
          lam = fmax(lam, cell_rate_fast<DIM>(W, A.gamma, 1.0 / B.dx[0], 1.0 / B.dx[1], 1.0 / B.dx[2]));
        } else {
          if (!load_prim<EOS>(p + z * plane, B.ncell, A.gamma, W)) {
            bad = 1;
            badblk = min(badblk, b);
            continue;
          }
          lam = fmax(lam, cell_rate<DIM, EOS>(W, A.gamma, B.dx[0], B.dx[1], B.dx[2]));
        }
      }
    }
  }
  flush_acc(A.acc, lam, bad, badblk, true);
}

// ------------------------------------------------------------------------
// Launchers.
// ------------------------------------------------------------------------
template <int DIM, bool MIXED, int STAGE, int SPEEDS, int RECON, int EOS = EOS_IDEAL, int OCC = 0>
static hipError_t launch_ks(int kmask, int grid, hipStream_t s, const StageArgs &a) {
  switch (kmask) {
    case 1:
      hipLaunchKernelGGL((k_stage<DIM, MIXED, STAGE, 1, SPEEDS, RECON, EOS, OCC>), dim3(grid), dim3(WG), 0, s, a);
      break;
    case 2:
      hipLaunchKernelGGL((k_stage<DIM, MIXED, STAGE, 2, SPEEDS, RECON, EOS, OCC>), dim3(grid), dim3(WG), 0, s, a);
      break;
    default:
      hipLaunchKernelGGL((k_stage<DIM, MIXED, STAGE, 3, SPEEDS, RECON, EOS, OCC>), dim3(grid), dim3(WG), 0, s, a);
      break;
  }
  return hipGetLastError();
}

template <int DIM, bool MIXED, int STAGE, int RECON>
static hipError_t launch_kr(int kmask, int speeds, int grid, hipStream_t s, const StageArgs &a) {
  switch (speeds) {
    case SPEEDS_EINFELDT:
      return launch_ks<DIM, MIXED, STAGE, SPEEDS_EINFELDT, RECON>(kmask, grid, s, a);
    case SPEEDS_PVRS:
      return launch_ks<DIM, MIXED, STAGE, SPEEDS_PVRS, RECON>(kmask, grid, s, a);
    default:
      return launch_ks<DIM, MIXED, STAGE, SPEEDS_DAVIS, RECON>(kmask, grid, s, a);
  }
}

// The default method (Davis bounds, primitive PLM, gamma law) with an
// occupancy request of occ (2, 3 or 4) waves per SIMD instead of the
// default register budget.
template <int DIM, bool MIXED, int STAGE>
static hipError_t launch_occ(int kmask, int occ, int grid, hipStream_t s, const StageArgs &a) {
  switch (occ) {
    case 2:
      return launch_ks<DIM, MIXED, STAGE, SPEEDS_DAVIS, RECON_PRIMITIVE, EOS_IDEAL, 2>(kmask, grid, s, a);
    case 3:
      return launch_ks<DIM, MIXED, STAGE, SPEEDS_DAVIS, RECON_PRIMITIVE, EOS_IDEAL, 3>(kmask, grid, s, a);
    default:
      return launch_ks<DIM, MIXED, STAGE, SPEEDS_DAVIS, RECON_PRIMITIVE, EOS_IDEAL, 4>(kmask, grid, s, a);
  }
}

template <int DIM, bool MIXED, int STAGE>
static hipError_t launch_k(int kmask, int speeds, int recon, int grid, hipStream_t s, const StageArgs &a) {
  switch (recon) {
    case RECON_CONSERVED:
      return launch_kr<DIM, MIXED, STAGE, RECON_CONSERVED>(kmask, speeds, grid, s, a);
    case RECON_CHARACTERISTIC:
      return launch_kr<DIM, MIXED, STAGE, RECON_CHARACTERISTIC>(kmask, speeds, grid, s, a);
    default:
      return launch_kr<DIM, MIXED, STAGE, RECON_PRIMITIVE>(kmask, speeds, grid, s, a);
  }
}

}  // namespace hyd
