// Device-side physics of the WENO5-CT step for gfx950: zone fluxes and wave
// speeds, the face eigensystem of Appendix A, the WENO5 interpolant of
// Sect. 2.2 and the per-face characteristic flux.  Everything here runs per
// lane on the VALU; nothing is a dense contraction (each face has its own 7x7
// eigenvector matrices used on ten vectors), so there is no MFMA path.
#pragma once
#include <hip/hip_runtime.h>

namespace wm {

struct Phys {
  double gamma;     // adiabatic index
  double inv_h;     // 1 / zone size
  double eps;       // WENO epsilon (Jiang-Shu)
  double eps_B;     // degeneracy threshold of Appendix A
  double eps_Z;     // WENO-Z epsilon
  int weno_z;       // 0: Jiang-Shu weights, 1: WENO-Z, 2: WENO-Z as printed
  double g1;        // (gamma - 1) / 2
  double g2;        // (gamma - 2) / (gamma - 1)
};

__host__ __device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Number of per-zone values a sweep stages in LDS.
enum ZoneVar {
  Z_RHO = 0, Z_MN, Z_MT1, Z_MT2, Z_BT1, Z_BT2, Z_E,        // q, 7 components
  Z_F0, Z_F1, Z_F2, Z_F3, Z_F4, Z_F5, Z_F6,                // F_n(q), 7 components
  Z_VN, Z_VT1, Z_VT2, Z_BN, Z_P,                           // primitives for the face state
  Z_CF, Z_CA, Z_CS,                                        // c_fast, c_A, c_slow
  Z_NVAR
};

// Scheduling fence: keeps the compiler from hoisting the LDS reads of later
// interfaces / passes above earlier ones, which bounds register pressure.
__host__ __device__ __forceinline__ void sched_fence() {
#ifdef __HIP_DEVICE_COMPILE__
  __builtin_amdgcn_sched_barrier(0);
#endif
}

// Reciprocal: the hardware estimate (relative error up to 4.6e-8 on MI355X,
// measured over 2^22 arguments) refined by two Newton steps, exact to rounding.
__host__ __device__ __forceinline__ double rcp_w(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(e, r, r);
  e = fma(-x, r, 1.0);
  return fma(e, r, r);
#else
  return 1.0 / x;
#endif
}
// hardware reciprocal without refinement (about 1 ulp), for scale factors
__host__ __device__ __forceinline__ float rcp_raw(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
__host__ __device__ __forceinline__ double rcp_raw(double x) { return rcp_w(x); }

__host__ __device__ __forceinline__ float rcp_w(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(fmaf(-x, r, 1.0f), r, r);
#else
  return 1.0f / x;
#endif
}
// One Newton step on the hardware estimate: relative error up to 2.2e-15
// (measured), for the common denominator of the FP64 WENO weights, where it
// scales the interpolant phi_N by at most that factor.  The FP32 form is rcp_w.
__host__ __device__ __forceinline__ double rcp_1(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  const double r = __builtin_amdgcn_rcp(x);
  return fma(fma(-x, r, 1.0), r, r);
#else
  return 1.0 / x;
#endif
}
__host__ __device__ __forceinline__ float rcp_1(float x) { return rcp_w(x); }

// 1/sqrt(x) for x > 0 from the hardware estimate (relative error up to 5.2e-8,
// measured) and two Newton steps (~1 ulp); sqrt(x) for x >= 0 from one Newton
// step on 1/sqrt (up to 4.3e-15) and one on the square root itself, which
// brings it to ~1 ulp (sqrt(0) = 0).
__host__ __device__ __forceinline__ double rsq_nr(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
#else
  return 1.0 / sqrt(x);
#endif
}
__host__ __device__ __forceinline__ double sqrt_nr(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  const double xc = fmax(x, 1e-300);
  const double y0 = __builtin_amdgcn_rsq(xc);
  const double y = fma(0.5 * y0, fma(-xc * y0, y0, 1.0), y0);
  const double r = x * y;
  return fma(0.5 * y, fma(-r, r, x), r);
#else
  return sqrt(x);
#endif
}

// Zone prologue of a sweep (step 2 of the 3D step list): primitives (eq. P),
// the flux along n (eq. fluxes, total pressure P + |B|^2/2), and the fast,
// Alfven and slow speeds.  Inputs are in the sweep frame (n, t1, t2).
struct ZoneVals {
  double v[Z_NVAR];
};

__host__ __device__ __forceinline__ void zone_prologue(double rho, double mn, double mt1, double mt2, double E,
                                              double Bn, double Bt1, double Bt2, double gamma,
                                              double* out) {
  // Every rounding step is written out (no implicit FMA contraction, whose
  // choice of product can differ between the kernels this is inlined into):
  // the sweep and the stand-alone time-step pass get bitwise the same speeds.
#pragma clang fp contract(off)
  const double irho = rcp_w(rho);
  const double vn = mn * irho, vt1 = mt1 * irho, vt2 = mt2 * irho;
  const double Bperp2 = fma(Bt2, Bt2, Bt1 * Bt1);
  const double B2 = fma(Bn, Bn, Bperp2);
  const double mv = fma(mt2, vt2, fma(mt1, vt1, mn * vn));
  const double P = (gamma - 1.0) * fma(-0.5, mv + B2, E);
  const double Pstar = fma(0.5, B2, P);
  const double vB = fma(vt2, Bt2, fma(vt1, Bt1, vn * Bn));
  const double rvn = rho * vn;
  out[Z_RHO] = rho; out[Z_MN] = mn; out[Z_MT1] = mt1; out[Z_MT2] = mt2;
  out[Z_BT1] = Bt1; out[Z_BT2] = Bt2; out[Z_E] = E;
  out[Z_F0] = rvn;
  out[Z_F1] = fma(-Bn, Bn, fma(rvn, vn, Pstar));
  out[Z_F2] = fma(-Bn, Bt1, rvn * vt1);
  out[Z_F3] = fma(-Bn, Bt2, rvn * vt2);
  out[Z_F4] = fma(Bt1, vn, -(Bn * vt1));
  out[Z_F5] = fma(Bt2, vn, -(Bn * vt2));
  out[Z_F6] = fma(E + Pstar, vn, -(Bn * vB));
  out[Z_VN] = vn; out[Z_VT1] = vt1; out[Z_VT2] = vt2; out[Z_BN] = Bn; out[Z_P] = P;
  // c_f,s^2 = (a^2 + b^2 +- D)/2, D = sqrt((a^2 - b^2)^2 + 4 a^2 b_perp^2),
  // c_slow^2 = a^2 b_n^2 / c_fast^2 (no cancellation), c_A = |B_n|/sqrt(rho)
  const double a2 = (gamma * P) * irho;
  const double bn2 = (Bn * Bn) * irho;
  const double dab = fma(-B2, irho, a2), apb = fma(B2, irho, a2);   // a^2 -+ b^2
  const double D = sqrt_nr(fma(dab, dab, (4.0 * a2) * (Bperp2 * irho)));
  const double cf2 = 0.5 * (apb + D);
  const double cs2 = cf2 > 0.0 ? (a2 * bn2) * rcp_w(cf2) : 0.0;
  out[Z_CF] = sqrt_nr(cf2);
  out[Z_CA] = sqrt_nr(bn2);
  out[Z_CS] = sqrt_nr(cs2);
}

// WENO5 interpolant phi_N(a, b, c, d) of Sect. 2.2.  With s_k = eps + IS_k the
// Jiang-Shu weights alpha_k = d_k / s_k^2 give
//   omega_0 = s1^2 s2^2 / Q,  omega_2 = 3 s0^2 s1^2 / Q,
//   Q = s1^2 s2^2 + 6 s0^2 s2^2 + 3 s0^2 s1^2,
// one reciprocal instead of four divisions.  WENO-Z: alpha_k = d_k (1 + u_k) with
// u_k = (tau_5/(eps_Z + IS_k))^2 (the dimensionless ratio squared), or, with `lit`,
// u_k = tau_5/(eps_Z + IS_k)^2 as Sect. 2.2 prints it.  Always evaluated in FP64:
// eps_Z (1e-40 in the paper) lies below the FP32 range.
template <bool WENO_Z, typename T>
__host__ __device__ __forceinline__ T phiN(T a, T b, T c, T d, T eps, double eps_Z, bool lit) {
  const T t0 = a - b, t1 = a - T(3) * b;
  const T t2 = b - c, t3 = b + c;
  const T t4 = c - d, t5 = T(3) * c - d;
  const T X = t0 - t2, Y = t2 - t4;   // a - 2b + c, b - 2c + d
  if (!WENO_Z) {
    (void)lit;
    // s_k/3 = eps/3 + IS_k/3: a common factor of the three s_k cancels in the
    // weights.  phi = [p12 X / 3 + (p01/4 - p12/12 - p02/2) Y] / Q with
    // p_ij = s_i^2 s_j^2 and Q = p12 + 6 p02 + 3 p01.
    const T e3 = eps * T(1.0 / 3.0);
    T s0 = fma(T(13.0 / 3.0) * t0, t0, fma(t1, t1, e3));
    T s1 = fma(T(13.0 / 3.0) * t2, t2, fma(t3, t3, e3));
    T s2 = fma(T(13.0 / 3.0) * t4, t4, fma(t5, t5, e3));
    s0 *= s0; s1 *= s1; s2 *= s2;
    if (sizeof(T) == 4) {   // FP32: normalise so the products cannot overflow; phi is
      // homogeneous of degree 0 in the s_k, so the scale need not be exact
      const T r = rcp_raw(fmax(s0, fmax(s1, s2)));
      s0 *= r; s1 *= r; s2 *= r;
    }
    const T p12 = s1 * s2, p02 = s0 * s2, p01 = s0 * s1;
    const T rq = rcp_1(fma(T(3), p01, fma(T(6), p02, p12)));
    const T cY = fma(T(0.25), p01, fma(T(-1.0 / 12.0), p12, T(-0.5) * p02));
    return rq * fma(cY, Y, (p12 * T(1.0 / 3.0)) * X);
  } else {
    if constexpr (sizeof(T) == 4)
      return T(phiN<true, double>(double(a), double(b), double(c), double(d), double(eps), eps_Z, lit));
    const T IS0 = T(13) * t0 * t0 + T(3) * t1 * t1;
    const T IS1 = T(13) * t2 * t2 + T(3) * t3 * t3;
    const T IS2 = T(13) * t4 * t4 + T(3) * t5 * t5;
    const T tau5 = fabs(IS0 - IS2);
    // alpha_k P^2 with P = s0 s1 s2, s_k = eps_Z + IS_k: d_k (P^2 + t m_k^2), m_k = P / s_k,
    // t = tau_5^2 (or tau_5 as printed); the common factor P^2 cancels in the
    // weights, so one reciprocal serves.  eps_Z >= 1e-50 keeps P^2 >= eps_Z^6 normal.
    const T s0 = eps_Z + IS0, s1 = eps_Z + IS1, s2 = eps_Z + IS2;
    const T m0 = s1 * s2, m1 = s0 * s2, m2 = s0 * s1;
    const T P = s0 * m0, P2 = P * P;
    const T t = lit ? tau5 : tau5 * tau5;
    const T al0 = fma(t * m0, m0, P2), al1 = T(6) * fma(t * m1, m1, P2), al2 = T(3) * fma(t * m2, m2, P2);
    const T inv = rcp_1(al0 + al1 + al2);
    return inv * (al0 * X * T(1.0 / 3.0) + (al2 - T(0.5) * (al0 + al1 + al2)) * Y * T(1.0 / 6.0));
  }
}

// phi^- - phi^+ of eq. (FWENO) from the split values of one characteristic
// field: v[0..3] = Delta F^+ at i-3/2 .. i+3/2, v[4..7] = Delta F^- at i-1/2 .. i+5/2.
template <bool WENO_Z, typename T>
__host__ __device__ __forceinline__ T weno_split(const T v[8], T eps, double eps_Z, bool lit) {
  return phiN<WENO_Z>(v[7], v[6], v[5], v[4], eps, eps_Z, lit) - phiN<WENO_Z>(v[0], v[1], v[2], v[3], eps, eps_Z, lit);
}

// Eigen-system scalars of Appendix A at one face (always FP64: the
// renormalisation near degeneracies is done in double precision).  qa2 =
// 1/(4 a^2) carries the 1/(2 c_s^2) of the fast and slow rows times the 1/2 of
// the Lax-Friedrichs split, which is folded into every left row.
struct FaceEig {
  double vn, vt1, vt2, Bt1, Bt2;
  double a2, cs, sr, isr, cf, cf2, csl, csl2;
  double by, bz, s, af, as;
  double v2, Gf, Ga, Gs, qa2, tau, g1, g2, omg;
};

// alpha_f^2 = (D + dab) / (2D) and alpha_s^2 = (D - dab) / (2D) of eq. (alpha),
// dab = a^2 - b^2, D = sqrt(dab^2 + p), p = 4 a^2 b_perp^2 >= 0, clamped to
// [0, 1].  The difference of nearly equal terms, D - |dab|, is formed as
// p / (D + |dab|), so the smaller of the two is exact to rounding also as
// b_perp -> 0 (it is exactly 0 at b_perp = 0, where 1 - dab/D would leave a
// rounding residue that the square root of alpha raises to ~1e-8).
__host__ __device__ __forceinline__ void alpha_sq(double dab, double D, double p, double& cfa, double& csa) {
  const double h = 0.5 * rcp_w(D);
  const double big = (D + fabs(dab)) * h;
  const double small = p * rcp_w(D + fabs(dab)) * h;
  cfa = fmin(fmax(dab >= 0.0 ? big : small, 0.0), 1.0);
  csa = fmin(fmax(dab >= 0.0 ? small : big, 0.0), 1.0);
}

__host__ __device__ __forceinline__ void face_eig(double rho, double vn, double vt1, double vt2, double Bn, double Bt1,
                                                  double Bt2, double P, const Phys& ph, FaceEig& e) {
  const double gamma = ph.gamma;
  e.vn = vn; e.vt1 = vt1; e.vt2 = vt2; e.Bt1 = Bt1; e.Bt2 = Bt2;
  e.isr = rsq_nr(rho);
  e.sr = rho * e.isr;
  const double irho = e.isr * e.isr;
  e.a2 = gamma * P * irho;
  e.cs = sqrt_nr(e.a2);
  const double ia2 = rcp_w(e.a2);
  const double Bperp2 = Bt1 * Bt1 + Bt2 * Bt2;
  const double b2 = (Bn * Bn + Bperp2) * irho;
  const double dab = e.a2 - b2;
  const double p4 = 4.0 * e.a2 * (Bperp2 * irho);
  const double D = sqrt_nr(dab * dab + p4);
  e.cf2 = 0.5 * (e.a2 + b2 + D);
  e.cf = sqrt_nr(e.cf2);
  e.csl2 = e.cf2 > 0.0 ? e.a2 * (Bn * Bn * irho) * rcp_w(e.cf2) : 0.0;
  e.csl = sqrt_nr(e.csl2);
  if (Bperp2 > ph.eps_B) {
    const double ib = rsq_nr(Bperp2);
    e.by = Bt1 * ib;
    e.bz = Bt2 * ib;
  } else {
    e.by = 0.70710678118654752440;
    e.bz = 0.70710678118654752440;
  }
  e.s = Bn >= ph.eps_B ? 1.0 : -1.0;
  if (D >= ph.eps_B * ph.eps_B) {
    double cfa, csa;
    alpha_sq(dab, D, p4, cfa, csa);
    e.af = sqrt_nr(cfa);
    e.as = sqrt_nr(csa);
  } else {
    e.af = 0.70710678118654752440;
    e.as = 0.70710678118654752440;
  }
  e.g1 = ph.g1;
  e.g2 = ph.g2;
  e.omg = 1.0 - gamma;
  e.qa2 = 0.25 * ia2;
  e.tau = (gamma - 1.0) * ia2;
  e.v2 = vn * vn + vt1 * vt1 + vt2 * vt2;
  const double bv = e.by * vt1 + e.bz * vt2;
  e.Gf = e.af * e.cf * vn - e.as * e.csl * e.s * bv;
  e.Ga = e.s * (e.bz * vt1 - e.by * vt2);
  e.Gs = e.as * e.csl * vn + e.af * e.cf * e.s * bv;
}

// Characteristic part of the interface flux at face i+1/2,
//   corr = sum_m R(:,m) (phi^-_m - phi^+_m),
// so that F_{i+1/2} = F_c + corr with the central term F_c in physical space
// (R L = I), eq. (FWENO).  L and R follow Appendix A: m = 1, 2, 3 take the
// upper signs and 7, 6, 5 the lower; m = 2, 6 are the Alfven waves and m = 3, 5
// the slow waves.  `al(m)` gives the Lax-Friedrichs speed of field m (0-based),
// `dl(j, k)` reads interface difference j of interface k.  Projections, split
// and weights run in T; the eigen scalars and the back-projection in FP64.
// corr is added to (the caller passes the central term F_c in it).
template <bool WENO_Z, typename T, class AL, class DL>
__host__ __device__ __forceinline__ void face_corr(const FaceEig& e, AL al, DL dl, const Phys& ph,
                                                   double corr[7]) {
  const T eps = T(ph.eps);
  const double epsZ = ph.eps_Z;
  const bool lit = ph.weno_z == 2;
  const double gm1 = -e.omg;
  const double sra = e.sr * e.cs;
  T vu[8], vl[8];
  // The fast and slow left rows share W = (g1 v2, omg vn, omg vt1, omg vt2,
  // omg Bt1, omg Bt2, gm1): fast S = qa2 (af W + sra as beta), slow S = qa2 (as W
  // - sra af beta) with beta = (0, 0, 0, 0, by, bz, 0), and the entropy row is
  // e0/2 - 2 qa2 W (ht = 2 qa2 (gamma - 1)).  The projections W.dF, W.dq of the
  // five interfaces are formed once, in the fast pair, and reused.
  // W.d = g1 v2 d0 + omg (vn d1 + vt1 d2 + vt2 d3 + Bt1 d4 + Bt2 d5) + gm1 d6, with the
  // uniform factors applied after the per-lane sum (fewer live registers than W itself)
  const T w0 = T(e.g1 * e.v2), wv[5] = {T(e.vn), T(e.vt1), T(e.vt2), T(e.Bt1), T(e.Bt2)};
  const T omgT = T(e.omg), gm1T = T(gm1);
  auto wdot = [&](const T* d) {
    T in = wv[0] * d[1];
#pragma unroll
    for (int j = 1; j < 5; ++j) in += wv[j] * d[1 + j];
    return omgT * in + (w0 * d[0] + gm1T * d[6]);
  };
  T WF[5], Wq[5];
  // Split values of a pair whose left rows are S + A (upper, lambda = v - c) and
  // S - A (lower), at interface k = 0..4 (i-3/2 .. i+5/2) from the projections
  // sF = S.dF, sq = S.dq, aF = A.dF, aq = A.dq (dl(j, k): j = 0..6 Delta F,
  // 7..13 Delta q).  Lax-Friedrichs: Delta F^+- = (Delta F^s +- alpha Delta q^s)/2,
  // the 1/2 carried by the rows; vu[0..3] / vu[4..7] feed phi^+ / phi^-.
  auto split_k = [&](int k, T sF, T sq, T aF, T aq, T alu, T all) {
    const T uF = sF + aF, uq = sq + aq, lF = sF - aF, lq = sq - aq;
    if (k <= 3) { vu[k] = uF + alu * uq; vl[k] = lF + all * lq; }
    if (k >= 1) { vu[3 + k] = uF - alu * uq; vl[3 + k] = lF - all * lq; }
  };
  // ---- fast pair (m = 1, 7)
  {
    const T cW = T(e.qa2 * e.af), cBy = T(e.qa2 * (sra * e.as) * e.by), cBz = T(e.qa2 * (sra * e.as) * e.bz);
    const T A[4] = {T(e.qa2 * e.Gf), T(-e.qa2 * (e.af * e.cf)), T(e.qa2 * (e.csl * e.as * e.by * e.s)),
                    T(e.qa2 * (e.csl * e.as * e.bz * e.s))};
    const T alu = al(0), all = al(6);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      T dF[7], dq[7];
#pragma unroll
      for (int j = 0; j < 7; ++j) { dF[j] = dl(j, k); dq[j] = dl(7 + j, k); }
      const T wF = wdot(dF), wq = wdot(dq);
      WF[k] = wF;
      Wq[k] = wq;
      T aF = A[0] * dF[0], aq = A[0] * dq[0];
#pragma unroll
      for (int j = 1; j < 4; ++j) { aF += A[j] * dF[j]; aq += A[j] * dq[j]; }
      split_k(k, cW * wF + (cBy * dF[4] + cBz * dF[5]), cW * wq + (cBy * dq[4] + cBz * dq[5]), aF, aq, alu, all);
      sched_fence();
    }
    const double fu = double(weno_split<WENO_Z>(vu, eps, epsZ, lit));
    const double fl = double(weno_split<WENO_Z>(vl, eps, epsZ, lit));
    const double sp = fu + fl, sm = fu - fl;
    corr[0] += e.af * sp;
    corr[1] += e.af * e.vn * sp - e.af * e.cf * sm;
    corr[2] += e.af * e.vt1 * sp + e.csl * e.as * e.by * e.s * sm;
    corr[3] += e.af * e.vt2 * sp + e.csl * e.as * e.bz * e.s * sm;
    corr[4] += e.cs * e.as * e.by * e.isr * sp;
    corr[5] += e.cs * e.as * e.bz * e.isr * sp;
    corr[6] += e.af * (0.5 * e.v2 + e.cf2 - e.g2 * e.a2) * sp - e.Gf * sm;
  }
  sched_fence();
  // ---- slow pair (m = 3, 5)
  {
    const T cW = T(e.qa2 * e.as), cBy = T(-e.qa2 * (sra * e.af) * e.by), cBz = T(-e.qa2 * (sra * e.af) * e.bz);
    const T A[4] = {T(e.qa2 * e.Gs), T(-e.qa2 * (e.as * e.csl)), T(-e.qa2 * (e.cf * e.af * e.by * e.s)),
                    T(-e.qa2 * (e.cf * e.af * e.bz * e.s))};
    const T alu = al(2), all = al(4);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      T dF[6], dq[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) { dF[j] = dl(j, k); dq[j] = dl(7 + j, k); }
      T aF = A[0] * dF[0], aq = A[0] * dq[0];
#pragma unroll
      for (int j = 1; j < 4; ++j) { aF += A[j] * dF[j]; aq += A[j] * dq[j]; }
      split_k(k, cW * WF[k] + (cBy * dF[4] + cBz * dF[5]), cW * Wq[k] + (cBy * dq[4] + cBz * dq[5]), aF, aq, alu,
              all);
      sched_fence();
    }
    const double fu = double(weno_split<WENO_Z>(vu, eps, epsZ, lit));
    const double fl = double(weno_split<WENO_Z>(vl, eps, epsZ, lit));
    const double sp = fu + fl, sm = fu - fl;
    corr[0] += e.as * sp;
    corr[1] += e.as * e.vn * sp - e.as * e.csl * sm;
    corr[2] += e.as * e.vt1 * sp - e.cf * e.af * e.by * e.s * sm;
    corr[3] += e.as * e.vt2 * sp - e.cf * e.af * e.bz * e.s * sm;
    corr[4] += -e.cs * e.af * e.by * e.isr * sp;
    corr[5] += -e.cs * e.af * e.bz * e.isr * sp;
    corr[6] += e.as * (0.5 * e.v2 + e.csl2 - e.g2 * e.a2) * sp - e.Gs * sm;
  }
  sched_fence();
  // ---- entropy (m = 4): L = (1 - tau v^2/2, tau v, tau B_t, -tau), times 1/2, = e0/2 - 2 qa2 W
  {
    const T cE = T(-2.0 * e.qa2);
    const T a4 = al(3);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const T sF = T(0.5) * dl(0, k) + cE * WF[k], sq = T(0.5) * dl(7, k) + cE * Wq[k];
      if (k <= 3) vu[k] = sF + a4 * sq;
      if (k >= 1) vu[3 + k] = sF - a4 * sq;
      sched_fence();
    }
    const double f4 = double(weno_split<WENO_Z>(vu, eps, epsZ, lit));
    corr[0] += f4;
    corr[1] += e.vn * f4;
    corr[2] += e.vt1 * f4;
    corr[3] += e.vt2 * f4;
    corr[6] += 0.5 * e.v2 * f4;
  }
  sched_fence();
  // ---- Alfven pair (m = 2, 6): L = (Ga/2, 0, -bz s/2, by s/2, -+sr bz/2, +-sr by/2, 0)
  {
    const T S0 = T(0.25 * e.Ga), S2 = T(-0.25 * e.bz * e.s), S3 = T(0.25 * e.by * e.s);
    const T A4 = T(-0.25 * e.sr * e.bz), A5 = T(0.25 * e.sr * e.by);
    const T alu = al(1), all = al(5);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const T sF = S0 * dl(0, k) + S2 * dl(2, k) + S3 * dl(3, k);
      const T sq = S0 * dl(7, k) + S2 * dl(9, k) + S3 * dl(10, k);
      const T aF = A4 * dl(4, k) + A5 * dl(5, k);
      const T aq = A4 * dl(11, k) + A5 * dl(12, k);
      split_k(k, sF, sq, aF, aq, alu, all);
      sched_fence();
    }
    const double fu = double(weno_split<WENO_Z>(vu, eps, epsZ, lit));
    const double fl = double(weno_split<WENO_Z>(vl, eps, epsZ, lit));
    const double sp = fu + fl, sm = fu - fl;
    corr[2] += -e.bz * e.s * sp;
    corr[3] += e.by * e.s * sp;
    corr[4] += -e.bz * e.isr * sm;
    corr[5] += e.by * e.isr * sm;
    corr[6] += -e.Ga * sp;
  }
}

}  // namespace wm
