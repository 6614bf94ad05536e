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
  int weno_z;       // 0: Jiang-Shu weights, 1: WENO-Z
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

// Zone prologue of a sweep (step 2 of the 3D step list): primitives (eq. P),
// the flux along n (eq. fluxes, total pressure P + |B|^2/2), and the fast,
// Alfven and slow speeds.  Inputs are in the sweep frame (n, t1, t2).
struct ZoneVals {
  double v[Z_NVAR];
};

__host__ __device__ __forceinline__ void zone_prologue(double rho, double mn, double mt1, double mt2, double E,
                                              double Bn, double Bt1, double Bt2, double gamma,
                                              double* out) {
  const double irho = 1.0 / rho;
  const double vn = mn * irho, vt1 = mt1 * irho, vt2 = mt2 * irho;
  const double Bperp2 = Bt1 * Bt1 + Bt2 * Bt2;
  const double B2 = Bn * Bn + Bperp2;
  const double P = (gamma - 1.0) * (E - 0.5 * ((mn * vn + mt1 * vt1 + mt2 * vt2) + B2));
  const double Pstar = P + 0.5 * B2;
  const double vB = vn * Bn + vt1 * Bt1 + vt2 * Bt2;
  out[Z_RHO] = rho; out[Z_MN] = mn; out[Z_MT1] = mt1; out[Z_MT2] = mt2;
  out[Z_BT1] = Bt1; out[Z_BT2] = Bt2; out[Z_E] = E;
  out[Z_F0] = rho * vn;
  out[Z_F1] = rho * vn * vn + Pstar - Bn * Bn;
  out[Z_F2] = rho * vn * vt1 - Bn * Bt1;
  out[Z_F3] = rho * vn * vt2 - Bn * Bt2;
  out[Z_F4] = Bt1 * vn - Bn * vt1;
  out[Z_F5] = Bt2 * vn - Bn * vt2;
  out[Z_F6] = (E + Pstar) * vn - Bn * vB;
  out[Z_VN] = vn; out[Z_VT1] = vt1; out[Z_VT2] = vt2; out[Z_BN] = Bn; out[Z_P] = P;
  // c_f,s^2 = (a^2 + b^2 +- D)/2, D = sqrt((a^2 - b^2)^2 + 4 a^2 b_perp^2),
  // c_slow^2 = a^2 b_n^2 / c_fast^2 (no cancellation), c_A = |B_n|/sqrt(rho)
  const double a2 = gamma * P * irho;
  const double b2 = B2 * irho;
  const double bn2 = Bn * Bn * irho;
  const double dab = a2 - b2;
  const double D = sqrt(dab * dab + 4.0 * a2 * (Bperp2 * irho));
  const double cf2 = 0.5 * (a2 + b2 + D);
  const double cs2 = cf2 > 0.0 ? a2 * bn2 / cf2 : 0.0;
  out[Z_CF] = sqrt(cf2);
  out[Z_CA] = sqrt(bn2);
  out[Z_CS] = sqrt(cs2);
}

// WENO5 interpolant phi_N(a, b, c, d) of Sect. 2.2.  With s_k = eps + IS_k the
// Jiang-Shu weights alpha_k = d_k / s_k^2 give
//   omega_0 = s1^2 s2^2 / Q,  omega_2 = 3 s0^2 s1^2 / Q,
//   Q = s1^2 s2^2 + 6 s0^2 s2^2 + 3 s0^2 s1^2,
// one division instead of four.  WENO-Z: alpha_k = d_k (1 + (tau_5/(eps_Z + IS_k))^2).
template <bool WENO_Z>
__host__ __device__ __forceinline__ double phiN(double a, double b, double c, double d, double eps, double eps_Z) {
  const double t0 = a - b, t1 = a - 3.0 * b;
  const double t2 = b - c, t3 = b + c;
  const double t4 = c - d, t5 = 3.0 * c - d;
  const double IS0 = 13.0 * t0 * t0 + 3.0 * t1 * t1;
  const double IS1 = 13.0 * t2 * t2 + 3.0 * t3 * t3;
  const double IS2 = 13.0 * t4 * t4 + 3.0 * t5 * t5;
  double w0, w2;
  if (!WENO_Z) {
    double s0 = eps + IS0, s1 = eps + IS1, s2 = eps + IS2;
    s0 *= s0; s1 *= s1; s2 *= s2;
    const double p12 = s1 * s2, p02 = s0 * s2, p01 = s0 * s1;
    const double inv = 1.0 / (p12 + 6.0 * p02 + 3.0 * p01);
    w0 = p12 * inv;
    w2 = 3.0 * p01 * inv;
  } else {
    const double tau5 = fabs(IS0 - IS2);
    const double r0 = tau5 / (eps_Z + IS0), r1 = tau5 / (eps_Z + IS1), r2 = tau5 / (eps_Z + IS2);
    const double al0 = 1.0 + r0 * r0, al1 = 6.0 * (1.0 + r1 * r1), al2 = 3.0 * (1.0 + r2 * r2);
    const double inv = 1.0 / (al0 + al1 + al2);
    w0 = al0 * inv;
    w2 = al2 * inv;
  }
  return w0 * (a - 2.0 * b + c) * (1.0 / 3.0) + (w2 - 0.5) * (b - 2.0 * c + d) * (1.0 / 6.0);
}

// phi^- - phi^+ of eq. (FWENO) for one characteristic field, from the projected
// differences pF[k], pq[k] at interfaces i-3/2 .. i+5/2 and the LF speed alpha.
template <bool WENO_Z>
__host__ __device__ __forceinline__ double weno_char(const double pF[5], const double pq[5], double alpha,
                                            double eps, double eps_Z) {
  double p0 = 0.5 * (pF[0] + alpha * pq[0]);
  double p1 = 0.5 * (pF[1] + alpha * pq[1]);
  double p2 = 0.5 * (pF[2] + alpha * pq[2]);
  double p3 = 0.5 * (pF[3] + alpha * pq[3]);
  double n1 = 0.5 * (pF[1] - alpha * pq[1]);
  double n2 = 0.5 * (pF[2] - alpha * pq[2]);
  double n3 = 0.5 * (pF[3] - alpha * pq[3]);
  double n4 = 0.5 * (pF[4] - alpha * pq[4]);
  return phiN<WENO_Z>(n4, n3, n2, n1, eps, eps_Z) - phiN<WENO_Z>(p0, p1, p2, p3, eps, eps_Z);
}

// Dot products of a row with the five differences of F and of q.
__host__ __device__ __forceinline__ void project7(const double l[7], const double dF[5][7], const double dq[5][7],
                                         double pF[5], double pq[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double sF = l[0] * dF[k][0], sq = l[0] * dq[k][0];
#pragma unroll
    for (int j = 1; j < 7; ++j) {
      sF += l[j] * dF[k][j];
      sq += l[j] * dq[k][j];
    }
    pF[k] = sF;
    pq[k] = sq;
  }
}

// Projections with a row split into its sign-even part S (full) and sign-odd
// part A (nonzero in components 0..3 only): rows S + A and S - A at once.
__host__ __device__ __forceinline__ void project_pair(const double S[7], const double A[4], const double dF[5][7],
                                             const double dq[5][7], double pFu[5], double pqu[5],
                                             double pFl[5], double pql[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double sF = S[0] * dF[k][0], sq = S[0] * dq[k][0];
#pragma unroll
    for (int j = 1; j < 7; ++j) {
      sF += S[j] * dF[k][j];
      sq += S[j] * dq[k][j];
    }
    double aF = A[0] * dF[k][0], aq = A[0] * dq[k][0];
#pragma unroll
    for (int j = 1; j < 4; ++j) {
      aF += A[j] * dF[k][j];
      aq += A[j] * dq[k][j];
    }
    pFu[k] = sF + aF; pqu[k] = sq + aq;
    pFl[k] = sF - aF; pql[k] = sq - aq;
  }
}

// Characteristic part of the WENO interface flux at face i+1/2:
//   corr = sum_m R(:,m) (phi^-_m - phi^+_m)
// so that F_{i+1/2} = F_c + corr with the central term F_c taken in physical
// space (R L = I), eq. (FWENO).  The face state is the mean of the primitive
// states of zones i and i+1 (arithmetic averaging, Sect. 2.2 / Appendix A);
// L and R follow Appendix A with m = 1, 2, 3 the upper signs and 7, 6, 5 the
// lower, m = 2, 6 Alfven and m = 3, 5 slow.
//
// Inputs: face primitives, zone speeds of zones i and i+1 for alpha(m), and
// the differences dF[k], dq[k] across interfaces i-3/2 .. i+5/2.
template <bool WENO_Z>
__host__ __device__ __forceinline__ void face_char_flux(
    double rho, double vn, double vt1, double vt2, double Bn, double Bt1, double Bt2, double P,
    double vnL, double cfL, double cAL, double csL, double vnR, double cfR, double cAR, double csR,
    const double dF[5][7], const double dq[5][7], const Phys& ph, double corr[7]) {
  const double gamma = ph.gamma;
  const double irho = 1.0 / rho;
  const double a2 = gamma * P * irho;
  const double cs = sqrt(a2);
  const double sr = sqrt(rho);
  const double isr = 1.0 / sr;
  const double Bperp2 = Bt1 * Bt1 + Bt2 * Bt2;
  const double b2 = (Bn * Bn + Bperp2) * irho;
  const double dab = a2 - b2;
  const double D = sqrt(dab * dab + 4.0 * a2 * (Bperp2 * irho));
  const double cf2 = 0.5 * (a2 + b2 + D);
  const double cf = sqrt(cf2);
  const double csl2 = cf2 > 0.0 ? a2 * (Bn * Bn * irho) / cf2 : 0.0;
  const double csl = sqrt(csl2);
  double by, bz;
  if (Bperp2 > ph.eps_B) {
    const double ib = 1.0 / sqrt(Bperp2);
    by = Bt1 * ib;
    bz = Bt2 * ib;
  } else {
    by = 0.70710678118654752440;
    bz = 0.70710678118654752440;
  }
  const double s = Bn >= ph.eps_B ? 1.0 : -1.0;
  double af, as;
  if (sqrt(D) >= ph.eps_B) {
    const double r = dab / D;
    af = sqrt(fmin(fmax(0.5 * (1.0 + r), 0.0), 1.0));
    as = sqrt(fmin(fmax(0.5 * (1.0 - r), 0.0), 1.0));
  } else {
    af = 0.70710678118654752440;
    as = 0.70710678118654752440;
  }
  const double g1 = 0.5 * (gamma - 1.0);
  const double g2 = (gamma - 2.0) / (gamma - 1.0);
  const double omg = 1.0 - gamma;
  const double ha2 = 0.5 / a2;
  const double tau = (gamma - 1.0) / a2;
  const double v2 = vn * vn + vt1 * vt1 + vt2 * vt2;
  const double bv = by * vt1 + bz * vt2;
  const double Gf = af * cf * vn - as * csl * s * bv;
  const double Ga = s * (bz * vt1 - by * vt2);
  const double Gs = as * csl * vn + af * cf * s * bv;
  const double sra = sr * cs;

  double pFu[5], pqu[5], pFl[5], pql[5];
  double fu, fl;   // phi^- - phi^+ of the upper / lower member of a pair

  // ---- fast pair, m = 1 (v - c_fast) and m = 7 (v + c_fast)
  {
    const double S[7] = {ha2 * (af * g1 * v2), ha2 * (omg * af * vn), ha2 * (omg * af * vt1),
                         ha2 * (omg * af * vt2), ha2 * (omg * af * Bt1 + sra * as * by),
                         ha2 * (omg * af * Bt2 + sra * as * bz), ha2 * ((gamma - 1.0) * af)};
    const double A[4] = {ha2 * Gf, -ha2 * (af * cf), ha2 * (csl * as * by * s), ha2 * (csl * as * bz * s)};
    project_pair(S, A, dF, dq, pFu, pqu, pFl, pql);
    const double alu = fmax(fabs(vnL - cfL), fabs(vnR - cfR));
    const double all = fmax(fabs(vnL + cfL), fabs(vnR + cfR));
    fu = weno_char<WENO_Z>(pFu, pqu, alu, ph.eps, ph.eps_Z);
    fl = weno_char<WENO_Z>(pFl, pql, all, ph.eps, ph.eps_Z);
    const double sp = fu + fl, sm = fu - fl;
    const double Rs6 = af * (0.5 * v2 + cf2 - g2 * a2);
    corr[0] = af * sp;
    corr[1] = af * vn * sp - af * cf * sm;
    corr[2] = af * vt1 * sp + csl * as * by * s * sm;
    corr[3] = af * vt2 * sp + csl * as * bz * s * sm;
    corr[4] = cs * as * by * isr * sp;
    corr[5] = cs * as * bz * isr * sp;
    corr[6] = Rs6 * sp - Gf * sm;
  }
  // ---- Alfven pair, m = 2 (v - c_A) and m = 6 (v + c_A)
  {
    const double S[4] = {0.5 * Ga, 0.0, -0.5 * bz * s, 0.5 * by * s};
    const double A4 = -0.5 * sr * bz, A5 = 0.5 * sr * by;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double sF = S[0] * dF[k][0] + S[2] * dF[k][2] + S[3] * dF[k][3];
      const double sq = S[0] * dq[k][0] + S[2] * dq[k][2] + S[3] * dq[k][3];
      const double aF = A4 * dF[k][4] + A5 * dF[k][5];
      const double aq = A4 * dq[k][4] + A5 * dq[k][5];
      pFu[k] = sF + aF; pqu[k] = sq + aq;
      pFl[k] = sF - aF; pql[k] = sq - aq;
    }
    const double alu = fmax(fabs(vnL - cAL), fabs(vnR - cAR));
    const double all = fmax(fabs(vnL + cAL), fabs(vnR + cAR));
    fu = weno_char<WENO_Z>(pFu, pqu, alu, ph.eps, ph.eps_Z);
    fl = weno_char<WENO_Z>(pFl, pql, all, ph.eps, ph.eps_Z);
    const double sp = fu + fl, sm = fu - fl;
    corr[2] += -bz * s * sp;
    corr[3] += by * s * sp;
    corr[4] += -bz * isr * sm;
    corr[5] += by * isr * sm;
    corr[6] += -Ga * sp;
  }
  // ---- slow pair, m = 3 (v - c_slow) and m = 5 (v + c_slow)
  {
    const double S[7] = {ha2 * (as * g1 * v2), ha2 * (omg * as * vn), ha2 * (omg * as * vt1),
                         ha2 * (omg * as * vt2), ha2 * (omg * as * Bt1 - sra * af * by),
                         ha2 * (omg * as * Bt2 - sra * af * bz), ha2 * ((gamma - 1.0) * as)};
    const double A[4] = {ha2 * Gs, -ha2 * (as * csl), -ha2 * (cf * af * by * s), -ha2 * (cf * af * bz * s)};
    project_pair(S, A, dF, dq, pFu, pqu, pFl, pql);
    const double alu = fmax(fabs(vnL - csL), fabs(vnR - csR));
    const double all = fmax(fabs(vnL + csL), fabs(vnR + csR));
    fu = weno_char<WENO_Z>(pFu, pqu, alu, ph.eps, ph.eps_Z);
    fl = weno_char<WENO_Z>(pFl, pql, all, ph.eps, ph.eps_Z);
    const double sp = fu + fl, sm = fu - fl;
    const double Rs6 = as * (0.5 * v2 + csl2 - g2 * a2);
    corr[0] += as * sp;
    corr[1] += as * vn * sp - as * csl * sm;
    corr[2] += as * vt1 * sp - cf * af * by * s * sm;
    corr[3] += as * vt2 * sp - cf * af * bz * s * sm;
    corr[4] += -cs * af * by * isr * sp;
    corr[5] += -cs * af * bz * isr * sp;
    corr[6] += Rs6 * sp - Gs * sm;
  }
  // ---- entropy, m = 4 (v)
  {
    const double l[7] = {1.0 - 0.5 * tau * v2, tau * vn, tau * vt1, tau * vt2, tau * Bt1, tau * Bt2, -tau};
    project7(l, dF, dq, pFu, pqu);
    const double al = fmax(fabs(vnL), fabs(vnR));
    const double f4 = weno_char<WENO_Z>(pFu, pqu, al, ph.eps, ph.eps_Z);
    corr[0] += f4;
    corr[1] += vn * f4;
    corr[2] += vt1 * f4;
    corr[3] += vt2 * f4;
    corr[6] += 0.5 * v2 * f4;
  }
}

}  // namespace wm
