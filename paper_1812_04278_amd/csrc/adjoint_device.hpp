// Reverse-mode (vector-Jacobian) counterparts of the per-zone and per-face
// computations of the WENO5-CT sweep, FP64, for the adjoint of a stage.
//
// Each *_vjp function recomputes what it needs of the forward pass and
// propagates a cotangent backwards through it.  Non-smooth points take the
// derivative of the branch the forward pass takes: max() of the Lax-Friedrichs
// speed follows the larger argument (ties: the first), |x| its sign (0 at 0),
// the clamps of alpha_f^2, alpha_s^2 and the degenerate constants of Appendix A
// (beta, sgn(B_n), alpha_f = alpha_s = 1/sqrt2) have zero derivative, and
// sqrt(0) contributes nothing.
#pragma once
#include "mhd_device.hpp"

namespace wm {

// ---------------------------------------------------------------------------
// phi_N: value and gradient with respect to its four arguments (Sect. 2.2).
// With omega = alpha/sum, g = X/3, h = Y/6 (X = a-2b+c, Y = b-2c+d) and
// W = g omega_0 + h omega_2, dphi/dalpha_k = (G_k - W)/sum, G = (g, 0, h).
// Jiang-Shu: s_k = eps + IS_k, alpha_k = d_k/s_k^2, so
//   dphi/ds_0 = (2 omega_0/s_0)(W - g), dphi/ds_1 = (2 omega_1/s_1) W,
//   dphi/ds_2 = (2 omega_2/s_2)(W - h).
// WENO-Z: alpha_k = d_k (1 + r_k^2), r_k = tau_5/(eps_Z + IS_k), tau_5 = |IS_0 - IS_2|.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// face eigen-system scalars: cotangents of the FaceEig members -> face state
// ---------------------------------------------------------------------------
// Materialises x in a register at this point of the program: the compiler may
// not sink the computation of x past it (without this, the terms of the
// cotangent sums below are kept live until their final use and spill).
__host__ __device__ __forceinline__ void pin(double& x) {
#ifdef __HIP_DEVICE_COMPILE__
  asm volatile("" : "+v"(x));
#else
  (void)x;
#endif
}

// Compiler-level memory clobber: loads after it are not merged with loads
// before it (re-reading the differences from LDS is cheaper than keeping them
// live in registers).
__host__ __device__ __forceinline__ void reload_fence() {
#ifdef __HIP_DEVICE_COMPILE__
  asm volatile("" ::: "memory");
#endif
}

struct FaceEigBar {
  double vn, vt1, vt2, Bt1, Bt2;
  double a2, cs, sr, isr, cf, cf2, csl, csl2;
  double by, bz, af, as;
  double v2, Gf, Ga, Gs, qa2, tau;
  __host__ __device__ void zero() {
    vn = vt1 = vt2 = Bt1 = Bt2 = a2 = cs = sr = isr = cf = cf2 = csl = csl2 = 0.0;
    by = bz = af = as = v2 = Gf = Ga = Gs = qa2 = tau = 0.0;
  }
  // pin_*: the members that the reverse of one pair writes
  __host__ __device__ __forceinline__ void pin_fast_slow_common() {
    pin(vn); pin(vt1); pin(vt2); pin(Bt1); pin(Bt2); pin(a2); pin(cs); pin(sr); pin(isr); pin(cf); pin(csl);
    pin(by); pin(bz); pin(af); pin(as); pin(v2); pin(qa2);
  }
  __host__ __device__ __forceinline__ void pin_fast() { pin_fast_slow_common(); pin(cf2); pin(Gf); }
  __host__ __device__ __forceinline__ void pin_slow() { pin_fast_slow_common(); pin(csl2); pin(Gs); }
  __host__ __device__ __forceinline__ void pin_alfven() { pin(bz); pin(by); pin(isr); pin(Ga); pin(sr); }
  __host__ __device__ __forceinline__ void pin_entropy() {
    pin(vn); pin(vt1); pin(vt2); pin(v2); pin(Bt1); pin(Bt2); pin(tau);
  }
};

// Reverse of face_eig: out[0..7] += d/d(rho, vn, vt1, vt2, Bn, Bt1, Bt2, P).
__host__ __device__ __forceinline__ void face_eig_vjp(const double fp[8], const Phys& ph, const FaceEig& e,
                                                      FaceEigBar eb, double out[8]) {
  const double rho = fp[0], vn = fp[1], vt1 = fp[2], vt2 = fp[3], Bn = fp[4], Bt1 = fp[5], Bt2 = fp[6], P = fp[7];
  const double gamma = ph.gamma;
  const double isr = rsq_nr(rho);
  const double irho = isr * isr;
  const double a2 = e.a2;
  const double ia2 = rcp_w(a2);
  const double Bp2 = Bt1 * Bt1 + Bt2 * Bt2;
  const double b2 = (Bn * Bn + Bp2) * irho;
  const double dab = a2 - b2;
  const double p4 = 4.0 * a2 * (Bp2 * irho);   // as in face_eig
  const double Q = dab * dab + p4;
  const double D = sqrt_nr(Q);
  const double cf2 = 0.5 * (a2 + b2 + D);
  const double bv = e.by * vt1 + e.bz * vt2;
  const double s = e.s;
  double l_vn = eb.vn, l_vt1 = eb.vt1, l_vt2 = eb.vt2, l_Bt1 = eb.Bt1, l_Bt2 = eb.Bt2;
  double l_a2 = eb.a2, l_cf = eb.cf, l_cf2 = eb.cf2, l_csl = eb.csl, l_csl2 = eb.csl2;
  double l_by = eb.by, l_bz = eb.bz, l_af = eb.af, l_as = eb.as, l_v2 = eb.v2;
  double l_isr = eb.isr, l_sr = eb.sr, l_cs = eb.cs;
  double l_bv = 0.0, l_ia2 = 0.0, l_Bp2 = 0.0, l_b2 = 0.0, l_dab = 0.0, l_D = 0.0, l_irho = 0.0;
  double l_rho = 0.0, l_Bn = 0.0, l_P = 0.0;
  // Gs = as csl vn + af cf s bv
  l_as += eb.Gs * e.csl * vn; l_csl += eb.Gs * e.as * vn; l_vn += eb.Gs * e.as * e.csl;
  l_af += eb.Gs * e.cf * s * bv; l_cf += eb.Gs * e.af * s * bv; l_bv += eb.Gs * e.af * e.cf * s;
  // Ga = s (bz vt1 - by vt2)
  l_bz += eb.Ga * s * vt1; l_vt1 += eb.Ga * s * e.bz; l_by -= eb.Ga * s * vt2; l_vt2 -= eb.Ga * s * e.by;
  // Gf = af cf vn - as csl s bv
  l_af += eb.Gf * e.cf * vn; l_cf += eb.Gf * e.af * vn; l_vn += eb.Gf * e.af * e.cf;
  l_as -= eb.Gf * e.csl * s * bv; l_csl -= eb.Gf * e.as * s * bv; l_bv -= eb.Gf * e.as * e.csl * s;
  // bv = by vt1 + bz vt2
  l_by += l_bv * vt1; l_vt1 += l_bv * e.by; l_bz += l_bv * vt2; l_vt2 += l_bv * e.bz;
  // v2
  l_vn += 2.0 * vn * l_v2; l_vt1 += 2.0 * vt1 * l_v2; l_vt2 += 2.0 * vt2 * l_v2;
  // qa2 = ia2/4, tau = (gamma-1) ia2
  l_ia2 += 0.25 * eb.qa2 + (gamma - 1.0) * eb.tau;
  // alpha_f, alpha_s (non-degenerate branch, unclamped interior)
  if (D >= ph.eps_B * ph.eps_B) {
    const double iD = rcp_w(D);
    const double r = dab * iD;
    double cfa, csa;   // the forward's clamped alpha^2 (same arithmetic), for the interior test
    alpha_sq(dab, D, p4, cfa, csa);
    double l_r = 0.0;
    if (cfa > 0.0 && cfa < 1.0 && e.af > 0.0) l_r += l_af * 0.25 * rcp_w(e.af);
    if (csa > 0.0 && csa < 1.0 && e.as > 0.0) l_r -= l_as * 0.25 * rcp_w(e.as);
    l_dab += l_r * iD;
    l_D -= l_r * r * iD;
  }
  // beta
  if (Bp2 > ph.eps_B) {
    const double ib = rsq_nr(Bp2);
    l_Bt1 += l_by * ib;
    l_Bt2 += l_bz * ib;
    l_Bp2 -= 0.5 * ib * ib * ib * (l_by * Bt1 + l_bz * Bt2);
  }
  // csl = sqrt(csl2)
  if (e.csl > 0.0) l_csl2 += l_csl * 0.5 * rcp_w(e.csl);
  // csl2 = a2 Bn^2 irho / cf2
  if (cf2 > 0.0) {
    const double icf2 = rcp_w(cf2);
    const double lN = l_csl2 * icf2;
    l_cf2 -= l_csl2 * e.csl2 * icf2;
    l_a2 += lN * Bn * Bn * irho;
    l_Bn += lN * 2.0 * a2 * Bn * irho;
    l_irho += lN * a2 * Bn * Bn;
  }
  // cf = sqrt(cf2)
  if (e.cf > 0.0) l_cf2 += l_cf * 0.5 * rcp_w(e.cf);
  // cf2 = (a2 + b2 + D)/2
  l_a2 += 0.5 * l_cf2; l_b2 += 0.5 * l_cf2; l_D += 0.5 * l_cf2;
  // D = sqrt(dab^2 + 4 a2 Bp2 irho)
  if (D > 0.0) {
    const double lQ = l_D * 0.5 * rcp_w(D);
    l_dab += 2.0 * dab * lQ;
    l_a2 += 4.0 * Bp2 * irho * lQ;
    l_Bp2 += 4.0 * a2 * irho * lQ;
    l_irho += 4.0 * a2 * Bp2 * lQ;
  }
  // dab = a2 - b2
  l_a2 += l_dab; l_b2 -= l_dab;
  // b2 = (Bn^2 + Bp2) irho
  l_Bn += 2.0 * Bn * irho * l_b2; l_Bp2 += irho * l_b2; l_irho += (Bn * Bn + Bp2) * l_b2;
  // Bp2
  l_Bt1 += 2.0 * Bt1 * l_Bp2; l_Bt2 += 2.0 * Bt2 * l_Bp2;
  // ia2 = 1/a2, cs = sqrt(a2)
  l_a2 -= ia2 * ia2 * l_ia2;
  if (e.cs > 0.0) l_a2 += l_cs * 0.5 * rcp_w(e.cs);
  // a2 = gamma P irho
  l_P += gamma * irho * l_a2; l_irho += gamma * P * l_a2;
  // irho = isr^2, sr = rho isr, isr = rho^(-1/2)
  l_isr += 2.0 * isr * l_irho;
  l_rho += isr * l_sr; l_isr += rho * l_sr;
  l_rho -= 0.5 * isr * isr * isr * l_isr;
  out[0] += l_rho; out[1] += l_vn; out[2] += l_vt1; out[3] += l_vt2;
  out[4] += l_Bn; out[5] += l_Bt1; out[6] += l_Bt2; out[7] += l_P;
}

// ---------------------------------------------------------------------------
// phi = omega_0 X/3 + (omega_2 - 1/2) Y/6 and its gradient
// ---------------------------------------------------------------------------
template <bool WZ>
__host__ __device__ __forceinline__ void phiN_val_grad(double a, double b, double c, double d, double eps,
                                                       double epsZ, bool lit, double& val, double gr[4]) {
  const double t0 = a - b, t1 = a - 3.0 * b;
  const double t2 = b - c, t3 = b + c;
  const double t4 = c - d, t5 = 3.0 * c - d;
  const double X = t0 - t2, Y = t2 - t4;   // a - 2b + c, b - 2c + d
  const double g = X * (1.0 / 3.0), h = Y * (1.0 / 6.0);
  double w0, w2, l0, l1, l2;   // normalised weights 0, 2 and dphi/dIS_k
  if constexpr (!WZ) {
    (void)epsZ;
    (void)lit;
    const double s0 = eps + 13.0 * t0 * t0 + 3.0 * t1 * t1;
    const double s1 = eps + 13.0 * t2 * t2 + 3.0 * t3 * t3;
    const double s2 = eps + 13.0 * t4 * t4 + 3.0 * t5 * t5;
    // 1/s_k from one reciprocal of s0 s1 s2 (s_k >= eps, so the product stays normal)
    const double s12 = s1 * s2, r = rcp_w(s0 * s12);
    const double i0 = s12 * r, i1 = s0 * s2 * r, i2 = s0 * s1 * r;
    const double al0 = i0 * i0, al1 = 6.0 * i1 * i1, al2 = 3.0 * i2 * i2;
    const double isum = rcp_w(al0 + al1 + al2);
    w0 = al0 * isum;
    const double w1 = al1 * isum;
    w2 = al2 * isum;
    const double W = g * w0 + h * w2;
    l0 = 2.0 * w0 * i0 * (W - g);
    l1 = 2.0 * w1 * i1 * W;
    l2 = 2.0 * w2 * i2 * (W - h);
  } else {
    // WENO-Z: alpha_k = d_k (1 + u_k), q_k = 1/(eps_Z + IS_k), r_k = tau5 q_k, tau5 = |IS_0 - IS_2|,
    // u_k = r_k^2, or u_k = tau5 q_k^2 = r_k q_k as printed (`lit`).  Both give
    // du_k/dIS_k = -2 u_k q_k; du_k/dtau5 is 2 r_k q_k, or q_k^2 as printed.
    (void)eps;
    const double IS0 = 13.0 * t0 * t0 + 3.0 * t1 * t1;
    const double IS1 = 13.0 * t2 * t2 + 3.0 * t3 * t3;
    const double IS2 = 13.0 * t4 * t4 + 3.0 * t5 * t5;
    const double dIS = IS0 - IS2, tau = fabs(dIS);
    const double q0 = rcp_w(epsZ + IS0), q1 = rcp_w(epsZ + IS1), q2 = rcp_w(epsZ + IS2);
    const double r0 = tau * q0, r1 = tau * q1, r2 = tau * q2;
    const double s0 = lit ? q0 : r0, s1 = lit ? q1 : r1, s2 = lit ? q2 : r2;
    const double u0 = r0 * s0, u1 = r1 * s1, u2 = r2 * s2;
    const double al0 = 1.0 + u0, al1 = 6.0 * (1.0 + u1), al2 = 3.0 * (1.0 + u2);
    const double isum = rcp_w(al0 + al1 + al2);
    w0 = al0 * isum;
    w2 = al2 * isum;
    const double W = g * w0 + h * w2;
    // dphi/du_k = (G_k - W)/sum(alpha) * d_k, G = (g, 0, h)
    const double M0 = (g - W) * isum, M1 = -W * isum * 6.0, M2 = (h - W) * isum * 3.0;
    const double ct = lit ? 1.0 : 2.0;   // du_k/dtau5 = ct s_k q_k
    const double ltau = ct * (M0 * s0 * q0 + M1 * s1 * q1 + M2 * s2 * q2);   // dphi/dtau5
    const double sg = dIS > 0.0 ? 1.0 : (dIS < 0.0 ? -1.0 : 0.0);
    l0 = -2.0 * M0 * u0 * q0 + sg * ltau;
    l1 = -2.0 * M1 * u1 * q1;
    l2 = -2.0 * M2 * u2 * q2 - sg * ltau;
  }
  const double cX = w0 * (1.0 / 3.0), cY = (w2 - 0.5) * (1.0 / 6.0);
  val = cX * X + cY * Y;
  // dIS_0/da = 26 t0 + 6 t1, dIS_0/db = -26 t0 - 18 t1
  // dIS_1/db = 26 t2 + 6 t3, dIS_1/dc = -26 t2 + 6 t3
  // dIS_2/dc = 26 t4 + 18 t5, dIS_2/dd = -26 t4 - 6 t5
  gr[0] = cX + l0 * (26.0 * t0 + 6.0 * t1);
  gr[1] = -2.0 * cX + cY + l0 * (-26.0 * t0 - 18.0 * t1) + l1 * (26.0 * t2 + 6.0 * t3);
  gr[2] = cX - 2.0 * cY + l1 * (-26.0 * t2 + 6.0 * t3) + l2 * (26.0 * t4 + 18.0 * t5);
  gr[3] = cY + l2 * (-26.0 * t4 - 6.0 * t5);
}

// ---------------------------------------------------------------------------
// eigen pairs: forward and reverse in a single pass
// ---------------------------------------------------------------------------
// A pair has the left rows S + A (upper) and S - A (lower) with the
// Lax-Friedrichs speeds alu, all; S is nonzero on the components in SM, A on
// A0 .. A0+NA-1 (TWO = false: the single row S).  Split values as in
// face_corr; f = phi(v7, v6, v5, v4) - phi(v0, v1, v2, v3) per row.  The
// cotangents lfu, lfl of the two f only involve the right eigenvectors, so they
// are known before the pass, which computes f (needed for the right-vector
// cotangents) and the cotangents of S, A, the two speeds and the interface
// differences.
struct PairRows {
  double S[7], A[4];
  double alu, all;   // Lax-Friedrichs speeds of the upper / lower row
  double lfu, lfl;   // cotangents of f_upper, f_lower
};
struct PairCot {
  double fu = 0.0, fl = 0.0;                       // forward values
  double lS[7] = {0, 0, 0, 0, 0, 0, 0}, lA[4] = {0, 0, 0, 0};
  double lalu = 0.0, lall = 0.0;                   // cotangents of the speeds
};

template <int A0, int NA, bool TWO, int SM>
struct PairShape {
  // projections of the rows at one interface: d[0..6] Delta F, d[7..13] Delta q
  __host__ __device__ static __forceinline__ void proj(const PairRows& r, const double d[14], double& uF, double& uq,
                                                       double& lF, double& lq) {
    double sF = 0.0, sq = 0.0, aF = 0.0, aq = 0.0;
#pragma unroll
    for (int j = 0; j < 7; ++j)
      if (SM & (1 << j)) { sF += r.S[j] * d[j]; sq += r.S[j] * d[7 + j]; }
#pragma unroll
    for (int j = 0; j < NA; ++j) { aF += r.A[j] * d[A0 + j]; aq += r.A[j] * d[7 + A0 + j]; }
    uF = sF + aF; uq = sq + aq; lF = sF - aF; lq = sq - aq;
  }
  // cotangents of S, A from one interface (sFb = lP_u + lP_l, aFb = lP_u - lP_l, ...)
  __host__ __device__ static __forceinline__ void rowcot(const double d[14], double sFb, double aFb, double sqb,
                                                         double aqb, PairCot& c) {
#pragma unroll
    for (int j = 0; j < 7; ++j)
      if (SM & (1 << j)) c.lS[j] += sFb * d[j] + sqb * d[7 + j];
#pragma unroll
    for (int j = 0; j < NA; ++j) c.lA[j] += aFb * d[A0 + j] + aqb * d[7 + A0 + j];
  }
  // cotangent of the interface differences: lD += (S + A) lP_u + (S - A) lP_l (F and q parts)
  __host__ __device__ static __forceinline__ void difcot(const PairRows& r, double sFb, double aFb, double sqb,
                                                         double aqb, double lD[14]) {
#pragma unroll
    for (int j = 0; j < 7; ++j)
      if (SM & (1 << j)) { lD[j] += r.S[j] * sFb; lD[7 + j] += r.S[j] * sqb; }
#pragma unroll
    for (int j = 0; j < NA; ++j) { lD[A0 + j] += r.A[j] * aFb; lD[7 + A0 + j] += r.A[j] * aqb; }
  }
};

// Split values, phi and its gradient for one row: from the projections uF, uq
// (interfaces 0..4) to f and the cotangents lP (of uF), lQ (of uq) and of alpha.
template <bool WZ>
__host__ __device__ __forceinline__ void row_split_grad(const double uF[5], const double uq[5], double al, double lf,
                                                        double eps, double epsZ, bool lit, double& f, double lP[5],
                                                        double lQ[5], double& lal) {
  double v[8];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = uF[k] + al * uq[k];
#pragma unroll
  for (int k = 1; k < 5; ++k) v[3 + k] = uF[k] - al * uq[k];
  double g[8], g4[4], pa, pb;
  phiN_val_grad<WZ>(v[7], v[6], v[5], v[4], eps, epsZ, lit, pa, g4);
  g[7] = g4[0] * lf; g[6] = g4[1] * lf; g[5] = g4[2] * lf; g[4] = g4[3] * lf;
  phiN_val_grad<WZ>(v[0], v[1], v[2], v[3], eps, epsZ, lit, pb, g4);
  g[0] = -g4[0] * lf; g[1] = -g4[1] * lf; g[2] = -g4[2] * lf; g[3] = -g4[3] * lf;
  f = pa - pb;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double pk = k <= 3 ? g[k] : 0.0, mk = k >= 1 ? g[3 + k] : 0.0;
    lP[k] = pk + mk;
    lQ[k] = al * (pk - mk);
    lal += uq[k] * (pk - mk);
  }
}

// Forward and reverse of two pairs at once: one read of the differences per
// interface serves both, and one barrier round per interface carries both
// pairs' cotangents (emit(k, lD[14])).
template <class PA, bool TWOA, class PB, bool TWOB, bool WZ, class DL, class EMIT>
__host__ __device__ __forceinline__ void pair2_rev(const PairRows& ra, const PairRows& rb, DL dl, double eps,
                                                   double epsZ, bool lit, PairCot& ca, PairCot& cb, EMIT emit) {
  double uFa[5], uqa[5], lFa[5], lqa[5], uFb[5], uqb[5], lFb[5], lqb[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double d[14];
#pragma unroll
    for (int j = 0; j < 14; ++j) d[j] = dl(j, k);
    PA::proj(ra, d, uFa[k], uqa[k], lFa[k], lqa[k]);
    PB::proj(rb, d, uFb[k], uqb[k], lFb[k], lqb[k]);
    sched_fence();
  }
  double lPua[5], lQua[5], lPla[5], lQla[5], lPub[5], lQub[5], lPlb[5], lQlb[5];
  row_split_grad<WZ>(uFa, uqa, ra.alu, ra.lfu, eps, epsZ, lit, ca.fu, lPua, lQua, ca.lalu);
  if (TWOA) row_split_grad<WZ>(lFa, lqa, ra.all, ra.lfl, eps, epsZ, lit, ca.fl, lPla, lQla, ca.lall);
  row_split_grad<WZ>(uFb, uqb, rb.alu, rb.lfu, eps, epsZ, lit, cb.fu, lPub, lQub, cb.lalu);
  if (TWOB) row_split_grad<WZ>(lFb, lqb, rb.all, rb.lfl, eps, epsZ, lit, cb.fl, lPlb, lQlb, cb.lall);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    if (!TWOA) { lPla[k] = 0.0; lQla[k] = 0.0; }
    if (!TWOB) { lPlb[k] = 0.0; lQlb[k] = 0.0; }
  }
  // cotangents of the rows (a second read of the differences, no synchronisation) ...
  reload_fence();
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double d[14];
#pragma unroll
    for (int j = 0; j < 14; ++j) d[j] = dl(j, k);
    PA::rowcot(d, lPua[k] + lPla[k], lPua[k] - lPla[k], lQua[k] + lQla[k], lQua[k] - lQla[k], ca);
    PB::rowcot(d, lPub[k] + lPlb[k], lPub[k] - lPlb[k], lQub[k] + lQlb[k], lQub[k] - lQlb[k], cb);
    sched_fence();
  }
#pragma unroll
  for (int j = 0; j < 7; ++j) { pin(ca.lS[j]); pin(cb.lS[j]); }
#pragma unroll
  for (int j = 0; j < 4; ++j) { pin(ca.lA[j]); pin(cb.lA[j]); }
  // ... then those of the interface differences, one barrier-separated round per k
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double lD[14];
#pragma unroll
    for (int j = 0; j < 14; ++j) lD[j] = 0.0;
    PA::difcot(ra, lPua[k] + lPla[k], lPua[k] - lPla[k], lQua[k] + lQla[k], lQua[k] - lQla[k], lD);
    PB::difcot(rb, lPub[k] + lPlb[k], lPub[k] - lPlb[k], lQub[k] + lQlb[k], lQub[k] - lQlb[k], lD);
    emit(k, lD);
  }
}

// ---------------------------------------------------------------------------
// rows and right-vector cotangents of each pair (Appendix A), with the
// reverse of the row construction into the eigen-scalar cotangents eb
// ---------------------------------------------------------------------------
// fast pair (m = 1, 7): S = qa2 t, A = qa2 u
template <class ALF, class LAM>
__host__ __device__ __forceinline__ void fast_rows(const FaceEig& e, ALF alf, LAM lamf, PairRows& r) {
  const double gm1 = -e.omg, omg = e.omg, qa2 = e.qa2, sra = e.sr * e.cs, s = e.s;
  const double t[7] = {e.af * e.g1 * e.v2, omg * e.af * e.vn, omg * e.af * e.vt1, omg * e.af * e.vt2,
                       omg * e.af * e.Bt1 + sra * e.as * e.by, omg * e.af * e.Bt2 + sra * e.as * e.bz, gm1 * e.af};
  const double u[4] = {e.Gf, -(e.af * e.cf), e.csl * e.as * e.by * s, e.csl * e.as * e.bz * s};
#pragma unroll
  for (int j = 0; j < 7; ++j) r.S[j] = qa2 * t[j];
#pragma unroll
  for (int j = 0; j < 4; ++j) r.A[j] = qa2 * u[j];
  const double lam[7] = {lamf(0), lamf(1), lamf(2), lamf(3), lamf(4), lamf(5), lamf(6)};
  const double Rs6 = e.af * (0.5 * e.v2 + e.cf2 - e.g2 * e.a2);
  // corr[0..6] = af sp; af vn sp - af cf sm; af vt1 sp + csl as by s sm; af vt2 sp + csl as bz s sm;
  //              cs as by isr sp; cs as bz isr sp; Rs6 sp - Gf sm   (sp = fu + fl, sm = fu - fl)
  const double lsp = e.af * lam[0] + e.af * e.vn * lam[1] + e.af * e.vt1 * lam[2] + e.af * e.vt2 * lam[3] +
                     e.cs * e.as * e.isr * (e.by * lam[4] + e.bz * lam[5]) + Rs6 * lam[6];
  const double lsm = -e.af * e.cf * lam[1] + e.csl * e.as * s * (e.by * lam[2] + e.bz * lam[3]) - e.Gf * lam[6];
  r.lfu = lsp + lsm;
  r.lfl = lsp - lsm;
  r.alu = alf(0);
  r.all = alf(6);
}
template <class LAM>
__host__ __device__ __forceinline__ void fast_post(const FaceEig& e, LAM lamf, const PairCot& c, FaceEigBar& eb) {
  const double gm1 = -e.omg, omg = e.omg, qa2 = e.qa2, sra = e.sr * e.cs, s = e.s;
  const double t[7] = {e.af * e.g1 * e.v2, omg * e.af * e.vn, omg * e.af * e.vt1, omg * e.af * e.vt2,
                       omg * e.af * e.Bt1 + sra * e.as * e.by, omg * e.af * e.Bt2 + sra * e.as * e.bz, gm1 * e.af};
  const double u[4] = {e.Gf, -(e.af * e.cf), e.csl * e.as * e.by * s, e.csl * e.as * e.bz * s};
  const double lam[7] = {lamf(0), lamf(1), lamf(2), lamf(3), lamf(4), lamf(5), lamf(6)};
  const double sp = c.fu + c.fl, sm = c.fu - c.fl;
  eb.af += sp * (lam[0] + e.vn * lam[1] + e.vt1 * lam[2] + e.vt2 * lam[3] +
                 (0.5 * e.v2 + e.cf2 - e.g2 * e.a2) * lam[6]) - sm * e.cf * lam[1];
  eb.vn += e.af * sp * lam[1]; eb.vt1 += e.af * sp * lam[2]; eb.vt2 += e.af * sp * lam[3];
  eb.cf -= e.af * sm * lam[1];
  eb.cf2 += e.af * sp * lam[6]; eb.v2 += 0.5 * e.af * sp * lam[6]; eb.a2 -= e.g2 * e.af * sp * lam[6];
  eb.csl += sm * e.as * s * (e.by * lam[2] + e.bz * lam[3]);
  eb.as += sm * e.csl * s * (e.by * lam[2] + e.bz * lam[3]) + sp * e.cs * e.isr * (e.by * lam[4] + e.bz * lam[5]);
  eb.by += sm * e.csl * e.as * s * lam[2] + sp * e.cs * e.as * e.isr * lam[4];
  eb.bz += sm * e.csl * e.as * s * lam[3] + sp * e.cs * e.as * e.isr * lam[5];
  eb.cs += sp * e.as * e.isr * (e.by * lam[4] + e.bz * lam[5]);
  eb.isr += sp * e.cs * e.as * (e.by * lam[4] + e.bz * lam[5]);
  eb.Gf -= sm * lam[6];
  // rows S = qa2 t, A = qa2 u
  double lt[7], lu[4];
#pragma unroll
  for (int j = 0; j < 7; ++j) { eb.qa2 += c.lS[j] * t[j]; lt[j] = qa2 * c.lS[j]; }
#pragma unroll
  for (int j = 0; j < 4; ++j) { eb.qa2 += c.lA[j] * u[j]; lu[j] = qa2 * c.lA[j]; }
  eb.af += lt[0] * e.g1 * e.v2 + omg * (lt[1] * e.vn + lt[2] * e.vt1 + lt[3] * e.vt2 + lt[4] * e.Bt1 +
                                        lt[5] * e.Bt2) + gm1 * lt[6];
  eb.v2 += lt[0] * e.af * e.g1;
  eb.vn += lt[1] * omg * e.af; eb.vt1 += lt[2] * omg * e.af; eb.vt2 += lt[3] * omg * e.af;
  eb.Bt1 += lt[4] * omg * e.af; eb.Bt2 += lt[5] * omg * e.af;
  eb.sr += e.cs * e.as * (lt[4] * e.by + lt[5] * e.bz);
  eb.cs += e.sr * e.as * (lt[4] * e.by + lt[5] * e.bz);
  eb.as += sra * (lt[4] * e.by + lt[5] * e.bz);
  eb.by += sra * e.as * lt[4]; eb.bz += sra * e.as * lt[5];
  eb.Gf += lu[0];
  eb.af -= lu[1] * e.cf; eb.cf -= lu[1] * e.af;
  eb.csl += e.as * s * (lu[2] * e.by + lu[3] * e.bz);
  eb.as += e.csl * s * (lu[2] * e.by + lu[3] * e.bz);
  eb.by += e.csl * e.as * s * lu[2]; eb.bz += e.csl * e.as * s * lu[3];
}

// slow pair (m = 3, 5): S = qa2 t, A = qa2 u
template <class ALF, class LAM>
__host__ __device__ __forceinline__ void slow_rows(const FaceEig& e, ALF alf, LAM lamf, PairRows& r) {
  const double gm1 = -e.omg, omg = e.omg, qa2 = e.qa2, sra = e.sr * e.cs, s = e.s;
  const double t[7] = {e.as * e.g1 * e.v2, omg * e.as * e.vn, omg * e.as * e.vt1, omg * e.as * e.vt2,
                       omg * e.as * e.Bt1 - sra * e.af * e.by, omg * e.as * e.Bt2 - sra * e.af * e.bz, gm1 * e.as};
  const double u[4] = {e.Gs, -(e.as * e.csl), -(e.cf * e.af * e.by * s), -(e.cf * e.af * e.bz * s)};
#pragma unroll
  for (int j = 0; j < 7; ++j) r.S[j] = qa2 * t[j];
#pragma unroll
  for (int j = 0; j < 4; ++j) r.A[j] = qa2 * u[j];
  const double lam[7] = {lamf(0), lamf(1), lamf(2), lamf(3), lamf(4), lamf(5), lamf(6)};
  const double Rs6 = e.as * (0.5 * e.v2 + e.csl2 - e.g2 * e.a2);
  // corr += as sp; as vn sp - as csl sm; as vt1 sp - cf af by s sm; as vt2 sp - cf af bz s sm;
  //         -cs af by isr sp; -cs af bz isr sp; Rs6 sp - Gs sm
  const double lsp = e.as * lam[0] + e.as * e.vn * lam[1] + e.as * e.vt1 * lam[2] + e.as * e.vt2 * lam[3] -
                     e.cs * e.af * e.isr * (e.by * lam[4] + e.bz * lam[5]) + Rs6 * lam[6];
  const double lsm = -e.as * e.csl * lam[1] - e.cf * e.af * s * (e.by * lam[2] + e.bz * lam[3]) - e.Gs * lam[6];
  r.lfu = lsp + lsm;
  r.lfl = lsp - lsm;
  r.alu = alf(2);
  r.all = alf(4);
}
template <class LAM>
__host__ __device__ __forceinline__ void slow_post(const FaceEig& e, LAM lamf, const PairCot& c, FaceEigBar& eb) {
  const double gm1 = -e.omg, omg = e.omg, qa2 = e.qa2, sra = e.sr * e.cs, s = e.s;
  const double t[7] = {e.as * e.g1 * e.v2, omg * e.as * e.vn, omg * e.as * e.vt1, omg * e.as * e.vt2,
                       omg * e.as * e.Bt1 - sra * e.af * e.by, omg * e.as * e.Bt2 - sra * e.af * e.bz, gm1 * e.as};
  const double u[4] = {e.Gs, -(e.as * e.csl), -(e.cf * e.af * e.by * s), -(e.cf * e.af * e.bz * s)};
  const double lam[7] = {lamf(0), lamf(1), lamf(2), lamf(3), lamf(4), lamf(5), lamf(6)};
  const double sp = c.fu + c.fl, sm = c.fu - c.fl;
  eb.as += sp * (lam[0] + e.vn * lam[1] + e.vt1 * lam[2] + e.vt2 * lam[3] +
                 (0.5 * e.v2 + e.csl2 - e.g2 * e.a2) * lam[6]) - sm * e.csl * lam[1];
  eb.vn += e.as * sp * lam[1]; eb.vt1 += e.as * sp * lam[2]; eb.vt2 += e.as * sp * lam[3];
  eb.csl -= e.as * sm * lam[1];
  eb.csl2 += e.as * sp * lam[6]; eb.v2 += 0.5 * e.as * sp * lam[6]; eb.a2 -= e.g2 * e.as * sp * lam[6];
  eb.cf -= sm * e.af * s * (e.by * lam[2] + e.bz * lam[3]);
  eb.af -= sm * e.cf * s * (e.by * lam[2] + e.bz * lam[3]) + sp * e.cs * e.isr * (e.by * lam[4] + e.bz * lam[5]);
  eb.by -= sm * e.cf * e.af * s * lam[2] + sp * e.cs * e.af * e.isr * lam[4];
  eb.bz -= sm * e.cf * e.af * s * lam[3] + sp * e.cs * e.af * e.isr * lam[5];
  eb.cs -= sp * e.af * e.isr * (e.by * lam[4] + e.bz * lam[5]);
  eb.isr -= sp * e.cs * e.af * (e.by * lam[4] + e.bz * lam[5]);
  eb.Gs -= sm * lam[6];
  double lt[7], lu[4];
#pragma unroll
  for (int j = 0; j < 7; ++j) { eb.qa2 += c.lS[j] * t[j]; lt[j] = qa2 * c.lS[j]; }
#pragma unroll
  for (int j = 0; j < 4; ++j) { eb.qa2 += c.lA[j] * u[j]; lu[j] = qa2 * c.lA[j]; }
  eb.as += lt[0] * e.g1 * e.v2 + omg * (lt[1] * e.vn + lt[2] * e.vt1 + lt[3] * e.vt2 + lt[4] * e.Bt1 +
                                        lt[5] * e.Bt2) + gm1 * lt[6];
  eb.v2 += lt[0] * e.as * e.g1;
  eb.vn += lt[1] * omg * e.as; eb.vt1 += lt[2] * omg * e.as; eb.vt2 += lt[3] * omg * e.as;
  eb.Bt1 += lt[4] * omg * e.as; eb.Bt2 += lt[5] * omg * e.as;
  eb.sr -= e.cs * e.af * (lt[4] * e.by + lt[5] * e.bz);
  eb.cs -= e.sr * e.af * (lt[4] * e.by + lt[5] * e.bz);
  eb.af -= sra * (lt[4] * e.by + lt[5] * e.bz);
  eb.by -= sra * e.af * lt[4]; eb.bz -= sra * e.af * lt[5];
  eb.Gs += lu[0];
  eb.as -= lu[1] * e.csl; eb.csl -= lu[1] * e.as;
  eb.cf -= e.af * s * (lu[2] * e.by + lu[3] * e.bz);
  eb.af -= e.cf * s * (lu[2] * e.by + lu[3] * e.bz);
  eb.by -= e.cf * e.af * s * lu[2]; eb.bz -= e.cf * e.af * s * lu[3];
}

// Alfven pair (m = 2, 6): S = (Ga/4, 0, -bz s/4, by s/4, 0, 0, 0), A = (-sr bz/4, sr by/4) on components 4, 5
template <class ALF, class LAM>
__host__ __device__ __forceinline__ void alfven_rows(const FaceEig& e, ALF alf, LAM lamf, PairRows& r) {
  const double s = e.s;
  r.S[0] = 0.25 * e.Ga; r.S[1] = 0.0; r.S[2] = -0.25 * e.bz * s; r.S[3] = 0.25 * e.by * s;
  r.S[4] = 0.0; r.S[5] = 0.0; r.S[6] = 0.0;
  r.A[0] = -0.25 * e.sr * e.bz; r.A[1] = 0.25 * e.sr * e.by; r.A[2] = 0.0; r.A[3] = 0.0;
  // corr += (0, 0, -bz s sp, by s sp, -bz isr sm, by isr sm, -Ga sp)
  const double lsp = -e.bz * s * lamf(2) + e.by * s * lamf(3) - e.Ga * lamf(6);
  const double lsm = -e.bz * e.isr * lamf(4) + e.by * e.isr * lamf(5);
  r.lfu = lsp + lsm;
  r.lfl = lsp - lsm;
  r.alu = alf(1);
  r.all = alf(5);
}
template <class LAM>
__host__ __device__ __forceinline__ void alfven_post(const FaceEig& e, LAM lamf, const PairCot& c, FaceEigBar& eb) {
  const double s = e.s;
  const double lam2 = lamf(2), lam3 = lamf(3), lam4 = lamf(4), lam5 = lamf(5), lam6 = lamf(6);
  const double sp = c.fu + c.fl, sm = c.fu - c.fl;
  eb.bz += -s * sp * lam2 - e.isr * sm * lam4;
  eb.by += s * sp * lam3 + e.isr * sm * lam5;
  eb.isr += sm * (-e.bz * lam4 + e.by * lam5);
  eb.Ga -= sp * lam6;
  eb.Ga += 0.25 * c.lS[0];
  eb.bz += -0.25 * s * c.lS[2] - 0.25 * e.sr * c.lA[0];
  eb.by += 0.25 * s * c.lS[3] + 0.25 * e.sr * c.lA[1];
  eb.sr += -0.25 * e.bz * c.lA[0] + 0.25 * e.by * c.lA[1];
}

// entropy (m = 4): the single row L/2 = (1/2 - tau v^2/4, tau vn/2, tau vt1/2, tau vt2/2, tau Bt1/2, tau Bt2/2, -tau/2)
template <class ALF, class LAM>
__host__ __device__ __forceinline__ void entropy_rows(const FaceEig& e, ALF alf, LAM lamf, PairRows& r) {
  const double ht = 0.5 * e.tau;
  r.S[0] = 0.5 - 0.5 * ht * e.v2; r.S[1] = ht * e.vn; r.S[2] = ht * e.vt1; r.S[3] = ht * e.vt2;
  r.S[4] = ht * e.Bt1; r.S[5] = ht * e.Bt2; r.S[6] = -ht;
  r.A[0] = r.A[1] = r.A[2] = r.A[3] = 0.0;
  // corr += (f4, vn f4, vt1 f4, vt2 f4, 0, 0, v2/2 f4)
  r.lfu = lamf(0) + e.vn * lamf(1) + e.vt1 * lamf(2) + e.vt2 * lamf(3) + 0.5 * e.v2 * lamf(6);
  r.lfl = 0.0;
  r.alu = alf(3);
  r.all = r.alu;
}
template <class LAM>
__host__ __device__ __forceinline__ void entropy_post(const FaceEig& e, LAM lamf, const PairCot& c, FaceEigBar& eb) {
  const double ht = 0.5 * e.tau;
  const double f4 = c.fu;
  eb.vn += f4 * lamf(1); eb.vt1 += f4 * lamf(2); eb.vt2 += f4 * lamf(3); eb.v2 += 0.5 * f4 * lamf(6);
  const double lht = -0.5 * e.v2 * c.lS[0] + e.vn * c.lS[1] + e.vt1 * c.lS[2] + e.vt2 * c.lS[3] +
                     e.Bt1 * c.lS[4] + e.Bt2 * c.lS[5] - c.lS[6];
  eb.v2 -= 0.5 * ht * c.lS[0];
  eb.vn += ht * c.lS[1]; eb.vt1 += ht * c.lS[2]; eb.vt2 += ht * c.lS[3]; eb.Bt1 += ht * c.lS[4];
  eb.Bt2 += ht * c.lS[5];
  eb.tau += 0.5 * lht;
}

using FastShape = PairShape<0, 4, true, 127>;
using SlowShape = PairShape<0, 4, true, 127>;
using AlfvenShape = PairShape<4, 2, true, 13>;
using EntropyShape = PairShape<0, 0, false, 127>;

// Reverse of face_corr (FP64) at one face: given the eigen scalars e, the
// Lax-Friedrichs speeds alf(m), the differences dl and the cotangent lamf(j)
// of corr, accumulates the cotangents of the eigen scalars (eb), of the LF
// speeds (lal[7]) and, via emit (five rounds per group), of the interface
// differences.  The face-state cotangents follow from face_eig_vjp(eb).  The
// pairs run in two groups, fast with slow and Alfven with entropy.
template <bool WZ, class ALF, class LAM, class DL, class EMIT>
__host__ __device__ __forceinline__ void face_corr_vjp(const FaceEig& e, ALF alf, LAM lamf, DL dl, const Phys& ph,
                                                       FaceEigBar& eb, double lal[7], EMIT emit) {
  {
    PairRows rf, rs;
    fast_rows(e, alf, lamf, rf);
    slow_rows(e, alf, lamf, rs);
    PairCot cf, cs;
    pair2_rev<FastShape, true, SlowShape, true, WZ>(rf, rs, dl, ph.eps, ph.eps_Z, ph.weno_z == 2, cf, cs, emit);
    fast_post(e, lamf, cf, eb);
    slow_post(e, lamf, cs, eb);
    lal[0] += cf.lalu; lal[6] += cf.lall; lal[2] += cs.lalu; lal[4] += cs.lall;
  }
  eb.pin_fast();
  eb.pin_slow();
  pin(lal[0]); pin(lal[6]); pin(lal[2]); pin(lal[4]);
  sched_fence();
  {
    PairRows ra, rn;
    alfven_rows(e, alf, lamf, ra);
    entropy_rows(e, alf, lamf, rn);
    PairCot ca, cn;
    pair2_rev<AlfvenShape, true, EntropyShape, false, WZ>(ra, rn, dl, ph.eps, ph.eps_Z, ph.weno_z == 2, ca, cn, emit);
    alfven_post(e, lamf, ca, eb);
    entropy_post(e, lamf, cn, eb);
    lal[1] += ca.lalu; lal[5] += ca.lall; lal[3] += cn.lalu;
  }
  eb.pin_alfven();
  eb.pin_entropy();
  pin(lal[1]); pin(lal[5]); pin(lal[3]);
}

// ---------------------------------------------------------------------------
// zone prologue: cotangents of (q, F, primitives, speeds) -> zone inputs
// ---------------------------------------------------------------------------
// Inputs in the sweep frame: u = (rho, m_n, m_t1, m_t2, E, B_n, B_t1, B_t2).
// lz[Z_NVAR] are the cotangents of the prologue outputs; out[8] += d/du.
__host__ __device__ __forceinline__ void zone_prologue_vjp(const double u[8], double gamma, const double lz[Z_NVAR],
                                                  double out[8]) {
  const double rho = u[0], mn = u[1], mt1 = u[2], mt2 = u[3], E = u[4], Bn = u[5], Bt1 = u[6], Bt2 = u[7];
  const double irho = rcp_w(rho);
  const double vn = mn * irho, vt1 = mt1 * irho, vt2 = mt2 * irho;
  const double Bp2 = Bt1 * Bt1 + Bt2 * Bt2;
  const double B2 = Bn * Bn + Bp2;
  const double P = (gamma - 1.0) * (E - 0.5 * ((mn * vn + mt1 * vt1 + mt2 * vt2) + B2));
  const double Pstar = P + 0.5 * B2;
  const double vB = vn * Bn + vt1 * Bt1 + vt2 * Bt2;
  const double a2 = gamma * P * irho, b2 = B2 * irho, bn2 = Bn * Bn * irho;
  const double dab = a2 - b2;
  const double D = sqrt_nr(dab * dab + 4.0 * a2 * (Bp2 * irho));
  const double cf2 = 0.5 * (a2 + b2 + D);
  const double icf2 = cf2 > 0.0 ? rcp_w(cf2) : 0.0;
  const double cs2 = a2 * bn2 * icf2;
  const double cf = sqrt_nr(cf2), cA = sqrt_nr(bn2), cs = sqrt_nr(cs2);
  double l_rho = lz[Z_RHO], l_mn = lz[Z_MN], l_mt1 = lz[Z_MT1], l_mt2 = lz[Z_MT2];
  double l_Bt1 = lz[Z_BT1], l_Bt2 = lz[Z_BT2], l_E = lz[Z_E];
  double l_vn = lz[Z_VN], l_vt1 = lz[Z_VT1], l_vt2 = lz[Z_VT2], l_Bn = lz[Z_BN], l_P = lz[Z_P];
  double l_cf2 = 0.0, l_cs2 = 0.0, l_bn2 = 0.0, l_a2 = 0.0, l_b2 = 0.0, l_D = 0.0, l_dab = 0.0;
  double l_irho = 0.0, l_Bp2 = 0.0, l_B2 = 0.0, l_Pstar = 0.0, l_vB = 0.0;
  // speeds
  if (cf > 0.0) l_cf2 += lz[Z_CF] * 0.5 * rcp_w(cf);
  if (cA > 0.0) l_bn2 += lz[Z_CA] * 0.5 * rcp_w(cA);
  if (cs > 0.0) l_cs2 += lz[Z_CS] * 0.5 * rcp_w(cs);
  if (cf2 > 0.0) {
    l_a2 += l_cs2 * bn2 * icf2;
    l_bn2 += l_cs2 * a2 * icf2;
    l_cf2 -= l_cs2 * cs2 * icf2;
  }
  l_a2 += 0.5 * l_cf2; l_b2 += 0.5 * l_cf2; l_D += 0.5 * l_cf2;
  if (D > 0.0) {
    const double lQ = l_D * 0.5 * rcp_w(D);
    l_dab += 2.0 * dab * lQ;
    l_a2 += 4.0 * Bp2 * irho * lQ;
    l_Bp2 += 4.0 * a2 * irho * lQ;
    l_irho += 4.0 * a2 * Bp2 * lQ;
  }
  l_a2 += l_dab; l_b2 -= l_dab;
  l_Bn += 2.0 * Bn * irho * l_bn2; l_irho += Bn * Bn * l_bn2;
  l_B2 += irho * l_b2; l_irho += B2 * l_b2;
  l_P += gamma * irho * l_a2; l_irho += gamma * P * l_a2;
  // fluxes
  const double F0 = lz[Z_F0], F1 = lz[Z_F1], F2 = lz[Z_F2], F3 = lz[Z_F3], F4 = lz[Z_F4], F5 = lz[Z_F5], F6 = lz[Z_F6];
  // F0 = rho vn
  l_rho += F0 * vn; l_vn += F0 * rho;
  // F1 = rho vn vn + Pstar - Bn Bn
  l_rho += F1 * vn * vn; l_vn += F1 * 2.0 * rho * vn; l_Pstar += F1; l_Bn -= F1 * 2.0 * Bn;
  // F2 = rho vn vt1 - Bn Bt1, F3 = rho vn vt2 - Bn Bt2
  l_rho += F2 * vn * vt1 + F3 * vn * vt2;
  l_vn += F2 * rho * vt1 + F3 * rho * vt2;
  l_vt1 += F2 * rho * vn; l_vt2 += F3 * rho * vn;
  l_Bn -= F2 * Bt1 + F3 * Bt2; l_Bt1 -= F2 * Bn; l_Bt2 -= F3 * Bn;
  // F4 = Bt1 vn - Bn vt1, F5 = Bt2 vn - Bn vt2
  l_Bt1 += F4 * vn; l_vn += F4 * Bt1 + F5 * Bt2; l_Bn -= F4 * vt1 + F5 * vt2; l_vt1 -= F4 * Bn;
  l_Bt2 += F5 * vn; l_vt2 -= F5 * Bn;
  // F6 = (E + Pstar) vn - Bn vB
  l_E += F6 * vn; l_Pstar += F6 * vn; l_vn += F6 * (E + Pstar); l_Bn -= F6 * vB; l_vB -= F6 * Bn;
  // vB = vn Bn + vt1 Bt1 + vt2 Bt2
  l_vn += l_vB * Bn; l_Bn += l_vB * vn; l_vt1 += l_vB * Bt1; l_Bt1 += l_vB * vt1; l_vt2 += l_vB * Bt2;
  l_Bt2 += l_vB * vt2;
  // Pstar = P + B2/2
  l_P += l_Pstar; l_B2 += 0.5 * l_Pstar;
  // P = (gamma-1)(E - (mn vn + mt1 vt1 + mt2 vt2 + B2)/2)
  const double gm = gamma - 1.0;
  l_E += gm * l_P;
  l_mn -= 0.5 * gm * l_P * vn; l_vn -= 0.5 * gm * l_P * mn;
  l_mt1 -= 0.5 * gm * l_P * vt1; l_vt1 -= 0.5 * gm * l_P * mt1;
  l_mt2 -= 0.5 * gm * l_P * vt2; l_vt2 -= 0.5 * gm * l_P * mt2;
  l_B2 -= 0.5 * gm * l_P;
  // B2 = Bn^2 + Bp2, Bp2 = Bt1^2 + Bt2^2
  l_Bn += 2.0 * Bn * l_B2; l_Bp2 += l_B2;
  l_Bt1 += 2.0 * Bt1 * l_Bp2; l_Bt2 += 2.0 * Bt2 * l_Bp2;
  // v = m irho
  l_mn += l_vn * irho; l_mt1 += l_vt1 * irho; l_mt2 += l_vt2 * irho;
  l_irho += l_vn * mn + l_vt1 * mt1 + l_vt2 * mt2;
  // irho = 1/rho
  l_rho -= irho * irho * l_irho;
  out[0] += l_rho; out[1] += l_mn; out[2] += l_mt1; out[3] += l_mt2;
  out[4] += l_E; out[5] += l_Bn; out[6] += l_Bt1; out[7] += l_Bt2;
}

}  // namespace wm
