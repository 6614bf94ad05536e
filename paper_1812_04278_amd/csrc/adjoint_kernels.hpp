// HIP kernels of the adjoint (vector-Jacobian product) of the semi-discrete
// right-hand side and of the SSP-RK3 stage map, FP64.
//
//   adj_emf_kernel       cotangent of the face-b right-hand side -> cotangents
//                        of the six transport fluxes (transposes of the b
//                        equations of Sect. 2.3 and of eq. ox1-ox3)
//   adj_sweep_kernel     one direction: recomputes the tile's forward data,
//                        runs the per-face reverse (adjoint_device.hpp) and
//                        the per-zone prologue reverse, and adds the zone
//                        cotangents of every zone its faces touch (own zones
//                        and the halo zones of the neighbouring tiles); the
//                        tiles of one launch touch disjoint zones
//   adj_bcell_kernel     face-b cotangent += transpose of the fourth-order
//                        zone interpolation
//   adj_glue kernels     the RK3 stage combinations
//   init_adj kernels     transpose of the initial-state map (curl_h A, m, E)
// Accumulation orders are fixed (LDS sub-rounds separated by barriers, no
// atomics), so results are bitwise reproducible.
#pragma once
#include <hip/hip_runtime.h>

#include "adjoint_device.hpp"
#include "kernels.hpp"

namespace wm {

// ---------------------------------------------------------------------------
// b equations and corner fluxes, transposed
// ---------------------------------------------------------------------------
// Forward (update_kernel): rhs_bx = -(Ez - Ez[j-1])/h + (Ey - Ey[k-1])/h,
// rhs_by = -(Ex - Ex[k-1])/h + (Ez - Ez[i-1])/h, rhs_bz = -(Ey - Ey[i-1])/h +
// (Ex - Ex[j-1])/h with Ez = (Tyx + Tyx[i+1])/2 - (Txy + Txy[j+1])/2,
// Ex = (Tzy + Tzy[j+1])/2 - (Tyz + Tyz[k+1])/2, Ey = (Txz + Txz[k+1])/2 - (Tzx + Tzx[i+1])/2.
// It also clears zero3 ([3][N], the zone-B cotangent that the sweeps then add into).
__global__ __launch_bounds__(256) void adj_emf_kernel(Grid g, double inv_h, const double* lam_k, double* lam_T,
                                                      double* zero3) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const size_t N = g.N;
  {
    const size_t c = g.at(i, j, k);
    zero3[c] = 0.0;
    zero3[N + c] = 0.0;
    zero3[2 * N + c] = 0.0;
  }
  const double* lbx = lam_k + 5 * N;
  const double* lby = lam_k + 6 * N;
  const double* lbz = lam_k + 7 * N;
  const int im = wrap(i - 1, g.nx), ip = wrap(i + 1, g.nx);
  const int jm = wrap(j - 1, g.ny), jp = wrap(j + 1, g.ny);
  const int km = wrap(k - 1, g.nz), kp = wrap(k + 1, g.nz);
  // cotangents of the corner fluxes at edge index (ii, jj, kk)
  auto lEz = [&](int ii, int jj, int kk) {
    const int jjp = wrap(jj + 1, g.ny), iip = wrap(ii + 1, g.nx);
    return (-lbx[g.at(ii, jj, kk)] + lbx[g.at(ii, jjp, kk)] + lby[g.at(ii, jj, kk)] - lby[g.at(iip, jj, kk)]) * inv_h;
  };
  auto lEx = [&](int ii, int jj, int kk) {
    const int kkp = wrap(kk + 1, g.nz), jjp = wrap(jj + 1, g.ny);
    return (-lby[g.at(ii, jj, kk)] + lby[g.at(ii, jj, kkp)] + lbz[g.at(ii, jj, kk)] - lbz[g.at(ii, jjp, kk)]) * inv_h;
  };
  auto lEy = [&](int ii, int jj, int kk) {
    const int kkp = wrap(kk + 1, g.nz), iip = wrap(ii + 1, g.nx);
    return (lbx[g.at(ii, jj, kk)] - lbx[g.at(ii, jj, kkp)] - lbz[g.at(ii, jj, kk)] + lbz[g.at(iip, jj, kk)]) * inv_h;
  };
  (void)ip; (void)jp; (void)kp;
  const size_t c0 = g.at(i, j, k);
  const double ez = lEz(i, j, k), ex = lEx(i, j, k), ey = lEy(i, j, k);
  // T layout: [0] Txy, [1] Txz, [2] Tyz, [3] Tyx, [4] Tzx, [5] Tzy
  lam_T[0 * N + c0] = -0.5 * (ez + lEz(i, jm, k));   // Txy feeds Ez(j) and Ez(j-1)
  lam_T[1 * N + c0] = 0.5 * (ey + lEy(i, j, km));    // Txz feeds Ey(k) and Ey(k-1)
  lam_T[2 * N + c0] = -0.5 * (ex + lEx(i, j, km));   // Tyz feeds Ex(k) and Ex(k-1)
  lam_T[3 * N + c0] = 0.5 * (ez + lEz(im, j, k));    // Tyx feeds Ez(i) and Ez(i-1)
  lam_T[4 * N + c0] = -0.5 * (ey + lEy(im, j, k));   // Tzx feeds Ey(i) and Ey(i-1)
  lam_T[5 * N + c0] = 0.5 * (ex + lEx(i, jm, k));    // Tzy feeds Ex(j) and Ex(j-1)
}

// ---------------------------------------------------------------------------
// adjoint of one directional sweep
// ---------------------------------------------------------------------------
struct AdjSweepArgs {
  Grid g;
  Phys ph;
  double inv_h;
  const double* hydro;   // forward state [5][N]
  const double* bcell;   // its zone B [3][N]
  const double* lam_k;   // [8][N] cotangent of the right-hand side (hydro part used)
  const double* lam_T;   // [2][N] cotangent of this sweep's transport fluxes T^n_t1, T^n_t2
  double* lam_h;         // [5][N] += zone cotangents of rho, m_x, m_y, m_z, E
  double* lam_Bz;        // [3][N] += zone cotangents of the zone field B_x, B_y, B_z
  int tile0;             // tile index along the axis of block 0 of this launch
  int tstride;           // tile index step between consecutive blocks along the axis
};

constexpr int ADJ_NP = 11;   // cotangents of zone primitives and speeds (P_* order)
// One thread per face; one 256-face tile per CU (LDS), so one wave per SIMD
// with up to 512 registers per thread.
constexpr int ADJ_THREADS = 256;
// adjoint tiles: TA faces along the sweep axis times TB across it, TA * TB = ADJ_THREADS
template <int AXIS> struct AdjTile { static constexpr int TA = 16, TB = 16; };
template <> struct AdjTile<0> { static constexpr int TA = 64, TB = 4; };

template <int AXIS>
struct AdjLds {
  static constexpr int TA = AdjTile<AXIS>::TA, TB = AdjTile<AXIS>::TB;
  static constexpr int NC = (TA + SW_HL + SW_HR) * TB, NIF = (TA + 4) * TB, NF = TA * TB;
  static constexpr size_t bytes = sizeof(double) * (size_t)(SW_NQ * NC + SW_NP * NC + ADJ_NP * NC + SW_NQ * NIF + 7 * NF);
};

// One block: TA x TB faces of one plane.  Every zone that a face of the tile
// touches (positions 0 .. tav+4 along the axis) gets its cotangent added to
// lam_h / lam_Bz by exactly one thread of the block; positions that wrap onto the
// same zone (a tile that spans the whole axis) are summed first.  Blocks of
// one launch touch disjoint zones (the host launches the tiles of an axis in
// conflict-free classes), so the additions need no atomics and the order of
// accumulation is fixed.
template <int AXIS, bool WZ>
__global__ __launch_bounds__(ADJ_THREADS, 1) void adj_sweep_kernel(AdjSweepArgs a) {
  constexpr int TA = AdjTile<AXIS>::TA, TB = AdjTile<AXIS>::TB;
  constexpr int NA = TA + SW_HL + SW_HR;
  constexpr int NI = TA + 4;
  constexpr int NC = NA * TB;
  constexpr int NIF = NI * TB;
  constexpr int NF = TA * TB;
  // LDS: zone q/F (later the differences) | zone primitives and speeds | their
  //      cotangents | interface-difference cotangents | face flux cotangents
  __shared__ double Q[SW_NQ * NC];
  __shared__ double Pz[SW_NP * NC];
  __shared__ double PB[ADJ_NP * NC];
  __shared__ double LD[SW_NQ * NIF];
  __shared__ double LF[7 * NF];
  const Grid& g = a.g;
  const int nA = AXIS == 0 ? g.nx : (AXIS == 1 ? g.ny : g.nz);
  const int nB = AXIS == 0 ? g.ny : g.nx;
  const int a0 = (a.tile0 + blockIdx.x * a.tstride) * TA;
  const int b0 = blockIdx.y * TB;
  const int c = blockIdx.z;
  const int tav = min(TA, nA - a0);            // valid faces (and own zones) along the axis
  constexpr int CN = AXIS, CT1 = (AXIS + 1) % 3, CT2 = (AXIS + 2) % 3;
  auto cidx = [](int aa, int bb) { return AXIS == 0 ? bb * NA + aa : aa * TB + bb; };
  auto iidx = [](int ia, int bb) { return AXIS == 0 ? bb * NI + ia : ia * TB + bb; };
  auto fidx = [](int fa, int bb) { return AXIS == 0 ? bb * TA + fa : fa * TB + bb; };
  auto gindex = [&](int aa_global, int bb_global) {
    int i, j, k;
    if (AXIS == 0)      { i = aa_global; j = bb_global; k = c; }
    else if (AXIS == 1) { i = bb_global; j = aa_global; k = c; }
    else                { i = bb_global; j = c;         k = aa_global; }
    return g.at(i, j, k);
  };

  const int tid = threadIdx.x;                   // face of this thread
  // ---- (0) global loads first: the states of this thread's cells (the same
  //          cells it handles in (4), kept in registers) and the right-hand-side
  //          cotangents of its face, so that the latencies overlap
  int fa, fb;
  if (AXIS == 0) { fa = tid % TA; fb = tid / TA; }
  else           { fb = tid % TB; fa = tid / TB; }
  const bool valid = fa < tav && b0 + fb < nB;
  constexpr int NCELL = (NC + ADJ_THREADS - 1) / ADJ_THREADS;
  double uz[NCELL][8];   // sweep frame: rho, m_n, m_t1, m_t2, E, B_n, B_t1, B_t2
#pragma unroll
  for (int k = 0; k < NCELL; ++k) {
    const int cell = min(threadIdx.x + k * ADJ_THREADS, (unsigned)NC - 1);
    int aa, bb;
    if (AXIS == 0) { aa = cell % NA; bb = cell / NA; }
    else           { bb = cell % TB; aa = cell / TB; }
    const size_t gi = gindex(wrap(a0 - SW_HL + aa, nA), min(b0 + bb, nB - 1));
    const double m[3] = {a.hydro[g.N + gi], a.hydro[2 * g.N + gi], a.hydro[3 * g.N + gi]};
    const double B[3] = {a.bcell[gi], a.bcell[g.N + gi], a.bcell[2 * g.N + gi]};
    double* u = uz[k];
    u[0] = a.hydro[gi]; u[1] = m[CN]; u[2] = m[CT1]; u[3] = m[CT2]; u[4] = a.hydro[4 * g.N + gi];
    u[5] = B[CN]; u[6] = B[CT1]; u[7] = B[CT2];
  }
  double lk0[5], lk1[5], lT[2];
  {
    const int ia = wrap(a0 + fa, nA), ia1 = wrap(a0 + fa + 1, nA);
    const int ib = min(b0 + fb, nB - 1);
    const size_t g0 = gindex(ia, ib), g1 = gindex(ia1, ib);
#pragma unroll
    for (int v = 0; v < 5; ++v) { lk0[v] = a.lam_k[v * g.N + g0]; lk1[v] = a.lam_k[v * g.N + g1]; }
    lT[0] = a.lam_T[g0];
    lT[1] = a.lam_T[g.N + g0];
  }

  // ---- (1) forward zone prologue into LDS
#pragma unroll
  for (int k = 0; k < NCELL; ++k) {   // branch-free: surplus threads repeat the last cell (equal values)
    const int cell = min(threadIdx.x + k * ADJ_THREADS, (unsigned)NC - 1);
    const double* u = uz[k];
    double z[Z_NVAR];
    zone_prologue(u[0], u[1], u[2], u[3], u[4], u[5], u[6], u[7], a.ph.gamma, z);
#pragma unroll
    for (int v = 0; v < SW_NQ; ++v) Q[v * NC + cell] = z[v];
    const int pv[SW_NP] = {Z_RHO, Z_VN, Z_VT1, Z_VT2, Z_BN, Z_BT1, Z_BT2, Z_P, Z_CF, Z_CA, Z_CS};
#pragma unroll
    for (int v = 0; v < SW_NP; ++v) Pz[v * NC + cell] = z[pv[v]];
  }
  __syncthreads();

  // ---- (2) per face: own interface differences, incoming flux cotangents
  const int cL = cidx(fa + 2, fb), cR = cidx(fa + 3, fb);
  {
    // zone variables: q in Q rows 0..6, F in rows 7..13; differences: Delta F
    // in rows 0..6, Delta q in rows 7..13
    constexpr int NV = SW_NQ;
    auto src_row = [](int v) { return v < 7 ? v + 7 : v - 7; };
    auto dst_row = [](int v) { return v; };
    double d0[NV], d1[NV];
    {
      const int c0 = cidx(fa, fb), c1 = cidx(fa + 1, fb);
#pragma unroll
      for (int v = 0; v < NV; ++v) d0[v] = Q[src_row(v) * NC + c1] - Q[src_row(v) * NC + c0];
      if (fa < 4) {
        const int c2 = cidx(TA + fa, fb), c3 = cidx(TA + fa + 1, fb);
#pragma unroll
        for (int v = 0; v < NV; ++v) d1[v] = Q[src_row(v) * NC + c3] - Q[src_row(v) * NC + c2];
      }
    }
    // incoming cotangents: flux divergence transposed, lam_F_v(face i+1/2) = (lam_k_v(i+1) - lam_k_v(i))/h,
    // in the sweep frame; the B_t components carry the transport-flux cotangents
    double lam[7];
    {
      double lg[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) lg[v] = (lk1[v] - lk0[v]) * a.inv_h;
      const double lm[3] = {lg[1], lg[2], lg[3]};
      const double msk = valid ? 1.0 : 0.0;
      lam[0] = msk * lg[0];
      lam[1] = msk * lm[CN];
      lam[2] = msk * lm[CT1];
      lam[3] = msk * lm[CT2];
      lam[4] = msk * lT[0];
      lam[5] = msk * lT[1];
      lam[6] = msk * lg[4];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) Q[dst_row(v) * NIF + iidx(fa, fb)] = d0[v];
    if (fa < 4) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Q[dst_row(v) * NIF + iidx(TA + fa, fb)] = d1[v];
    }
#pragma unroll
    for (int v = 0; v < 7; ++v) LF[v * NF + fidx(fa, fb)] = lam[v];
  }
  for (int t = threadIdx.x; t < SW_NQ * NIF; t += ADJ_THREADS) LD[t] = 0.0;
  for (int t = threadIdx.x; t < ADJ_NP * NC; t += ADJ_THREADS) PB[t] = 0.0;
  __syncthreads();

  // ---- (3) per-face reverse; interface cotangents in barrier-separated sub-rounds
  // LF speed of field m: max(|v_L + sg c_L|, |v_R + sg c_R|); c index: fast 0, Alfven 1, slow 2, none (entropy)
  // sign and speed index of field m: m < 3 minus, m = 3 none, m > 3 plus
  auto sgm = [](int m) { return m < 3 ? -1 : (m == 3 ? 0 : 1); };
  auto spi = [](int m) { return (m == 0 || m == 6) ? 0 : ((m == 1 || m == 5) ? 1 : 2); };
  auto xarg = [&](int m, int cz) {
    const double v = Pz[P_VN * NC + cz];
    return sgm(m) == 0 ? v : v + sgm(m) * Pz[(P_CF + spi(m)) * NC + cz];
  };
  auto alf = [&](int m) { return fmax(fabs(xarg(m, cL)), fabs(xarg(m, cR))); };
  auto lamf = [&](int j) { return LF[j * NF + fidx(fa, fb)]; };
  auto dl = [&](int j, int k) -> double { return Q[j * NIF + iidx(fa + k, fb)]; };
  // round k: every face adds its cotangent of interface difference fa + k
  auto emit = [&](int k, const double* v) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SW_NQ; ++j) LD[j * NIF + iidx(fa + k, fb)] += v[j];
  };
  double lal[7] = {0, 0, 0, 0, 0, 0, 0};
  double lfp[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  {
    // eigen scalars of the face state (the mean of the two zones' primitives)
    auto eig = [&]() {
      double fp[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) fp[v] = 0.5 * (Pz[v * NC + cL] + Pz[v * NC + cR]);
      FaceEig e;
      face_eig(fp[0], fp[1], fp[2], fp[3], fp[4], fp[5], fp[6], fp[7], a.ph, e);
      return e;
    };
    const FaceEig e = eig();
    FaceEigBar eb;
    eb.zero();
    face_corr_vjp<WZ>(e, alf, lamf, dl, a.ph, eb, lal, emit);
    double fp[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) fp[v] = 0.5 * (Pz[v * NC + cL] + Pz[v * NC + cR]);
    face_eig_vjp(fp, a.ph, e, eb, lfp);
  }
  // zone-primitive cotangents of zones L (i) and R (i+1): face-state means,
  // LF speeds (branch of the larger argument; ties -> L) and transport-flux means
  double pl[ADJ_NP], pr[ADJ_NP];
#pragma unroll
  for (int v = 0; v < ADJ_NP; ++v) { pl[v] = v < 8 ? 0.5 * lfp[v] : 0.0; pr[v] = pl[v]; }
#pragma unroll
  for (int m = 0; m < 7; ++m) {
    const double xl = xarg(m, cL), xr = xarg(m, cR);
    const bool left = fabs(xl) >= fabs(xr);
    const double x = left ? xl : xr;
    const double sx = x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0);
    // to the zone of the larger argument (weights instead of a pointer select,
    // which would move pl, pr to scratch memory)
    const double gl = left ? lal[m] * sx : 0.0, gr = left ? 0.0 : lal[m] * sx;
    pl[P_VN] += gl;
    pr[P_VN] += gr;
    if (sgm(m) != 0) {
      pl[P_CF + spi(m)] += gl * sgm(m);
      pr[P_CF + spi(m)] += gr * sgm(m);
    }
  }
  {
    const double ltc1 = lamf(4), ltc2 = lamf(5);
    const double BnL = Pz[P_BN * NC + cL], BnR = Pz[P_BN * NC + cR];
    pl[P_BN] += 0.5 * (ltc1 * Pz[P_VT1 * NC + cL] + ltc2 * Pz[P_VT2 * NC + cL]);
    pr[P_BN] += 0.5 * (ltc1 * Pz[P_VT1 * NC + cR] + ltc2 * Pz[P_VT2 * NC + cR]);
    pl[P_VT1] += 0.5 * ltc1 * BnL; pr[P_VT1] += 0.5 * ltc1 * BnR;
    pl[P_VT2] += 0.5 * ltc2 * BnL; pr[P_VT2] += 0.5 * ltc2 * BnR;
  }
  // cotangent sums of this thread's cells in (4), loaded ahead of the sub-rounds
  const int span = tav + SW_HL + SW_HR;          // positions touched by the valid faces
  const int nz_own = min(span, nA);              // distinct zones among them
  double lm[NCELL][8];
  size_t gcell[NCELL];
  bool own[NCELL];
#pragma unroll
  for (int k = 0; k < NCELL; ++k) {
    const int cell = threadIdx.x + k * ADJ_THREADS;
    int aa, bb;
    if (AXIS == 0) { aa = cell % NA; bb = cell / NA; }
    else           { bb = cell % TB; aa = cell / TB; }
    own[k] = cell < NC && aa < nz_own && b0 + bb < nB;
    gcell[k] = own[k] ? gindex(wrap(a0 - SW_HL + aa, nA), b0 + bb) : 0;
#pragma unroll
    for (int v = 0; v < 8; ++v) lm[k][v] = own[k] ? (v < 5 ? a.lam_h : a.lam_Bz - 5 * g.N)[v * g.N + gcell[k]] : 0.0;
  }
  // two sub-rounds: zone L, then zone R
  __syncthreads();
#pragma unroll
  for (int v = 0; v < ADJ_NP; ++v) PB[v * NC + cL] += pl[v];
  __syncthreads();
#pragma unroll
  for (int v = 0; v < ADJ_NP; ++v) PB[v * NC + cR] += pr[v];
  __syncthreads();

  // ---- (4) per zone: gather, prologue reverse, add
  // cotangents of the prologue outputs at tile position aa (lz += ...)
  auto gather = [&](int aa, int bb, double* lz) {
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      double lFj = 0.0, lqj = 0.0;
      // interface differences: D(ia) = X(ia+1) - X(ia)
      if (aa >= 1) { lFj += LD[j * NIF + iidx(aa - 1, bb)]; lqj += LD[(7 + j) * NIF + iidx(aa - 1, bb)]; }
      if (aa < NI) { lFj -= LD[j * NIF + iidx(aa, bb)]; lqj -= LD[(7 + j) * NIF + iidx(aa, bb)]; }
      // central term: face f (local) uses zones f+1 (-1/12), f+2 (7/12), f+3 (7/12), f+4 (-1/12)
      const int f1 = aa - 1, f2 = aa - 2, f3 = aa - 3, f4 = aa - 4;
      if (f1 >= 0 && f1 < TA) lFj -= LF[j * NF + fidx(f1, bb)] * (1.0 / 12.0);
      if (f2 >= 0 && f2 < TA) lFj += LF[j * NF + fidx(f2, bb)] * (7.0 / 12.0);
      if (f3 >= 0 && f3 < TA) lFj += LF[j * NF + fidx(f3, bb)] * (7.0 / 12.0);
      if (f4 >= 0 && f4 < TA) lFj -= LF[j * NF + fidx(f4, bb)] * (1.0 / 12.0);
      lz[Z_F0 + j] += lFj;
      lz[Z_RHO + j] += lqj;
    }
    const int cz = cidx(aa, bb);
    lz[Z_RHO] += PB[P_RHO * NC + cz];
    lz[Z_VN] += PB[P_VN * NC + cz];
    lz[Z_VT1] += PB[P_VT1 * NC + cz];
    lz[Z_VT2] += PB[P_VT2 * NC + cz];
    lz[Z_BN] += PB[P_BN * NC + cz];
    lz[Z_BT1] += PB[P_BT1 * NC + cz];
    lz[Z_BT2] += PB[P_BT2 * NC + cz];
    lz[Z_P] += PB[P_P * NC + cz];
    lz[Z_CF] += PB[P_CF * NC + cz];
    lz[Z_CA] += PB[P_CA * NC + cz];
    lz[Z_CS] += PB[P_CS * NC + cz];
  };
#pragma unroll
  for (int k = 0; k < NCELL; ++k) {   // branch-free over the cells (the stores are predicated)
    const int cell = min(threadIdx.x + k * ADJ_THREADS, (unsigned)NC - 1);
    int aa, bb;
    if (AXIS == 0) { aa = cell % NA; bb = cell / NA; }
    else           { bb = cell % TB; aa = cell / TB; }
    double lz[Z_NVAR];
#pragma unroll
    for (int v = 0; v < Z_NVAR; ++v) lz[v] = 0.0;
    gather(aa, bb, lz);
    if (span > nA)   // a tile that wraps onto itself: other positions of the same zone
      for (int q = aa + nA; q < span; q += nA) gather(q, bb, lz);
    double lu[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    zone_prologue_vjp(uz[k], a.ph.gamma, lz, lu);
    double out[8];
    out[0] = lu[0];
    out[1 + CN] = lu[1]; out[1 + CT1] = lu[2]; out[1 + CT2] = lu[3];
    out[4] = lu[4];
    out[5 + CN] = lu[5]; out[5 + CT1] = lu[6]; out[5 + CT2] = lu[7];
    if (own[k]) {
#pragma unroll
      for (int v = 0; v < 8; ++v) (v < 5 ? a.lam_h : a.lam_Bz - 5 * g.N)[v * g.N + gcell[k]] = lm[k][v] + out[v];
    }
  }
}

// face b cotangent += transpose of B_i = (-b_{i-2} + 9 b_{i-1} + 9 b_i - b_{i+1})/16:
// lam_b_j += (-lam_B_{j+2} + 9 lam_B_{j+1} + 9 lam_B_j - lam_B_{j-1})/16
__global__ __launch_bounds__(256) void adj_bcell_kernel(Grid g, const double* lam_B, double* lam_b) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const size_t N = g.N, c0 = g.at(i, j, k);
  const double* Lx = lam_B;
  const double* Ly = lam_B + N;
  const double* Lz = lam_B + 2 * N;
  lam_b[c0] += (-Lx[g.at(wrap(i + 2, g.nx), j, k)] + 9.0 * Lx[g.at(wrap(i + 1, g.nx), j, k)] + 9.0 * Lx[c0] -
                Lx[g.at(wrap(i - 1, g.nx), j, k)]) * (1.0 / 16.0);
  lam_b[N + c0] += (-Ly[g.at(i, wrap(j + 2, g.ny), k)] + 9.0 * Ly[g.at(i, wrap(j + 1, g.ny), k)] + 9.0 * Ly[c0] -
                    Ly[g.at(i, wrap(j - 1, g.ny), k)]) * (1.0 / 16.0);
  lam_b[2 * N + c0] += (-Lz[g.at(i, j, wrap(k + 2, g.nz))] + 9.0 * Lz[g.at(i, j, wrap(k + 1, g.nz))] + 9.0 * Lz[c0] -
                        Lz[g.at(i, j, wrap(k - 1, g.nz))]) * (1.0 / 16.0);
}

// y = a x (n doubles)
__global__ __launch_bounds__(256) void scale_kernel(size_t n, double a, const double* x, double* y) {
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (c < n) y[c] = a * x[c];
}
__global__ __launch_bounds__(256) void fill_kernel(size_t n, double v, double* y) {
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (c < n) y[c] = v;
}
// y = x widened from float (n values): FP32 states enter the FP64 adjoint
__global__ __launch_bounds__(256) void widen_kernel(size_t n, const float* x, double* y) {
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (c < n) y[c] = double(x[c]);
}

// The stage combinations of the adjoint step over the 8N cotangent entries
// (hydro [5][N] then face b [3][N]).  lam3, the incoming cotangent, is read in
// place from (lh, lb), which keep it until the last combination overwrites them:
//   glue_a: lk = c lam3, z = 0
//   glue_b: lk = a lam3 + b x, z = 0
//   glue_c: lk = a lam3 + b x + c y, (lh, lb) = lam3 + x + y
//   glue_d: lk = a lam3 + b x, (lh, lb) = lam3 + x + y + z (the four-stage sum of RK4)
__device__ __forceinline__ double lam3_at(size_t i, size_t N, const double* lh, const double* lb) {
  return i < 5 * N ? lh[i] : lb[i - 5 * N];
}
__global__ __launch_bounds__(256) void adj_glue_a_kernel(size_t N, double c, const double* lh, const double* lb,
                                                         double* lk, double* z) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= 8 * N) return;
  lk[i] = c * lam3_at(i, N, lh, lb);
  z[i] = 0.0;
}
__global__ __launch_bounds__(256) void adj_glue_b_kernel(size_t N, double a, const double* lh, const double* lb,
                                                         double b, const double* x, double* lk, double* z) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= 8 * N) return;
  lk[i] = a * lam3_at(i, N, lh, lb) + b * x[i];
  z[i] = 0.0;
}
__global__ __launch_bounds__(256) void adj_glue_c_kernel(size_t N, double a, double b, const double* x, double c,
                                                         const double* y, double* lk, double* lh, double* lb) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= 8 * N) return;
  const double wi = lam3_at(i, N, lh, lb), xi = x[i], yi = y[i];
  lk[i] = a * wi + b * xi + c * yi;
  const double s = wi + xi + yi;
  if (i < 5 * N) lh[i] = s;
  else lb[i - 5 * N] = s;
}
__global__ __launch_bounds__(256) void adj_glue_d_kernel(size_t N, double a, double b, const double* x,
                                                         const double* y, const double* z, double* lk, double* lh,
                                                         double* lb) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= 8 * N) return;
  const double wi = lam3_at(i, N, lh, lb), xi = x[i];
  lk[i] = a * wi + b * xi;
  const double s = wi + xi + y[i] + z[i];
  if (i < 5 * N) lh[i] = s;
  else lb[i - 5 * N] = s;
}

// Initial-state map transposed, per zone: m = rho v, E = P0/(gamma-1) + (rho v^2 + B^2)/2
// with B the zone interpolation of b:  lam_v = rho lam_m + rho v lam_E,  lam_B = B lam_E.
__global__ __launch_bounds__(256) void init_adj_zone_kernel(size_t N, const double* rho, const double* v,
                                                            const double* B, const double* lam_h, double* g_v,
                                                            double* lam_B) {
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= N) return;
  const double r = rho[c], lE = lam_h[4 * N + c];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    g_v[d * N + c] = r * lam_h[(1 + d) * N + c] + r * v[d * N + c] * lE;
    lam_B[d * N + c] = B[d * N + c] * lE;
  }
}

// curl_h transposed: b_x = (Az - Az[j-1] - Ay + Ay[k-1])/h, b_y = (Ax - Ax[k-1] - Az + Az[i-1])/h,
// b_z = (Ay - Ay[i-1] - Ax + Ax[j-1])/h  =>  per edge value of A:
// g_Ax = (lby - lby[k+1] - lbz + lbz[j+1])/h, g_Ay = (lbz - lbz[i+1] - lbx + lbx[k+1])/h,
// g_Az = (lbx - lbx[j+1] - lby + lby[i+1])/h
__global__ __launch_bounds__(256) void curl_adj_kernel(Grid g, double inv_h, const double* lam_b, double* g_A) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const size_t N = g.N, c0 = g.at(i, j, k);
  const double* lbx = lam_b;
  const double* lby = lam_b + N;
  const double* lbz = lam_b + 2 * N;
  const int ip = wrap(i + 1, g.nx), jp = wrap(j + 1, g.ny), kp = wrap(k + 1, g.nz);
  g_A[c0] = (lby[c0] - lby[g.at(i, j, kp)] - lbz[c0] + lbz[g.at(i, jp, k)]) * inv_h;
  g_A[N + c0] = (lbz[c0] - lbz[g.at(ip, j, k)] - lbx[c0] + lbx[g.at(i, j, kp)]) * inv_h;
  g_A[2 * N + c0] = (lbx[c0] - lbx[g.at(i, jp, k)] - lby[c0] + lby[g.at(ip, j, k)]) * inv_h;
}

}  // namespace wm
