// HIP kernels of the WENO5-CT step for gfx950 (wave64, 256-thread blocks).
//
//   sweep_kernel<AXIS>   face fluxes along one axis: zone prologue staged in
//                        LDS, one face per lane, eigensystem + projections in
//                        registers.  Writes the five hydro flux components
//                        (global frame) and the two CT transport fluxes.
//   update_kernel<STAGE> flux divergence, corner fluxes, face-B right-hand
//                        side and the SSP-RK3 increment, one zone per lane.
//   bcell_kernel         zone B = fourth-order interpolation of the face field.
//   init kernels, dt and diagnostics reductions.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mhd_device.hpp"

namespace wm {

struct Grid {
  int nx, ny, nz;
  size_t N;   // nx * ny * nz
  int wall[3];  // 1: reflecting conducting walls at both ends of the axis
  int wide;     // 1: the sweep takes 64-bit addresses also for arrays under 4 GiB (testing)
  __device__ __forceinline__ size_t at(int i, int j, int k) const {
    return ((size_t)k * ny + j) * nx + i;
  }
  // the same index in 32 bits (N < 2^31 always)
  __device__ __forceinline__ unsigned at32(int i, int j, int k) const {
    return ((unsigned)k * (unsigned)ny + (unsigned)j) * (unsigned)nx + (unsigned)i;
  }
};

// Raw buffer access to one array of at most 4 GiB: the array's base lives in a
// scalar descriptor and the hardware adds the lane's 32-bit byte offset, so an
// access costs no 64-bit address arithmetic.  Word 3 of the descriptor is the
// gfx9 value for untyped 32-bit accesses.
using BufRsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ BufRsrc buf_rsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)(unsigned)bytes, 0x00020000);
}
typedef unsigned BufU2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double buf_load(BufRsrc r, unsigned off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float buf_load(BufRsrc r, unsigned off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void buf_store(BufRsrc r, unsigned off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(BufU2, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store(BufRsrc r, unsigned off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}

// The four normal-field faces b_f, f = c-2 .. c+1, that the zone-B
// interpolation of zone c reads along an axis of n faces: periodic wrap, or at
// walls the mirror ghost faces (odd about the wall faces -1/2 and n-1/2; the
// lower wall face, index -1, is zero).  Index and sign only, with selects, so
// that the caller issues its loads together (a walled axis has n >= 3).
__device__ __forceinline__ void face_stencil(int c, int n, int wall, int idx[4], double sg[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int f = c - 2 + q;
    if (wall) {
      const bool ghost = f < -1 || f > n - 1;
      idx[q] = f < -1 ? -2 - f : (f > n - 1 ? 2 * n - 2 - f : max(f, 0));
      sg[q] = f == -1 ? 0.0 : (ghost ? -1.0 : 1.0);
    } else {   // periodic: f lies in [-2, n], so one add or subtract wraps it (n = 1: zone 0)
      idx[q] = n == 1 ? 0 : (f < 0 ? f + n : (f >= n ? f - n : f));
      sg[q] = 1.0;
    }
  }
}

// ---------------------------------------------------------------------------
// directional sweep
// ---------------------------------------------------------------------------
// Tile of TA faces along the sweep axis by TB faces across it (256 lanes, one
// face each), for work type TW.  The x sweep uses 128 x 2 (266 zones for 256
// faces; a wave reads whole 128-byte lines of a row), 0.5% faster than 64 x 4.
// The y and z sweeps have x across: in FP64 32 x 8 (296 zones; rows of 64
// bytes), which fits three blocks per CU in LDS, against 16 x 16 (336 zones,
// 128-byte rows) in the FP32 work type (32 x 8 measured 1% slower there); 64 x 4
// (276 zones, 32-byte rows) measured 4% slower in FP64.
template <int AXIS, typename TW> struct SweepTile {
  static constexpr int TA = sizeof(TW) == 8 ? 32 : 16, TB = sizeof(TW) == 8 ? 8 : 16;
};
template <typename TW> struct SweepTile<0, TW> { static constexpr int TA = 128, TB = 2; };
constexpr int SW_THREADS = 256;
constexpr int SW_HL = 2, SW_HR = 3;          // stencil zones i-2 .. i+3
constexpr int SW_NQ = 14;                    // q (7) and F (7) per zone
constexpr int SW_NP = 11;                    // rho, v_n, v_t1, v_t2, B_n, B_t1, B_t2, P, c_f, c_A, c_s
enum { P_RHO = 0, P_VN, P_VT1, P_VT2, P_BN, P_BT1, P_BT2, P_P, P_CF, P_CA, P_CS };
// the forward sweep's zone primitives and speeds: rho, B_t1 and B_t2 are read
// from the zone q in LDS instead
constexpr int SW_NPF = 8;
enum { FP_VN = 0, FP_VT1, FP_VT2, FP_BN, FP_P, FP_CF, FP_CA, FP_CS };

// S: storage type of the state and of the face values (double, or float for
// the FP32-state form); arithmetic is in double / TW as described below.
__device__ __forceinline__ double nanmax(double a, double b) {   // NaN-propagating max (either argument)
  if (a != a) return a;
  if (b != b) return b;
  return b > a ? b : a;
}

// Signal speed |v_n| + c_fast of eq. (cfl) from a zone prologue along n, as
// the bit pattern of the double: the sweep of the first stage of a step and the
// stand-alone time-step pass both take it from zone_prologue, so their maxima
// agree bitwise.  Non-negative doubles order like their bit patterns read as
// unsigned integers, so the maximum is an integer max.  A fast speed that is
// not real (a negative argument of its square roots, which sqrt_nr returns as
// a negative value) makes the speed negative, and a NaN state makes it NaN:
// both keys lie above every non-negative speed's, and dt_final_kernel turns
// such a maximum into NaN.
typedef unsigned long long SpeedKey;
__device__ __forceinline__ SpeedKey cfl_key(const double* z) {
  return __builtin_bit_cast(SpeedKey, fabs(z[Z_VN]) + z[Z_CF]);
}
__device__ __forceinline__ SpeedKey kmax(SpeedKey a, SpeedKey b) { return b > a ? b : a; }

// Maximum of a 32-bit unsigned value over the 64 lanes of a wave, returned to
// every lane: maxima over the preceding 1, 2, 4, 8 lanes of each row of 16
// (DPP row shifts), then row 0's into row 1 and row 2's into row 3 (row
// broadcast of lane 15), then rows 0-1 into rows 2-3 (broadcast of lane 31):
// lane 63 ends with the maximum.  Lanes without a source keep 0, the identity.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  auto step = [](unsigned x, auto ctrl, auto rows) {
    const unsigned y = (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, decltype(ctrl)::value,
                                                             decltype(rows)::value, 0xf, false);
    return y > x ? y : x;
  };
  v = step(v, std::integral_constant<int, 0x111>{}, std::integral_constant<int, 0xf>{});   // row_shr:1
  v = step(v, std::integral_constant<int, 0x112>{}, std::integral_constant<int, 0xf>{});   // row_shr:2
  v = step(v, std::integral_constant<int, 0x114>{}, std::integral_constant<int, 0xf>{});   // row_shr:4
  v = step(v, std::integral_constant<int, 0x118>{}, std::integral_constant<int, 0xf>{});   // row_shr:8
  v = step(v, std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xa>{});   // row_bcast:15
  v = step(v, std::integral_constant<int, 0x143>{}, std::integral_constant<int, 0xc>{});   // row_bcast:31
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}
// the same for a 64-bit key, exactly: the high words' maximum, then the
// maximum of the low words of the lanes that hold it
__device__ __forceinline__ SpeedKey wave_max_key(SpeedKey k) {
  const unsigned hi = (unsigned)(k >> 32), lo = (unsigned)k;
  const unsigned hm = wave_max_u32(hi);
  const unsigned lm = wave_max_u32(hi == hm ? lo : 0u);
  return ((SpeedKey)hm << 32) | lm;
}

template <typename S>
struct SweepArgs {
  Grid g;
  Phys ph;
  const S* hydro;        // [5][N] rho, mx, my, mz, E
  const S* bcell;        // [3][N] zone B
  S* fhydro;             // [5][N] interface flux, global frame (rho, mx, my, mz, E)
  S* T;                  // [2][N] transport fluxes T^n_t1, T^n_t2
  double* dbg;           // optional [9][N]: 7 sweep-frame flux components + 2 T
  S* wallF;              // walled sweep axis: [5][nB * nC] fluxes through the lower wall face
  SpeedKey* smax_blk;    // optional: per wave (4 per block), the maximum of |v_n| + c_fast over its zones (cfl_key)
#ifdef WM_SWEEP_CLOCK
  unsigned long long* clk;   // clock build: [block][wave][8] phase stamps, or null
#endif
};

// Zone index along a sweep axis of n zones for a stencil position z: periodic
// wrap, or at walls the mirror zone, with flip = -1 where the normal momentum
// and field change sign (ghost zones, R20).  The mirror is the periodic
// extension of the mirror-doubled axis (period 2n), so any z -- also the
// positions of a tile longer than the axis, whose faces are discarded --
// maps into [0, n); for z in [-n, 2n) it is the plain reflection.
// Positions within one period of [0, p) wrap with one add or subtract; the
// modulo (an integer division by the runtime length) is left for tiles longer
// than the axis.
__device__ __forceinline__ int wrap_near(int z, int p) {
  if (z >= -p && z < 2 * p) return z < 0 ? z + p : (z >= p ? z - p : z);
  return wrap(z, p);
}
__device__ __forceinline__ int sweep_zone(int z, int n, int wall, double& flip) {
  flip = 1.0;
  if (!wall) return wrap_near(z, n);
  const int zz = wrap_near(z, 2 * n);
  if (zz >= n) { flip = -1.0; return 2 * n - 1 - zz; }
  return zz;
}

// LDS per block, two arrays: zone q and F in FP64 (the differences are formed
// in FP64, then stored over them), and the zone primitives and speeds in the
// work type TW.
template <int AXIS, typename TW> constexpr int sweep_zones() {
  return (SweepTile<AXIS, TW>::TA + SW_HL + SW_HR) * SweepTile<AXIS, TW>::TB;
}
template <int AXIS, typename TW> constexpr size_t sweep_q_doubles() {
  return (size_t)SW_NQ * sweep_zones<AXIS, TW>();
}
template <int AXIS, typename TW> constexpr size_t sweep_p_doubles() {
  return ((size_t)SW_NPF * sweep_zones<AXIS, TW>() * sizeof(TW) + 7) / 8;
}

// Phases: (1) zone prologue of the tile and its halo into LDS; (2) per face:
// central flux, face state, Lax-Friedrichs speeds and the interface
// differences Delta F, Delta q (formed in FP64); (3) per face: eigen-system
// and characteristic WENO in registers, reading the differences (in TW) from
// LDS one eigen pair at a time.  TW = double: everything in FP64.  TW = float
// (mixed): projections, split, weights, zone primitives, LF speeds and the
// transport-flux mean in FP32; the zone prologue (pressure recovery), the
// differences, the central flux and the face eigen-system (renormalisation of
// alpha_f, alpha_s, beta) in FP64.  DTMAX: each wave also writes the maximum
// of the eq. (cfl) signal speed over its zones to a.smax_blk (the first stage
// of a step), a separate instantiation so that the other sweeps carry none of it.

template <int AXIS, bool WENO_Z, typename TW, typename S, bool DTMAX = false>
__global__ __launch_bounds__(SW_THREADS, 3) void sweep_kernel(SweepArgs<S> a) {
  constexpr int TA = SweepTile<AXIS, TW>::TA, TB = SweepTile<AXIS, TW>::TB;
  constexpr int NA = TA + SW_HL + SW_HR;     // zones along the axis
  constexpr int NI = TA + 4;                 // interfaces i-3/2 .. i+TA+3/2
  constexpr int NC = NA * TB;
  constexpr int NIF = NI * TB;
  static_assert(TA * TB == SW_THREADS, "one face per lane");
  static_assert(TA >= 4, "extra interfaces are built by lanes fa < 4");
  __shared__ double sQ[sweep_q_doubles<AXIS, TW>()];
  __shared__ double sP[sweep_p_doubles<AXIS, TW>()];
  double* Q = sQ;                            // [14][NC] zone q and F, later the differences
  TW* Pz = reinterpret_cast<TW*>(sP);        // [11][NC] zone primitives and speeds
  TW* Dl = reinterpret_cast<TW*>(sQ);        // [14][NIF] interface differences (aliases Q)

  const Grid& g = a.g;
  const int nA = AXIS == 0 ? g.nx : (AXIS == 1 ? g.ny : g.nz);
  const int nB = AXIS == 0 ? g.ny : g.nx;
  constexpr int CN = AXIS, CT1 = (AXIS + 1) % 3, CT2 = (AXIS + 2) % 3;
  auto cidx = [](int aa, int bb) { return AXIS == 0 ? bb * NA + aa : aa * TB + bb; };
  auto iidx = [](int ia, int bb) { return AXIS == 0 ? bb * NI + ia : ia * TB + bb; };
  // faces 0 .. nA-1 (i+1/2), and with walls also the lower wall face -1/2
  const int wl = g.wall[AXIS];
  const int a0 = blockIdx.x * TA - wl;
  const int b0 = blockIdx.y * TB;
  const int c = blockIdx.z;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid) / 64;   // uniform: held in a scalar register
  // every array of the state and the fluxes within 4 GiB: buffer accesses with 32-bit offsets
  const size_t abytes = g.N * sizeof(S);
  const bool off32 = !g.wide && abytes < (size_t(1) << 32);
#ifdef WM_SWEEP_CLOCK
  // clock build: per-wave shader-clock stamps at the phase boundaries
  unsigned long long stamp[8];
  stamp[0] = clock64();
#endif

  // ---- (1) zone prologue, zones i-2 .. i+TA+2 along the axis (periodic wrap
  // or wall mirror).  The tile has more zones than lanes (NR = 2 per lane at
  // most): every lane issues the loads of all its zones before evaluating any,
  // so the block waits for one round trip to memory, not two.  Lanes past the
  // last zone load it again and discard it.
  constexpr int NR = (NC + SW_THREADS - 1) / SW_THREADS;
  double raw[NR][8];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int cell = min(tid + r * SW_THREADS, NC - 1);
    int aa, bb;
    if (AXIS == 0) { aa = cell % NA; bb = cell / NA; }
    else           { bb = cell % TB; aa = cell / TB; }
    double flip;
    const int ia = sweep_zone(a0 - SW_HL + aa, nA, wl, flip);
    const int ib = min(b0 + bb, nB - 1);
    int i, j, k;
    if (AXIS == 0)      { i = ia; j = ib; k = c; }
    else if (AXIS == 1) { i = ib; j = ia; k = c; }
    else                { i = ib; j = c;  k = ia; }
    if (off32) {
      const unsigned off = g.at32(i, j, k) * (unsigned)sizeof(S);
#pragma unroll
      for (int v = 0; v < 5; ++v) raw[r][v] = double(buf_load(buf_rsrc(a.hydro + v * g.N, abytes), off, S()));
#pragma unroll
      for (int v = 0; v < 3; ++v) raw[r][5 + v] = double(buf_load(buf_rsrc(a.bcell + v * g.N, abytes), off, S()));
    } else {
      const size_t gi = g.at(i, j, k);
#pragma unroll
      for (int v = 0; v < 5; ++v) raw[r][v] = double(a.hydro[v * g.N + gi]);
#pragma unroll
      for (int v = 0; v < 3; ++v) raw[r][5 + v] = double(a.bcell[v * g.N + gi]);
    }
    raw[r][1 + CN] *= flip;
    raw[r][5 + CN] *= flip;
  }
  SpeedKey key = 0;   // the lane's maximum over its zones (cfl_key)
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int cell = tid + r * SW_THREADS;
    if (cell >= NC) continue;
    const double* m = raw[r] + 1;
    const double* B = raw[r] + 5;
    double z[Z_NVAR];
    zone_prologue(raw[r][0], m[CN], m[CT1], m[CT2], raw[r][4], B[CN], B[CT1], B[CT2], a.ph.gamma, z);
    if constexpr (DTMAX) key = kmax(key, cfl_key(z));
#pragma unroll
    for (int v = 0; v < SW_NQ; ++v) Q[v * NC + cell] = z[v];
    Pz[FP_VN * NC + cell] = TW(z[Z_VN]);
    Pz[FP_VT1 * NC + cell] = TW(z[Z_VT1]);
    Pz[FP_VT2 * NC + cell] = TW(z[Z_VT2]);
    Pz[FP_BN * NC + cell] = TW(z[Z_BN]);
    Pz[FP_P * NC + cell] = TW(z[Z_P]);
    Pz[FP_CF * NC + cell] = TW(z[Z_CF]);
    Pz[FP_CA * NC + cell] = TW(z[Z_CA]);
    Pz[FP_CS * NC + cell] = TW(z[Z_CS]);
  }
  if constexpr (DTMAX) {   // the wave's maximum, one value per wave
    static_assert(SW_THREADS == 256, "four waves per block");
    const SpeedKey wk = wave_max_key(key);
    if (__lane_id() == 0)
      a.smax_blk[((blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * 4 + wave] = wk;
  }
#ifdef WM_SWEEP_CLOCK
  stamp[1] = clock64();
#endif
  __syncthreads();
#ifdef WM_SWEEP_CLOCK
  stamp[2] = clock64();
#endif

  // ---- (2) per face: central flux, face state, LF speeds, own interface differences
  int fa, fb;
  if (AXIS == 0) { fa = tid % TA; fb = tid / TA; }
  else           { fb = tid % TB; fa = tid / TB; }
  const int cL = cidx(fa + 2, fb), cR = cidx(fa + 3, fb);
  double Fc[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const double* F = Q + (SW_NQ / 2 + j) * NC;
    Fc[j] = (-F[cidx(fa + 1, fb)] + 7.0 * F[cL] + 7.0 * F[cR] - F[cidx(fa + 4, fb)]) * (1.0 / 12.0);
  }
  auto PL = [&](int v) { return double(Pz[v * NC + cL]); };
  auto PR = [&](int v) { return double(Pz[v * NC + cR]); };
  auto QL = [&](int v) { return Q[v * NC + cL]; };
  auto QR = [&](int v) { return Q[v * NC + cR]; };
  // face state: mean of the primitive states of zones i and i+1 (rho, B_t from q)
  const double fp[8] = {0.5 * (QL(Z_RHO) + QR(Z_RHO)), 0.5 * (PL(FP_VN) + PR(FP_VN)),
                        0.5 * (PL(FP_VT1) + PR(FP_VT1)), 0.5 * (PL(FP_VT2) + PR(FP_VT2)),
                        0.5 * (PL(FP_BN) + PR(FP_BN)), 0.5 * (QL(Z_BT1) + QR(Z_BT1)),
                        0.5 * (QL(Z_BT2) + QR(Z_BT2)), 0.5 * (PL(FP_P) + PR(FP_P))};
  double d0[SW_NQ], d1[SW_NQ];
  {
    const int c0 = cidx(fa, fb), c1 = cidx(fa + 1, fb);
#pragma unroll
    for (int v = 0; v < SW_NQ; ++v) d0[v] = Q[v * NC + c1] - Q[v * NC + c0];
    if (fa < 4) {
      const int c2 = cidx(TA + fa, fb), c3 = cidx(TA + fa + 1, fb);
#pragma unroll
      for (int v = 0; v < SW_NQ; ++v) d1[v] = Q[v * NC + c3] - Q[v * NC + c2];
    }
  }
#ifdef WM_SWEEP_CLOCK
  stamp[3] = clock64();
#endif
  __syncthreads();
  // differences stored as (Delta F, Delta q): j = 0..6 flux, 7..13 state
#pragma unroll
  for (int v = 0; v < 7; ++v) {
    Dl[v * NIF + iidx(fa, fb)] = TW(d0[7 + v]);
    Dl[(7 + v) * NIF + iidx(fa, fb)] = TW(d0[v]);
  }
  if (fa < 4) {
#pragma unroll
    for (int v = 0; v < 7; ++v) {
      Dl[v * NIF + iidx(TA + fa, fb)] = TW(d1[7 + v]);
      Dl[(7 + v) * NIF + iidx(TA + fa, fb)] = TW(d1[v]);
    }
  }
  __syncthreads();
#ifdef WM_SWEEP_CLOCK
  stamp[4] = clock64();
#endif

  // ---- (3) characteristic WENO flux of this face
  auto dl = [&](int j, int k) -> TW { return Dl[j * NIF + iidx(fa + k, fb)]; };
  // Lax-Friedrichs speed of field m (0-based), read when its pair needs it:
  // max(|v_L + sg c_L|, |v_R + sg c_R|), c = c_f (m = 0, 6), c_A (1, 5), c_s (2, 4), 0 (3)
  auto alf = [&](int m) -> TW {
    const double vL = PL(FP_VN), vR = PR(FP_VN);
    if (m == 3) return TW(fmax(fabs(vL), fabs(vR)));
    const int sp = (m == 0 || m == 6) ? FP_CF : ((m == 1 || m == 5) ? FP_CA : FP_CS);
    const double sg = m < 3 ? -1.0 : 1.0;
    return TW(fmax(fabs(vL + sg * PL(sp)), fabs(vR + sg * PR(sp))));
  };
  FaceEig e;
  face_eig(fp[0], fp[1], fp[2], fp[3], fp[4], fp[5], fp[6], fp[7], a.ph, e);
  // F = F_c + corr: the characteristic part is added onto the central term
  double Ff[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) Ff[j] = Fc[j];
  face_corr<WENO_Z, TW>(e, alf, dl, a.ph, Ff);
  // CT transport-flux correction: face mean of B_n v_t (eq. fct1-fct6)
  const double tc1 = 0.5 * (PL(FP_BN) * PL(FP_VT1) + PR(FP_BN) * PR(FP_VT1));
  const double tc2 = 0.5 * (PL(FP_BN) * PL(FP_VT2) + PR(FP_BN) * PR(FP_VT2));
  const double T1 = Ff[4] + tc1;
  const double T2 = Ff[5] + tc2;
#ifdef WM_SWEEP_CLOCK
  stamp[5] = clock64();
#endif

  // keep the face computation ahead of the range guard: sinking it into the
  // guarded block defeats register allocation (hundreds of spills)
#pragma unroll
  for (int j = 0; j < 7; ++j) asm volatile("" : "+v"(Ff[j]));
  // FP64: the face's coordinates again, from the wave index and the lane id,
  // for the stores: holding them through phase 3 cost a spilled register (the
  // FP32 work type has registers to spare and measured 0.7% slower with this)
  if constexpr (sizeof(TW) == 8) {
    const int t = wave * 64 + (int)__lane_id();
    if (AXIS == 0) { fa = t % TA; fb = t / TA; }
    else           { fb = t % TB; fa = t / TB; }
  }
  if (a0 + fa < 0 && b0 + fb < nB) {          // the lower wall face (-1/2): hydro fluxes only
    double fm[3];
    fm[CN] = Ff[1]; fm[CT1] = Ff[2]; fm[CT2] = Ff[3];
    const size_t wi = (size_t)(b0 + fb) + (size_t)nB * c;
    const size_t P = (size_t)nB * (AXIS == 2 ? g.ny : g.nz);
    a.wallF[wi] = S(Ff[0]);
    a.wallF[P + wi] = S(fm[0]);
    a.wallF[2 * P + wi] = S(fm[1]);
    a.wallF[3 * P + wi] = S(fm[2]);
    a.wallF[4 * P + wi] = S(Ff[6]);
  } else if (a0 + fa < nA && b0 + fb < nB) {
  int i, j, k;
  if (AXIS == 0)      { i = a0 + fa; j = b0 + fb; k = c; }
  else if (AXIS == 1) { i = b0 + fb; j = a0 + fa; k = c; }
  else                { i = b0 + fb; j = c;       k = a0 + fa; }
  const size_t gi = g.at(i, j, k);
  double fm[3];
  fm[CN] = Ff[1]; fm[CT1] = Ff[2]; fm[CT2] = Ff[3];
  if (off32) {
    const unsigned off = g.at32(i, j, k) * (unsigned)sizeof(S);
    buf_store(buf_rsrc(a.fhydro, abytes), off, S(Ff[0]));
    buf_store(buf_rsrc(a.fhydro + g.N, abytes), off, S(fm[0]));
    buf_store(buf_rsrc(a.fhydro + 2 * g.N, abytes), off, S(fm[1]));
    buf_store(buf_rsrc(a.fhydro + 3 * g.N, abytes), off, S(fm[2]));
    buf_store(buf_rsrc(a.fhydro + 4 * g.N, abytes), off, S(Ff[6]));
    buf_store(buf_rsrc(a.T, abytes), off, S(T1));
    buf_store(buf_rsrc(a.T + g.N, abytes), off, S(T2));
  } else {
    a.fhydro[gi] = S(Ff[0]);
    a.fhydro[g.N + gi] = S(fm[0]);
    a.fhydro[2 * g.N + gi] = S(fm[1]);
    a.fhydro[3 * g.N + gi] = S(fm[2]);
    a.fhydro[4 * g.N + gi] = S(Ff[6]);
    a.T[gi] = S(T1);
    a.T[g.N + gi] = S(T2);
  }
  if (a.dbg) {
#pragma unroll
    for (int v = 0; v < 7; ++v) a.dbg[v * g.N + gi] = Ff[v];
    a.dbg[7 * g.N + gi] = T1;
    a.dbg[8 * g.N + gi] = T2;
  }
  }
#ifdef WM_SWEEP_CLOCK
  stamp[6] = clock64();
  stamp[7] = __smid();
  if (a.clk && (tid & 63) == 0) {
    const size_t blk = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    unsigned long long* o = a.clk + (blk * (SW_THREADS / 64) + tid / 64) * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = stamp[q];
  }
#endif
}

// ---------------------------------------------------------------------------
// divergence + CT + RK stage
// ---------------------------------------------------------------------------
template <typename S>
struct UpdateArgs {
  Grid g;
  double inv_h;
  const S* faces;        // [21][N]: F^x[5], F^y[5], F^z[5], T^x[2], T^y[2], T^z[2]
  const S* Un;           // hydro [5][N] of U^n
  const S* bn;           // bface [3][N] of U^n
  S* acc;                // [8][N] accumulated increments
  S* hyd_out;            // hydro [5][N] of the stage result
  S* b_out;              // bface [3][N] of the stage result
  double* rhs_out;       // optional [8][N]: the right-hand side itself (no state update)
  const double* dt;      // device scalar
  const S* wallF[3];     // per walled axis: [5][nB * nC] fluxes through the lower wall face
};

// The update's streams that are used once (U^n and the accumulator read, the
// stage state and the accumulator written) as nontemporal accesses: they pass
// the caches by, which keeps the face fluxes the update re-reads at tile edges
// cached (update -3.2% for the stores and -4.4% more for the loads at 256^3
// FP64, the sweeps unchanged).
template <typename S>
__device__ __forceinline__ void nt_store(S* p, S x) {
  __builtin_nontemporal_store(x, p);
}
template <typename S>
__device__ __forceinline__ S nt_load(const S* p) {
  return __builtin_nontemporal_load(p);
}
template <typename S> struct NtV2;
template <> struct NtV2<float> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct NtV2<double> { typedef double T __attribute__((ext_vector_type(2))); };
template <typename S>
__device__ __forceinline__ void nt_store2(S* p, S x, S y) {
  typename NtV2<S>::T v;
  v.x = x;
  v.y = y;
  __builtin_nontemporal_store(v, reinterpret_cast<typename NtV2<S>::T*>(p));
}

// corner fluxes (eq. ox1-ox3), each from four transport fluxes:
//   Ez(i+1/2, j+1/2, k) = (Tyx(i) + Tyx(i+1))/2 - (Txy(j) + Txy(j+1))/2   [Omega_x]
//   Ex(i, j+1/2, k+1/2) = (Tzy(j) + Tzy(j+1))/2 - (Tyz(k) + Tyz(k+1))/2   [Omega_y]
//   Ey(i+1/2, j, k+1/2) = (Txz(k) + Txz(k+1))/2 - (Tzx(i) + Tzx(i+1))/2   [Omega_z]
template <typename S>
struct TView {
  const S *xy, *xz, *yz, *yx, *zx, *zy;
};

// RK = 3: SSP-RK3 (Shu-Osher) in increment form, acc = k0, k0 + k1;
//   U1 = U^n + dt k0, U2 = U^n + dt/4 (k0 + k1), U^{n+1} = U^n + dt/6 (k0 + k1 + 4 k2).
// RK = 4: the classical RK4 of Sect. 2.1 in increment form, acc = k0, k0 + 2 k1,
//   k0 + 2 k1 + 2 k2; U1 = U^n + dt/2 k0, U2 = U^n + dt/2 k1, U3 = U^n + dt k2,
//   U^{n+1} = U^n + dt/6 (k0 + 2 k1 + 2 k2 + k3) -- the paper's q_save sum
//   -4/3 q0 + q1/3 + 2 q2/3 + q3/3 + q4 written out.
template <int RK, int STAGE, typename S>
__global__ __launch_bounds__(256) void update_kernel(UpdateArgs<S> a) {
  static_assert((RK == 3 && STAGE >= 0 && STAGE < 3) || (RK == 4 && STAGE >= 0 && STAGE < 4), "stage of the scheme");
  const Grid& g = a.g;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const int im = i == 0 ? g.nx - 1 : i - 1, ip = i + 1 == g.nx ? 0 : i + 1;
  const int jm = j == 0 ? g.ny - 1 : j - 1, jp = j + 1 == g.ny ? 0 : j + 1;
  const int km = k == 0 ? g.nz - 1 : k - 1, kp = k + 1 == g.nz ? 0 : k + 1;
  const size_t N = g.N;
  const size_t c0 = g.at(i, j, k);
  const size_t cxm = g.at(im, j, k), cym = g.at(i, jm, k), czm = g.at(i, j, km);
  const double ih = a.inv_h;
  const S* Fx = a.faces;
  const S* Fy = a.faces + 5 * N;
  const S* Fz = a.faces + 10 * N;
  double kv[8];
  // the face behind the zone: at a lower wall, the flux through the wall face
  // (per-axis plane buffers indexed like the sweep's (across, plane) tiles)
  const bool lwx = g.wall[0] && i == 0, lwy = g.wall[1] && j == 0, lwz = g.wall[2] && k == 0;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const size_t o = v * N;
    const double fxm = lwx ? double(a.wallF[0][(size_t)v * g.ny * g.nz + j + (size_t)g.ny * k]) : double(Fx[o + cxm]);
    const double fym = lwy ? double(a.wallF[1][(size_t)v * g.nx * g.nz + i + (size_t)g.nx * k]) : double(Fy[o + cym]);
    const double fzm = lwz ? double(a.wallF[2][(size_t)v * g.nx * g.ny + i + (size_t)g.nx * j]) : double(Fz[o + czm]);
    const double dx = -(double(Fx[o + c0]) - fxm) * ih;
    const double dy = -(double(Fy[o + c0]) - fym) * ih;
    const double dz = -(double(Fz[o + c0]) - fzm) * ih;
    kv[v] = (dx + dy) + dz;
  }
  TView<S> T;
  T.xy = a.faces + 15 * N; T.xz = a.faces + 16 * N;
  T.yz = a.faces + 17 * N; T.yx = a.faces + 18 * N;
  T.zx = a.faces + 19 * N; T.zy = a.faces + 20 * N;
  // corner fluxes on edges that lie in a wall plane vanish (conducting wall);
  // with walls the lower wall's edges wrap to index n-1, the upper wall's
  auto Ez = [&](int ii, int jj, int kk) -> double {
    if ((g.wall[0] && ii == g.nx - 1) || (g.wall[1] && jj == g.ny - 1)) return 0.0;
    const int iip = ii + 1 == g.nx ? 0 : ii + 1, jjp = jj + 1 == g.ny ? 0 : jj + 1;
    return 0.5 * (double(T.yx[g.at(ii, jj, kk)]) + double(T.yx[g.at(iip, jj, kk)])) -
           0.5 * (double(T.xy[g.at(ii, jj, kk)]) + double(T.xy[g.at(ii, jjp, kk)]));
  };
  auto Ex = [&](int ii, int jj, int kk) -> double {
    if ((g.wall[1] && jj == g.ny - 1) || (g.wall[2] && kk == g.nz - 1)) return 0.0;
    const int jjp = jj + 1 == g.ny ? 0 : jj + 1, kkp = kk + 1 == g.nz ? 0 : kk + 1;
    return 0.5 * (double(T.zy[g.at(ii, jj, kk)]) + double(T.zy[g.at(ii, jjp, kk)])) -
           0.5 * (double(T.yz[g.at(ii, jj, kk)]) + double(T.yz[g.at(ii, jj, kkp)]));
  };
  auto Ey = [&](int ii, int jj, int kk) -> double {
    if ((g.wall[0] && ii == g.nx - 1) || (g.wall[2] && kk == g.nz - 1)) return 0.0;
    const int iip = ii + 1 == g.nx ? 0 : ii + 1, kkp = kk + 1 == g.nz ? 0 : kk + 1;
    return 0.5 * (double(T.xz[g.at(ii, jj, kk)]) + double(T.xz[g.at(ii, jj, kkp)])) -
           0.5 * (double(T.zx[g.at(ii, jj, kk)]) + double(T.zx[g.at(iip, jj, kk)]));
  };
  (void)ip; (void)jp; (void)kp;
  const double ez = Ez(i, j, k), ez_jm = Ez(i, jm, k), ez_im = Ez(im, j, k);
  const double ex = Ex(i, j, k), ex_km = Ex(i, j, km), ex_jm = Ex(i, jm, k);
  const double ey = Ey(i, j, k), ey_km = Ey(i, j, km), ey_im = Ey(im, j, k);
  // Sect. 2.3 face-field equations
  kv[5] = -(ez - ez_jm) * ih + (ey - ey_km) * ih;
  kv[6] = -(ex - ex_km) * ih + (ez - ez_im) * ih;
  kv[7] = -(ey - ey_im) * ih + (ex - ex_jm) * ih;
  // the normal field on a wall face stays zero
  if (g.wall[0] && i == g.nx - 1) kv[5] = 0.0;
  if (g.wall[1] && j == g.ny - 1) kv[6] = 0.0;
  if (g.wall[2] && k == g.nz - 1) kv[7] = 0.0;

  if (a.rhs_out) {
#pragma unroll
    for (int v = 0; v < 8; ++v) a.rhs_out[v * N + c0] = kv[v];
    return;
  }
  const double dt = *a.dt;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const double un = double(nt_load(v < 5 ? a.Un + v * N + c0 : a.bn + (v - 5) * N + c0));
    double out;
    if constexpr (RK == 3) {
      if constexpr (STAGE == 0) {
        nt_store(a.acc + v * N + c0, S(kv[v]));
        out = un + dt * kv[v];
      } else if constexpr (STAGE == 1) {
        const double s = double(nt_load(a.acc + v * N + c0)) + kv[v];
        nt_store(a.acc + v * N + c0, S(s));
        out = un + (0.25 * dt) * s;
      } else {
        const double s = double(nt_load(a.acc + v * N + c0)) + 4.0 * kv[v];
        out = un + (dt / 6.0) * s;
      }
    } else {
      if constexpr (STAGE == 0) {
        nt_store(a.acc + v * N + c0, S(kv[v]));
        out = un + (0.5 * dt) * kv[v];
      } else if constexpr (STAGE < 3) {
        nt_store(a.acc + v * N + c0, S(double(nt_load(a.acc + v * N + c0)) + 2.0 * kv[v]));
        out = un + (STAGE == 1 ? 0.5 * dt : dt) * kv[v];
      } else {
        const double s = double(nt_load(a.acc + v * N + c0)) + kv[v];
        out = un + (dt / 6.0) * s;
      }
    }
    if (v < 5) nt_store(a.hyd_out + v * N + c0, S(out));
    else nt_store(a.b_out + (v - 5) * N + c0, S(out));
  }
}

// Two storage values as one load or store (8 bytes for float, 16 for double).
template <typename S> struct Pair2;
template <> struct Pair2<float> { using T = float2; };
template <> struct Pair2<double> { using T = double2; };

// The update with two x-adjacent zones (i0 even, i0 + 1) per thread: every load
// and store of the zone pair is one vector access, so a wave keeps more bytes
// in flight per instruction (with 4-byte values, one zone per thread keeps
// half the bytes of the FP64 kernel, and the update is bound by the latency
// of its many streams).  Needs nx even and arrays at even element offsets.
// Blocks of PAIR_ROW_ZONES x PAIR_ROWS zones: long rows (a wave covers 128
// contiguous zones of a row) keep the x-neighbour reads at the row ends few;
// 256 x 2 measured 1.252 ms per FP64 update at 256^3 against 1.260 (128 x 4)
// and 1.329 (64 x 8), and 0.632 ms against 0.643 and 0.700 for the FP32 state.
// Each zone's arithmetic is update_kernel's, term by term in the same order
// (the compiler may still fuse a different product into an FMA).
constexpr int PAIR_ROW_ZONES = 256;
constexpr int PAIR_ROWS = 2 * 256 / PAIR_ROW_ZONES;   // 256 threads, two zones each
template <int RK, int STAGE, typename S>
__global__ __launch_bounds__(256) void update_pair_kernel(UpdateArgs<S> a) {
  using V2 = typename Pair2<S>::T;
  static_assert((RK == 3 && STAGE >= 0 && STAGE < 3) || (RK == 4 && STAGE >= 0 && STAGE < 4), "stage of the scheme");
  const Grid& g = a.g;
  const int i0 = blockIdx.x * PAIR_ROW_ZONES + 2 * (threadIdx.x % (PAIR_ROW_ZONES / 2));
  const int j = blockIdx.y * PAIR_ROWS + threadIdx.x / (PAIR_ROW_ZONES / 2);
  const int k = blockIdx.z;
  if (i0 >= g.nx || j >= g.ny) return;
  const int nx = g.nx;
  const int jm = j == 0 ? g.ny - 1 : j - 1, jp = j + 1 == g.ny ? 0 : j + 1;
  const int km = k == 0 ? g.nz - 1 : k - 1, kp = k + 1 == g.nz ? 0 : k + 1;
  const int imm = i0 == 0 ? nx - 2 : i0 - 2;          // pair holding zone i0 - 1 (as .y)
  const int ipp = i0 + 2 == nx ? 0 : i0 + 2;          // pair holding zone i0 + 2 (as .x)
  const size_t N = g.N;
  const size_t c0 = g.at(i0, j, k);
  const double ih = a.inv_h;
  struct D2 { double x, y; };
  auto pr = [&](const S* q, int jj, int kk) -> D2 {      // zones i0, i0 + 1
    const V2 t = *reinterpret_cast<const V2*>(q + g.at(i0, jj, kk));
    return {double(t.x), double(t.y)};
  };
  auto lo = [&](const S* q, int jj, int kk) -> double {  // zone i0 - 1
    return double(reinterpret_cast<const V2*>(q + g.at(imm, jj, kk))->y);
  };
  auto hi = [&](const S* q, int jj, int kk) -> double {  // zone i0 + 2
    return double(reinterpret_cast<const V2*>(q + g.at(ipp, jj, kk))->x);
  };
  const S* Fx = a.faces;
  const S* Fy = a.faces + 5 * N;
  const S* Fz = a.faces + 10 * N;
  double kv[2][8];
  const bool lwx = g.wall[0] && i0 == 0, lwy = g.wall[1] && j == 0, lwz = g.wall[2] && k == 0;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const size_t o = v * N;
    const D2 fx = pr(Fx + o, j, k), fy = pr(Fy + o, j, k), fz = pr(Fz + o, j, k);
    const double fxm0 = lwx ? double(a.wallF[0][(size_t)v * g.ny * g.nz + j + (size_t)g.ny * k]) : lo(Fx + o, j, k);
    D2 fym, fzm;
    // the wall-face planes may start at an odd element offset: two scalar loads
    if (lwy) {
      const S* w = a.wallF[1] + (size_t)v * nx * g.nz + i0 + (size_t)nx * k;
      fym = {double(w[0]), double(w[1])};
    } else {
      fym = pr(Fy + o, jm, k);
    }
    if (lwz) {
      const S* w = a.wallF[2] + (size_t)v * nx * g.ny + i0 + (size_t)nx * j;
      fzm = {double(w[0]), double(w[1])};
    } else {
      fzm = pr(Fz + o, j, km);
    }
    kv[0][v] = (-(fx.x - fxm0) * ih + -(fy.x - fym.x) * ih) + -(fz.x - fzm.x) * ih;
    kv[1][v] = (-(fx.y - fx.x) * ih + -(fy.y - fym.y) * ih) + -(fz.y - fzm.y) * ih;
  }
  const S* Txy = a.faces + 15 * N;
  const S* Txz = a.faces + 16 * N;
  const S* Tyz = a.faces + 17 * N;
  const S* Tyx = a.faces + 18 * N;
  const S* Tzx = a.faces + 19 * N;
  const S* Tzy = a.faces + 20 * N;
  // corner fluxes (eq. ox1-ox3) as in update_kernel; x positions: m = i0 - 1,
  // 0 = i0, 1 = i0 + 1, p = i0 + 2; zero on edges in a wall plane
  const bool w0top = g.wall[0] && i0 + 1 == nx - 1;   // zone i0 + 1's upper x edge lies in the wall
  const bool w1 = g.wall[1], w2 = g.wall[2];
  const bool w0m = g.wall[0] && i0 == 0;              // the edge below zone i0 (index nx - 1) is a wall edge
  // Ez(ii, jj) = (Tyx(ii) + Tyx(ii+1))/2 - (Txy(jj) + Txy(jj+1))/2
  const D2 yxj = pr(Tyx, j, k), yxm = pr(Tyx, jm, k);
  const double yxj_m = lo(Tyx, j, k), yxj_p = hi(Tyx, j, k), yxm_p = hi(Tyx, jm, k);
  const D2 xyj = pr(Txy, j, k), xyp = pr(Txy, jp, k), xym = pr(Txy, jm, k);
  const double xyj_m = lo(Txy, j, k), xyp_m = lo(Txy, jp, k);
  const bool zj = w1 && j == g.ny - 1, zjm = w1 && jm == g.ny - 1;
  const double ez0 = zj ? 0.0 : 0.5 * (yxj.x + yxj.y) - 0.5 * (xyj.x + xyp.x);
  const double ez1 = (zj || w0top) ? 0.0 : 0.5 * (yxj.y + yxj_p) - 0.5 * (xyj.y + xyp.y);
  const double ezm = (zj || w0m) ? 0.0 : 0.5 * (yxj_m + yxj.x) - 0.5 * (xyj_m + xyp_m);
  const double ez0_jm = zjm ? 0.0 : 0.5 * (yxm.x + yxm.y) - 0.5 * (xym.x + xyj.x);
  const double ez1_jm = (zjm || w0top) ? 0.0 : 0.5 * (yxm.y + yxm_p) - 0.5 * (xym.y + xyj.y);
  // Ex(jj, kk) = (Tzy(jj) + Tzy(jj+1))/2 - (Tyz(kk) + Tyz(kk+1))/2, at each zone's own x
  const D2 zy_jk = pr(Tzy, j, k), zy_pk = pr(Tzy, jp, k), zy_jkm = pr(Tzy, j, km), zy_pkm = pr(Tzy, jp, km);
  const D2 zy_mk = pr(Tzy, jm, k);
  const D2 yz_jk = pr(Tyz, j, k), yz_jkp = pr(Tyz, j, kp), yz_jkm = pr(Tyz, j, km), yz_mk = pr(Tyz, jm, k),
           yz_mkp = pr(Tyz, jm, kp);
  const bool zk = w2 && k == g.nz - 1, zkm = w2 && km == g.nz - 1;
  auto exf = [](double a0, double a1, double b0, double b1) { return 0.5 * (a0 + a1) - 0.5 * (b0 + b1); };
  const double ex0 = (zj || zk) ? 0.0 : exf(zy_jk.x, zy_pk.x, yz_jk.x, yz_jkp.x);
  const double ex1 = (zj || zk) ? 0.0 : exf(zy_jk.y, zy_pk.y, yz_jk.y, yz_jkp.y);
  const double ex0_km = (zj || zkm) ? 0.0 : exf(zy_jkm.x, zy_pkm.x, yz_jkm.x, yz_jk.x);
  const double ex1_km = (zj || zkm) ? 0.0 : exf(zy_jkm.y, zy_pkm.y, yz_jkm.y, yz_jk.y);
  const double ex0_jm = (zjm || zk) ? 0.0 : exf(zy_mk.x, zy_jk.x, yz_mk.x, yz_mkp.x);
  const double ex1_jm = (zjm || zk) ? 0.0 : exf(zy_mk.y, zy_jk.y, yz_mk.y, yz_mkp.y);
  // Ey(ii, kk) = (Txz(kk) + Txz(kk+1))/2 - (Tzx(ii) + Tzx(ii+1))/2
  const D2 xzk = pr(Txz, j, k), xzp = pr(Txz, j, kp), xzm = pr(Txz, j, km);
  const double xzk_m = lo(Txz, j, k), xzp_m = lo(Txz, j, kp);
  const D2 zxk = pr(Tzx, j, k), zxm = pr(Tzx, j, km);
  const double zxk_m = lo(Tzx, j, k), zxk_p = hi(Tzx, j, k), zxm_p = hi(Tzx, j, km);
  const double ey0 = zk ? 0.0 : 0.5 * (xzk.x + xzp.x) - 0.5 * (zxk.x + zxk.y);
  const double ey1 = (zk || w0top) ? 0.0 : 0.5 * (xzk.y + xzp.y) - 0.5 * (zxk.y + zxk_p);
  const double eym = (zk || w0m) ? 0.0 : 0.5 * (xzk_m + xzp_m) - 0.5 * (zxk_m + zxk.x);
  const double ey0_km = zkm ? 0.0 : 0.5 * (xzm.x + xzk.x) - 0.5 * (zxm.x + zxm.y);
  const double ey1_km = (zkm || w0top) ? 0.0 : 0.5 * (xzm.y + xzk.y) - 0.5 * (zxm.y + zxm_p);
  // Sect. 2.3 face-field equations, per zone
  const double ez[2] = {ez0, ez1}, ez_jm[2] = {ez0_jm, ez1_jm}, ez_im[2] = {ezm, ez0};
  const double ex[2] = {ex0, ex1}, ex_km[2] = {ex0_km, ex1_km}, ex_jm[2] = {ex0_jm, ex1_jm};
  const double ey[2] = {ey0, ey1}, ey_km[2] = {ey0_km, ey1_km}, ey_im[2] = {eym, ey0};
#pragma unroll
  for (int z = 0; z < 2; ++z) {
    kv[z][5] = -(ez[z] - ez_jm[z]) * ih + (ey[z] - ey_km[z]) * ih;
    kv[z][6] = -(ex[z] - ex_km[z]) * ih + (ez[z] - ez_im[z]) * ih;
    kv[z][7] = -(ey[z] - ey_im[z]) * ih + (ex[z] - ex_jm[z]) * ih;
  }
  if (g.wall[0] && i0 + 1 == nx - 1) kv[1][5] = 0.0;
  if (g.wall[1] && j == g.ny - 1) { kv[0][6] = 0.0; kv[1][6] = 0.0; }
  if (g.wall[2] && k == g.nz - 1) { kv[0][7] = 0.0; kv[1][7] = 0.0; }

  if (a.rhs_out) {
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      a.rhs_out[v * N + c0] = kv[0][v];
      a.rhs_out[v * N + c0 + 1] = kv[1][v];
    }
    return;
  }
  const double dt = *a.dt;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const S* unp = v < 5 ? a.Un + v * N : a.bn + (v - 5) * N;
    using NV = typename NtV2<S>::T;
    const NV u = __builtin_nontemporal_load(reinterpret_cast<const NV*>(unp + c0));
    const double un[2] = {double(u.x), double(u.y)};
    V2* accp = reinterpret_cast<V2*>(a.acc + v * N + c0);
    double out[2], acc_new[2];
    double acc_old[2] = {0.0, 0.0};
    if constexpr (STAGE > 0) {
      const NV t = __builtin_nontemporal_load(reinterpret_cast<const NV*>(accp));
      acc_old[0] = double(t.x);
      acc_old[1] = double(t.y);
    }
#pragma unroll
    for (int z = 0; z < 2; ++z) {
      if constexpr (RK == 3) {
        if constexpr (STAGE == 0) {
          acc_new[z] = kv[z][v];
          out[z] = un[z] + dt * kv[z][v];
        } else if constexpr (STAGE == 1) {
          const double s = acc_old[z] + kv[z][v];
          acc_new[z] = s;
          out[z] = un[z] + (0.25 * dt) * s;
        } else {
          const double s = acc_old[z] + 4.0 * kv[z][v];
          out[z] = un[z] + (dt / 6.0) * s;
        }
      } else {
        if constexpr (STAGE == 0) {
          acc_new[z] = kv[z][v];
          out[z] = un[z] + (0.5 * dt) * kv[z][v];
        } else if constexpr (STAGE < 3) {
          acc_new[z] = acc_old[z] + 2.0 * kv[z][v];
          out[z] = un[z] + (STAGE == 1 ? 0.5 * dt : dt) * kv[z][v];
        } else {
          const double s = acc_old[z] + kv[z][v];
          out[z] = un[z] + (dt / 6.0) * s;
        }
      }
    }
    constexpr bool writes_acc = RK == 3 ? STAGE < 2 : STAGE < 3;
    if constexpr (writes_acc) {
      nt_store2(a.acc + v * N + c0, S(acc_new[0]), S(acc_new[1]));
    }
    S* outp = v < 5 ? a.hyd_out + v * N : a.b_out + (v - 5) * N;
    nt_store2(outp + c0, S(out[0]), S(out[1]));
  }
}

// zone B = (-b_{i-2} + 9 b_{i-1} + 9 b_i - b_{i+1}) / 16 along each component's own axis
// Blocks of BCELL_ROW_ZONES x BCELL_ROWS zones (256 threads): 64 x 4 measured
// 0.191 ms per 256^3 FP64 pass against 0.192 (128 x 2) and 0.200 (256 x 1).
constexpr int BCELL_ROW_ZONES = 64;
constexpr int BCELL_ROWS = 256 / BCELL_ROW_ZONES;
template <typename S>
__global__ __launch_bounds__(256) void bcell_kernel(Grid g, const S* b, S* B) {
  const int i = blockIdx.x * BCELL_ROW_ZONES + threadIdx.x % BCELL_ROW_ZONES;
  const int j = blockIdx.y * BCELL_ROWS + threadIdx.x / BCELL_ROW_ZONES;
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const size_t N = g.N, c0 = g.at(i, j, k);
  const S* bx = b;
  const S* by = b + N;
  const S* bz = b + 2 * N;
  int ix[4], iy[4], iz[4];
  double sx[4], sy[4], sz[4];
  face_stencil(i, g.nx, g.wall[0], ix, sx);
  face_stencil(j, g.ny, g.wall[1], iy, sy);
  face_stencil(k, g.nz, g.wall[2], iz, sz);
  double vx[4], vy[4], vz[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    vx[q] = double(bx[g.at(ix[q], j, k)]);
    vy[q] = double(by[g.at(i, iy[q], k)]);
    vz[q] = double(bz[g.at(i, j, iz[q])]);
  }
  // the sign after the loads (a select, so the zero face ignores the value read)
  auto sgn = [](double s, double v) { return s == 1.0 ? v : (s == 0.0 ? 0.0 : -v); };
  auto interp = [&](const double* v, const double* sg) {
    return (-sgn(sg[0], v[0]) + 9.0 * sgn(sg[1], v[1]) + 9.0 * sgn(sg[2], v[2]) - sgn(sg[3], v[3])) * (1.0 / 16.0);
  };
  B[c0] = S(interp(vx, sx));
  B[N + c0] = S(interp(vy, sy));
  B[2 * N + c0] = S(interp(vz, sz));
}

// b = B0 + curl_h A (first-order differences on the edge potential)
template <typename S>
__global__ __launch_bounds__(256) void init_b_kernel(Grid g, double inv_h, const double* A, double B0x,
                                                     double B0y, double B0z, S* b) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const size_t N = g.N, c0 = g.at(i, j, k);
  const double* Ax = A;
  const double* Ay = A + N;
  const double* Az = A + 2 * N;
  const int im = wrap(i - 1, g.nx), jm = wrap(j - 1, g.ny), km = wrap(k - 1, g.nz);
  b[c0] = S(B0x + ((Az[c0] - Az[g.at(i, jm, k)]) * inv_h - (Ay[c0] - Ay[g.at(i, j, km)]) * inv_h));
  b[N + c0] = S(B0y + ((Ax[c0] - Ax[g.at(i, j, km)]) * inv_h - (Az[c0] - Az[g.at(im, j, k)]) * inv_h));
  b[2 * N + c0] = S(B0z + ((Ay[c0] - Ay[g.at(im, j, k)]) * inv_h - (Ax[c0] - Ax[g.at(i, jm, k)]) * inv_h));
  // a wall face carries no normal field
  if (g.wall[0] && i == g.nx - 1) b[c0] = S(0.0);
  if (g.wall[1] && j == g.ny - 1) b[N + c0] = S(0.0);
  if (g.wall[2] && k == g.nz - 1) b[2 * N + c0] = S(0.0);
}

// m = rho v, E = P0/(gamma-1) + (rho v^2 + B^2)/2 (zone B already interpolated)
template <typename S>
__global__ __launch_bounds__(256) void init_hydro_kernel(size_t N, double gamma, double P0, const double* rho,
                                                         const double* v, const S* B, S* hydro) {
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= N) return;
  const double r = rho[c];
  const double vx = v[c], vy = v[N + c], vz = v[2 * N + c];
  const double Bx = B[c], By = B[N + c], Bz = B[2 * N + c];
  hydro[c] = S(r);
  hydro[N + c] = S(r * vx);
  hydro[2 * N + c] = S(r * vy);
  hydro[3 * N + c] = S(r * vz);
  hydro[4 * N + c] = S(P0 / (gamma - 1.0) + 0.5 * (r * (vx * vx + vy * vy + vz * vz) + (Bx * Bx + By * By + Bz * Bz)));
}

// ---------------------------------------------------------------------------
// reductions (fixed order, no atomics: results are bitwise reproducible)
// ---------------------------------------------------------------------------
constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;

// max over zones of |v_d| + c_fast^d, d = x, y, z -> part[3 * block + d] (cfl_key);
// the signal speed along d is the one the sweep along d forms (zone_prologue in
// its frame n = d, t1 = d + 1, t2 = d + 2), so a step that takes the maxima from
// its first stage's sweeps finds bitwise the same dt
template <typename S>
__global__ __launch_bounds__(RED_THREADS) void speed_partial_kernel(size_t N, double gamma, const S* hydro,
                                                                    const S* bcell, SpeedKey* part) {
  __shared__ SpeedKey red[3][RED_THREADS];
  SpeedKey mx[3] = {0, 0, 0};
  for (size_t c = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; c < N; c += (size_t)gridDim.x * RED_THREADS) {
    const double rho = double(hydro[c]), E = double(hydro[4 * N + c]);
    const double m[3] = {double(hydro[N + c]), double(hydro[2 * N + c]), double(hydro[3 * N + c])};
    const double B[3] = {double(bcell[c]), double(bcell[N + c]), double(bcell[2 * N + c])};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
      double z[Z_NVAR];
      zone_prologue(rho, m[d], m[t1], m[t2], E, B[d], B[t1], B[t2], gamma, z);
      mx[d] = kmax(mx[d], cfl_key(z));
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = mx[d];
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = kmax(red[d][threadIdx.x], red[d][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) part[3 * blockIdx.x + d] = red[d][0];
  }
}

// The maxima of the first stage's sweeps: part holds n[0] + n[1] + n[2] block
// keys (the x, y, z sweeps in turn) -> out[3 * block + d], for dt_final_kernel
__global__ __launch_bounds__(RED_THREADS) void speed_blocks_kernel(const SpeedKey* part, unsigned n0, unsigned n1,
                                                                   unsigned n2, SpeedKey* out) {
  __shared__ SpeedKey red[3][RED_THREADS];
  const unsigned n[3] = {n0, n1, n2};
  const SpeedKey* base[3] = {part, part + n0, part + (size_t)n0 + n1};
  SpeedKey mx[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < 3; ++d)
    for (unsigned b = blockIdx.x * RED_THREADS + threadIdx.x; b < n[d]; b += gridDim.x * RED_THREADS)
      mx[d] = kmax(mx[d], base[d][b]);
#pragma unroll
  for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = mx[d];
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = kmax(red[d][threadIdx.x], red[d][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) out[3 * blockIdx.x + d] = red[d][0];
  }
}

// dt = cfl h / sum_d max_d (eq. cfl); also keeps the three maxima.  A maximum
// whose key has the sign bit set (a negative speed) or is NaN gives NaN.
__global__ __launch_bounds__(RED_THREADS) void dt_final_kernel(int nblocks, double cfl_h, const SpeedKey* part,
                                                               double* dt, double* smax) {
  __shared__ SpeedKey red[3][RED_THREADS];
  SpeedKey mx[3] = {0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) {
#pragma unroll
    for (int d = 0; d < 3; ++d) mx[d] = kmax(mx[d], part[3 * b + d]);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = mx[d];
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = kmax(red[d][threadIdx.x], red[d][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double m[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const SpeedKey k = red[d][0];
      m[d] = (k >> 63) ? __builtin_nan("") : __builtin_bit_cast(double, k);
    }
    const double s = (m[0] + m[1]) + m[2];
    *dt = cfl_h / s;
    smax[0] = m[0]; smax[1] = m[1]; smax[2] = m[2];
  }
}

__global__ void set_scalar_kernel(double* p, double v) { *p = v; }

// Opt-in floors on a stage result (hydro [5][N] with its zone field): rho below
// rho_f is raised to it (momentum kept), then P below p_f (eq. P) is raised to
// it by adding internal energy.  part[block] = activations of the block (a
// density and a pressure activation count separately).
template <typename S>
__global__ __launch_bounds__(RED_THREADS) void floor_kernel(size_t N, double gamma, double rho_f, double p_f,
                                                            S* hydro, const S* bcell, double* part) {
  __shared__ double red[RED_THREADS];
  double cnt = 0.0;
  for (size_t c = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; c < N; c += (size_t)gridDim.x * RED_THREADS) {
    double rho = hydro[c];
    if (rho_f > 0.0 && rho < rho_f) {
      rho = rho_f;
      hydro[c] = S(rho);
      cnt += 1.0;
    }
    if (p_f > 0.0) {
      const double m[3] = {hydro[N + c], hydro[2 * N + c], hydro[3 * N + c]};
      const double B[3] = {bcell[c], bcell[N + c], bcell[2 * N + c]};
      const double E = hydro[4 * N + c];
      const double r = double(S(rho));
      const double P = (gamma - 1.0) * (E - 0.5 * ((m[0] * (m[0] / r) + m[1] * (m[1] / r) + m[2] * (m[2] / r)) +
                                                   (B[0] * B[0] + B[1] * B[1] + B[2] * B[2])));
      if (P < p_f) {
        hydro[4 * N + c] = S(E + (p_f - P) / (gamma - 1.0));
        cnt += 1.0;
      }
    }
  }
  red[threadIdx.x] = cnt;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// total += sum of the block counts (one thread, fixed order)
__global__ void floor_final_kernel(int nblocks, const double* part, double* total, int reset) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = reset ? 0.0 : *total;
  for (int b = 0; b < nblocks; ++b) s += part[b];
  *total = s;
}

// diagnostics partials: per block, Neumaier sums of rho, m(3), E, b(3) and
// max|div b|, min rho, min P, unphysical count
struct Acc2 {
  double s, c;
  __device__ void add(double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
  }
};

template <typename S>
__global__ __launch_bounds__(RED_THREADS) void diag_partial_kernel(Grid g, double gamma, double inv_h,
                                                                   const S* hydro, const S* b,
                                                                   const S* bcell, double* part) {
  // part layout per block: [0..7] sums, [8..15] compensations, [16] max|divb|, [17] min rho,
  // [18] min P, [19] unphysical count
  const size_t N = g.N;
  Acc2 acc[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) { acc[v].s = 0.0; acc[v].c = 0.0; }
  double mdiv = 0.0, mrho = 1.0e308, mp = 1.0e308, nbad = 0.0;
  for (size_t c = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; c < N; c += (size_t)gridDim.x * RED_THREADS) {
    const int i = (int)(c % g.nx);
    const int j = (int)((c / g.nx) % g.ny);
    const int k = (int)(c / ((size_t)g.nx * g.ny));
    const double rho = hydro[c];
    const double m[3] = {hydro[N + c], hydro[2 * N + c], hydro[3 * N + c]};
    const double E = hydro[4 * N + c];
    acc[0].add(rho);
    acc[1].add(m[0]); acc[2].add(m[1]); acc[3].add(m[2]);
    acc[4].add(E);
    auto bf = [&](size_t q) { return double(b[q]); };
    acc[5].add(bf(c)); acc[6].add(bf(N + c)); acc[7].add(bf(2 * N + c));
    const double div = ((bf(c) - bf(g.at(wrap(i - 1, g.nx), j, k))) + (bf(N + c) - bf(N + g.at(i, wrap(j - 1, g.ny), k))) +
                        (bf(2 * N + c) - bf(2 * N + g.at(i, j, wrap(k - 1, g.nz))))) * inv_h;
    mdiv = nanmax(mdiv, fabs(div));
    const double Bx = bcell[c], By = bcell[N + c], Bz = bcell[2 * N + c];
    const double P = (gamma - 1.0) * (E - 0.5 * ((m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / rho + (Bx * Bx + By * By + Bz * Bz)));
    mrho = fmin(mrho, rho);
    mp = fmin(mp, P);
    const bool bad = !(rho > 0.0) || !(P > 0.0) || !isfinite(E) || !isfinite(rho) || !isfinite(P);
    nbad += bad ? 1.0 : 0.0;
  }
  // wave-level then block-level reduction in fixed order
  double vals[20];
#pragma unroll
  for (int v = 0; v < 8; ++v) { vals[v] = acc[v].s; vals[8 + v] = acc[v].c; }
  vals[16] = mdiv; vals[17] = mrho; vals[18] = mp; vals[19] = nbad;
  __shared__ double tmp[20][RED_THREADS];
#pragma unroll
  for (int v = 0; v < 20; ++v) tmp[v][threadIdx.x] = vals[v];
  __syncthreads();
  if (threadIdx.x == 0) {
    Acc2 s[8];
    for (int v = 0; v < 8; ++v) { s[v].s = 0.0; s[v].c = 0.0; }
    double a16 = 0.0, a17 = 1.0e308, a18 = 1.0e308, a19 = 0.0;
    for (int t = 0; t < RED_THREADS; ++t) {
      for (int v = 0; v < 8; ++v) { s[v].add(tmp[v][t]); s[v].c += tmp[8 + v][t]; }
      a16 = nanmax(a16, tmp[16][t]);
      a17 = fmin(a17, tmp[17][t]);
      a18 = fmin(a18, tmp[18][t]);
      a19 += tmp[19][t];
    }
    double* o = part + 20 * blockIdx.x;
    for (int v = 0; v < 8; ++v) { o[v] = s[v].s; o[8 + v] = s[v].c; }
    o[16] = a16; o[17] = a17; o[18] = a18; o[19] = a19;
  }
}

__global__ void diag_final_kernel(int nblocks, const double* part, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Acc2 s[8];
  for (int v = 0; v < 8; ++v) { s[v].s = 0.0; s[v].c = 0.0; }
  double a16 = 0.0, a17 = 1.0e308, a18 = 1.0e308, a19 = 0.0;
  for (int b = 0; b < nblocks; ++b) {
    const double* p = part + 20 * b;
    for (int v = 0; v < 8; ++v) { s[v].add(p[v]); s[v].c += p[8 + v]; }
    a16 = nanmax(a16, p[16]);
    a17 = fmin(a17, p[17]);
    a18 = fmin(a18, p[18]);
    a19 += p[19];
  }
  for (int v = 0; v < 8; ++v) out[v] = s[v].s + s[v].c;
  out[8] = a16; out[9] = a17; out[10] = a18; out[11] = a19;
}

}  // namespace wm
