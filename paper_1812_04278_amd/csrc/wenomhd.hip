// C ABI of the WENO5-CT MHD step (declarations and contracts in
// include/wenomhd.h).  Host-side orchestration only: argument checks, the
// scratch layout, and stream-ordered kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/wenomhd.h"
#include "adjoint_kernels.hpp"

using namespace wm;

#ifdef WM_SWEEP_CLOCK
#include "../../include/wenomhd_clock.h"
// clock build: process-wide per-axis stamp buffers (device) and their capacity
static unsigned long long* g_sweep_clk[3] = {nullptr, nullptr, nullptr};
static size_t g_sweep_clk_n[3] = {0, 0, 0};
#endif

// Device scratch of wm_step_static, for callers that cannot allocate: one copy
// of this array per GPU the library runs on, held until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// it is only a stand-in for the symbol); it uses the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {

thread_local char g_err[512] = "";

wm_status fail(wm_status s, const char* fmt, const char* detail = "") {
  std::snprintf(g_err, sizeof(g_err), fmt, detail);
  return s;
}

wm_status hip_check(hipError_t e, const char* where) {
  if (e != hipSuccess) {
    std::snprintf(g_err, sizeof(g_err), "%s: %s", where, hipGetErrorString(e));
    return WM_ERR_HIP;
  }
  return WM_OK;
}

#define WM_LAUNCH_CHECK(where)                                      \
  do {                                                              \
    wm_status _s = hip_check(hipGetLastError(), where);             \
    if (_s != WM_OK) return _s;                                     \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// scratch layout (bytes, each region 256-aligned), elements of the state's
// storage type (double, or float for WM_MIXED_F32STATE):
//   Us    [11][N]  stage state: hydro 5, bface 3, bcell 3
//   acc   [8][N]   RK increment accumulator
//   faces [21][N]  F^x, F^y, F^z (5 each), T^x, T^y, T^z (2 each)
//   red            (doubles) dt, 3 signal-speed maxima, reduction partials
//   wall  [5][ny nz] + [5][nx nz] + [5][nx ny]  lower-wall-face fluxes (walls)
struct Layout {
  size_t us, acc, faces, wall, red, total;
};

// red: dt, 3 signal-speed maxima, speed partials (3/block), diagnostics partials
// (20/block), 12 diagnostics results and the floor count, floor partials (1/block)
constexpr size_t kRedDoubles = 4 + 3 * RED_BLOCKS + 20 * RED_BLOCKS + 13 + RED_BLOCKS + 8;

bool valid_config(const wm_config* c, const char** why) {
  if (!c) { *why = "null config"; return false; }
  if (c->nx < 1 || c->ny < 1 || c->nz < 1) { *why = "grid sizes must be >= 1"; return false; }
  if (c->nx > 8192 || c->ny > 8192 || c->nz > 8192) { *why = "grid size above 8192"; return false; }
  const double n = (double)c->nx * c->ny * c->nz;
  if (n > 2147483647.0) { *why = "more than 2^31-1 zones"; return false; }
  if (!(c->h > 0.0) || !std::isfinite(c->h)) { *why = "h must be positive"; return false; }
  if (!(c->gamma > 1.0)) { *why = "gamma must exceed 1"; return false; }
  if (!(c->cfl > 0.0)) { *why = "cfl must be positive"; return false; }
  if (!(c->eps_weno > 0.0) || !(c->eps_B >= 0.0) || !(c->eps_Z > 0.0)) { *why = "epsilons must be positive"; return false; }
  if (!(c->eps_Z >= 1e-50)) { *why = "eps_Z below 1e-50 (the WENO-Z weights need eps_Z^6 in the FP64 range)"; return false; }
  if (c->weights != WM_WENO_JS && c->weights != WM_WENO_Z && c->weights != WM_WENO_Z_PRINTED) {
    *why = "unknown weights";
    return false;
  }
  if (c->precision != WM_FP64 && c->precision != WM_MIXED && c->precision != WM_MIXED_F32STATE) {
    *why = "unknown precision mode";
    return false;
  }
  if (c->integrator != WM_SSPRK3 && c->integrator != WM_RK4) { *why = "unknown integrator"; return false; }
  const int n3[3] = {c->nx, c->ny, c->nz};
  for (int d = 0; d < 3; ++d) {
    if (c->walls[d] != 0 && c->walls[d] != 1) { *why = "walls must be 0 or 1"; return false; }
    if (c->walls[d] && n3[d] < 3) { *why = "a walled axis needs at least 3 zones"; return false; }
  }
  if (!(c->rho_floor >= 0.0) || !(c->p_floor >= 0.0) || !std::isfinite(c->rho_floor) || !std::isfinite(c->p_floor)) {
    *why = "floors must be finite and >= 0";
    return false;
  }
  if ((c->rho_floor > 0.0 || c->p_floor > 0.0) && c->integrator != WM_SSPRK3) {
    *why = "floors are applied to the SSP-RK3 stages";
    return false;
  }
  return true;
}

size_t state_elem_bytes(const wm_config* c) {
  return c->precision == WM_MIXED_F32STATE ? sizeof(float) : sizeof(double);
}

Layout layout(const wm_config* c) {
  const size_t N = (size_t)c->nx * c->ny * c->nz;
  const size_t es = state_elem_bytes(c);
  Layout L;
  size_t off = 0;
  L.us = off;    off = align_up(off + 11 * N * es);
  L.acc = off;   off = align_up(off + 8 * N * es);
  L.faces = off; off = align_up(off + 21 * N * es);
  L.wall = off;
  off = align_up(off + 5 * ((size_t)c->ny * c->nz + (size_t)c->nx * c->nz + (size_t)c->nx * c->ny) * es);
  L.red = off;   off = align_up(off + kRedDoubles * sizeof(double));
  L.total = off;
  return L;
}

// adjoint scratch (doubles, N each unless noted): recomputed stage states U1,
// U2 (11 each: hydro, face b, zone B), zone B of the linearisation state (3),
// transport-flux cotangents (6), zone-B cotangent (3), rhs cotangent (8), stage
// cotangents lamU2, lamU1 (8 each), lam3 (8), then the dt slot.
enum AdjOff { A_U1 = 0, A_U2 = 11, A_BZ = 22, A_LT = 25, A_LBZ = 31, A_LK = 34, A_LU2 = 42, A_LU1 = 50,
              A_WORK = 58, A_NARR = 66,
              // RK4 only: the third stage state and its cotangent
              A_U3 = 66, A_LU3 = 77, A_NARR4 = 85 };

// Launch classes of the adjoint sweep along one axis: n zones in tiles of TA
// faces; tile t adds into the zones t*TA - 2 .. t*TA + tav + 2 (periodic).
// Neighbouring tiles on the ring share zones, and so do tiles 0 and nt-2 when
// the last tile has at most 4 zones (their halos reach into it from both
// sides).  Classes: even tiles, odd tiles, and the tile left over (nt odd:
// the last; nt even with a short last tile: tile nt-2).
struct TileRun { int first, stride, count; };
struct TilePlan { TileRun run[4]; int n; };

bool plan_disjoint(int n, int TA, const TilePlan& pl) {
  std::vector<int> stamp(n, -1);
  for (int r = 0; r < pl.n; ++r) {
    const TileRun& t = pl.run[r];
    for (int i = 0; i < t.count; ++i) {
      const int tile = t.first + i * t.stride;
      const int tav = std::min(TA, n - tile * TA);
      if (tav <= 0) return false;
      const int span = std::min(tav + SW_HL + SW_HR, n);   // distinct zones (wrapped positions are summed)
      for (int q = 0; q < span; ++q) {
        const int z = ((tile * TA - SW_HL + q) % n + n) % n;
        if (stamp[z] == r * 1000000 + tile) continue;
        if (stamp[z] >= r * 1000000) return false;       // another tile of the same class
        stamp[z] = r * 1000000 + tile;
      }
    }
  }
  // every tile in exactly one class
  std::vector<int> seen((n + TA - 1) / TA, 0);
  for (int r = 0; r < pl.n; ++r)
    for (int i = 0; i < pl.run[r].count; ++i) ++seen[pl.run[r].first + i * pl.run[r].stride];
  for (int v : seen)
    if (v != 1) return false;
  return true;
}

TilePlan plan_tiles(int n, int TA) {
  TilePlan pl{};
  const int nt = (n + TA - 1) / TA;
  const int last = n - (nt - 1) * TA;
  auto add = [&](int first, int stride, int count) {
    if (count > 0) pl.run[pl.n++] = TileRun{first, stride, count};
  };
  if (nt == 1) {
    add(0, 1, 1);
  } else if (nt % 2 == 1) {
    add(0, 2, (nt - 1) / 2);
    add(1, 2, (nt - 1) / 2);
    add(nt - 1, 1, 1);
  } else if (nt == 2 || last > SW_HL + SW_HR - 1) {
    add(0, 2, nt / 2);
    add(1, 2, nt / 2);
  } else {
    add(0, 2, nt / 2 - 1);
    add(1, 2, nt / 2);
    add(nt - 2, 1, 1);
  }
  return pl;
}

// arrays of N doubles in the adjoint scratch (the dt scalar follows them).  A
// patch with an FP32 state adds, after the arrays above, U^n widened to FP64
// (8) and room for the FP32 stage states the adjoint recomputes ([11][N]
// floats each: 11 arrays for SSP-RK3's two, 17 for RK4's three).
int adjoint_base_arrays(const wm_config* c) { return c->integrator == WM_RK4 ? A_NARR4 : A_NARR; }
int adjoint_arrays(const wm_config* c) {
  int n = adjoint_base_arrays(c);
  if (c->precision == WM_MIXED_F32STATE) n += 8 + (c->integrator == WM_RK4 ? 17 : 11);
  return n;
}

size_t adjoint_bytes(const wm_config* c) {
  const size_t N = (size_t)c->nx * c->ny * c->nz;
  return align_up(adjoint_arrays(c) * N * sizeof(double) + 256);
}

}  // namespace

struct wm_patch {
  wm_config cfg;
  hipStream_t stream;
  Grid g;
  Phys ph;
  char* scratch;
  Layout lay;
  bool f32 = false;          // state, stage states, accumulator and face values in FP32
  void* hydro = nullptr;     // bound state (storage type: double, or float when f32)
  void* bface = nullptr;
  void* bcell = nullptr;
  bool floors = false;       // opt-in floors configured
  bool floor_reset = true;   // the floor count restarts at the next floor pass
  int stage_done = -1;       // last completed stage of the current step (-1: none)
  bool dt_valid = false;
  TilePlan adj_plan[3];      // adjoint sweep launch classes per axis (grid sizes >= 3)
  // event timing (wm_profile)
  bool prof = false;
  std::vector<hipEvent_t> ev;       // pool, 2 per record
  std::vector<int> ev_class;        // kernel class per record
  size_t n_rec = 0;

  template <typename S> S* us() const { return reinterpret_cast<S*>(scratch + lay.us); }
  template <typename S> S* acc() const { return reinterpret_cast<S*>(scratch + lay.acc); }
  template <typename S> S* faces() const { return reinterpret_cast<S*>(scratch + lay.faces); }
  template <typename S> S* hyd() const { return reinterpret_cast<S*>(hydro); }
  template <typename S> S* bf() const { return reinterpret_cast<S*>(bface); }
  template <typename S> S* bc() const { return reinterpret_cast<S*>(bcell); }
  double* red() const { return reinterpret_cast<double*>(scratch + lay.red); }
  double* dt_dev() const { return red(); }                 // red[0]
  double* smax_dev() const { return red() + 1; }           // red[1..3]
  double* diag_out() const { return red() + 4 + 3 * RED_BLOCKS + 20 * RED_BLOCKS; }  // 12 values + floor count
  double* floor_total() const { return diag_out() + 12; }
  double* floor_part() const { return diag_out() + 13; }
  // lower-wall-face fluxes of a walled axis: [5][nB * nC], the sweep's (across, plane) order
  template <typename S> S* wallF(int axis) const {
    S* w = reinterpret_cast<S*>(scratch + lay.wall);
    const size_t yz = (size_t)g.ny * g.nz, xz = (size_t)g.nx * g.nz;
    return axis == 0 ? w : (axis == 1 ? w + 5 * yz : w + 5 * (yz + xz));
  }
  SpeedKey* speed_part() const { return reinterpret_cast<SpeedKey*>(red() + 4); }   // cfl_key maxima
  double* diag_part() const { return red() + 4 + 3 * RED_BLOCKS; }
};

namespace {

constexpr size_t kMaxRec = 8192;
enum KClass { K_SWEEP = 0, K_UPDATE = 1, K_BCELL = 2, K_DT = 3, K_OTHER = 4, K_NCLASS = 5 };

// Records a start event before a launch of class c; returns the record index or -1.
long prof_begin(wm_patch* p, int c) {
  if (!p->prof || p->n_rec >= kMaxRec) return -1;
  const size_t r = p->n_rec;
  while (p->ev.size() < 2 * (r + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    p->ev.push_back(e);
  }
  if (p->ev_class.size() < r + 1) p->ev_class.resize(r + 1);
  p->ev_class[r] = c;
  if (hipEventRecord(p->ev[2 * r], p->stream) != hipSuccess) return -1;
  return (long)r;
}

void prof_end(wm_patch* p, long r) {
  if (r < 0) return;
  if (hipEventRecord(p->ev[2 * r + 1], p->stream) == hipSuccess) p->n_rec = (size_t)r + 1;
}

dim3 zone_grid(const Grid& g) { return dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz); }

// Runs fn(S{}) with S the patch's storage type.
template <class Fn>
wm_status with_storage(const wm_patch* p, Fn&& fn) {
  return p->f32 ? fn(float{}) : fn(double{});
}

// Launch grid of the sweep along AXIS: the tile depends on the work type
// (FP32 for the FP32 state and the mixed form); with walls the sweep also
// computes the lower wall face (-1/2)
template <int AXIS>
dim3 sweep_grid(const wm_patch* p) {
  const int nA = AXIS == 0 ? p->g.nx : (AXIS == 1 ? p->g.ny : p->g.nz);
  const int nB = AXIS == 0 ? p->g.ny : p->g.nx;
  const int nC = AXIS == 2 ? p->g.ny : p->g.nz;
  auto grid_for = [&](auto tw) {
    using TW = decltype(tw);
    constexpr int TA = SweepTile<AXIS, TW>::TA, TB = SweepTile<AXIS, TW>::TB;
    return dim3((nA + p->g.wall[AXIS] + TA - 1) / TA, (nB + TB - 1) / TB, nC);
  };
  const bool f32_work = p->f32 || p->cfg.precision == WM_MIXED;
  return f32_work ? grid_for(float{}) : grid_for(double{});
}

size_t sweep_blocks(const dim3& g) { return (size_t)g.x * g.y * g.z; }

template <int AXIS, typename S>
wm_status launch_sweep(wm_patch* p, const S* hydro, const S* bcell, S* fh, S* T, double* dbg,
                       SpeedKey* smax_blk = nullptr) {
  SweepArgs<S> a;
  a.g = p->g;
  a.ph = p->ph;
  a.hydro = hydro;
  a.bcell = bcell;
  a.fhydro = fh;
  a.T = T;
  a.dbg = dbg;
  a.wallF = p->g.wall[AXIS] ? p->wallF<S>(AXIS) : nullptr;
  a.smax_blk = smax_blk;
#ifdef WM_SWEEP_CLOCK
  a.clk = nullptr;
#endif
  const dim3 grid = sweep_grid<AXIS>(p);
#ifdef WM_SWEEP_CLOCK
  if ((size_t)grid.x * grid.y * grid.z * (SW_THREADS / 64) * 8 <= g_sweep_clk_n[AXIS]) a.clk = g_sweep_clk[AXIS];
#endif
  const long r = prof_begin(p, K_SWEEP);
  // kernel choice: work type (FP32 for the FP32 state and the mixed form),
  // weights, and whether the block writes its signal-speed maximum
  auto go = [&](auto tw, auto wz, auto dtmax) {
    hipLaunchKernelGGL((sweep_kernel<AXIS, decltype(wz)::value, decltype(tw), S, decltype(dtmax)::value>), grid,
                       dim3(SW_THREADS), 0, p->stream, a);
  };
  auto pick_dt = [&](auto tw, auto wz) {
    if (smax_blk) go(tw, wz, std::true_type{});
    else go(tw, wz, std::false_type{});
  };
  auto pick_wz = [&](auto tw) {
    if (p->ph.weno_z) pick_dt(tw, std::true_type{});
    else pick_dt(tw, std::false_type{});
  };
  if constexpr (sizeof(S) == 4) {   // FP32 state: the mixed arithmetic
    pick_wz(float{});
  } else {
    if (p->cfg.precision == WM_MIXED) pick_wz(float{});
    else pick_wz(double{});
  }
  WM_LAUNCH_CHECK("sweep kernel");
  prof_end(p, r);
  return WM_OK;
}

// smax: optional, the per-wave signal-speed maxima of the three sweeps in turn
// (4 per block of each axis' grid), for the fused time step
template <typename S>
wm_status sweeps(wm_patch* p, const S* hydro, const S* bcell, SpeedKey* smax = nullptr) {
  const size_t N = p->g.N;
  S* f = p->faces<S>();
  SpeedKey* s1 = smax ? smax + 4 * sweep_blocks(sweep_grid<0>(p)) : nullptr;
  SpeedKey* s2 = smax ? s1 + 4 * sweep_blocks(sweep_grid<1>(p)) : nullptr;
  wm_status s;
  if ((s = launch_sweep<0, S>(p, hydro, bcell, f, f + 15 * N, nullptr, smax)) != WM_OK) return s;
  if ((s = launch_sweep<1, S>(p, hydro, bcell, f + 5 * N, f + 17 * N, nullptr, s1)) != WM_OK) return s;
  if ((s = launch_sweep<2, S>(p, hydro, bcell, f + 10 * N, f + 19 * N, nullptr, s2)) != WM_OK) return s;
  return WM_OK;
}

int n_stages(const wm_patch* p) { return p->cfg.integrator == WM_RK4 ? 4 : 3; }

// Launches the update of one stage: with nx even and every array aligned to
// two elements, the two-zone kernel (vector loads), else one zone per thread.
constexpr bool kUpdatePairs = true;
template <int RK, int STAGE, typename S>
void launch_update_kernel(wm_patch* p, const UpdateArgs<S>& a) {
  if (kUpdatePairs) {
    auto al = [](const void* q) { return q == nullptr || (reinterpret_cast<uintptr_t>(q) % (2 * sizeof(S))) == 0; };
    const bool pair = p->g.nx % 2 == 0 && al(a.faces) && al(a.Un) && al(a.bn) && al(a.acc) && al(a.hyd_out) &&
                      al(a.b_out);
    if (pair) {
      const dim3 grid((p->g.nx + PAIR_ROW_ZONES - 1) / PAIR_ROW_ZONES, (p->g.ny + PAIR_ROWS - 1) / PAIR_ROWS, p->g.nz);
      hipLaunchKernelGGL((update_pair_kernel<RK, STAGE, S>), grid, dim3(256), 0, p->stream, a);
      return;
    }
  }
  hipLaunchKernelGGL((update_kernel<RK, STAGE, S>), zone_grid(p->g), dim3(256), 0, p->stream, a);
}

template <typename S>
void launch_update_stage(wm_patch* p, const UpdateArgs<S>& a, bool rk4, int stage) {
  if (rk4) {
    switch (stage) {
      case 0: launch_update_kernel<4, 0, S>(p, a); break;
      case 1: launch_update_kernel<4, 1, S>(p, a); break;
      case 2: launch_update_kernel<4, 2, S>(p, a); break;
      default: launch_update_kernel<4, 3, S>(p, a); break;
    }
  } else {
    switch (stage) {
      case 0: launch_update_kernel<3, 0, S>(p, a); break;
      case 1: launch_update_kernel<3, 1, S>(p, a); break;
      default: launch_update_kernel<3, 2, S>(p, a); break;
    }
  }
}

template <typename S>
wm_status launch_update(wm_patch* p, int stage, double* rhs_out) {
  const size_t N = p->g.N;
  UpdateArgs<S> a;
  a.g = p->g;
  a.inv_h = 1.0 / p->cfg.h;
  a.faces = p->faces<S>();
  a.Un = p->hyd<S>();
  a.bn = p->bf<S>();
  a.acc = p->acc<S>();
  a.rhs_out = rhs_out;
  a.dt = p->dt_dev();
  for (int d = 0; d < 3; ++d) a.wallF[d] = p->g.wall[d] ? p->wallF<S>(d) : nullptr;
  if (stage == n_stages(p) - 1) {
    a.hyd_out = p->hyd<S>();
    a.b_out = p->bf<S>();
  } else {
    a.hyd_out = p->us<S>();
    a.b_out = p->us<S>() + 5 * N;
  }
  const long r = prof_begin(p, K_UPDATE);
  launch_update_stage<S>(p, a, p->cfg.integrator == WM_RK4, stage);
  WM_LAUNCH_CHECK("update kernel");
  prof_end(p, r);
  return WM_OK;
}

template <typename S>
wm_status launch_bcell(wm_patch* p, const S* b, S* B) {
  const long r = prof_begin(p, K_BCELL);
  const dim3 grid((p->g.nx + BCELL_ROW_ZONES - 1) / BCELL_ROW_ZONES, (p->g.ny + BCELL_ROWS - 1) / BCELL_ROWS, p->g.nz);
  hipLaunchKernelGGL(bcell_kernel<S>, grid, dim3(256), 0, p->stream, p->g, b, B);
  WM_LAUNCH_CHECK("bcell kernel");
  prof_end(p, r);
  return WM_OK;
}

int red_blocks(const Grid& g) {
  size_t b = (g.N + RED_THREADS - 1) / RED_THREADS;
  return (int)(b < (size_t)RED_BLOCKS ? b : (size_t)RED_BLOCKS);
}

wm_status check_bound(wm_patch* p) {
  if (!p) return fail(WM_ERR_ARG, "null patch");
  if (!p->hydro || !p->bface || !p->bcell) return fail(WM_ERR_STATE, "state not bound (wm_bind_state)");
  return WM_OK;
}

dim3 lin_grid(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

template <int AXIS>
wm_status launch_adj_sweep(wm_patch* p, const double* hydro, const double* bcell, const double* lam_k,
                           const double* lam_T, double* acc_h, double* lam_Bz) {
  AdjSweepArgs a;
  a.g = p->g;
  a.ph = p->ph;
  a.inv_h = 1.0 / p->cfg.h;
  a.hydro = hydro;
  a.bcell = bcell;
  a.lam_k = lam_k;
  a.lam_T = lam_T;
  a.lam_h = acc_h;
  a.lam_Bz = lam_Bz;
  const int nB = AXIS == 0 ? p->g.ny : p->g.nx;
  const int nC = AXIS == 2 ? p->g.ny : p->g.nz;
  constexpr int TB = AdjTile<AXIS>::TB;
  const TilePlan& pl = p->adj_plan[AXIS];
  const long r = prof_begin(p, K_OTHER);
  for (int c = 0; c < pl.n; ++c) {   // classes in order: each launch adds into disjoint zones
    a.tile0 = pl.run[c].first;
    a.tstride = pl.run[c].stride;
    const dim3 grid(pl.run[c].count, (nB + TB - 1) / TB, nC);
    if (p->ph.weno_z) hipLaunchKernelGGL((adj_sweep_kernel<AXIS, true>), grid, dim3(ADJ_THREADS), 0, p->stream, a);
    else hipLaunchKernelGGL((adj_sweep_kernel<AXIS, false>), grid, dim3(ADJ_THREADS), 0, p->stream, a);
    WM_LAUNCH_CHECK("adjoint sweep kernel");
  }
  prof_end(p, r);
  return WM_OK;
}

wm_status check_adjoint(wm_patch* p, void* adj) {
  if (!p) return fail(WM_ERR_ARG, "null patch");
  if (!adj || reinterpret_cast<uintptr_t>(adj) % kAlign) return fail(WM_ERR_ARG, "adjoint scratch null or misaligned");
  if (p->cfg.nx < 3 || p->cfg.ny < 3 || p->cfg.nz < 3) return fail(WM_ERR_ARG, "the adjoint needs grid sizes >= 3");
  if (p->g.wall[0] || p->g.wall[1] || p->g.wall[2] || p->floors)
    return fail(WM_ERR_ARG, "the adjoint is for periodic boxes without floors");
  return WM_OK;
}

// (dL/dU)^T lam_k at U = (hydro, bface) -> out (hydro 5, bface 3); A = adjoint scratch base
// (acc_h, acc_b) += (dL/dU)^T lam_k at U = (hydro, bface)
wm_status rhs_vjp_acc(wm_patch* p, double* A, const double* hydro, const double* bface, const double* lam_k,
                      double* acc_h, double* acc_b) {
  const size_t N = p->g.N;
  wm_status s;
  double* Bz = A + A_BZ * N;
  double* lT = A + A_LT * N;
  double* lBz = A + A_LBZ * N;
  if ((s = launch_bcell<double>(p, bface, Bz)) != WM_OK) return s;
  hipLaunchKernelGGL(adj_emf_kernel, zone_grid(p->g), dim3(256), 0, p->stream, p->g, 1.0 / p->cfg.h, lam_k, lT,
                     lBz);
  WM_LAUNCH_CHECK("adjoint emf kernel");
  if ((s = launch_adj_sweep<0>(p, hydro, Bz, lam_k, lT, acc_h, lBz)) != WM_OK) return s;
  if ((s = launch_adj_sweep<1>(p, hydro, Bz, lam_k, lT + 2 * N, acc_h, lBz)) != WM_OK) return s;
  if ((s = launch_adj_sweep<2>(p, hydro, Bz, lam_k, lT + 4 * N, acc_h, lBz)) != WM_OK) return s;
  // face b from the zone-B cotangent
  hipLaunchKernelGGL(adj_bcell_kernel, zone_grid(p->g), dim3(256), 0, p->stream, p->g, lBz, acc_b);
  WM_LAUNCH_CHECK("adjoint bcell kernel");
  return WM_OK;
}

// The intermediate stage states of one step from U^n (SSP-RK3: U1, U2; RK4:
// U1, U2, U3), each [11][N] (hydro, face b, zone B) in the storage type S of
// the patch's forward, with the given device dt.
template <typename S>
wm_status forward_stages(wm_patch* p, const S* Uh, const S* Ub, S* Bz, const double* dtp, S* U1, S* U2, S* U3,
                         S* acc) {
  const size_t N = p->g.N;
  const bool rk4 = p->cfg.integrator == WM_RK4;
  S* outs[3] = {U1, U2, U3};
  wm_status s;
  if ((s = launch_bcell<S>(p, Ub, Bz)) != WM_OK) return s;
  for (int st = 0; st < (rk4 ? 3 : 2); ++st) {
    const S* hin = st == 0 ? Uh : outs[st - 1];
    const S* bcin = st == 0 ? Bz : outs[st - 1] + 8 * N;
    if ((s = sweeps<S>(p, hin, bcin)) != WM_OK) return s;
    UpdateArgs<S> a;
    a.g = p->g;
    a.inv_h = 1.0 / p->cfg.h;
    a.faces = p->faces<S>();
    a.Un = Uh;
    a.bn = Ub;
    a.acc = acc;
    a.rhs_out = nullptr;
    a.dt = dtp;
    for (int d = 0; d < 3; ++d) a.wallF[d] = nullptr;   // the adjoint is for periodic boxes
    S* out = outs[st];
    a.hyd_out = out;
    a.b_out = out + 5 * N;
    launch_update_stage<S>(p, a, rk4, st);
    WM_LAUNCH_CHECK("update kernel");
    if ((s = launch_bcell<S>(p, out + 5 * N, out + 8 * N)) != WM_OK) return s;
  }
  return WM_OK;
}

wm_status widen(wm_patch* p, const void* x, size_t n, double* y) {
  hipLaunchKernelGGL(widen_kernel, lin_grid(n), dim3(256), 0, p->stream, n, reinterpret_cast<const float*>(x), y);
  WM_LAUNCH_CHECK("widen kernel");
  return WM_OK;
}

// U^n of an FP32-state patch widened into the adjoint scratch: (hydro, face b)
wm_status widen_state(wm_patch* p, double* A, const void* hydro, const void* bface, const double** Uh,
                      const double** Ub) {
  const size_t N = p->g.N;
  double* W = A + adjoint_base_arrays(&p->cfg) * N;
  wm_status s;
  if ((s = widen(p, hydro, 5 * N, W)) != WM_OK) return s;
  if ((s = widen(p, bface, 3 * N, W + 5 * N)) != WM_OK) return s;
  *Uh = W;
  *Ub = W + 5 * N;
  return WM_OK;
}

// Fields of a patch for a valid configuration, its stream and its scratch.
void setup_patch(wm_patch* p, const wm_config* cfg, void* hip_stream, void* scratch_buf, const Layout& L) {
  p->cfg = *cfg;
  p->stream = reinterpret_cast<hipStream_t>(hip_stream);
  p->g.nx = cfg->nx; p->g.ny = cfg->ny; p->g.nz = cfg->nz;
  p->g.N = (size_t)cfg->nx * cfg->ny * cfg->nz;
  for (int d = 0; d < 3; ++d) p->g.wall[d] = cfg->walls[d];
  p->g.wide = 0;
  p->floors = cfg->rho_floor > 0.0 || cfg->p_floor > 0.0;
  p->floor_reset = true;
  p->ph.gamma = cfg->gamma;
  p->ph.inv_h = 1.0 / cfg->h;
  p->ph.eps = cfg->eps_weno;
  p->ph.eps_B = cfg->eps_B;
  p->ph.eps_Z = cfg->eps_Z;
  p->ph.weno_z = cfg->weights == WM_WENO_Z ? 1 : (cfg->weights == WM_WENO_Z_PRINTED ? 2 : 0);
  p->ph.g1 = 0.5 * (cfg->gamma - 1.0);
  p->ph.g2 = (cfg->gamma - 2.0) / (cfg->gamma - 1.0);
  p->scratch = reinterpret_cast<char*>(scratch_buf);
  p->lay = L;
  p->f32 = cfg->precision == WM_MIXED_F32STATE;
}

// Opt-in floors on a stage result (hydro with its zone field) and the count.
template <typename S>
wm_status launch_floors(wm_patch* p, S* hydro, const S* bcell) {
  const int nb = red_blocks(p->g);
  hipLaunchKernelGGL(floor_kernel<S>, dim3(nb), dim3(RED_THREADS), 0, p->stream, p->g.N, p->cfg.gamma,
                     p->cfg.rho_floor, p->cfg.p_floor, hydro, bcell, p->floor_part());
  WM_LAUNCH_CHECK("floor kernel");
  hipLaunchKernelGGL(floor_final_kernel, dim3(1), dim3(1), 0, p->stream, nb, p->floor_part(), p->floor_total(),
                     p->floor_reset ? 1 : 0);
  WM_LAUNCH_CHECK("floor count kernel");
  p->floor_reset = false;
  return WM_OK;
}

// Device address of `scratch` on the current device, looked up once per device
// (with that device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};

wm_status static_scratch_address(void** out) {
  int dev = -1;
  wm_status s = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (s != WM_OK) return s;
  if (dev < 0 || dev >= kMaxDevices) return fail(WM_ERR_ARG, "device index beyond the static scratch table%s");
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* ptr = nullptr;
    if ((s = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)")) != WM_OK)
      return s;
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % kAlign) return fail(WM_ERR_HIP, "static scratch address invalid%s");
    g_static_ptr[dev] = ptr;
  }
  *out = g_static_ptr[dev];
  return WM_OK;
}

}  // namespace

extern "C" {

void wm_config_default(wm_config* c, int n) {
  if (!c) return;
  c->nx = c->ny = c->nz = n;
  c->h = n > 0 ? 1.0 / n : 0.0;
  c->gamma = 5.0 / 3.0;
  c->cfl = 0.4;
  c->eps_weno = 1e-6;
  c->eps_B = 1e-30;
  c->eps_Z = 1e-40;
  c->weights = WM_WENO_JS;
  c->precision = WM_FP64;
  c->integrator = WM_SSPRK3;
  c->walls[0] = c->walls[1] = c->walls[2] = 0;
  c->rho_floor = 0.0;
  c->p_floor = 0.0;
}

size_t wm_scratch_bytes(const wm_config* cfg) {
  const char* why = "";
  if (!valid_config(cfg, &why)) return 0;
  return layout(cfg).total;
}

wm_status wm_patch_create(const wm_config* cfg, void* hip_stream, void* scratch_buf, size_t scratch_bytes,
                          wm_patch** out) {
  const char* why = "";
  if (!out) return fail(WM_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (!valid_config(cfg, &why)) return fail(WM_ERR_ARG, "invalid config: %s", why);
  const Layout L = layout(cfg);
  if (!scratch_buf) return fail(WM_ERR_ARG, "null scratch");
  if (reinterpret_cast<uintptr_t>(scratch_buf) % kAlign) return fail(WM_ERR_ARG, "scratch not 256-byte aligned");
  if (scratch_bytes < L.total) return fail(WM_ERR_ARG, "scratch smaller than wm_scratch_bytes");
  wm_patch* p = new (std::nothrow) wm_patch;
  if (!p) return fail(WM_ERR_ARG, "host allocation failed");
  setup_patch(p, cfg, hip_stream, scratch_buf, L);
  if (cfg->nx >= 3 && cfg->ny >= 3 && cfg->nz >= 3) {
    const int n3[3] = {cfg->nx, cfg->ny, cfg->nz};
    const int ta[3] = {AdjTile<0>::TA, AdjTile<1>::TA, AdjTile<2>::TA};
    for (int d = 0; d < 3; ++d) {
      p->adj_plan[d] = plan_tiles(n3[d], ta[d]);
      if (!plan_disjoint(n3[d], ta[d], p->adj_plan[d])) {
        delete p;
        return fail(WM_ERR_ARG, "internal: adjoint tile classes overlap");
      }
    }
  }
  *out = p;
  g_err[0] = 0;
  return WM_OK;
}

wm_status wm_patch_destroy(wm_patch* p) {
  if (p) {
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  }
  delete p;
  return WM_OK;
}

wm_status wm_bind_state(wm_patch* p, void* hydro, void* bface, void* bcell) {
  if (!p) return fail(WM_ERR_ARG, "null patch");
  if (!hydro || !bface || !bcell) return fail(WM_ERR_ARG, "null state pointer");
  p->hydro = hydro;
  p->bface = bface;
  p->bcell = bcell;
  p->stage_done = -1;
  p->dt_valid = false;
  p->floor_reset = true;
  return WM_OK;
}

wm_status wm_init_from_potential(wm_patch* p, const double* rho, const double* v, const double* A_edge, double P0,
                                 const double B0[3]) {
  wm_status s = check_bound(p);
  if (s != WM_OK) return s;
  if (!rho || !v || !A_edge || !B0) return fail(WM_ERR_ARG, "null input pointer");
  s = with_storage(p, [&](auto tag) -> wm_status {
    using S = decltype(tag);
    hipLaunchKernelGGL(init_b_kernel<S>, zone_grid(p->g), dim3(256), 0, p->stream, p->g, 1.0 / p->cfg.h, A_edge,
                       B0[0], B0[1], B0[2], p->bf<S>());
    WM_LAUNCH_CHECK("init_b kernel");
    wm_status st = launch_bcell<S>(p, p->bf<S>(), p->bc<S>());
    if (st != WM_OK) return st;
    const size_t N = p->g.N;
    hipLaunchKernelGGL(init_hydro_kernel<S>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, p->stream, N,
                       p->cfg.gamma, P0, rho, v, p->bc<S>(), p->hyd<S>());
    WM_LAUNCH_CHECK("init_hydro kernel");
    return WM_OK;
  });
  if (s != WM_OK) return s;
  p->stage_done = -1;
  p->dt_valid = false;
  p->floor_reset = true;
  return WM_OK;
}

wm_status wm_refresh_zone_field(wm_patch* p) {
  wm_status s = check_bound(p);
  if (s != WM_OK) return s;
  p->floor_reset = true;
  return with_storage(p, [&](auto tag) {
    using S = decltype(tag);
    return launch_bcell<S>(p, p->bf<S>(), p->bc<S>());
  });
}

wm_status wm_compute_dt(wm_patch* p, double* dt_host) {
  wm_status s = check_bound(p);
  if (s != WM_OK) return s;
  const int nb = red_blocks(p->g);
  const long r = prof_begin(p, K_DT);
  if (p->f32)
    hipLaunchKernelGGL(speed_partial_kernel<float>, dim3(nb), dim3(RED_THREADS), 0, p->stream, p->g.N, p->cfg.gamma,
                       p->hyd<float>(), p->bc<float>(), p->speed_part());
  else
    hipLaunchKernelGGL(speed_partial_kernel<double>, dim3(nb), dim3(RED_THREADS), 0, p->stream, p->g.N, p->cfg.gamma,
                       p->hyd<double>(), p->bc<double>(), p->speed_part());
  WM_LAUNCH_CHECK("speed kernel");
  hipLaunchKernelGGL(dt_final_kernel, dim3(1), dim3(RED_THREADS), 0, p->stream, nb, p->cfg.cfl * p->cfg.h,
                     p->speed_part(), p->dt_dev(), p->smax_dev());
  WM_LAUNCH_CHECK("dt kernel");
  prof_end(p, r);
  p->dt_valid = true;
  if (dt_host) {
    if ((s = hip_check(hipMemcpyAsync(dt_host, p->dt_dev(), sizeof(double), hipMemcpyDeviceToHost, p->stream),
                       "dt copy")) != WM_OK)
      return s;
    if ((s = hip_check(hipStreamSynchronize(p->stream), "dt sync")) != WM_OK) return s;
  }
  return WM_OK;
}

namespace {

// The fused time step: the sweeps of a step's first stage write per-wave
// maxima of the eq. (cfl) signal speed (4 per block) into the accumulator
// region (free until that stage's update writes it), and speed_blocks_kernel +
// dt_final_kernel turn them into dt before the update.  Returns the number of
// wave values, or 0 when they do not fit there, in which case the step runs the
// stand-alone time-step pass first (very thin grids, e.g. 1 x 1 x n).
size_t fused_dt_blocks(const wm_patch* p) {
  const size_t nb =
      4 * (sweep_blocks(sweep_grid<0>(p)) + sweep_blocks(sweep_grid<1>(p)) + sweep_blocks(sweep_grid<2>(p)));
  const size_t acc_bytes = 8 * p->g.N * (p->f32 ? sizeof(float) : sizeof(double));
  // (at most 2^31 values: the kernels index them in 32 bits)
  return nb * sizeof(SpeedKey) <= acc_bytes && nb <= (size_t(1) << 31) ? nb : 0;
}

wm_status launch_fused_dt(wm_patch* p) {
  const unsigned n0 = (unsigned)(4 * sweep_blocks(sweep_grid<0>(p))),
                 n1 = (unsigned)(4 * sweep_blocks(sweep_grid<1>(p))),
                 n2 = (unsigned)(4 * sweep_blocks(sweep_grid<2>(p)));
  const unsigned nmax = std::max(n0, std::max(n1, n2));
  const int nb = (int)std::min<unsigned>((nmax + RED_THREADS - 1) / RED_THREADS, (unsigned)RED_BLOCKS);
  const long r = prof_begin(p, K_DT);
  hipLaunchKernelGGL(speed_blocks_kernel, dim3(nb), dim3(RED_THREADS), 0, p->stream,
                     reinterpret_cast<const SpeedKey*>(p->acc<char>()), n0, n1, n2, p->speed_part());
  WM_LAUNCH_CHECK("speed blocks kernel");
  hipLaunchKernelGGL(dt_final_kernel, dim3(1), dim3(RED_THREADS), 0, p->stream, nb, p->cfg.cfl * p->cfg.h,
                     p->speed_part(), p->dt_dev(), p->smax_dev());
  WM_LAUNCH_CHECK("dt kernel");
  prof_end(p, r);
  p->dt_valid = true;
  return WM_OK;
}

// One stage (after the caller's checks); fuse_dt (stage 0 only): dt from the
// stage's own sweeps
wm_status run_stage(wm_patch* p, int stage, bool fuse_dt) {
  const int ns = n_stages(p);
  const size_t N = p->g.N;
  wm_status s = with_storage(p, [&](auto tag) -> wm_status {
    using S = decltype(tag);
    const S* hyd_in = stage == 0 ? p->hyd<S>() : p->us<S>();
    const S* bcell_in = stage == 0 ? p->bc<S>() : p->us<S>() + 8 * N;
    wm_status st;
    SpeedKey* smax = fuse_dt ? reinterpret_cast<SpeedKey*>(p->acc<char>()) : nullptr;
    if ((st = sweeps<S>(p, hyd_in, bcell_in, smax)) != WM_OK) return st;
    if (fuse_dt && (st = launch_fused_dt(p)) != WM_OK) return st;
    if ((st = launch_update<S>(p, stage, nullptr)) != WM_OK) return st;
    S* hyd_out = stage == ns - 1 ? p->hyd<S>() : p->us<S>();
    S* b_out = stage == ns - 1 ? p->bf<S>() : p->us<S>() + 5 * N;
    S* bc_out = stage == ns - 1 ? p->bc<S>() : p->us<S>() + 8 * N;
    if ((st = launch_bcell<S>(p, b_out, bc_out)) != WM_OK) return st;
    return p->floors ? launch_floors<S>(p, hyd_out, bc_out) : WM_OK;
  });
  if (s != WM_OK) return s;
  if (stage == ns - 1) {
    p->stage_done = -1;
    p->dt_valid = false;
  } else {
    p->stage_done = stage;
  }
  return WM_OK;
}

}  // namespace

wm_status wm_rk_stage(wm_patch* p, int stage, const double* dt_host) {
  wm_status s = check_bound(p);
  if (s != WM_OK) return s;
  const int ns = n_stages(p);
  if (stage < 0 || stage >= ns) return fail(WM_ERR_ARG, "stage out of range for the integrator (SSP-RK3: 0..2, RK4: 0..3)");
  if (stage > 0 && p->stage_done != stage - 1) return fail(WM_ERR_STATE, "stages must run in order from 0");
  if (dt_host) {
    if (!std::isfinite(*dt_host)) return fail(WM_ERR_ARG, "dt is not finite");
    hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, p->stream, p->dt_dev(), *dt_host);
    WM_LAUNCH_CHECK("set dt");
    p->dt_valid = true;
  } else if (!p->dt_valid) {
    return fail(WM_ERR_STATE, "no dt: call wm_compute_dt or pass dt");
  }
  return run_stage(p, stage, false);
}

wm_status wm_step(wm_patch* p, double* dt_used) {
  wm_status s = check_bound(p);
  if (s != WM_OK) return s;
  p->stage_done = -1;
  const bool fuse = fused_dt_blocks(p) > 0;
  if (!fuse && (s = wm_compute_dt(p, nullptr)) != WM_OK) return s;
  for (int st = 0; st < n_stages(p); ++st)
    if ((s = run_stage(p, st, fuse && st == 0)) != WM_OK) return s;
  if (dt_used) {
    if ((s = hip_check(hipMemcpyAsync(dt_used, p->dt_dev(), sizeof(double), hipMemcpyDeviceToHost, p->stream),
                       "dt copy")) != WM_OK)
      return s;
    if ((s = hip_check(hipStreamSynchronize(p->stream), "step sync")) != WM_OK) return s;
  }
  return WM_OK;
}

wm_status wm_step_static(const wm_config* cfg, void* hip_stream, void* hydro, void* bface, void* bcell,
                         double* dt_used) {
  const char* why = "";
  if (!valid_config(cfg, &why)) return fail(WM_ERR_ARG, "invalid config: %s", why);
  if (!hydro || !bface || !bcell) return fail(WM_ERR_ARG, "null state pointer");
  const Layout L = layout(cfg);
  if (L.total > kStaticScratchBytes) {
    std::snprintf(g_err, sizeof(g_err),
                  "wm_step_static: this configuration needs %zu bytes of scratch, above the static maximum of %zu "
                  "bytes (64 MiB); use wm_patch_create with caller-owned scratch",
                  L.total, kStaticScratchBytes);
    return WM_ERR_ARG;
  }
  void* ptr = nullptr;
  wm_status s = static_scratch_address(&ptr);
  if (s != WM_OK) return s;
  wm_patch p;   // on the stack: profiling stays off, so its event lists stay empty
  setup_patch(&p, cfg, hip_stream, ptr, L);
  p.hydro = hydro;
  p.bface = bface;
  p.bcell = bcell;
  if ((s = wm_step(&p, dt_used)) != WM_OK) return s;
  g_err[0] = 0;
  return WM_OK;
}

wm_status wm_diagnostics(wm_patch* p, wm_diag* out) {
  wm_status s = check_bound(p);
  if (s != WM_OK) return s;
  if (!out) return fail(WM_ERR_ARG, "null output");
  const int nb = red_blocks(p->g);
  if (p->f32)
    hipLaunchKernelGGL(diag_partial_kernel<float>, dim3(nb), dim3(RED_THREADS), 0, p->stream, p->g, p->cfg.gamma,
                       1.0 / p->cfg.h, p->hyd<float>(), p->bf<float>(), p->bc<float>(), p->diag_part());
  else
    hipLaunchKernelGGL(diag_partial_kernel<double>, dim3(nb), dim3(RED_THREADS), 0, p->stream, p->g, p->cfg.gamma,
                       1.0 / p->cfg.h, p->hyd<double>(), p->bf<double>(), p->bc<double>(), p->diag_part());
  WM_LAUNCH_CHECK("diag kernel");
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, p->stream, nb, p->diag_part(), p->diag_out());
  WM_LAUNCH_CHECK("diag final kernel");
  double h[13];
  if ((s = hip_check(hipMemcpyAsync(h, p->diag_out(), sizeof(h), hipMemcpyDeviceToHost, p->stream), "diag copy")) !=
      WM_OK)
    return s;
  if ((s = hip_check(hipStreamSynchronize(p->stream), "diag sync")) != WM_OK) return s;
  out->mass = h[0];
  out->mom[0] = h[1]; out->mom[1] = h[2]; out->mom[2] = h[3];
  out->energy = h[4];
  out->bflux[0] = h[5]; out->bflux[1] = h[6]; out->bflux[2] = h[7];
  out->max_divb = h[8];
  out->min_rho = h[9];
  out->min_p = h[10];
  out->n_unphysical = (long long)h[11];
  out->n_floored = (p->floors && !p->floor_reset) ? (long long)h[12] : 0;
  if (out->n_unphysical > 0) return fail(WM_ERR_UNPHYSICAL, "unphysical zones in the state%s");
  return WM_OK;
}

wm_status wm_debug_wide_addressing(wm_patch* p, int on) {
  if (!p) return fail(WM_ERR_ARG, "null patch");
  p->g.wide = on != 0;
  return WM_OK;
}

wm_status wm_debug_sweep(wm_patch* p, int axis, void* out) {
  wm_status s = check_bound(p);
  if (s != WM_OK) return s;
  if (!out) return fail(WM_ERR_ARG, "null output");
  const size_t N = p->g.N;
  double* o = reinterpret_cast<double*>(out);
  if (axis < 0 || axis > 2) return fail(WM_ERR_ARG, "axis must be 0, 1 or 2");
  return with_storage(p, [&](auto tag) {
    using S = decltype(tag);
    S* f = p->faces<S>();
    switch (axis) {
      case 0: return launch_sweep<0, S>(p, p->hyd<S>(), p->bc<S>(), f, f + 15 * N, o);
      case 1: return launch_sweep<1, S>(p, p->hyd<S>(), p->bc<S>(), f + 5 * N, f + 17 * N, o);
      default: return launch_sweep<2, S>(p, p->hyd<S>(), p->bc<S>(), f + 10 * N, f + 19 * N, o);
    }
  });
}

wm_status wm_debug_rhs(wm_patch* p, void* out) {
  wm_status s = check_bound(p);
  if (s != WM_OK) return s;
  if (!out) return fail(WM_ERR_ARG, "null output");
  return with_storage(p, [&](auto tag) {
    using S = decltype(tag);
    wm_status st = sweeps<S>(p, p->hyd<S>(), p->bc<S>());
    if (st != WM_OK) return st;
    return launch_update<S>(p, 0, reinterpret_cast<double*>(out));
  });
}

size_t wm_adjoint_scratch_bytes(const wm_config* cfg) {
  const char* why = "";
  if (!valid_config(cfg, &why)) return 0;
  return adjoint_bytes(cfg);
}

wm_status wm_rhs_vjp(wm_patch* p, void* adj_scratch, const void* hydro, const void* bface, const void* lam_k,
                     void* lam_out) {
  wm_status s = check_adjoint(p, adj_scratch);
  if (s != WM_OK) return s;
  if (!hydro || !bface || !lam_k || !lam_out) return fail(WM_ERR_ARG, "null pointer");
  const size_t N = p->g.N;
  double* A = reinterpret_cast<double*>(adj_scratch);
  const double* Uh = reinterpret_cast<const double*>(hydro);
  const double* Ub = reinterpret_cast<const double*>(bface);
  if (p->f32 && (s = widen_state(p, A, hydro, bface, &Uh, &Ub)) != WM_OK) return s;
  double* out = reinterpret_cast<double*>(lam_out);
  hipLaunchKernelGGL(fill_kernel, lin_grid(8 * N), dim3(256), 0, p->stream, 8 * N, 0.0, out);
  WM_LAUNCH_CHECK("fill kernel");
  return rhs_vjp_acc(p, A, Uh, Ub, reinterpret_cast<const double*>(lam_k), out, out + 5 * N);
}

wm_status wm_adjoint_step(wm_patch* p, void* adj_scratch, const void* Un_hydro, const void* Un_bface,
                          const void* U1_stage, const void* U2_stage, double dt, void* lam_hydro, void* lam_bface) {
  wm_status s = check_adjoint(p, adj_scratch);
  if (s != WM_OK) return s;
  const bool rk4 = p->cfg.integrator == WM_RK4;
  if (!Un_hydro || !Un_bface || !lam_hydro || !lam_bface) return fail(WM_ERR_ARG, "null pointer");
  if ((U1_stage == nullptr) != (U2_stage == nullptr)) return fail(WM_ERR_ARG, "give both stage states or neither");
  if (rk4 && U1_stage) return fail(WM_ERR_ARG, "the RK4 step adjoint recomputes its stage states (pass NULL)");
  if (!std::isfinite(dt)) return fail(WM_ERR_ARG, "dt is not finite");
  const size_t N = p->g.N;
  double* A = reinterpret_cast<double*>(adj_scratch);
  const double* Uh = reinterpret_cast<const double*>(Un_hydro);
  const double* Ub = reinterpret_cast<const double*>(Un_bface);
  double* lh = reinterpret_cast<double*>(lam_hydro);
  double* lb = reinterpret_cast<double*>(lam_bface);
  const double* U1 = reinterpret_cast<const double*>(U1_stage);
  const double* U2 = reinterpret_cast<const double*>(U2_stage);
  const double* U3 = nullptr;
  if (!U1 && p->stage_done >= 0)
    return fail(WM_ERR_STATE, "a step is in progress (wm_rk_stage): recomputing the stage states would overwrite "
                              "its scratch%s");
  if (p->f32) {
    // FP32 state: U^n and the stage states are widened to FP64 and the FP64
    // method is linearised there; missing stage states come from the FP32-state
    // forward (the forward scratch's stage state and accumulator are free
    // outside a step)
    if ((s = widen_state(p, A, Un_hydro, Un_bface, &Uh, &Ub)) != WM_OK) return s;
    double* base = A + adjoint_base_arrays(&p->cfg) * N;
    if (U1) {
      if ((s = widen(p, U1_stage, 8 * N, A + A_U1 * N)) != WM_OK) return s;
      if ((s = widen(p, U2_stage, 8 * N, A + A_U2 * N)) != WM_OK) return s;
    } else {
      double* dtp = A + adjoint_arrays(&p->cfg) * N;
      hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, p->stream, dtp, dt);
      WM_LAUNCH_CHECK("set dt");
      float* F = reinterpret_cast<float*>(base + 8 * N);
      if ((s = forward_stages<float>(p, reinterpret_cast<const float*>(Un_hydro),
                                     reinterpret_cast<const float*>(Un_bface), p->us<float>() + 8 * N, dtp, F,
                                     F + 11 * N, rk4 ? F + 22 * N : nullptr, p->acc<float>())) != WM_OK)
        return s;
      if ((s = widen(p, F, 8 * N, A + A_U1 * N)) != WM_OK) return s;
      if ((s = widen(p, F + 11 * N, 8 * N, A + A_U2 * N)) != WM_OK) return s;
      if (rk4 && (s = widen(p, F + 22 * N, 8 * N, A + A_U3 * N)) != WM_OK) return s;
    }
    U1 = A + A_U1 * N;
    U2 = A + A_U2 * N;
    U3 = A + A_U3 * N;
  } else if (!U1) {   // recompute the stage states from U^n
    double* dtp = A + adjoint_arrays(&p->cfg) * N;
    hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, p->stream, dtp, dt);
    WM_LAUNCH_CHECK("set dt");
    // the stage accumulator of the forward scratch is free outside wm_step
    if ((s = forward_stages<double>(p, Uh, Ub, A + A_BZ * N, dtp, A + A_U1 * N, A + A_U2 * N,
                                    rk4 ? A + A_U3 * N : nullptr, p->acc<double>())) != WM_OK)
      return s;
    U1 = A + A_U1 * N;
    U2 = A + A_U2 * N;
    U3 = A + A_U3 * N;
  }
  double* lk = A + A_LK * N;
  double* lU2 = A + A_LU2 * N;
  double* lU1 = A + A_LU1 * N;
  const dim3 g8 = lin_grid(8 * N);
  if (rk4) {
    // U^{n+1} = U^n + dt/6 (k0 + 2 k1 + 2 k2 + k3), k_s = L(U_s), U1 = U^n + dt/2 k0,
    // U2 = U^n + dt/2 k1, U3 = U^n + dt k2; lam3 = the incoming cotangent, in (lh, lb)
    double* lU3 = A + A_LU3 * N;
    // k3 = L(U3): dt/6 lam3
    hipLaunchKernelGGL(adj_glue_a_kernel, g8, dim3(256), 0, p->stream, N, dt / 6.0, lh, lb, lk, lU3);
    WM_LAUNCH_CHECK("adjoint glue kernel");
    if ((s = rhs_vjp_acc(p, A, U3, U3 + 5 * N, lk, lU3, lU3 + 5 * N)) != WM_OK) return s;
    // k2 = L(U2): dt/3 lam3 + dt lamU3
    hipLaunchKernelGGL(adj_glue_b_kernel, g8, dim3(256), 0, p->stream, N, dt / 3.0, lh, lb, dt, lU3, lk, lU2);
    WM_LAUNCH_CHECK("adjoint glue kernel");
    if ((s = rhs_vjp_acc(p, A, U2, U2 + 5 * N, lk, lU2, lU2 + 5 * N)) != WM_OK) return s;
    // k1 = L(U1): dt/3 lam3 + dt/2 lamU2
    hipLaunchKernelGGL(adj_glue_b_kernel, g8, dim3(256), 0, p->stream, N, dt / 3.0, lh, lb, 0.5 * dt, lU2, lk, lU1);
    WM_LAUNCH_CHECK("adjoint glue kernel");
    if ((s = rhs_vjp_acc(p, A, U1, U1 + 5 * N, lk, lU1, lU1 + 5 * N)) != WM_OK) return s;
    // k0 = L(U^n): dt/6 lam3 + dt/2 lamU1; lam^n = lam3 + lamU1 + lamU2 + lamU3 + (dL/dU^n)^T lam_k0
    hipLaunchKernelGGL(adj_glue_d_kernel, g8, dim3(256), 0, p->stream, N, dt / 6.0, 0.5 * dt, lU1, lU2, lU3, lk, lh,
                       lb);
    WM_LAUNCH_CHECK("adjoint glue kernel");
    return rhs_vjp_acc(p, A, Uh, Ub, lk, lh, lb);
  }
  // SSP-RK3: k2 = L(U2), weight 4 dt/6
  hipLaunchKernelGGL(adj_glue_a_kernel, g8, dim3(256), 0, p->stream, N, 4.0 * dt / 6.0, lh, lb, lk, lU2);
  WM_LAUNCH_CHECK("adjoint glue kernel");
  if ((s = rhs_vjp_acc(p, A, U2, U2 + 5 * N, lk, lU2, lU2 + 5 * N)) != WM_OK) return s;
  // k1 = L(U1): dt/6 lam3 + dt/4 lamU2
  hipLaunchKernelGGL(adj_glue_b_kernel, g8, dim3(256), 0, p->stream, N, dt / 6.0, lh, lb, 0.25 * dt, lU2, lk, lU1);
  WM_LAUNCH_CHECK("adjoint glue kernel");
  if ((s = rhs_vjp_acc(p, A, U1, U1 + 5 * N, lk, lU1, lU1 + 5 * N)) != WM_OK) return s;
  // k0 = L(U^n): dt/6 lam3 + dt/4 lamU2 + dt lamU1; lam^n = lam3 + lamU2 + lamU1 + (dL/dU^n)^T lam_k0
  hipLaunchKernelGGL(adj_glue_c_kernel, g8, dim3(256), 0, p->stream, N, dt / 6.0, 0.25 * dt, lU2, dt, lU1, lk, lh, lb);
  WM_LAUNCH_CHECK("adjoint glue kernel");
  return rhs_vjp_acc(p, A, Uh, Ub, lk, lh, lb);
}

wm_status wm_step_record(wm_patch* p, double dt, void* U1_out, void* U2_out) {
  wm_status s = check_bound(p);
  if (s != WM_OK) return s;
  if (p->cfg.integrator != WM_SSPRK3) return fail(WM_ERR_ARG, "stage recording is for the SSP-RK3 step");
  if (!U1_out || !U2_out) return fail(WM_ERR_ARG, "null pointer");
  if (!std::isfinite(dt)) return fail(WM_ERR_ARG, "dt is not finite");
  const size_t bytes = 8 * p->g.N * state_elem_bytes(&p->cfg);
  p->stage_done = -1;
  if ((s = wm_rk_stage(p, 0, &dt)) != WM_OK) return s;
  if ((s = hip_check(hipMemcpyAsync(U1_out, p->us<char>(), bytes, hipMemcpyDeviceToDevice, p->stream), "stage copy")) !=
      WM_OK)
    return s;
  if ((s = wm_rk_stage(p, 1, nullptr)) != WM_OK) return s;
  if ((s = hip_check(hipMemcpyAsync(U2_out, p->us<char>(), bytes, hipMemcpyDeviceToDevice, p->stream), "stage copy")) !=
      WM_OK)
    return s;
  return wm_rk_stage(p, 2, nullptr);
}

wm_status wm_zone_field_vjp(wm_patch* p, const void* lam_bcell, void* lam_bface) {
  if (!p) return fail(WM_ERR_ARG, "null patch");
  if (!lam_bcell || !lam_bface) return fail(WM_ERR_ARG, "null pointer");
  hipLaunchKernelGGL(adj_bcell_kernel, zone_grid(p->g), dim3(256), 0, p->stream, p->g,
                     reinterpret_cast<const double*>(lam_bcell), reinterpret_cast<double*>(lam_bface));
  WM_LAUNCH_CHECK("adjoint bcell kernel");
  return WM_OK;
}

wm_status wm_init_adjoint(wm_patch* p, void* adj_scratch, const double* rho, const double* v, const double* A_edge,
                          const double B0[3], const void* lam_hydro, const void* lam_bface, double* g_A,
                          double* g_v) {
  wm_status s = check_adjoint(p, adj_scratch);
  if (s != WM_OK) return s;
  if (!rho || !v || !A_edge || !B0 || !lam_hydro || !lam_bface || !g_A || !g_v) return fail(WM_ERR_ARG, "null pointer");
  const size_t N = p->g.N;
  double* A = reinterpret_cast<double*>(adj_scratch);
  double* b0 = A + A_U1 * N;          // initial face field
  double* B0z = A + A_U1 * N + 3 * N; // its zone interpolation
  double* lB = A + A_WORK * N;        // zone-B cotangent
  double* lb = A + A_WORK * N + 3 * N;  // total face-b cotangent
  hipLaunchKernelGGL(init_b_kernel<double>, zone_grid(p->g), dim3(256), 0, p->stream, p->g, 1.0 / p->cfg.h, A_edge, B0[0],
                     B0[1], B0[2], b0);
  WM_LAUNCH_CHECK("init_b kernel");
  if ((s = launch_bcell<double>(p, b0, B0z)) != WM_OK) return s;
  hipLaunchKernelGGL(init_adj_zone_kernel, lin_grid(N), dim3(256), 0, p->stream, N, rho, v, B0z,
                     reinterpret_cast<const double*>(lam_hydro), g_v, lB);
  WM_LAUNCH_CHECK("init adjoint kernel");
  hipLaunchKernelGGL(scale_kernel, lin_grid(3 * N), dim3(256), 0, p->stream, 3 * N, 1.0,
                     reinterpret_cast<const double*>(lam_bface), lb);
  WM_LAUNCH_CHECK("copy kernel");
  hipLaunchKernelGGL(adj_bcell_kernel, zone_grid(p->g), dim3(256), 0, p->stream, p->g, lB, lb);
  WM_LAUNCH_CHECK("adjoint bcell kernel");
  hipLaunchKernelGGL(curl_adj_kernel, zone_grid(p->g), dim3(256), 0, p->stream, p->g, 1.0 / p->cfg.h, lb, g_A);
  WM_LAUNCH_CHECK("curl adjoint kernel");
  return WM_OK;
}

wm_status wm_profile(wm_patch* p, int enable) {
  if (!p) return fail(WM_ERR_ARG, "null patch");
  p->prof = enable != 0;
  if (enable) p->n_rec = 0;
  return WM_OK;
}

wm_status wm_profile_report(wm_patch* p, double* out, int n_out) {
  if (!p) return fail(WM_ERR_ARG, "null patch");
  if (!out || n_out < 2 * K_NCLASS) return fail(WM_ERR_ARG, "output needs 10 doubles");
  wm_status s = hip_check(hipStreamSynchronize(p->stream), "profile sync");
  if (s != WM_OK) return s;
  for (int c = 0; c < 2 * K_NCLASS; ++c) out[c] = 0.0;
  for (size_t r = 0; r < p->n_rec; ++r) {
    float ms = 0.f;
    if ((s = hip_check(hipEventElapsedTime(&ms, p->ev[2 * r], p->ev[2 * r + 1]), "event time")) != WM_OK) return s;
    out[2 * p->ev_class[r]] += 1.0;
    out[2 * p->ev_class[r] + 1] += ms;
  }
  return WM_OK;
}

const char* wm_last_error(void) { return g_err; }

}  // extern "C"

#ifdef WM_SWEEP_CLOCK
extern "C" wm_status wm_clock_sweep_buffer(int axis, void* stamps, size_t n_stamps) {
  if (axis < 0 || axis > 2) return fail(WM_ERR_ARG, "axis must be 0, 1 or 2");
  if (stamps == nullptr) n_stamps = 0;
  g_sweep_clk[axis] = static_cast<unsigned long long*>(stamps);
  g_sweep_clk_n[axis] = n_stamps;
  return WM_OK;
}
#endif
