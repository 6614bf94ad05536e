"""Per-phase clock split of the directional sweep (measurement build).

Loads libwenomhd_clock.so (``python -m paper_1812_04278_amd.build --clock``),
runs one SSP-RK3 stage of the Mach-2 box (three sweeps) with every wave's
phase stamps recorded (include/wenomhd_clock.h), and prints per axis the mean
shader-clock cycles a wave spends in each phase, their share of the wave's
life, and the mean number of resident waves per compute unit.

Usage (GPU): ``python -m paper_1812_04278_amd.sweep_clock [--n 256] [--precision 0]``
"""
from __future__ import annotations

import argparse
import ctypes
import json

import numpy as np
import torch

from . import binding as B
from . import build as _build
from . import inputs

PHASES = ["zone loads + prologue", "barrier 1", "phase 2 (central flux, face state, differences)",
          "barriers 2-3 + difference stores", "phase 3 (eigensystem + WENO)", "flux stores"]
TILES = {0: (128, 2), 1: (32, 8), 2: (32, 8)}         # FP64 work type
TILES_F32 = {0: (128, 2), 1: (16, 16), 2: (16, 16)}   # mixed and FP32 state
WAVES_PER_BLOCK = 4


def analyse(st: np.ndarray) -> dict:
    """st: [waves, 8] stamps of one sweep launch."""
    d = np.diff(st[:, :7], axis=1).astype(np.float64)
    life = (st[:, 6] - st[:, 0]).astype(np.float64)
    cu = st[:, 7] & 0xFFFFFFFF
    resident = []
    for c in np.unique(cu):
        m = cu == c
        span = float(st[m, 6].max() - st[m, 0].min())
        if span > 0:
            resident.append(life[m].sum() / span)
    return {
        "waves": int(len(st)),
        "mean_life_cycles": float(life.mean()),
        "mean_cycles": {p: float(d[:, i].mean()) for i, p in enumerate(PHASES)},
        "share": {p: float(d[:, i].sum() / life.sum()) for i, p in enumerate(PHASES)},
        "resident_waves_per_cu": float(np.mean(resident)),
        "compute_units": int(len(resident)),
    }


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--precision", type=int, default=B.WM_FP64)
    ap.add_argument("--seed", type=int, default=1)
    args = ap.parse_args()
    n = args.n
    lib = B.load(_build.CLOCK_LIB)
    lib.wm_clock_sweep_buffer.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t]
    lib.wm_clock_sweep_buffer.restype = ctypes.c_int
    f = inputs.random_fields(n, seed=args.seed, v_rms=2.0, device="cuda")
    p = B.Patch(B.config(n, precision=args.precision))
    p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
    for _ in range(2):
        p.step()
    torch.cuda.synchronize()
    bufs = []
    tiles = TILES if args.precision == B.WM_FP64 else TILES_F32
    for ax in range(3):
        TA, TB = tiles[ax]
        nblk = -(-n // TA) * -(-n // TB) * n
        b = torch.zeros(nblk * WAVES_PER_BLOCK * 8, dtype=torch.int64, device="cuda")
        if lib.wm_clock_sweep_buffer(ax, ctypes.c_void_p(b.data_ptr()), b.numel()) != 0:
            raise RuntimeError("wm_clock_sweep_buffer failed")
        bufs.append(b)
    dt = p.compute_dt()
    p.rk_stage(0, dt)
    torch.cuda.synchronize()
    for ax in range(3):
        lib.wm_clock_sweep_buffer(ax, None, 0)
    out = {"n": n, "precision": args.precision}
    print(f"| axis | waves | life (cycles) | " + " | ".join(PHASES) + " | resident waves / CU |")
    print("|---|---|---|" + "---|" * len(PHASES) + "---|")
    for ax in range(3):
        st = bufs[ax].view(-1, 8).cpu().numpy().view(np.uint64).astype(np.int64)
        if not (st[:, 6] >= st[:, 0]).all() or (st[:, 0] == 0).any():
            raise RuntimeError(f"axis {ax}: missing or unordered stamps")
        r = analyse(st)
        out[f"axis{ax}"] = r
        cells = [f"{r['mean_cycles'][q]:.0f} ({100 * r['share'][q]:.0f}%)" for q in PHASES]
        print(f"| {'xyz'[ax]} | {r['waves']} | {r['mean_life_cycles']:.0f} | " + " | ".join(cells) +
              f" | {r['resident_waves_per_cu']:.2f} |", flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
