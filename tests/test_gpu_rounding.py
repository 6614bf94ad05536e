"""Rounding floor of a long FP64 run: one period of the grid-aligned linear fast
wave (Sect. 4.1 setup, A0 = 1e-5) on 256 x 4 x 4 zones with dt = 0.25 h^(5/3),
20,643 SSP-RK3 steps.  The error of the k = 1 Fourier amplitude against the
exact travelling wave is then about the scheme's truncation error (~1.2e-14 by
extrapolating the fifth-order trend from N = 64, 128).  An arrangement of the
stages whose rounding is correlated with the solution -- e.g. reading the earlier
increments off the rounded stage states instead of keeping them in the
accumulator -- lifts it to ~2e-13; the bar is 4e-14."""
import sys

import numpy as np
import pytest
import torch

from paper_1812_04278_amd import binding as B, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()


def k1(U):
    comps = [U["rho"], U["m"][0], U["m"][1], U["m"][2], U["E"], U["b"][0], U["b"][1], U["b"][2]]
    return np.array([np.fft.rfft(np.asarray(x, dtype=np.float64).mean(axis=(0, 1)))[1] / x.shape[-1] for x in comps])


def test_long_run_rounding_floor():
    n, A0 = 256, 1e-5
    print(f"long run: fast wave N={n}, A0={A0}", flush=True)
    sys.stdout.flush()
    U0, U1 = inputs.fast_wave(n, A0=A0), inputs.fast_wave(n, t=0.5, A0=A0)
    p = B.Patch(B.config(nx=n, ny=4, nz=4, h=1.0 / n))
    p.set_state(U0["rho"], U0["m"], U0["E"], U0["b"])
    nt = int(np.ceil(0.5 / (0.25 * (1.0 / n) ** (5.0 / 3.0))))
    for _ in range(nt):
        p.step_dt(0.5 / nt)
    err = float(np.linalg.norm(k1(p.state()) - k1(U1)))
    print(f"  {nt} steps, k = 1 amplitude error {err:.3e}", flush=True)
    assert err <= 4e-14, err
