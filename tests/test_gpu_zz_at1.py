"""GPU parity of AT1 with penalised irreversibility (phase_model 1) against
the bar's scalar equation and the oracle.

* Homogeneous bar (9 x 70 elements) on a loading and on an unloading-
  reloading path: d to the staggered tolerance of the closed form (both
  stop at ||F_d|| <= tol_stag ||sum 2 Psi+ N||), the reaction force to 1e-4,
  two u-solves per step for ST.
* Notched 16^2 panel, 8 load steps through nucleation: the histories of the
  other parity tests (counts within +-1, u to 1e-7 / 1e-6, d to 1e-5, force
  curve to 1e-4 of its peak), FP64 for ST, S1 and S3, mixed for S1, and S1
  on LDS tiles.
* The 64^2 tension panel at l = 2h (the length-scale ratio of the 512^2
  configuration), load steps 1-2: the regime in which a later staggered
  iteration's phase solve starts from a converged d and can only stop at
  the rounding floor of F_d (tests/test_at1_stop_rule.py emulates it on the
  CPU); ST and S1 against the oracle under the same protocol.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from test_gpu_parity import compare_history
from test_oracle_at1 import LOADING, UNLOADING, bar_at1_history

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
@pytest.mark.parametrize("loads", [LOADING, UNLOADING], ids=["loading", "unloading"])
def test_at1_bar_closed_form(gpu_lib, scheme, precision, loads):
    p = dataclasses.replace(W.homogeneous_bar(nx=9, ny=70, lx=1.0, ly=1.0, steps=len(loads)),
                            loads=np.asarray(loads, float), phase_model=1)
    ref = bar_at1_history(p)
    ctx = gpu_lib.Context(p, scheme=scheme, precision=precision)
    for lam, (d_ref, F_ref) in zip(p.loads, ref):
        st = ctx.load_step(float(lam))
        print(f"lam={lam:.3e} n_stag={st['n_stag']} d_ref={d_ref:.6e} F={st['force'][1]:.6f} "
              f"F_ref={F_ref:.6f}", flush=True)
        assert st["converged"] == 1
        _, d, _ = ctx.get_state()
        np.testing.assert_allclose(d, d_ref, rtol=0, atol=1e-9 + 2 * p.tol_stag)
        assert np.isclose(st["force"][1], F_ref, rtol=1e-4)
        if scheme == 0:
            assert st["n_stag"] == 2
    ctx.close()


PANEL = [(0, 0, 0), (1, 0, 0), (3, 0, 0), (1, 1, 0), (1, 0, 1)]


@pytest.mark.parametrize("scheme,precision,rows", PANEL)
def test_at1_panel_history(gpu_lib, scheme, precision, rows):
    p = dataclasses.replace(W.tension_panel(n=16, l=0.1, du=1e-3, steps=8), phase_model=1)
    compare_history(gpu_lib, p, scheme, precision, 8, 1e-7 if precision == 0 else 1e-6,
                    march_rows=rows)


@pytest.mark.parametrize("scheme,precision", [(0, 0), (1, 0), (1, 1)])
def test_at1_l2h_panel_first_steps(gpu_lib, scheme, precision):
    n = 64
    p = dataclasses.replace(W.tension_panel(n=n, l=2.0 / n, du=6e-5, steps=2),
                            phase_model=1)
    compare_history(gpu_lib, p, scheme, precision, 2, 1e-7 if precision == 0 else 1e-6)
