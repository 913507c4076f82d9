"""Teacher-forced parity through crack nucleation and growth (GPU).

The committed fixtures under tests/golden/teacher_forced/ hold FP64 oracle
states, written by tests/golden/make_teacher_forced.py from oracle/ and
workloads/ only.  Each test injects the oracle's committed state before one
load step into a fresh context (pf_set_state), runs that one step on the GPU
and compares it with the oracle's result of the same step, under the parity
protocol (tests/_parity.py):

* 64^2 notched tension panel (l = 0.03 mm, 3e-4 mm per step), ST, S1 and
  S3: step 10 (the last step before the crack runs), step 11 (nucleation:
  the largest staggered count of the first crack, where the fixed-stress
  schemes differ most from ST, Section 4.1) and step 19 (the ligament
  breaks); FP64 and mixed precision;
* 32^2 spectral shear panel, ST and S1: the first step past the peak of the
  reaction curve.

The reaction force of the step is compared with the oracle's at 1e-4 of the
largest force of the fixture's curve.
"""
import os

import numpy as np
import pytest

import workloads as W
from _parity import check_step

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FIX = os.path.join(HERE, "golden", "teacher_forced")
SCHEME = {"ST": 0, "S1": 1, "S2": 2, "S3": 3}


def _load(name):
    return np.load(os.path.join(FIX, name + ".npz"), allow_pickle=False)


def forced_step(pf, p, scheme, precision, z, step, **opts):
    """Inject the state after step-1, run step, compare with the fixture."""
    k = step - 1                                  # index of the step's record
    ctx = pf.Context(p, scheme=scheme, precision=precision, **opts)
    ctx.set_state(z[f"u_{step - 1}"], z[f"d_{step - 1}"], z[f"H_{step - 1}"])
    sg = ctx.load_step(float(p.loads[k]))
    u, d, _ = ctx.get_state()
    ctx.close()
    tol = 1e-7 if precision == 0 else 1e-6
    check_step(f"step {step} (prec {precision})", int(z["n_stag"][k]), float(z["last_du"][k]),
               float(z["last_dd"][k]), z[f"u_{step}"], z[f"d_{step}"], sg["n_stag"], u, d, tol)
    F_scale = np.abs(z["force"]).max()
    eF = abs(sg["force"][p.load_comp] - z["force"][k]) / F_scale
    print(f"  force gpu={sg['force'][p.load_comp]:.6f} oracle={z['force'][k]:.6f} "
          f"err={eF:.1e}; converged gpu={sg['converged']} oracle={int(z['converged'][k])}",
          flush=True)
    assert eF <= 1e-4, eF
    assert sg["converged"] == int(z["converged"][k])
    return sg


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("step", [10, 11, 19])
@pytest.mark.parametrize("scheme", ["ST", "S1", "S3"])
def test_tension64_forced_step(gpu_lib, scheme, step, precision):
    z = _load(f"tension64_{scheme}")
    assert int(z["scheme"]) == SCHEME[scheme]
    forced_step(gpu_lib, W.config_tension64(), SCHEME[scheme], precision, z, step)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheme", ["ST", "S1"])
def test_shear32_spectral_post_peak_step(gpu_lib, scheme, precision):
    z = _load(f"shear32_{scheme}")
    step = int(z["step"])
    p = W.shear_panel(n=32, l=0.06, du=3e-3, steps=14, name="shear32")
    assert z["force"][step - 1] < z["force"][:step - 1].max()     # past the peak
    forced_step(gpu_lib, p, SCHEME[scheme], precision, z, step)


def test_tension64_forced_nucleation_lds_tiles_chebyshev(gpu_lib):
    """The nucleation step of S1 in the benchmark's launch configuration
    (mixed, LDS tiles, Jacobi-Chebyshev of degree 3)."""
    z = _load("tension64_S1")
    forced_step(gpu_lib, W.config_tension64(), 1, 1, z, 11, precond=1, cheb_degree=3,
                march_rows=1)
