"""Free-running load histories against stored FP64 oracle histories (GPU).

The fixtures hold whole oracle histories, written by the scripts beside them
from oracle/ and workloads/ only (tests/golden/make_teacher_forced.py and
tests/golden/make_reduced_histories.py).  Each test runs the same history on
the GPU from the zero state, with no state injected, and compares:

* every step's staggered count with the oracle's, within +-1 (or both at the
  step cap: a step that stops at max_stag has no converged state to match);
* every step's converged flag and reaction force, the force within 1e-4 of
  the largest force of the oracle's curve;
* u and d after the stored steps (the step with the most staggered
  iterations, the one after it, the last step) under the one-step parity
  protocol of tests/_parity.py, except after a step that both sides ended
  at the cap.

The panels: the 64^2 notched tension panel over its 20 steps (ST, S1, S3;
the crack nucleates at step 11 and breaks the ligament by step 19), and
reduced versions of the three larger configurations with their l/h ratio:
the 128^2 tension panel (ST, S1, S3), the 128^2 spectral shear panel (ST,
S1, S2, S3) and the 256^2 masked L-shaped panel (ST, S1, S2).
"""
import dataclasses
import os

import numpy as np
import pytest

import workloads as W
from _parity import check_step

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")
SCHEME = {"ST": 0, "S1": 1, "S2": 2, "S3": 3}


def _load(sub, name):
    return np.load(os.path.join(GOLD, sub, name + ".npz"), allow_pickle=False)


def reduced_problem(kind, max_stag):
    # the same panels as tests/golden/make_reduced_histories.py
    if kind == "tension128":
        p = W.tension_panel(n=128, l=0.016, du=2e-4, steps=20, name="tension128")
    elif kind == "shear128":
        p = W.shear_panel(n=128, l=0.016, du=1e-3, steps=20, name="shear128")
    else:
        p = W.lshape_panel(n=256, steps=10, total=0.3, name="lshape256")
    return dataclasses.replace(p, max_stag=max_stag)


def free_run(pf, p, scheme, precision, z, stored, **opts):
    """Run the whole history on the GPU and compare it step by step."""
    n_steps = z["n_stag"].size
    assert p.loads.size >= n_steps
    tol = 1e-7 if precision == 0 else 1e-6
    F_scale = np.abs(z["force"]).max()
    ctx = pf.Context(p, scheme=scheme, precision=precision, **opts)
    worst_F = 0.0
    stats = []
    try:
        for n in range(1, n_steps + 1):
            k = n - 1
            sg = ctx.load_step(float(p.loads[k]))
            stats.append(sg)
            n_o, n_g = int(z["n_stag"][k]), int(sg["n_stag"])
            F_g = float(sg["force"][p.load_comp])
            eF = abs(F_g - float(z["force"][k])) / F_scale
            worst_F = max(worst_F, eF)
            print(f"  step {n}: stag oracle={n_o} gpu={n_g} converged oracle="
                  f"{int(z['converged'][k])} gpu={sg['converged']} force err={eF:.1e}",
                  flush=True)
            capped = n_o == p.max_stag and n_g == p.max_stag
            assert capped or abs(n_o - n_g) <= 1, (n, n_o, n_g)
            assert sg["converged"] == int(z["converged"][k]), n
            assert eF <= 1e-4, (n, eF)
            if n in stored and capped:
                print(f"  state after step {n} not compared: both sides stopped at the cap",
                      flush=True)
            elif n in stored:
                u, d, _ = ctx.get_state()
                check_step(f"state after step {n}", n_o, float(z["last_du"][k]),
                           float(z["last_dd"][k]), z[f"u_{n}"], z[f"d_{n}"], n_g, u, d, tol)
    finally:
        ctx.close()
    print(f"  largest force error over the history {worst_F:.1e}", flush=True)
    return stats


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheme", ["ST", "S1", "S3"])
def test_tension64_whole_history(gpu_lib, scheme, precision):
    z = _load("teacher_forced", f"tension64_{scheme}")
    assert int(z["steps"]) == 20
    stored = sorted(int(k[2:]) for k in z.files if k.startswith("u_"))
    free_run(gpu_lib, W.config_tension64(), SCHEME[scheme], precision, z, stored)


def test_tension64_whole_history_benchmark_launch(gpu_lib):
    """S1 mixed in the benchmark's launch configuration (LDS tiles, Jacobi-
    Chebyshev of degree 3)."""
    z = _load("teacher_forced", "tension64_S1")
    stored = sorted(int(k[2:]) for k in z.files if k.startswith("u_"))
    free_run(gpu_lib, W.config_tension64(), 1, 1, z, stored, precond=1, cheb_degree=3,
             march_rows=1)


# each configuration's schemes (the tension panel: ST and S1/S3; the spectral
# shear panel: S1/S2/S3 against ST; the L-shape: S1 and S2 against ST), in
# FP64 and mixed precision
REDUCED = [("tension128", "ST", 0), ("tension128", "S1", 0), ("tension128", "S1", 1),
           ("tension128", "S3", 1),
           ("shear128", "ST", 0), ("shear128", "S1", 0), ("shear128", "S1", 1),
           ("shear128", "S2", 0), ("shear128", "S2", 1), ("shear128", "S3", 1),
           ("lshape256", "ST", 0), ("lshape256", "S1", 0), ("lshape256", "S1", 1),
           ("lshape256", "S2", 0), ("lshape256", "S2", 1)]


@pytest.mark.parametrize("kind,scheme,precision", REDUCED)
def test_reduced_configuration_history(gpu_lib, kind, scheme, precision):
    z = _load("reduced", f"{kind}_{scheme}")
    assert int(z["scheme"]) == SCHEME[scheme]
    p = reduced_problem(kind, int(z["max_stag"]))
    free_run(gpu_lib, p, SCHEME[scheme], precision, z, [int(s) for s in z["stored_steps"]])


@pytest.mark.parametrize("scheme,precision,opts", [
    ("S1", 1, {"precond": 1, "cheb_degree": 3, "march_rows": 1}),
    ("ST", 0, {"precond": 1, "cheb_degree": 5, "march_rows": 2}),
    ("S3", 1, {})])
def test_tension64_whole_history_with_starting_guesses(gpu_lib, scheme, precision, opts):
    """Displacement solves started from the projection onto the last four
    solutions (guess_vectors = 4) give the same history as the oracle, under
    the same protocol, with fewer displacement CG iterations than the same
    run from zero."""
    z = _load("teacher_forced", f"tension64_{scheme}")
    stored = sorted(int(k[2:]) for k in z.files if k.startswith("u_"))
    p = W.config_tension64()
    with_guess = free_run(gpu_lib, p, SCHEME[scheme], precision, z, stored, guess_vectors=4,
                          **opts)
    ctx = gpu_lib.Context(p, scheme=SCHEME[scheme], precision=precision, **opts)
    plain = [ctx.load_step(float(lam)) for lam in p.loads[:len(with_guess)]]
    ctx.close()
    cg_guess = sum(st["n_cg_u"] for st in with_guess)
    cg_plain = sum(st["n_cg_u"] for st in plain)
    print(f"  displacement CG iterations: {cg_guess} with starting guesses, {cg_plain} from zero",
          flush=True)
    assert cg_guess < cg_plain
