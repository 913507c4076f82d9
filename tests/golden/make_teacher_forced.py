"""Write the teacher-forcing fixtures: committed oracle states before and
after the load steps where a crack nucleates and runs.

Every value stored here comes from the FP64 oracle (``oracle/``) on the
synthetic inputs of ``workloads/``; nothing is read from the HIP path.  The
steps were chosen from the oracle's own history of each panel:

* ``tension64_<scheme>.npz`` - the 64^2 notched tension panel (20 steps of
  3e-4 mm, l = 0.03 mm), schemes ST, S1 and S3, FP64 oracle, load steps
  1-20 (the whole load history of the panel).  Step 10 is the last step
  before the crack runs, step 11 is the nucleation step (the largest
  staggered count of the first crack, where the fixed-stress schemes gain
  most: Section 4.1), step 19 is the step in which the ligament breaks.
  Stored: the per-step record of every step (staggered
  count, reaction, residual, converged flag, size of the last staggered
  iteration) and the committed u and d after steps 9, 10, 11, 18, 19 and
  20, with H after steps 9, 10 and 18 (the inputs of the forced steps 10,
  11 and 19).
* ``shear32_<scheme>.npz`` - a 32^2 shear panel with the spectral split
  (l = 0.06 mm, 3e-3 mm per step), schemes ST and S1: the committed state
  before and after the first step past the peak of the reaction curve
  (post-peak), with the per-step records up to it.

Run from the repository root (CPU only, about ten minutes per tension
scheme): ``python tests/golden/make_teacher_forced.py [case ...]`` with
case in tension64_ST, tension64_S1, tension64_S3, shear32_ST, shear32_S1.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import Oracle  # noqa: E402

OUT = os.path.join(HERE, "teacher_forced")
SCHEMES = {"ST": 0, "S1": 1, "S2": 2, "S3": 3}

TENSION_STEPS = 20
TENSION_KEEP = (9, 10, 11, 18, 19, 20)  # committed u, d after these steps
TENSION_KEEP_H = (9, 10, 18)           # H after these (inputs of 10, 11, 19)
SHEAR_MAX_STEPS = 14


def tension64_problem():
    return W.config_tension64()


def shear32_problem():
    return W.shear_panel(n=32, l=0.06, du=3e-3, steps=SHEAR_MAX_STEPS, name="shear32")


def _record(st):
    return (st.n_stag, st.force, st.r_stag, int(st.converged), st.last_du, st.last_dd)


def _save(path, rows, states, Hs, extra):
    rows = np.array(rows, dtype=np.float64)
    arrays = {"n_stag": rows[:, 0].astype(np.int64), "force": rows[:, 1], "r_stag": rows[:, 2],
              "converged": rows[:, 3].astype(np.int64), "last_du": rows[:, 4],
              "last_dd": rows[:, 5]}
    for n, (u, d) in states.items():
        arrays[f"u_{n}"] = u
        arrays[f"d_{n}"] = d
    for n, H in Hs.items():
        arrays[f"H_{n}"] = H
    arrays.update(extra)
    np.savez_compressed(path, **arrays)


def make_tension(name):
    scheme = SCHEMES[name]
    p = tension64_problem()
    orc = Oracle(p, scheme)
    rows, states, Hs = [], {}, {}
    t0 = time.perf_counter()
    for n in range(1, TENSION_STEPS + 1):
        st = orc.load_step(float(p.loads[n - 1]))
        rows.append(_record(st))
        u, d, H = orc.get_state()
        if n in TENSION_KEEP:
            states[n] = (u, d)
        if n in TENSION_KEEP_H:
            Hs[n] = H
        print(f"tension64 {name} step {n}: n_stag={st.n_stag} F={st.force:.6f} "
              f"converged={st.converged} last_dd={st.last_dd:.2e} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
    _save(os.path.join(OUT, f"tension64_{name}.npz"), rows, states, Hs,
          {"scheme": np.int64(scheme), "steps": np.int64(TENSION_STEPS)})


def make_shear(name):
    scheme = SCHEMES[name]
    p = shear32_problem()
    orc = Oracle(p, scheme)
    rows = []
    peak = -np.inf
    t0 = time.perf_counter()
    for n in range(1, min(SHEAR_MAX_STEPS, p.loads.size) + 1):
        before = orc.get_state()
        st = orc.load_step(float(p.loads[n - 1]))
        rows.append(_record(st))
        print(f"shear32 {name} step {n}: n_stag={st.n_stag} F={st.force:.6f} "
              f"converged={st.converged} ({time.perf_counter() - t0:.0f} s)", flush=True)
        if st.force < peak:
            u, d, _ = orc.get_state()
            _save(os.path.join(OUT, f"shear32_{name}.npz"), rows,
                  {n - 1: before[:2], n: (u, d)}, {n - 1: before[2]},
                  {"scheme": np.int64(scheme), "step": np.int64(n)})
            return
        peak = max(peak, st.force)
    raise RuntimeError(f"shear32 {name}: no post-peak step within {SHEAR_MAX_STEPS} steps")


def main(argv):
    os.makedirs(OUT, exist_ok=True)
    cases = argv or ["tension64_ST", "tension64_S1", "tension64_S3", "shear32_ST", "shear32_S1"]
    for c in cases:
        kind, name = c.split("_")
        if kind == "tension64":
            make_tension(name)
        elif kind == "shear32":
            make_shear(name)
        else:
            raise SystemExit(f"unknown case {c}")


if __name__ == "__main__":
    main(sys.argv[1:])
