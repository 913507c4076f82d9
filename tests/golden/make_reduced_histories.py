"""Write the free-running history fixtures: FP64 oracle histories of the
reduced-resolution panels, for comparison with free-running GPU histories.

Every value stored here comes from the FP64 oracle (``oracle/``) on the
synthetic inputs of ``workloads/``; nothing is read from the HIP path.  The
panels are reduced versions of the benchmark configurations, with the same
ratio of regularisation length to element size as the full ones:

* ``tension128_<scheme>``: the notched tension panel at 128^2, l = 2.05 h
  (0.016 mm), 20 load steps of 2e-4 mm: the crack nucleates and runs within
  the history (the 512^2 configuration at a quarter of its resolution);
* ``shear128_<scheme>``: the notched shear panel with the spectral split at
  128^2, l = 0.016 mm, 20 load steps of 1e-3 mm (the 1024^2 configuration's
  panel at an eighth of its resolution);
* ``lshape256_<scheme>``: the masked L-shaped panel at 256^2, 10 load steps
  to 0.3 mm (the 2048^2 configuration at an eighth of its resolution).

Stored per step: staggered count, reaction, residual, converged flag and the
size of the last staggered iteration; u and d after the step with the most
staggered iterations, after the one following it, and after the last step.
The step cap is 300 staggered iterations.

Run from the repository root (CPU only, minutes to an hour per case):
``python tests/golden/make_reduced_histories.py [case ...]``.
"""
from __future__ import annotations

import dataclasses
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

OUT = os.path.join(HERE, "reduced")
SCHEMES = {"ST": 0, "S1": 1, "S2": 2, "S3": 3}
MAX_STAG = 300


def problem(kind):
    if kind == "tension128":
        p = W.tension_panel(n=128, l=0.016, du=2e-4, steps=20, name="tension128")
    elif kind == "shear128":
        p = W.shear_panel(n=128, l=0.016, du=1e-3, steps=20, name="shear128")
    elif kind == "lshape256":
        p = W.lshape_panel(n=256, steps=10, total=0.3, name="lshape256")
    else:
        raise SystemExit(f"unknown panel {kind}")
    return dataclasses.replace(p, max_stag=MAX_STAG)


def run(case):
    kind, name = case.split("_")
    p = problem(kind)
    orc = Oracle(p, SCHEMES[name])
    rows, states = [], {}
    t0 = time.perf_counter()
    for n in range(1, p.loads.size + 1):
        st = orc.load_step(float(p.loads[n - 1]))
        rows.append((st.n_stag, st.force, st.r_stag, int(st.converged), st.last_du, st.last_dd))
        u, d, _ = orc.get_state()
        states[n] = (u, d)
        # keep only what the stored steps need (the largest count so far,
        # the step after it, and the latest)
        counts = [r[0] for r in rows]
        peak = int(np.argmax(counts)) + 1
        keep = {peak, peak + 1, n}
        states = {k: v for k, v in states.items() if k in keep}
        print(f"{case} step {n}: n_stag={st.n_stag} F={st.force:.6f} converged={st.converged} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
    rows = np.array(rows, dtype=np.float64)
    arrays = {"n_stag": rows[:, 0].astype(np.int64), "force": rows[:, 1], "r_stag": rows[:, 2],
              "converged": rows[:, 3].astype(np.int64), "last_du": rows[:, 4],
              "last_dd": rows[:, 5], "scheme": np.int64(SCHEMES[name]),
              "max_stag": np.int64(MAX_STAG), "stored_steps": np.array(sorted(states))}
    for k, (u, d) in states.items():
        arrays[f"u_{k}"] = u
        arrays[f"d_{k}"] = d
    np.savez_compressed(os.path.join(OUT, f"{case}.npz"), **arrays)


def main(argv):
    os.makedirs(OUT, exist_ok=True)
    cases = argv or ["tension128_ST", "tension128_S1", "tension128_S3", "shear128_ST",
                     "shear128_S1", "shear128_S2", "shear128_S3", "lshape256_ST",
                     "lshape256_S1", "lshape256_S2"]
    for c in cases:
        run(c)


if __name__ == "__main__":
    main(sys.argv[1:])
