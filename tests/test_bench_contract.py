"""The benchmark's host-side contract (no device): the one-GPU refusal, the
counter-traffic lookup's guards, and the algorithmic byte counts the
roofline divides by (each a count of the arrays the kernel must move)."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    line = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_traffic_lookup_guards():
    b = bench()
    import hashlib
    rec = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic_tension512.json")))
    src_path = os.path.join(ROOT, "paper_2209_07969_amd", "csrc", "pf_kernels.hip")
    sha = hashlib.sha256(open(src_path, "rb").read()).hexdigest()
    traffic, src = b.measured_traffic(rec["kernel"])
    if rec["kernel_source_sha256"] == sha:
        # counters taken on this very source: reported, with their origin
        assert traffic == rec["traffic_bytes_per_launch"]
        assert "hbm_traffic_tension512.json" in src and sha[:16] in src
    else:
        # the kernels changed since the counters were taken: nothing reported
        assert (traffic, src) == (None, None)
    # another kernel's name never borrows it
    assert b.measured_traffic("k_cg_updcheb<1, OpUpdCheb<OpTangent<float>>>") == (None, None)


def test_algorithmic_bytes_per_node():
    b = bench()
    f32, flag = 4, 1
    # apply: z, p_old, p_new, q (2 comps), d; node and element flags
    assert b.fused_apply_bytes_per_node() == (4 * 2 + 1) * f32 + 2 * flag
    # Chebyshev step: d_{k-1}, z, res, D^-1 in; d_k, z, res out (2 comps); d; flags
    assert b.cheb_step_bytes_per_node() == (7 * 2 + 1) * f32 + 2 * flag
    # update + first step: r, q, D^-1, x, p in; x, r, d_1, z, res out; d; flags
    assert b.updcheb_bytes_per_node() == (10 * 2 + 1) * f32 + 2 * flag
    # update + two steps: r, q, D^-1, x, p in; x, r, z out (d_2, res_2 when more follow)
    assert b.updcheb2_bytes_per_node(True) == (8 * 2 + 1) * f32 + 2 * flag
    assert b.updcheb2_bytes_per_node(False) == (10 * 2 + 1) * f32 + 2 * flag
    # vector update: x, p, q, r, D^-1 in; x, r, z out, per DOF
    assert b.update_bytes_per_node() == 2 * 8 * f32


def test_step_record_is_one_json_line():
    b = bench()
    st = {"n_stag": 5, "n_newton": 7, "n_trial": 2, "n_dsolve": 4, "n_cg_u": 900, "n_cg_d": 80,
          "n_cg_trial": 40, "gated_max": 12, "floor_hits": 3, "r_stag": 8e-6,
          "force": [0.0, 123.5], "time_ms": 42.0, "time_u_ms": 30.0, "time_d_ms": 9.0,
          "dof_updates": 1.5e6, "converged": 1,
          "cg_not_converged": 0, "extra": "ignored"}
    line = b.step_record("s1_mixed", 3, True, st)
    assert "\n" not in line
    rec = json.loads(line)
    assert rec["run"] == "s1_mixed" and rec["step"] == 3 and rec["timed"] is True
    assert rec["force"] == [0.0, 123.5] and rec["n_cg_trial"] == 40
    assert set(rec) == {"run", "step", "timed", *b.STEP_FIELDS}


def test_sweep_part_is_validated_before_any_device_work():
    """--sweep-part K/M must name a residue class of the 64 instances; a bad
    one ends the run before a context is created (pf is never touched)."""
    import types

    import pytest
    b = bench()
    for bad in ("2/2", "-1/2", "0/0"):
        args = types.SimpleNamespace(sweep_part=bad, steps=1, warmup=1, sweep_modes="shared",
                                     sweep_rows=4, workers=1, stats_jsonl="")
        with pytest.raises(SystemExit):
            b.run_sweep(None, args)
