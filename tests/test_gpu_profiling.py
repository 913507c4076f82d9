"""Sampled kernel timing (GPU): pf_set_profiling / pf_kernel_time on every
work decomposition and Jacobi-Chebyshev degree of the two-kernel CG.  Every
timing event pair the CG driver reads must have been recorded: kernel 0
(apply) and 2 (update, fused with the first polynomial step or, on LDS
tiles from degree 3, the first two) always have samples; kernel 3 (the
first separate Chebyshev step of the displacement solves) only where such a
step exists."""
import math

import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rows", [1, 2])
@pytest.mark.parametrize("degree", [0, 1, 2, 3, 4])
def test_profiling_samples_match_the_kernels_run(gpu_lib, rows, degree):
    p = W.tension_panel(n=16, l=0.1, du=1e-3, steps=2)
    opts = {} if degree == 0 else {"precond": 1, "cheb_degree": degree}
    ctx = gpu_lib.Context(p, scheme=1, precision=1, march_rows=rows, **opts)
    ctx.set_profiling(True)
    st = ctx.load_step(float(p.loads[0]))
    assert st["converged"] == 1
    separate = 0 if degree <= 1 else degree - (3 if (rows == 1 and degree >= 3) else 2)
    for kid in range(4):
        n, ms, nodes = ctx.kernel_time(kid)
        print(f"rows={rows} degree={degree} kernel {kid}: {n} launches, {ms:.3f} ms, "
              f"{nodes} nodes", flush=True)
        assert math.isfinite(ms) and ms >= 0.0
        if kid in (0, 2):
            assert n > 0 and ms > 0.0
        if kid == 3:
            assert (n > 0) == (separate > 0)
    ctx.close()
