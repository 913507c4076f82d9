"""The allocation-free tangent apply (GPU): pf_tangent_apply_noalloc through
the C ABI against pf_op_tangent_apply of a context on the same mesh, which
runs the same kernels with the indicator bytes in a buffer of its own.  Two
calls in a row, the second on a smaller mesh, so the second reuses the
device scratch array the first filled; both must equal the context's result
bit for bit (same kernels, same work decomposition, same summation order).
Masked L-shape and spectral split cases cover the mask pointer and the
other tangent."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _fields(torch, p, seed):
    N = (p.nx + 1) * (p.ny + 1)
    g = torch.Generator(device="cuda").manual_seed(seed)
    # strains of mixed sign, so both branches of the split are active
    u = (torch.rand(2 * N, dtype=torch.float64, device="cuda", generator=g) - 0.5) * 1e-3
    d = torch.rand(N, dtype=torch.float64, device="cuda", generator=g)
    pv = torch.rand(2 * N, dtype=torch.float64, device="cuda", generator=g) - 0.5
    return u, d, pv


def _check(pf, torch, p, seed):
    ctx = pf.Context(p)
    u, d, pv = _fields(torch, p, seed)
    q_ref = torch.empty_like(u)
    ctx.op_tangent_apply(u, d, pv, q_ref)
    mask = None
    if p.elem_active is not None:
        mask = torch.from_numpy(np.ascontiguousarray(p.elem_active, dtype=np.uint8)).cuda()
    q = torch.full_like(u, np.nan)
    pf.tangent_apply_noalloc(p, u, d, pv, q, elem_active=mask)
    torch.cuda.synchronize()
    ctx.close()
    a, b = q.cpu().numpy(), q_ref.cpu().numpy()
    assert np.isfinite(a).all()
    np.testing.assert_array_equal(a, b)
    return a


@pytest.mark.parametrize("case", ["tension_vd", "lshape_masked", "shear_spectral"])
def test_noalloc_tangent_apply_matches_context(gpu_lib, case):
    import torch
    if case == "tension_vd":
        big, small = W.tension_panel(n=96), W.tension_panel(n=20)
        big.nx, big.ny = 133, 77          # ragged: several strips, chunks and tiles
    elif case == "lshape_masked":
        big, small = W.lshape_panel(n=64, steps=2), W.lshape_panel(n=16, steps=2)
    else:
        big, small = W.shear_panel(n=80, steps=2), W.shear_panel(n=12, steps=2)
    first = _check(gpu_lib, torch, big, 1)
    second = _check(gpu_lib, torch, small, 2)
    assert first.size > second.size
