"""External device allocator (pf_set_allocator) on the GPU: moving a live
context's buffers into PyTorch's caching allocator and back keeps its state
and its later results bit-identical to a context that never moved."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_torch_allocator_moves_buffers_and_keeps_results(gpu_lib):
    import torch
    p = W.tension_panel(n=16, l=0.1, du=1e-3, steps=6)
    a = gpu_lib.Context(p, scheme=1, precision=1)
    b = gpu_lib.Context(p, scheme=1, precision=1)
    for lam in p.loads[:2]:
        a.load_step(float(lam))
        b.load_step(float(lam))
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    b.use_torch_allocator()
    moved = torch.cuda.memory_allocated() - before
    # at least the FP64 state (u, u_try, d, four QP planes) lives there now
    assert moved >= 8 * (4 * b.N + 16 * b.E), moved
    for x, y in zip(a.get_state(), b.get_state()):
        np.testing.assert_array_equal(x, y)
    for lam in p.loads[2:4]:
        sa = a.load_step(float(lam))
        sb = b.load_step(float(lam))
        assert sa["n_stag"] == sb["n_stag"] and sa["n_cg_u"] == sb["n_cg_u"]
        np.testing.assert_array_equal(sa["force"], sb["force"])
    b.use_default_allocator()
    assert torch.cuda.memory_allocated() == before
    for lam in p.loads[4:]:
        sa = a.load_step(float(lam))
        sb = b.load_step(float(lam))
        np.testing.assert_array_equal(sa["force"], sb["force"])
    for x, y in zip(a.get_state(), b.get_state()):
        np.testing.assert_array_equal(x, y)
    a.close()
    b.close()


def test_torch_allocator_released_on_destroy(gpu_lib):
    import torch
    p = W.tension_panel(n=8, l=0.1, du=1e-3, steps=2)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    c = gpu_lib.Context(p, scheme=0)
    c.use_torch_allocator()
    assert torch.cuda.memory_allocated() > before
    c.set_dirichlet_d(p.dir_d_nodes, p.dir_d_values)    # reallocates group lists
    c.load_step(float(p.loads[0]))
    c.close()
    assert torch.cuda.memory_allocated() == before
