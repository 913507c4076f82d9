"""The Python binding's own checks (not GPU): what it verifies before a
device pointer reaches the C ABI, which cannot see sizes or dtypes, and the
batch's refusal to step once a member context is closed."""
import ctypes

import pytest
import torch

import paper_2209_07969_amd as pf


def test_device_argument_checks():
    n = 12
    ok = torch.zeros(n, dtype=torch.float64)
    with pytest.raises(TypeError, match="torch.Tensor"):
        pf._dev_arg(ok.numpy(), torch.float64, n, 0, "u")
    with pytest.raises(TypeError, match="dtype"):
        pf._dev_arg(ok.float(), torch.float64, n, 0, "u")
    with pytest.raises(TypeError, match="dtype"):
        pf._dev_arg(torch.zeros(n, dtype=torch.int8), torch.uint8, n, 0, "flags")
    with pytest.raises(ValueError, match="needs 13 elements"):
        pf._dev_arg(ok, torch.float64, n + 1, 0, "u")
    with pytest.raises(ValueError, match="contiguous"):
        pf._dev_arg(torch.zeros(2 * n, dtype=torch.float64)[::2], torch.float64, n, 0, "u")
    # every host-visible property right: refused only for living in host memory
    with pytest.raises(ValueError, match="device tensor"):
        pf._dev_arg(ok, torch.float64, n, 0, "u")
    with pytest.raises(ValueError, match="device tensor"):
        pf._dev_arg(ok.reshape(3, 4), torch.float64, n, 0, "H")


class _Member:
    """Stands in for a Context: pf_batch_create only records the handles."""

    def __init__(self, addr):
        self.h = ctypes.c_void_p(addr)


def test_batch_refuses_a_closed_member():
    members = [_Member(0x1000), _Member(0x2000)]
    b = pf.Batch(members)
    members[1].h = None
    with pytest.raises(RuntimeError, match="closed"):
        b.load_step([1.0, 1.0])
    b.close()


def test_every_entry_fails_loudly_without_a_device():
    """The product path has no CPU fallback: without a HIP device every
    class that would run kernels raises before touching the library's
    compute entry points (not GPU; skipped where a device is visible)."""
    if torch.cuda.is_available():
        import pytest as _pytest
        _pytest.skip("a HIP device is visible")
    import workloads as W
    p2 = W.tension_panel(n=4, steps=1)
    p3 = W.uniaxial_bar3d(n=1, steps=1)
    for make in (lambda: pf.Context(p2), lambda: pf.Hex3DOps(p3),
                 lambda: pf.Hex3DContext(p3)):
        with pytest.raises(RuntimeError, match="no HIP device"):
            make()
