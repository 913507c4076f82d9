"""End-to-end parity of the HIP staggered solver against the FP64 oracle (GPU).

Every load step is compared (tests/_parity.py): staggered counts within +-1;
where the counts agree, relative L2 of u <= 1e-7 (FP64) / 1e-6 (mixed) and
max |d diff| <= 1e-5; where they differ by one, the same bounds plus twice
the oracle's own last staggered change of that step.  Reaction-force curve
error <= 1e-4 of its maximum, and at most one step per history compared at
the one-iteration bound only.
"""
import numpy as np
import pytest

import workloads as W
from _parity import check_step, compare_history, soa
from oracle import Oracle

pytestmark = pytest.mark.gpu


def bar_closed_form(p, lam):
    m = p.material
    Ep = m.E / (1 - m.nu ** 2)
    eps = lam / p.ly
    d = m.l * Ep * eps ** 2 / (m.Gc + m.l * Ep * eps ** 2)
    return d, ((1 - d) ** 2 + m.eta) * Ep * eps * p.lx


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_homogeneous_bar_closed_form(gpu_lib, scheme, precision):
    p = W.homogeneous_bar(nx=9, ny=70, lx=1.0, ly=1.0, du=5e-3, steps=6)
    ctx = gpu_lib.Context(p, scheme=scheme, precision=precision)
    for lam in p.loads:
        st = ctx.load_step(float(lam))
        d_ref, F_ref = bar_closed_form(p, lam)
        u, d, H = ctx.get_state()
        np.testing.assert_allclose(d, d_ref, rtol=1e-8 if precision == 0 else 1e-6)
        assert np.isclose(st["force"][1], F_ref, rtol=1e-8 if precision == 0 else 1e-6)
        assert st["converged"] == 1
        assert st["n_stag"] <= 3
    ctx.close()


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_small_panel_history_fp64(gpu_lib, scheme):
    p = W.tension_panel(n=16, l=0.1, du=1e-3, steps=8)
    compare_history(gpu_lib, p, scheme, 0, 8, 1e-7)


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_small_panel_history_mixed(gpu_lib, scheme):
    p = W.tension_panel(n=16, l=0.1, du=1e-3, steps=8)
    compare_history(gpu_lib, p, scheme, 1, 8, 1e-6)


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_shear_spectral_history_fp64(gpu_lib, scheme):
    """Shear panel with the spectral split: cracks under mixed-sign
    principal strains; S* predictors active from step 5."""
    p = W.shear_panel(n=16, l=0.1, du=2e-3, steps=8)
    compare_history(gpu_lib, p, scheme, 0, 8, 1e-7)


@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_shear_spectral_history_mixed(gpu_lib, scheme):
    p = W.shear_panel(n=16, l=0.1, du=2e-3, steps=8)
    compare_history(gpu_lib, p, scheme, 1, 8, 1e-6)


@pytest.mark.parametrize("scheme", [0, 1, 2])
def test_lshape_masked_history_fp64(gpu_lib, scheme):
    """L-shaped panel on a 32^2 grid with the upper-right quadrant masked
    out, the load patch and the d = 0 zone; steps 1-3 include nucleation."""
    p = W.lshape_panel(n=32, steps=10, total=0.3)
    compare_history(gpu_lib, p, scheme, 0, 3, 1e-7)


@pytest.mark.parametrize("scheme", [0, 1, 2])
def test_lshape_masked_history_mixed(gpu_lib, scheme):
    """The masked L-shape in mixed precision (FP32 inner solves): ST, and
    the S1 and S2 schemes that the 2048^2 L-shape configuration compares."""
    p = W.lshape_panel(n=32, steps=10, total=0.3)
    compare_history(gpu_lib, p, scheme, 1, 3, 1e-6)


@pytest.mark.parametrize("rows", [0, 1])
@pytest.mark.parametrize("degree", [1, 2, 3, 4])
@pytest.mark.parametrize("precision", [0, 1])
def test_chebyshev_preconditioner_history(gpu_lib, precision, degree, rows):
    """Jacobi-Chebyshev preconditioned solves reach the same fixed points:
    degree 1 (update only), 2 (fused update is the last step), 3 and 4 (odd
    and even buffer alternation), on both work decompositions."""
    p = W.tension_panel(n=16, l=0.1, du=1e-3, steps=6)
    compare_history(gpu_lib, p, 1, precision, 6, 1e-7 if precision == 0 else 1e-6,
                    precond=1, cheb_degree=degree, march_rows=rows)


def test_chebyshev_spectral_masked(gpu_lib):
    """Jacobi-Chebyshev on the spectral shear panel (mixed) and the masked
    L-shape (FP64)."""
    compare_history(gpu_lib, W.shear_panel(n=16, l=0.1, du=2e-3, steps=8), 3, 1, 8, 1e-6,
                    precond=1, cheb_degree=3)
    compare_history(gpu_lib, W.lshape_panel(n=32, steps=10, total=0.3), 1, 0, 3, 1e-7,
                    precond=1, cheb_degree=5)


def _ragged_panel():
    p = W.tension_panel(n=16, l=0.08, du=1e-3, steps=5)
    p.nx, p.ny = 133, 40
    nx, ny = p.nx, p.ny
    p.dir_u = [W._fix(W._edge_nodes(nx, ny, "bottom"), (0, 1)),
               W.DirichletU(W._edge_nodes(nx, ny, "top"), np.ones(nx + 1, np.int8),
                            np.ones(nx + 1))]
    p.dir_d_nodes = W.notch_nodes(nx, ny, 1.0, 1.0, 0.5)
    p.dir_d_values = np.ones(p.dir_d_nodes.shape)
    return p


@pytest.mark.parametrize("case", ["tension_s1_mixed", "tension_st_fp64", "shear_s3_mixed",
                                  "lshape_s1_fp64", "ragged_s1_mixed"])
def test_lds_tiles_history(gpu_lib, case):
    """The LDS-tile work decomposition (march_rows 1) reaches the oracle's
    fixed points: VD and spectral, masked, ragged, FP64 and mixed."""
    if case == "tension_s1_mixed":
        p, sch, prec, n, tol = W.tension_panel(n=16, l=0.1, du=1e-3, steps=8), 1, 1, 8, 1e-6
    elif case == "tension_st_fp64":
        p, sch, prec, n, tol = W.tension_panel(n=16, l=0.1, du=1e-3, steps=8), 0, 0, 8, 1e-7
    elif case == "shear_s3_mixed":
        p, sch, prec, n, tol = W.shear_panel(n=16, l=0.1, du=2e-3, steps=8), 3, 1, 8, 1e-6
    elif case == "lshape_s1_fp64":
        p, sch, prec, n, tol = W.lshape_panel(n=32, steps=10, total=0.3), 1, 0, 3, 1e-7
    else:
        p, sch, prec, n, tol = _ragged_panel(), 1, 1, 5, 1e-6
    compare_history(gpu_lib, p, sch, prec, n, tol, march_rows=1)


def test_ragged_panel_history_fp64(gpu_lib):
    """Non-square ragged mesh spanning several wave strips and chunks."""
    p = W.tension_panel(n=16, l=0.08, du=1e-3, steps=5)
    p.nx, p.ny = 133, 40
    nx, ny = p.nx, p.ny
    p.dir_u = [W._fix(W._edge_nodes(nx, ny, "bottom"), (0, 1)),
               W.DirichletU(W._edge_nodes(nx, ny, "top"), np.ones(nx + 1, np.int8),
                            np.ones(nx + 1))]
    p.dir_d_nodes = W.notch_nodes(nx, ny, 1.0, 1.0, 0.5)
    p.dir_d_values = np.ones(p.dir_d_nodes.shape)
    compare_history(gpu_lib, p, 1, 0, 5, 1e-7)


@pytest.mark.parametrize("scheme", [0, 1, 3])
def test_teacher_forced_nucleation_step(gpu_lib, scheme):
    """Inject the oracle's committed state before the nucleation step and
    compare that one step."""
    p = W.tension_panel(n=16, l=0.1, du=1e-3, steps=8)
    orc = Oracle(p, scheme)
    for lam in p.loads[:3]:
        orc.load_step(float(lam))
    u, d, H = orc.get_state()
    ctx = gpu_lib.Context(p, scheme=scheme)
    ctx.set_state(u, d, H)
    lam = float(p.loads[3])
    so = orc.load_step(lam)
    sg = ctx.load_step(lam)
    ug, dg, Hg = ctx.get_state()
    check_step("forced step 4", so.n_stag, so.last_du, so.last_dd, soa(orc.u), orc.d,
               sg["n_stag"], ug, dg, 1e-7)
    assert abs(sg["force"][1] - so.force) <= 1e-4 * abs(so.force)
    ctx.close()


def test_config_tension64_first_steps(gpu_lib):
    """64^2 notched tension panel, the first 8 load steps (pre-nucleation)."""
    p = W.config_tension64()
    compare_history(gpu_lib, p, 0, 0, 8, 1e-7)


def test_state_roundtrip_and_errors(gpu_lib):
    p = W.tension_panel(n=8, l=0.1, du=1e-3, steps=2)
    ctx = gpu_lib.Context(p, scheme=1)
    ctx.load_step(p.loads[0])
    u, d, H = ctx.get_state()
    ctx2 = gpu_lib.Context(p, scheme=1)
    ctx2.set_state(u, d, H)
    u2, d2, H2 = ctx2.get_state()
    np.testing.assert_array_equal(u, u2)
    np.testing.assert_array_equal(d, d2)
    np.testing.assert_array_equal(H, H2)
    bad = d.copy()
    bad[3] = np.nan
    with pytest.raises(gpu_lib.PhaseFieldError):
        ctx2.set_state(d=bad)
    # staggered_iterate / commit protocol
    s0 = ctx2.staggered_iterate(p.loads[1])
    assert s0["n_stag"] == 1
    with pytest.raises(gpu_lib.PhaseFieldError):
        ctx2.staggered_iterate(p.loads[1] * 2)
    while s0["r_stag"] > p.tol_stag:
        s0 = ctx2.staggered_iterate(p.loads[1])
    ctx2.commit_step()
    with pytest.raises(gpu_lib.PhaseFieldError):
        ctx2.commit_step()
    ref = ctx.load_step(p.loads[1])
    assert ref["n_stag"] == s0["n_stag"]
    np.testing.assert_allclose(ctx2.reaction_force(1), ref["force"], rtol=1e-12)
    ctx.close()
    ctx2.close()


def test_max_stag_reports_not_converged(gpu_lib):
    p = W.tension_panel(n=16, l=0.1, du=1e-3, steps=4)
    ctx = gpu_lib.Context(p, scheme=0, max_stag=2)
    st = None
    for lam in p.loads[:4]:
        st = ctx.load_step(lam)
    assert st["converged"] == 0 and st["n_stag"] == 2
    ctx.close()
