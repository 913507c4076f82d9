"""Pins for the oracle's 3-D hexahedral path (not GPU).

* Plane-strain equivalence: the 2-D notched panel extruded into a slab with
  u_z = 0 on both faces (one or two element layers) is plane strain; its
  fields are the 2-D oracle's on every node layer, its staggered counts the
  same, and its reaction force the 2-D force per unit thickness times the
  thickness.  This ties the 3-D kinematics, split, tangent, phase operator
  and staggered loop to the independently pinned 2-D oracle.
* Uniaxial stress: a cube on rollers pulled on one face has the affine
  displacement u = eps (-nu x, y, -nu z), Psi+ = E eps^2 / 2 (the trace
  eps (1 - 2 nu) is positive), so d = l E eps^2 / (Gc + l E eps^2) and the
  reaction force is g(d) E eps times the face area (textbook 3-D values,
  with E, not the plane-strain modulus).
"""
import numpy as np
import pytest

import workloads as W
from oracle import Oracle
from oracle.hex3d import Oracle3D


@pytest.mark.parametrize("nz", [1, 2])
@pytest.mark.parametrize("scheme", [0, 1, 3])
def test_slab_is_plane_strain(scheme, nz):
    # steps 1-2: the second already runs gated trial solves (S1, S3)
    p2 = W.tension_panel(n=8, l=0.2, du=2e-3, steps=2)
    lz = 0.1
    p3 = W.slab_from_panel(p2, nz=nz, lz=lz)
    o2, o3 = Oracle(p2, scheme), Oracle3D(p3, scheme)
    P = (p2.nx + 1) * (p2.ny + 1)
    trials = 0
    for lam in p2.loads:
        s2, s3 = o2.load_step(float(lam)), o3.load_step(float(lam))
        assert s2.converged and s3.converged
        assert s2.n_stag == s3.n_stag, (scheme, lam, s2.n_stag, s3.n_stag)
        trials += s3.n_trial
        for k in range(nz + 1):
            lay = slice(k * P, (k + 1) * P)
            np.testing.assert_allclose(o3.d[lay], o2.d, rtol=1e-8, atol=1e-12)
            np.testing.assert_allclose(o3.u[3 * k * P:3 * (k + 1) * P][0::3], o2.u[0::2],
                                       rtol=1e-8, atol=1e-14)
            np.testing.assert_allclose(o3.u[3 * k * P:3 * (k + 1) * P][1::3], o2.u[1::2],
                                       rtol=1e-8, atol=1e-14)
        assert np.abs(o3.u[2::3]).max() < 1e-14
        assert np.isclose(s3.force, s2.force * lz, rtol=1e-8)
    if scheme != 0:
        assert trials > 0


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_uniaxial_bar3d_closed_form(scheme):
    p = W.uniaxial_bar3d(n=3, l=0.03, du=5e-3, steps=6)
    m = p.material
    o = Oracle3D(p, scheme)
    for lam in p.loads:
        st = o.load_step(float(lam))
        eps = lam / p.ly
        d_ref = m.l * m.E * eps ** 2 / (m.Gc + m.l * m.E * eps ** 2)
        F_ref = ((1 - d_ref) ** 2 + m.eta) * m.E * eps * p.lx * p.lz
        assert st.converged
        np.testing.assert_allclose(o.d, d_ref, rtol=1e-9)
        assert np.isclose(st.force, F_ref, rtol=1e-9)
        # lateral contraction: u_x = -nu eps x on the face x = 1
        nodes = np.arange(o.mesh.n_nodes)
        xface = nodes[(nodes % (p.nx + 1)) == p.nx]
        np.testing.assert_allclose(o.u[3 * xface], -m.nu * eps * p.lx, rtol=1e-9)
        if scheme == 0:
            assert st.n_stag == 2
        else:
            assert st.n_stag <= 3
