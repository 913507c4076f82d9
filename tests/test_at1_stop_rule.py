"""The AT1 phase solve's stop rules, emulated on the CPU (not GPU).

The device's semismooth Newton for F_d(d) = 0 (AT1 with the penalty,
Section 2) stops on ||F_d|| <= max(tol_pcg ||F_d(start)||, 1e-13 ||b||), or
once the active set has stopped changing and a step no longer halves
||F_d||.  This test mirrors that loop step for step: the same first step at
the kink, single-reduction (Chronopoulos-Gear) Jacobi CG to 1e-10 of each
step's residual as the device's FP64 solves, the same targets.  It uses the
oracle's AT1 residual and matrices and its displacement solves, on the
notched tension panel at l = 2h (the length-scale ratio of the 512^2
configuration), at 64^2.

A later staggered iteration starts the phase solve from an already
converged d: its target then lies below the rounding floor of F_d, and
without the stall rule the loop runs to its cap of 60 steps, the failure
the device showed at 512^2.  With the rule the load steps converge.
"""
import dataclasses

import numpy as np

import workloads as W
from oracle import Oracle, at1

MAX_NEWTON = 60


def cg_single_reduction(A, b, rtol):
    """Jacobi PCG with one reduction per iteration (Chronopoulos-Gear), to
    ||r|| <= rtol ||b|| on the recursively updated residual."""
    Dinv = 1.0 / A.diagonal()
    x = np.zeros_like(b)
    r = b.copy()
    z = Dinv * r
    w = A @ z
    gam, dl, rr0 = r @ z, w @ z, r @ r
    alpha, beta = gam / dl, 0.0
    p = np.zeros_like(b)
    s = np.zeros_like(b)
    for _ in range(100000):
        p = z + beta * p
        s = w + beta * s
        x += alpha * p
        r -= alpha * s
        if r @ r <= rtol ** 2 * rr0:
            break
        z = Dinv * r
        w = A @ z
        gn, dl = r @ z, w @ z
        beta = gn / gam
        alpha = gn / (dl - beta * gn / alpha)
        gam = gn
    return x


def phase_solve(o, psi, d, stall_rule):
    """Semismooth Newton on F_d with the device's stop rules; returns the
    new d and why the loop ended ('target', 'stall' or 'cap')."""
    mesh, f = o.mesh, o.d_free
    nb = at1.driving_scale(mesh, psi, f)
    chi_prev, nR0, nR_prev = None, None, 0.0
    for it in range(MAX_NEWTON + 1):
        dq, pq = mesh.interp(d), mesh.interp(o.d_prev)
        chi = (dq < pq) | ((dq == pq) if it == 0 else False)
        unchanged = chi_prev is not None and not np.any(chi != chi_prev)
        chi_prev = chi
        R = at1.residual(mesh, psi, d, o.d_prev, o.Gc, o.l, o.gamma)
        nR = np.linalg.norm(R[f])
        if nR0 is None:
            nR0 = nR
        if it > 0 and nR <= max(1e-10 * nR0, 1e-13 * nb):
            return d, "target"
        if stall_rule and it > 0 and unchanged and nR > 0.5 * nR_prev:
            return d, "stall"
        if it == MAX_NEWTON:
            return d, "cap"
        J = at1.matrix(mesh, at1.jacobian_coefficient(psi, chi, o.gamma), o.Gc, o.l)
        J = J.tocsr()[f][:, f]
        d = d.copy()
        d[f] += cg_single_reduction(J, -R[f], 1e-10)
        nR_prev = nR
    raise AssertionError("unreachable")


def run_steps(stall_rule, n=64, steps=2):
    p = dataclasses.replace(W.tension_panel(n=n, l=2.0 / n, du=6e-5, steps=steps),
                            phase_model=1)
    o = Oracle(p, 0)
    ends, counts, converged = [], [], []
    for lam in p.loads:
        lam = float(lam)
        u = o.u.copy()
        u[o.u_fixed] = lam * o.u_unit[o.u_fixed]
        d = o.d.copy()
        d[o.d_fixed] = o.d_val[o.d_fixed]
        R0 = np.linalg.norm(o.residual_u(u, d)[o.u_free])
        Rref = R0 if R0 > 0 else 1.0
        u, _, _ = o.newton(u, d, Rref)
        psi = o.energies(u, d)["psi_plus"]
        r, k = o.stag_residual(d, psi), 1
        while r > p.tol_stag and k < 20:
            d, why = phase_solve(o, psi, d, stall_rule)
            ends.append(why)
            u, _, _ = o.newton(u, d, Rref)
            psi = o.energies(u, d)["psi_plus"]
            r, k = o.stag_residual(d, psi), k + 1
        o.u, o.d = u, d
        o.d_prev = d.copy()
        counts.append(k)
        converged.append(r <= p.tol_stag)
    return ends, counts, converged


def test_without_the_stall_rule_a_later_solve_runs_to_the_cap():
    ends, _, _ = run_steps(stall_rule=False)
    assert "cap" in ends


def test_with_the_stall_rule_the_steps_converge():
    ends, counts, converged = run_steps(stall_rule=True)
    assert all(converged)
    assert "cap" not in ends and "stall" in ends
    assert max(counts) <= 5
