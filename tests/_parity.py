"""Step-by-step comparison of the HIP solver with the FP64 oracle.

Tolerances (one load step):
* staggered counts within +-1;
* where the counts agree, both sides end on the same staggered iterate:
  relative L2 of u <= u_tol (1e-7 FP64, 1e-6 mixed) and max |d diff| <= 1e-5;
* where they differ by one, one side has taken one staggered iteration more
  than the other.  The two end states then differ by about one iteration's
  change, which the oracle measures in its own last iteration of the step
  (``last_du``: ||u^k - u^{k-1}|| / ||u^k||, ``last_dd``: max |d^k - d^{k-1}|).
  The bound is the full tolerance plus twice that change (the factor covers
  a contraction rate near 1 in the slow steps of crack growth).

Every step is compared; a history also has to reach a minimum number of
steps compared at the full tolerance, so that it cannot pass on counts and
forces alone.
"""
from __future__ import annotations

import numpy as np

D_TOL = 1e-5
STAG_MARGIN = 2.0


def soa(o_u):
    """Interleaved oracle displacement [2N] -> [2][N] (the library's layout)."""
    return np.stack([o_u[0::2], o_u[1::2]])


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def check_step(tag, n_orc, last_du, last_dd, u_orc, d_orc, n_gpu, u_gpu, d_gpu, u_tol):
    """Compare one step; returns True when it was compared at full tolerance.

    u_orc and u_gpu are [2][N]; n_* are the staggered counts."""
    dn = abs(int(n_orc) - int(n_gpu))
    eu = rel_l2(u_gpu, u_orc)
    ed = float(np.abs(d_gpu - d_orc).max()) if d_orc.size else 0.0
    full = dn == 0
    bu = u_tol if full else u_tol + STAG_MARGIN * last_du
    bd = D_TOL if full else D_TOL + STAG_MARGIN * last_dd
    print(f"  {tag}: stag oracle={n_orc} gpu={n_gpu} rel-L2(u)={eu:.2e} (<= {bu:.1e}) "
          f"max|dd|={ed:.2e} (<= {bd:.1e}){'' if full else ' [counts differ]'}", flush=True)
    assert dn <= 1, (tag, n_orc, n_gpu)
    assert eu <= bu, (tag, eu, bu)
    assert ed <= bd, (tag, ed, bd)
    return full


def compare_history(pf, p, scheme, precision, n_steps, u_tol, min_full=None, orc=None,
                    ctx=None, **opts):
    """Run n_steps load steps on both sides and compare every step.

    min_full defaults to n_steps - 1: at most one step may be compared at the
    staggered (one-iteration) tolerance only."""
    from oracle import Oracle
    orc = Oracle(p, scheme) if orc is None else orc
    own = ctx is None
    ctx = pf.Context(p, scheme=scheme, precision=precision, **opts) if own else ctx
    F_o, F_g = [], []
    n_full = 0
    for n, lam in enumerate(p.loads[:n_steps]):
        so = orc.load_step(float(lam))
        sg = ctx.load_step(float(lam))
        F_o.append(so.force)
        F_g.append(sg["force"][p.load_comp])
        u, d, _ = ctx.get_state()
        n_full += check_step(f"step {n + 1} lam={lam:.3e}", so.n_stag, so.last_du, so.last_dd,
                             soa(orc.u), orc.d, sg["n_stag"], u, d, u_tol)
    F_o, F_g = np.array(F_o), np.array(F_g)
    err = np.abs(F_g - F_o).max() / np.abs(F_o).max()
    need = n_steps - 1 if min_full is None else min_full
    print(f"  force curve error {err:.2e}; steps at full tolerance {n_full}/{n_steps} "
          f"(need {need})", flush=True)
    assert err <= 1e-4, err
    assert n_full >= need, (n_full, need)
    if own:
        ctx.close()
    return n_full
