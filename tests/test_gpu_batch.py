"""Batched sweeps and autotuning (GPU): a batch of members on their own streams
gives bit-identical results to stepping them one by one; autotuning keeps
parity with the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import Oracle

pytestmark = pytest.mark.gpu


def test_batch_matches_sequential(gpu_lib):
    import torch
    probs = [W.tension_panel(n=n, l=0.1, du=1e-3, steps=4, notch=a)
             for n, a in ((16, 0.5), (24, 0.375), (20, 0.45))]
    seq = [gpu_lib.Context(p, scheme=s) for p, s in zip(probs, (1, 0, 3))]
    streams = [torch.cuda.Stream() for _ in probs]
    bat = [gpu_lib.Context(p, scheme=s, stream=st.cuda_stream)
           for p, s, st in zip(probs, (1, 0, 3), streams)]
    B = gpu_lib.Batch(bat, workers=3)
    for k in range(4):
        lams = [float(p.loads[k]) for p in probs]
        sb = B.load_step(lams)
        for i, c in enumerate(seq):
            s = c.load_step(lams[i])
            assert s["n_stag"] == sb[i]["n_stag"]
            assert s["force"] == sb[i]["force"]
    for a, b in zip(seq, bat):
        ua, da, Ha = a.get_state()
        ub, db, Hb = b.get_state()
        np.testing.assert_array_equal(ua, ub)
        np.testing.assert_array_equal(da, db)
        np.testing.assert_array_equal(Ha, Hb)
    B.close()


def _mixed_members():
    """Uneven mixed-precision members: several work decompositions, a
    spectral member, a masked L-shape and a Chebyshev-preconditioned member,
    so the shared launches hold several apply groups and both operator
    kinds while one member solves on its own stream."""
    return [
        (W.tension_panel(n=16, l=0.1, du=1e-3, steps=4, notch=0.5), 1, {}),
        (W.tension_panel(n=24, l=0.1, du=1e-3, steps=4, notch=0.375), 1, {"march_rows": 2}),
        (W.tension_panel(n=20, l=0.1, du=1e-3, steps=4, notch=0.45), 0, {"march_rows": 8}),
        (W.shear_panel(n=16, l=0.1, du=2e-3, steps=4), 3, {}),
        (W.lshape_panel(n=32, steps=4, total=0.12), 1, {}),
        # Jacobi-Chebyshev member: its solves stay on its own stream
        (W.tension_panel(n=18, l=0.1, du=1e-3, steps=4, notch=0.4), 1,
         {"precond": 1, "cheb_degree": 3, "march_rows": 1}),
    ]


@pytest.mark.parametrize("shared", [True, False])
def test_batch_mixed_matches_sequential(gpu_lib, shared):
    import torch
    mem = _mixed_members()
    seq = [gpu_lib.Context(p, scheme=s, precision=1, **kw) for p, s, kw in mem]
    streams = [torch.cuda.Stream() for _ in mem]
    bat = [gpu_lib.Context(p, scheme=s, precision=1, stream=st.cuda_stream, **kw)
           for (p, s, kw), st in zip(mem, streams)]
    B = gpu_lib.Batch(bat, workers=3, shared=shared)
    for k in range(4):
        lams = [float(p.loads[k]) for p, _, _ in mem]
        sb = B.load_step(lams)
        for i, c in enumerate(seq):
            s = c.load_step(lams[i])
            for key in ("n_stag", "n_newton", "n_cg_u", "n_cg_d", "n_cg_trial"):
                assert s[key] == sb[i][key], (shared, k, i, key, s[key], sb[i][key])
            assert s["force"] == sb[i]["force"]
    for a, b in zip(seq, bat):
        for x, y in zip(a.get_state(), b.get_state()):
            np.testing.assert_array_equal(x, y)
    B.close()
    for c in seq + bat:
        c.close()


def test_autotune_keeps_parity(gpu_lib):
    p = W.tension_panel(n=16, l=0.1, du=1e-3, steps=5)
    ctx = gpu_lib.Context(p, scheme=1)
    orc = Oracle(p, 1)
    for lam in p.loads[:2]:
        ctx.load_step(float(lam))
        orc.load_step(float(lam))
    ch = ctx.autotune(5)
    assert ch in (2, 4, 8)
    for lam in p.loads[2:]:
        sg = ctx.load_step(float(lam))
        so = orc.load_step(float(lam))
        assert abs(sg["n_stag"] - so.n_stag) <= 1
        assert abs(sg["force"][1] - so.force) <= 1e-4 * abs(so.force)
    ctx.close()


def _oracle_batch_members():
    """Eight uneven mixed-precision members of a tension sweep (meshes 12^2
    to 24^2, two regularisation lengths, four notch lengths, S1/S2/S3 and one
    ST member): each is compared with its own oracle run."""
    spec = [(16, 0.1, 0.5, 1), (24, 0.1, 0.375, 1), (20, 0.08, 0.45, 2), (12, 0.12, 0.5, 3),
            (18, 0.1, 0.4, 1), (22, 0.09, 0.3, 0), (14, 0.1, 0.6, 1), (16, 0.08, 0.35, 3)]
    return [(W.tension_panel(n=n, l=l, du=1e-3, steps=5, notch=a), s) for n, l, a, s in spec]


@pytest.mark.parametrize("shared", [True, False])
def test_batch_members_match_oracle(gpu_lib, shared):
    """Every member of an 8-instance mixed batch (shared CG launches or
    concurrent streams) against its own FP64 oracle history, step by step
    under the parity protocol."""
    import torch
    from _parity import check_step, soa
    mem = _oracle_batch_members()
    streams = [torch.cuda.Stream() for _ in mem]
    ctxs = [gpu_lib.Context(p, scheme=s, precision=1, stream=st.cuda_stream)
            for (p, s), st in zip(mem, streams)]
    orcs = [Oracle(p, s) for p, s in mem]
    B = gpu_lib.Batch(ctxs, workers=4, shared=shared)
    n_steps = 5
    F = [([], []) for _ in mem]
    n_full = [0] * len(mem)
    for k in range(n_steps):
        sb = B.load_step([float(p.loads[k]) for p, _ in mem])
        for i, ((p, s), orc, ctx) in enumerate(zip(mem, orcs, ctxs)):
            so = orc.load_step(float(p.loads[k]))
            u, d, _ = ctx.get_state()
            n_full[i] += check_step(f"member {i} (n={p.nx}, scheme {s}) step {k + 1}",
                                    so.n_stag, so.last_du, so.last_dd, soa(orc.u), orc.d,
                                    sb[i]["n_stag"], u, d, 1e-6)
            F[i][0].append(so.force)
            F[i][1].append(sb[i]["force"][1])
    B.close()
    for i, (fo, fg) in enumerate(F):
        fo, fg = np.array(fo), np.array(fg)
        err = np.abs(fg - fo).max() / np.abs(fo).max()
        assert err <= 1e-4, (i, err)
        assert n_full[i] >= n_steps - 1, (i, n_full[i])
    for c in ctxs:
        c.close()
